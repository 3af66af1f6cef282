// Linearised measurement operator (Eq. (1)), the data term of the loss
// (Eq. (4), mean-squared form), the output head and the fused Adam update.
//
// J is stored compacted to the voxels of the imaging region (M x qa_pad,
// row-major, zero-padded columns): the products J sigma and J^T g each stream
// it once from HBM with 16-byte loads; sums over column or row blocks land in
// partial buffers that a second pass reduces in a fixed order.
#include <algorithm>

#include "kernels.h"

namespace d2ip {
namespace {

__global__ void k_gather_columns(const float* __restrict__ J, int M, int Q,
                                 const int* __restrict__ idx, int qa, int qa_pad,
                                 float* __restrict__ Jc) {
  const size_t total = (size_t)M * qa_pad;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int q = (int)(i % qa_pad);
    const size_t m = i / qa_pad;
    Jc[i] = q < qa ? J[m * Q + idx[q]] : 0.f;
  }
}

// Members of a group share J: each block reads its J tile once and forms the
// partial products for every member (up to kJMaxB per launch).  Each wave
// owns kJvecRows / 4 rows and issues all of their loads before reducing, so
// a lane keeps 16 independent 16-byte loads in flight.
constexpr int kJvecRowsPerWave = kJvecRows / 4;
__global__ __launch_bounds__(256) void k_jvec(const float* __restrict__ Jc, int M, int qa_pad,
                                              const int* __restrict__ idx, const float* sigma,
                                              float* ppart, int B, long long istride) {
  extern __shared__ __align__(16) float sv[];  // [B][kJvecCols]
  const int q0 = blockIdx.x * kJvecCols;
  const int qn = min(kJvecCols, qa_pad - q0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m0 = blockIdx.y * kJvecRows + wave * kJvecRowsPerWave;
  constexpr int KV = kJvecCols / 256;  // float4 per lane per row
  // issue order: the gather indices, this wave's J rows, then the image
  // values at the indices, so the dependent gather overlaps the J stream.
  // Addresses are clamped in bounds (qn >= 64, a multiple of 64) so the loads
  // carry no branches: a clamped column meets a zero image value and a
  // clamped row's sum is not stored
  int iq[KV];
#pragma unroll
  for (int k = 0; k < KV; ++k) iq[k] = idx[q0 + min((int)threadIdx.x + 256 * k, qn - 1)];
  float4 jv[kJvecRowsPerWave][KV];
#pragma unroll
  for (int r = 0; r < kJvecRowsPerWave; ++r) {
    const int m = m0 + r;
    const float* row = Jc + (size_t)min(m, M - 1) * qa_pad + q0;
#pragma unroll
    for (int k = 0; k < KV; ++k) {
      const int j = lane * 4 + 256 * k;
      jv[r][k] = *reinterpret_cast<const float4*>(row + min(j, qn - 4));
    }
  }
  {
    float gv[KV];
#pragma unroll
    for (int k = 0; k < KV; ++k) gv[k] = sigma[iq[k]];
#pragma unroll
    for (int k = 0; k < KV; ++k) {
      const int q = threadIdx.x + 256 * k;
      sv[q] = q < qn ? gv[k] : 0.f;
    }
  }
  for (int b = 1; b < B; ++b) {
    const float* sg = ishift(sigma, b * istride);
#pragma unroll
    for (int k = 0; k < KV; ++k) {
      const int q = threadIdx.x + 256 * k;
      sv[b * kJvecCols + q] = q < qn ? sg[iq[k]] : 0.f;
    }
  }
  __syncthreads();
  for (int b = 0; b < B; ++b) {
#pragma unroll
    for (int r = 0; r < kJvecRowsPerWave; ++r) {
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < KV; ++k) {
        const float4 sb = *reinterpret_cast<const float4*>(&sv[b * kJvecCols + lane * 4 + 256 * k]);
        acc += jv[r][k].x * sb.x + jv[r][k].y * sb.y + jv[r][k].z * sb.z + jv[r][k].w * sb.w;
      }
      const float v = wave_sum(acc);
      const int m = m0 + r;
      if (lane == 0 && m < M) ishift(ppart, b * istride)[(size_t)blockIdx.x * M + m] = v;
    }
  }
}

// Residual, loss partial and data gradient of the kJtRows rows of a block,
// from the column-block partials of J sigma: 8 threads per row sum column
// blocks k = j, j+8, .. in increasing order and combine by a butterfly, the
// same order as the fused path of k_jtvec.  g_p = (2/M) r
// is written over column block 0's partial of its row, a slot only the thread
// that reads it writes.
__global__ __launch_bounds__(256) void k_resid(float* ppart, int nqb, int M, const float* dv,
                                               double* rsum, long long istride) {
  {
    const long long off = (long long)blockIdx.y * istride;
    ppart = ishift(ppart, off); dv = ishift(dv, off); rsum = ishift(rsum, off);
  }
  __shared__ double sh[16];
  const int m0 = blockIdx.x * kJtRows;
  const int mn = min(kJtRows, M - m0);
  const int r = threadIdx.x >> 3, j = threadIdx.x & 7;
  float p = 0.f;
  if (r < mn) {
    // up to 32 column blocks per thread in flight at once (addresses clamped,
    // clamped values added as zeros), summed in increasing order
    const float* col = ppart + m0 + r;
    for (int k0 = j; k0 < nqb; k0 += 8 * 32) {
      float v[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) v[u] = col[(size_t)min(k0 + 8 * u, nqb - 1) * M];
#pragma unroll
      for (int u = 0; u < 32; ++u) p += k0 + 8 * u < nqb ? v[u] : 0.f;
    }
  }
#pragma unroll
  for (int o = 4; o > 0; o >>= 1) p += __shfl_xor(p, o, 8);
  double rr = 0.0;
  if (j == 0 && r < mn) {
    const float res = p - dv[m0 + r];
    ppart[m0 + r] = (2.f / (float)M) * res;
    rr = (double)res * res;
  }
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) rsum[blockIdx.x] = rr;
}

// J^T g over row groups of rpg rows (large grids): the data gradient of every
// row is in column block 0 of ppart (k_resid).  Each thread accumulates its 4
// columns over the group's rows in batches of 8, the next batch loading under
// the current one's arithmetic; addresses are clamped (a clamped row weighs
// zero, a clamped column is not stored).
__global__ __launch_bounds__(256) void k_jt_rows(const float* __restrict__ Jc, int M, int qa_pad,
                                                 const float* gp, int rpg, float* tpart, int B,
                                                 long long istride) {
  constexpr int kB = 8;
  const int m0 = blockIdx.y * rpg;
  const int mn = min(rpg, M - m0);
  const int q = (blockIdx.x * 256 + threadIdx.x) * 4;
  const float* base = Jc + (size_t)m0 * qa_pad + min(q, qa_pad - 4);
  auto jrow = [&](int r) {
    return *reinterpret_cast<const float4*>(base + (size_t)min(r, mn - 1) * qa_pad);
  };
  float4 acc[kJMaxB];
#pragma unroll
  for (int b = 0; b < kJMaxB; ++b) acc[b] = make_float4(0.f, 0.f, 0.f, 0.f);
  // member 0's data gradient of a batch: two aligned float4 (rpg and kB are
  // multiples of 8 and the partial buffer is 256-byte aligned); rows past the
  // group read (and drop) the next rows of the buffer, which holds
  // nqb > kJtFuseMax column blocks of M rows, so m0 + r0 + 8 <= M + 8 stays
  // inside it
  auto gload = [&](int r0, float4& lo, float4& hi) {
    lo = *reinterpret_cast<const float4*>(gp + m0 + r0);
    hi = *reinterpret_cast<const float4*>(gp + m0 + r0 + 4);
  };
  float4 jv[kB], glo, ghi;
#pragma unroll
  for (int r = 0; r < kB; ++r) jv[r] = jrow(r);
  gload(0, glo, ghi);
  for (int r0 = 0; r0 < mn; r0 += kB) {
    // the next batch (clamped: past the group it repeats the last row)
    float4 nx[kB], nlo, nhi;
#pragma unroll
    for (int r = 0; r < kB; ++r) nx[r] = jrow(r0 + kB + r);
    gload(r0 + kB < mn ? r0 + kB : r0, nlo, nhi);
    const float g0[kB] = {glo.x, glo.y, glo.z, glo.w, ghi.x, ghi.y, ghi.z, ghi.w};
#pragma unroll
    for (int r = 0; r < kB; ++r) {
      const bool ok = r0 + r < mn;
#pragma unroll
      for (int b = 0; b < kJMaxB; ++b) {
        if (b >= B) break;
        const float gv = b == 0 ? g0[r] : ishift(gp, b * istride)[m0 + r0 + r];
        const float g = ok ? gv : 0.f;
        acc[b].x += jv[r].x * g;
        acc[b].y += jv[r].y * g;
        acc[b].z += jv[r].z * g;
        acc[b].w += jv[r].w * g;
      }
    }
#pragma unroll
    for (int r = 0; r < kB; ++r) jv[r] = nx[r];
    glo = nlo;
    ghi = nhi;
  }
  if (q >= qa_pad) return;
#pragma unroll
  for (int b = 0; b < kJMaxB; ++b) {
    if (b >= B) break;
    *reinterpret_cast<float4*>(ishift(tpart, b * istride) + (size_t)blockIdx.y * qa_pad + q) =
        acc[b];
  }
}

__global__ __launch_bounds__(256) void k_jtvec(const float* __restrict__ Jc, int M, int qa_pad,
                                               const float* ppart, int nqb, const float* dv,
                                               double* rsum, float* tpart, int B,
                                               long long istride) {
  __shared__ float gs[kJMaxB][kJtRows];
  __shared__ double sh[16];
  const int m0 = blockIdx.y * kJtRows;
  const int mn = min(kJtRows, M - m0);
  // Issue order: member 0's residual inputs (the first kJtPre column-block
  // partials of this thread's row, and its measurement), then the first
  // kJtBatch J rows of this thread's 4 columns, which load while the residual
  // is formed.  Addresses are clamped in bounds (a clamped partial is
  // dropped, a clamped row has a zero residual weight, a clamped column is not
  // stored), so the loads carry no branches.
  constexpr int kJtBatch = 8, kJtPre = 4;
  const int r = threadIdx.x >> 3, j = threadIdx.x & 7;
  const int rc = m0 + min(r, mn - 1);
  float pv[kJtPre];
#pragma unroll
  for (int i = 0; i < kJtPre; ++i) pv[i] = ppart[(size_t)min(j + 8 * i, nqb - 1) * M + rc];
  const float dv0 = dv[rc];
  __builtin_amdgcn_sched_barrier(0);  // keep these loads ahead of the J rows
  const int q = (blockIdx.x * 256 + threadIdx.x) * 4;
  const float* base = Jc + (size_t)m0 * qa_pad + min(q, qa_pad - 4);
  auto jrow = [&](int rr) {
    return *reinterpret_cast<const float4*>(base + (size_t)min(rr, mn - 1) * qa_pad);
  };
  float4 jv[kJtBatch];
#pragma unroll
  for (int rr = 0; rr < kJtBatch; ++rr) jv[rr] = jrow(rr);
  // residual of this block's rows for every member: 8 threads per row,
  // column blocks k = j, j+8, .. combined by a butterfly (fixed order)
  for (int b = 0; b < B; ++b) {
    const long long off = b * istride;
    const float* pp = ishift(ppart, off);
    float p = 0.f;
    if (b == 0) {
#pragma unroll
      for (int i = 0; i < kJtPre; ++i) p += j + 8 * i < nqb ? pv[i] : 0.f;
      if (r < mn)
        for (int k = j + 8 * kJtPre; k < nqb; k += 8) p += pp[(size_t)k * M + m0 + r];
    } else if (r < mn) {
      for (int k = j; k < nqb; k += 8) p += pp[(size_t)k * M + m0 + r];
    }
#pragma unroll
    for (int o = 4; o > 0; o >>= 1) p += __shfl_xor(p, o, 8);
    double rr = 0.0;
    if (j == 0 && r < kJtRows) {
      const float res = r < mn ? p - (b == 0 ? dv0 : ishift(dv, off)[m0 + r]) : 0.f;
      gs[b][r] = (2.f / (float)M) * res;
      rr = (double)res * res;
    }
    if (blockIdx.x == 0) {
      rr = block_sum(rr, sh);
      if (threadIdx.x == 0) ishift(rsum, off)[blockIdx.y] = rr;
    }
  }
  __syncthreads();
  float4 acc[kJMaxB];
#pragma unroll
  for (int b = 0; b < kJMaxB; ++b) acc[b] = make_float4(0.f, 0.f, 0.f, 0.f);
  // all kJtRows rows in batches (rows beyond mn weigh zero), the next batch
  // loading under the current one's arithmetic
#pragma unroll
  for (int r0 = 0; r0 < kJtRows; r0 += kJtBatch) {
    float4 nx[kJtBatch];
    if (r0 + kJtBatch < kJtRows) {
#pragma unroll
      for (int r = 0; r < kJtBatch; ++r) nx[r] = jrow(r0 + kJtBatch + r);
    }
#pragma unroll
    for (int r = 0; r < kJtBatch; ++r) {
#pragma unroll
      for (int b = 0; b < kJMaxB; ++b) {
        if (b >= B) break;
        const float g = gs[b][r0 + r];
        acc[b].x += jv[r].x * g;
        acc[b].y += jv[r].y * g;
        acc[b].z += jv[r].z * g;
        acc[b].w += jv[r].w * g;
      }
    }
    if (r0 + kJtBatch < kJtRows) {
#pragma unroll
      for (int r = 0; r < kJtBatch; ++r) jv[r] = nx[r];
    }
  }
  if (q >= qa_pad) return;
#pragma unroll
  for (int b = 0; b < kJMaxB; ++b) {
    if (b >= B) break;
    *reinterpret_cast<float4*>(ishift(tpart, b * istride) + (size_t)blockIdx.y * qa_pad + q) =
        acc[b];
  }
}

__global__ void k_tail_fwd(const float* d0, int C, const float* w, const float* b,
                           const float* __restrict__ mask, size_t V, float* sigma,
                           long long istride) {
  {
    const long long off = (long long)blockIdx.y * istride;
    d0 = ishift(d0, off); w = ishift(w, off); b = ishift(b, off); sigma = ishift(sigma, off);
  }
  for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < V;
       v += (size_t)gridDim.x * blockDim.x) {
    const float4* row = reinterpret_cast<const float4*>(d0 + v * C);
    float acc = b[0];
    for (int c4 = 0; c4 < C / 4; ++c4) {
      const float4 x = row[c4];
      acc += w[4 * c4] * x.x + w[4 * c4 + 1] * x.y + w[4 * c4 + 2] * x.z + w[4 * c4 + 3] * x.w;
    }
    sigma[v] = mask[v] * acc;
  }
}

constexpr int kTailVoxels = 256;

__global__ __launch_bounds__(256) void k_tail_bwd(const float* tpart, int nmb, int qa_pad,
                                                  const int* __restrict__ inv, const float* d0,
                                                  int C, const float* w, size_t V, float* gd0,
                                                  double* part, const float* gtv,
                                                  long long istride) {
  {
    const long long off = (long long)blockIdx.y * istride;
    tpart = ishift(tpart, off); d0 = ishift(d0, off); w = ishift(w, off);
    gd0 = ishift(gd0, off); part = ishift(part, off); gtv = ishift(gtv, off);
  }
  __shared__ float gsv[kTailVoxels];
  __shared__ double sh[256];
  const int tid = threadIdx.x;
  const size_t v0 = (size_t)blockIdx.x * kTailVoxels;
  {
    const size_t v = v0 + tid;
    float g = 0.f;
    if (v < V) {
      const int q = inv[v];
      if (q >= 0) {
        // eight row-group partials in flight, added in row-group order
        for (int k0 = 0; k0 < nmb; k0 += 8) {
          float t[8];
#pragma unroll
          for (int e = 0; e < 8; ++e)
            t[e] = k0 + e < nmb ? tpart[(size_t)(k0 + e) * qa_pad + q] : 0.f;
#pragma unroll
          for (int e = 0; e < 8; ++e) g += t[e];
        }
        if (gtv) g += gtv[v];  // the image is masked: d sigma / d out = mask
      }
    }
    gsv[tid] = g;
  }
  __syncthreads();
  // channel-major sweep: thread (c, r0) covers voxels r0, r0 + 256/C, ...
  const int c = tid % C, r0 = tid / C, rpi = 256 / C;
  const float wc = w[c];
  double s = 0.0;
  for (int r = r0; r < kTailVoxels; r += rpi) {
    const size_t v = v0 + r;
    if (v >= V) break;
    const float g = gsv[r];
    gd0[v * C + c] = g * wc;
    s += (double)g * d0[v * C + c];
  }
  sh[tid] = s;
  __syncthreads();
  const size_t pb = (size_t)blockIdx.x * (C + 1);
  if (tid < C) {
    double a = 0.0;
    for (int k = tid; k < 256; k += C) a += sh[k];
    part[pb + tid] = a;
  }
  __syncthreads();
  // bias partial: the block's voxel gradients, summed by the fixed wave
  // butterflies of block_sum
  const double a = block_sum((double)gsv[tid], sh);
  if (tid == 0) part[pb + C] = a;
}

__global__ void k_adam(float* theta, const float* g, float* m, float* v, size_t P, float lr,
                       float beta1, float beta2, float eps, IterState* it,
                       long long istride) {
  {
    const long long off = (long long)blockIdx.y * istride;
    theta = ishift(theta, off); g = ishift(g, off); m = ishift(m, off); v = ishift(v, off);
    it = ishift(it, off);
  }
  __shared__ float sbc[2];
  if (threadIdx.x == 0) {
    const int t = it->t + 1;
    sbc[0] = (float)(1.0 - pow((double)beta1, (double)t));
    sbc[1] = (float)(1.0 - pow((double)beta2, (double)t));
  }
  __syncthreads();
  const float bc1 = sbc[0], bc2 = sbc[1];
  const float step = lr / bc1;
  const float rs2 = 1.f / sqrtf(bc2);
  bool bad = false;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < P;
       i += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float th = theta[i] - step * mi / (sqrtf(vi) * rs2 + eps);
    theta[i] = th;
    bad |= !isfinite(th);
  }
  // a non-finite parameter raises the instance's flag (bit 1; bit 0 is the loss)
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(&it->nonfinite, 2);
}

__device__ __forceinline__ void put_bf(uint16_t* w, long long i, long long lo_off, float val) {
  const uint16_t hi = f2bf(val);
  w[i] = hi;
  if (lo_off) w[lo_off + i] = f2bf(val - bf2f(hi));
}

// p[0] + p[1] + ... + p[n-1], added in index order, with eight loads in
// flight (one thread).
__device__ __forceinline__ double ordered_sum(const double* p, int n) {
  double s = 0.0;
  int k = 0;
  for (; k + 8 <= n; k += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[k + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  double v[7];
#pragma unroll
  for (int u = 0; u < 7; ++u) v[u] = k + u < n ? p[k + u] : 0.0;
#pragma unroll
  for (int u = 0; u < 7; ++u)
    if (k + u < n) s += v[u];
  return s;
}

__global__ void k_pack_weights(const ConvPack* __restrict__ packs, const float* theta,
                               float* wf32, uint16_t* wbf16, long long lo_off, IterState* it,
                               const double* rsum, int nrs, int M, const double* tvsum, int ntv,
                               long long istride) {
  {
    const long long off = (long long)blockIdx.z * istride;
    theta = ishift(theta, off); wf32 = ishift(wf32, off); wbf16 = ishift(wbf16, off);
    it = ishift(it, off); rsum = ishift(rsum, off); tvsum = ishift(tvsum, off);
  }
  if (it && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    double L = ordered_sum(rsum, nrs);
    L /= M;
    const double R = ordered_sum(tvsum, ntv);
    L += R;
    it->loss = L;
    if (!isfinite(L)) it->nonfinite = 1;
    it->t = it->t + 1;
  }
  const ConvPack pk = packs[blockIdx.y];
  const int per_co = pk.cin_real * pk.taps;
  const int total = pk.cout * per_co;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int co = e / per_co;
    const int rem = e - co * per_co;
    const int ci = rem / pk.taps;
    const int tap = rem - ci * pk.taps;
    const float val = theta[pk.th_off + e];
    const long long fi = pk.wf_off + ((long long)co * pk.taps + tap) * pk.cin + ci;
    if (wf32) wf32[fi] = val;
    if (wbf16) put_bf(wbf16, fi, lo_off, val);
    if (pk.need_dgrad) {
      const long long di =
          pk.wd_off + ((long long)ci * pk.taps + (pk.taps - 1 - tap)) * pk.cout + co;
      if (wf32) wf32[di] = val;
      if (wbf16) put_bf(wbf16, di, lo_off, val);
    }
  }
}

// Dense J products of the standalone operators (J is M x Q row-major FP32,
// Q a multiple of 4).  p[m] = sum_q J[m][q] sigma[q]: one block per row,
// fixed-order block reduction.
__global__ __launch_bounds__(256) void k_jv_dense(const float* J, int M, int Q, const float* sig,
                                                  float* p) {
  __shared__ double sh[8];
  const float4* r = reinterpret_cast<const float4*>(J + (size_t)blockIdx.x * Q);
  const float4* s4 = reinterpret_cast<const float4*>(sig);
  float acc = 0.f;
  for (int q = threadIdx.x; q < Q / 4; q += 256) {
    const float4 a = r[q], b = s4[q];
    acc += a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;
  }
  const double t = block_sum((double)acc, sh);
  if (threadIdx.x == 0) p[blockIdx.x] = (float)t;
}

// part[rs][q] = sum over rows m = rs, rs + RS, ... of J[m][q] g[m] (4 columns
// per thread, rows in order); k_jt_sum adds the RS slices in order.
constexpr int kJtSlices = 8;
__global__ __launch_bounds__(256) void k_jt_dense(const float* J, int M, int Q, const float* g,
                                                  float* part) {
  const int q4 = blockIdx.x * 256 + threadIdx.x;
  if (q4 * 4 >= Q) return;
  const int rs = blockIdx.y;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int m = rs; m < M; m += kJtSlices) {
    const float4 j = reinterpret_cast<const float4*>(J + (size_t)m * Q)[q4];
    const float gm = g[m];
    acc.x += j.x * gm;
    acc.y += j.y * gm;
    acc.z += j.z * gm;
    acc.w += j.w * gm;
  }
  reinterpret_cast<float4*>(part + (size_t)rs * Q)[q4] = acc;
}

__global__ void k_jt_sum(const float* part, int Q, float* out) {
  const int q4 = blockIdx.x * 256 + threadIdx.x;
  if (q4 * 4 >= Q) return;
  float4 acc = reinterpret_cast<const float4*>(part)[q4];
  for (int rs = 1; rs < kJtSlices; ++rs) {
    const float4 v = reinterpret_cast<const float4*>(part + (size_t)rs * Q)[q4];
    acc.x += v.x;
    acc.y += v.y;
    acc.z += v.z;
    acc.w += v.w;
  }
  reinterpret_cast<float4*>(out)[q4] = acc;
}

// Data term of Eq. (4) in the mean-squared form: r = p - dv (FP32), loss =
// (1/M) sum r^2 accumulated in FP64 and reduced in one block in a fixed
// order, gp = (2/M) r.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ p,
                                             const float* __restrict__ dv, int M,
                                             float* __restrict__ gp, double* __restrict__ loss) {
  __shared__ double sh[4];
  double acc = 0.0;
  const float two_m = 2.f / (float)M;
  for (int m = threadIdx.x; m < M; m += 256) {
    const float r = p[m] - dv[m];
    acc += (double)r * (double)r;
    if (gp) gp[m] = two_m * r;
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) *loss = t / (double)M;
}

// 4D-TV of one image (Sec. III-E, Eqs. (11)-(13)), one thread per voxel.
// Spatial: q(v) = sqrt(dz^2 + dy^2 + dx^2 + eps) of the forward differences
// (0 where the neighbour is outside the grid); v's gradient collects -d/q(v)
// of its own differences and +d/q(u) of the differences of u = v - e that
// end at v.  Temporal: sum_k w_k sqrt((s - h_k)^2 + eps) over the history.
// Writes gtv[v] and one FP64 partial of lam * R per block (fixed order).
__device__ __forceinline__ float tv_q(const float* s, int z, int y, int x, int n, float eps) {
  const size_t v = ((size_t)z * n + y) * n + x;
  const float c = s[v];
  const float dz = z + 1 < n ? s[v + (size_t)n * n] - c : 0.f;
  const float dy = y + 1 < n ? s[v + n] - c : 0.f;
  const float dx = x + 1 < n ? s[v + 1] - c : 0.f;
  return sqrtf(dz * dz + dy * dy + dx * dx + eps);
}

__global__ __launch_bounds__(256) void k_tv(const float* sigma, int n, const float* hist,
                                            const TvState* ts, TvCoef c, float* gtv,
                                            double* tvsum, long long istride) {
  {
    const long long off = (long long)blockIdx.y * istride;
    sigma = ishift(sigma, off); hist = ishift(hist, off); ts = ishift(ts, off);
    gtv = ishift(gtv, off); tvsum = ishift(tvsum, off);
  }
  __shared__ double sh[8];
  const size_t V = (size_t)n * n * n;
  const size_t v = (size_t)blockIdx.x * 256 + threadIdx.x;
  double part = 0.0;
  if (v < V) {
    const int x = (int)(v % n), y = (int)((v / n) % n), z = (int)(v / ((size_t)n * n));
    const float s = sigma[v];
    const float dz = z + 1 < n ? sigma[v + (size_t)n * n] - s : 0.f;
    const float dy = y + 1 < n ? sigma[v + n] - s : 0.f;
    const float dx = x + 1 < n ? sigma[v + 1] - s : 0.f;
    const float q = sqrtf(dz * dz + dy * dy + dx * dx + c.eps);
    float gs = -(dz + dy + dx) / q;
    if (z > 0) gs += (s - sigma[v - (size_t)n * n]) / tv_q(sigma, z - 1, y, x, n, c.eps);
    if (y > 0) gs += (s - sigma[v - n]) / tv_q(sigma, z, y - 1, x, n, c.eps);
    if (x > 0) gs += (s - sigma[v - 1]) / tv_q(sigma, z, y, x - 1, n, c.eps);
    const float invV = 1.f / (float)V;
    float gt = 0.f;
    double rt = 0.0;
    const int cnt = ts->count, head = ts->head;
    for (int k = 1; k <= cnt; ++k) {
      const int slot = (head - k + 1 + kTvHistory) % kTvHistory;
      const float d = s - hist[(size_t)slot * V + v];
      const float qt = sqrtf(d * d + c.eps);
      gt += ts->w[k - 1] * (d / qt);
      rt += (double)ts->w[k - 1] * qt;
    }
    gtv[v] = c.lam * (c.lam_s * gs * invV + c.lam_t * gt);
    part = (double)c.lam * ((double)c.lam_s * q / (double)V + (double)c.lam_t * rt);
  }
  part = block_sum(part, sh);
  if (threadIdx.x == 0) tvsum[blockIdx.x] = part;
}

inline int grid_for(size_t work) {
  size_t b = (work + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

void gather_columns(const float* J, int M, int Q, const int* idx, int qa, int qa_pad, float* Jc,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_gather_columns, dim3(grid_for((size_t)M * qa_pad)), dim3(256), 0, s, J, M,
                     Q, idx, qa, qa_pad, Jc);
}

void jvec(const float* Jc, int M, int qa_pad, const int* idx, const float* sigma, float* ppart,
          int batch, long long istride, hipStream_t s) {
  dim3 grid(jvec_qblocks(qa_pad), (M + kJvecRows - 1) / kJvecRows);
  for (int b0 = 0; b0 < batch; b0 += kJMaxB)
    hipLaunchKernelGGL(k_jvec, grid, dim3(256),
                       (size_t)std::min(kJMaxB, batch - b0) * kJvecCols * sizeof(float), s, Jc,
                       M, qa_pad, idx,
                       ishift(sigma, b0 * istride), ishift(ppart, b0 * istride),
                       std::min(kJMaxB, batch - b0), istride);
}

void jtvec(const float* Jc, int M, int qa_pad, const float* ppart, int nqb, const float* dv,
           double* rsum, float* tpart, int batch, long long istride, hipStream_t s) {
  const int qb = (qa_pad / 4 + 255) / 256;
  const bool large = nqb > kJtFuseMax;
  const int rpg = jt_rows_per_group(M, qa_pad);
  for (int b0 = 0; b0 < batch; b0 += kJMaxB) {
    const int nb = std::min(kJMaxB, batch - b0);
    if (large) {
      hipLaunchKernelGGL(k_resid, dim3(jt_mblocks(M), nb), dim3(256), 0, s,
                         const_cast<float*>(ishift(ppart, b0 * istride)), nqb, M,
                         ishift(dv, b0 * istride), ishift(rsum, b0 * istride), istride);
      hipLaunchKernelGGL(k_jt_rows, dim3(qb, jt_partials(M, qa_pad)), dim3(256), 0, s, Jc, M,
                         qa_pad, ishift(ppart, b0 * istride), rpg, ishift(tpart, b0 * istride),
                         nb, istride);
    } else {
      hipLaunchKernelGGL(k_jtvec, dim3(qb, jt_mblocks(M)), dim3(256), 0, s, Jc, M, qa_pad,
                         ishift(ppart, b0 * istride), nqb, ishift(dv, b0 * istride),
                         ishift(rsum, b0 * istride), ishift(tpart, b0 * istride), nb, istride);
    }
  }
}

void tail_fwd(const float* d0, int C, const float* w, const float* b, const float* mask, size_t V,
              float* sigma, int batch, long long istride, hipStream_t s) {
  hipLaunchKernelGGL(k_tail_fwd, dim3(grid_for(V), batch), dim3(256), 0, s, d0, C, w, b, mask, V,
                     sigma, istride);
}

int tail_bwd_blocks(size_t V, int C) {
  (void)C;
  return (int)((V + kTailVoxels - 1) / kTailVoxels);
}

void tail_bwd(const float* tpart, int nmb, int qa_pad, const int* inv, const float* d0, int C,
              const float* w, size_t V, float* gd0, double* part, const float* gtv, int batch,
              long long istride, hipStream_t s) {
  hipLaunchKernelGGL(k_tail_bwd, dim3(tail_bwd_blocks(V, C), batch), dim3(256), 0, s, tpart, nmb,
                     qa_pad, inv, d0, C, w, V, gd0, part, gtv, istride);
}

void adam(float* theta, const float* g, float* m, float* v, size_t P, float lr, float beta1,
          float beta2, float eps, IterState* it, int batch, long long istride,
          hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(grid_for(P), batch), dim3(256), 0, s, theta, g, m, v, P, lr,
                     beta1, beta2, eps, it, istride);
}

void pack_weights(const ConvPack* packs, int npacks, int max_elems, const float* theta,
                  float* wf32, uint16_t* wbf16, long long lo_off, IterState* it,
                  const double* rsum, int nrs, int M, const double* tvsum, int ntv, int batch,
                  long long istride, hipStream_t s) {
  dim3 grid((max_elems + 255) / 256, npacks, batch);
  if (grid.x > 1024) grid.x = 1024;
  hipLaunchKernelGGL(k_pack_weights, grid, dim3(256), 0, s, packs, theta, wf32, wbf16, lo_off, it,
                     rsum, nrs, M, tvsum, ntv, istride);
}

void jv_dense(const float* J, int M, int Q, const float* sigma, float* p, hipStream_t s) {
  hipLaunchKernelGGL(k_jv_dense, dim3(M), dim3(256), 0, s, J, M, Q, sigma, p);
}

size_t jt_dense_scratch(int Q) { return (size_t)kJtSlices * Q; }

void mse_loss(const float* p, const float* dv, int M, float* gp, double* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, s, p, dv, M, gp, loss);
}

void jt_dense(const float* J, int M, int Q, const float* g, float* part, float* out,
              hipStream_t s) {
  const int bx = (Q / 4 + 255) / 256;
  hipLaunchKernelGGL(k_jt_dense, dim3(bx, kJtSlices), dim3(256), 0, s, J, M, Q, g, part);
  hipLaunchKernelGGL(k_jt_sum, dim3(bx), dim3(256), 0, s, part, Q, out);
}

int tv_blocks(size_t V) { return (int)((V + 255) / 256); }

void tv_reg(const float* sigma, int n, const float* hist, const TvState* ts, TvCoef c, float* gtv,
            double* tvsum, int batch, long long istride, hipStream_t s) {
  const size_t V = (size_t)n * n * n;
  hipLaunchKernelGGL(k_tv, dim3(tv_blocks(V), batch), dim3(256), 0, s, sigma, n, hist, ts, c, gtv,
                     tvsum, istride);
}

}  // namespace d2ip
