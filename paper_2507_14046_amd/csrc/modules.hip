// Output head and attention unit of the 3D-FastResUNet (Sec. III-D) on
// channels-last FP32 tensors, forward and backward.
//
// Head: t[v] = b + sum_c w[c] x[v][c] (a 1x1x1 convolution to one channel),
// out[v] = mask[v] * t[v] (linear) or mask[v] * (2 sigmoid(t[v]) - 1) (the
// sigmoid tail scaled to (-1, 1)).  One thread per voxel, float4 rows.
//
// Attention unit of a decoder stage (attention, then interpolation): the
// skip x [n^3][c] is gated by coefficients formed on the grid of the coarser
// decoder output g [(n/2)^3][cu]:
//   xs[u] = mean of x over the 8 children of coarse voxel u,
//   a[u][k] = b[k] + sum_j wx[k][j] xs[u][j] + sum_j wg[k][j] g[u][j],
//   alpha[u] = sigmoid(bpsi + sum_k psi[k] relu(a[u][k])),
//   y[v] = alpha[parent(v)] x[v].
// Both products with weights (the pre-activations a = [xs, g] W^T and, in
// the backward, the weight gradient and the gradients of xs and g) run on the
// matrix cores; the children's x and gy quads stay in registers from the
// pooling to the output, so each tensor crosses HBM once.  Parameter
// gradients are accumulated per block and reduced in FP64 in a fixed order
// (deterministic).
//
// Channel slices and ReLU: the ASPP's concatenation of its branches (each
// branch copied into its channel range of the concatenated tensor, and the
// gradient's ranges copied back out) and its output activation.
#include <algorithm>

#include "kernels.h"

namespace d2ip {
namespace {

// ---- head -------------------------------------------------------------------

__device__ __forceinline__ float head_t(const float* __restrict__ x, const float* __restrict__ w,
                                        float b, int C, size_t v) {
  const float4* r = reinterpret_cast<const float4*>(x + v * C);
  const float4* w4 = reinterpret_cast<const float4*>(w);
  float t = b;
  for (int q = 0; q < C / 4; ++q) {
    const float4 a = r[q], c = w4[q];
    t += a.x * c.x + a.y * c.y + a.z * c.z + a.w * c.w;
  }
  return t;
}

__global__ __launch_bounds__(256) void k_head_fwd(const float* __restrict__ x,
                                                  const float* __restrict__ w,
                                                  const float* __restrict__ b,
                                                  const float* __restrict__ mask, size_t V, int C,
                                                  int sig, float* __restrict__ out) {
  for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < V;
       v += (size_t)gridDim.x * blockDim.x) {
    const float t = head_t(x, w, b[0], C, v);
    float o = sig ? 2.f / (1.f + expf(-t)) - 1.f : t;
    if (mask) o *= mask[v];
    out[v] = o;
  }
}

// ---- fixed-order column sums ----------------------------------------------

constexpr int kColSlices = 32;

// Stage 1 of out[i] = sum_k part[k][i] (k < nrows, i < ncols): slice s of the
// rows (contiguous, S slices) is summed per column in FP64 by four row lanes
// (rows r0 + l, r0 + l + 4, ...) whose sums are then added in lane order.
// Grid (ceil(ncols / 64), S), 256 threads.
template <class T>
__global__ __launch_bounds__(256) void k_colsum1(const T* __restrict__ part, int nrows, int ncols,
                                                 double* __restrict__ tmp) {
  __shared__ double red[4][64];
  const int cl = threadIdx.x & 63, ln = threadIdx.x >> 6;
  const int col = blockIdx.x * 64 + cl;
  const int S = gridDim.y, sl = blockIdx.y;
  const int r0 = (int)((long long)nrows * sl / S), r1 = (int)((long long)nrows * (sl + 1) / S);
  double acc = 0.0;
  if (col < ncols)
    for (int k0 = r0 + ln; k0 < r1; k0 += 32) {
      // eight loads in flight, then added in row order
      double v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = k0 + 4 * e;
        v[e] = k < r1 ? (double)part[(size_t)k * ncols + col] : 0.0;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) acc += v[e];
    }
  red[ln][cl] = acc;
  __syncthreads();
  if (ln == 0 && col < ncols)
    tmp[(size_t)sl * ncols + col] = ((red[0][cl] + red[1][cl]) + red[2][cl]) + red[3][cl];
}

// Output tensors of a column sum: column i lands in dst[j][i - start[j]] for
// start[j] <= i < start[j + 1] (a null dst[j] drops its columns).
struct ColOut {
  float* dst[5];
  int start[6];
  int nseg;
};

// Stage 2: the S slice sums of every column added in slice order.
__global__ __launch_bounds__(256) void k_colsum2(const double* __restrict__ tmp, int S, int ncols,
                                                 ColOut o) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncols) return;
  // every slice's load in flight, then added in slice order (S <= kColSlices)
  double v[kColSlices];
#pragma unroll
  for (int k = 0; k < kColSlices; ++k) v[k] = k < S ? tmp[(size_t)k * ncols + i] : 0.0;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kColSlices; ++k) s += v[k];
  for (int j = 0; j < o.nseg; ++j)
    if (i >= o.start[j] && i < o.start[j + 1]) {
      if (o.dst[j]) o.dst[j][i - o.start[j]] = (float)s;
      break;
    }
}

int colsum_slices(int nrows) { return nrows < kColSlices ? nrows : kColSlices; }

template <class T>
void colsum(const T* part, int nrows, int ncols, double* tmp, const ColOut& o, hipStream_t s) {
  const int S = colsum_slices(nrows);
  hipLaunchKernelGGL(k_colsum1<T>, dim3((ncols + 63) / 64, S), dim3(256), 0, s, part, nrows,
                     ncols, tmp);
  hipLaunchKernelGGL(k_colsum2, dim3((ncols + 255) / 256), dim3(256), 0, s, tmp, S, ncols, o);
}

// ---- head backward ----------------------------------------------------------

// gt[v] = gout[v] mask[v] dout/dt; gx[v][c] = gt w[c]; one FP64 partial per
// block of (sum_v gt x[v][c], sum_v gt).  A block walks chunks of 256 voxels
// (chunk k, k + gridDim, ...): each thread forms one voxel's gt into LDS, then
// thread (q, r) takes channel quad q of voxels r, r + R, ... (R = 256 / (C/4)),
// coalesced rows; the R row lanes are added in lane order at the end.
constexpr int kHeadMaxC = 256;
constexpr int kHeadChunk = 256;
__global__ __launch_bounds__(256) void k_head_bwd(const float* __restrict__ x,
                                                  const float* __restrict__ w,
                                                  const float* __restrict__ b,
                                                  const float* __restrict__ mask,
                                                  const float* __restrict__ gout, size_t V, int C,
                                                  int sig, float* __restrict__ gx,
                                                  double* __restrict__ part) {
  __shared__ float gts[kHeadChunk];
  __shared__ double red[256][5];
  const int C4 = C / 4;
  const int R = 256 / C4, q = threadIdx.x % C4, r = threadIdx.x / C4;
  const float4 wq = reinterpret_cast<const float4*>(w)[q];
  double acc[4] = {0.0, 0.0, 0.0, 0.0}, accb = 0.0;
  for (size_t c0 = (size_t)blockIdx.x * kHeadChunk; c0 < V; c0 += (size_t)gridDim.x * kHeadChunk) {
    const int nv = (int)min((size_t)kHeadChunk, V - c0);
    if ((int)threadIdx.x < nv) {
      const size_t v = c0 + threadIdx.x;
      float gt = gout[v];
      if (mask) gt *= mask[v];
      if (sig) {
        const float sg = 1.f / (1.f + expf(-head_t(x, w, b[0], C, v)));
        gt *= 2.f * sg * (1.f - sg);
      }
      gts[threadIdx.x] = gt;
    }
    __syncthreads();
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
    float ab = 0.f;
    for (int rr = r; rr < nv; rr += R) {
      const size_t v = c0 + rr;
      const float gt = gts[rr];
      const float4 xv = reinterpret_cast<const float4*>(x + v * C)[q];
      a.x += gt * xv.x;
      a.y += gt * xv.y;
      a.z += gt * xv.z;
      a.w += gt * xv.w;
      ab += gt;
      if (gx)
        reinterpret_cast<float4*>(gx + v * C)[q] =
            make_float4(gt * wq.x, gt * wq.y, gt * wq.z, gt * wq.w);
    }
    acc[0] += a.x;
    acc[1] += a.y;
    acc[2] += a.z;
    acc[3] += a.w;
    accb += ab;
    __syncthreads();  // gts is refilled by the next chunk
  }
  for (int e = 0; e < 4; ++e) red[threadIdx.x][e] = acc[e];
  red[threadIdx.x][4] = accb;
  __syncthreads();
  if ((int)threadIdx.x < C4) {
    double sm[4] = {0.0, 0.0, 0.0, 0.0}, sb = 0.0;
    for (int rr = 0; rr < R; ++rr) {
      const int t = rr * C4 + threadIdx.x;
      for (int e = 0; e < 4; ++e) sm[e] += red[t][e];
      sb += red[t][4];
    }
    double* p = part + (size_t)blockIdx.x * (C + 1);
    for (int e = 0; e < 4; ++e) p[4 * threadIdx.x + e] = sm[e];
    if (threadIdx.x == 0) p[C] = sb;
  }
}

// ---- attention unit ---------------------------------------------------------
//
// A tile is kAttU = 64 coarse voxels (four row tiles of 16, one per wave).
// LDS (sized per launch): Z [u][0, c) the pooled skip rows and Z [u][c, K)
// the gating rows (K = c + cu; zero past the tile's voxels and up to K16, the
// next multiple of 16); W [k][j] = [wx[k][:], wg[k][:]] staged once per
// block with the same row stride.  The matrix-core step is
// v_mfma_f32_16x16x4f32: lane l = l16 + 16 g supplies A[row l16][slot g] and
// B[slot g][col l16] and receives D[row 4 g + i][col l16] in register i.

constexpr int kAttU = 64;
constexpr int kAttMaxC = 64;   // skip channels
constexpr int kAttMaxCu = 128; // gating channels

struct AttArgs {
  const float *x, *g, *wx, *wg, *b, *psi, *bpsi;
  int n, c, cu;
};

// LDS layout in floats (every offset a multiple of 4).
struct AttLds {
  int K16, Zs, Ap, Pp;
  int z, w, a, pd, al, gt, red, total;
};

__host__ __device__ inline AttLds att_lds(int c, int cu, bool bwd) {
  AttLds L;
  L.K16 = (c + cu + 15) & ~15;
  L.Zs = L.K16 + 4;
  L.Ap = c + 4;
  L.Pp = c / 4 + 1;
  int o = 0;
  L.z = o;
  o += kAttU * L.Zs;
  L.w = o;
  o += c * L.Zs;
  L.a = o;
  o += bwd ? kAttU * L.Ap : 0;
  L.pd = o;
  o += bwd ? kAttU * L.Pp : 0;
  L.al = o;
  o += kAttU;
  L.gt = o;
  o += bwd ? kAttU : 0;
  L.red = o;
  o += bwd ? 512 : 0;
  L.total = o;
  return L;
}

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float comp4(const float4& v, int s) {
  return s == 0 ? v.x : s == 1 ? v.y : s == 2 ? v.z : v.w;
}

// Offset (floats) of child ch (0..7, bits z y x) of coarse voxel uc.
__device__ __forceinline__ size_t att_child(const AttArgs& A, int uc, int ch) {
  const int m = A.n / 2;
  const int xx = uc % m, yy = (uc / m) % m, zz = uc / (m * m);
  const int fz = 2 * zz + (ch >> 2), fy = 2 * yy + ((ch >> 1) & 1), fx = 2 * xx + (ch & 1);
  return ((size_t)(fz * A.n + fy) * A.n + fx) * A.c;
}

// W into LDS: Ws [k][j] for k < c, j < K16 (zero for j >= K).
__device__ __forceinline__ void att_stage_w(const AttArgs& A, const AttLds& L, float* Ws) {
  const int w4 = L.K16 / 4;
  for (int it = threadIdx.x; it < A.c * w4; it += blockDim.x) {
    const int k = it / w4, j0 = 4 * (it - k * w4);
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (j0 < A.c)
      v = *reinterpret_cast<const float4*>(A.wx + (size_t)k * A.c + j0);
    else if (j0 < A.c + A.cu)
      v = *reinterpret_cast<const float4*>(A.wg + (size_t)k * A.cu + (j0 - A.c));
    *reinterpret_cast<float4*>(Ws + k * L.Zs + j0) = v;
  }
}

// Gating rows (and zero padding) of the tile into Z [u][c, K16).
__device__ __forceinline__ void att_stage_g(const AttArgs& A, const AttLds& L, int u0, int nu,
                                            float* Z) {
  const int w4 = (L.K16 - A.c) / 4;
  for (int it = threadIdx.x; it < kAttU * w4; it += blockDim.x) {
    const int u = it / w4, j0 = A.c + 4 * (it - u * w4);
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (u < nu && j0 < A.c + A.cu)
      v = *reinterpret_cast<const float4*>(A.g + (size_t)(u0 + u) * A.cu + (j0 - A.c));
    *reinterpret_cast<float4*>(Z + u * L.Zs + j0) = v;
  }
}

// a [u][k] = b[k] + sum_j Z[u][j] W[k][j] for the wave's rows u = 16 w ..
// 16 w + 15 (into As when given), and alpha[u] = sigmoid(bpsi + sum_k psi[k]
// relu(a[u][k])) into al: each column tile's psi-weighted terms are added over
// its 16 lanes by a butterfly, the tiles in order, and lane 16 g keeps the sums
// of rows 4 g .. 4 g + 3.
__device__ __forceinline__ void att_preact_alpha(const AttArgs& A, const AttLds& L, const float* Z,
                                                 const float* Ws, float* As, float* al) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, g = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  float sacc[4] = {0.f, 0.f, 0.f, 0.f};
  for (int nt = 0; nt * 16 < A.c; ++nt) {
    const int k = 16 * nt + l16;
    const bool kin = k < A.c;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k16 = 0; k16 < L.K16; k16 += 16) {
      const float4 a = *reinterpret_cast<const float4*>(Z + (16 * wave + l16) * L.Zs + k16 + 4 * g);
      float4 bw = make_float4(0.f, 0.f, 0.f, 0.f);
      if (kin) bw = *reinterpret_cast<const float4*>(Ws + k * L.Zs + k16 + 4 * g);
#pragma unroll
      for (int s = 0; s < 4; ++s) acc = mfma4(comp4(a, s), comp4(bw, s), acc);
    }
    const float bk = kin ? A.b[k] : 0.f, pk = kin ? A.psi[k] : 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float av = acc[i] + bk;
      if (As && kin) As[(16 * wave + 4 * g + i) * L.Ap + k] = av;
      float v = pk * fmaxf(av, 0.f);
      v += __shfl_xor(v, 8, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 1, 64);
      sacc[i] += v;
    }
  }
  if (l16 == 0) {
    const float bp = A.bpsi[0];
#pragma unroll
    for (int i = 0; i < 4; ++i) al[16 * wave + 4 * g + i] = 1.f / (1.f + expf(-(bp + sacc[i])));
  }
}

// Forward.  ITEMS = ceil(c / 16): a thread owns items it = tid + 256 i
// (coarse voxel u = it / (c/4), channel quad q), whose eight children's x
// quads it keeps in registers from the pooling to the output.
template <int ITEMS>
__global__ __launch_bounds__(256) void k_att_fwd(AttArgs A, int ntiles, float* __restrict__ y,
                                                 float* __restrict__ alpha) {
  extern __shared__ __align__(16) float smem[];
  const AttLds L = att_lds(A.c, A.cu, false);
  float *Z = smem + L.z, *Ws = smem + L.w, *al = smem + L.al;
  const int c4 = A.c / 4;
  const int m = A.n / 2, mc = m * m * m;
  att_stage_w(A, L, Ws);
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int u0 = tile * kAttU, nu = min(kAttU, mc - u0);
    float4 xr[ITEMS][8];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int it = threadIdx.x + 256 * i, u = it / c4, q = it - u * c4;
      if (it >= kAttU * c4) continue;
      float4 sm = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int ch = 0; ch < 8; ++ch) {
        xr[i][ch] = u < nu ? reinterpret_cast<const float4*>(A.x + att_child(A, u0 + u, ch))[q]
                           : make_float4(0.f, 0.f, 0.f, 0.f);
        sm.x += xr[i][ch].x;
        sm.y += xr[i][ch].y;
        sm.z += xr[i][ch].z;
        sm.w += xr[i][ch].w;
      }
      *reinterpret_cast<float4*>(Z + u * L.Zs + 4 * q) =
          make_float4(0.125f * sm.x, 0.125f * sm.y, 0.125f * sm.z, 0.125f * sm.w);
    }
    att_stage_g(A, L, u0, nu, Z);
    __syncthreads();
    att_preact_alpha(A, L, Z, Ws, nullptr, al);
    __syncthreads();
    if (alpha && (int)threadIdx.x < nu) alpha[u0 + threadIdx.x] = al[threadIdx.x];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int it = threadIdx.x + 256 * i, u = it / c4, q = it - u * c4;
      if (it >= kAttU * c4 || u >= nu) continue;
      const float a = al[u];
#pragma unroll
      for (int ch = 0; ch < 8; ++ch)
        reinterpret_cast<float4*>(y + att_child(A, u0 + u, ch))[q] =
            make_float4(a * xr[i][ch].x, a * xr[i][ch].y, a * xr[i][ch].z, a * xr[i][ch].w);
    }
    __syncthreads();  // Z and al are refilled by the next tile
  }
}

// Parameter-gradient partial layout per block: wx [c][c], wg [c][cu], b [c],
// psi [c], bpsi [1].
__host__ __device__ inline int att_nparams(int c, int cu) { return c * c + c * cu + 2 * c + 1; }

// Backward of a block's tiles (tile k, k + gridDim, ...): the same items as
// the forward keep the children's gy quads in registers; dL/dalpha[u] is the
// sum of gy x over the children, added per quad and then over the quads in
// order.  ga [u][k] = psi[k] gt[u] where a > 0; the psi, b and bpsi sums run
// over fixed voxel subsets per thread, combined in order.  The weight
// gradient gW [k][j] += sum_u ga[u][k] Z[u][j] accumulates over the block's
// tiles in the matrix-core registers (wave w: column tiles w, w + 4, w + 8);
// the pooled and gating gradients gZ [u][j] = sum_k ga[u][k] W[k][j] (wave w:
// rows 16 w ..) give gg directly and gx = alpha gy + gZ[u][j] / 8.
template <int ITEMS>
__global__ __launch_bounds__(256) void k_att_bwd(AttArgs A, int ntiles, const float* __restrict__ gy,
                                                 float* __restrict__ gx, float* __restrict__ gg,
                                                 float* __restrict__ part) {
  extern __shared__ __align__(16) float smem[];
  const AttLds L = att_lds(A.c, A.cu, true);
  float *Z = smem + L.z, *Ws = smem + L.w, *As = smem + L.a, *Pd = smem + L.pd;
  float *al = smem + L.al, *gt = smem + L.gt, *red = smem + L.red;
  const int c = A.c, c4 = c / 4, K = c + A.cu;
  const int m = A.n / 2, mc = m * m * m;
  const int lane = threadIdx.x & 63, l16 = lane & 15, g = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int MT = (c + 15) / 16;  // row tiles of gW (k)
  const int NL = 256 / c;        // voxel lanes of the psi and b sums
  f32x4 gw[4][3];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int t = 0; t < 3; ++t) gw[mt][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float acc_psi = 0.f, acc_b = 0.f, acc_bpsi = 0.f;
  att_stage_w(A, L, Ws);
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int u0 = tile * kAttU, nu = min(kAttU, mc - u0);
    float4 gr[ITEMS][8];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int it = threadIdx.x + 256 * i, u = it / c4, q = it - u * c4;
      if (it >= kAttU * c4) continue;
      float4 sm = make_float4(0.f, 0.f, 0.f, 0.f);
      float d = 0.f;
#pragma unroll
      for (int ch = 0; ch < 8; ++ch) {
        float4 xv = make_float4(0.f, 0.f, 0.f, 0.f);
        gr[i][ch] = xv;
        if (u < nu) {
          const size_t o = att_child(A, u0 + u, ch);
          xv = reinterpret_cast<const float4*>(A.x + o)[q];
          gr[i][ch] = reinterpret_cast<const float4*>(gy + o)[q];
        }
        sm.x += xv.x;
        sm.y += xv.y;
        sm.z += xv.z;
        sm.w += xv.w;
        d += gr[i][ch].x * xv.x + gr[i][ch].y * xv.y + gr[i][ch].z * xv.z + gr[i][ch].w * xv.w;
      }
      *reinterpret_cast<float4*>(Z + u * L.Zs + 4 * q) =
          make_float4(0.125f * sm.x, 0.125f * sm.y, 0.125f * sm.z, 0.125f * sm.w);
      Pd[u * L.Pp + q] = d;
    }
    att_stage_g(A, L, u0, nu, Z);
    __syncthreads();
    att_preact_alpha(A, L, Z, Ws, As, al);
    __syncthreads();
    if ((int)threadIdx.x < kAttU) {
      const int u = threadIdx.x;
      float t = 0.f;
      if (u < nu) {
        float d = 0.f;
        for (int q = 0; q < c4; ++q) d += Pd[u * L.Pp + q];
        const float a = al[u];
        t = d * a * (1.f - a);  // through the sigmoid
      }
      gt[u] = t;
    }
    __syncthreads();
    // psi (relu(a) gt), then ga in place and b; voxel lane l takes u = l, l + NL, ...
    if ((int)threadIdx.x < c * NL) {
      const int k = threadIdx.x % c, l = threadIdx.x / c;
      const float pk = A.psi[k];
      float sp = 0.f, sb = 0.f;
      for (int u = l; u < kAttU; u += NL) {
        const float av = As[u * L.Ap + k], tu = gt[u];
        const bool in = u < nu;
        if (in) sp += fmaxf(av, 0.f) * tu;
        const float ga = (in && av > 0.f) ? pk * tu : 0.f;  // ReLU derivative 0 at 0
        sb += ga;
        As[u * L.Ap + k] = ga;
      }
      red[l * c + k] = sp;
      red[256 + l * c + k] = sb;
    }
    if (wave == 0) {
      float v = lane < nu ? gt[lane] : 0.f;
      v = wave_sum(v);
      if (lane == 0) acc_bpsi += v;
    }
    __syncthreads();
    if ((int)threadIdx.x < c) {
      float sp = 0.f, sb = 0.f;
      for (int l = 0; l < NL; ++l) {
        sp += red[l * c + threadIdx.x];
        sb += red[256 + l * c + threadIdx.x];
      }
      acc_psi += sp;
      acc_b += sb;
    }
    // gW [k][j] += sum_u ga[u][k] Z[u][j]: slot g of step u4 is voxel u4 + g
    for (int u4 = 0; u4 < kAttU; u4 += 4) {
      float av[4], bv[3];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        const int k = 16 * mt + l16;
        av[mt] = (mt < MT && k < c) ? As[(u4 + g) * L.Ap + k] : 0.f;
      }
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const int jt = wave + 4 * t;
        bv[t] = 16 * jt < L.K16 ? Z[(u4 + g) * L.Zs + 16 * jt + l16] : 0.f;
      }
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int t = 0; t < 3; ++t)
          if (mt < MT && 16 * (wave + 4 * t) < L.K16) gw[mt][t] = mfma4(av[mt], bv[t], gw[mt][t]);
    }
    __syncthreads();  // Z is overwritten below
    // gZ [u][j] = sum_k ga[u][k] W[k][j] for the wave's 16 rows
    for (int jt = 0; 16 * jt < K; ++jt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      const int j = 16 * jt + l16;
      for (int k4 = 0; k4 < c4; ++k4)
        acc = mfma4(As[(16 * wave + l16) * L.Ap + 4 * k4 + g], Ws[(4 * k4 + g) * L.Zs + j], acc);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int u = 16 * wave + 4 * g + i;
        if (j < c) {
          Z[u * L.Zs + j] = 0.125f * acc[i];
        } else if (j < K && u < nu && gg) {
          gg[(size_t)(u0 + u) * A.cu + (j - c)] = acc[i];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int it = threadIdx.x + 256 * i, u = it / c4, q = it - u * c4;
      if (it >= kAttU * c4 || u >= nu || !gx) continue;
      const float a = al[u];
      const float4 p = *reinterpret_cast<const float4*>(Z + u * L.Zs + 4 * q);
#pragma unroll
      for (int ch = 0; ch < 8; ++ch)
        reinterpret_cast<float4*>(gx + att_child(A, u0 + u, ch))[q] =
            make_float4(a * gr[i][ch].x + p.x, a * gr[i][ch].y + p.y, a * gr[i][ch].z + p.z,
                        a * gr[i][ch].w + p.w);
    }
    __syncthreads();  // Z, As, Pd, al, gt and red are refilled by the next tile
  }
  float* P = part + (size_t)blockIdx.x * att_nparams(c, A.cu);
  const int o_wg = c * c, o_b = o_wg + c * A.cu, o_psi = o_b + c, o_bpsi = o_psi + c;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int jt = wave + 4 * t, j = 16 * jt + l16;
      if (mt >= MT || 16 * jt >= L.K16 || j >= K) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = 16 * mt + 4 * g + i;
        if (k < c) P[j < c ? k * c + j : o_wg + k * A.cu + (j - c)] = gw[mt][t][i];
      }
    }
  if ((int)threadIdx.x < c) {
    P[o_b + threadIdx.x] = acc_b;
    P[o_psi + threadIdx.x] = acc_psi;
  }
  if (threadIdx.x == 0) P[o_bpsi] = acc_bpsi;
}

// ---- attention unit, wide channels -------------------------------------------
//
// Skip channels above kAttMaxC or gating channels above kAttMaxCu: the unit
// is composed from pieces that scale with the channel counts.  Z [u][K]
// (K = c + cu) holds the pooled skip and the gating rows, Wcat [c][K] the
// weights [wx | wg]; a = Z Wcat^T + b and, in the backward, gW = ga^T Z and
// gZ = ga Wcat run on the pointwise matrix-core GEMM; the gate, the scaling
// and their gradients are the kernels below.  One wave per coarse voxel where
// a voxel's values are summed (butterfly, lane 0's result), so every result
// is run-to-run identical.

// Z [u][0, c) = mean of x over the 8 children of u, Z [u][c, K) = g [u].
__global__ __launch_bounds__(256) void k_attw_stage(const float* __restrict__ x,
                                                    const float* __restrict__ g, int n, int c,
                                                    int cu, float* __restrict__ Z) {
  const int m = n / 2, K4 = (c + cu) / 4, c4 = c / 4;
  const size_t total = (size_t)m * m * m * K4;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t u = i / K4;
    const int q = (int)(i - u * K4);
    float4 v;
    if (q < c4) {
      const int xx = (int)(u % m), yy = (int)((u / m) % m), zz = (int)(u / ((size_t)m * m));
      float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int ch = 0; ch < 8; ++ch) {
        const int fz = 2 * zz + (ch >> 2), fy = 2 * yy + ((ch >> 1) & 1), fx = 2 * xx + (ch & 1);
        const float4 a =
            reinterpret_cast<const float4*>(x + ((size_t)(fz * n + fy) * n + fx) * c)[q];
        s.x += a.x;
        s.y += a.y;
        s.z += a.z;
        s.w += a.w;
      }
      v = make_float4(0.125f * s.x, 0.125f * s.y, 0.125f * s.z, 0.125f * s.w);
    } else {
      v = reinterpret_cast<const float4*>(g + u * cu)[q - c4];
    }
    reinterpret_cast<float4*>(Z + u * (size_t)(c + cu))[q] = v;
  }
}

// Wcat [k][K] = [wx [k][:], wg [k][:]].
__global__ void k_attw_catw(const float* __restrict__ wx, const float* __restrict__ wg, int c,
                            int cu, float* __restrict__ W) {
  const int K = c + cu;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < c * K; i += gridDim.x * blockDim.x) {
    const int k = i / K, j = i - k * K;
    W[i] = j < c ? wx[k * c + j] : wg[k * cu + (j - c)];
  }
}

// al[u] = sigmoid(bpsi + sum_k psi[k] relu(a[u][k])): wave per coarse voxel.
__global__ __launch_bounds__(256) void k_attw_gate(const float* __restrict__ a,
                                                   const float* __restrict__ psi,
                                                   const float* __restrict__ bpsi, size_t Vc,
                                                   int c, float* __restrict__ al,
                                                   float* __restrict__ alpha) {
  const int lane = threadIdx.x & 63;
  const size_t w0 = blockIdx.x * (size_t)4 + (threadIdx.x >> 6);
  for (size_t u = w0; u < Vc; u += (size_t)gridDim.x * 4) {
    float s = 0.f;
    for (int k = lane; k < c; k += 64) s += psi[k] * fmaxf(a[u * c + k], 0.f);
    s = wave_sum(s);
    if (lane == 0) {
      const float v = 1.f / (1.f + expf(-(bpsi[0] + s)));
      al[u] = v;
      if (alpha) alpha[u] = v;
    }
  }
}

// y[v] = al[parent(v)] x[v] (float4 quads).
__global__ __launch_bounds__(256) void k_attw_scale(const float* __restrict__ x,
                                                    const float* __restrict__ al, int n, int c,
                                                    float* __restrict__ y) {
  const int c4 = c / 4, m = n / 2;
  const size_t total = (size_t)n * n * n * c4;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t v = i / c4;
    const int fx = (int)(v % n), fy = (int)((v / n) % n), fz = (int)(v / ((size_t)n * n));
    const float a = al[((size_t)(fz / 2) * m + fy / 2) * m + fx / 2];
    const float4 t = reinterpret_cast<const float4*>(x)[i];
    reinterpret_cast<float4*>(y)[i] = make_float4(a * t.x, a * t.y, a * t.z, a * t.w);
  }
}

// gt[u] = (sum over the children and channels of gy x) al (1 - al): wave per
// coarse voxel, lanes over (child, quad) items.
__global__ __launch_bounds__(256) void k_attw_gdot(const float* __restrict__ x,
                                                   const float* __restrict__ gy,
                                                   const float* __restrict__ al, int n, int c,
                                                   float* __restrict__ gt) {
  const int lane = threadIdx.x & 63, c4 = c / 4, m = n / 2;
  const size_t Vc = (size_t)m * m * m;
  const size_t w0 = blockIdx.x * (size_t)4 + (threadIdx.x >> 6);
  for (size_t u = w0; u < Vc; u += (size_t)gridDim.x * 4) {
    const int xx = (int)(u % m), yy = (int)((u / m) % m), zz = (int)(u / ((size_t)m * m));
    float s = 0.f;
    for (int it = lane; it < 8 * c4; it += 64) {
      const int ch = it / c4, q = it - ch * c4;
      const int fz = 2 * zz + (ch >> 2), fy = 2 * yy + ((ch >> 1) & 1), fx = 2 * xx + (ch & 1);
      const size_t o = ((size_t)(fz * n + fy) * n + fx) * c;
      const float4 a = reinterpret_cast<const float4*>(x + o)[q];
      const float4 b = reinterpret_cast<const float4*>(gy + o)[q];
      s += a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;
    }
    s = wave_sum(s);
    if (lane == 0) {
      const float a = al[u];
      gt[u] = s * a * (1.f - a);
    }
  }
}

// ga[u][k] = psi[k] gt[u] where a[u][k] > 0 (else 0); one FP64 partial per
// block of (sum_u relu(a[u][k]) gt[u] for every k, sum_u gt[u]): thread
// (quad q, row lane r) takes rows r, r + R, ... of the block's chunk of
// kAttwRows coarse voxels, the row lanes added in lane order at the end.
constexpr int kAttwRows = 256;
__global__ __launch_bounds__(256) void k_attw_gate_bwd(const float* __restrict__ a,
                                                       const float* __restrict__ psi,
                                                       const float* __restrict__ gt, size_t Vc,
                                                       int c, float* __restrict__ ga,
                                                       double* __restrict__ part) {
  __shared__ double red[256][5];
  const int c4 = c / 4, R = 256 / c4, q = threadIdx.x % c4, r = threadIdx.x / c4;
  const float4 pq = reinterpret_cast<const float4*>(psi)[q];
  double acc[4] = {0.0, 0.0, 0.0, 0.0}, accb = 0.0;
  for (size_t u0 = blockIdx.x * (size_t)kAttwRows; u0 < Vc; u0 += (size_t)gridDim.x * kAttwRows) {
    const int nu = (int)min((size_t)kAttwRows, Vc - u0);
    if (r < R)
      for (int rr = r; rr < nu; rr += R) {
        const size_t u = u0 + rr;
        const float t = gt[u];
        const float4 av = reinterpret_cast<const float4*>(a + u * c)[q];
        acc[0] += (double)(fmaxf(av.x, 0.f) * t);
        acc[1] += (double)(fmaxf(av.y, 0.f) * t);
        acc[2] += (double)(fmaxf(av.z, 0.f) * t);
        acc[3] += (double)(fmaxf(av.w, 0.f) * t);
        if (q == 0) accb += (double)t;
        reinterpret_cast<float4*>(ga + u * c)[q] =
            make_float4(av.x > 0.f ? pq.x * t : 0.f, av.y > 0.f ? pq.y * t : 0.f,
                        av.z > 0.f ? pq.z * t : 0.f, av.w > 0.f ? pq.w * t : 0.f);
      }
  }
  for (int e = 0; e < 4; ++e) red[threadIdx.x][e] = acc[e];
  red[threadIdx.x][4] = accb;
  __syncthreads();
  if ((int)threadIdx.x < c4) {
    double sm[4] = {0.0, 0.0, 0.0, 0.0}, sb = 0.0;
    for (int rr = 0; rr < R; ++rr) {
      const int t = rr * c4 + threadIdx.x;
      for (int e = 0; e < 4; ++e) sm[e] += red[t][e];
      sb += red[t][4];
    }
    double* p = part + (size_t)blockIdx.x * (c + 1);
    for (int e = 0; e < 4; ++e) p[4 * threadIdx.x + e] = sm[e];
    if (threadIdx.x == 0) p[c] = sb;
  }
}

// gx[v] = al[parent(v)] gy[v] + gZ[parent(v)][0, c) / 8.
__global__ __launch_bounds__(256) void k_attw_scale_bwd(const float* __restrict__ gy,
                                                        const float* __restrict__ al,
                                                        const float* __restrict__ gZ, int n,
                                                        int c, int K, float* __restrict__ gx) {
  const int c4 = c / 4, m = n / 2;
  const size_t total = (size_t)n * n * n * c4;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t v = i / c4;
    const int q = (int)(i - v * c4);
    const int fx = (int)(v % n), fy = (int)((v / n) % n), fz = (int)(v / ((size_t)n * n));
    const size_t u = ((size_t)(fz / 2) * m + fy / 2) * m + fx / 2;
    const float a = al[u];
    const float4 t = reinterpret_cast<const float4*>(gy)[i];
    const float4 z = reinterpret_cast<const float4*>(gZ + u * K)[q];
    reinterpret_cast<float4*>(gx)[i] = make_float4(a * t.x + 0.125f * z.x, a * t.y + 0.125f * z.y,
                                                   a * t.z + 0.125f * z.z, a * t.w + 0.125f * z.w);
  }
}

// ---- channel slices, ReLU ---------------------------------------------------

// dst[v][doff + j] = src[v][soff + j] for j < c (all counts and offsets
// multiples of 4: one float4 per thread and step).
__global__ __launch_bounds__(256) void k_chan_copy(const float* __restrict__ src, int sC, int soff,
                                                   float* __restrict__ dst, int dC, int doff,
                                                   int c4, size_t V) {
  const size_t total = V * (size_t)c4;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t v = i / c4;
    const int q = (int)(i - v * c4);
    *reinterpret_cast<float4*>(dst + v * dC + doff + 4 * q) =
        *reinterpret_cast<const float4*>(src + v * sC + soff + 4 * q);
  }
}

// In place allowed (y == x, gx == gy): each value is read, then written, by
// the one thread that owns it.
__global__ __launch_bounds__(256) void k_relu_fwd(const float4* x, float4* y, size_t n4) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4;
       i += (size_t)gridDim.x * blockDim.x) {
    const float4 a = x[i];
    y[i] = make_float4(fmaxf(a.x, 0.f), fmaxf(a.y, 0.f), fmaxf(a.z, 0.f), fmaxf(a.w, 0.f));
  }
}

// gx = gy where y > 0, else 0 (the derivative at the kink taken as 0).
__global__ __launch_bounds__(256) void k_relu_bwd(const float4* y, const float4* gy, float4* gx,
                                                  size_t n4) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4;
       i += (size_t)gridDim.x * blockDim.x) {
    const float4 a = y[i], g = gy[i];
    gx[i] = make_float4(a.x > 0.f ? g.x : 0.f, a.y > 0.f ? g.y : 0.f, a.z > 0.f ? g.z : 0.f,
                        a.w > 0.f ? g.w : 0.f);
  }
}

unsigned elementwise_blocks(size_t work) {
  return (unsigned)std::max<size_t>(1, std::min<size_t>((work + 255) / 256, 16384));
}

int head_blocks(size_t V) {
  const size_t b = (V + kHeadChunk - 1) / kHeadChunk;
  return (int)std::max<size_t>(1, std::min<size_t>(b, 1024));
}

int att_tiles(int n) {
  const int m = n / 2;
  return (m * m * m + kAttU - 1) / kAttU;
}

int att_bwd_blocks(int n) { return std::max(1, std::min(att_tiles(n), 512)); }

}  // namespace

size_t colsum_tmp_doubles(int nrows, int ncols) {
  return (size_t)colsum_slices(nrows) * ncols;
}

void colsum_f64(const double* part, int nrows, int ncols, double* tmp, float* out,
                hipStream_t s) {
  ColOut o{{out, nullptr, nullptr, nullptr, nullptr}, {0, ncols, 0, 0, 0, 0}, 1};
  colsum(part, nrows, ncols, tmp, o, s);
}

int att_max_c() { return kAttMaxC; }
int att_max_cu() { return kAttMaxCu; }
int head_max_c() { return kHeadMaxC; }

size_t head_scratch_bytes(size_t V, int C) {
  const int nb = head_blocks(V);
  return (size_t)(nb + colsum_slices(nb)) * (C + 1) * sizeof(double);
}

void head_forward(const float* x, const float* w, const float* b, const float* mask, size_t V,
                  int C, int sig, float* out, hipStream_t s) {
  const size_t blocks = std::min<size_t>((V + 255) / 256, 8192);
  hipLaunchKernelGGL(k_head_fwd, dim3((unsigned)std::max<size_t>(1, blocks)), dim3(256), 0, s, x,
                     w, b, mask, V, C, sig, out);
}

void head_backward(const float* x, const float* w, const float* b, const float* mask,
                   const float* gout, size_t V, int C, int sig, float* gx, float* gw, float* gb,
                   void* scratch, hipStream_t s) {
  const int nb = head_blocks(V);
  double* part = reinterpret_cast<double*>(scratch);
  hipLaunchKernelGGL(k_head_bwd, dim3(nb), dim3(256), 0, s, x, w, b, mask, gout, V, C, sig, gx,
                     part);
  if (gw || gb) {
    ColOut o{{gw, gb, nullptr, nullptr, nullptr}, {0, C, C + 1, 0, 0, 0}, 2};
    colsum(part, nb, C + 1, part + (size_t)nb * (C + 1), o, s);
  }
}

namespace {

size_t vox3(int n) { return (size_t)n * n * n; }

// Wide channels (composed form): workspace pieces, 256-byte aligned.
struct AttwWs {
  float *Z = nullptr, *W = nullptr, *a = nullptr, *al = nullptr, *gt = nullptr, *ga = nullptr,
        *gZ = nullptr, *gW = nullptr, *pwp = nullptr;
  double *gp = nullptr, *tmp = nullptr;
  int nbg = 0;
  size_t bytes = 0;
};

AttwWs attw_carve(char* base, int n, int c, int cu, bool bwd) {
  AttwWs w;
  const size_t m = n / 2, Vc = m * m * m, K = c + cu;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = (off + 255) & ~size_t(255);
    char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  w.Z = reinterpret_cast<float*>(take(Vc * K * 4));
  w.W = reinterpret_cast<float*>(take((size_t)c * K * 4));
  w.a = reinterpret_cast<float*>(take(Vc * c * 4));
  w.al = reinterpret_cast<float*>(take(Vc * 4));
  if (bwd) {
    w.nbg = (int)std::max<size_t>(1, std::min<size_t>((Vc + kAttwRows - 1) / kAttwRows, 1024));
    w.gt = reinterpret_cast<float*>(take(Vc * 4));
    w.ga = reinterpret_cast<float*>(take(Vc * c * 4));
    w.gZ = reinterpret_cast<float*>(take(Vc * K * 4));
    w.gW = reinterpret_cast<float*>(take((size_t)c * K * 4));
    w.pwp = reinterpret_cast<float*>(take(pw_partials(Vc, (int)K, c) * 4));
    w.gp = reinterpret_cast<double*>(take((size_t)w.nbg * (c + 1) * 8));
    w.tmp = reinterpret_cast<double*>(take((size_t)colsum_slices(w.nbg) * (c + 1) * 8));
  }
  w.bytes = off;
  return w;
}

bool att_wide(int c, int cu) { return c > kAttMaxC || cu > kAttMaxCu; }

unsigned wave_blocks(size_t items) {  // four waves per block, one item per wave
  return (unsigned)std::max<size_t>(1, std::min<size_t>((items + 3) / 4, 8192));
}

// a = Z Wcat^T + b and the gate, from x and g (both forms of the wide path).
void attw_gate_fwd(const AttArgs& A, const AttwWs& w, float* alpha, hipStream_t s) {
  const int c = A.c, cu = A.cu, K = c + cu, m = A.n / 2;
  const size_t Vc = (size_t)m * m * m;
  hipLaunchKernelGGL(k_attw_stage, dim3(elementwise_blocks(Vc * (K / 4))), dim3(256), 0, s, A.x,
                     A.g, A.n, c, cu, w.Z);
  hipLaunchKernelGGL(k_attw_catw, dim3((c * K + 255) / 256), dim3(256), 0, s, A.wx, A.wg, c, cu,
                     w.W);
  pw_gemm(w.Z, w.W, A.b, w.a, Vc, K, c, false, s);
  hipLaunchKernelGGL(k_attw_gate, dim3(wave_blocks(Vc)), dim3(256), 0, s, w.a, A.psi, A.bpsi, Vc, c,
                     w.al, alpha);
}

}  // namespace

int att_max_c_wide() { return 256; }
int att_max_cu_wide() { return 512; }

size_t att_scratch_bytes(int n, int c, int cu) {
  if (att_wide(c, cu)) return attw_carve(nullptr, n, c, cu, true).bytes + 256;
  const int nb = att_bwd_blocks(n);
  const size_t np = att_nparams(c, cu);
  return (size_t)nb * np * sizeof(float) + (size_t)colsum_slices(nb) * np * sizeof(double) + 256;
}

size_t att_lds_bytes(int c, int cu, bool bwd) { return (size_t)att_lds(c, cu, bwd).total * 4; }

template <class Kern>
void att_launch(Kern k, size_t lds, dim3 grid, hipStream_t s, const AttArgs& A, int nt, float* p0,
                float* p1) {
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k, grid, dim3(256), lds, s, A, nt, p0, p1);
}

void att_forward(const float* x, const float* g, const float* wx, const float* wg, const float* b,
                 const float* psi, const float* bpsi, float* y, float* alpha, int n, int c, int cu,
                 void* scratch, hipStream_t s) {
  AttArgs A{x, g, wx, wg, b, psi, bpsi, n, c, cu};
  if (att_wide(c, cu)) {
    const AttwWs w = attw_carve(reinterpret_cast<char*>(scratch), n, c, cu, false);
    attw_gate_fwd(A, w, alpha, s);
    hipLaunchKernelGGL(k_attw_scale, dim3(elementwise_blocks(vox3(n) * (c / 4))), dim3(256), 0, s,
                       x, w.al, n, c, y);
    return;
  }
  const int nt = att_tiles(n), items = (c + 15) / 16;
  const size_t lds = att_lds_bytes(c, cu, false);
  const dim3 grid(nt);
  switch (items) {
    case 1: att_launch(k_att_fwd<1>, lds, grid, s, A, nt, y, alpha); break;
    case 2: att_launch(k_att_fwd<2>, lds, grid, s, A, nt, y, alpha); break;
    case 3: att_launch(k_att_fwd<3>, lds, grid, s, A, nt, y, alpha); break;
    default: att_launch(k_att_fwd<4>, lds, grid, s, A, nt, y, alpha); break;
  }
}

void att_backward(const float* x, const float* g, const float* wx, const float* wg,
                  const float* b, const float* psi, const float* bpsi, const float* gy,
                  float* gx, float* gg, float* gwx, float* gwg, float* gb, float* gpsi,
                  float* gbpsi, int n, int c, int cu, void* scratch, hipStream_t s) {
  AttArgs A{x, g, wx, wg, b, psi, bpsi, n, c, cu};
  if (att_wide(c, cu)) {
    const AttwWs w = attw_carve(reinterpret_cast<char*>(scratch), n, c, cu, true);
    const int K = c + cu, m = n / 2;
    const size_t Vc = (size_t)m * m * m;
    attw_gate_fwd(A, w, nullptr, s);
    hipLaunchKernelGGL(k_attw_gdot, dim3(wave_blocks(Vc)), dim3(256), 0, s, x, gy, w.al, n, c,
                       w.gt);
    hipLaunchKernelGGL(k_attw_gate_bwd, dim3(w.nbg), dim3(256), 0, s, w.a, psi, w.gt, Vc, c, w.ga,
                       w.gp);
    if (gpsi || gbpsi) {
      ColOut o{{gpsi, gbpsi, nullptr, nullptr, nullptr}, {0, c, c + 1, 0, 0, 0}, 2};
      colsum(w.gp, w.nbg, c + 1, w.tmp, o, s);
    }
    // gW = ga^T Z (then split into wx and wg), gb = column sums of ga
    if (gwx || gwg || gb) {
      pw_wgrad(w.Z, w.ga, w.pwp, w.gW, gb, Vc, K, c, s);
      if (gwx) channel_copy(w.gW, K, 0, gwx, c, 0, c, (size_t)c, s);
      if (gwg) channel_copy(w.gW, K, c, gwg, cu, 0, cu, (size_t)c, s);
    }
    if (gx || gg) {
      pw_gemm(w.ga, w.W, nullptr, w.gZ, Vc, c, K, true, s);  // gZ = ga Wcat
      if (gg) channel_copy(w.gZ, K, c, gg, cu, 0, cu, Vc, s);
      if (gx)
        hipLaunchKernelGGL(k_attw_scale_bwd, dim3(elementwise_blocks(vox3(n) * (c / 4))), dim3(256),
                           0, s, gy, w.al, w.gZ, n, c, K, gx);
    }
    return;
  }
  const int nt = att_tiles(n), nb = att_bwd_blocks(n), items = (c + 15) / 16;
  float* part = reinterpret_cast<float*>(scratch);
  const int np = att_nparams(c, cu);
  const size_t lds = att_lds_bytes(c, cu, true);
  const dim3 grid(nb);
  auto launch = [&](auto kern) {
    if (lds > 64 * 1024)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, A, nt, gy, gx, gg, part);
  };
  switch (items) {
    case 1: launch(k_att_bwd<1>); break;
    case 2: launch(k_att_bwd<2>); break;
    case 3: launch(k_att_bwd<3>); break;
    default: launch(k_att_bwd<4>); break;
  }
  const int o_wg = c * c, o_b = o_wg + c * cu, o_psi = o_b + c, o_bpsi = o_psi + c;
  // the FP64 slice sums start at the next 256-byte boundary after the partials
  const size_t pb = ((size_t)nb * np * sizeof(float) + 255) / 256 * 256;
  double* tmp = reinterpret_cast<double*>(reinterpret_cast<char*>(scratch) + pb);
  ColOut o{{gwx, gwg, gb, gpsi, gbpsi}, {0, o_wg, o_b, o_psi, o_bpsi, np}, 5};
  colsum(part, nb, np, tmp, o, s);
}

void channel_copy(const float* src, int sC, int soff, float* dst, int dC, int doff, int c,
                  size_t V, hipStream_t s) {
  hipLaunchKernelGGL(k_chan_copy, dim3(elementwise_blocks(V * (c / 4))), dim3(256), 0, s, src, sC,
                     soff, dst, dC, doff, c / 4, V);
}

void relu_forward(const float* x, float* y, size_t count, hipStream_t s) {
  const size_t n4 = count / 4;
  hipLaunchKernelGGL(k_relu_fwd, dim3(elementwise_blocks(n4)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(x), reinterpret_cast<float4*>(y), n4);
}

void relu_backward(const float* y, const float* gy, float* gx, size_t count, hipStream_t s) {
  const size_t n4 = count / 4;
  hipLaunchKernelGGL(k_relu_bwd, dim3(elementwise_blocks(n4)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(y), reinterpret_cast<const float4*>(gy),
                     reinterpret_cast<float4*>(gx), n4);
}

}  // namespace d2ip
