// Whole-volume LayerNorm (statistics over all channels and voxels of one
// instance, per-channel affine), ReLU, 2x2x2 average pooling, nearest x2
// up-sampling with channel concatenation, and their backward passes.
// Activations are NDHWC fp32; reductions accumulate in FP64 and combine
// per-block partials in a fixed order, so results are run-to-run identical.
#include "kernels.h"


namespace d2ip {
namespace {

constexpr int kElemsPerBlock = 1024;

__global__ void k_ln_apply(const float4* h, PairRef sr, const float* g, const float* b,
                           const float4* skip, float4* y, size_t n4, int C, long long istride) {
  {
    const long long off = (long long)blockIdx.y * istride;
    h = ishift(h, off); sr.part = ishift(sr.part, off); g = ishift(g, off); b = ishift(b, off);
    skip = ishift(skip, off); y = ishift(y, off);
  }
  // the first element's loads are in flight while the statistics are reduced
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  float4 vn = z4, sn = z4;
  if (i < n4) {
    vn = h[i];
    if (skip) sn = skip[i];
  }
  const LnStat st = stat_of(sr);
  const float mean = st.mean, rstd = st.rstd;
  for (; i < n4; i += stride) {
    const int c = (int)((i * 4) % C);
    const float4 v = vn, s = sn;
    if (i + stride < n4) {
      vn = h[i + stride];
      if (skip) sn = skip[i + stride];
    }
    float4 o;
    o.x = fmaxf(g[c + 0] * ((v.x - mean) * rstd) + b[c + 0] + s.x, 0.f);
    o.y = fmaxf(g[c + 1] * ((v.y - mean) * rstd) + b[c + 1] + s.y, 0.f);
    o.z = fmaxf(g[c + 2] * ((v.z - mean) * rstd) + b[c + 2] + s.z, 0.f);
    o.w = fmaxf(g[c + 3] * ((v.w - mean) * rstd) + b[c + 3] + s.w, 0.f);
    y[i] = o;
  }
}

// gz = gy * mask and the block's partial sums: part_c[blk] = per-channel
// (sum gz*xhat [C], sum gz [C]); part_ab[blk] = (sum_c gamma_c sum gz,
// sum_c gamma_c sum gz*xhat).
__global__ __launch_bounds__(256) void k_ln_bwd(
    const float* gy, int mask_mode, const float* my, const float* mg, const float* mb,
    const float* h, PairRef sr, float* gz, double* part_c, double* part_ab, int V, int C, int vpb,
    const float* gamma, long long istride) {
  {
    const long long off = (long long)blockIdx.y * istride;
    gy = ishift(gy, off); my = ishift(my, off); mg = ishift(mg, off); mb = ishift(mb, off);
    h = ishift(h, off); sr.part = ishift(sr.part, off); gz = ishift(gz, off);
    part_c = ishift(part_c, off); part_ab = ishift(part_ab, off); gamma = ishift(gamma, off);
  }
  __shared__ double sh1[256], sh2[256];
  const int tid = threadIdx.x;
  const int c = tid % C, r0 = tid / C, rpi = 256 / C;
  const int v0 = blockIdx.x * vpb;
  const int v1 = min(V, v0 + vpb);
  // the first kLnPre elements of this thread are loaded while the statistics
  // are reduced (vpb <= kLnPre * rpi for every C the plan uses)
  constexpr int kLnPre = 4;
  float hp[kLnPre], gp[kLnPre], mp[kLnPre];
#pragma unroll
  for (int k = 0; k < kLnPre; ++k) {
    const int v = v0 + r0 + k * rpi;
    hp[k] = gp[k] = mp[k] = 0.f;
    if (v < v1) {
      const size_t i = (size_t)v * C + c;
      hp[k] = h[i];
      gp[k] = gy[i];
      if (mask_mode == LNMASK_Y) mp[k] = my[i];
    }
  }
  const LnStat st = stat_of(sr);
  const float mean = st.mean, rstd = st.rstd;
  const float gam = mask_mode == LNMASK_LN ? mg[c] : 0.f;
  const float bet = mask_mode == LNMASK_LN ? mb[c] : 0.f;
  double s1 = 0.0, s2 = 0.0;
  auto elem = [&](size_t i, float hv, float gv, float mv) {
    const float xh = (hv - mean) * rstd;
    if (mask_mode == LNMASK_Y) gv = mv > 0.f ? gv : 0.f;
    else if (mask_mode == LNMASK_LN) gv = (gam * xh + bet) > 0.f ? gv : 0.f;
    gz[i] = gv;
    s1 += gv;
    s2 += (double)gv * xh;
  };
#pragma unroll
  for (int k = 0; k < kLnPre; ++k) {
    const int v = v0 + r0 + k * rpi;
    if (v < v1) elem((size_t)v * C + c, hp[k], gp[k], mp[k]);
  }
  for (int v = v0 + r0 + kLnPre * rpi; v < v1; v += rpi) {
    const size_t i = (size_t)v * C + c;
    elem(i, h[i], gy[i], mask_mode == LNMASK_Y ? my[i] : 0.f);
  }
  sh1[tid] = s1;
  sh2[tid] = s2;
  __syncthreads();
  double ga = 0.0, gb = 0.0;
  if (tid < C) {
    double a = 0.0, b = 0.0;
    for (int k = tid; k < 256; k += C) {
      a += sh1[k];
      b += sh2[k];
    }
    part_c[(size_t)blockIdx.x * 2 * C + tid] = b;      // dgamma partial
    part_c[(size_t)blockIdx.x * 2 * C + C + tid] = a;  // dbeta partial
    ga = (double)gamma[tid] * a;
    gb = (double)gamma[tid] * b;
  }
  __syncthreads();
  ga = block_sum(ga, sh1);
  gb = block_sum(gb, sh2);
  if (tid == 0) {
    part_ab[2 * (size_t)blockIdx.x] = ga;
    part_ab[2 * (size_t)blockIdx.x + 1] = gb;
  }
}

// y = relu(LN(h) + skip) for 2x2x2 groups of voxels, and the group mean of y
// (the average-pooled input of the next encoder level) when `pooled` is set.
// Thread t handles child t % 8 of coarse element t / 8 (a float4 of channels);
// the eight threads of a group are adjacent lanes, and the child-0 lane adds
// the group's values in child order.
__global__ void k_ln_apply_pool(const float4* h, PairRef sr, const float* g, const float* b,
                                const float4* skip, float4* y, float4* pooled, int n, int C4,
                                long long istride) {
  {
    const long long off = (long long)blockIdx.y * istride;
    h = ishift(h, off); sr.part = ishift(sr.part, off); g = ishift(g, off); b = ishift(b, off);
    skip = ishift(skip, off); y = ishift(y, off); pooled = ishift(pooled, off);
  }
  const int m = n / 2;
  const size_t total8 = (size_t)m * m * m * C4 * 8;
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  const int lane = threadIdx.x & 63, k = lane & 7, g0 = lane & ~7;
  // fine-grid element of child k of coarse element i
  auto child = [&](size_t i) {
    const int c4 = (int)(i % C4);
    const size_t vc = i / C4;
    const int xx = (int)(vc % m), yy = (int)((vc / m) % m), zz = (int)(vc / ((size_t)m * m));
    const int fz = 2 * zz + (k >> 2), fy = 2 * yy + ((k >> 1) & 1), fx = 2 * xx + (k & 1);
    return ((size_t)(fz * n + fy) * n + fx) * C4 + c4;
  };
  // the first element is loaded while the statistics are reduced
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t t0 = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  float4 hv = z4, sv = z4;
  if (t0 < total8) {
    const size_t j = child(t0 >> 3);
    hv = h[j];
    if (skip) sv = skip[j];
  }
  const LnStat st = stat_of(sr);
  const float mean = st.mean, rstd = st.rstd;
  // whole blocks iterate together (the group sums read other lanes)
  for (size_t base = blockIdx.x * (size_t)blockDim.x; base < total8; base += stride) {
    const size_t t = base + threadIdx.x;
    const bool ok = t < total8;
    const size_t i = t >> 3;
    const int c = 4 * (int)(i % C4);
    float4 o = z4;
    if (ok) {
      const size_t j = child(i);
      float4 v, sk;
      if (t == t0) {
        v = hv;
        sk = sv;
      } else {
        v = h[j];
        sk = skip ? skip[j] : z4;
      }
      o.x = fmaxf(g[c + 0] * ((v.x - mean) * rstd) + b[c + 0] + sk.x, 0.f);
      o.y = fmaxf(g[c + 1] * ((v.y - mean) * rstd) + b[c + 1] + sk.y, 0.f);
      o.z = fmaxf(g[c + 2] * ((v.z - mean) * rstd) + b[c + 2] + sk.z, 0.f);
      o.w = fmaxf(g[c + 3] * ((v.w - mean) * rstd) + b[c + 3] + sk.w, 0.f);
      y[j] = o;
    }
    if (pooled) {
      float4 s = z4;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        s.x += __shfl(o.x, g0 + q, 64);
        s.y += __shfl(o.y, g0 + q, 64);
        s.z += __shfl(o.z, g0 + q, 64);
        s.w += __shfl(o.w, g0 + q, 64);
      }
      if (ok && k == 0)
        pooled[i] = make_float4(0.125f * s.x, 0.125f * s.y, 0.125f * s.z, 0.125f * s.w);
    }
  }
}

// y[v'][c] = mean of the 8 children (fine grid n, coarse n/2).
__global__ void k_avgpool2(const float4* __restrict__ x, int n, int C4, float4* __restrict__ y) {
  const int m = n / 2;
  const size_t total = (size_t)m * m * m * C4;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int c4 = (int)(i % C4);
    const size_t vc = i / C4;
    const int xx = (int)(vc % m), yy = (int)((vc / m) % m), zz = (int)(vc / ((size_t)m * m));
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int fz = 2 * zz + (k >> 2), fy = 2 * yy + ((k >> 1) & 1), fx = 2 * xx + (k & 1);
      const float4 v = x[((size_t)(fz * n + fy) * n + fx) * C4 + c4];
      s.x += v.x; s.y += v.y; s.z += v.z; s.w += v.w;
    }
    y[i] = make_float4(0.125f * s.x, 0.125f * s.y, 0.125f * s.z, 0.125f * s.w);
  }
}

// cat[v][0..Cu) = d[parent(v)], cat[v][Cu..Cu+Cs) = e[v]  (fine grid n).
__global__ void k_up_concat(const float4* d, int Cu4, const float4* e, int Cs4, int n, float4* cat,
                            long long istride) {
  {
    const long long off = (long long)blockIdx.y * istride;
    d = ishift(d, off); e = ishift(e, off); cat = ishift(cat, off);
  }
  const int m = n / 2, C4 = Cu4 + Cs4;
  const size_t total = (size_t)n * n * n * C4;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int c4 = (int)(i % C4);
    const size_t v = i / C4;
    if (c4 < Cu4) {
      const int xx = (int)(v % n), yy = (int)((v / n) % n), zz = (int)(v / ((size_t)n * n));
      cat[i] = d[((size_t)((zz >> 1) * m + (yy >> 1)) * m + (xx >> 1)) * Cu4 + c4];
    } else {
      cat[i] = e[v * Cs4 + (c4 - Cu4)];
    }
  }
}

// gu[v'][c] = sum of gcat[child][c] over the 8 children, c < Cu (coarse grid).
__global__ void k_up_bwd(const float4* gcat, int C4, int Cu4, int n, float4* gu,
                         long long istride) {
  {
    const long long off = (long long)blockIdx.y * istride;
    gcat = ishift(gcat, off); gu = ishift(gu, off);
  }
  const int m = n / 2;
  const size_t total = (size_t)m * m * m * Cu4;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int c4 = (int)(i % Cu4);
    const size_t vc = i / Cu4;
    const int xx = (int)(vc % m), yy = (int)((vc / m) % m), zz = (int)(vc / ((size_t)m * m));
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int fz = 2 * zz + (k >> 2), fy = 2 * yy + ((k >> 1) & 1), fx = 2 * xx + (k & 1);
      const float4 v = gcat[((size_t)(fz * n + fy) * n + fx) * C4 + c4];
      s.x += v.x; s.y += v.y; s.z += v.z; s.w += v.w;
    }
    gu[i] = s;
  }
}

// gs[v][c] = gcat[v][Cu + c]
__global__ void k_cat_split(const float4* gcat, int C4, int Cu4, int Cs4, size_t V, float4* gs,
                            long long istride) {
  {
    const long long off = (long long)blockIdx.y * istride;
    gcat = ishift(gcat, off); gs = ishift(gs, off);
  }
  const size_t total = V * Cs4;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t v = i / Cs4;
    gs[i] = gcat[v * C4 + Cu4 + (i % Cs4)];
  }
}

// gy[v][c] = add[v][c] + gx[parent(v)][c] / 8   (fine grid n; add may be null)
__global__ void k_pool_bwd_add(const float4* gx, const float4* add, int n, int C4, float4* gy,
                               long long istride) {
  {
    const long long off = (long long)blockIdx.y * istride;
    gx = ishift(gx, off); add = ishift(add, off); gy = ishift(gy, off);
  }
  const int m = n / 2;
  const size_t total = (size_t)n * n * n * C4;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int c4 = (int)(i % C4);
    const size_t v = i / C4;
    const int xx = (int)(v % n), yy = (int)((v / n) % n), zz = (int)(v / ((size_t)n * n));
    const float4 p = gx[((size_t)((zz >> 1) * m + (yy >> 1)) * m + (xx >> 1)) * C4 + c4];
    const float4 a = add ? add[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    gy[i] = make_float4(a.x + 0.125f * p.x, a.y + 0.125f * p.y, a.z + 0.125f * p.z,
                        a.w + 0.125f * p.w);
  }
}

// zp[v][0] = z[v], zp[v][1..8) = 0
__global__ void k_pad_input(const float* __restrict__ z, size_t V, float* __restrict__ zp) {

  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < V * 8;
       i += (size_t)gridDim.x * blockDim.x)
    zp[i] = (i % 8) == 0 ? z[i / 8] : 0.f;
}

inline int grid_for(size_t work, int per_thread = 1) {
  size_t b = (work / per_thread + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

// Per-block FP64 (sum, sum of squares) partials of x[0..n): block b covers a
// contiguous range of `per` values (a multiple of 4; x 16-byte aligned, n a
// multiple of 4), read as float4 quads, four per thread in flight and added
// in quad order, so the partials (and any fixed-order sum of them) are
// run-to-run identical.  The statistics a standalone LayerNorm needs.
__global__ __launch_bounds__(256) void k_block_stats(const float4* x, size_t n, size_t per,
                                                     double* part) {
  __shared__ double sh[8];
  const size_t q0 = blockIdx.x * per / 4, q1 = min(n, (blockIdx.x + 1) * per) / 4;
  double s1 = 0.0, s2 = 0.0;
  for (size_t q = q0 + threadIdx.x; q < q1; q += 1024) {
    float4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const size_t i = q + 256 * k;
      v[k] = i < q1 ? x[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double a = v[k].x, b = v[k].y, c = v[k].z, d = v[k].w;
      s1 += ((a + b) + c) + d;
      s2 += ((a * a + b * b) + c * c) + d * d;
    }
  }
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1;
    part[2 * blockIdx.x + 1] = s2;
  }
}

// LayerNorm input gradient: gx = rstd * (gamma_c * gz - A - xhat * B), with
// the statistics of h and the coefficients (A, B) reduced from partials.
__global__ void k_ln_dx(const float4* gz, const float4* h, PairRef st, PairRef bw,
                        const float* gamma, float4* gx, size_t n4, int C) {
  LnStat s;
  LnBwd k;
  stat_coef_of(st, bw, s, k);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4;
       i += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)((i * 4) % C);
    const float4 g = gz[i], x = h[i];
    float4 o;
    o.x = s.rstd * (gamma[c + 0] * g.x - k.A - ((x.x - s.mean) * s.rstd) * k.B);
    o.y = s.rstd * (gamma[c + 1] * g.y - k.A - ((x.y - s.mean) * s.rstd) * k.B);
    o.z = s.rstd * (gamma[c + 2] * g.z - k.A - ((x.z - s.mean) * s.rstd) * k.B);
    o.w = s.rstd * (gamma[c + 3] * g.w - k.A - ((x.w - s.mean) * s.rstd) * k.B);
    gx[i] = o;
  }
}

}  // namespace

void ln_apply(const float* h, PairRef st, const float* g, const float* b, const float* skip,
              float* y, size_t V, int C, int batch, long long istride, hipStream_t s) {
  const size_t n4 = V * C / 4;
  hipLaunchKernelGGL(k_ln_apply, dim3(grid_for(n4), batch), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(h), st, g, b,
                     reinterpret_cast<const float4*>(skip), reinterpret_cast<float4*>(y), n4, C,
                     istride);
}

int ln_bwd_blocks(size_t V, int C) {
  const int vpb = ln_bwd_vpb(C);
  return (int)((V + vpb - 1) / vpb);
}

int ln_bwd_vpb(int C) {
  int vpb = kElemsPerBlock / C;
  if (vpb < 256 / C) vpb = 256 / C;
  return vpb;
}

void ln_bwd(const float* gy, int mask_mode, const float* my, const float* mg, const float* mb,
            const float* h, PairRef st, float* gz, double* part_c, double* part_ab, size_t V,
            int C, const float* gamma, int batch, long long istride, hipStream_t s) {
  hipLaunchKernelGGL(k_ln_bwd, dim3(ln_bwd_blocks(V, C), batch), dim3(256), 0, s, gy, mask_mode,
                     my, mg, mb, h, st, gz, part_c, part_ab, (int)V, C, ln_bwd_vpb(C), gamma,
                     istride);
}

void ln_apply_pool(const float* h, PairRef st, const float* g, const float* b, const float* skip,
                   float* y, float* pooled, int n, int C, int batch, long long istride,
                   hipStream_t s) {
  const size_t work = (size_t)(n / 2) * (n / 2) * (n / 2) * (C / 4) * 8;  // thread per child
  hipLaunchKernelGGL(k_ln_apply_pool, dim3(grid_for(work), batch), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(h), st, g, b,
                     reinterpret_cast<const float4*>(skip), reinterpret_cast<float4*>(y),
                     reinterpret_cast<float4*>(pooled), n, C / 4, istride);
}

void avgpool2(const float* x, int n, int C, float* y, hipStream_t s) {
  const size_t work = (size_t)(n / 2) * (n / 2) * (n / 2) * (C / 4);
  hipLaunchKernelGGL(k_avgpool2, dim3(grid_for(work)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(x), n, C / 4, reinterpret_cast<float4*>(y));
}

void up_concat(const float* d, int Cu, const float* e, int Cs, int n, float* cat, int batch,
               long long istride, hipStream_t s) {
  const size_t work = (size_t)n * n * n * ((Cu + Cs) / 4);
  hipLaunchKernelGGL(k_up_concat, dim3(grid_for(work), batch), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(d), Cu / 4,
                     reinterpret_cast<const float4*>(e), Cs / 4, n,
                     reinterpret_cast<float4*>(cat), istride);
}

void up_concat_bwd(const float* gcat, int Cu, int Cs, int n, float* gu, float* gs, int batch,
                   long long istride, hipStream_t s) {
  const int C4 = (Cu + Cs) / 4;
  const size_t wu = (size_t)(n / 2) * (n / 2) * (n / 2) * (Cu / 4);
  hipLaunchKernelGGL(k_up_bwd, dim3(grid_for(wu), batch), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(gcat), C4, Cu / 4, n,
                     reinterpret_cast<float4*>(gu), istride);
  const size_t V = (size_t)n * n * n;
  hipLaunchKernelGGL(k_cat_split, dim3(grid_for(V * (Cs / 4)), batch), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(gcat), C4, Cu / 4, Cs / 4, V,
                     reinterpret_cast<float4*>(gs), istride);
}

void pool_bwd_add(const float* gx, const float* add, int n, int C, float* gy, int batch,
                  long long istride, hipStream_t s) {
  const size_t work = (size_t)n * n * n * (C / 4);
  hipLaunchKernelGGL(k_pool_bwd_add, dim3(grid_for(work), batch), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(gx), reinterpret_cast<const float4*>(add), n,
                     C / 4, reinterpret_cast<float4*>(gy), istride);
}

__global__ void k_zero_words(int* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

void zero_words(void* p, size_t n, hipStream_t s) {
  if (n == 0) return;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)blocks), dim3(256), 0, s,
                     reinterpret_cast<int*>(p), n);
}

void pad_input(const float* z, size_t V, float* zp, hipStream_t s) {
  hipLaunchKernelGGL(k_pad_input, dim3(grid_for(V * 8)), dim3(256), 0, s, z, V, zp);
}

// About 2048 values per block (enough blocks to cover the chip from 32^3 x 16
// on), at most 1024 blocks (the consumers add the partials in one pass).
int block_stats_blocks(size_t n) {
  size_t b = (n + 2047) / 2048;
  if (b > 1024) b = 1024;
  return (int)(b < 1 ? 1 : b);
}

void block_stats(const float* x, size_t n, double* part, hipStream_t s) {
  const int nb = block_stats_blocks(n);
  const size_t per = ((n + nb - 1) / nb + 3) / 4 * 4;
  hipLaunchKernelGGL(k_block_stats, dim3(nb), dim3(256), 0, s, reinterpret_cast<const float4*>(x),
                     n, per, part);
}

void ln_dx(const float* gz, const float* h, PairRef st, PairRef bw, const float* gamma, float* gx,
           size_t V, int C, hipStream_t s) {
  const size_t n4 = V * C / 4;
  hipLaunchKernelGGL(k_ln_dx, dim3(grid_for(n4)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(gz), reinterpret_cast<const float4*>(h), st,
                     bw, gamma, reinterpret_cast<float4*>(gx), n4, C);
}

}  // namespace d2ip
