// Whole-volume LayerNorm (statistics over all channels and voxels of one
// instance, per-channel affine), ReLU, 2x2x2 average pooling, nearest x2
// up-sampling with channel concatenation, and their backward passes.
// Activations are NDHWC fp32; reductions accumulate in FP64 and combine
// per-block partials in a fixed order, so results are run-to-run identical.
#include "kernels.h"


namespace d2ip {
namespace {

constexpr int kElemsPerBlock = 4096;

__global__ void k_ln_finalize(const double* __restrict__ part, int nparts, double count, float eps,
                              LnStat* out) {
  __shared__ double sh[16];
  double s1 = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
    s1 += part[2 * i];
    s2 += part[2 * i + 1];
  }
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    const double mean = s1 / count;
    double var = s2 / count - mean * mean;
    if (var < 0.0) var = 0.0;
    out->mean = (float)mean;
    out->rstd = (float)(1.0 / sqrt(var + (double)eps));
  }
}

__global__ void k_ln_apply(const float4* __restrict__ h, const LnStat* __restrict__ st,
                           const float* __restrict__ g, const float* __restrict__ b,
                           const float4* __restrict__ skip, float4* __restrict__ y, size_t n4,
                           int C) {
  const float mean = st->mean, rstd = st->rstd;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4;
       i += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)((i * 4) % C);
    float4 v = h[i];
    float4 s = skip ? skip[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    float4 o;
    o.x = fmaxf(g[c + 0] * ((v.x - mean) * rstd) + b[c + 0] + s.x, 0.f);
    o.y = fmaxf(g[c + 1] * ((v.y - mean) * rstd) + b[c + 1] + s.y, 0.f);
    o.z = fmaxf(g[c + 2] * ((v.z - mean) * rstd) + b[c + 2] + s.z, 0.f);
    o.w = fmaxf(g[c + 3] * ((v.w - mean) * rstd) + b[c + 3] + s.w, 0.f);
    y[i] = o;
  }
}

// gz = gy * mask; per-block per-channel partial sums of gz and gz * xhat.
__global__ __launch_bounds__(256) void k_ln_bwd_sums(
    const float* gy, int mask_mode, const float* __restrict__ my,
    const float* __restrict__ mg, const float* __restrict__ mb, const float* __restrict__ h,
    const LnStat* __restrict__ st, float* gz, double* __restrict__ part, int V,
    int C, int vpb) {
  __shared__ double sh1[256], sh2[256];
  const int tid = threadIdx.x;
  const int c = tid % C, r0 = tid / C, rpi = 256 / C;
  const float mean = st->mean, rstd = st->rstd;
  const float gam = mask_mode == LNMASK_LN ? mg[c] : 0.f;
  const float bet = mask_mode == LNMASK_LN ? mb[c] : 0.f;
  double s1 = 0.0, s2 = 0.0;
  const int v0 = blockIdx.x * vpb;
  const int v1 = min(V, v0 + vpb);
  for (int v = v0 + r0; v < v1; v += rpi) {
    const size_t i = (size_t)v * C + c;
    const float xh = (h[i] - mean) * rstd;
    float gv = gy[i];
    if (mask_mode == LNMASK_Y) gv = my[i] > 0.f ? gv : 0.f;
    else if (mask_mode == LNMASK_LN) gv = (gam * xh + bet) > 0.f ? gv : 0.f;
    gz[i] = gv;
    s1 += gv;
    s2 += (double)gv * xh;
  }
  sh1[tid] = s1;
  sh2[tid] = s2;
  __syncthreads();
  if (tid < C) {
    double a = 0.0, b = 0.0;
    for (int k = tid; k < 256; k += C) {
      a += sh1[k];
      b += sh2[k];
    }
    part[((size_t)blockIdx.x * C + tid) * 2] = a;
    part[((size_t)blockIdx.x * C + tid) * 2 + 1] = b;
  }
}

__global__ void k_ln_bwd_finalize(const double* __restrict__ part, int nparts, int C, double count,
                                  const float* __restrict__ gamma, float* dgamma, float* dbeta,
                                  LnBwd* coef) {
  __shared__ double sh[16];
  double a = 0.0, b = 0.0;
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    double s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < nparts; ++k) {
      s1 += part[((size_t)k * C + c) * 2];
      s2 += part[((size_t)k * C + c) * 2 + 1];
    }
    dgamma[c] = (float)s2;
    dbeta[c] = (float)s1;
    a += (double)gamma[c] * s1;
    b += (double)gamma[c] * s2;
  }
  a = block_sum(a, sh);
  b = block_sum(b, sh);
  if (threadIdx.x == 0) {
    coef->A = (float)(a / count);
    coef->B = (float)(b / count);
  }
}

__global__ void k_ln_bwd_apply(const float4* __restrict__ gz, const float4* __restrict__ h,
                               const LnStat* __restrict__ st, const float* __restrict__ gamma,
                               const LnBwd* __restrict__ coef, float4* __restrict__ gh, size_t n4,
                               int C) {
  const float mean = st->mean, rstd = st->rstd, A = coef->A, B = coef->B;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4;
       i += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)((i * 4) % C);
    const float4 g = gz[i], x = h[i];
    float4 o;
    o.x = rstd * (gamma[c + 0] * g.x - A - ((x.x - mean) * rstd) * B);
    o.y = rstd * (gamma[c + 1] * g.y - A - ((x.y - mean) * rstd) * B);
    o.z = rstd * (gamma[c + 2] * g.z - A - ((x.z - mean) * rstd) * B);
    o.w = rstd * (gamma[c + 3] * g.w - A - ((x.w - mean) * rstd) * B);
    gh[i] = o;
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
__global__ void k_up_concat(const float4* __restrict__ d, int Cu4, const float4* __restrict__ e,
                            int Cs4, int n, float4* __restrict__ cat) {
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
__global__ void k_up_bwd(const float4* __restrict__ gcat, int C4, int Cu4, int n,
                         float4* __restrict__ gu) {
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
__global__ void k_cat_split(const float4* __restrict__ gcat, int C4, int Cu4, int Cs4, size_t V,
                            float4* __restrict__ gs) {
  const size_t total = V * Cs4;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t v = i / Cs4;
    gs[i] = gcat[v * C4 + Cu4 + (i % Cs4)];
  }
}

// gy[v][c] = add[v][c] + gx[parent(v)][c] / 8   (fine grid n)
__global__ void k_pool_bwd_add(const float4* __restrict__ gx, const float4* __restrict__ add,
                               int n, int C4, float4* __restrict__ gy) {
  const int m = n / 2;
  const size_t total = (size_t)n * n * n * C4;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int c4 = (int)(i % C4);
    const size_t v = i / C4;
    const int xx = (int)(v % n), yy = (int)((v / n) % n), zz = (int)(v / ((size_t)n * n));
    const float4 p = gx[((size_t)((zz >> 1) * m + (yy >> 1)) * m + (xx >> 1)) * C4 + c4];
    const float4 a = add[i];
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

}  // namespace

void ln_finalize(const double* part, int nparts, double count, float eps, LnStat* out,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_ln_finalize, dim3(1), dim3(256), 0, s, part, nparts, count, eps, out);
}

void ln_apply(const float* h, const LnStat* st, const float* g, const float* b, const float* skip,
              float* y, size_t V, int C, hipStream_t s) {
  const size_t n4 = V * C / 4;
  hipLaunchKernelGGL(k_ln_apply, dim3(grid_for(n4)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(h), st, g, b,
                     reinterpret_cast<const float4*>(skip), reinterpret_cast<float4*>(y), n4, C);
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

void ln_bwd_sums(const float* gy, int mask_mode, const float* my, const float* mg, const float* mb,
                 const float* h, const LnStat* st, float* gz, double* part, size_t V, int C,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_ln_bwd_sums, dim3(ln_bwd_blocks(V, C)), dim3(256), 0, s, gy, mask_mode, my,
                     mg, mb, h, st, gz, part, (int)V, C, ln_bwd_vpb(C));
}

void ln_bwd_finalize(const double* part, int nparts, int C, double count, const float* gamma,
                     float* dgamma, float* dbeta, LnBwd* coef, hipStream_t s) {
  hipLaunchKernelGGL(k_ln_bwd_finalize, dim3(1), dim3(256), 0, s, part, nparts, C, count, gamma,
                     dgamma, dbeta, coef);
}

void ln_bwd_apply(const float* gz, const float* h, const LnStat* st, const float* gamma,
                  const LnBwd* coef, float* gh, size_t V, int C, hipStream_t s) {
  const size_t n4 = V * C / 4;
  hipLaunchKernelGGL(k_ln_bwd_apply, dim3(grid_for(n4)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(gz), reinterpret_cast<const float4*>(h), st,
                     gamma, coef, reinterpret_cast<float4*>(gh), n4, C);
}

void avgpool2(const float* x, int n, int C, float* y, hipStream_t s) {
  const size_t work = (size_t)(n / 2) * (n / 2) * (n / 2) * (C / 4);
  hipLaunchKernelGGL(k_avgpool2, dim3(grid_for(work)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(x), n, C / 4, reinterpret_cast<float4*>(y));
}

void up_concat(const float* d, int Cu, const float* e, int Cs, int n, float* cat, hipStream_t s) {
  const size_t work = (size_t)n * n * n * ((Cu + Cs) / 4);
  hipLaunchKernelGGL(k_up_concat, dim3(grid_for(work)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(d), Cu / 4,
                     reinterpret_cast<const float4*>(e), Cs / 4, n,
                     reinterpret_cast<float4*>(cat));
}

void up_concat_bwd(const float* gcat, int Cu, int Cs, int n, float* gu, float* gs, hipStream_t s) {
  const int C4 = (Cu + Cs) / 4;
  const size_t wu = (size_t)(n / 2) * (n / 2) * (n / 2) * (Cu / 4);
  hipLaunchKernelGGL(k_up_bwd, dim3(grid_for(wu)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(gcat), C4, Cu / 4, n,
                     reinterpret_cast<float4*>(gu));
  const size_t V = (size_t)n * n * n;
  hipLaunchKernelGGL(k_cat_split, dim3(grid_for(V * (Cs / 4))), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(gcat), C4, Cu / 4, Cs / 4, V,
                     reinterpret_cast<float4*>(gs));
}

void pool_bwd_add(const float* gx, const float* add, int n, int C, float* gy, hipStream_t s) {
  const size_t work = (size_t)n * n * n * (C / 4);
  hipLaunchKernelGGL(k_pool_bwd_add, dim3(grid_for(work)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(gx), reinterpret_cast<const float4*>(add), n,
                     C / 4, reinterpret_cast<float4*>(gy));
}

void pad_input(const float* z, size_t V, float* zp, hipStream_t s) {
  hipLaunchKernelGGL(k_pad_input, dim3(grid_for(V * 8)), dim3(256), 0, s, z, V, zp);
}

}  // namespace d2ip
