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
// A block takes kAttU coarse voxels: their pooled skip and gating rows and
// the pre-activations a go through LDS, the per-voxel sums run in fixed
// order.  The backward recomputes a and alpha, writes gx and gg and one
// partial of every parameter gradient per block, reduced in FP64 in block
// order by a second kernel (deterministic).
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

// gt = gout * mask * dout/dt; gx[v][c] = gt w[c]; one partial per block of
// (sum_v gt x[v][c], sum_v gt) over the block's voxels, reduced across the
// block's threads in a fixed order.
constexpr int kHeadMaxC = 256;
__global__ __launch_bounds__(256) void k_head_bwd(const float* __restrict__ x,
                                                  const float* __restrict__ w,
                                                  const float* __restrict__ b,
                                                  const float* __restrict__ mask,
                                                  const float* __restrict__ gout, size_t V, int C,
                                                  int sig, float* __restrict__ gx,
                                                  double* __restrict__ part) {
  __shared__ float red[256][5];
  const int C4 = C / 4;
  // thread t accumulates channel quad (t % C4) over the voxels v = v0 + r,
  // r = t / C4, t / C4 + R, ...  (R = 256 / C4 voxel lanes)
  const int R = 256 / C4, q = threadIdx.x % C4, r = threadIdx.x / C4;
  const size_t per = (V + gridDim.x - 1) / gridDim.x;
  const size_t v0 = blockIdx.x * per, v1 = min(V, v0 + per);
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  float accb = 0.f;
  const float4 wq = reinterpret_cast<const float4*>(w)[q];
  if (r < R) {
    for (size_t v = v0 + r; v < v1; v += R) {
      float gt = gout[v];
      if (mask) gt *= mask[v];
      if (sig) {
        const float s = 1.f / (1.f + expf(-head_t(x, w, b[0], C, v)));
        gt *= 2.f * s * (1.f - s);
      }
      const float4 xv = reinterpret_cast<const float4*>(x + v * C)[q];
      acc.x += gt * xv.x;
      acc.y += gt * xv.y;
      acc.z += gt * xv.z;
      acc.w += gt * xv.w;
      if (q == 0) accb += gt;
      if (gx)
        reinterpret_cast<float4*>(gx + v * C)[q] =
            make_float4(gt * wq.x, gt * wq.y, gt * wq.z, gt * wq.w);
    }
  }
  red[threadIdx.x][0] = acc.x;
  red[threadIdx.x][1] = acc.y;
  red[threadIdx.x][2] = acc.z;
  red[threadIdx.x][3] = acc.w;
  red[threadIdx.x][4] = accb;
  __syncthreads();
  if (threadIdx.x < C4) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    double sb = 0.0;
    for (int rr = 0; rr < R; ++rr) {
      const int t = rr * C4 + threadIdx.x;
      for (int e = 0; e < 4; ++e) s[e] += red[t][e];
      if (threadIdx.x == 0) sb += red[t][4];
    }
    double* p = part + (size_t)blockIdx.x * (C + 1);
    for (int e = 0; e < 4; ++e) p[4 * threadIdx.x + e] = s[e];
    if (threadIdx.x == 0) p[C] = sb;
  }
}

// out[i] = sum over blocks k of part[k][i] (fixed order), i < n
__global__ void k_part_sum(const double* __restrict__ part, int nblocks, int n,
                           float* __restrict__ out0, int n0, float* __restrict__ out1) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < nblocks; ++k) s += part[(size_t)k * n + i];
  if (i < n0) {
    if (out0) out0[i] = (float)s;
  } else if (out1) {
    out1[i - n0] = (float)s;
  }
}

// ---- attention unit ---------------------------------------------------------

constexpr int kAttU = 32;      // coarse voxels per block
constexpr int kAttMaxC = 64;   // skip channels
constexpr int kAttMaxCu = 128; // gating channels

struct AttArgs {
  const float *x, *g, *wx, *wg, *b, *psi, *bpsi;
  int n, c, cu;
};

// Stage the block's pooled skip rows xs[u][c], gating rows gg[u][cu] and
// pre-activations a[u][c]; returns the block's coarse voxel count.
__device__ int att_stage(const AttArgs& A, int u0, float* xs, float* gs, float* as) {
  const int m = A.n / 2;
  const int mc = m * m * m;
  const int nu = min(kAttU, mc - u0);
  const int c4 = A.c / 4, cu4 = A.cu / 4;
  for (int i = threadIdx.x; i < nu * c4; i += blockDim.x) {
    const int u = i / c4, q = i - u * c4;
    const int cu_ = u0 + u;
    const int xx = cu_ % m, yy = (cu_ / m) % m, zz = cu_ / (m * m);
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int fz = 2 * zz + (k >> 2), fy = 2 * yy + ((k >> 1) & 1), fx = 2 * xx + (k & 1);
      const float4 v =
          reinterpret_cast<const float4*>(A.x + ((size_t)(fz * A.n + fy) * A.n + fx) * A.c)[q];
      s.x += v.x;
      s.y += v.y;
      s.z += v.z;
      s.w += v.w;
    }
    float* d = xs + u * A.c + 4 * q;
    d[0] = 0.125f * s.x;
    d[1] = 0.125f * s.y;
    d[2] = 0.125f * s.z;
    d[3] = 0.125f * s.w;
  }
  for (int i = threadIdx.x; i < nu * cu4; i += blockDim.x) {
    const int u = i / cu4, q = i - u * cu4;
    const float4 v = reinterpret_cast<const float4*>(A.g + (size_t)(u0 + u) * A.cu)[q];
    float* d = gs + u * A.cu + 4 * q;
    d[0] = v.x;
    d[1] = v.y;
    d[2] = v.z;
    d[3] = v.w;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nu * A.c; i += blockDim.x) {
    const int u = i / A.c, k = i - u * A.c;
    float t = A.b[k];
    const float* wr = A.wx + (size_t)k * A.c;
    const float* xr = xs + u * A.c;
    for (int j = 0; j < A.c; ++j) t += wr[j] * xr[j];
    const float* gr = A.wg + (size_t)k * A.cu;
    const float* gsr = gs + u * A.cu;
    for (int j = 0; j < A.cu; ++j) t += gr[j] * gsr[j];
    as[u * A.c + k] = t;
  }
  __syncthreads();
  return nu;
}

__device__ __forceinline__ float att_alpha(const AttArgs& A, const float* as, int u) {
  float s = A.bpsi[0];
  const float* ar = as + u * A.c;
  for (int k = 0; k < A.c; ++k) s += A.psi[k] * fmaxf(ar[k], 0.f);
  return 1.f / (1.f + expf(-s));
}

__global__ __launch_bounds__(256) void k_att_fwd(AttArgs A, float* __restrict__ y,
                                                 float* __restrict__ alpha) {
  __shared__ float xs[kAttU * kAttMaxC];
  __shared__ float gs[kAttU * kAttMaxCu];
  __shared__ float as[kAttU * kAttMaxC];
  __shared__ float al[kAttU];
  const int m = A.n / 2;
  const int u0 = blockIdx.x * kAttU;
  const int nu = att_stage(A, u0, xs, gs, as);
  if (threadIdx.x < nu) {
    al[threadIdx.x] = att_alpha(A, as, threadIdx.x);
    if (alpha) alpha[u0 + threadIdx.x] = al[threadIdx.x];
  }
  __syncthreads();
  const int c4 = A.c / 4;
  for (int i = threadIdx.x; i < nu * 8 * c4; i += blockDim.x) {
    const int q = i % c4, ch = (i / c4) & 7, u = i / (8 * c4);
    const int cu_ = u0 + u;
    const int xx = cu_ % m, yy = (cu_ / m) % m, zz = cu_ / (m * m);
    const int fz = 2 * zz + (ch >> 2), fy = 2 * yy + ((ch >> 1) & 1), fx = 2 * xx + (ch & 1);
    const size_t o = ((size_t)(fz * A.n + fy) * A.n + fx) * A.c;
    const float4 v = reinterpret_cast<const float4*>(A.x + o)[q];
    const float a = al[u];
    reinterpret_cast<float4*>(y + o)[q] = make_float4(a * v.x, a * v.y, a * v.z, a * v.w);
  }
}

// Parameter-gradient partial layout per block: wx [c][c], wg [c][cu], b [c],
// psi [c], bpsi [1].
__host__ __device__ inline int att_nparams(int c, int cu) { return c * c + c * cu + 2 * c + 1; }

__global__ __launch_bounds__(256) void k_att_bwd(AttArgs A, const float* __restrict__ gy,
                                                 float* __restrict__ gx, float* __restrict__ gg,
                                                 float* __restrict__ part) {
  __shared__ float xs[kAttU * kAttMaxC];
  __shared__ float gs[kAttU * kAttMaxCu];
  __shared__ float as[kAttU * kAttMaxC];   // a, then ga = dL/da
  __shared__ float al[kAttU], gt[kAttU];
  const int m = A.n / 2;
  const int u0 = blockIdx.x * kAttU;
  const int nu = att_stage(A, u0, xs, gs, as);
  const int c = A.c, cu = A.cu, c4 = c / 4;
  // dL/dalpha[u] = sum over the 8 children and channels of gy * x (fixed order)
  if (threadIdx.x < nu) {
    const int u = threadIdx.x;
    const float a = att_alpha(A, as, u);
    const int cu_ = u0 + u;
    const int xx = cu_ % m, yy = (cu_ / m) % m, zz = cu_ / (m * m);
    float s = 0.f;
    for (int ch = 0; ch < 8; ++ch) {
      const int fz = 2 * zz + (ch >> 2), fy = 2 * yy + ((ch >> 1) & 1), fx = 2 * xx + (ch & 1);
      const size_t o = ((size_t)(fz * A.n + fy) * A.n + fx) * c;
      for (int q = 0; q < c4; ++q) {
        const float4 gv = reinterpret_cast<const float4*>(gy + o)[q];
        const float4 xv = reinterpret_cast<const float4*>(A.x + o)[q];
        s += gv.x * xv.x + gv.y * xv.y + gv.z * xv.z + gv.w * xv.w;
      }
    }
    al[u] = a;
    gt[u] = s * a * (1.f - a);  // through the sigmoid
  }
  __syncthreads();
  // psi and bpsi partials use relu(a) before a is overwritten by ga
  float* P = part + (size_t)blockIdx.x * att_nparams(c, cu);
  const int o_wg = c * c, o_b = o_wg + c * cu, o_psi = o_b + c, o_bpsi = o_psi + c;
  for (int k = threadIdx.x; k < c; k += blockDim.x) {
    float s = 0.f;
    for (int u = 0; u < nu; ++u) s += fmaxf(as[u * c + k], 0.f) * gt[u];
    P[o_psi + k] = s;
  }
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int u = 0; u < nu; ++u) s += gt[u];
    P[o_bpsi] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nu * c; i += blockDim.x) {
    const int u = i / c, k = i - u * c;
    as[i] = as[i] > 0.f ? A.psi[k] * gt[u] : 0.f;  // ga (ReLU derivative 0 at 0)
  }
  __syncthreads();
  // parameter partials: wx[k][j] = sum_u ga[u][k] xs[u][j], wg, b
  for (int i = threadIdx.x; i < c * c; i += blockDim.x) {
    const int k = i / c, j = i - k * c;
    float s = 0.f;
    for (int u = 0; u < nu; ++u) s += as[u * c + k] * xs[u * c + j];
    P[i] = s;
  }
  for (int i = threadIdx.x; i < c * cu; i += blockDim.x) {
    const int k = i / cu, j = i - k * cu;
    float s = 0.f;
    for (int u = 0; u < nu; ++u) s += as[u * c + k] * gs[u * cu + j];
    P[o_wg + i] = s;
  }
  for (int k = threadIdx.x; k < c; k += blockDim.x) {
    float s = 0.f;
    for (int u = 0; u < nu; ++u) s += as[u * c + k];
    P[o_b + k] = s;
  }
  // gating gradient gg[u][j] = sum_k wg[k][j] ga[u][k]
  if (gg)
    for (int i = threadIdx.x; i < nu * cu; i += blockDim.x) {
      const int u = i / cu, j = i - u * cu;
      float s = 0.f;
      for (int k = 0; k < c; ++k) s += A.wg[(size_t)k * cu + j] * as[u * c + k];
      gg[(size_t)(u0 + u) * cu + j] = s;
    }
  // skip gradient gx[v][j] = alpha gy[v][j] + (1/8) sum_k wx[k][j] ga[u][k]
  if (gx) {
    // the pooled part per (u, j) first, into xs (no longer needed)
    __syncthreads();
    for (int i = threadIdx.x; i < nu * c; i += blockDim.x) {
      const int u = i / c, j = i - u * c;
      float s = 0.f;
      for (int k = 0; k < c; ++k) s += A.wx[(size_t)k * c + j] * as[u * c + k];
      xs[i] = 0.125f * s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nu * 8 * c4; i += blockDim.x) {
      const int q = i % c4, ch = (i / c4) & 7, u = i / (8 * c4);
      const int cu_ = u0 + u;
      const int xx = cu_ % m, yy = (cu_ / m) % m, zz = cu_ / (m * m);
      const int fz = 2 * zz + (ch >> 2), fy = 2 * yy + ((ch >> 1) & 1), fx = 2 * xx + (ch & 1);
      const size_t o = ((size_t)(fz * A.n + fy) * A.n + fx) * c;
      const float4 gv = reinterpret_cast<const float4*>(gy + o)[q];
      const float a = al[u];
      const float* p = xs + u * c + 4 * q;
      reinterpret_cast<float4*>(gx + o)[q] =
          make_float4(a * gv.x + p[0], a * gv.y + p[1], a * gv.z + p[2], a * gv.w + p[3]);
    }
  }
}

// out[i] = sum over blocks of fpart[k][i] in FP64, block order, split into
// the parameter tensors
__global__ void k_att_reduce(const float* __restrict__ part, int nblocks, int c, int cu,
                             float* gwx, float* gwg, float* gb, float* gpsi, float* gbpsi) {
  const int np = att_nparams(c, cu);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  double s = 0.0;
  for (int k = 0; k < nblocks; ++k) s += part[(size_t)k * np + i];
  const int o_wg = c * c, o_b = o_wg + c * cu, o_psi = o_b + c, o_bpsi = o_psi + c;
  float* dst = nullptr;
  int j = 0;
  if (i < o_wg) {
    dst = gwx;
    j = i;
  } else if (i < o_b) {
    dst = gwg;
    j = i - o_wg;
  } else if (i < o_psi) {
    dst = gb;
    j = i - o_b;
  } else if (i < o_bpsi) {
    dst = gpsi;
    j = i - o_psi;
  } else {
    dst = gbpsi;
    j = 0;
  }
  if (dst) dst[j] = (float)s;
}

int head_blocks(size_t V) {
  size_t b = (V + 2047) / 2048;
  return (int)std::max<size_t>(1, std::min<size_t>(b, 1024));
}

}  // namespace

int att_max_c() { return kAttMaxC; }
int att_max_cu() { return kAttMaxCu; }
int head_max_c() { return kHeadMaxC; }

size_t head_scratch_bytes(size_t V, int C) {
  return (size_t)head_blocks(V) * (C + 1) * sizeof(double);
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
  if (gw || gb)
    hipLaunchKernelGGL(k_part_sum, dim3((C + 1 + 255) / 256), dim3(256), 0, s, part, nb, C + 1,
                       gw, C, gb);
}

int att_blocks(int n) {
  const int m = n / 2;
  return (m * m * m + kAttU - 1) / kAttU;
}

size_t att_scratch_bytes(int n, int c, int cu) {
  return (size_t)att_blocks(n) * att_nparams(c, cu) * sizeof(float);
}

void att_forward(const float* x, const float* g, const float* wx, const float* wg, const float* b,
                 const float* psi, const float* bpsi, float* y, float* alpha, int n, int c, int cu,
                 hipStream_t s) {
  AttArgs A{x, g, wx, wg, b, psi, bpsi, n, c, cu};
  hipLaunchKernelGGL(k_att_fwd, dim3(att_blocks(n)), dim3(256), 0, s, A, y, alpha);
}

void att_backward(const float* x, const float* g, const float* wx, const float* wg,
                  const float* b, const float* psi, const float* bpsi, const float* gy,
                  float* gx, float* gg, float* gwx, float* gwg, float* gb, float* gpsi,
                  float* gbpsi, int n, int c, int cu, void* scratch, hipStream_t s) {
  AttArgs A{x, g, wx, wg, b, psi, bpsi, n, c, cu};
  const int nb = att_blocks(n);
  float* part = reinterpret_cast<float*>(scratch);
  hipLaunchKernelGGL(k_att_bwd, dim3(nb), dim3(256), 0, s, A, gy, gx, gg, part);
  const int np = att_nparams(c, cu);
  hipLaunchKernelGGL(k_att_reduce, dim3((np + 255) / 256), dim3(256), 0, s, part, nb, c, cu, gwx,
                     gwg, gb, gpsi, gbpsi);
}

}  // namespace d2ip
