// Conv entry points: mode dispatch, launch-shape helpers and the batched,
// deterministic reduction of all weight-gradient partials of an iteration.
#include "conv_impl.h"

namespace d2ip {
namespace {

// Sum of the strided values x[k * stride], k = first, first + step, ... < n,
// with eight loads in flight: eight running sums over interleaved subsets,
// combined in a fixed tree, so the order depends on n alone.
__device__ __forceinline__ float strided_sum(const float* x, long long stride, int first, int step,
                                             int n) {
  float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  int k = first;
  for (; k + 7 * step < n; k += 8 * step) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = x[(long long)(k + u * step) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += v[u];
  }
  float r[7];  // at most 7 left: all loads issued, then added in the same order
#pragma unroll
  for (int u = 0; u < 7; ++u) r[u] = k + u * step < n ? x[(long long)(k + u * step) * stride] : 0.f;
#pragma unroll
  for (int u = 0; u < 7; ++u)
    if (k + u * step < n) a[u] += r[u];
  return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// One block row per conv segment.  A block owns 64 consecutive partial
// elements (layout [co][tap][ci]); its 4 thread groups sum interleaved split
// subsets, combined in group order, so the sum order is fixed.
__global__ void k_grad_reduce(const GradSeg* __restrict__ segs, const float* part,
                              const float* partb, const double* dpart, float* grad,
                              long long istride) {
  __shared__ float sh[4][64];
  const GradSeg sg = segs[blockIdx.y];
  {
    const long long off = (long long)blockIdx.z * istride;  // group member
    part = ishift(part, off);
    partb = ishift(partb, off);
    dpart = ishift(dpart, off);
    grad = ishift(grad, off);
  }
  if (sg.kind == 1) {
    // column sums of double partials [splits][cout]: 8 columns per pass, 32
    // row groups (rows g, g + 32, ...) combined in group order; a group adds
    // its rows in row order, eight loads in flight
    __shared__ double shd[32][8];
    const double* D = dpart + sg.part_off;
    const int col = threadIdx.x & 7, rg = threadIdx.x >> 3;
    for (int k0 = blockIdx.x * 8; k0 < sg.cout; k0 += gridDim.x * 8) {
      const int k = k0 + col;
      double acc = 0.0;
      if (k < sg.cout) {
        int i = rg;
        for (; i + 7 * 32 < sg.splits; i += 8 * 32) {
          double v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) v[u] = D[(long long)(i + 32 * u) * sg.cout + k];
#pragma unroll
          for (int u = 0; u < 8; ++u) acc += v[u];
        }
        double r[7];  // at most 7 rows left
#pragma unroll
        for (int u = 0; u < 7; ++u)
          r[u] = i + 32 * u < sg.splits ? D[(long long)(i + 32 * u) * sg.cout + k] : 0.0;
#pragma unroll
        for (int u = 0; u < 7; ++u)
          if (i + 32 * u < sg.splits) acc += r[u];
      }
      shd[rg][col] = acc;
      __syncthreads();
      if (rg == 0 && k < sg.cout) {
        double t = 0.0;
        for (int q = 0; q < 32; ++q) t += shd[q][col];
        grad[sg.th_w + k] = (float)t;
      }
      __syncthreads();
    }
    return;
  }
  const int cout16 = (sg.cout + 15) & ~15;
  const long long per = (long long)cout16 * sg.taps * sg.cin;
  const int total = sg.cout * sg.taps * sg.cin;
  const float* P = part + sg.part_off;
  const int j = threadIdx.x & 63, q = threadIdx.x >> 6;
  for (int base = blockIdx.x * 64; base < total; base += gridDim.x * 64) {
    const int f = base + j;
    sh[q][j] = f < total ? strided_sum(P + f, per, q, 4, sg.splits) : 0.f;
    __syncthreads();
    if (q == 0 && f < total) {
      const float v = ((sh[0][j] + sh[1][j]) + sh[2][j]) + sh[3][j];
      const int ci = f % sg.cin;
      const int tap = (f / sg.cin) % sg.taps;
      const int co = f / (sg.cin * sg.taps);
      if (ci < sg.cin_real) grad[sg.th_w + ((long long)co * sg.cin_real + ci) * sg.taps + tap] = v;
    }
    __syncthreads();
  }
  if (blockIdx.x == 0) {
    // bias: 16 channels per pass, 16 split groups each, combined in group order
    const float* PB = partb + sg.partb_off;
    const int cl = threadIdx.x & 15, sgp = threadIdx.x >> 4;
    float* shb = &sh[0][0];
    for (int c0 = 0; c0 < sg.cout; c0 += 16) {
      const int co = c0 + cl;
      shb[sgp * 16 + cl] = co < sg.cout ? strided_sum(PB + co, cout16, sgp, 16, sg.splits) : 0.f;
      __syncthreads();
      if (sgp == 0 && co < sg.cout) {
        float t = 0.f;
        for (int k = 0; k < 16; ++k) t += shb[k * 16 + cl];
        grad[sg.th_b + co] = t;
      }
      __syncthreads();
    }
  }
}

}  // namespace

int conv_tiles(int n, int tile) { return conv_detail::spatial_tiles(n, tile); }

int conv_fwd_blocks(const ConvFwd& a) {
  return conv_detail::spatial_tiles(a.n, a.tile) * ((a.cout + a.bn - 1) / a.bn);
}

void conv_fwd(const ConvFwd& a, hipStream_t s) {
  switch (a.prec) {
    case PREC_BF16: conv_fwd_bf16(a, s); break;
    case PREC_BF16X3: conv_fwd_bf16x3(a, s); break;
    default: conv_fwd_f32(a, s); break;
  }
  if (a.ksplit > 1) conv_detail::launch_finish(a, s);
}

int conv_wgrad_groups(int taps, int ck) {
  const int cols = conv_detail::wg_cols(taps, ck);
  return (taps * ck + cols - 1) / cols;
}

void conv_wgrad(const ConvWgrad& a, hipStream_t s) {
  switch (a.prec) {
    case PREC_BF16: conv_wgrad_bf16(a, s); break;
    case PREC_BF16X3: conv_wgrad_bf16x3(a, s); break;
    default: conv_wgrad_f32(a, s); break;
  }
}

size_t conv_fwd_lds_bytes(int tile, int taps, int bn, int ck, int prec) {
  return conv_detail::fwd_lds_bytes(tile, taps, bn, ck, prec);
}

size_t conv_wgrad_lds_bytes(int tile, int taps, int ck, int prec) {
  return conv_detail::wg_lds_bytes(tile, taps, ck, prec);
}

void grad_reduce(const GradSeg* segs, int nsegs, int max_elems, const float* part,
                 const float* partb, const double* dpart, float* grad, int batch,
                 long long istride, hipStream_t s) {
  int bx = (max_elems + 63) / 64;
  if (bx > 1024) bx = 1024;
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(k_grad_reduce, dim3(bx, nsegs, batch), dim3(256), 0, s, segs, part, partb,
                     dpart, grad, istride);
}

}  // namespace d2ip
