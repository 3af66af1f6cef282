// Conv entry points: mode dispatch, launch-shape helpers and the deterministic
// reduction of weight-gradient partials.
#include "conv_impl.h"

namespace d2ip {
namespace {

__global__ void k_wgrad_reduce(const float* __restrict__ part, const float* __restrict__ partb,
                               int splits, int cout, int taps, int cin, int cin_real, float* gw,
                               float* gb) {
  const int cout16 = (cout + 15) & ~15;
  const size_t per = (size_t)cout16 * taps * cin;
  const size_t total = (size_t)cout * taps * cin;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int ci = (int)(i % cin);
    const int tap = (int)((i / cin) % taps);
    const int co = (int)(i / ((size_t)cin * taps));
    if (ci >= cin_real) continue;
    float s = 0.f;
    for (int k = 0; k < splits; ++k) s += part[k * per + i];
    gw[((size_t)co * cin_real + ci) * taps + tap] = s;
  }
  if (gb && blockIdx.x == 0) {
    for (int co = threadIdx.x; co < cout; co += blockDim.x) {
      float s = 0.f;
      for (int k = 0; k < splits; ++k) s += partb[(size_t)k * cout16 + co];
      gb[co] = s;
    }
  }
}

}  // namespace

int conv_fwd_blocks(const ConvFwd& a) {
  const int bn = conv_detail::pick_bn(a.cout);
  return conv_detail::spatial_tiles(a.n, a.tile) * ((a.cout + bn - 1) / bn);
}

void conv_fwd(const ConvFwd& a, hipStream_t s) {
  switch (a.prec) {
    case PREC_BF16: conv_fwd_bf16(a, s); break;
    case PREC_BF16X3: conv_fwd_bf16x3(a, s); break;
    default: conv_fwd_f32(a, s); break;
  }
}

int conv_wgrad_splits(int n, int cin, int cout, int tile) {
  const int per = (cin / conv_detail::pick_ck(cin)) * ((cout + 15) / 16);
  const int tiles = conv_detail::spatial_tiles(n, tile);
  int s = (1024 + per - 1) / per;
  if (s > tiles) s = tiles;
  if (s < 1) s = 1;
  return s;
}

size_t conv_wgrad_part_floats(int n, int cin, int cout, int taps, int tile) {
  const int s = conv_wgrad_splits(n, cin, cout, tile);
  return (size_t)s * ((cout + 15) & ~15) * taps * cin;
}

void conv_wgrad(const ConvWgrad& a, hipStream_t s) {
  switch (a.prec) {
    case PREC_BF16: conv_wgrad_bf16(a, s); break;
    case PREC_BF16X3: conv_wgrad_bf16x3(a, s); break;
    default: conv_wgrad_f32(a, s); break;
  }
}

void wgrad_reduce(const float* part, const float* partb, int splits, int cout, int taps, int cin,
                  int cin_real, float* gw, float* gb, hipStream_t s) {
  const size_t total = (size_t)cout * taps * cin;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(blocks), dim3(256), 0, s, part, partb, splits, cout,
                     taps, cin, cin_real, gw, gb);
}

}  // namespace d2ip
