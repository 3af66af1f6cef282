// Depthwise 3x3x3 convolution of the lightweight backbone's depthwise-
// separable convolutions (Sec. III-D): forward, input gradient and weight
// gradient on channels-last FP32 tensors [n^3][C], C a multiple of 4.  An
// output needs 27 multiply-adds per input value read, far too few for the
// matrix cores to matter: the operator is bound by HBM.  A block stages the
// halo of a voxel tile for KQ channel quads in LDS with coalesced loads (lanes
// run over the quads of a voxel first, so a wave reads whole 16*KQ-byte
// voxel rows), and each thread walks a z column of 4 outputs, so that every
// LDS value loaded serves the three output planes it touches.
#include "kernels.h"

namespace d2ip {
namespace {

constexpr int kDwParts = 28;  // per channel: 27 tap sums, then the bias sum

// Tile of a block with KQ channel quads per voxel: 256 / KQ (y, x) columns of
// 4 voxels along z, one thread per (column, quad).
template <int KQ>
struct DwGeo {
  static constexpr int TZ = 4, TY = KQ >= 4 ? 8 : 16, TX = 256 / KQ / TY;
  static constexpr int HY = TY + 2, HX = TX + 2, HALO = (TZ + 2) * HY * HX;
  static constexpr int SHIFT = KQ == 8 ? 3 : KQ == 4 ? 2 : KQ == 2 ? 1 : 0;
  static constexpr int NLOAD = (HALO * KQ + 255) / 256;  // halo loads per thread
};

// Physical block -> logical block, so that consecutive logical blocks (which
// are neighbouring tiles) run on the same XCD and share its L2: the hardware
// deals blocks round-robin to the 8 XCDs.  The grid is padded to a multiple
// of 8; logical indices past `nb` return at once.
__device__ __forceinline__ int dw_logical(int nb) {
  const int per = (nb + 7) >> 3;
  return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

template <int KQ>
struct DwTile {
  int z0, y0, x0;
  __device__ DwTile(int t, int n) {
    using G = DwGeo<KQ>;
    const int ntx = (n + G::TX - 1) / G::TX, nty = (n + G::TY - 1) / G::TY;
    x0 = (t % ntx) * G::TX;
    t /= ntx;
    y0 = (t % nty) * G::TY;
    z0 = (t / nty) * G::TZ;
  }
};

// Loads the halo of the tile at (z0, y0, x0) for channel quads
// c0/4 .. c0/4 + KQ - 1 (zeros outside the grid) and writes it to hal
// [(hz * HY + hy) * HX + hx][q].  Every load is issued before the first LDS
// write, from clamped (always valid) addresses.
// Loads are issued in batches of BATCH per thread (all of a batch before its
// LDS writes), which bounds the registers the staging holds.
template <int KQ, int BATCH>
__device__ __forceinline__ void dw_stage(float4* hal, const float* __restrict__ x, int n, int C,
                                         int c0, int z0, int y0, int x0) {
  using G = DwGeo<KQ>;
  constexpr int total = G::HALO * KQ;
#pragma unroll
  for (int i0 = 0; i0 < G::NLOAD; i0 += BATCH) {
    float4 r[BATCH];
    bool in[BATCH];
#pragma unroll
    for (int j = 0; j < BATCH; ++j) {
      const int e = min((int)threadIdx.x + 256 * (i0 + j), total - 1);
      const int q = e & (KQ - 1), p = e >> G::SHIFT;
      const int hx = p % G::HX, hy = (p / G::HX) % G::HY, hz = p / (G::HX * G::HY);
      const int gz = z0 + hz - 1, gy = y0 + hy - 1, gx = x0 + hx - 1;
      in[j] = (unsigned)gz < (unsigned)n && (unsigned)gy < (unsigned)n &&
              (unsigned)gx < (unsigned)n;
      const int cz = min(max(gz, 0), n - 1), cy = min(max(gy, 0), n - 1),
                cx = min(max(gx, 0), n - 1);
      r[j] = *reinterpret_cast<const float4*>(x + ((size_t)(cz * n + cy) * n + cx) * C + c0 +
                                              4 * q);
    }
#pragma unroll
    for (int j = 0; j < BATCH; ++j) {
      const int e = (int)threadIdx.x + 256 * (i0 + j);
      if (i0 + j < G::NLOAD && e < total) hal[e] = in[j] ? r[j] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
}

// Keeps the compiler from sinking the accumulation of a below this point
// (into the guarded stores), which would keep every LDS value loaded live.
__device__ __forceinline__ void dw_pin(float4& a) {
  asm volatile("" : "+v"(a.x), "+v"(a.y), "+v"(a.z), "+v"(a.w));
}

__device__ __forceinline__ void fma4(float4& a, const float4& k, const float4& v) {
  a.x += k.x * v.x;
  a.y += k.y * v.y;
  a.z += k.z * v.z;
  a.w += k.w * v.w;
}

// y[v][c] = b[c] + sum_tap w[c][tap] x[v + offset(tap)][c]; with flip the
// taps are taken in reverse (w[c][26 - tap]) and b is ignored, which makes
// the kernel the input gradient of the forward one.  Logical blocks:
// (voxel tile) fastest, then channel chunk of KQ quads.
template <int KQ>
__global__ __launch_bounds__(256, 3) void k_dw_fwd(const float* __restrict__ x,
                                                const float* __restrict__ w,
                                                const float* __restrict__ b, float* __restrict__ y,
                                                int n, int C, int ntiles, int flip) {
  using G = DwGeo<KQ>;
  __shared__ float4 hal[G::HALO * KQ];
  __shared__ float4 wl[27 * KQ];
  const int nchunks = C / (4 * KQ);
  const int L = dw_logical(ntiles * nchunks);
  if (L >= ntiles * nchunks) return;  // whole block: no barrier reached
  const int c0 = (L / ntiles) * 4 * KQ;
  const DwTile<KQ> t(L % ntiles, n);
  dw_stage<KQ, DwGeo<KQ>::NLOAD>(hal, x, n, C, c0, t.z0, t.y0, t.x0);
  if (threadIdx.x < 27 * KQ) {
    const int tap = threadIdx.x >> G::SHIFT, q = threadIdx.x & (KQ - 1);
    const float* wc = w + (size_t)(c0 + 4 * q) * 27 + (flip ? 26 - tap : tap);
    wl[threadIdx.x] = make_float4(wc[0], wc[27], wc[54], wc[81]);
  }
  __syncthreads();
  const int q = threadIdx.x & (KQ - 1), col = threadIdx.x >> G::SHIFT;
  const int tx = col % G::TX, ty = col / G::TX;
  float4 k[27];
#pragma unroll
  for (int i = 0; i < 27; ++i) k[i] = wl[i * KQ + q];
  const float4 b0 = (b && !flip) ? *reinterpret_cast<const float4*>(b + c0 + 4 * q)
                                 : make_float4(0.f, 0.f, 0.f, 0.f);
  float4 acc[G::TZ];
#pragma unroll
  for (int o = 0; o < G::TZ; ++o) acc[o] = b0;
  // halo plane pz feeds output plane o = pz - dz through tap (dz, dy, dx)
#pragma unroll
  for (int pz = 0; pz < G::TZ + 2; ++pz)
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const float4 v = hal[((pz * G::HY + ty + dy) * G::HX + tx + dx) * KQ + q];
#pragma unroll
        for (int dz = 0; dz < 3; ++dz) {
          const int o = pz - dz;
          if (o >= 0 && o < G::TZ) fma4(acc[o], k[(dz * 3 + dy) * 3 + dx], v);
        }
        // one plane's nine LDS values in registers at a time
        if (dy == 2 && dx == 2)
#pragma unroll
          for (int o = 0; o < G::TZ; ++o) dw_pin(acc[o]);
      }
  const int gy = t.y0 + ty, gx = t.x0 + tx;
  if (gy >= n || gx >= n) return;
#pragma unroll
  for (int o = 0; o < G::TZ; ++o)
    if (t.z0 + o < n)
      *reinterpret_cast<float4*>(y + ((size_t)((t.z0 + o) * n + gy) * n + gx) * C + c0 + 4 * q) =
          acc[o];
}

// Weight-gradient partials: the block of (y, x) tile `txy`, z group `zg`
// (zs consecutive z tiles) and channel chunk sums, over its voxels v,
// gy[v][c] x[v + offset(tap)][c] (27 taps) and gy[v][c] (bias) and writes
// them to part[(c * 28 + k) * nP + txy + ntxy * zg], nP = ntxy * nzg: one
// partial per (y, x) tile and z group, column-major so that the reduction
// reads them contiguously.  Threads sum in a fixed order, lanes of equal quad
// by a fixed butterfly, waves in index order.
template <int KQ>
__global__ __launch_bounds__(256, 2) void k_dw_wgrad(const float* __restrict__ x,
                                                  const float* __restrict__ gyv,
                                                  float* __restrict__ part, int n, int C,
                                                  int ntxy, int nzg, int zs) {
  using G = DwGeo<KQ>;
  __shared__ float4 hal[G::HALO * KQ];
  static_assert(G::HALO * KQ >= 4 * kDwParts * KQ, "reduction buffer fits in the halo");
  const int nchunks = C / (4 * KQ);
  const int nb = ntxy * nzg * nchunks;
  const int L = dw_logical(nb);
  if (L >= nb) return;  // whole block
  const int txy = L % ntxy, zg = (L / ntxy) % nzg, c0 = (L / (ntxy * nzg)) * 4 * KQ;
  const int ntz = (n + G::TZ - 1) / G::TZ;
  const int q = threadIdx.x & (KQ - 1), col = threadIdx.x >> G::SHIFT;
  const int tx = col % G::TX, ty = col / G::TX;
  const DwTile<KQ> t0(txy, n);  // z0 = 0: the (y, x) origin
  const int gy = t0.y0 + ty, gx = t0.x0 + tx;
  const bool colin = gy < n && gx < n;
  const int cy = min(gy, n - 1), cx = min(gx, n - 1);
  float4 acc[kDwParts];
#pragma unroll
  for (int i = 0; i < kDwParts; ++i) acc[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  const int zt_end = min(ntz, (zg + 1) * zs);
  for (int zt = zg * zs; zt < zt_end; ++zt) {
    const int z0 = zt * G::TZ;
    float4 g[G::TZ];
#pragma unroll
    for (int o = 0; o < G::TZ; ++o) {
      const int z = min(z0 + o, n - 1);
      g[o] = *reinterpret_cast<const float4*>(gyv + ((size_t)(z * n + cy) * n + cx) * C + c0 +
                                              4 * q);
    }
    if (zt > zg * zs) __syncthreads();  // the previous tile's halo is consumed
    dw_stage<KQ, 4>(hal, x, n, C, c0, z0, t0.y0, t0.x0);
#pragma unroll
    for (int o = 0; o < G::TZ; ++o)
      if (!colin || z0 + o >= n) g[o] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
#pragma unroll
    for (int pz = 0; pz < G::TZ + 2; ++pz)
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          const float4 v = hal[((pz * G::HY + ty + dy) * G::HX + tx + dx) * KQ + q];
#pragma unroll
          for (int dz = 0; dz < 3; ++dz) {
            const int o = pz - dz;
            if (o >= 0 && o < G::TZ) fma4(acc[(dz * 3 + dy) * 3 + dx], g[o], v);
          }
          if (dy == 2 && dx == 2) __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
    for (int o = 0; o < G::TZ; ++o) fma4(acc[27], make_float4(1.f, 1.f, 1.f, 1.f), g[o]);
  }
  // lanes of one quad: butterfly over lane offsets 32 .. KQ
#pragma unroll
  for (int i = 0; i < kDwParts; ++i)
#pragma unroll
    for (int off = 32; off >= KQ; off >>= 1) {
      acc[i].x += __shfl_xor(acc[i].x, off, 64);
      acc[i].y += __shfl_xor(acc[i].y, off, 64);
      acc[i].z += __shfl_xor(acc[i].z, off, 64);
      acc[i].w += __shfl_xor(acc[i].w, off, 64);
    }
  __syncthreads();  // halo no longer read: reuse it for the wave sums
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane < KQ)
#pragma unroll
    for (int i = 0; i < kDwParts; ++i) hal[(wave * kDwParts + i) * KQ + lane] = acc[i];
  __syncthreads();
  if (threadIdx.x < kDwParts * KQ) {
    const int i = threadIdx.x / KQ, qq = threadIdx.x & (KQ - 1);
    float4 s = hal[i * KQ + qq];
#pragma unroll
    for (int w2 = 1; w2 < 4; ++w2) {
      const float4 v = hal[(w2 * kDwParts + i) * KQ + qq];
      s.x += v.x;
      s.y += v.y;
      s.z += v.z;
      s.w += v.w;
    }
    const size_t nP = (size_t)ntxy * nzg, P = txy + (size_t)ntxy * zg;
    const int c = c0 + 4 * qq;
    part[((size_t)(c + 0) * kDwParts + i) * nP + P] = s.x;
    part[((size_t)(c + 1) * kDwParts + i) * nP + P] = s.y;
    part[((size_t)(c + 2) * kDwParts + i) * nP + P] = s.z;
    part[((size_t)(c + 3) * kDwParts + i) * nP + P] = s.w;
  }
}

// gw[c][tap] and gb[c] from the partials: one wave per (c, k), lanes over the
// partials with eight loads in flight, then a fixed butterfly.
__global__ __launch_bounds__(256) void k_dw_wreduce(const float* __restrict__ part, int nP, int C,
                                                    float* gw, float* gb) {
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (e >= C * kDwParts) return;  // whole wave
  const float* p = part + (size_t)e * nP;
  float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  int j = lane;
  for (; j + 7 * 64 < nP; j += 8 * 64) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[j + 64 * u];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += v[u];
  }
#pragma unroll
  for (int u = 0; u < 7; ++u)
    if (j + 64 * u < nP) a[u] += p[j + 64 * u];
  const float s = wave_sum(((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7])));
  if (lane == 0) {
    const int c = e / kDwParts, k = e - c * kDwParts;
    if (k < 27) {
      if (gw) gw[(size_t)c * 27 + k] = s;
    } else if (gb) {
      gb[c] = s;
    }
  }
}

// Channel quads per block: the largest power of two <= 8 dividing C / 4.
int dw_kq(int C) {
  const int c4 = C / 4;
  return c4 % 8 == 0 ? 8 : c4 % 4 == 0 ? 4 : c4 % 2 == 0 ? 2 : 1;
}

template <int KQ>
int dw_tiles_kq(int n) {
  using G = DwGeo<KQ>;
  return ((n + G::TX - 1) / G::TX) * ((n + G::TY - 1) / G::TY) * ((n + G::TZ - 1) / G::TZ);
}

template <int KQ>
void dw_shape(int n, int C, int* ntxy, int* nzg, int* zs) {
  using G = DwGeo<KQ>;
  *ntxy = ((n + G::TX - 1) / G::TX) * ((n + G::TY - 1) / G::TY);
  const int ntz = (n + G::TZ - 1) / G::TZ, nch = C / (4 * KQ);
  // fewest partials that still give about 1024 blocks
  int s = 1;
  while (2 * s <= ntz && (long long)*ntxy * ((ntz + 2 * s - 1) / (2 * s)) * nch >= 1024) s *= 2;
  *zs = s;
  *nzg = (ntz + s - 1) / s;
}

void dw_shape_any(int n, int C, int* ntxy, int* nzg, int* zs) {
  switch (dw_kq(C)) {
    case 8: dw_shape<8>(n, C, ntxy, nzg, zs); break;
    case 4: dw_shape<4>(n, C, ntxy, nzg, zs); break;
    case 2: dw_shape<2>(n, C, ntxy, nzg, zs); break;
    default: dw_shape<1>(n, C, ntxy, nzg, zs); break;
  }
}

template <int KQ>
void launch_fwd(const float* x, const float* w, const float* b, float* y, int n, int C, bool flip,
                hipStream_t s) {
  const int nt = dw_tiles_kq<KQ>(n), nb = nt * (C / (4 * KQ));
  hipLaunchKernelGGL(k_dw_fwd<KQ>, dim3((nb + 7) / 8 * 8), dim3(256), 0, s, x, w, b, y, n, C, nt,
                     flip ? 1 : 0);
}

template <int KQ>
void launch_wgrad(const float* x, const float* gy, float* part, int n, int C, hipStream_t s) {
  int ntxy, nzg, zs;
  dw_shape<KQ>(n, C, &ntxy, &nzg, &zs);
  const int nb = ntxy * nzg * (C / (4 * KQ));
  hipLaunchKernelGGL(k_dw_wgrad<KQ>, dim3((nb + 7) / 8 * 8), dim3(256), 0, s, x, gy, part, n, C,
                     ntxy, nzg, zs);
}

}  // namespace

size_t dw_partials(int n, int C) {
  int ntxy, nzg, zs;
  dw_shape_any(n, C, &ntxy, &nzg, &zs);
  return (size_t)ntxy * nzg * C * kDwParts;
}

void dw_forward(const float* x, const float* w, const float* b, float* y, int n, int C, bool flip,
                hipStream_t s) {
  switch (dw_kq(C)) {
    case 8: launch_fwd<8>(x, w, b, y, n, C, flip, s); break;
    case 4: launch_fwd<4>(x, w, b, y, n, C, flip, s); break;
    case 2: launch_fwd<2>(x, w, b, y, n, C, flip, s); break;
    default: launch_fwd<1>(x, w, b, y, n, C, flip, s); break;
  }
}

void dw_wgrad(const float* x, const float* gy, float* part, float* gw, float* gb, int n, int C,
              hipStream_t s) {
  switch (dw_kq(C)) {
    case 8: launch_wgrad<8>(x, gy, part, n, C, s); break;
    case 4: launch_wgrad<4>(x, gy, part, n, C, s); break;
    case 2: launch_wgrad<2>(x, gy, part, n, C, s); break;
    default: launch_wgrad<1>(x, gy, part, n, C, s); break;
  }
  int ntxy, nzg, zs;
  dw_shape_any(n, C, &ntxy, &nzg, &zs);
  hipLaunchKernelGGL(k_dw_wreduce, dim3((C * kDwParts + 3) / 4), dim3(256), 0, s, part,
                     ntxy * nzg, C, gw, gb);
}

}  // namespace d2ip
