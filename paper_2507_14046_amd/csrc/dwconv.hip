// Depthwise 3x3x3 convolution of the lightweight backbone's depthwise-
// separable convolutions (Sec. III-D): forward, input gradient and weight
// gradient on channels-last FP32 tensors [n^3][C], C a multiple of 4.  An
// output value needs 27 multiply-adds per 8 bytes of HBM traffic (its input
// read once, itself written once): a per-channel stencil, not a contraction,
// so the matrix cores do not apply, and the FP32 vector rate puts the
// arithmetic within reach of the HBM time.  A block takes a (y, x) tile for
// KQ channel quads and streams a segment of z planes through LDS, loading the
// halo plane with coalesced float4 loads (lanes run over the quads of a voxel
// first) while the previous planes are computed; each thread walks one z
// column, and every value it reads from LDS serves the three output planes it
// touches.
#include "kernels.h"

namespace d2ip {
namespace {

constexpr int kDwParts = 28;  // per channel: 27 tap sums, then the bias sum
constexpr int kDwFwdGroup = 4;  // halo planes per group: forward / input gradient
constexpr int kDwWgGroup = 4;   // weight gradient (its accumulators leave fewer registers)
constexpr int kDwRedChunk = 4;  // accumulators per step of the weight gradient's block sum

// A block covers a (y, x) tile of 256 / KQ columns for KQ channel quads and
// walks a segment of z planes; one thread per (column, quad).  A halo plane
// holds (TY + 2) x (TX + 2) positions x KQ quads.
template <int KQ>
struct DwGeo {
  static constexpr int TY = KQ >= 4 ? 8 : 16, TX = 256 / KQ / TY;
  static constexpr int HY = TY + 2, HX = TX + 2, PLANE = HY * HX * KQ;  // float4
  static constexpr int SHIFT = KQ == 8 ? 3 : KQ == 4 ? 2 : KQ == 2 ? 1 : 0;
  static constexpr int NL = (PLANE + 255) / 256;  // halo-plane loads per thread
};

// Physical block -> logical block, so that consecutive logical blocks (which
// are neighbouring tiles) run on the same XCD and share its L2: the hardware
// deals blocks round-robin to the 8 XCDs.  The grid is padded to a multiple
// of 8; logical indices past `nb` return at once.
__device__ __forceinline__ int dw_logical(int nb) {
  const int per = (nb + 7) >> 3;
  return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

// Block coordinates: (y, x) tile fastest, then z segment, then channel chunk.
template <int KQ>
struct DwBlock {
  int x0, y0, zb, ze, sg, txy, c0;
  __device__ DwBlock(int L, int n, int ntxy, int nseg, int seglen) {
    using G = DwGeo<KQ>;
    txy = L % ntxy;
    sg = (L / ntxy) % nseg;
    c0 = (L / (ntxy * nseg)) * 4 * KQ;
    const int ntx = (n + G::TX - 1) / G::TX;
    x0 = (txy % ntx) * G::TX;
    y0 = (txy / ntx) * G::TY;
    zb = sg * seglen;
    ze = min(n, zb + seglen);
  }
};

// The thread's share of a halo plane: element e = tid + 256 i of the plane
// (position (hy, hx), quad q) sits at a fixed (y, x) for every plane, so its
// clamped in-plane offset and in-grid flag are computed once.
template <int KQ>
struct DwStager {
  using G = DwGeo<KQ>;
  size_t off[G::NL];
  bool xyin[G::NL];
  size_t plane_stride;
  int n;
  __device__ DwStager(int n_, int C, int c0, int y0, int x0) : n(n_) {
    plane_stride = (size_t)n * n * C;
#pragma unroll
    for (int i = 0; i < G::NL; ++i) {
      const int e = min((int)threadIdx.x + 256 * i, G::PLANE - 1);
      const int q = e & (KQ - 1), p = e >> G::SHIFT;
      const int gy = y0 + p / G::HX - 1, gx = x0 + p % G::HX - 1;
      xyin[i] = (unsigned)gy < (unsigned)n && (unsigned)gx < (unsigned)n;
      off[i] = ((size_t)min(max(gy, 0), n - 1) * n + min(max(gx, 0), n - 1)) * C + c0 + 4 * q;
    }
  }
  // Issue the loads of plane z (clamped into the grid; always valid).
  __device__ __forceinline__ void load(const float* __restrict__ x, int z, float4 (&r)[G::NL]) const {
    const float* base = x + (size_t)min(max(z, 0), n - 1) * plane_stride;
#pragma unroll
    for (int i = 0; i < G::NL; ++i) r[i] = *reinterpret_cast<const float4*>(base + off[i]);
  }
  // Write plane z's loaded values to LDS (zeros outside the grid).
  __device__ __forceinline__ void store(float4* hal, int z, const float4 (&r)[G::NL]) const {
    const bool zin = (unsigned)z < (unsigned)n;
#pragma unroll
    for (int i = 0; i < G::NL; ++i) {
      const int e = (int)threadIdx.x + 256 * i;
      if (e < G::PLANE) hal[e] = (zin && xyin[i]) ? r[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
};

__device__ __forceinline__ void fma4(float4& a, const float4& k, const float4& v) {
  a.x += k.x * v.x;
  a.y += k.y * v.y;
  a.z += k.z * v.z;
  a.w += k.w * v.w;
}

// Keeps the compiler from sinking an accumulation below this point (into a
// guarded store), which would keep every LDS value loaded live.
__device__ __forceinline__ void dw_pin(float4& a) {
  asm volatile("" : "+v"(a.x), "+v"(a.y), "+v"(a.z), "+v"(a.w));
}

// y[v][c] = b[c] + sum_tap w[c][tap] x[v + offset(tap)][c]; with flip the
// taps are taken in reverse (w[c][26 - tap]) and b is ignored, which makes
// the kernel the input gradient of the forward one.  Input planes zb-1 .. ze
// pass through LDS in groups of D, the next group loading while one is
// computed; when plane
// p is in LDS the thread adds its 3 x 3 neighbourhood into outputs p+1 (taps
// dz = 0), p (dz = 1) and p-1 (dz = 2), and output p-1 is then complete.
template <int KQ, int D>
__global__ __launch_bounds__(256, 2) void k_dw_fwd(const float* __restrict__ x,
                                                   const float* __restrict__ w,
                                                   const float* __restrict__ b,
                                                   float* __restrict__ y, int n, int C, int ntxy,
                                                   int nseg, int seglen, int flip) {
  using G = DwGeo<KQ>;
  __shared__ float4 hal[D][G::PLANE];
  __shared__ float4 wl[27 * KQ];
  const int nb = ntxy * nseg * (C / (4 * KQ));
  const int L = dw_logical(nb);
  if (L >= nb) return;  // whole block: no barrier reached
  const DwBlock<KQ> bk(L, n, ntxy, nseg, seglen);
  const DwStager<KQ> st(n, C, bk.c0, bk.y0, bk.x0);
  float4 r[D][G::NL];
#pragma unroll
  for (int j = 0; j < D; ++j) st.load(x, min(bk.zb - 1 + j, bk.ze), r[j]);
  if (threadIdx.x < 27 * KQ) {
    const int tap = threadIdx.x >> G::SHIFT, q = threadIdx.x & (KQ - 1);
    const float* wc = w + (size_t)(bk.c0 + 4 * q) * 27 + (flip ? 26 - tap : tap);
    wl[threadIdx.x] = make_float4(wc[0], wc[27], wc[54], wc[81]);
  }
  __syncthreads();
  const int q = threadIdx.x & (KQ - 1), col = threadIdx.x >> G::SHIFT;
  const int tx = col % G::TX, ty = col / G::TX;
  const int gy = bk.y0 + ty, gx = bk.x0 + tx;
  const bool colin = gy < n && gx < n;
  float4 k[27];
#pragma unroll
  for (int i = 0; i < 27; ++i) k[i] = wl[i * KQ + q];
  const float4 b0 = (b && !flip) ? *reinterpret_cast<const float4*>(b + bk.c0 + 4 * q)
                                 : make_float4(0.f, 0.f, 0.f, 0.f);
  float* yc = y + ((size_t)min(gy, n - 1) * n + min(gx, n - 1)) * C + bk.c0 + 4 * q;
  const size_t pstride = (size_t)n * n * C;
  float4 a_prev = b0, a_cur = b0, a_next = b0;  // outputs p-1, p, p+1
  const int np = bk.ze - bk.zb + 2;             // input planes zb-1 .. ze
  for (int s = 0; s < np; s += D) {
#pragma unroll
    for (int j = 0; j < D; ++j)
      if (s + j < np) st.store(hal[j], bk.zb - 1 + s + j, r[j]);
    __syncthreads();
    if (s + D < np)  // uniform: the next group's loads fly during this group
#pragma unroll
      for (int j = 0; j < D; ++j) st.load(x, min(bk.zb - 1 + s + D + j, bk.ze), r[j]);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      if (s + j < np) {  // uniform
        const int p = bk.zb - 1 + s + j;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) {
            const float4 v = hal[j][((ty + dy) * G::HX + tx + dx) * KQ + q];
            fma4(a_next, k[dy * 3 + dx], v);
            fma4(a_cur, k[9 + dy * 3 + dx], v);
            fma4(a_prev, k[18 + dy * 3 + dx], v);
          }
        dw_pin(a_prev);
        dw_pin(a_cur);
        dw_pin(a_next);
        if (p - 1 >= bk.zb && colin)
          *reinterpret_cast<float4*>(yc + (size_t)(p - 1) * pstride) = a_prev;
        a_prev = a_cur;
        a_cur = a_next;
        a_next = b0;
      }
    }
    __syncthreads();  // the group's planes are consumed before the next are written
  }
}

// Weight-gradient partials.  The block streams its z segment like the
// forward kernel; when input plane p is in LDS the thread adds
// g[p+1] * x (taps dz = 0), g[p] * x (dz = 1) and g[p-1] * x (dz = 2) over the
// 3 x 3 neighbourhood, g being zero outside the segment and the grid, so each
// output voxel is counted by exactly one block.  The block's sums go to
// part[(c * 28 + k) * nP + txy + ntxy * sg], nP = ntxy * nseg (column-major,
// so the reduction reads them contiguously).  Threads sum in plane order,
// then threads of equal quad in a fixed order through LDS.
template <int KQ, int D>
__global__ __launch_bounds__(256, 2) void k_dw_wgrad(const float* __restrict__ x,
                                                     const float* __restrict__ gyv,
                                                     float* __restrict__ part, int n, int C,
                                                     int ntxy, int nseg, int seglen) {
  using G = DwGeo<KQ>;
  __shared__ float4 hal[D][G::PLANE];
  const int nb = ntxy * nseg * (C / (4 * KQ));
  const int L = dw_logical(nb);
  if (L >= nb) return;  // whole block
  const DwBlock<KQ> bk(L, n, ntxy, nseg, seglen);
  const DwStager<KQ> st(n, C, bk.c0, bk.y0, bk.x0);
  const int q = threadIdx.x & (KQ - 1), col = threadIdx.x >> G::SHIFT;
  const int tx = col % G::TX, ty = col / G::TX;
  const int gy = bk.y0 + ty, gx = bk.x0 + tx;
  const bool colin = gy < n && gx < n;
  const float* gc = gyv + ((size_t)min(gy, n - 1) * n + min(gx, n - 1)) * C + bk.c0 + 4 * q;
  const size_t pstride = (size_t)n * n * C;
  // g of output plane o, clamped into the segment (always a valid address)
  auto gload = [&](int o) {
    return *reinterpret_cast<const float4*>(gc + (size_t)min(max(o, bk.zb), bk.ze - 1) * pstride);
  };
  auto gmask = [&](int o, float4 v) {
    return (colin && o >= bk.zb && o < bk.ze) ? v : make_float4(0.f, 0.f, 0.f, 0.f);
  };
  float4 r[D][G::NL], gq[D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    st.load(x, min(bk.zb - 1 + j, bk.ze), r[j]);
    gq[j] = gload(bk.zb + 1 + j);
  }
  float4 g0 = make_float4(0.f, 0.f, 0.f, 0.f), g1 = g0;  // g of planes p-1, p
  float4 g2 = gmask(bk.zb, gload(bk.zb));               // g of plane p+1
  float4 acc[kDwParts];
#pragma unroll
  for (int i = 0; i < kDwParts; ++i) acc[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  const int np = bk.ze - bk.zb + 2;
  for (int s = 0; s < np; s += D) {
    float4 gn[D];  // g of planes p + 2 for this group's planes p
#pragma unroll
    for (int j = 0; j < D; ++j) {
      if (s + j < np) st.store(hal[j], bk.zb - 1 + s + j, r[j]);
      gn[j] = gmask(bk.zb + 1 + s + j, gq[j]);
    }
    __syncthreads();
    if (s + D < np)  // uniform: the next group's loads fly during this group
#pragma unroll
      for (int j = 0; j < D; ++j) {
        st.load(x, min(bk.zb - 1 + s + D + j, bk.ze), r[j]);
        gq[j] = gload(bk.zb + 1 + s + D + j);
      }
#pragma unroll
    for (int j = 0; j < D; ++j) {
      if (s + j < np) {  // uniform
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) {
            const float4 v = hal[j][((ty + dy) * G::HX + tx + dx) * KQ + q];
            fma4(acc[dy * 3 + dx], g2, v);
            fma4(acc[9 + dy * 3 + dx], g1, v);
            fma4(acc[18 + dy * 3 + dx], g0, v);
          }
        fma4(acc[27], make_float4(1.f, 1.f, 1.f, 1.f), g1);
        g0 = g1;
        g1 = g2;
        g2 = gn[j];
      }
    }
    __syncthreads();  // the group's planes are consumed before the next are written
  }
  // Sum over the threads of equal quad through LDS, kDwRedChunk
  // accumulators at a time: each thread's values go to red[c][tid]; thread
  // (o, part) of NO = chunk * KQ outputs sums M of them in order, then the
  // P = 256 / NO part sums of each output are added in order.
  constexpr int CH = kDwRedChunk, NO = CH * KQ, P = 256 / NO, M = 256 / KQ / P;
  static_assert(D * G::PLANE >= CH * 256, "reduction buffer fits in the planes");
  float4* red = &hal[0][0];
  const int o = threadIdx.x % NO, part_i = threadIdx.x / NO;
  const int oc = o / KQ, oq = o % KQ;
  const size_t nP = (size_t)ntxy * nseg, P0 = bk.txy + (size_t)ntxy * bk.sg;
#pragma unroll
  for (int i0 = 0; i0 < kDwParts; i0 += CH) {
    __syncthreads();  // the previous chunk (or the planes) fully read
#pragma unroll
    for (int c = 0; c < CH; ++c) red[c * 256 + threadIdx.x] = acc[i0 + c];
    __syncthreads();
    float4 sum = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const float4 v = red[oc * 256 + oq + KQ * (part_i * M + m)];
      sum.x += v.x;
      sum.y += v.y;
      sum.z += v.z;
      sum.w += v.w;
    }
    __syncthreads();
    red[part_i * NO + o] = sum;
    __syncthreads();
    if (threadIdx.x < NO) {
      float4 t = red[threadIdx.x];
#pragma unroll
      for (int pp = 1; pp < P; ++pp) {
        const float4 v = red[pp * NO + threadIdx.x];
        t.x += v.x;
        t.y += v.y;
        t.z += v.z;
        t.w += v.w;
      }
      const int i = i0 + oc, c = bk.c0 + 4 * oq;
      part[((size_t)(c + 0) * kDwParts + i) * nP + P0] = t.x;
      part[((size_t)(c + 1) * kDwParts + i) * nP + P0] = t.y;
      part[((size_t)(c + 2) * kDwParts + i) * nP + P0] = t.z;
      part[((size_t)(c + 3) * kDwParts + i) * nP + P0] = t.w;
    }
  }
}

// Dilated depthwise convolution (taps `dil` voxels apart, the atrous branches
// of an ASPP module), direct form for the small grids it runs on: thread per
// (voxel, channel quad), 27 clamped float4 loads masked outside the grid; flip
// reverses the taps (input gradient; b ignored).  Grid: ceil(V * C4 / 256).
__global__ __launch_bounds__(256) void k_dwd_fwd(const float* __restrict__ x,
                                                 const float* __restrict__ w,
                                                 const float* __restrict__ b,
                                                 float* __restrict__ y, int n, int C, int dil,
                                                 int flip) {
  const int C4 = C >> 2;
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long long)n * n * n * C4) return;
  const int q = (int)(e % C4);
  const int v = (int)(e / C4);
  const int vx = v % n, vy = (v / n) % n, vz = v / (n * n);
  float4 acc = (b && !flip) ? *reinterpret_cast<const float4*>(b + 4 * q)
                            : make_float4(0.f, 0.f, 0.f, 0.f);
  const float* wq = w + (size_t)(4 * q) * 27;
#pragma unroll
  for (int t = 0; t < 27; ++t) {
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    const int gz = vz + dil * dz, gy = vy + dil * dy, gx = vx + dil * dx;
    const bool in = (unsigned)gz < (unsigned)n && (unsigned)gy < (unsigned)n &&
                    (unsigned)gx < (unsigned)n;
    const int cz = min(max(gz, 0), n - 1), cy = min(max(gy, 0), n - 1), cx = min(max(gx, 0), n - 1);
    float4 xv = *reinterpret_cast<const float4*>(x + ((size_t)(cz * n + cy) * n + cx) * C + 4 * q);
    if (!in) xv = make_float4(0.f, 0.f, 0.f, 0.f);
    const int tt = flip ? 26 - t : t;
    acc.x += wq[tt] * xv.x;
    acc.y += wq[27 + tt] * xv.y;
    acc.z += wq[54 + tt] * xv.z;
    acc.w += wq[81 + tt] * xv.w;
  }
  *reinterpret_cast<float4*>(y + (size_t)v * C + 4 * q) = acc;
}

// Weight-gradient partials of the dilated depthwise convolution: block b of
// a chunk of `chunk` voxels; thread (r, q) of R = 256 / C4 row lanes sums
// gy[v] x[v + dil (t - 1)] (27 taps) and gy[v] (bias) over voxels
// v0 + r, v0 + r + R, ...; the lanes of a quad are added in order through
// LDS, four sums at a time, into part[(c * 28 + k) * nP + b].
__global__ __launch_bounds__(256) void k_dwd_wgrad(const float* __restrict__ x,
                                                   const float* __restrict__ gyv,
                                                   float* __restrict__ part, int n, int C,
                                                   int dil, int chunk, int nP) {
  __shared__ float4 red[4 * 256];
  const int C4 = C >> 2, R = 256 / C4;
  const int q = threadIdx.x % C4, r = threadIdx.x / C4;
  const int V = n * n * n;
  const int v0 = blockIdx.x * chunk, v1 = min(V, v0 + chunk);
  float4 acc[kDwParts];
#pragma unroll
  for (int i = 0; i < kDwParts; ++i) acc[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  if (r < R)
    for (int v = v0 + r; v < v1; v += R) {
      const int vx = v % n, vy = (v / n) % n, vz = v / (n * n);
      const float4 g = *reinterpret_cast<const float4*>(gyv + (size_t)v * C + 4 * q);
#pragma unroll
      for (int t = 0; t < 27; ++t) {
        const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
        const int gz = vz + dil * dz, gy = vy + dil * dy, gx = vx + dil * dx;
        const bool in = (unsigned)gz < (unsigned)n && (unsigned)gy < (unsigned)n &&
                        (unsigned)gx < (unsigned)n;
        const int cz = min(max(gz, 0), n - 1), cy = min(max(gy, 0), n - 1),
                  cx = min(max(gx, 0), n - 1);
        float4 xv =
            *reinterpret_cast<const float4*>(x + ((size_t)(cz * n + cy) * n + cx) * C + 4 * q);
        if (!in) xv = make_float4(0.f, 0.f, 0.f, 0.f);
        fma4(acc[t], g, xv);
      }
      fma4(acc[27], make_float4(1.f, 1.f, 1.f, 1.f), g);
    }
#pragma unroll
  for (int i0 = 0; i0 < kDwParts; i0 += 4) {
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 4; ++c) red[c * 256 + threadIdx.x] = acc[i0 + c];
    __syncthreads();
    if (threadIdx.x < 4 * C4) {
      const int c = threadIdx.x / C4, qq = threadIdx.x % C4;
      float4 s = red[c * 256 + qq];
      for (int rr = 1; rr < R; ++rr) {
        const float4 t = red[c * 256 + rr * C4 + qq];
        s.x += t.x;
        s.y += t.y;
        s.z += t.z;
        s.w += t.w;
      }
      const int k = i0 + c, ch = 4 * qq;
      part[((size_t)(ch + 0) * kDwParts + k) * nP + blockIdx.x] = s.x;
      part[((size_t)(ch + 1) * kDwParts + k) * nP + blockIdx.x] = s.y;
      part[((size_t)(ch + 2) * kDwParts + k) * nP + blockIdx.x] = s.z;
      part[((size_t)(ch + 3) * kDwParts + k) * nP + blockIdx.x] = s.w;
    }
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
  float r[7];  // the rest: every load issued, then added in the same order
#pragma unroll
  for (int u = 0; u < 7; ++u) r[u] = j + 64 * u < nP ? p[j + 64 * u] : 0.f;
#pragma unroll
  for (int u = 0; u < 7; ++u)
    if (j + 64 * u < nP) a[u] += r[u];
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

// (y, x) tiles and z segments: segments of 32 planes, halved (down to 4)
// while the grid has fewer than `target` blocks.
struct DwPlan {
  int kq, ntxy, nseg, seglen, nb;
};

constexpr int kDwFwdBlocks = 512;  // grid targets (two blocks fit a CU): forward / input gradient
constexpr int kDwWgBlocks = 512;   // weight gradient

DwPlan dw_plan(int n, int C, int target) {
  DwPlan p;
  p.kq = dw_kq(C);
  const int ty = p.kq >= 4 ? 8 : 16, tx = 256 / p.kq / ty;
  p.ntxy = ((n + tx - 1) / tx) * ((n + ty - 1) / ty);
  const int nch = C / (4 * p.kq);
  p.seglen = 32;
  while (p.seglen > 4 && (long long)p.ntxy * ((n + p.seglen - 1) / p.seglen) * nch < target)
    p.seglen /= 2;
  p.nseg = (n + p.seglen - 1) / p.seglen;
  p.nb = p.ntxy * p.nseg * nch;
  return p;
}

template <int KQ>
void launch_fwd(const DwPlan& p, const float* x, const float* w, const float* b, float* y, int n,
                int C, bool flip, hipStream_t s) {
  hipLaunchKernelGGL((k_dw_fwd<KQ, kDwFwdGroup>), dim3((p.nb + 7) / 8 * 8), dim3(256), 0, s, x, w, b, y, n, C,
                     p.ntxy, p.nseg, p.seglen, flip ? 1 : 0);
}

template <int KQ>
void launch_wgrad(const DwPlan& p, const float* x, const float* gy, float* part, int n, int C,
                  hipStream_t s) {
  hipLaunchKernelGGL((k_dw_wgrad<KQ, kDwWgGroup>), dim3((p.nb + 7) / 8 * 8), dim3(256), 0, s, x, gy, part, n,
                     C, p.ntxy, p.nseg, p.seglen);
}

}  // namespace

// Voxel chunks of the dilated weight gradient: at most 256, whole lane passes.
static void dwd_chunks(int n, int C, int* chunk, int* nchunks) {
  const int V = n * n * n, R = 256 / (C / 4);
  int len = (V + 255) / 256;
  len = (len + R - 1) / R * R;
  *chunk = len;
  *nchunks = (V + len - 1) / len;
}

size_t dwd_partials(int n, int C) {
  int chunk, nchunks;
  dwd_chunks(n, C, &chunk, &nchunks);
  return (size_t)nchunks * C * kDwParts;
}

void dwd_forward(const float* x, const float* w, const float* b, float* y, int n, int C, int dil,
                 bool flip, hipStream_t s) {
  const long long total = (long long)n * n * n * (C / 4);
  hipLaunchKernelGGL(k_dwd_fwd, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, x, w, b, y,
                     n, C, dil, flip ? 1 : 0);
}

void dwd_wgrad(const float* x, const float* gy, float* part, float* gw, float* gb, int n, int C,
               int dil, hipStream_t s) {
  int chunk, nchunks;
  dwd_chunks(n, C, &chunk, &nchunks);
  hipLaunchKernelGGL(k_dwd_wgrad, dim3(nchunks), dim3(256), 0, s, x, gy, part, n, C, dil, chunk,
                     nchunks);
  hipLaunchKernelGGL(k_dw_wreduce, dim3((C * kDwParts + 3) / 4), dim3(256), 0, s, part, nchunks,
                     C, gw, gb);
}

size_t dw_partials(int n, int C) {
  const DwPlan p = dw_plan(n, C, kDwWgBlocks);
  return (size_t)p.ntxy * p.nseg * C * kDwParts;
}

void dw_forward(const float* x, const float* w, const float* b, float* y, int n, int C, bool flip,
                hipStream_t s) {
  const DwPlan p = dw_plan(n, C, kDwFwdBlocks);
  switch (p.kq) {
    case 8: launch_fwd<8>(p, x, w, b, y, n, C, flip, s); break;
    case 4: launch_fwd<4>(p, x, w, b, y, n, C, flip, s); break;
    case 2: launch_fwd<2>(p, x, w, b, y, n, C, flip, s); break;
    default: launch_fwd<1>(p, x, w, b, y, n, C, flip, s); break;
  }
}

void dw_wgrad(const float* x, const float* gy, float* part, float* gw, float* gb, int n, int C,
              hipStream_t s) {
  const DwPlan p = dw_plan(n, C, kDwWgBlocks);
  switch (p.kq) {
    case 8: launch_wgrad<8>(p, x, gy, part, n, C, s); break;
    case 4: launch_wgrad<4>(p, x, gy, part, n, C, s); break;
    case 2: launch_wgrad<2>(p, x, gy, part, n, C, s); break;
    default: launch_wgrad<1>(p, x, gy, part, n, C, s); break;
  }
  hipLaunchKernelGGL(k_dw_wreduce, dim3((C * kDwParts + 3) / 4), dim3(256), 0, s, part,
                     p.ntxy * p.nseg, C, gw, gb);
}

}  // namespace d2ip
