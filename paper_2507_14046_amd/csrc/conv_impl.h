// 3D convolutions of the image prior (3x3x3 and 1x1x1, zero padding) as
// implicit GEMMs on the gfx950 matrix cores.
//
// Forward / input-gradient kernel: GEMM rows are the output voxels of a
// TZ x TY x TX spatial tile, columns are output channels (BN per block), the
// reduction runs over (tap, input channel).  Each block stages the input halo
// of its tile for a chunk of CK channels in LDS, applying the producer's
// pending transform on the fly (LayerNorm+ReLU, or the LayerNorm backward),
// then each wave issues 16x16 MFMAs: v_mfma_f32_16x16x4_f32 (FP32 operands)
// or v_mfma_f32_16x16x32_bf16 (BF16 operands); accumulation is FP32.  Coarse
// grids split the channel chunks over blocks (split-K); a second launch sums
// each output's partials in split order.  The epilogue adds bias / residual,
// stores, and emits per-tile FP64 (sum, sumsq) partials, which the consumer
// reduces into the LayerNorm statistics of the output.
//
// Weight-gradient kernel: rows are output channels (16 per block), columns
// (tap, channel) in groups of 128 per block, the reduction runs over voxels;
// blocks split the voxel range and write partial sums that one batched
// kernel per iteration reduces in a fixed order (deterministic).
//
// Operand modes: PREC_F32 (one FP32 MFMA per k-step), PREC_BF16 (operands
// rounded to bf16, one MFMA), PREC_BF16X3 (each operand x split into
// hi = bf16(x) and lo = bf16(x - hi); the product is hi*hi + hi*lo + lo*hi on
// three BF16 MFMAs, leaving a relative product error near 2^-16).
// This header is included by one translation unit per mode.
#pragma once
#include <type_traits>

#include "kernels.h"

namespace d2ip {
namespace conv_detail {

constexpr int kCkMax = 32;       // largest channel chunk staged at once
constexpr int kWgNg1 = 2;        // 1x1x1 weight-gradient column tiles (chunks <= 32)
// Columns (tap, channel) of a weight-gradient block.  1x1x1: every wave works
// on the chunk's (at most 2) column tiles over a quarter of the voxel k-steps;
// 3x3x3: each wave owns wg_nj(ck) column tiles over all k-steps (4 for 8
// channels = 13.5 tiles, 7 for 16 and 32 = 27 and 54 tiles), so one staged
// halo feeds up to 28 tiles, the MFMAs need no guards and no cross-wave
// exchange is needed.
__host__ __device__ constexpr int wg_nj(int ck) { return ck == 8 ? 4 : 7; }
__host__ __device__ constexpr int wg_cols(int taps, int ck) {
  return taps == 27 ? 4 * wg_nj(ck) * 16 : kWgNg1 * 16;
}

template <int TILE>
struct TileDims;
template <>
struct TileDims<TILE_2x4x16> {
  static constexpr int Z = 2, Y = 4, X = 16;
};
template <>
struct TileDims<TILE_1x4x16> {
  static constexpr int Z = 1, Y = 4, X = 16;
};
template <>
struct TileDims<TILE_1x8x8> {
  static constexpr int Z = 1, Y = 8, X = 8;
};

template <int MODE>
struct Mode {
  static constexpr bool BF = MODE != PREC_F32;        // bf16 operands
  static constexpr bool SPLIT = MODE == PREC_BF16X3;  // hi + lo parts
  static constexpr int KPL = BF ? 8 : 1;              // k per lane per MFMA
  static constexpr int KSTEP = 4 * KPL;               // k per MFMA
  static constexpr int PAD = BF ? 8 : 1;              // LDS row padding (elements)
  using ST = typename std::conditional<BF, uint16_t, float>::type;  // LDS element
  using FT = typename std::conditional<BF, bf16x8, float>::type;    // MFMA operand
};

// LDS row pitch (elements) of the forward weight slab: FP32 pitches are
// 2 mod 32 words so the 16 rows x 4 k of a fragment hit distinct banks; BF16
// pitches keep 16-byte alignment.
__host__ __device__ inline int fwd_wrow(int taps, int ck, bool bf) {
  const int base = taps * ck;
  if (bf) return base + 8;
  return base + ((2 - base % 32) + 32) % 32;
}

__host__ inline size_t fwd_lds_bytes(int tile, int taps, int bn, int ck, int mode) {
  int tz, ty, tx;
  if (tile == TILE_2x4x16) {
    tz = 2; ty = 4; tx = 16;
  } else if (tile == TILE_1x4x16) {
    tz = 1; ty = 4; tx = 16;
  } else {
    tz = 1; ty = 8; tx = 8;
  }
  const int r = taps == 27 ? 1 : 0;
  const size_t hp = (size_t)(tz + 2 * r) * (ty + 2 * r) * (tx + 2 * r);
  const bool bf = mode != PREC_F32;
  const int parts = mode == PREC_BF16X3 ? 2 : 1;
  const size_t el = bf ? 2 : 4;
  const size_t ckp = ck + (bf ? 8 : 1);
  const size_t stage = parts * el * (hp * ckp + (size_t)bn * fwd_wrow(taps, ck, bf));
  const size_t xch = (size_t)4 * (tz * ty * tx / 16) * (bn / 16) * 64 * 16;  // 4 waves x tiles
  const int kstep = bf ? 32 : 4;
  const size_t ktab = (size_t)4 * 4 * ((taps * ck + kstep - 1) / kstep);  // k-offset table
  return (((stage > xch ? stage : xch) + 15) & ~(size_t)15) + ktab;
}

// Offset (in LDS elements) of the k-offset table of the forward kernel.
__host__ __device__ inline int fwd_ktab_offset_bytes(int hp, int bn, int ck, int taps, int mode,
                                                     int mt, int nt) {
  const bool bf = mode != PREC_F32;
  const int parts = mode == PREC_BF16X3 ? 2 : 1;
  const int el = bf ? 2 : 4;
  const int ckp = ck + (bf ? 8 : 1);
  const int stage = parts * el * (hp * ckp + bn * fwd_wrow(taps, ck, bf));
  const int xch = 4 * mt * nt * 64 * 16;
  return ((stage > xch ? stage : xch) + 15) & ~15;
}

__device__ __forceinline__ f32x4 mfma(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Split an fp32 value into bf16 hi and lo parts (lo = bf16(x - hi)).
__device__ __forceinline__ void split_bf(float x, uint16_t& hi, uint16_t& lo) {
  hi = f2bf(x);
  lo = f2bf(x - bf2f(hi));
}

__device__ __forceinline__ uint32_t pack2(uint16_t a, uint16_t b) {
  return (uint32_t)a | ((uint32_t)b << 16);
}

// Prologue constants of a source, reduced from the producers' partials by
// the whole block (call from every thread).
template <int PRO>
__device__ __forceinline__ void src_consts(const ConvSrc& s, float& mean, float& rstd, float& A,
                                           float& B) {
  mean = 0.f;
  rstd = 1.f;
  A = 0.f;
  B = 0.f;
  if (PRO == PRO_LN_RELU) {
    const LnStat st = stat_of(s.st);
    mean = st.mean;
    rstd = st.rstd;
  } else if (PRO == PRO_LN_BWD) {
    LnStat st;
    LnBwd c;
    stat_coef_of(s.st, s.bw, st, c);
    mean = st.mean;
    rstd = st.rstd;
    A = c.A;
    B = c.B;
  }
}

// Store four values at LDS element offset o (and the lo parts in split mode).
template <int MODE>
__device__ __forceinline__ void put4(typename Mode<MODE>::ST* hi, typename Mode<MODE>::ST* lo,
                                     int o, float4 v) {
  if constexpr (Mode<MODE>::SPLIT) {
    uint16_t h0, h1, h2, h3, l0, l1, l2, l3;
    split_bf(v.x, h0, l0);
    split_bf(v.y, h1, l1);
    split_bf(v.z, h2, l2);
    split_bf(v.w, h3, l3);
    *reinterpret_cast<uint2*>(hi + o) = make_uint2(pack2(h0, h1), pack2(h2, h3));
    *reinterpret_cast<uint2*>(lo + o) = make_uint2(pack2(l0, l1), pack2(l2, l3));
  } else if constexpr (Mode<MODE>::BF) {
    *reinterpret_cast<uint2*>(hi + o) =
        make_uint2(pack2(f2bf(v.x), f2bf(v.y)), pack2(f2bf(v.z), f2bf(v.w)));
  } else {
    hi[o + 0] = v.x;
    hi[o + 1] = v.y;
    hi[o + 2] = v.z;
    hi[o + 3] = v.w;
  }
}

// Staging goes through registers in two phases: every global load of a
// pass is issued first (all in flight together, and across chunks or tiles
// while the previous one is being computed), then the values are
// transformed and written to LDS.  Element k of a thread's pass is
// p = k * 256 + tid; with Q = ck / 4 channel quads per voxel (Q divides 256)
// a thread always handles the same quad, tid % Q.
template <int NB, int PRO>
struct Quads {
  float4 v[NB];
  float4 h[PRO == PRO_LN_BWD ? NB : 1];  // LayerNorm-backward input
  unsigned in;                           // bit k: element k lies inside the grid
};

// Element k's LayerNorm-backward input (zero for other prologues).
template <int NB, int PRO>
__device__ __forceinline__ float4 quad_h(const Quads<NB, PRO>& r, int k) {
  if constexpr (PRO == PRO_LN_BWD) return r.h[k];
  return make_float4(0.f, 0.f, 0.f, 0.f);
}

// Channel constants of a source prologue for the channels c..c+3.
struct ChanConsts {
  float4 g, b;
};

template <int PRO>
__device__ __forceinline__ ChanConsts chan_consts(const ConvSrc& s, int c) {
  ChanConsts k;
  k.g = make_float4(1.f, 1.f, 1.f, 1.f);
  k.b = make_float4(0.f, 0.f, 0.f, 0.f);
  if (PRO != PRO_NONE) k.g = make_float4(s.gamma[c], s.gamma[c + 1], s.gamma[c + 2], s.gamma[c + 3]);
  if (PRO == PRO_LN_RELU) k.b = make_float4(s.beta[c], s.beta[c + 1], s.beta[c + 2], s.beta[c + 3]);
  return k;
}

// The source's pending transform on four channels (inside the grid only: the
// conv's zero padding stays zero).
template <int PRO>
__device__ __forceinline__ float4 apply_pro(float4 v, float4 h, const ChanConsts& k, float mean,
                                            float rstd, float A, float B) {
  if (PRO == PRO_LN_RELU) {
    v.x = fmaxf(k.g.x * ((v.x - mean) * rstd) + k.b.x, 0.f);
    v.y = fmaxf(k.g.y * ((v.y - mean) * rstd) + k.b.y, 0.f);
    v.z = fmaxf(k.g.z * ((v.z - mean) * rstd) + k.b.z, 0.f);
    v.w = fmaxf(k.g.w * ((v.w - mean) * rstd) + k.b.w, 0.f);
  } else if (PRO == PRO_LN_BWD) {
    v.x = rstd * (k.g.x * v.x - A - ((h.x - mean) * rstd) * B);
    v.y = rstd * (k.g.y * v.y - A - ((h.y - mean) * rstd) * B);
    v.z = rstd * (k.g.z * v.z - A - ((h.z - mean) * rstd) * B);
    v.w = rstd * (k.g.w * v.w - A - ((h.w - mean) * rstd) * B);
  }
  return v;
}

// Number of staging elements per thread for a halo of HP voxels at the
// largest channel chunk.
template <int HP>
constexpr int halo_nb() {
  return (HP * (kCkMax / 4) + 255) / 256;
}

// Per-thread geometry of its halo elements, the same for every tile and
// chunk of a launch: the element's position inside the halo (hz, hy, hx in
// bytes 0..2; -1 when the element lies beyond the halo) and its offset from
// the halo origin in the source tensor.
template <int NB>
struct HaloIdx {
  int pos[NB];
  int rel[NB];
};

template <int NB, int HZ, int HY, int HX>
__device__ __forceinline__ void halo_prep(HaloIdx<NB>& hi, int n, int stride, int qs) {
  constexpr int HP = HZ * HY * HX;
  const int total = HP << qs;
  const int q = threadIdx.x & ((1 << qs) - 1);
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const int p = k * 256 + threadIdx.x;
    const int pos = p >> qs;
    const int hx = pos % HX, hy = (pos / HX) % HY, hz = pos / (HX * HY);
    hi.pos[k] = p < total ? (hz | (hy << 8) | (hx << 16)) : -1;
    hi.rel[k] = ((hz * n + hy) * n + hx) * stride + 4 * q;
  }
}

// Issue the loads of a (HZ x HY x HX) halo of ck = 4 << qs channels starting
// at ci0, anchored at (z0, y0, x0) - R.
template <int NB, int PRO, int HZ, int HY, int HX>
__device__ __forceinline__ void halo_load(Quads<NB, PRO>& r, const HaloIdx<NB>& hi,
                                          const ConvSrc& s, int n, int qs, int ci0, int z0,
                                          int y0, int x0, int R) {
  constexpr int HP = HZ * HY * HX;
  const int total = HP << qs;
  const int oz = z0 - R, oy = y0 - R, ox = x0 - R;
  const long long base = ((long long)(oz * n + oy) * n + ox) * s.stride + ci0;
  r.in = 0u;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    r.v[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (PRO == PRO_LN_BWD) r.h[k] = r.v[k];
    if (k * 256 >= total) continue;  // uniform: dead for smaller chunks
    const int ps = hi.pos[k];
    const bool ok = ps >= 0 && (unsigned)(oz + (ps & 255)) < (unsigned)n &&
                    (unsigned)(oy + ((ps >> 8) & 255)) < (unsigned)n &&
                    (unsigned)(ox + (ps >> 16)) < (unsigned)n;
    if (ok) {
      const long long i = base + hi.rel[k];
      r.v[k] = *reinterpret_cast<const float4*>(s.x + i);
      if constexpr (PRO == PRO_LN_BWD) r.h[k] = *reinterpret_cast<const float4*>(s.h + i);
    }
    r.in |= (ok ? 1u : 0u) << k;
  }
}

// Write a loaded halo to LDS rows of ckp elements (forward layout
// [voxel][channel]).
template <int MODE, int NB, int PRO, int HP>
__device__ __forceinline__ void halo_store(typename Mode<MODE>::ST* hal,
                                           typename Mode<MODE>::ST* hal_lo,
                                           const Quads<NB, PRO>& r, int qs, int ckp,
                                           const ChanConsts& kc, float mean, float rstd, float A,
                                           float B) {
  const int total = HP << qs;
  const int q = threadIdx.x & ((1 << qs) - 1);
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (k * 256 >= total) break;  // uniform
    const int p = k * 256 + threadIdx.x;
    if (p < total) {
      float4 v = r.v[k];
      if (PRO != PRO_NONE && ((r.in >> k) & 1u))
        v = apply_pro<PRO>(v, quad_h(r, k), kc, mean, rstd, A, B);
      put4<MODE>(hal, hal_lo, (p >> qs) * ckp + 4 * q, v);
    }
  }
}

__device__ __forceinline__ int tap_offset(int tap, int HY, int HX) {
  const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
  return (dz * HY + dy) * HX + dx;
}

// MFMA operand fragment at p (always an in-bounds LDS address), zeroed
// where ok is false; a select, not a branch.
template <int MODE>
__device__ __forceinline__ typename Mode<MODE>::FT frag(const typename Mode<MODE>::ST* p, bool ok) {
  if constexpr (Mode<MODE>::BF) {
    u32x4 v = *reinterpret_cast<const u32x4*>(p);
    const unsigned m = ok ? 0xffffffffu : 0u;
    v.x &= m;
    v.y &= m;
    v.z &= m;
    v.w &= m;
    return __builtin_bit_cast(bf16x8, v);
  } else {
    const float v = *p;
    return ok ? v : 0.f;
  }
}

// CK: the channel chunk, fixed at compile time for 3x3x3 (8, 16 or 32; it
// sizes the halo prefetch), 0 for 1x1x1 (read from the arguments).
// Epilogue of a forward tile: y = result (+ bias) (+ add) (+ y) and the
// tile's (sum, sum of squares) of y.  fin[j] holds this lane's part of
// accumulator tile t = wave + 4 j: rows 4 g .. 4 g + 3 of row block t / NT,
// column l16 of column block t % NT.  Contains barriers (block_sum).
template <int TILE, int BN, int TPW>
__device__ __forceinline__ void fwd_epilogue(const ConvFwd& a, const f32x4 (&fin)[TPW], int x0,
                                             int y0, int z0, int co0, int tile_id, double* red) {
  using TD = TileDims<TILE>;
  constexpr int TZ = TD::Z, TY = TD::Y, TX = TD::X;
  constexpr int MT = TZ * TY * TX / 16, NT = BN / 16, NTILE = MT * NT;
  static_assert(TPW == (NTILE + 3) / 4, "tiles per wave");
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, g = lane >> 4;
  const int n = a.n;
  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    const int t = wave + 4 * j;
    if (t >= NTILE) continue;
    const int mt = t / NT, nt = t - mt * NT;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int li = mt * 16 + 4 * g + r;
      const int tz = li / (TY * TX), ty = (li / TX) % TY, tx = li % TX;
      const int gz = z0 + tz, gy = y0 + ty, gx = x0 + tx;
      const int co = co0 + nt * 16 + l16;
      if (gz >= n || gy >= n || gx >= n || co >= a.cout) continue;
      const size_t o = ((size_t)(gz * n + gy) * n + gx) * a.cout + co;
      float v = fin[j][r];
      if (a.bias) v += a.bias[co];
      if (a.add) v += a.add[o];
      if (a.accumulate) v += a.y[o];
      a.y[o] = v;
      s1 += v;
      s2 += (double)v * v;
    }
  }
  if (a.stat_part) {
    s1 = block_sum(s1, red);
    s2 = block_sum(s2, red);
    if (tid == 0) {
      a.stat_part[2 * tile_id] = s1;
      a.stat_part[2 * tile_id + 1] = s2;
    }
  }
}

template <int MODE, int TAPS, int TILE, int BN, int PRO, int CK>
__global__ __launch_bounds__(256) void k_conv_fwd(ConvFwd a) {
  // grid z = member * ksplit + split
  const int ksplit = a.ksplit;
  const int kz = blockIdx.z % ksplit;
  {
    const long long off = (long long)(blockIdx.z / ksplit) * a.istride;
    a.src = shift_src(a.src, off);
    a.w = ishift(a.w, off);
    a.bias = ishift(a.bias, off);
    a.add = ishift(a.add, off);
    a.y = ishift(a.y, off);
    a.stat_part = ishift(a.stat_part, off);
    a.kpart = ishift(a.kpart, off);
  }
  using MD = Mode<MODE>;
  using ST = typename MD::ST;
  using FT = typename MD::FT;
  using TD = TileDims<TILE>;
  constexpr int TZ = TD::Z, TY = TD::Y, TX = TD::X;
  constexpr int R = TAPS == 27 ? 1 : 0;
  constexpr int HZ = TZ + 2 * R, HY = TY + 2 * R, HX = TX + 2 * R, HP = HZ * HY * HX;
  constexpr int KPL = MD::KPL, KSTEP = MD::KSTEP;
  constexpr int BM = TZ * TY * TX, MT = BM / 16, NT = BN / 16;
  static_assert(MT * NT <= 16, "accumulator tile too large");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[8];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: scalar k-loop
  const int l16 = lane & 15, g = lane >> 4;
  const int n = a.n;
  const int ck = CK ? CK : a.ck, ckp = ck + MD::PAD;
  const int ck_shift = __builtin_ctz(ck);
  // LDS: halo [HP][ckp] (+ lo parts), weight slab [BN][wrp] (+ lo parts); the
  // same space holds the cross-wave accumulator exchange after the K loop
  const int wrp = fwd_wrow(TAPS, ck, MD::BF);
  ST* hal = reinterpret_cast<ST*>(smem);
  ST* hal_lo = hal + (MD::SPLIT ? HP * ckp : 0);
  ST* wsm = hal + (MD::SPLIT ? 2 : 1) * HP * ckp;
  ST* wsm_lo = wsm + (MD::SPLIT ? BN * wrp : 0);
  const int ntx = (n + TX - 1) / TX, nty = (n + TY - 1) / TY;
  int b = blockIdx.x;
  const int x0 = (b % ntx) * TX;
  b /= ntx;
  const int y0 = (b % nty) * TY;
  b /= nty;
  const int z0 = b * TZ;
  const int co0 = blockIdx.y * BN;

  // every wave accumulates all MT x NT tiles over every 4th k-step
  f32x4 acc[MT][NT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};

  // LDS offsets of this lane's A rows (halo voxels) and B rows (weight rows)
  int abase[MT], bbase[NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int li = mt * 16 + l16;
    const int tz = li / (TY * TX), ty = (li / TX) % TY, tx = li % TX;
    abase[mt] = ((tz * HY + ty) * HX + tx) * ckp;
  }
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) bbase[nt] = (nt * 16 + l16) * wrp;
  // k-offset table: for k-step s and lane group gg, the halo offset of its
  // (tap, channel) in the low 16 bits and the weight-slab column in the high
  // 16 bits; k beyond the taps points at the zeroed pad column of every
  // weight row (only BF16 steps overrun)
  const int nstep = (TAPS * ck + KSTEP - 1) / KSTEP;
  uint32_t* ktab = reinterpret_cast<uint32_t*>(
      smem + fwd_ktab_offset_bytes(HP, BN, ck, TAPS, MODE, MT, NT));
  for (int e = tid; e < nstep * 4; e += 256) {
    const int kl = (e >> 2) * KSTEP + (e & 3) * KPL;
    const int tap = kl >> ck_shift, c = kl & (ck - 1);
    uint32_t hoff = 0, woff = TAPS * ck;
    if (tap < TAPS) {
      hoff = (TAPS == 27 ? tap_offset(tap, HY, HX) : 0) * ckp + c;
      woff = tap * ck + c;
    }
    ktab[e] = hoff | (woff << 16);
  }
  if constexpr (MD::BF) {
    // zero pad columns [TAPS * ck, wrp) of every weight row (hi and lo)
    const int padw = wrp - TAPS * ck;
    for (int e = tid; e < BN * padw; e += 256) {
      const int r = e / padw, j = e - r * padw;
      wsm[r * wrp + TAPS * ck + j] = 0;
      if constexpr (MD::SPLIT) wsm_lo[r * wrp + TAPS * ck + j] = 0;
    }
  }

  const ST* __restrict__ W = reinterpret_cast<const ST*>(a.w);
  const ST* __restrict__ Wlo = W + a.w_lo_off;
  const int nchunks = a.cin >> ck_shift;
  const int cps = nchunks / ksplit;
  const int qs = ck_shift - 2;
  constexpr int NBH = CK ? (HP * (CK / 4) + 255) / 256 : halo_nb<HP>();
  Quads<NBH, PRO> hq;
  HaloIdx<NBH> hidx;
  halo_prep<NBH, HZ, HY, HX>(hidx, n, a.src.stride, qs);
  // weight slab of a chunk: rows co0.., for every tap ck channels, in batches
  // of NBW 16-byte vectors per thread; the first batch of the next chunk is
  // loaded into registers under the current chunk's MFMAs
  constexpr int EV = MD::BF ? 8 : 4;  // elements per 16-byte vector
  constexpr int NBW = 8;              // loads in flight per thread
  const int vs = ck_shift - (MD::BF ? 3 : 2);  // log2(vectors per (row, tap))
  const int nv = (BN * TAPS) << vs;
  u32x4 wv[NBW], wvl[MD::SPLIT ? NBW : 1];
  auto w_issue = [&](int ci0, int p0) {
#pragma unroll
    for (int k = 0; k < NBW; ++k) {
      const int p = p0 + k * 256 + tid;
      const int rt = p >> vs, q = p & ((1 << vs) - 1);
      const int r = rt / TAPS, tap = rt - r * TAPS;
      const int co = co0 + r;
      wv[k] = (u32x4){0u, 0u, 0u, 0u};
      if constexpr (MD::SPLIT) wvl[k] = (u32x4){0u, 0u, 0u, 0u};
      if (p < nv && co < a.w_rows) {
        const size_t wi = ((size_t)co * TAPS + tap) * a.cin + ci0 + q * EV;
        wv[k] = *reinterpret_cast<const u32x4*>(W + wi);
        if constexpr (MD::SPLIT) wvl[k] = *reinterpret_cast<const u32x4*>(Wlo + wi);
      }
    }
  };
  auto w_store = [&](int p0) {
#pragma unroll
    for (int k = 0; k < NBW; ++k) {
      const int p = p0 + k * 256 + tid;
      if (p >= nv) continue;
      const int rt = p >> vs, q = p & ((1 << vs) - 1);
      const int r = rt / TAPS, tap = rt - r * TAPS;
      const int o = r * wrp + tap * ck + q * EV;
      if constexpr (MD::BF) {
        *reinterpret_cast<u32x4*>(wsm + o) = wv[k];
        if constexpr (MD::SPLIT) *reinterpret_cast<u32x4*>(wsm_lo + o) = wvl[k];
      } else {
        // FP32 rows are padded to an even pitch: 4-byte stores
        ST* d = wsm + o;
        d[0] = __uint_as_float(wv[k].x);
        d[1] = __uint_as_float(wv[k].y);
        d[2] = __uint_as_float(wv[k].z);
        d[3] = __uint_as_float(wv[k].w);
      }
    }
  };
  // first chunk's halo and weights in flight while the prologue statistics
  // are reduced
  halo_load<NBH, PRO, HZ, HY, HX>(hq, hidx, a.src, n, qs, (kz * cps) << ck_shift, z0, y0, x0,
                                  R);
  w_issue((kz * cps) << ck_shift, 0);
  float pmean, prstd, pA, pB;
  src_consts<PRO>(a.src, pmean, prstd, pA, pB);
  for (int ch = kz * cps; ch < (kz + 1) * cps; ++ch) {
    const int ci0 = ch << ck_shift;
    const ChanConsts kc = chan_consts<PRO>(a.src, ci0 + 4 * (tid & ((1 << qs) - 1)));
    halo_store<MODE, NBH, PRO, HP>(hal, hal_lo, hq, qs, ckp, kc, pmean, prstd, pA, pB);
    w_store(0);
    for (int p0 = 256 * NBW; p0 < nv; p0 += 256 * NBW) {  // slabs beyond one batch
      w_issue(ci0, p0);
      w_store(p0);
    }
    __syncthreads();
    // next chunk's halo and first weight batch load under this chunk's MFMAs
    if (ch + 1 < (kz + 1) * cps) {
      halo_load<NBH, PRO, HZ, HY, HX>(hq, hidx, a.src, n, qs, (ch + 1) << ck_shift, z0, y0, x0,
                                      R);
      w_issue((ch + 1) << ck_shift, 0);
    }
#pragma unroll 2
    for (int step = wave; step < nstep; step += 4) {
      const uint32_t ko = ktab[step * 4 + g];
      const int hoff = ko & 0xffffu, woff = ko >> 16;
      FT A[MT], B[NT];
      FT Al[MD::SPLIT ? MT : 1], Bl[MD::SPLIT ? NT : 1];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        A[mt] = frag<MODE>(hal + abase[mt] + hoff, true);
        if constexpr (MD::SPLIT) Al[mt] = frag<MODE>(hal_lo + abase[mt] + hoff, true);
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        B[nt] = frag<MODE>(wsm + bbase[nt] + woff, true);
        if constexpr (MD::SPLIT) Bl[nt] = frag<MODE>(wsm_lo + bbase[nt] + woff, true);
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          if constexpr (MD::SPLIT) {
            acc[mt][nt] = mfma(Al[mt], B[nt], acc[mt][nt]);
            acc[mt][nt] = mfma(A[mt], Bl[nt], acc[mt][nt]);
          }
          acc[mt][nt] = mfma(A[mt], B[nt], acc[mt][nt]);
        }
    }
    __syncthreads();
  }

  // cross-wave exchange: wave w finishes tiles t = w, w + 4, ... by adding the
  // four waves' accumulators in wave order
  f32x4* xch = reinterpret_cast<f32x4*>(smem);
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) xch[((wave * MT + mt) * NT + nt) * 64 + lane] = acc[mt][nt];
  __syncthreads();
  constexpr int NTILE = MT * NT;
  constexpr int TPW = (NTILE + 3) / 4;  // tiles per wave
  f32x4 fin[TPW];
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    const int t = wave + 4 * j;
    f32x4 v = (f32x4){0.f, 0.f, 0.f, 0.f};
    if (t < NTILE) {
#pragma unroll
      for (int w = 0; w < 4; ++w) v += xch[(w * NTILE + t) * 64 + lane];
    }
    fin[j] = v;
  }

  const int tile_id = blockIdx.y * gridDim.x + blockIdx.x;
  if (ksplit > 1) {
    // split-K: publish this block's partial tile; k_fwd_finish sums the
    // splits in split order and runs the epilogue after this launch
    const size_t V = (size_t)n * n * n;
    float* kp = a.kpart + (size_t)kz * V * a.cout;
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      const int t = wave + 4 * j;
      if (t >= NTILE) continue;
      const int mt = t / NT, nt = t - mt * NT;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int li = mt * 16 + 4 * g + r;
        const int tz = li / (TY * TX), ty = (li / TX) % TY, tx = li % TX;
        const int gz = z0 + tz, gy = y0 + ty, gx = x0 + tx;
        const int co = co0 + nt * 16 + l16;
        if (gz >= n || gy >= n || gx >= n || co >= a.cout) continue;
        kp[((size_t)(gz * n + gy) * n + gx) * a.cout + co] = fin[j][r];
      }
    }
    return;
  }
  fwd_epilogue<TILE, BN>(a, fin, x0, y0, z0, co0, tile_id, red);
}

// Sum of the split-K partial tiles of a forward pass, in split order, then
// the epilogue; same grid (x, y) as the pass, z = group member.  Partials
// written by the previous launch are visible at the kernel boundary, so no
// block of the pass waits on or signals another.
template <int TILE, int BN>
__global__ __launch_bounds__(256) void k_fwd_finish(ConvFwd a) {
  {
    const long long off = (long long)blockIdx.z * a.istride;
    a.bias = ishift(a.bias, off);
    a.add = ishift(a.add, off);
    a.y = ishift(a.y, off);
    a.stat_part = ishift(a.stat_part, off);
    a.kpart = ishift(a.kpart, off);
  }
  using TD = TileDims<TILE>;
  constexpr int TZ = TD::Z, TY = TD::Y, TX = TD::X;
  constexpr int MT = TZ * TY * TX / 16, NT = BN / 16, NTILE = MT * NT, TPW = (NTILE + 3) / 4;
  __shared__ double red[8];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, g = lane >> 4;
  const int n = a.n;
  const int ntx = (n + TX - 1) / TX, nty = (n + TY - 1) / TY;
  int b = blockIdx.x;
  const int x0 = (b % ntx) * TX;
  b /= ntx;
  const int y0 = (b % nty) * TY;
  b /= nty;
  const int z0 = b * TZ;
  const int co0 = blockIdx.y * BN;
  const size_t V = (size_t)n * n * n;
  // every element sums the splits in split order; one split's loads of all
  // this lane's elements are in flight together
  size_t o[TPW][4];
  bool ok[TPW][4];
  f32x4 fin[TPW];
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    const int t = wave + 4 * j;
    const int mt = t / NT, nt = t - mt * NT;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int li = mt * 16 + 4 * g + r;
      const int tz = li / (TY * TX), ty = (li / TX) % TY, tx = li % TX;
      const int gz = z0 + tz, gy = y0 + ty, gx = x0 + tx;
      const int co = co0 + nt * 16 + l16;
      ok[j][r] = t < NTILE && gz < n && gy < n && gx < n && co < a.cout;
      o[j][r] = ok[j][r] ? ((size_t)(gz * n + gy) * n + gx) * a.cout + co : 0;
      fin[j][r] = 0.f;
    }
  }
  for (int k = 0; k < a.ksplit; ++k) {
    const float* kp = a.kpart + (size_t)k * V * a.cout;
    float v[TPW][4];
#pragma unroll
    for (int j = 0; j < TPW; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) v[j][r] = ok[j][r] ? kp[o[j][r]] : 0.f;
#pragma unroll
    for (int j = 0; j < TPW; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (ok[j][r]) fin[j][r] += v[j][r];
  }
  fwd_epilogue<TILE, BN>(a, fin, x0, y0, z0, co0, blockIdx.y * gridDim.x + blockIdx.x, red);
}

// Weight-gradient LDS (dynamic): halo, g tile and the cross-wave exchange.
//  FP32: halo [HP][ck+1] floats, g tile [BM][17] floats.
//  BF16: halo channel-major in three copies shifted by dx = 0, 1, 2 so that
//        8 consecutive voxels of a row are one aligned 16-byte read:
//        [3][ck][HZ*HY*TX + 8] (hi, then lo parts), g tile [16][BM + 8].
__host__ __device__ inline size_t wg_lds_bytes(int tile, int taps, int ck, int mode) {
  int tz, ty, tx;
  if (tile == TILE_2x4x16) {
    tz = 2; ty = 4; tx = 16;
  } else if (tile == TILE_1x4x16) {
    tz = 1; ty = 4; tx = 16;
  } else {
    tz = 1; ty = 8; tx = 8;
  }
  const int r = taps == 27 ? 1 : 0;
  const size_t bm = (size_t)tz * ty * tx;
  size_t stage;
  if (mode == PREC_F32) {
    const size_t hp = (size_t)(tz + 2 * r) * (ty + 2 * r) * (tx + 2 * r);
    stage = 4 * (hp * (ck + 1) + bm * 17);
  } else {
    const int parts = mode == PREC_BF16X3 ? 2 : 1;
    const size_t plane = (size_t)(tz + 2 * r) * (ty + 2 * r) * tx + 8;
    stage = parts * 2 * ((taps == 27 ? 3 : 1) * ck * plane + 16 * (bm + 8));
  }
  const size_t xch = taps == 27 ? 0 : (size_t)4 * kWgNg1 * 64 * 16;
  return stage > xch ? stage : xch;
}

// CK: the channel chunk, fixed at compile time for 3x3x3 (8, 16 or 32; it
// sizes the halo prefetch and the column tiles of a wave), 0 for 1x1x1 (read
// from the arguments).
template <int MODE, int TAPS, int TILE, int PRO, int GPRO, int CK>
__global__ __launch_bounds__(256) void k_conv_wgrad(ConvWgrad a) {
  // grid z = member * cout tiles + cout tile
  const int cotiles = (a.cout + 15) / 16;
  const int cz = blockIdx.z % cotiles;
  {
    const long long off = (long long)(blockIdx.z / cotiles) * a.istride;
    a.src = shift_src(a.src, off);
    a.gsrc = shift_src(a.gsrc, off);
    a.part = ishift(a.part, off);
    a.partb = ishift(a.partb, off);
  }
  using MD = Mode<MODE>;
  using ST = typename MD::ST;
  using FT = typename MD::FT;
  using TD = TileDims<TILE>;
  constexpr int TZ = TD::Z, TY = TD::Y, TX = TD::X;
  constexpr int R = TAPS == 27 ? 1 : 0;
  constexpr int HZ = TZ + 2 * R, HY = TY + 2 * R, HX = TX + 2 * R;
  constexpr int HP = HZ * HY * HX;
  constexpr int KPL = MD::KPL, KSTEP = MD::KSTEP;
  constexpr int BM = TZ * TY * TX;
  constexpr int NSTEP = BM / KSTEP;
  constexpr int NCOPY = TAPS == 27 ? 3 : 1;       // BF16: dx-shifted halo copies
  constexpr int PLANE = HZ * HY * TX + 8;          // BF16: elements per (copy, channel)
  constexpr int GP = MD::BF ? BM + 8 : 17;         // g tile row pitch
  constexpr int GSZ = MD::BF ? 16 * GP : BM * GP;
  constexpr bool WCOLS = TAPS == 27;               // waves own column tiles
  static_assert(!WCOLS || CK == 8 || CK == 16 || CK == 32, "3x3x3 needs a fixed chunk");
  constexpr int NJ = WCOLS ? wg_nj(CK) : kWgNg1;   // column tiles per wave
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ float4 bred[256];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, g = lane >> 4;
  const int n = a.n;
  const int ck = CK ? CK : a.ck;
  const int ck_shift = __builtin_ctz(ck);
  const int ckp = ck + 1;                          // FP32 halo row pitch
  const int ntot = TAPS * ck;
  const int ngroups = (ntot + wg_cols(TAPS, ck) - 1) / wg_cols(TAPS, ck);
  const int chunk = blockIdx.y / ngroups, grp = blockIdx.y - chunk * ngroups;
  const int ntx = (n + TX - 1) / TX, nty = (n + TY - 1) / TY, ntz = (n + TZ - 1) / TZ;
  const int ntiles = ntx * nty * ntz;
  const int ci0 = chunk << ck_shift;
  const int co0 = cz * 16;
  const bool do_bias = blockIdx.y == 0;

  // LDS carve
  ST* hal = reinterpret_cast<ST*>(smem);
  const int hal_sz = MD::BF ? NCOPY * ck * PLANE : HP * ckp;
  ST* hal_lo = hal + (MD::SPLIT ? hal_sz : 0);
  ST* gs = hal + (MD::SPLIT ? 2 : 1) * hal_sz;
  ST* gs_lo = gs + (MD::SPLIT ? GSZ : 0);

  // this wave's column tiles (tap, channel): 3x3x3 tile grp*4*NJ + 4j + wave
  // (interleaved, so a wave's tiles past the last column are at its end; their
  // operands read as zero), 1x1x1 tile grp*2 + j shared by all waves
  auto col_tile = [&](int j) { return WCOLS ? grp * 4 * NJ + 4 * j + wave : grp * NJ + j; };
  f32x4 acc[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) acc[j] = (f32x4){0.f, 0.f, 0.f, 0.f};
  int ctap[NJ], cc[NJ], coff[NJ];
  bool cval[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int nn = col_tile(j) * 16 + l16;
    cval[j] = nn < ntot;
    ctap[j] = cval[j] ? nn >> ck_shift : 0;
    cc[j] = nn & (ck - 1);
    if constexpr (MD::BF) {
      // copy dx, channel c, plane offset of (dz, dy)
      const int dz = TAPS == 27 ? ctap[j] / 9 : 0, dy = TAPS == 27 ? (ctap[j] / 3) % 3 : 0;
      const int dx = TAPS == 27 ? ctap[j] % 3 : 0;
      coff[j] = (dx * ck + cc[j]) * PLANE + (dz * HY + dy) * TX;
    } else {
      coff[j] = (TAPS == 27 ? tap_offset(ctap[j], HY, HX) : 0) * ckp + cc[j];
    }
  }
  float4 bacc = make_float4(0.f, 0.f, 0.f, 0.f);

  // staging of a voxel tile (halo of ck input channels, g tile of 16 output
  // channels) goes through registers: the next tile's loads are issued before
  // the current tile's MFMAs
  constexpr int NBH = CK ? (HP * (CK / 4) + 255) / 256 : halo_nb<HP>();
  constexpr int NBG = (BM * 4 + 255) / 256;
  const int qs = ck_shift - 2;
  const int gco = co0 + 4 * (tid & 3);  // output channels of this thread's g quads
  Quads<NBH, PRO> hq;
  Quads<NBG, GPRO> gq;
  HaloIdx<NBH> hidx;
  halo_prep<NBH, HZ, HY, HX>(hidx, n, a.src.stride, qs);
  auto issue = [&](int t) {
    int b = t;
    const int x0 = (b % ntx) * TX;
    b /= ntx;
    const int y0 = (b % nty) * TY;
    b /= nty;
    const int z0 = b * TZ;
    halo_load<NBH, PRO, HZ, HY, HX>(hq, hidx, a.src, n, qs, ci0, z0, y0, x0, R);
    gq.in = 0u;
#pragma unroll
    for (int k = 0; k < NBG; ++k) {
      const int p = k * 256 + tid;
      const int v = p >> 2;
      const int tz = v / (TY * TX), ty = (v / TX) % TY, tx = v % TX;
      const int gz = z0 + tz, gy = y0 + ty, gx = x0 + tx;
      const bool ok = p < BM * 4 && gz < n && gy < n && gx < n && gco < a.cout;
      float4 val = make_float4(0.f, 0.f, 0.f, 0.f), h = val;
      if (ok) {
        const size_t i = ((size_t)(gz * n + gy) * n + gx) * a.cout + gco;
        val = *reinterpret_cast<const float4*>(a.gsrc.x + i);
        if (GPRO == PRO_LN_BWD) h = *reinterpret_cast<const float4*>(a.gsrc.h + i);
      }
      gq.v[k] = val;
      if constexpr (GPRO == PRO_LN_BWD) gq.h[k] = h;
      gq.in |= (ok ? 1u : 0u) << k;
    }
  };
  if ((int)blockIdx.x < ntiles) issue(blockIdx.x);

  float gmean, grstd, gA, gB;
  src_consts<GPRO>(a.gsrc, gmean, grstd, gA, gB);
  float xmean, xrstd, xA, xB;
  src_consts<PRO>(a.src, xmean, xrstd, xA, xB);
  const ChanConsts xk = chan_consts<PRO>(a.src, ci0 + 4 * (tid & ((1 << qs) - 1)));
  ChanConsts gk;
  gk.g = make_float4(1.f, 1.f, 1.f, 1.f);
  gk.b = make_float4(0.f, 0.f, 0.f, 0.f);
  if (gco < a.cout) gk = chan_consts<GPRO>(a.gsrc, gco);

  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    // ---- halo of ck channels
    {
      const int total = HP << qs;
      const int q = tid & ((1 << qs) - 1);
#pragma unroll
      for (int k = 0; k < NBH; ++k) {
        if (k * 256 >= total) break;  // uniform
        const int p = k * 256 + tid;
        if (p >= total) continue;
        const int pos = p >> qs;
        float4 v = hq.v[k];
        if (PRO != PRO_NONE && ((hq.in >> k) & 1u))
          v = apply_pro<PRO>(v, quad_h(hq, k), xk, xmean, xrstd, xA, xB);
        if constexpr (MD::BF) {
          // scatter into the dx copies that contain column hx
          const int hx = pos % HX, hy = (pos / HX) % HY, hz = pos / (HX * HY);
          const float e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int dx = 0; dx < NCOPY; ++dx) {
            const int tx = hx - dx;
            if (tx < 0 || tx >= TX) continue;
            const int base = (hz * HY + hy) * TX + tx;
#pragma unroll
            for (int e4 = 0; e4 < 4; ++e4) {
              const int o = (dx * ck + 4 * q + e4) * PLANE + base;
              if constexpr (MD::SPLIT) {
                uint16_t hi, lo;
                split_bf(e[e4], hi, lo);
                hal[o] = hi;
                hal_lo[o] = lo;
              } else {
                hal[o] = f2bf(e[e4]);
              }
            }
          }
        } else {
          float* d = hal + pos * ckp + 4 * q;
          d[0] = v.x;
          d[1] = v.y;
          d[2] = v.z;
          d[3] = v.w;
        }
      }
    }
    // ---- g tile: BM voxels x 16 output channels (zero outside the grid / cout)
#pragma unroll
    for (int k = 0; k < NBG; ++k) {
      const int p = k * 256 + tid;
      if (p >= BM * 4) continue;
      const int v = p >> 2, q = p & 3;
      float4 val = gq.v[k];
      if (GPRO != PRO_NONE && ((gq.in >> k) & 1u))
        val = apply_pro<GPRO>(val, quad_h(gq, k), gk, gmean, grstd, gA, gB);
      bacc.x += val.x;
      bacc.y += val.y;
      bacc.z += val.z;
      bacc.w += val.w;
      if constexpr (MD::BF) {
        const float e[4] = {val.x, val.y, val.z, val.w};
#pragma unroll
        for (int e4 = 0; e4 < 4; ++e4) {
          if constexpr (MD::SPLIT) {
            uint16_t h, l;
            split_bf(e[e4], h, l);
            gs[(4 * q + e4) * GP + v] = h;
            gs_lo[(4 * q + e4) * GP + v] = l;
          } else {
            gs[(4 * q + e4) * GP + v] = f2bf(e[e4]);
          }
        }
      } else {
        float* d = gs + v * GP + 4 * q;
        d[0] = val.x;
        d[1] = val.y;
        d[2] = val.z;
        d[3] = val.w;
      }
    }
    __syncthreads();
    if (t + (int)gridDim.x < ntiles) issue(t + gridDim.x);
    // ---- 3x3x3: every wave its own column tiles over all voxel k-steps;
    // 1x1x1: every wave all column tiles over k-steps ks = wave, wave + 4, ...
    // A column past the last (tap, channel) reads an in-range halo word
    // (tap 0): column j of an MFMA product depends on column j of B alone, and
    // those accumulators are never written out, so FP32 needs no zero select.
#pragma unroll 8
    for (int ks = WCOLS ? 0 : wave; ks < NSTEP; ks += WCOLS ? 1 : 4) {
      FT A, Al;
      FT B[NJ], Bl[MD::SPLIT ? NJ : 1];
      if constexpr (MD::BF) {
        const int v0 = ks * KSTEP + g * KPL;  // 8 consecutive voxels of one row
        A = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(gs + l16 * GP + v0));
        if constexpr (MD::SPLIT)
          Al = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(gs_lo + l16 * GP + v0));
        const int tz = v0 / (TY * TX), ty = (v0 / TX) % TY, tx = v0 % TX;
        const int vb = (tz * HY + ty) * TX + tx;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          B[j] = frag<MODE>(hal + coff[j] + vb, cval[j]);
          if constexpr (MD::SPLIT) Bl[j] = frag<MODE>(hal_lo + coff[j] + vb, cval[j]);
        }
      } else {
        const int v = ks * KSTEP + g;
        A = gs[v * GP + l16];
        const int tz = v / (TY * TX), ty = (v / TX) % TY, tx = v % TX;
        const int vp = ((tz * HY + ty) * HX + tx) * ckp;
#pragma unroll
        for (int j = 0; j < NJ; ++j) B[j] = frag<MODE>(hal + vp + coff[j], true);
      }
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        if constexpr (MD::SPLIT) {
          acc[j] = mfma(Al, B[j], acc[j]);
          acc[j] = mfma(A, Bl[j], acc[j]);
        }
        acc[j] = mfma(A, B[j], acc[j]);
      }
    }
    __syncthreads();
  }

  const int cout16 = (a.cout + 15) & ~15;
  float* part = a.part + (size_t)blockIdx.x * cout16 * TAPS * a.cin;
  if constexpr (WCOLS) {
    // ---- every wave writes its own column tiles
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int nn = col_tile(j) * 16 + l16;
      if (nn >= ntot) continue;
      const int tap = nn >> ck_shift, c = nn & (ck - 1);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int co = co0 + 4 * g + r;
        if (co < a.cout) part[((size_t)co * TAPS + tap) * a.cin + ci0 + c] = acc[j][r];
      }
    }
  } else {
    // ---- cross-wave exchange (fixed wave order), then this block's partials
    f32x4* xch = reinterpret_cast<f32x4*>(smem);
#pragma unroll
    for (int j = 0; j < NJ; ++j) xch[(wave * NJ + j) * 64 + lane] = acc[j];
    __syncthreads();
    for (int j = wave; j < NJ; j += 4) {
      f32x4 v = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int w = 0; w < 4; ++w) v += xch[(w * NJ + j) * 64 + lane];
      const int nn = col_tile(j) * 16 + l16;
      if (nn >= ntot) continue;
      const int tap = nn >> ck_shift, c = nn & (ck - 1);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int co = co0 + 4 * g + r;
        if (co < a.cout) part[((size_t)co * TAPS + tap) * a.cin + ci0 + c] = v[r];
      }
    }
  }
  if (do_bias) {
    // threads with equal tid & 3 staged the same four channels
    bred[tid] = bacc;
    __syncthreads();
    if (tid < 16) {
      const int q = tid >> 2, e = tid & 3;
      float s = 0.f;
      for (int k = q; k < 256; k += 4) {
        const float4 v = bred[k];
        s += e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
      }
      if (co0 + tid < a.cout) a.partb[(size_t)blockIdx.x * cout16 + co0 + tid] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// dispatch (per mode)
// ---------------------------------------------------------------------------

inline void tile_dims(int tile, int& tz, int& ty, int& tx) {
  if (tile == TILE_2x4x16) {
    tz = 2; ty = 4; tx = 16;
  } else if (tile == TILE_1x4x16) {
    tz = 1; ty = 4; tx = 16;
  } else {
    tz = 1; ty = 8; tx = 8;
  }
}

inline int spatial_tiles(int n, int tile) {
  int tz, ty, tx;
  tile_dims(tile, tz, ty, tx);
  return ((n + tx - 1) / tx) * ((n + ty - 1) / ty) * ((n + tz - 1) / tz);
}

template <int MODE, int TAPS, int TILE, int BN, int PRO>
void launch_fwd(const ConvFwd& a, hipStream_t s) {
  dim3 grid(spatial_tiles(a.n, TILE), (a.cout + BN - 1) / BN, a.ksplit * a.batch);
  const size_t lds = fwd_lds_bytes(TILE, TAPS, BN, a.ck, MODE);
  if constexpr (TAPS == 27) {
    // the plan admits chunks of 8, 16 and 32 channels only
    if (a.ck == 8)
      hipLaunchKernelGGL((k_conv_fwd<MODE, TAPS, TILE, BN, PRO, 8>), grid, dim3(256), lds, s, a);
    else if (a.ck == 16)
      hipLaunchKernelGGL((k_conv_fwd<MODE, TAPS, TILE, BN, PRO, 16>), grid, dim3(256), lds, s, a);
    else
      hipLaunchKernelGGL((k_conv_fwd<MODE, TAPS, TILE, BN, PRO, 32>), grid, dim3(256), lds, s, a);
  } else {
    hipLaunchKernelGGL((k_conv_fwd<MODE, TAPS, TILE, BN, PRO, 0>), grid, dim3(256), lds, s, a);
  }
}

template <int MODE, int TAPS, int TILE, int BN>
void fwd_pro(const ConvFwd& a, hipStream_t s) {
  if constexpr (TAPS == 27) {
    if (a.src.prologue == PRO_LN_RELU) return launch_fwd<MODE, TAPS, TILE, BN, PRO_LN_RELU>(a, s);
    if (a.src.prologue == PRO_LN_BWD) return launch_fwd<MODE, TAPS, TILE, BN, PRO_LN_BWD>(a, s);
  }
  launch_fwd<MODE, TAPS, TILE, BN, PRO_NONE>(a, s);
}

// The 128-voxel tile holds at most 32 output channels per block (16
// accumulator tiles per wave); the engine never asks it for 64.
template <int MODE, int TAPS, int TILE>
void fwd_bn(const ConvFwd& a, hipStream_t s) {
  switch (a.bn) {
    case 16: fwd_pro<MODE, TAPS, TILE, 16>(a, s); break;
    case 32: fwd_pro<MODE, TAPS, TILE, 32>(a, s); break;
    default:
      if constexpr (TILE != TILE_2x4x16) fwd_pro<MODE, TAPS, TILE, 64>(a, s);
      break;
  }
}

template <int TILE, int BN>
void launch_finish_bn(const ConvFwd& a, hipStream_t s) {
  dim3 grid(spatial_tiles(a.n, TILE), (a.cout + BN - 1) / BN, a.batch);
  hipLaunchKernelGGL((k_fwd_finish<TILE, BN>), grid, dim3(256), 0, s, a);
}

template <int TILE>
void launch_finish_tile(const ConvFwd& a, hipStream_t s) {
  switch (a.bn) {
    case 16: launch_finish_bn<TILE, 16>(a, s); break;
    case 32: launch_finish_bn<TILE, 32>(a, s); break;
    default:
      if constexpr (TILE != TILE_2x4x16) launch_finish_bn<TILE, 64>(a, s);
      break;
  }
}

// The split-K finishing launch of a forward pass (ksplit > 1).
inline void launch_finish(const ConvFwd& a, hipStream_t s) {
  switch (a.tile) {
    case TILE_2x4x16: launch_finish_tile<TILE_2x4x16>(a, s); break;
    case TILE_1x4x16: launch_finish_tile<TILE_1x4x16>(a, s); break;
    default: launch_finish_tile<TILE_1x8x8>(a, s); break;
  }
}

template <int MODE, int TAPS>
void fwd_tile(const ConvFwd& a, hipStream_t s) {
  switch (a.tile) {
    case TILE_2x4x16: fwd_bn<MODE, TAPS, TILE_2x4x16>(a, s); break;
    case TILE_1x4x16: fwd_bn<MODE, TAPS, TILE_1x4x16>(a, s); break;
    default: fwd_bn<MODE, TAPS, TILE_1x8x8>(a, s); break;
  }
}

template <int MODE, int TAPS, int TILE, int PRO, int GPRO>
void launch_wg(const ConvWgrad& a, hipStream_t s) {
  dim3 grid(a.splits, (a.cin / a.ck) * conv_wgrad_groups(a.taps, a.ck),
            ((a.cout + 15) / 16) * a.batch);
  const size_t lds = wg_lds_bytes(TILE, TAPS, a.ck, MODE);
  if constexpr (TAPS == 27) {
    // the plan admits chunks of 8, 16 and 32 channels only
    if (a.ck == 8)
      hipLaunchKernelGGL((k_conv_wgrad<MODE, TAPS, TILE, PRO, GPRO, 8>), grid, dim3(256), lds, s, a);
    else if (a.ck == 16)
      hipLaunchKernelGGL((k_conv_wgrad<MODE, TAPS, TILE, PRO, GPRO, 16>), grid, dim3(256), lds, s, a);
    else
      hipLaunchKernelGGL((k_conv_wgrad<MODE, TAPS, TILE, PRO, GPRO, 32>), grid, dim3(256), lds, s, a);
  } else {
    hipLaunchKernelGGL((k_conv_wgrad<MODE, TAPS, TILE, PRO, GPRO, 0>), grid, dim3(256), lds, s, a);
  }
}

template <int MODE, int TAPS, int TILE>
void wg_pro(const ConvWgrad& a, hipStream_t s) {
  if constexpr (TAPS == 27) {
    const bool xr = a.src.prologue == PRO_LN_RELU, gb = a.gsrc.prologue == PRO_LN_BWD;
    if (xr && gb) return launch_wg<MODE, TAPS, TILE, PRO_LN_RELU, PRO_LN_BWD>(a, s);
    if (xr) return launch_wg<MODE, TAPS, TILE, PRO_LN_RELU, PRO_NONE>(a, s);
    if (gb) return launch_wg<MODE, TAPS, TILE, PRO_NONE, PRO_LN_BWD>(a, s);
  }
  launch_wg<MODE, TAPS, TILE, PRO_NONE, PRO_NONE>(a, s);
}

template <int MODE, int TAPS>
void wg_tile(const ConvWgrad& a, hipStream_t s) {
  switch (a.tile) {
    case TILE_2x4x16: wg_pro<MODE, TAPS, TILE_2x4x16>(a, s); break;
    case TILE_1x4x16: wg_pro<MODE, TAPS, TILE_1x4x16>(a, s); break;
    default: wg_pro<MODE, TAPS, TILE_1x8x8>(a, s); break;
  }
}

template <int MODE>
void conv_fwd_mode(const ConvFwd& a, hipStream_t s) {
  if (a.taps == 27) fwd_tile<MODE, 27>(a, s); else fwd_tile<MODE, 1>(a, s);
}

template <int MODE>
void conv_wgrad_mode(const ConvWgrad& a, hipStream_t s) {
  if (a.taps == 27) wg_tile<MODE, 27>(a, s); else wg_tile<MODE, 1>(a, s);
}

}  // namespace conv_detail

// one instantiation per translation unit
void conv_fwd_f32(const ConvFwd& a, hipStream_t s);
void conv_fwd_bf16(const ConvFwd& a, hipStream_t s);
void conv_fwd_bf16x3(const ConvFwd& a, hipStream_t s);
void conv_wgrad_f32(const ConvWgrad& a, hipStream_t s);
void conv_wgrad_bf16(const ConvWgrad& a, hipStream_t s);
void conv_wgrad_bf16x3(const ConvWgrad& a, hipStream_t s);

}  // namespace d2ip
