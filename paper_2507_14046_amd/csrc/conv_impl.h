// 3D convolutions of the image prior (3x3x3 and 1x1x1, zero padding) as
// implicit GEMMs on the gfx950 matrix cores.
//
// Forward / input-gradient kernel: the GEMM rows are output voxels of a
// TZ x TY x TX spatial tile, the columns are output channels, the reduction
// runs over (tap, input channel).  Each block stages the input halo of its tile
// for a chunk of CK channels in LDS (applying the LayerNorm+ReLU of the
// producing layer on the fly when asked), then every wave issues 16x16 MFMAs:
// v_mfma_f32_16x16x4_f32 (FP32 operands) or v_mfma_f32_16x16x32_bf16 (BF16
// operands, rounded to nearest even while staging); accumulation is FP32.
// The epilogue adds bias / residual, stores, and emits per-block (sum, sumsq)
// partials in FP64 for the following whole-volume LayerNorm.
//
// Weight-gradient kernel: rows are output channels, columns (tap, channel),
// the reduction runs over voxels; blocks split the voxel range and write
// partial sums that a second kernel reduces in a fixed order (deterministic).
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


template <int TILE>
struct TileDims;
template <>
struct TileDims<TILE_2x4x16> {
  static constexpr int Z = 2, Y = 4, X = 16;
};
template <>
struct TileDims<TILE_2x8x8> {
  static constexpr int Z = 2, Y = 8, X = 8;
};

template <int MODE>
struct Mode {
  static constexpr bool BF = MODE != PREC_F32;        // bf16 operands
  static constexpr bool SPLIT = MODE == PREC_BF16X3;  // hi + lo parts
  static constexpr int KPL = BF ? 8 : 1;              // k per lane per MFMA
  static constexpr int KSTEP = 4 * KPL;               // k per MFMA
  using ST = typename std::conditional<BF, uint16_t, float>::type;  // LDS element
  using FT = typename std::conditional<BF, bf16x8, float>::type;    // MFMA operand
};

__device__ __forceinline__ float ln_relu(float h, float mean, float rstd, float g, float b) {
  float v = g * ((h - mean) * rstd) + b;
  return v > 0.f ? v : 0.f;
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

// Stage a (HZ x HY x HX) halo of CK channels starting at ci0 into LDS
// (rows of CKP elements); the LayerNorm+ReLU prologue is applied to in-grid
// voxels, out-of-grid voxels are the conv's zero padding.
template <int MODE, int CK, int HZ, int HY, int HX, int CKP, int PRO>
__device__ __forceinline__ void stage_halo(typename Mode<MODE>::ST* hal,
                                           typename Mode<MODE>::ST* hal_lo,
                                           const float* __restrict__ x, int n, int cin_stride,
                                           int ci0, int z0, int y0, int x0, int R,
                                           const LnStat* ln, const float* lng, const float* lnb) {
  constexpr int Q = CK / 4;
  constexpr int HP = HZ * HY * HX;
  float mean = 0.f, rstd = 1.f;
  if (PRO == PRO_LN_RELU) {
    mean = ln->mean;
    rstd = ln->rstd;
  }
  for (int p = threadIdx.x; p < HP * Q; p += 256) {
    const int pos = p / Q, q = p - pos * Q;
    const int hx = pos % HX, hy = (pos / HX) % HY, hz = pos / (HX * HY);
    const int gz = z0 + hz - R, gy = y0 + hy - R, gx = x0 + hx - R;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (gz >= 0 && gz < n && gy >= 0 && gy < n && gx >= 0 && gx < n) {
      const int c = ci0 + 4 * q;
      v = *reinterpret_cast<const float4*>(x + (size_t)((gz * n + gy) * n + gx) * cin_stride + c);
      if (PRO == PRO_LN_RELU) {
        v.x = ln_relu(v.x, mean, rstd, lng[c + 0], lnb[c + 0]);
        v.y = ln_relu(v.y, mean, rstd, lng[c + 1], lnb[c + 1]);
        v.z = ln_relu(v.z, mean, rstd, lng[c + 2], lnb[c + 2]);
        v.w = ln_relu(v.w, mean, rstd, lng[c + 3], lnb[c + 3]);
      }
    }
    const int o = pos * CKP + 4 * q;
    if constexpr (Mode<MODE>::SPLIT) {
      uint16_t h0, h1, h2, h3, l0, l1, l2, l3;
      split_bf(v.x, h0, l0);
      split_bf(v.y, h1, l1);
      split_bf(v.z, h2, l2);
      split_bf(v.w, h3, l3);
      *reinterpret_cast<uint2*>(hal + o) = make_uint2(pack2(h0, h1), pack2(h2, h3));
      *reinterpret_cast<uint2*>(hal_lo + o) = make_uint2(pack2(l0, l1), pack2(l2, l3));
    } else if constexpr (Mode<MODE>::BF) {
      *reinterpret_cast<uint2*>(hal + o) =
          make_uint2(pack2(f2bf(v.x), f2bf(v.y)), pack2(f2bf(v.z), f2bf(v.w)));
    } else {
      hal[o + 0] = v.x;
      hal[o + 1] = v.y;
      hal[o + 2] = v.z;
      hal[o + 3] = v.w;
    }
  }
}

__device__ __forceinline__ int tap_offset(int tap, int HY, int HX) {
  const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
  return (dz * HY + dy) * HX + dx;
}

template <int MODE>
__device__ __forceinline__ typename Mode<MODE>::FT lds_frag(const typename Mode<MODE>::ST* p,
                                                            bool ok) {
  if constexpr (Mode<MODE>::BF) {
    u32x4 v = {0u, 0u, 0u, 0u};
    if (ok) v = *reinterpret_cast<const u32x4*>(p);
    return __builtin_bit_cast(bf16x8, v);
  } else {
    return ok ? *p : 0.f;
  }
}

template <int MODE>
__device__ __forceinline__ typename Mode<MODE>::FT glb_frag(const typename Mode<MODE>::ST* p,
                                                            bool ok) {
  if constexpr (Mode<MODE>::BF) {
    u32x4 v = {0u, 0u, 0u, 0u};
    if (ok) v = *reinterpret_cast<const u32x4*>(p);
    return __builtin_bit_cast(bf16x8, v);
  } else {
    return ok ? *p : 0.f;
  }
}

template <int MODE, int TAPS, int CK, int TILE, int BN, int PRO>
__global__ __launch_bounds__(256) void k_conv_fwd(ConvFwd a) {
  using MD = Mode<MODE>;
  using ST = typename MD::ST;
  using FT = typename MD::FT;
  using TD = TileDims<TILE>;
  constexpr int TZ = TD::Z, TY = TD::Y, TX = TD::X;
  constexpr int R = TAPS == 27 ? 1 : 0;
  constexpr int HZ = TZ + 2 * R, HY = TY + 2 * R, HX = TX + 2 * R, HP = HZ * HY * HX;
  constexpr int KPL = MD::KPL, KSTEP = MD::KSTEP;
  constexpr int NSTEP = (TAPS * CK + KSTEP - 1) / KSTEP;
  constexpr bool KEXACT = (TAPS * CK) % KSTEP == 0;
  constexpr int CKP = MD::BF ? CK + 8 : CK + 1;
  constexpr int BM = TZ * TY * TX, MT = BM / 16, MTW = MT / 4, NT = BN / 16;
  static_assert(MT % 4 == 0, "tile must hold a multiple of 64 voxels");
  __shared__ __align__(16) ST hal[HP * CKP];
  __shared__ __align__(16) ST hal_lo[MD::SPLIT ? HP * CKP : 8];
  __shared__ double red[8];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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

  f32x4 acc[MTW][NT];
#pragma unroll
  for (int i = 0; i < MTW; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};

  int apos[MTW];
#pragma unroll
  for (int mt = 0; mt < MTW; ++mt) {
    const int li = (wave * MTW + mt) * 16 + l16;
    const int tz = li / (TY * TX), ty = (li / TX) % TY, tx = li % TX;
    apos[mt] = (tz * HY + ty) * HX + tx;
  }

  const ST* __restrict__ W = reinterpret_cast<const ST*>(a.w);
  const ST* __restrict__ Wlo = W + a.w_lo_off;
  for (int ci0 = 0; ci0 < a.cin; ci0 += CK) {
    stage_halo<MODE, CK, HZ, HY, HX, CKP, PRO>(hal, hal_lo, a.x, n, a.cin_stride, ci0, z0, y0, x0,
                                               R, a.ln, a.ln_g, a.ln_b);
    __syncthreads();
#pragma unroll 2
    for (int step = 0; step < NSTEP; ++step) {
      const int kl = step * KSTEP + g * KPL;
      const int tap = kl / CK, c = kl - tap * CK;
      const bool kv = KEXACT || tap < TAPS;
      const int toff = TAPS == 27 ? tap_offset(tap, HY, HX) : 0;
      FT A[MTW], B[NT];
      FT Al[MD::SPLIT ? MTW : 1], Bl[MD::SPLIT ? NT : 1];
#pragma unroll
      for (int mt = 0; mt < MTW; ++mt) {
        const int o = (apos[mt] + toff) * CKP + c;
        A[mt] = lds_frag<MODE>(hal + o, kv);
        if constexpr (MD::SPLIT) Al[mt] = lds_frag<MODE>(hal_lo + o, kv);
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int co = co0 + nt * 16 + l16;
        const bool ok = kv && co < a.w_rows;
        const size_t wi = ((size_t)co * TAPS + tap) * a.cin + ci0 + c;
        B[nt] = glb_frag<MODE>(W + wi, ok);
        if constexpr (MD::SPLIT) Bl[nt] = glb_frag<MODE>(Wlo + wi, ok);
      }
#pragma unroll
      for (int mt = 0; mt < MTW; ++mt)
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

  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int mt = 0; mt < MTW; ++mt) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int li = (wave * MTW + mt) * 16 + 4 * g + r;
      const int tz = li / (TY * TX), ty = (li / TX) % TY, tx = li % TX;
      const int gz = z0 + tz, gy = y0 + ty, gx = x0 + tx;
      if (gz >= n || gy >= n || gx >= n) continue;
      const size_t vox = (size_t)(gz * n + gy) * n + gx;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int co = co0 + nt * 16 + l16;
        if (co >= a.cout) continue;
        const size_t o = vox * a.cout + co;
        float v = acc[mt][nt][r];
        if (a.bias) v += a.bias[co];
        if (a.add) v += a.add[o];
        if (a.accumulate) v += a.y[o];
        a.y[o] = v;
        s1 += v;
        s2 += (double)v * v;
      }
    }
  }
  if (a.stat_part) {
    s1 = block_sum(s1, red);
    s2 = block_sum(s2, red);
    if (tid == 0) {
      const size_t pb = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
      a.stat_part[2 * pb] = s1;
      a.stat_part[2 * pb + 1] = s2;
    }
  }
}

template <int MODE, int TAPS, int CK, int TILE, int PRO>
__global__ __launch_bounds__(256) void k_conv_wgrad(ConvWgrad a) {
  using MD = Mode<MODE>;
  using ST = typename MD::ST;
  using FT = typename MD::FT;
  using TD = TileDims<TILE>;
  constexpr int TZ = TD::Z, TY = TD::Y, TX = TD::X;
  constexpr int R = TAPS == 27 ? 1 : 0;
  constexpr int HZ = TZ + 2 * R, HY = TY + 2 * R, HX = TX + 2 * R;
  constexpr int HP = HZ * HY * HX;
  constexpr int KPL = MD::KPL, KSTEP = MD::KSTEP;
  constexpr int CKP = MD::BF ? CK + 8 : CK + 1;
  constexpr int BM = TZ * TY * TX;
  constexpr int NTOT = TAPS * CK;
  constexpr int NT = (NTOT + 15) / 16;
  constexpr int NTW = (NT + 3) / 4;
  constexpr int GP = MD::BF ? BM + 8 : 17;  // g tile row pitch
  constexpr int GSZ = MD::BF ? 16 * GP : BM * GP;
  __shared__ __align__(16) ST hal[HP * CKP];
  __shared__ __align__(16) ST hal_lo[MD::SPLIT ? HP * CKP : 8];
  // BF16: gs[co][voxel]; FP32: gs[voxel][co]
  __shared__ __align__(16) ST gs[GSZ];
  __shared__ __align__(16) ST gs_lo[MD::SPLIT ? GSZ : 8];
  __shared__ float bred[256];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const int n = a.n;
  const int ntx = (n + TX - 1) / TX, nty = (n + TY - 1) / TY, ntz = (n + TZ - 1) / TZ;
  const int ntiles = ntx * nty * ntz;
  const int ci0 = blockIdx.y * CK;
  const int co0 = blockIdx.z * 16;
  const bool do_bias = a.partb != nullptr && blockIdx.y == 0;

  f32x4 acc[NTW];
#pragma unroll
  for (int j = 0; j < NTW; ++j) acc[j] = (f32x4){0.f, 0.f, 0.f, 0.f};
  float bacc = 0.f;

  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int b = t;
    const int x0 = (b % ntx) * TX;
    b /= ntx;
    const int y0 = (b % nty) * TY;
    b /= nty;
    const int z0 = b * TZ;
    stage_halo<MODE, CK, HZ, HY, HX, CKP, PRO>(hal, hal_lo, a.x, n, a.cin_stride, ci0, z0, y0, x0,
                                               R, a.ln, a.ln_g, a.ln_b);
    // g tile: BM voxels x 16 output channels (zero outside the grid / cout)
    for (int p = tid; p < BM * 4; p += 256) {
      const int v = p >> 2, q = p & 3;
      const int tz = v / (TY * TX), ty = (v / TX) % TY, tx = v % TX;
      const int gz = z0 + tz, gy = y0 + ty, gx = x0 + tx;
      const int co = co0 + 4 * q;
      float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
      if (gz < n && gy < n && gx < n && co < a.cout)
        val = *reinterpret_cast<const float4*>(a.g + ((size_t)(gz * n + gy) * n + gx) * a.cout + co);
      if constexpr (MD::BF) {
        const float e[4] = {val.x, val.y, val.z, val.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if constexpr (MD::SPLIT) {
            uint16_t h, l;
            split_bf(e[k], h, l);
            gs[(4 * q + k) * GP + v] = h;
            gs_lo[(4 * q + k) * GP + v] = l;
          } else {
            gs[(4 * q + k) * GP + v] = f2bf(e[k]);
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
    // bias partial in FP32 from the unrounded gradient
    if (do_bias) {
      const int co = tid & 15;
      if (co0 + co < a.cout) {
        for (int v = tid >> 4; v < BM; v += 16) {
          const int tz = v / (TY * TX), ty = (v / TX) % TY, tx = v % TX;
          const int gz = z0 + tz, gy = y0 + ty, gx = x0 + tx;
          if (gz < n && gy < n && gx < n)
            bacc += a.g[((size_t)(gz * n + gy) * n + gx) * a.cout + co0 + co];
        }
      }
    }
#pragma unroll 2
    for (int ks = 0; ks < BM / KSTEP; ++ks) {
      FT A, Al;
      FT B[NTW], Bl[MD::SPLIT ? NTW : 1];
      if constexpr (MD::BF) {
        const int v0 = ks * KSTEP + g * KPL;
        A = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(gs + l16 * GP + v0));
        if constexpr (MD::SPLIT)
          Al = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(gs_lo + l16 * GP + v0));
#pragma unroll
        for (int j = 0; j < NTW; ++j) {
          const int nn = (wave + 4 * j) * 16 + l16;
          uint16_t e[8], el[8];
          if (nn < NTOT) {
            const int tap = nn / CK, c = nn - tap * CK;
            const int toff = TAPS == 27 ? tap_offset(tap, HY, HX) : 0;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const int v = v0 + q;
              const int tz = v / (TY * TX), ty = (v / TX) % TY, tx = v % TX;
              const int o = ((tz * HY + ty) * HX + tx + toff) * CKP + c;
              e[q] = hal[o];
              if constexpr (MD::SPLIT) el[q] = hal_lo[o];
            }
          } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              e[q] = 0;
              el[q] = 0;
            }
          }
          u32x4 pk = {pack2(e[0], e[1]), pack2(e[2], e[3]), pack2(e[4], e[5]), pack2(e[6], e[7])};
          B[j] = __builtin_bit_cast(bf16x8, pk);
          if constexpr (MD::SPLIT) {
            u32x4 pl = {pack2(el[0], el[1]), pack2(el[2], el[3]), pack2(el[4], el[5]),
                        pack2(el[6], el[7])};
            Bl[j] = __builtin_bit_cast(bf16x8, pl);
          }
        }
      } else {
        const int v = ks * KSTEP + g;
        A = gs[v * GP + l16];
        const int tz = v / (TY * TX), ty = (v / TX) % TY, tx = v % TX;
        const int vp = (tz * HY + ty) * HX + tx;
#pragma unroll
        for (int j = 0; j < NTW; ++j) {
          const int nn = (wave + 4 * j) * 16 + l16;
          float e = 0.f;
          if (nn < NTOT) {
            const int tap = nn / CK, c = nn - tap * CK;
            const int toff = TAPS == 27 ? tap_offset(tap, HY, HX) : 0;
            e = hal[(vp + toff) * CKP + c];
          }
          B[j] = e;
        }
      }
#pragma unroll
      for (int j = 0; j < NTW; ++j) {
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
#pragma unroll
  for (int j = 0; j < NTW; ++j) {
    const int nt = wave + 4 * j;
    if (nt >= NT) continue;
    const int nn = nt * 16 + l16;
    if (nn >= NTOT) continue;
    const int tap = nn / CK, c = nn - tap * CK;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int co = co0 + 4 * g + r;
      if (co < a.cout) part[((size_t)co * TAPS + tap) * a.cin + ci0 + c] = acc[j][r];
    }
  }
  if (do_bias) {
    bred[tid] = bacc;
    __syncthreads();
    if (tid < 16) {
      float s = 0.f;
      for (int k = tid; k < 256; k += 16) s += bred[k];
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
  } else {
    tz = 2; ty = 8; tx = 8;
  }
}

inline int spatial_tiles(int n, int tile) {
  int tz, ty, tx;
  tile_dims(tile, tz, ty, tx);
  return ((n + tx - 1) / tx) * ((n + ty - 1) / ty) * ((n + tz - 1) / tz);
}

inline int pick_ck(int cin) {
  if (cin % 32 == 0) return 32;
  if (cin % 16 == 0) return 16;
  return 8;
}

inline int pick_bn(int cout) {
  if (cout <= 16) return 16;
  if (cout <= 32) return 32;
  return 64;
}

template <int MODE, int TAPS, int CK, int TILE, int BN, int PRO>
void launch_fwd(const ConvFwd& a, hipStream_t s) {
  dim3 grid(spatial_tiles(a.n, TILE), (a.cout + BN - 1) / BN);
  hipLaunchKernelGGL((k_conv_fwd<MODE, TAPS, CK, TILE, BN, PRO>), grid, dim3(256), 0, s, a);
}

template <int MODE, int TAPS, int CK, int TILE, int BN>
void fwd_pro(const ConvFwd& a, hipStream_t s) {
  if (a.prologue == PRO_LN_RELU && TAPS == 27)
    launch_fwd<MODE, TAPS, CK, TILE, BN, PRO_LN_RELU>(a, s);
  else
    launch_fwd<MODE, TAPS, CK, TILE, BN, PRO_NONE>(a, s);
}

template <int MODE, int TAPS, int CK, int TILE>
void fwd_bn(const ConvFwd& a, hipStream_t s) {
  switch (pick_bn(a.cout)) {
    case 16: fwd_pro<MODE, TAPS, CK, TILE, 16>(a, s); break;
    case 32: fwd_pro<MODE, TAPS, CK, TILE, 32>(a, s); break;
    default: fwd_pro<MODE, TAPS, CK, TILE, 64>(a, s); break;
  }
}

template <int MODE, int TAPS, int CK>
void fwd_tile(const ConvFwd& a, hipStream_t s) {
  if (a.tile == TILE_2x4x16)
    fwd_bn<MODE, TAPS, CK, TILE_2x4x16>(a, s);
  else
    fwd_bn<MODE, TAPS, CK, TILE_2x8x8>(a, s);
}

template <int MODE, int TAPS>
void fwd_ck(const ConvFwd& a, hipStream_t s) {
  switch (pick_ck(a.cin)) {
    case 32: fwd_tile<MODE, TAPS, 32>(a, s); break;
    case 16: fwd_tile<MODE, TAPS, 16>(a, s); break;
    default: fwd_tile<MODE, TAPS, 8>(a, s); break;
  }
}

template <int MODE, int TAPS, int CK, int TILE, int PRO>
void launch_wg(const ConvWgrad& a, hipStream_t s) {
  dim3 grid(a.splits, a.cin / CK, (a.cout + 15) / 16);
  hipLaunchKernelGGL((k_conv_wgrad<MODE, TAPS, CK, TILE, PRO>), grid, dim3(256), 0, s, a);
}

template <int MODE, int TAPS, int CK, int TILE>
void wg_pro(const ConvWgrad& a, hipStream_t s) {
  if (a.prologue == PRO_LN_RELU && TAPS == 27)
    launch_wg<MODE, TAPS, CK, TILE, PRO_LN_RELU>(a, s);
  else
    launch_wg<MODE, TAPS, CK, TILE, PRO_NONE>(a, s);
}

template <int MODE, int TAPS, int CK>
void wg_tile(const ConvWgrad& a, hipStream_t s) {
  if (a.tile == TILE_2x4x16)
    wg_pro<MODE, TAPS, CK, TILE_2x4x16>(a, s);
  else
    wg_pro<MODE, TAPS, CK, TILE_2x8x8>(a, s);
}

template <int MODE, int TAPS>
void wg_ck(const ConvWgrad& a, hipStream_t s) {
  switch (pick_ck(a.cin)) {
    case 32: wg_tile<MODE, TAPS, 32>(a, s); break;
    case 16: wg_tile<MODE, TAPS, 16>(a, s); break;
    default: wg_tile<MODE, TAPS, 8>(a, s); break;
  }
}

template <int MODE>
void conv_fwd_mode(const ConvFwd& a, hipStream_t s) {
  if (a.taps == 27) fwd_ck<MODE, 27>(a, s); else fwd_ck<MODE, 1>(a, s);
}

template <int MODE>
void conv_wgrad_mode(const ConvWgrad& a, hipStream_t s) {
  if (a.taps == 27) wg_ck<MODE, 27>(a, s); else wg_ck<MODE, 1>(a, s);
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
