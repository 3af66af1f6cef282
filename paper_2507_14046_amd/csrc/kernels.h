// Internal launch interface of the D2IP kernels (not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.h"

namespace d2ip {

// Input transform applied while a conv stages its input tile.
enum Prologue { PRO_NONE = 0, PRO_LN_RELU = 1 };

// Operand precision of the conv MFMAs (accumulation is always FP32).
enum ConvPrec { PREC_F32 = 0, PREC_BF16 = 1, PREC_BF16X3 = 2 };

// Spatial output tile of a conv block (TZ x TY x TX voxels).
enum TileCfg { TILE_2x4x16 = 0, TILE_2x8x8 = 1, TILE_COUNT = 2 };

// y[v][co] (+)= sum_{tap, ci} Wp[co][tap][ci] * T(x)[v + off(tap)][ci] (+ bias[co])
// (+ add[v][co]); NDHWC tensors on an n^3 grid, zero padding.  Used for the
// forward conv (Wp = forward packing) and for the input gradient (Wp = flipped,
// transposed packing).
struct ConvFwd {
  const float* x;        // [n^3][cin_stride], fp32
  int n, cin, cin_stride;  // cin: multiple of 8, channels read
  const void* w;         // packed weights [w_rows][taps][cin], fp32 or bf16
  long long w_lo_off;    // PREC_BF16X3: elements from w to its lo-part copy
  int w_rows;            // rows present in w (>= cout)
  const float* bias;     // [cout] or null
  const float* add;      // [n^3][cout] residual added in the epilogue, or null
  int cout;              // output channels written
  int accumulate;        // 1: y += result
  float* y;              // [n^3][cout]
  int taps;              // 27 or 1
  int prologue;          // Prologue
  const LnStat* ln;      // statistics of x (PRO_LN_RELU)
  const float* ln_g;     // gamma[cin] (PRO_LN_RELU)
  const float* ln_b;     // beta[cin]
  double* stat_part;     // per-block (sum, sumsq) of y, or null
  int prec;              // ConvPrec
  int tile;              // TileCfg
};
int conv_fwd_blocks(const ConvFwd& a);  // number of blocks (= stat partials)
void conv_fwd(const ConvFwd& a, hipStream_t s);

// Weight gradient: part[s][co][tap][ci] = sum over voxels of split s of
// g[v][co] * T(x)[v + off(tap)][ci]; bias partials partb[s][co] = sum g[v][co].
struct ConvWgrad {
  const float* x;        // [n^3][cin_stride]
  int n, cin, cin_stride;
  const float* g;        // [n^3][cout]
  int cout;
  int taps;
  int prologue;
  const LnStat* ln;
  const float* ln_g;
  const float* ln_b;
  float* part;           // [splits][cout16][taps][cin]
  float* partb;          // [splits][cout16] or null
  int splits;
  int prec;
  int tile;
};
int conv_wgrad_splits(int n, int cin, int cout, int tile);
size_t conv_wgrad_part_floats(int n, int cin, int cout, int taps, int tile);
void conv_wgrad(const ConvWgrad& a, hipStream_t s);

// gw[co][ci][tap] (canonical) = sum_s part[s][co][tap][ci] for ci < cin_real;
// gb[co] = sum_s partb[s][co].
void wgrad_reduce(const float* part, const float* partb, int splits, int cout, int taps,
                  int cin, int cin_real, float* gw, float* gb, hipStream_t s);


// ---- LayerNorm, ReLU, pooling, up-sampling (norm.hip) ----------------------
enum LnMask { LNMASK_NONE = 0, LNMASK_Y = 1, LNMASK_LN = 2 };

// mean / rstd from `nparts` (sum, sumsq) FP64 partials over `count` elements.
void ln_finalize(const double* part, int nparts, double count, float eps, LnStat* out,
                 hipStream_t s);
// y = relu(g[c] * (h - mean) * rstd + b[c] (+ skip)), [V][C]
void ln_apply(const float* h, const LnStat* st, const float* g, const float* b, const float* skip,
              float* y, size_t V, int C, hipStream_t s);
int ln_bwd_vpb(int C);
int ln_bwd_blocks(size_t V, int C);
// gz = gy * relu'(.) (mask from y > 0, or from g*xhat + b > 0), per-block
// per-channel partial sums of gz and gz * xhat.
void ln_bwd_sums(const float* gy, int mask_mode, const float* my, const float* mg, const float* mb,
                 const float* h, const LnStat* st, float* gz, double* part, size_t V, int C,
                 hipStream_t s);
// dgamma, dbeta and the coefficients A = sum_c gamma_c S1_c / count,
// B = sum_c gamma_c S2_c / count.
void ln_bwd_finalize(const double* part, int nparts, int C, double count, const float* gamma,
                     float* dgamma, float* dbeta, LnBwd* coef, hipStream_t s);
// gh = rstd * (gamma_c * gz - A - xhat * B)
void ln_bwd_apply(const float* gz, const float* h, const LnStat* st, const float* gamma,
                  const LnBwd* coef, float* gh, size_t V, int C, hipStream_t s);
void avgpool2(const float* x, int n, int C, float* y, hipStream_t s);
void up_concat(const float* d, int Cu, const float* e, int Cs, int n, float* cat, hipStream_t s);
void up_concat_bwd(const float* gcat, int Cu, int Cs, int n, float* gu, float* gs, hipStream_t s);
void pool_bwd_add(const float* gx, const float* add, int n, int C, float* gy, hipStream_t s);
void pad_input(const float* z, size_t V, float* zp, hipStream_t s);

// ---- measurement operator, loss, tail, Adam (jops.hip) ----------------------
struct IterState {
  double loss;      // data term of the last iteration
  int t;            // Adam step counter
  int nonfinite;    // set when a non-finite loss was seen
  float bc1, bc2;   // 1 - beta1^t, 1 - beta2^t
};

struct ConvPack {  // one conv of the flat parameter vector
  int th_off, cout, cin_real, cin, taps, need_dgrad;
  long long wf_off, wd_off;  // element offsets in the packed buffers
};

constexpr int kJvecCols = 1024;   // columns per J*sigma block
constexpr int kJvecRows = 16;     // rows per J*sigma block
constexpr int kJtRows = 32;       // rows per J^T g block
inline int jvec_qblocks(int qa_pad) { return (qa_pad + kJvecCols - 1) / kJvecCols; }
inline int jt_mblocks(int M) { return (M + kJtRows - 1) / kJtRows; }

void gather_columns(const float* J, int M, int Q, const int* idx, int qa, int qa_pad, float* Jc,
                    hipStream_t s);
// ppart[qb][m] = sum_{q in block qb} Jc[m][q] * sigma[idx[q]]
void jvec(const float* Jc, int M, int qa_pad, const int* idx, const float* sigma, float* ppart,
          hipStream_t s);
// r = sum_qb ppart - dv; loss = (1/M) sum r^2 (FP64); gp = (2/M) r; t += 1.
void data_loss(const float* ppart, int nqb, const float* dv, int M, float* gp, IterState* it,
               float beta1, float beta2, hipStream_t s);
// tpart[mb][q] = sum_{m in block mb} Jc[m][q] * gp[m]
void jtvec(const float* Jc, int M, int qa_pad, const float* gp, float* tpart, hipStream_t s);
// sigma[v] = mask[v] * (b + sum_c w[c] d0[v][c])
void tail_fwd(const float* d0, int C, const float* w, const float* b, const float* mask, size_t V,
              float* sigma, hipStream_t s);
int tail_bwd_blocks(size_t V, int C);
// gs[v] = sum_mb tpart[mb][inv[v]] (0 where inv < 0); gd0[v][c] = gs[v] w[c];
// part[blk][c] = sum gs*d0[.][c], part[blk][C] = sum gs.
void tail_bwd(const float* tpart, int nmb, int qa_pad, const int* inv, const float* d0, int C,
              const float* w, size_t V, float* gd0, double* part, hipStream_t s);
// dst[k] = sum_i part[i][k]  (k < K)
void reduce_cols(const double* part, int nparts, int K, float* dst, hipStream_t s);
void adam(float* theta, const float* g, float* m, float* v, size_t P, float lr, float beta1,
          float beta2, float eps, const IterState* it, hipStream_t s);
// Packed conv weights from theta; with lo_off > 0 the bf16 lo parts
// (bf16(w - bf16(w))) are written lo_off elements after the hi parts.
void pack_weights(const ConvPack* packs, int npacks, int max_elems, const float* theta,
                  float* wf32, uint16_t* wbf16, long long lo_off, hipStream_t s);

}  // namespace d2ip
