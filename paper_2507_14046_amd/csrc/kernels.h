// Internal launch interface of the D2IP kernels (not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.h"

namespace d2ip {

// Input transform applied while a conv stages an operand tile.
//   PRO_LN_RELU: x -> relu(gamma_c * (x - mean) * rstd + beta_c)
//   PRO_LN_BWD : gz -> rstd * (gamma_c * gz - A - xhat * B), xhat from the
//                pre-norm activation h (LayerNorm backward, whole volume)
enum Prologue { PRO_NONE = 0, PRO_LN_RELU = 1, PRO_LN_BWD = 2 };

// Operand precision of the conv MFMAs (accumulation is always FP32).
enum ConvPrec { PREC_F32 = 0, PREC_BF16 = 1, PREC_BF16X3 = 2 };

// Spatial output tile of a conv block (TZ x TY x TX voxels).
enum TileCfg { TILE_2x4x16 = 0, TILE_1x4x16 = 1, TILE_1x8x8 = 2, TILE_COUNT = 3 };

// Operand tile source with its prologue.
struct ConvSrc {
  const float* x;        // [n^3][stride] fp32
  int stride;
  int prologue;          // Prologue
  PairRef st;            // statistics partials of the normalised tensor
  const float* gamma;    // [channels]
  const float* beta;     // [channels] (PRO_LN_RELU)
  const float* h;        // PRO_LN_BWD: pre-norm activation, same layout as x
  PairRef bw;            // PRO_LN_BWD: partials of the coefficients A, B
};

// Shift every per-member pointer of a source by `off` bytes.
__host__ __device__ inline ConvSrc shift_src(ConvSrc s, long long off) {
  s.x = ishift(s.x, off);
  s.gamma = ishift(s.gamma, off);
  s.beta = ishift(s.beta, off);
  s.h = ishift(s.h, off);
  s.st.part = ishift(s.st.part, off);
  s.bw.part = ishift(s.bw.part, off);
  return s;
}

// y[v][co] (+)= sum_{tap, ci} Wp[co][tap][ci] * T(x)[v + off(tap)][ci] (+ bias[co])
// (+ add[v][co]); NDHWC tensors on an n^3 grid, zero padding.  Used for the
// forward conv (Wp = forward packing) and the input gradient (Wp = flipped,
// transposed packing).  With ksplit > 1 the channel chunks are split over
// blocks, which store partial tiles; a second launch (conv_fwd issues it)
// sums them in split order and runs the epilogue.  With stat_part set, every output tile writes
// the (sum, sumsq) pair of its outputs for the following LayerNorm.
struct ConvFwd {
  ConvSrc src;
  int n, cin;            // cin: multiple of ck, channels read
  const void* w;         // packed weights [w_rows][taps][cin], fp32 or bf16
  long long w_lo_off;    // PREC_BF16X3: elements from w to its lo-part copy
  int w_rows;            // rows present in w (>= cout)
  const float* bias;     // [cout] or null
  const float* add;      // [n^3][cout] residual added in the epilogue, or null
  int cout;              // output channels written
  int accumulate;        // 1: y += result
  float* y;              // [n^3][cout]
  int taps;              // 27 or 1
  double* stat_part;     // per-tile (sum, sumsq) of y, or null
  int prec, tile, bn, ck, ksplit;
  float* kpart;          // [ksplit][n^3][cout] (ksplit > 1; a second launch sums them)
  int batch;             // group members (grid z = ksplit * batch)
  long long istride;     // bytes between members' data
};
int conv_tiles(int n, int tile);
int conv_fwd_blocks(const ConvFwd& a);  // output tiles (= stat partials)
// dynamic LDS of a forward/input-gradient launch (halo + weight slab)
size_t conv_fwd_lds_bytes(int tile, int taps, int bn, int ck, int prec);
void conv_fwd(const ConvFwd& a, hipStream_t s);

// Weight gradient partials: part[s][co][tap][ci] = sum over the voxels of
// split s of T(g)[v][co] * T(x)[v + off(tap)][ci]; partb[s][co] = sum T(g)[v][co].
struct ConvWgrad {
  ConvSrc src;           // x operand
  ConvSrc gsrc;          // g operand (PRO_NONE or PRO_LN_BWD), stride = cout
  int n, cin, cout, taps;
  float* part;           // [splits][cout16][taps][cin]
  float* partb;          // [splits][cout16]
  int splits, prec, tile, ck;
  int batch;             // group members (grid z = cout tiles * batch)
  long long istride;
};
int conv_wgrad_groups(int taps, int ck);
size_t conv_wgrad_lds_bytes(int tile, int taps, int ck, int prec);
void conv_wgrad(const ConvWgrad& a, hipStream_t s);

// One slice of the batched gradient reduction at the end of an iteration.
//  kind 0 (conv): g[th_w + (co*cin_real + ci)*taps + tap] = sum_s part[s][co][tap][ci]
//                 and g[th_b + co] = sum_s partb[s][co]   (float partials)
//  kind 1 (columns): g[th_w + k] = sum_i dpart[i][k], k < cout (double
//                 partials [splits][cout]: LayerNorm gains/shifts, output head)
struct GradSeg {
  int kind;
  long long part_off, partb_off;  // offsets in the partial buffers
  int splits, cout, taps, cin, cin_real;
  int th_w, th_b;
};
void grad_reduce(const GradSeg* segs, int nsegs, int max_elems, const float* part,
                 const float* partb, const double* dpart, float* grad, int batch,
                 long long istride, hipStream_t s);

// ---- LayerNorm, ReLU, pooling, up-sampling (norm.hip) ----------------------
enum LnMask { LNMASK_NONE = 0, LNMASK_Y = 1, LNMASK_LN = 2 };

// y = relu(g[c] * (h - mean) * rstd + b[c] (+ skip)), [V][C]
void ln_apply(const float* h, PairRef st, const float* g, const float* b, const float* skip,
              float* y, size_t V, int C, int batch, long long istride, hipStream_t s);
// the same on an n^3 grid (n even), also writing the 2x2x2 average of y
// (the next encoder input) when `pooled` is not null
void ln_apply_pool(const float* h, PairRef st, const float* g, const float* b, const float* skip,
                   float* y, float* pooled, int n, int C, int batch, long long istride,
                   hipStream_t s);
int ln_bwd_vpb(int C);
int ln_bwd_blocks(size_t V, int C);
// gz = gy * relu'(.) (mask from y > 0, or from g*xhat + b > 0); per block:
// part_c[blk][c] = sum gz*xhat (dgamma), part_c[blk][C + c] = sum gz (dbeta),
// part_ab[blk] = (sum_c gamma_c sum gz, sum_c gamma_c sum gz*xhat), whose
// totals over `count` elements are the coefficients A, B of
// dh = rstd * (gamma_c * gz - A - xhat * B).
void ln_bwd(const float* gy, int mask_mode, const float* my, const float* mg, const float* mb,
            const float* h, PairRef st, float* gz, double* part_c, double* part_ab, size_t V,
            int C, const float* gamma, int batch, long long istride, hipStream_t s);
void avgpool2(const float* x, int n, int C, float* y, hipStream_t s);
void up_concat(const float* d, int Cu, const float* e, int Cs, int n, float* cat, int batch,
               long long istride, hipStream_t s);
void up_concat_bwd(const float* gcat, int Cu, int Cs, int n, float* gu, float* gs, int batch,
                   long long istride, hipStream_t s);
void pool_bwd_add(const float* gx, const float* add, int n, int C, float* gy, int batch,
                  long long istride, hipStream_t s);
void pad_input(const float* z, size_t V, float* zp, hipStream_t s);
// out[i] = sum over rows k of part[k][i] (FP64 partials, i < ncols), summed
// in a fixed order in two passes (tmp holds colsum_tmp_doubles values).
size_t colsum_tmp_doubles(int nrows, int ncols);
void colsum_f64(const double* part, int nrows, int ncols, double* tmp, float* out, hipStream_t s);
// ---- output head and attention unit (modules.hip) ---------------------------
int head_max_c();
size_t head_scratch_bytes(size_t V, int C);
void head_forward(const float* x, const float* w, const float* b, const float* mask, size_t V,
                  int C, int sig, float* out, hipStream_t s);
void head_backward(const float* x, const float* w, const float* b, const float* mask,
                   const float* gout, size_t V, int C, int sig, float* gx, float* gw, float* gb,
                   void* scratch, hipStream_t s);
// Channel range copy between channels-last tensors (counts and offsets
// multiples of 4) and ReLU forward / backward on count values (count % 4 == 0).
void channel_copy(const float* src, int sC, int soff, float* dst, int dC, int doff, int c,
                  size_t V, hipStream_t s);
void relu_forward(const float* x, float* y, size_t count, hipStream_t s);
void relu_backward(const float* y, const float* gy, float* gx, size_t count, hipStream_t s);
int att_max_c();
int att_max_cu();
// Wider channels run the composed form (pointwise GEMMs and gate kernels).
int att_max_c_wide();
int att_max_cu_wide();
size_t att_scratch_bytes(int n, int c, int cu);
void att_forward(const float* x, const float* g, const float* wx, const float* wg, const float* b,
                 const float* psi, const float* bpsi, float* y, float* alpha, int n, int c, int cu,
                 void* scratch, hipStream_t s);
void att_backward(const float* x, const float* g, const float* wx, const float* wg,
                  const float* b, const float* psi, const float* bpsi, const float* gy,
                  float* gx, float* gg, float* gwx, float* gwg, float* gb, float* gpsi,
                  float* gbpsi, int n, int c, int cu, void* scratch, hipStream_t s);

// n 4-byte words at p set to zero by a kernel (a graph records a kernel node)
void zero_words(void* p, size_t n, hipStream_t s);

// ---- measurement operator, loss, tail, Adam (jops.hip) ----------------------
struct IterState {
  double loss;      // data term of the last iteration
  int t;            // Adam step counter
  int nonfinite;    // set when a non-finite loss was seen
  float bc1, bc2;   // 1 - beta1^t, 1 - beta2^t
};

// 4D-TV state of one instance (Sec. III-E): the last `count` frames' images
// sit in a ring of kTvHistory slots, the k-th most recent (k = 1..count) in
// slot (head - k + 1) mod kTvHistory, with normalised weight w[k - 1].
constexpr int kTvHistory = 32;
struct TvState {
  int count, head;
  float w[kTvHistory];
};
// Coefficients of the 4D-TV term.
struct TvCoef {
  float lam, lam_s, lam_t, eps;
};

struct ConvPack {  // one conv of the flat parameter vector
  int th_off, cout, cin_real, cin, taps, need_dgrad;
  long long wf_off, wd_off;  // element offsets in the packed buffers
};

constexpr int kJvecCols = 1024;   // columns per J*sigma block
constexpr int kJvecRows = 8;      // rows per J*sigma block
constexpr int kJtRows = 32;       // rows per J^T g block
constexpr int kJMaxB = 8;         // group members per J-product launch (J read once)
inline int jvec_qblocks(int qa_pad) { return (qa_pad + kJvecCols - 1) / kJvecCols; }
inline int jt_mblocks(int M) { return (M + kJtRows - 1) / kJtRows; }
// Column blocks of J sigma partials up to which every J^T g block forms its
// rows' residual itself; above it (large grids) the residual is formed once
// (k_resid) and J^T g runs over longer row groups, about 1024 blocks in all,
// so it writes fewer partials.
constexpr int kJtFuseMax = 32;
inline int jt_rows_per_group(int M, int qa_pad) {
  const int nqb = jvec_qblocks(qa_pad);
  if (nqb <= kJtFuseMax) return kJtRows;
  int R = (1024 + nqb - 1) / nqb;
  if (R > jt_mblocks(M)) R = jt_mblocks(M);
  if (R < 1) R = 1;
  return ((M + R - 1) / R + 7) / 8 * 8;  // a multiple of 8: aligned batches of rows
}
// Row groups of J^T g partials (tpart rows) for an M x qa_pad compact J.
inline int jt_partials(int M, int qa_pad) {
  const int rpg = jt_rows_per_group(M, qa_pad);
  return (M + rpg - 1) / rpg;
}

void gather_columns(const float* J, int M, int Q, const int* idx, int qa, int qa_pad, float* Jc,
                    hipStream_t s);
// ppart[qb][m] = sum_{q in column block qb} Jc[m][q] * sigma[idx[q]]
void jvec(const float* Jc, int M, int qa_pad, const int* idx, const float* sigma, float* ppart,
          int batch, long long istride, hipStream_t s);
// For every group of kJtRows rows: p = sum_qb ppart (column-block order),
// r = p - dv, gp = (2/M) r and rsum[mb] = sum r^2 (FP64); then for each of
// the jt_partials(M, qa_pad) row groups g: tpart[g][q] = sum_{m in g}
// Jc[m][q] gp[m].  (Few column blocks: every J^T g block forms its rows'
// residual; many: one residual launch first, then longer row groups.)
void jtvec(const float* Jc, int M, int qa_pad, const float* ppart, int nqb, const float* dv,
           double* rsum, float* tpart, int batch, long long istride, hipStream_t s);
// sigma[v] = mask[v] * (b + sum_c w[c] d0[v][c])
void tail_fwd(const float* d0, int C, const float* w, const float* b, const float* mask, size_t V,
              float* sigma, int batch, long long istride, hipStream_t s);
int tail_bwd_blocks(size_t V, int C);
// gs[v] = sum_mb tpart[mb][inv[v]] (0 where inv < 0); gd0[v][c] = gs[v] w[c];
// part[blk][c] = sum gs*d0[.][c], part[blk][C] = sum gs (gradient of the head,
// reduced by grad_reduce).
void tail_bwd(const float* tpart, int nmb, int qa_pad, const int* inv, const float* d0, int C,
              const float* w, size_t V, float* gd0, double* part, const float* gtv, int batch,
              long long istride, hipStream_t s);
// Adam step t + 1 (t = it->t, bias corrections 1 - beta^(t+1)); a non-finite
// updated parameter sets bit 1 of it->nonfinite.
void adam(float* theta, const float* g, float* m, float* v, size_t P, float lr, float beta1,
          float beta2, float eps, IterState* it, int batch, long long istride,
          hipStream_t s);
// Packed conv weights from theta; with lo_off > 0 the bf16 lo parts
// (bf16(w - bf16(w))) are written lo_off elements after the hi parts.  When
// `it` is set this ends an iteration: it->loss = sum(rsum[0..nrs)) / M (FP64),
// the non-finite flag, and t += 1.
void pack_weights(const ConvPack* packs, int npacks, int max_elems, const float* theta,
                  float* wf32, uint16_t* wbf16, long long lo_off, IterState* it,
                  const double* rsum, int nrs, int M, const double* tvsum, int ntv, int batch,
                  long long istride, hipStream_t s);
int tv_blocks(size_t V);
// 4D-TV of the image sigma (n^3): gtv = d(lam * R_4D-TV)/d sigma and per-block
// partial sums of lam * R_4D-TV (Eqs. (11)-(13)); history per TvState.
void tv_reg(const float* sigma, int n, const float* hist, const TvState* ts, TvCoef c, float* gtv,
            double* tvsum, int batch, long long istride, hipStream_t s);

// ---- standalone operators (op-level C-ABI) ----
int block_stats_blocks(size_t n);
// part[b] = (sum, sum of squares) of a contiguous range of x (FP64).
void block_stats(const float* x, size_t n, double* part, hipStream_t s);
// gx = rstd * (gamma_c * gz - A - xhat * B) (LayerNorm input gradient).
void ln_dx(const float* gz, const float* h, PairRef st, PairRef bw, const float* gamma, float* gx,
           size_t V, int C, hipStream_t s);
// p = J sigma and out = J^T g for a dense row-major M x Q J (Q % 4 == 0).
void jv_dense(const float* J, int M, int Q, const float* sigma, float* p, hipStream_t s);
size_t jt_dense_scratch(int Q);  // floats of `part`
// loss = (1/M) sum (p - dv)^2 (FP64 accumulation, one block), gp = (2/M)(p - dv)
void mse_loss(const float* p, const float* dv, int M, float* gp, double* loss, hipStream_t s);
void jt_dense(const float* J, int M, int Q, const float* g, float* part, float* out,
              hipStream_t s);
// Depthwise 3x3x3 convolution (channels-last [n^3][C], C % 4 == 0, w [C][27]):
// y = b + depthwise(x, w), or with flip the input gradient (taps reversed, b
// unused); dw_wgrad writes dw_partials(n, C) floats of `part` and reduces them
// into gw [C][27] and gb [C] (either may be null).
size_t dw_partials(int n, int C);
void dw_forward(const float* x, const float* w, const float* b, float* y, int n, int C, bool flip,
                hipStream_t s);
void dw_wgrad(const float* x, const float* gy, float* part, float* gw, float* gb, int n, int C,
              hipStream_t s);
// The same convolution with taps `dil` voxels apart (direct form, for small
// grids): forward / input gradient and the weight gradient through
// dwd_partials(n, C) floats of `part`.
size_t dwd_partials(int n, int C);
void dwd_forward(const float* x, const float* w, const float* b, float* y, int n, int C, int dil,
                 bool flip, hipStream_t s);
void dwd_wgrad(const float* x, const float* gy, float* part, float* gw, float* gb, int n, int C,
               int dil, hipStream_t s);
// Pointwise (1x1x1) convolution as FP32 matrix-core GEMMs on channels-last
// tensors: Y[M][N] = X[M][K] B + bias with B[k][n] = W[n][k] (W [N][K]) or,
// with transw, W[k][n] (W [K][N]); pw_wgrad writes pw_partials(M, K, N) floats
// of `part` and reduces them into gw [N][K] = G^T X and gb [N] = column sums
// of G (either may be null).  K and N multiples of 4.
size_t pw_partials(size_t M, int K, int N);
void pw_gemm(const float* X, const float* W, const float* bias, float* Y, size_t M, int K, int N,
             bool transw, hipStream_t s);
void pw_wgrad(const float* X, const float* G, float* part, float* gw, float* gb, size_t M, int K,
              int N, hipStream_t s);
// Squeeze-and-Excitation unit on channels-last [V][C] (C % 4 == 0, C <= 1024,
// H <= 256): w1 [H][C], b1 [H], w2 [C][H], b2 [C]; `ws` holds
// se_scratch(V, C, H) floats (256-byte aligned).  The backward recomputes the
// pooled state from x; any gradient output may be null.
size_t se_scratch(int V, int C, int H);
void se_forward(const float* x, const float* w1, const float* b1, const float* w2,
                const float* b2, float* y, int V, int C, int H, float* ws, hipStream_t s);
void se_backward(const float* x, const float* w1, const float* b1, const float* w2,
                 const float* b2, const float* gy, float* gx, float* gw1, float* gb1, float* gw2,
                 float* gb2, int V, int C, int H, float* ws, hipStream_t s);
// The launch shape the plan's heuristic picks for a forward / input-gradient
// pass with `cin` inputs and `cout` outputs (precision: PREC_*).
void default_conv_shape(int n, int cin, int cout, int taps, int prec, int* tile, int* bn, int* ck,
                        int* ksplit);

}  // namespace d2ip
