/*
 * d2ip.h - C-ABI of the MI355X (gfx950) library for the per-frame fitting
 * iteration of D2IP, "Deep Dynamic Image Prior for 3D Time-sequence
 * Pulmonary Impedance Imaging" (arXiv 2507.14046).
 *
 * The library fits the parameters theta of a 3D residual U-Net image prior
 * phi(theta | Z) to one frame of boundary-voltage differences:
 *
 *   image        d_sigma = mask * phi(theta | Z)                Eq. (3)
 *   prediction   p = J d_sigma                                  Eq. (1)
 *   data loss    L = (1/M) sum_m (p_m - dv_m)^2                 Eq. (4), l2 data term
 *   update       Adam on theta                                  Sec. III-A
 *
 * and carries theta from frame to frame (Temporal Parameter Propagation,
 * Eq. (9)): d2ip_set_frame replaces dv and leaves theta untouched.  The image
 * of a frame is read after its last update (Eq. (5)).
 *
 * Network (plain residual U-Net reading of Sec. III-D), with L levels and C
 * base channels, level l having C*2^l channels on an (n/2^l)^3 grid:
 *   stem conv3(1->C)+LN+ReLU; encoder ResBlocks at every level joined by 2x2x2
 *   average pooling; decoder ResBlocks(3c_l -> c_l) on [nearest-up x2, skip];
 *   tail conv1(C->1); ResBlock(a->b) = conv3, LN, ReLU, conv3, LN, + skip
 *   (1x1x1 conv if a != b), ReLU.  LN normalises each instance over all
 *   channels and voxels (eps 1e-5, biased variance) with a per-channel affine.
 *
 * Conventions for every entry point
 *  - Status: every function returns a d2ip_status; 0 is success.  On failure
 *    d2ip_last_error() describes the cause and the context keeps its previous
 *    valid state.  No C++ exception crosses the ABI.
 *  - Memory: the caller owns every buffer it passes.  `on_device` = 0 means a
 *    host pointer: the call copies and returns when the copy is complete.
 *    `on_device` = 1 means a device pointer in the same HIP device (e.g. a
 *    torch tensor's data_ptr()): the work is enqueued on the context stream and
 *    the caller keeps the buffer alive until that stream has passed the point.
 *  - Workspace: all device memory the library uses lives in one
 *    caller-allocated workspace (size from d2ip_workspace_bytes, 256-byte
 *    aligned) that the context borrows for its lifetime.  The library itself
 *    allocates no device memory.
 *  - Layouts: voxel index q = (z*n + y)*n + x (x fastest) for Z, mask and
 *    images; J is M x n^3 row-major FP32 with columns in that order.
 *    theta uses the flat order: stem, enc_0..enc_{L-1}, dec_{L-2}..dec_0,
 *    tail; inside a module conv W[Cout][Cin][kz][ky][kx] then b, norm gamma
 *    then beta, ResBlock order conv1, norm1, conv2, norm2, proj.
 *  - Threads: a context is not thread-safe; distinct contexts are independent.
 */
#ifndef D2IP_H
#define D2IP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct d2ip_ctx d2ip_ctx;

typedef enum {
  D2IP_OK = 0,
  D2IP_EINVAL = -1,     /* bad argument (NULL, shape, range)                 */
  D2IP_ENOMEM = -2,     /* workspace too small                               */
  D2IP_EHIP = -3,       /* a HIP runtime call failed                         */
  D2IP_ESTATE = -4,     /* call out of order (e.g. run before set_geometry)  */
  D2IP_ENONFINITE = -5  /* a non-finite loss was produced                    */
} d2ip_status;

/* Operand precision of the convolutions (forward, input gradient and weight
 * gradient); accumulation is always FP32, and the J products, LayerNorm, loss
 * and Adam are FP32 (the loss reduced in FP64).
 *   D2IP_PLAIN_FP32   FP32 operands (FP32 matrix-core instructions)
 *   D2IP_BF16_CONV    operands rounded to bfloat16 (one BF16 MFMA per product)
 *   D2IP_BF16X3_CONV  each FP32 operand split into bf16 hi + bf16 lo; products
 *                     hi*hi + hi*lo + lo*hi on three BF16 MFMAs (relative
 *                     product error near 2^-16) */
typedef enum { D2IP_PLAIN_FP32 = 0, D2IP_BF16_CONV = 1, D2IP_BF16X3_CONV = 2 } d2ip_precision;

/* d2ip_create flags */
#define D2IP_FLAG_GRAPH 1u /* capture one iteration in a hipGraph, replay it */

/* A measurement geometry: grid edge n (n^3 voxels) and M measurements. */
typedef struct {
  int n;
  int M;
} d2ip_geometry_desc;

/* One fitted instance (one sequence): its geometry index, levels L (2..5) and
 * base channels C (8, 16 or 32); n must be divisible by 2^(L-1) with
 * n / 2^(L-1) >= 2, and C * 2^(L-1) <= 256. */
typedef struct {
  int geometry;
  int levels;
  int base_ch;
} d2ip_instance_desc;

/* Adam hyper-parameters (defaults lr 1e-3, beta1 0.9, beta2 0.999, eps 1e-8). */
typedef struct {
  float lr, beta1, beta2, eps;
} d2ip_adam_cfg;

/* Text of the last error on this thread ("" if none); valid until the next call. */
const char* d2ip_last_error(void);

/* Number of parameters of a network with `levels` levels and `base_ch` base
 * channels.  Host only; needs no GPU. */
d2ip_status d2ip_param_count(int levels, int base_ch, size_t* out);

/* Kaiming initialisation of the network's parameters (Sec. III-B: the
 * network starts from Kaiming-initialised weights), host only: every conv
 * weight W[Cout][Cin][taps] ~ N(0, 2 / (Cin * taps)) (fan-in, ReLU gain),
 * biases 0, LayerNorm gamma 1 and beta 0, written to `theta` (n =
 * d2ip_param_count floats, flat order).  The normals come from a
 * counter-based generator (SplitMix64 outputs 2k, 2k + 1 of the seed's
 * sequence, Box-Muller) so value k depends only on `seed` and k.  A
 * convenience for callers without their own generator; parity inputs are
 * drawn by the caller and passed with d2ip_set_params. */
d2ip_status d2ip_init_params_host(int levels, int base_ch, uint64_t seed, float* theta, size_t n);

/* HIP_VERSION the library was compiled against, and the version of the HIP
 * runtime it is bound to in this process (hipRuntimeGetVersion).  A runtime
 * older than the compile-time headers is reported, not refused. */
d2ip_status d2ip_runtime_versions(int* compiled, int* loaded);

/* Workspace bytes needed by d2ip_create with the same arguments.  Host only. */
d2ip_status d2ip_workspace_bytes(const d2ip_geometry_desc* geos, int n_geo,
                                 const d2ip_instance_desc* insts, int n_inst, int precision,
                                 unsigned flags, size_t* out);

/* Host-only self check: plan the workspace for these arguments at a fake
 * address and walk one iteration's launch schedule without launching,
 * verifying that every kernel argument's extent lies inside one workspace
 * allocation for every instance.  D2IP_EINVAL with the violations in
 * d2ip_last_error() if not.  Needs no GPU. */
d2ip_status d2ip_check_launches(const d2ip_geometry_desc* geos, int n_geo,
                                const d2ip_instance_desc* insts, int n_inst, int precision,
                                unsigned flags);

/* Create a context over `workspace` (device memory, >= d2ip_workspace_bytes)
 * that enqueues on `hip_stream` (a hipStream_t; NULL = default stream).
 * All instances start with theta = 0, Adam state zero and no frame. */
d2ip_status d2ip_create(const d2ip_geometry_desc* geos, int n_geo, const d2ip_instance_desc* insts,
                        int n_inst, int precision, unsigned flags, void* workspace, size_t bytes,
                        void* hip_stream, d2ip_ctx** out);

/* Release host resources (waits for the stream).  The workspace is not freed. */
d2ip_status d2ip_destroy(d2ip_ctx* ctx);

/* Sensitivity matrix of geometry `geo` (Eq. (1)): J is M x n^3 FP32 row-major,
 * mask n^3 bytes (non-zero = voxel inside the imaging region).  J is
 * compacted to the mask's voxels on the device; masked columns of J are
 * ignored and masked image voxels are 0. */
d2ip_status d2ip_set_geometry(d2ip_ctx* ctx, int geo, const float* J, const uint8_t* mask,
                              int on_device);

/* theta of instance `inst` (n = d2ip_param_count floats, flat order). */
d2ip_status d2ip_set_params(d2ip_ctx* ctx, int inst, const float* theta, size_t n, int on_device);
d2ip_status d2ip_get_params(d2ip_ctx* ctx, int inst, float* theta, size_t n, int on_device);

/* theta of `inst` from d2ip_init_params_host(levels, base_ch, seed) (Kaiming,
 * Sec. III-B), uploaded as by d2ip_set_params. */
d2ip_status d2ip_init_params(d2ip_ctx* ctx, int inst, uint64_t seed);

/* Fixed noise input Z of instance `inst` (Eq. (3)): n^3 FP32. */
d2ip_status d2ip_set_noise_input(d2ip_ctx* ctx, int inst, const float* z, int on_device);

/* Voltage differences dv of the current frame of `inst` (M FP32).  theta is
 * not touched (Temporal Parameter Propagation, Eq. (9)). */
d2ip_status d2ip_set_frame(d2ip_ctx* ctx, int inst, const float* dv, int on_device);

/* Adam hyper-parameters for all instances. */
d2ip_status d2ip_set_adam(d2ip_ctx* ctx, const d2ip_adam_cfg* cfg);

/* Zero the Adam moments and step counter of `inst` (call between frames to
 * restart the optimiser while theta carries over). */
d2ip_status d2ip_reset_optimizer(d2ip_ctx* ctx, int inst);

/* Full optimiser state of `inst`: theta_m_v = [theta | m | v] (3 * P FP32),
 * t = Adam step count.  Restoring a saved state resumes bit-exactly. */
d2ip_status d2ip_get_state(d2ip_ctx* ctx, int inst, float* theta_m_v, int64_t* t, int on_device);
d2ip_status d2ip_set_state(d2ip_ctx* ctx, int inst, const float* theta_m_v, int64_t t,
                           int on_device);

/* Run k iterations of every instance (forward, J d_sigma, loss, J^T, backward,
 * Adam).  Asynchronous unless `last_loss` (n_inst doubles, may be NULL) is
 * given: then it synchronises and stores, per instance, the data loss of the
 * last iteration (evaluated before its update), and returns D2IP_ENONFINITE
 * if a loss or an updated parameter was not finite in any iteration since the
 * parameters were last set (the flag is raised on the device by the loss
 * reduction and by the Adam kernel, and cleared by d2ip_set_params,
 * d2ip_set_state and d2ip_init_params). */
d2ip_status d2ip_run(d2ip_ctx* ctx, int k, double* last_loss);

/* Gradient dL/dtheta of the data loss computed by the last iteration of
 * `inst` (before that iteration's Adam update), flat order, n = P floats. */
d2ip_status d2ip_get_grad(d2ip_ctx* ctx, int inst, float* grad, size_t n, int on_device);

/* Kernels d2ip_time_kernel can time in isolation. */
typedef enum {
  D2IP_KERNEL_JVEC = 0,        /* p = J d_sigma (streams J once)                  */
  D2IP_KERNEL_JTVEC = 1,       /* J^T g (streams J once)                          */
  D2IP_KERNEL_ADAM = 2,        /* fused Adam over all parameters (updates state!) */
  D2IP_KERNEL_CONV_FWD = 3,    /* forward of conv1 of block `block`               */
  D2IP_KERNEL_CONV_DGRAD = 4,  /* input gradient of that conv                     */
  D2IP_KERNEL_CONV_WGRAD = 5   /* weight gradient of that conv (+ its reduction)  */
} d2ip_kernel;

/* Benchmark helper: launch kernel `which` of instance `inst` `reps` times on
 * the context stream (after one untimed launch) and store the mean duration
 * per launch in ms, measured with HIP events.  `block` indexes the ResBlocks
 * in flat order (enc_0.., dec_{L-2}..dec_0) for the conv kernels.  Must
 * follow at least one d2ip_run (buffers hold that iteration's data).  The
 * Adam variant advances theta and the moments. */
d2ip_status d2ip_time_kernel(d2ip_ctx* ctx, int inst, int which, int block, int reps,
                             double* avg_ms);

/* Image of `inst` at its current theta: mask * phi(theta | Z), n^3 FP32 (Eq. (5)). */
d2ip_status d2ip_read_image(d2ip_ctx* ctx, int inst, float* sigma, int on_device);

/* ---- 4D total variation (Sec. III-E) ------------------------------------
 * With lambda_tv > 0 every iteration's loss is the data term plus
 *   lambda_tv * (lambda_s * R_spatial(s) + lambda_t * R_temporal(history, s))
 * (Eqs. (11)-(14)) for the current image s = mask * phi(theta | Z):
 *   R_spatial  = (1/V) sum_v sqrt(dz^2 + dy^2 + dx^2 + eps), forward
 *                differences, 0 where the neighbour is outside the grid;
 *   R_temporal = sum_k w_k sum_v sqrt((s - h_k)^2 + eps) over the images h_k
 *                of the k-th previous frame (k = 1 the newest), w_k =
 *                exp(-k) / sum_k exp(-k); 0 with no history.
 * The history holds at most 32 frames (an older frame's weight is below
 * exp(-32) of the newest's, under FP32 resolution).  The paper's values are
 * lambda_tv 0.002, lambda_s 1, lambda_t 0.1; eps (unstated) 1e-8. */
typedef struct {
  float lambda_tv, lambda_s, lambda_t, eps;
} d2ip_tv_cfg;

/* Set the 4D-TV coefficients of every instance (lambda_tv 0 switches the term
 * off, the default).  Drops a captured graph. */
d2ip_status d2ip_set_tv(d2ip_ctx* ctx, const d2ip_tv_cfg* cfg);

/* End the current frame of `inst`: its image at the current theta becomes
 * the newest entry of the temporal history.  Call before d2ip_set_frame of
 * the next frame. */
d2ip_status d2ip_commit_frame(d2ip_ctx* ctx, int inst);

/* Empty the temporal history of `inst` (a new sequence). */
d2ip_status d2ip_clear_history(d2ip_ctx* ctx, int inst);

/* ---- the 3D-FastResUNet fitting iteration (Sec. III-D) -------------------
 * One instance of the fitting iteration with the paper's lightweight
 * modules switched on individually: depthwise-separable ResBlock convs
 * (sep), an SE unit after every encoder ResBlock (se_ratio r > 0: hidden
 * width max(1, c / r)), an ASPP module at the bottleneck (aspp: a 1x1x1
 * branch and depthwise-separable atrous branches at dilations 1, 2, 3,
 * concatenated, projected, ReLU), attention units on the decoder skips
 * (att: the gate formed on the coarser decoder output's grid, then
 * interpolated) and the output head 2 sigmoid(t) - 1 (sigmoid_tail).  One
 * iteration: the forward from the fixed noise input, p = J sigma (Eq. (2)),
 * the data term (1/M) sum (p - dv)^2 reduced in FP64 and its gradient
 * (Eq. (4)), J^T, the backward of every module and an Adam step (Eq. (5)).
 * Every step runs the kernels of the standalone operators below; the
 * iteration is FP32 throughout (FP64 in the loss reduction), eager launches
 * on the caller's stream.
 *
 * theta's flat order: stem (W [C][1][3][3][3], b, gamma, beta); encoder
 * modules 0 .. L-1 (conv1, norm1, conv2, norm2, projection when the
 * channels change, then the SE unit's w1 [H][c], b1, w2 [c][H], b2); the
 * ASPP module (w0 [c][c], b0, then per dilation dw [c][27], dwb, pw [c][c],
 * pwb, then wp [c][4c], bp); decoder modules L-2 .. 0 (the ResBlock, then
 * the attention unit's wx [c][c], wg [c][c_up], b [c], psi [c], bpsi [1]);
 * head w [C], b.  A separable conv is dw [Cin][27], dwb, pw [Cout][Cin],
 * pwb in place of W, b.  J is M x n^3 row-major FP32 (the full grid),
 * mask n^3 bytes (0 outside), z the n^3 noise input.
 *
 * Limits: levels 2..5, base_ch 8, 16 or 32, base_ch 2^(levels-1) <= 256, n a
 * multiple of 2^(levels-1) with n / 2^(levels-1) >= 2 and n <= 128.
 * The workspace (256-byte aligned, d2ip_mnet_workspace_bytes) holds J,
 * every activation, gradients, Adam moments and the operators' scratch; the
 * context keeps pointers into it until d2ip_mnet_destroy, which waits for
 * the stream.  Host inputs are copied before the call returns. */
typedef struct d2ip_mnet d2ip_mnet;

/* graph != 0: the first d2ip_mnet_run captures one iteration in a hipGraph
 * (on a stream of the context's own) and every iteration replays it on the
 * caller's stream; d2ip_mnet_set_adam discards the graph (its Adam step holds
 * the hyper-parameters), the next run captures again. */
typedef struct {
  int n, M, levels, base_ch;
  int sep, se_ratio, att, sigmoid_tail, aspp;
  int graph;
} d2ip_mnet_desc;

d2ip_status d2ip_mnet_param_count(const d2ip_mnet_desc* desc, size_t* out);
d2ip_status d2ip_mnet_workspace_bytes(const d2ip_mnet_desc* desc, size_t* out);
d2ip_status d2ip_mnet_create(const d2ip_mnet_desc* desc, void* workspace, size_t bytes,
                             void* hip_stream, d2ip_mnet** out);
d2ip_status d2ip_mnet_destroy(d2ip_mnet* net);
/* J [M][n^3] FP32, mask [n^3] bytes, z [n^3] FP32: host or device memory. */
d2ip_status d2ip_mnet_set_problem(d2ip_mnet* net, const float* J, const uint8_t* mask,
                                  const float* z, int on_device);
/* theta in the flat order above (n must equal d2ip_mnet_param_count); also
 * restarts Adam (moments and step count). */
d2ip_status d2ip_mnet_set_params(d2ip_mnet* net, const float* theta, size_t n, int on_device);
d2ip_status d2ip_mnet_get_params(d2ip_mnet* net, float* theta, size_t n, int on_device);
/* dL/dtheta of the last iteration, at the parameters it started from. */
d2ip_status d2ip_mnet_get_grad(d2ip_mnet* net, float* grad, size_t n, int on_device);
/* The frame's measured voltage differences dv [M]; theta is kept (Eq. (9)). */
d2ip_status d2ip_mnet_set_frame(d2ip_mnet* net, const float* dv, int on_device);
d2ip_status d2ip_mnet_set_adam(d2ip_mnet* net, const d2ip_adam_cfg* cfg);
d2ip_status d2ip_mnet_reset_optimizer(d2ip_mnet* net);
/* k iterations; with last_loss the call waits and returns the last
 * iteration's loss (at the parameters before its update), and reports
 * D2IP_ENONFINITE if a loss or parameter was not finite. */
d2ip_status d2ip_mnet_run(d2ip_mnet* net, int k, double* last_loss);
/* sigma = mask * phi(theta | z) at the current theta (n^3 values). */
d2ip_status d2ip_mnet_read_image(d2ip_mnet* net, float* sigma, int on_device);

/* ---- launch shapes of the convolutions (for autotuning) ----------------
 * Every 3x3x3 / 1x1x1 convolution of the network (Eq. (3): the prior phi is
 * built from them) runs three passes: 0 forward, 1 input gradient, 2 weight
 * gradient.  A pass's launch shape trades parallelism against per-block
 * work; the plan picks one by a heuristic unless the tuning table holds an
 * entry for that pass. */
typedef struct {
  int tile;  /* voxel tile per block: 0 = 2x4x16, 1 = 1x4x16, 2 = 1x8x8 (z x y x x) */
  int bn;    /* passes 0/1: output channels per block, 16, 32 or 64 (not 64 with tile 0) */
  int ck;    /* input channels staged per step: 8, 16 or 32, dividing the pass's input */
  int split; /* passes 0/1: blocks sharing the channel chunks (split-K; divides
                the chunk count; 1 for forward 1x1 convs); pass 2: voxel
                splits, 1..min(256, voxel tiles) */
} d2ip_conv_shape;

/* One pass of one convolution and its shape.  The convolution is named by
 * its forward channels: grid n^3, cin inputs (8 for the padded 1-channel
 * stem), cout outputs, taps 27 or 1.  `prologue` is the operand transform the
 * pass fuses into its staging: passes 0/1: 0 none, 1 LayerNorm + ReLU of the
 * input (pass 0), 2 LayerNorm backward of the incoming gradient (pass 1);
 * pass 2: 3 * (input transform: 0 or 1) + (gradient transform: 0 or 2).
 * `precision` is a d2ip_precision. */
typedef struct {
  int n, cin, cout, taps;
  int pass;
  int prologue;
  int precision;
  d2ip_conv_shape shape;
} d2ip_tuning_entry;

/* Replace the process-wide tuning table with `count` entries (0 clears it).
 * Plans made afterwards (d2ip_workspace_bytes, d2ip_create,
 * d2ip_check_launches, d2ip_plan_convs) use an entry's shape for every pass
 * that matches all its key fields.  Every entry is validated first; on
 * D2IP_EINVAL (the reason in d2ip_last_error) the table is unchanged.  Not
 * thread-safe with concurrent planning.  Host only. */
d2ip_status d2ip_set_tuning(const d2ip_tuning_entry* table, int count);

/* The passes of every convolution of instance `inst` of the plan for these
 * arguments, in schedule order, with the shapes the plan chose.  Writes at
 * most `cap` entries to `out` (may be NULL with cap 0) and the total to
 * *count.  Host only. */
d2ip_status d2ip_plan_convs(const d2ip_geometry_desc* geos, int n_geo,
                            const d2ip_instance_desc* insts, int n_inst, int precision,
                            unsigned flags, int inst, d2ip_tuning_entry* out, int cap,
                            int* count);

/* Device workspace bytes d2ip_time_conv needs for entry `e`.  Host only. */
d2ip_status d2ip_time_conv_bytes(const d2ip_tuning_entry* e, size_t* out);

/* Time one pass of one convolution with the shape in `e`, in isolation, on
 * zero-filled operands carved from the caller's device `workspace` (256-byte
 * aligned, at least d2ip_time_conv_bytes): one untimed launch, then `reps`
 * launches on `hip_stream` between HIP events; the mean ms per launch goes to
 * *avg_ms.  The weight-gradient pass times its partial-sum kernel only. */
d2ip_status d2ip_time_conv(const d2ip_tuning_entry* e, void* workspace, size_t bytes,
                           void* hip_stream, int reps, double* avg_ms);

/* ---- standalone operators --------------------------------------------
 * The building blocks of the prior (Sec. III-D, Eq. (3)) and of the data term
 * (Eqs. (1), (4)) on caller buffers, for composing the network in a framework
 * with its own autograd.  They run the fitting iteration's kernels.  All
 * tensors are device pointers to FP32 (BF16 forms round the conv operands
 * internally); activations are channels-last: x[v][c] with v = (z*n + y)*n + x
 * over an n^3 grid.  Each call enqueues on `hip_stream` and returns; buffers
 * must stay alive until the stream passes that point.  `workspace` (device,
 * 256-byte aligned, at least the matching *_bytes) is scratch owned by the
 * caller; one workspace must not be used by two calls in flight at once.
 * These calls read no host memory after they return: their small tables are
 * written by kernels from kernel arguments. */

/* Workspace bytes of d2ip_op_conv3d_forward / _backward.  cin and cout
 * multiples of 8 in [8, 1024], taps 27 (3x3x3, zero padding) or 1. */
d2ip_status d2ip_op_conv3d_bytes(int n, int cin, int cout, int taps, int precision, size_t* out);

/* y[v][co] = b[co] + sum_{tap, ci} w[co][ci][tap] x[v + offset(tap)][ci]
 * (cross-correlation, zero padding; w in the canonical [cout][cin][kz][ky][kx]
 * order, b may be NULL). */
d2ip_status d2ip_op_conv3d_forward(const float* x, const float* w, const float* b, float* y, int n,
                                   int cin, int cout, int taps, int precision, void* workspace,
                                   size_t bytes, void* hip_stream);

/* Gradients of that convolution given gy = dL/dy: gx = dL/dx (input
 * gradient: the flipped, transposed convolution), gw = dL/dw (canonical
 * order) and gb = dL/db; any of the three outputs may be NULL.  Sums over
 * voxels are reduced in a fixed order (deterministic). */
d2ip_status d2ip_op_conv3d_backward(const float* x, const float* w, const float* gy, float* gx,
                                    float* gw, float* gb, int n, int cin, int cout, int taps,
                                    int precision, void* workspace, size_t bytes,
                                    void* hip_stream);

/* Workspace bytes of the LayerNorm + ReLU operators (C a power of two in
 * [4, 256]). */
d2ip_status d2ip_op_ln_relu_bytes(int n, int C, size_t* out);

/* y = relu(gamma_c * (x - mean) / sqrt(var + 1e-5) + beta_c + skip), with
 * mean and (biased) variance over all n^3 x C values of x; skip may be NULL.
 * x, y and skip 16-byte aligned (D2IP_EINVAL otherwise). */
d2ip_status d2ip_op_ln_relu_forward(const float* x, const float* gamma, const float* beta,
                                    const float* skip, float* y, int n, int C, void* workspace,
                                    size_t bytes, void* hip_stream);

/* Backward of d2ip_op_ln_relu_forward given its input x, output y and
 * gy = dL/dy: gx = dL/dx, gskip = dL/dskip (the ReLU-masked gy) and
 * dgamma_dbeta = [dL/dgamma (C), dL/dbeta (C)]; outputs may be NULL.
 * x, y, gy, gx and gskip 16-byte aligned (D2IP_EINVAL otherwise). */
d2ip_status d2ip_op_ln_relu_backward(const float* x, const float* y, const float* gamma,
                                     const float* gy, float* gx, float* gskip,
                                     float* dgamma_dbeta, int n, int C, void* workspace,
                                     size_t bytes, void* hip_stream);

/* Workspace bytes of d2ip_op_dwconv3d_backward's weight gradient (C a
 * multiple of 4 in [4, 1024]). */
d2ip_status d2ip_op_dwconv3d_bytes(int n, int C, size_t* out);

/* Depthwise 3x3x3 convolution, the first half of a depthwise-separable
 * convolution of the lightweight backbone (Sec. III-D):
 * y[v][c] = b[c] + sum_tap w[c][tap] x[v + offset(tap)][c] (cross-correlation,
 * zero padding; w [C][kz][ky][kx], i.e. the canonical [C][1][3][3][3]; b may be
 * NULL).  x, y (and b) 16-byte aligned.  The second half is the pointwise
 * convolution d2ip_op_pwconv3d_forward.  Needs no workspace and uploads
 * nothing. */
d2ip_status d2ip_op_dwconv3d_forward(const float* x, const float* w, const float* b, float* y,
                                     int n, int C, void* hip_stream);

/* Gradients of d2ip_op_dwconv3d_forward given gy = dL/dy: gx = dL/dx (the
 * same convolution with the taps reversed), gw = dL/dw [C][27] and
 * gb = dL/db [C]; any output may be NULL; x is needed only for gw / gb, w only
 * for gx, and the workspace only for gw / gb.  Sums over voxels are reduced
 * in a fixed order (deterministic). */
d2ip_status d2ip_op_dwconv3d_backward(const float* x, const float* w, const float* gy, float* gx,
                                      float* gw, float* gb, int n, int C, void* workspace,
                                      size_t bytes, void* hip_stream);

/* Workspace bytes of d2ip_op_dwconv3d_dilated_backward's weight gradient. */
d2ip_status d2ip_op_dwconv3d_dilated_bytes(int n, int C, int dilation, size_t* out);

/* The depthwise 3x3x3 convolution with its taps `dilation` voxels apart
 * (dilation in [1, 256]; the atrous branches of the ASPP module at the
 * bottleneck, Sec. III-D): y[v][c] = b[c] + sum_tap w[c][tap]
 * x[v + dilation (tap - 1)][c], zero outside the grid.  A direct kernel for
 * the small grids it runs on; otherwise as d2ip_op_dwconv3d_forward. */
d2ip_status d2ip_op_dwconv3d_dilated_forward(const float* x, const float* w, const float* b,
                                             float* y, int n, int C, int dilation,
                                             void* hip_stream);

/* Gradients of d2ip_op_dwconv3d_dilated_forward, as d2ip_op_dwconv3d_backward. */
d2ip_status d2ip_op_dwconv3d_dilated_backward(const float* x, const float* w, const float* gy,
                                              float* gx, float* gw, float* gb, int n, int C,
                                              int dilation, void* workspace, size_t bytes,
                                              void* hip_stream);

/* Workspace bytes of d2ip_op_pwconv3d_backward's weight gradient (cin and
 * cout multiples of 4 in [4, 1024]). */
d2ip_status d2ip_op_pwconv3d_bytes(int n, int cin, int cout, size_t* out);

/* Pointwise 1x1x1 convolution, the second half of a depthwise-separable
 * convolution (Sec. III-D), as an FP32 matrix-core GEMM:
 * y[v][co] = b[co] + sum_ci w[co][ci] x[v][ci] (w [cout][cin], the canonical
 * [cout][cin][1][1][1]; b may be NULL).  x, w and y 16-byte aligned.  Needs no
 * workspace and uploads nothing. */
d2ip_status d2ip_op_pwconv3d_forward(const float* x, const float* w, const float* b, float* y,
                                     int n, int cin, int cout, void* hip_stream);

/* Gradients of d2ip_op_pwconv3d_forward given gy: gx = gy w, gw = gy^T x
 * ([cout][cin]) and gb = column sums of gy; any output may be NULL; x is
 * needed only for gw / gb, w only for gx, the workspace only for gw / gb.
 * Voxel sums are reduced in a fixed order (deterministic). */
d2ip_status d2ip_op_pwconv3d_backward(const float* x, const float* w, const float* gy, float* gx,
                                      float* gw, float* gb, int n, int cin, int cout,
                                      void* workspace, size_t bytes, void* hip_stream);

/* Workspace bytes of the Squeeze-and-Excitation operators (C a multiple of
 * 4 in [4, 1024], hidden width H in [1, 256]). */
d2ip_status d2ip_op_se_bytes(int n, int C, int H, size_t* out);

/* Squeeze-and-Excitation unit of the 3D-FastResUNet (Sec. III-D): the channel
 * means s[c] = (1/n^3) sum_v x[v][c], the gate
 * e = sigmoid(w2 relu(w1 s + b1) + b2) (w1 [H][C], b1 [H], w2 [C][H], b2 [C])
 * and y[v][c] = e[c] x[v][c].  x and y 16-byte aligned. */
d2ip_status d2ip_op_se_forward(const float* x, const float* w1, const float* b1, const float* w2,
                               const float* b2, float* y, int n, int C, int H, void* workspace,
                               size_t bytes, void* hip_stream);

/* Gradients of d2ip_op_se_forward given its input x and gy = dL/dy: gx and the
 * weight and bias gradients (any output may be NULL).  The pooled state is
 * recomputed from x; voxel sums are reduced in a fixed order. */
d2ip_status d2ip_op_se_backward(const float* x, const float* w1, const float* b1, const float* w2,
                                const float* b2, const float* gy, float* gx, float* gw1,
                                float* gb1, float* gw2, float* gb2, int n, int C, int H,
                                void* workspace, size_t bytes, void* hip_stream);

/* ---- routing and module operators of the network (Sec. III-D) -----------
 * Channels-last FP32 tensors, channel counts multiples of 4, 16-byte aligned;
 * n is the finer grid of the pair (even). */

/* y [(n/2)^3][C] = the 2x2x2 average of x [n^3][C] (the encoder's down-sampling). */
d2ip_status d2ip_op_pool2_forward(const float* x, float* y, int n, int C, void* hip_stream);
/* gx [n^3][C] = gy[parent(v)] / 8, the adjoint of d2ip_op_pool2_forward. */
d2ip_status d2ip_op_pool2_backward(const float* gy, float* gx, int n, int C, void* hip_stream);

/* cat [n^3][Cu + Cs] = [up2(d), e]: the coarser decoder output d [(n/2)^3][Cu]
 * interpolated to the finer grid (nearest neighbour, x2) and the encoder skip
 * e [n^3][Cs], concatenated in that order (the decoder's fusion). */
d2ip_status d2ip_op_up2_concat_forward(const float* d, int Cu, const float* e, int Cs, int n,
                                       float* cat, void* hip_stream);
/* gd [(n/2)^3][Cu] = sum over each coarse voxel's 8 children of gcat[v][0..Cu),
 * ge [n^3][Cs] = gcat[v][Cu..Cu+Cs). */
d2ip_status d2ip_op_up2_concat_backward(const float* gcat, int Cu, int Cs, int n, float* gd,
                                        float* ge, void* hip_stream);

/* Channel range copy between channels-last tensors of `voxels` rows:
 * dst[v][dst_off + j] = src[v][src_off + j] for j < ch; src has src_ch
 * channels per voxel, dst dst_ch.  All counts and offsets multiples of 4,
 * both tensors 16-byte aligned and not overlapping (D2IP_EINVAL otherwise).
 * The ASPP module (Sec. III-D: parallel atrous branches fused into one
 * tensor) concatenates its branches with one call per branch and splits the
 * gradient back out the same way. */
d2ip_status d2ip_op_channel_copy(const float* src, int src_ch, int src_off, float* dst, int dst_ch,
                                 int dst_off, int ch, size_t voxels, void* hip_stream);

/* y = max(x, 0) over count values (count % 4 == 0; y may equal x), and its
 * gradient gx = gy where y > 0, else 0 (gx may equal gy). */
d2ip_status d2ip_op_relu_forward(const float* x, float* y, size_t count, void* hip_stream);
d2ip_status d2ip_op_relu_backward(const float* y, const float* gy, float* gx, size_t count,
                                  void* hip_stream);

/* Output head (Sec. III-D: a Conv3D layer and, for the sigmoid tail, a
 * sigmoid): t[v] = b[0] + sum_c w[c] x[v][c] over x [n^3][C] (C a power of
 * two in [4, 256]); out[v] = mask[v] * t[v], or with sigmoid_tail != 0
 * mask[v] * (2 sigmoid(t[v]) - 1) (range (-1, 1)); mask may be NULL (all 1). */
d2ip_status d2ip_op_head_bytes(int n, int C, size_t* out);
d2ip_status d2ip_op_head_forward(const float* x, const float* w, const float* b,
                                 const float* mask, float* out, int n, int C, int sigmoid_tail,
                                 void* hip_stream);
/* Gradients of the head given gout = dL/dout: gx [n^3][C], gw [C], gb [1]
 * (each may be NULL); the voxel sums are reduced in FP64 in a fixed order. */
d2ip_status d2ip_op_head_backward(const float* x, const float* w, const float* b,
                                  const float* mask, const float* gout, float* gx, float* gw,
                                  float* gb, int n, int C, int sigmoid_tail, void* workspace,
                                  size_t bytes, void* hip_stream);

/* Attention unit of a decoder stage (Sec. III-D: each up-sampling stage is
 * an attention mechanism followed by interpolation and a ResConv3D block):
 * x [n^3][c] is the encoder skip, g [(n/2)^3][cu] the coarser decoder output.
 * On g's grid: xs = 2x2x2 average of x, a = wx xs + wg g + b (wx [c][c],
 * wg [c][cu], b [c]), alpha = sigmoid(bpsi + psi . relu(a)) (psi [c],
 * bpsi [1]); then y [n^3][c] = alpha[parent(v)] x[v] (the coefficients
 * interpolated, nearest neighbour).  alpha [(n/2)^3] may be NULL.  c and cu
 * multiples of 4, c <= 256, cu <= 512 (up to 64 / 128 one fused pass; wider
 * through pointwise matrix-core GEMMs); x, g, y (gy, gx), wx and wg 16-byte
 * aligned.  The workspace (256-byte aligned, d2ip_op_attention_bytes, the
 * same for forward and backward) holds the wide form's intermediates and the
 * backward's partial sums. */
d2ip_status d2ip_op_attention_bytes(int n, int c, int cu, size_t* out);
d2ip_status d2ip_op_attention_forward(const float* x, const float* g, const float* wx,
                                      const float* wg, const float* b, const float* psi,
                                      const float* bpsi, float* y, float* alpha, int n, int c,
                                      int cu, void* workspace, size_t bytes, void* hip_stream);
/* Gradients of the attention unit given gy = dL/dy: gx, gg (on g's grid) and
 * the parameter gradients (any output may be NULL except that the parameter
 * gradients are written together); the ReLU derivative is 0 at 0.  Sums over
 * coarse voxels are per-block partials reduced in FP64 in block order. */
d2ip_status d2ip_op_attention_backward(const float* x, const float* g, const float* wx,
                                       const float* wg, const float* b, const float* psi,
                                       const float* bpsi, const float* gy, float* gx, float* gg,
                                       float* gwx, float* gwg, float* gb, float* gpsi,
                                       float* gbpsi, int n, int c, int cu, void* workspace,
                                       size_t bytes, void* hip_stream);

/* p = J sigma for a dense row-major M x Q J (Eq. (1)); Q a multiple of 4. */
d2ip_status d2ip_op_j_forward(const float* J, const float* sigma, float* p, int M, int Q,
                              void* hip_stream);

/* Data term of Eq. (4) in its mean-squared form (Sec. V-A calls it the MSE
 * loss) for M predicted voltages p against the measured dv: r = p - dv,
 * *loss = (1/M) sum r^2 (one double in device memory), accumulated in FP64 in
 * a fixed order, and gp = (2/M) r (M floats; may be NULL). */
d2ip_status d2ip_op_mse_loss(const float* p, const float* dv, float* gp, double* loss, int M,
                             void* hip_stream);

/* Workspace bytes of d2ip_op_jt. */
d2ip_status d2ip_op_jt_bytes(int M, int Q, size_t* out);

/* out = J^T g (Q values), the adjoint of d2ip_op_j_forward, summed over rows
 * in a fixed order. */
d2ip_status d2ip_op_jt(const float* J, const float* g, float* out, int M, int Q, void* workspace,
                       size_t bytes, void* hip_stream);

/* d2ip_op_jt without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments minus the workspace, same kernels and
 * summation order, so the result equals d2ip_op_jt's bit for bit.  The row
 * partial sums live in a static 8 MiB device array inside the library (one
 * per GPU, held until the process ends; its address is looked up on the first
 * call on each device), which limits Q to 262144 (64^3) columns: larger Q is
 * rejected with D2IP_EINVAL before anything is enqueued.  J and out must be
 * 16-byte aligned.  Allocates nothing.  Every call on one GPU shares that
 * array: calls that overlap on one GPU (two streams, or two threads) race and
 * must be serialised by the caller. */
d2ip_status d2ip_op_jt_noalloc(const float* J, const float* g, float* out, int M, int Q,
                               void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* D2IP_H */
