// Standalone operators of the C-ABI: one convolution (forward, input and
// weight gradients), LayerNorm + ReLU (forward and backward) and the dense J
// products, on caller buffers and the caller's stream.  They run the same
// kernels as the fitting iteration and let a framework compose the network
// with its own autograd.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "d2ip.h"
#include "kernels.h"

namespace d2ip {
d2ip_status api_fail(d2ip_status s, const std::string& m);
int default_wgrad_splits(int n, int cin, int cout, int taps, int tile, int ck);
int default_tile(int n);
int default_ck(int cin);
}  // namespace d2ip

using namespace d2ip;

namespace {

// One small descriptor written to device memory from a kernel argument: the
// host value it comes from may end with the calling frame, and the write is
// an ordinary kernel node when a caller captures the operator in a graph.
template <class T>
__global__ void k_put(T* dst, T v) {
  if (threadIdx.x == 0) *dst = v;
}

#define OPCHK(expr)                                                                      \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return api_fail(D2IP_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

// Carves 256-byte aligned pieces off a workspace (sizes only when base is null).
struct Piece {
  char* base = nullptr;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

int prec_of(int precision) {
  return precision == D2IP_BF16_CONV ? PREC_BF16 : precision == D2IP_BF16X3_CONV ? PREC_BF16X3
                                                                                 : PREC_F32;
}

// Launch shapes and scratch of one convolution.
struct ConvOp {
  int n = 0, cin = 0, cout = 0, taps = 0, prec = PREC_F32;
  size_t V = 0;
  int f_tile, f_bn, f_ck, f_split;  // forward
  int d_tile, d_bn, d_ck, d_split;  // input gradient
  int w_tile, w_ck, w_split;        // weight gradient
  ConvPack* pack = nullptr;
  GradSeg* seg = nullptr;
  float* wf32 = nullptr;
  uint16_t* wbf16 = nullptr;
  long long wtotal = 0;
  float *kpart = nullptr, *part = nullptr, *partb = nullptr, *grad = nullptr;
};

d2ip_status conv_check(int n, int cin, int cout, int taps, int precision) {
  if (n < 1 || n > 256) return api_fail(D2IP_EINVAL, "n must be in [1, 256]");
  if (taps != 27 && taps != 1) return api_fail(D2IP_EINVAL, "taps must be 27 or 1");
  if (cin < 8 || cout < 8 || cin % 8 || cout % 8 || cin > 1024 || cout > 1024)
    return api_fail(D2IP_EINVAL, "cin and cout must be multiples of 8 in [8, 1024]");
  if (precision < D2IP_PLAIN_FP32 || precision > D2IP_BF16X3_CONV)
    return api_fail(D2IP_EINVAL, "unknown precision");
  return D2IP_OK;
}

void conv_plan(ConvOp& c, int n, int cin, int cout, int taps, int precision, Piece& w) {
  c.n = n;
  c.cin = cin;
  c.cout = cout;
  c.taps = taps;
  c.prec = prec_of(precision);
  c.V = (size_t)n * n * n;
  default_conv_shape(n, cin, cout, taps, c.prec, &c.f_tile, &c.f_bn, &c.f_ck, &c.f_split);
  default_conv_shape(n, cout, cin, taps, c.prec, &c.d_tile, &c.d_bn, &c.d_ck, &c.d_split);
  c.w_tile = default_tile(n);
  c.w_ck = default_ck(cin);
  while (c.w_ck > 8 && conv_wgrad_lds_bytes(c.w_tile, taps, c.w_ck, c.prec) > 60 * 1024)
    c.w_ck >>= 1;
  c.w_split = default_wgrad_splits(n, cin, cout, taps, c.w_tile, c.w_ck);
  const size_t wel = (size_t)cout * taps * cin;
  c.wtotal = (long long)(2 * wel);  // forward packing, then input-gradient packing
  c.pack = w.take<ConvPack>(1);
  c.seg = w.take<GradSeg>(1);
  if (c.prec == PREC_F32)
    c.wf32 = w.take<float>(c.wtotal);
  else
    c.wbf16 = w.take<uint16_t>((c.prec == PREC_BF16X3 ? 2 : 1) * c.wtotal);
  const size_t kp = std::max((size_t)c.f_split * c.V * cout, (size_t)c.d_split * c.V * cin);
  c.kpart = w.take<float>(std::max<size_t>(1, kp));
  const size_t cout16 = (cout + 15) / 16 * 16;
  c.part = w.take<float>((size_t)c.w_split * cout16 * taps * cin);
  c.partb = w.take<float>((size_t)c.w_split * cout16);
  c.grad = w.take<float>(wel + cout);
}

ConvPack make_pack(const ConvOp& c) {
  ConvPack p;
  std::memset(&p, 0, sizeof(p));
  p.th_off = 0;
  p.cout = c.cout;
  p.cin_real = c.cin;
  p.cin = c.cin;
  p.taps = c.taps;
  p.need_dgrad = 1;
  p.wf_off = 0;
  p.wd_off = (long long)c.cout * c.taps * c.cin;
  return p;
}

// Upload the packing table once per call and pack w into the forward and
// input-gradient layouts.
d2ip_status conv_prepare(ConvOp& c, const float* w, hipStream_t s) {
  hipLaunchKernelGGL(k_put<ConvPack>, dim3(1), dim3(64), 0, s, c.pack, make_pack(c));
  pack_weights(c.pack, 1, c.cout * c.cin * c.taps, w, c.wf32, c.wbf16,
               c.prec == PREC_BF16X3 ? c.wtotal : 0, nullptr, nullptr, 0, 1, nullptr, 0, 1, 0, s);
  return D2IP_OK;
}

ConvSrc plain(const float* x, int stride) {
  ConvSrc s;
  std::memset(&s, 0, sizeof(s));
  s.x = x;
  s.stride = stride;
  s.prologue = PRO_NONE;
  return s;
}

ConvFwd fwd_of(const ConvOp& c, bool dgrad, const float* src, const float* bias, float* y) {
  ConvFwd a;
  std::memset(&a, 0, sizeof(a));
  const int kin = dgrad ? c.cout : c.cin, kout = dgrad ? c.cin : c.cout;
  const long long off = dgrad ? (long long)c.cout * c.taps * c.cin : 0;
  a.src = plain(src, kin);
  a.n = c.n;
  a.cin = kin;
  a.w = c.prec == PREC_F32 ? (const void*)(c.wf32 + off) : (const void*)(c.wbf16 + off);
  a.w_lo_off = c.prec == PREC_BF16X3 ? c.wtotal : 0;
  a.w_rows = kout;
  a.bias = bias;
  a.cout = kout;
  a.y = y;
  a.taps = c.taps;
  a.prec = c.prec;
  a.tile = dgrad ? c.d_tile : c.f_tile;
  a.bn = dgrad ? c.d_bn : c.f_bn;
  a.ck = dgrad ? c.d_ck : c.f_ck;
  a.ksplit = dgrad ? c.d_split : c.f_split;
  a.kpart = c.kpart;
  a.batch = 1;
  return a;
}

d2ip_status ws_check(void* ws, size_t bytes, size_t need) {
  if (!ws) return api_fail(D2IP_EINVAL, "null workspace");
  if (((uintptr_t)ws & 255) != 0) return api_fail(D2IP_EINVAL, "workspace not 256-byte aligned");
  if (bytes < need)
    return api_fail(D2IP_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  return D2IP_OK;
}

d2ip_status ln_check(int n, int C) {
  if (n < 1 || n > 256) return api_fail(D2IP_EINVAL, "n must be in [1, 256]");
  if (C < 4 || C > 256 || 256 % C != 0)
    return api_fail(D2IP_EINVAL, "C must be a power of two in [4, 256]");
  return D2IP_OK;
}

d2ip_status dw_check(int n, int C) {
  if (n < 1 || n > 256) return api_fail(D2IP_EINVAL, "n must be in [1, 256]");
  if (C < 4 || C > 1024 || C % 4 != 0)
    return api_fail(D2IP_EINVAL, "C must be a multiple of 4 in [4, 1024]");
  return D2IP_OK;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

d2ip_status se_check(int n, int C, int H) {
  if (n < 1 || n > 256) return api_fail(D2IP_EINVAL, "n must be in [1, 256]");
  if (C < 4 || C > 1024 || C % 4 != 0)
    return api_fail(D2IP_EINVAL, "C must be a multiple of 4 in [4, 1024]");
  if (H < 1 || H > 256) return api_fail(D2IP_EINVAL, "H must be in [1, 256]");
  return D2IP_OK;
}

d2ip_status pw_check(int n, int cin, int cout) {
  if (n < 1 || n > 256) return api_fail(D2IP_EINVAL, "n must be in [1, 256]");
  if (cin < 4 || cout < 4 || cin % 4 || cout % 4 || cin > 1024 || cout > 1024)
    return api_fail(D2IP_EINVAL, "cin and cout must be multiples of 4 in [4, 1024]");
  return D2IP_OK;
}

struct LnOp {
  double *st = nullptr, *part_c = nullptr, *part_ab = nullptr, *ctmp = nullptr;
  float* gz = nullptr;
  int nst = 0, nb = 0;
};

void ln_plan(LnOp& l, int n, int C, Piece& w) {
  const size_t V = (size_t)n * n * n;
  l.nst = block_stats_blocks(V * C);
  l.nb = ln_bwd_blocks(V, C);
  l.st = w.take<double>(2 * (size_t)l.nst);
  l.part_c = w.take<double>((size_t)l.nb * 2 * C);
  l.part_ab = w.take<double>(2 * (size_t)l.nb);
  l.gz = w.take<float>(V * C);
  l.ctmp = w.take<double>(colsum_tmp_doubles(l.nb, 2 * C));
}

// Scratch of d2ip_op_jt_noalloc: the per-slice partial sums of J^T g for up
// to kNoAllocMaxQ columns, in a file-scope device array (one copy per GPU,
// held until the process ends).  Host code never uses the array's name as an
// address: its device address is looked up once per device and kept.
constexpr int kNoAllocMaxQ = 64 * 64 * 64;
constexpr size_t kNoAllocScratchBytes = (size_t)8 * kNoAllocMaxQ * sizeof(float);  // 8 MiB
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kNoAllocMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kNoAllocMaxDevices] = {};

d2ip_status head_check(int n, int C) {
  if (n < 1 || n > 512) return api_fail(D2IP_EINVAL, "n must be in [1, 512]");
  if (C < 4 || C > head_max_c() || (C & (C - 1)))
    return api_fail(D2IP_EINVAL, "C must be a power of two in [4, 256]");
  return D2IP_OK;
}
d2ip_status att_check(int n, int c, int cu) {
  if (n < 2 || n % 2 || n > 512) return api_fail(D2IP_EINVAL, "n must be even, in [2, 512]");
  if (c < 4 || c % 4 || c > att_max_c_wide() || cu < 4 || cu % 4 || cu > att_max_cu_wide())
    return api_fail(D2IP_EINVAL, "need c % 4 == 0 <= 256 and cu % 4 == 0 <= 512");
  return D2IP_OK;
}

// Device address of `scratch` on the current device (looked up on the first
// call on that device).
d2ip_status scratch_address(void** out) {
  int dev = -1;
  OPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices) return api_fail(D2IP_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    OPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return api_fail(D2IP_EHIP, "no device address for the scratch array");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return D2IP_OK;
}

}  // namespace

extern "C" {

d2ip_status d2ip_op_conv3d_bytes(int n, int cin, int cout, int taps, int precision, size_t* out) {
  if (!out) return api_fail(D2IP_EINVAL, "null output");
  d2ip_status st = conv_check(n, cin, cout, taps, precision);
  if (st != D2IP_OK) return st;
  Piece w;
  ConvOp c;
  conv_plan(c, n, cin, cout, taps, precision, w);
  *out = w.off + 256;
  return D2IP_OK;
}

d2ip_status d2ip_op_conv3d_forward(const float* x, const float* w, const float* b, float* y, int n,
                                   int cin, int cout, int taps, int precision, void* workspace,
                                   size_t bytes, void* hip_stream) {
  d2ip_status st = conv_check(n, cin, cout, taps, precision);
  if (st != D2IP_OK) return st;
  if (!x || !w || !y) return api_fail(D2IP_EINVAL, "null x, w or y");
  size_t need = 0;
  d2ip_op_conv3d_bytes(n, cin, cout, taps, precision, &need);
  if ((st = ws_check(workspace, bytes, need)) != D2IP_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  Piece pc;
  pc.base = reinterpret_cast<char*>(workspace);
  ConvOp c;
  conv_plan(c, n, cin, cout, taps, precision, pc);
  if ((st = conv_prepare(c, w, s)) != D2IP_OK) return st;
  conv_fwd(fwd_of(c, false, x, b, y), s);
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_conv3d_backward(const float* x, const float* w, const float* gy, float* gx,
                                    float* gw, float* gb, int n, int cin, int cout, int taps,
                                    int precision, void* workspace, size_t bytes,
                                    void* hip_stream) {
  d2ip_status st = conv_check(n, cin, cout, taps, precision);
  if (st != D2IP_OK) return st;
  if (!x || !w || !gy) return api_fail(D2IP_EINVAL, "null x, w or gy");
  size_t need = 0;
  d2ip_op_conv3d_bytes(n, cin, cout, taps, precision, &need);
  if ((st = ws_check(workspace, bytes, need)) != D2IP_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  Piece pc;
  pc.base = reinterpret_cast<char*>(workspace);
  ConvOp c;
  conv_plan(c, n, cin, cout, taps, precision, pc);
  if ((st = conv_prepare(c, w, s)) != D2IP_OK) return st;
  if (gx) conv_fwd(fwd_of(c, true, gy, nullptr, gx), s);
  if (gw || gb) {
    ConvWgrad a;
    std::memset(&a, 0, sizeof(a));
    a.src = plain(x, cin);
    a.gsrc = plain(gy, cout);
    a.n = n;
    a.cin = cin;
    a.cout = cout;
    a.taps = taps;
    a.part = c.part;
    a.partb = c.partb;
    a.splits = c.w_split;
    a.prec = c.prec;
    a.tile = c.w_tile;
    a.ck = c.w_ck;
    a.batch = 1;
    conv_wgrad(a, s);
    GradSeg g;
    std::memset(&g, 0, sizeof(g));
    g.kind = 0;
    g.splits = c.w_split;
    g.cout = cout;
    g.taps = taps;
    g.cin = cin;
    g.cin_real = cin;
    g.th_w = 0;
    g.th_b = cout * cin * taps;
    hipLaunchKernelGGL(k_put<GradSeg>, dim3(1), dim3(64), 0, s, c.seg, g);
    grad_reduce(c.seg, 1, cout * cin * taps, c.part, c.partb, nullptr, c.grad, 1, 0, s);
    const size_t wel = (size_t)cout * cin * taps;
    if (gw) OPCHK(hipMemcpyAsync(gw, c.grad, wel * 4, hipMemcpyDeviceToDevice, s));
    if (gb) OPCHK(hipMemcpyAsync(gb, c.grad + wel, (size_t)cout * 4, hipMemcpyDeviceToDevice, s));
  }
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_ln_relu_bytes(int n, int C, size_t* out) {
  if (!out) return api_fail(D2IP_EINVAL, "null output");
  d2ip_status st = ln_check(n, C);
  if (st != D2IP_OK) return st;
  Piece w;
  LnOp l;
  ln_plan(l, n, C, w);
  *out = w.off + 256;
  return D2IP_OK;
}

d2ip_status d2ip_op_ln_relu_forward(const float* x, const float* gamma, const float* beta,
                                    const float* skip, float* y, int n, int C, void* workspace,
                                    size_t bytes, void* hip_stream) {
  d2ip_status st = ln_check(n, C);
  if (st != D2IP_OK) return st;
  if (!x || !gamma || !beta || !y) return api_fail(D2IP_EINVAL, "null x, gamma, beta or y");
  if (!aligned16(x) || !aligned16(y) || (skip && !aligned16(skip)))
    return api_fail(D2IP_EINVAL, "x, y and skip must be 16-byte aligned");
  size_t need = 0;
  d2ip_op_ln_relu_bytes(n, C, &need);
  if ((st = ws_check(workspace, bytes, need)) != D2IP_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  Piece pc;
  pc.base = reinterpret_cast<char*>(workspace);
  LnOp l;
  ln_plan(l, n, C, pc);
  const size_t V = (size_t)n * n * n;
  block_stats(x, V * C, l.st, s);
  ln_apply(x, PairRef{l.st, l.nst, (double)V * C}, gamma, beta, skip, y, V, C, 1, 0, s);
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_ln_relu_backward(const float* x, const float* y, const float* gamma,
                                     const float* gy, float* gx, float* gskip,
                                     float* dgamma_dbeta, int n, int C, void* workspace,
                                     size_t bytes, void* hip_stream) {
  d2ip_status st = ln_check(n, C);
  if (st != D2IP_OK) return st;
  if (!x || !y || !gamma || !gy) return api_fail(D2IP_EINVAL, "null x, y, gamma or gy");
  if (!aligned16(x) || !aligned16(y) || !aligned16(gy) || (gx && !aligned16(gx)) ||
      (gskip && !aligned16(gskip)))
    return api_fail(D2IP_EINVAL, "x, y, gy, gx and gskip must be 16-byte aligned");
  size_t need = 0;
  d2ip_op_ln_relu_bytes(n, C, &need);
  if ((st = ws_check(workspace, bytes, need)) != D2IP_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  Piece pc;
  pc.base = reinterpret_cast<char*>(workspace);
  LnOp l;
  ln_plan(l, n, C, pc);
  const size_t V = (size_t)n * n * n;
  const PairRef stat{l.st, l.nst, (double)V * C};
  block_stats(x, V * C, l.st, s);
  float* gz = gskip ? gskip : l.gz;
  ln_bwd(gy, LNMASK_Y, y, nullptr, nullptr, x, stat, gz, l.part_c, l.part_ab, V, C, gamma, 1, 0,
         s);
  if (gx) ln_dx(gz, x, stat, PairRef{l.part_ab, l.nb, (double)V * C}, gamma, gx, V, C, s);
  if (dgamma_dbeta) colsum_f64(l.part_c, l.nb, 2 * C, l.ctmp, dgamma_dbeta, s);
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_dwconv3d_bytes(int n, int C, size_t* out) {
  if (!out) return api_fail(D2IP_EINVAL, "null output");
  d2ip_status st = dw_check(n, C);
  if (st != D2IP_OK) return st;
  *out = dw_partials(n, C) * sizeof(float) + 256;
  return D2IP_OK;
}

d2ip_status d2ip_op_dwconv3d_forward(const float* x, const float* w, const float* b, float* y,
                                     int n, int C, void* hip_stream) {
  d2ip_status st = dw_check(n, C);
  if (st != D2IP_OK) return st;
  if (!x || !w || !y) return api_fail(D2IP_EINVAL, "null x, w or y");
  if (!aligned16(x) || !aligned16(y) || (b && !aligned16(b)))
    return api_fail(D2IP_EINVAL, "x, y and b must be 16-byte aligned");
  dw_forward(x, w, b, y, n, C, false, reinterpret_cast<hipStream_t>(hip_stream));
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_dwconv3d_backward(const float* x, const float* w, const float* gy, float* gx,
                                      float* gw, float* gb, int n, int C, void* workspace,
                                      size_t bytes, void* hip_stream) {
  d2ip_status st = dw_check(n, C);
  if (st != D2IP_OK) return st;
  if (!gy || (gx && !w) || ((gw || gb) && !x))
    return api_fail(D2IP_EINVAL, "null gy, or null w with gx, or null x with gw / gb");
  if (!aligned16(gy) || (gx && !aligned16(gx)) || (x && !aligned16(x)))
    return api_fail(D2IP_EINVAL, "x, gy and gx must be 16-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  if (gw || gb) {
    size_t need = 0;
    d2ip_op_dwconv3d_bytes(n, C, &need);
    if ((st = ws_check(workspace, bytes, need)) != D2IP_OK) return st;
    dw_wgrad(x, gy, reinterpret_cast<float*>(workspace), gw, gb, n, C, s);
  }
  if (gx) dw_forward(gy, w, nullptr, gx, n, C, true, s);
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_dwconv3d_dilated_bytes(int n, int C, int dilation, size_t* out) {
  if (!out) return api_fail(D2IP_EINVAL, "null output");
  d2ip_status st = dw_check(n, C);
  if (st != D2IP_OK) return st;
  if (dilation < 1 || dilation > 256) return api_fail(D2IP_EINVAL, "dilation must be in [1, 256]");
  *out = dwd_partials(n, C) * sizeof(float) + 256;
  return D2IP_OK;
}

d2ip_status d2ip_op_dwconv3d_dilated_forward(const float* x, const float* w, const float* b,
                                             float* y, int n, int C, int dilation,
                                             void* hip_stream) {
  d2ip_status st = dw_check(n, C);
  if (st != D2IP_OK) return st;
  if (dilation < 1 || dilation > 256) return api_fail(D2IP_EINVAL, "dilation must be in [1, 256]");
  if (!x || !w || !y) return api_fail(D2IP_EINVAL, "null x, w or y");
  if (!aligned16(x) || !aligned16(y) || (b && !aligned16(b)))
    return api_fail(D2IP_EINVAL, "x, y and b must be 16-byte aligned");
  dwd_forward(x, w, b, y, n, C, dilation, false, reinterpret_cast<hipStream_t>(hip_stream));
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_dwconv3d_dilated_backward(const float* x, const float* w, const float* gy,
                                              float* gx, float* gw, float* gb, int n, int C,
                                              int dilation, void* workspace, size_t bytes,
                                              void* hip_stream) {
  d2ip_status st = dw_check(n, C);
  if (st != D2IP_OK) return st;
  if (dilation < 1 || dilation > 256) return api_fail(D2IP_EINVAL, "dilation must be in [1, 256]");
  if (!gy || (gx && !w) || ((gw || gb) && !x))
    return api_fail(D2IP_EINVAL, "null gy, or null w with gx, or null x with gw / gb");
  if (!aligned16(gy) || (gx && !aligned16(gx)) || (x && !aligned16(x)))
    return api_fail(D2IP_EINVAL, "x, gy and gx must be 16-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  if (gw || gb) {
    size_t need = 0;
    d2ip_op_dwconv3d_dilated_bytes(n, C, dilation, &need);
    if ((st = ws_check(workspace, bytes, need)) != D2IP_OK) return st;
    dwd_wgrad(x, gy, reinterpret_cast<float*>(workspace), gw, gb, n, C, dilation, s);
  }
  if (gx) dwd_forward(gy, w, nullptr, gx, n, C, dilation, true, s);
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_pwconv3d_bytes(int n, int cin, int cout, size_t* out) {
  if (!out) return api_fail(D2IP_EINVAL, "null output");
  d2ip_status st = pw_check(n, cin, cout);
  if (st != D2IP_OK) return st;
  *out = pw_partials((size_t)n * n * n, cin, cout) * sizeof(float) + 256;
  return D2IP_OK;
}

d2ip_status d2ip_op_pwconv3d_forward(const float* x, const float* w, const float* b, float* y,
                                     int n, int cin, int cout, void* hip_stream) {
  d2ip_status st = pw_check(n, cin, cout);
  if (st != D2IP_OK) return st;
  if (!x || !w || !y) return api_fail(D2IP_EINVAL, "null x, w or y");
  if (!aligned16(x) || !aligned16(w) || !aligned16(y))
    return api_fail(D2IP_EINVAL, "x, w and y must be 16-byte aligned");
  pw_gemm(x, w, b, y, (size_t)n * n * n, cin, cout, false,
          reinterpret_cast<hipStream_t>(hip_stream));
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_pwconv3d_backward(const float* x, const float* w, const float* gy, float* gx,
                                      float* gw, float* gb, int n, int cin, int cout,
                                      void* workspace, size_t bytes, void* hip_stream) {
  d2ip_status st = pw_check(n, cin, cout);
  if (st != D2IP_OK) return st;
  if (!gy || (gx && !w) || ((gw || gb) && !x))
    return api_fail(D2IP_EINVAL, "null gy, or null w with gx, or null x with gw / gb");
  if (!aligned16(gy) || (gx && (!aligned16(gx) || !aligned16(w))) || (x && !aligned16(x)))
    return api_fail(D2IP_EINVAL, "x, w, gy and gx must be 16-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const size_t V = (size_t)n * n * n;
  if (gw || gb) {
    size_t need = 0;
    d2ip_op_pwconv3d_bytes(n, cin, cout, &need);
    if ((st = ws_check(workspace, bytes, need)) != D2IP_OK) return st;
    pw_wgrad(x, gy, reinterpret_cast<float*>(workspace), gw, gb, V, cin, cout, s);
  }
  if (gx) pw_gemm(gy, w, nullptr, gx, V, cout, cin, true, s);
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_se_bytes(int n, int C, int H, size_t* out) {
  if (!out) return api_fail(D2IP_EINVAL, "null output");
  d2ip_status st = se_check(n, C, H);
  if (st != D2IP_OK) return st;
  *out = se_scratch(n * n * n, C, H) * sizeof(float) + 256;
  return D2IP_OK;
}

d2ip_status d2ip_op_se_forward(const float* x, const float* w1, const float* b1, const float* w2,
                               const float* b2, float* y, int n, int C, int H, void* workspace,
                               size_t bytes, void* hip_stream) {
  d2ip_status st = se_check(n, C, H);
  if (st != D2IP_OK) return st;
  if (!x || !w1 || !b1 || !w2 || !b2 || !y) return api_fail(D2IP_EINVAL, "null x, y or weights");
  if (!aligned16(x) || !aligned16(y)) return api_fail(D2IP_EINVAL, "x and y must be 16-byte aligned");
  size_t need = 0;
  d2ip_op_se_bytes(n, C, H, &need);
  if ((st = ws_check(workspace, bytes, need)) != D2IP_OK) return st;
  se_forward(x, w1, b1, w2, b2, y, n * n * n, C, H, reinterpret_cast<float*>(workspace),
             reinterpret_cast<hipStream_t>(hip_stream));
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_se_backward(const float* x, const float* w1, const float* b1, const float* w2,
                                const float* b2, const float* gy, float* gx, float* gw1,
                                float* gb1, float* gw2, float* gb2, int n, int C, int H,
                                void* workspace, size_t bytes, void* hip_stream) {
  d2ip_status st = se_check(n, C, H);
  if (st != D2IP_OK) return st;
  if (!x || !w1 || !b1 || !w2 || !b2 || !gy)
    return api_fail(D2IP_EINVAL, "null x, gy or weights");
  if (!aligned16(x) || !aligned16(gy) || (gx && !aligned16(gx)))
    return api_fail(D2IP_EINVAL, "x, gy and gx must be 16-byte aligned");
  size_t need = 0;
  d2ip_op_se_bytes(n, C, H, &need);
  if ((st = ws_check(workspace, bytes, need)) != D2IP_OK) return st;
  se_backward(x, w1, b1, w2, b2, gy, gx, gw1, gb1, gw2, gb2, n * n * n, C, H,
              reinterpret_cast<float*>(workspace), reinterpret_cast<hipStream_t>(hip_stream));
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_j_forward(const float* J, const float* sigma, float* p, int M, int Q,
                              void* hip_stream) {
  if (!J || !sigma || !p) return api_fail(D2IP_EINVAL, "null J, sigma or p");
  if (M < 1 || Q < 4 || Q % 4 != 0) return api_fail(D2IP_EINVAL, "need M >= 1 and Q % 4 == 0");
  jv_dense(J, M, Q, sigma, p, reinterpret_cast<hipStream_t>(hip_stream));
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_jt_bytes(int M, int Q, size_t* out) {
  if (!out) return api_fail(D2IP_EINVAL, "null output");
  if (M < 1 || Q < 4 || Q % 4 != 0) return api_fail(D2IP_EINVAL, "need M >= 1 and Q % 4 == 0");
  *out = jt_dense_scratch(Q) * sizeof(float) + 256;
  return D2IP_OK;
}

d2ip_status d2ip_op_jt(const float* J, const float* g, float* out, int M, int Q, void* workspace,
                       size_t bytes, void* hip_stream) {
  if (!J || !g || !out) return api_fail(D2IP_EINVAL, "null J, g or out");
  size_t need = 0;
  d2ip_status st = d2ip_op_jt_bytes(M, Q, &need);
  if (st != D2IP_OK) return st;
  if ((st = ws_check(workspace, bytes, need)) != D2IP_OK) return st;
  jt_dense(J, M, Q, g, reinterpret_cast<float*>(workspace), out,
           reinterpret_cast<hipStream_t>(hip_stream));
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_pool2_forward(const float* x, float* y, int n, int C, void* hip_stream) {
  if (!x || !y) return api_fail(D2IP_EINVAL, "null x or y");
  if (n < 2 || n % 2 || n > 512 || C < 4 || C % 4) return api_fail(D2IP_EINVAL, "need even n and C % 4 == 0");
  if (!aligned16(x) || !aligned16(y)) return api_fail(D2IP_EINVAL, "x and y must be 16-byte aligned");
  avgpool2(x, n, C, y, reinterpret_cast<hipStream_t>(hip_stream));
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_pool2_backward(const float* gy, float* gx, int n, int C, void* hip_stream) {
  if (!gy || !gx) return api_fail(D2IP_EINVAL, "null gy or gx");
  if (n < 2 || n % 2 || n > 512 || C < 4 || C % 4) return api_fail(D2IP_EINVAL, "need even n and C % 4 == 0");
  if (!aligned16(gx) || !aligned16(gy)) return api_fail(D2IP_EINVAL, "gx and gy must be 16-byte aligned");
  pool_bwd_add(gy, nullptr, n, C, gx, 1, 0, reinterpret_cast<hipStream_t>(hip_stream));
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_up2_concat_forward(const float* d, int Cu, const float* e, int Cs, int n,
                                       float* cat, void* hip_stream) {
  if (!d || !e || !cat) return api_fail(D2IP_EINVAL, "null d, e or cat");
  if (n < 2 || n % 2 || n > 512 || Cu < 4 || Cu % 4 || Cs < 4 || Cs % 4)
    return api_fail(D2IP_EINVAL, "need even n and channel counts multiples of 4");
  if (!aligned16(d) || !aligned16(e) || !aligned16(cat))
    return api_fail(D2IP_EINVAL, "tensors must be 16-byte aligned");
  up_concat(d, Cu, e, Cs, n, cat, 1, 0, reinterpret_cast<hipStream_t>(hip_stream));
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_up2_concat_backward(const float* gcat, int Cu, int Cs, int n, float* gd,
                                        float* ge, void* hip_stream) {
  if (!gcat || !gd || !ge) return api_fail(D2IP_EINVAL, "null gcat, gd or ge");
  if (n < 2 || n % 2 || n > 512 || Cu < 4 || Cu % 4 || Cs < 4 || Cs % 4)
    return api_fail(D2IP_EINVAL, "need even n and channel counts multiples of 4");
  if (!aligned16(gcat) || !aligned16(gd) || !aligned16(ge))
    return api_fail(D2IP_EINVAL, "tensors must be 16-byte aligned");
  up_concat_bwd(gcat, Cu, Cs, n, gd, ge, 1, 0, reinterpret_cast<hipStream_t>(hip_stream));
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_channel_copy(const float* src, int src_ch, int src_off, float* dst, int dst_ch,
                                 int dst_off, int ch, size_t voxels, void* hip_stream) {
  if (!src || !dst) return api_fail(D2IP_EINVAL, "null src or dst");
  if (ch < 4 || src_ch < 4 || dst_ch < 4 || ch % 4 || src_ch % 4 || dst_ch % 4 || src_off % 4 ||
      dst_off % 4 || src_off < 0 || dst_off < 0)
    return api_fail(D2IP_EINVAL, "channel counts and offsets must be non-negative multiples of 4");
  if (src_off + ch > src_ch || dst_off + ch > dst_ch)
    return api_fail(D2IP_EINVAL, "channel range exceeds the tensor's channels");
  if (voxels == 0) return D2IP_OK;
  if (!aligned16(src) || !aligned16(dst)) return api_fail(D2IP_EINVAL, "tensors must be 16-byte aligned");
  const size_t sb = voxels * (size_t)src_ch * 4, db = voxels * (size_t)dst_ch * 4;
  const char *s0 = reinterpret_cast<const char*>(src), *d0 = reinterpret_cast<const char*>(dst);
  if (s0 < d0 + db && d0 < s0 + sb) return api_fail(D2IP_EINVAL, "src and dst overlap");
  channel_copy(src, src_ch, src_off, dst, dst_ch, dst_off, ch, voxels,
               reinterpret_cast<hipStream_t>(hip_stream));
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_relu_forward(const float* x, float* y, size_t count, void* hip_stream) {
  if (!x || !y) return api_fail(D2IP_EINVAL, "null x or y");
  if (count % 4) return api_fail(D2IP_EINVAL, "count must be a multiple of 4");
  if (count == 0) return D2IP_OK;
  if (!aligned16(x) || !aligned16(y)) return api_fail(D2IP_EINVAL, "x and y must be 16-byte aligned");
  relu_forward(x, y, count, reinterpret_cast<hipStream_t>(hip_stream));
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_relu_backward(const float* y, const float* gy, float* gx, size_t count,
                                  void* hip_stream) {
  if (!y || !gy || !gx) return api_fail(D2IP_EINVAL, "null y, gy or gx");
  if (count % 4) return api_fail(D2IP_EINVAL, "count must be a multiple of 4");
  if (count == 0) return D2IP_OK;
  if (!aligned16(y) || !aligned16(gy) || !aligned16(gx))
    return api_fail(D2IP_EINVAL, "tensors must be 16-byte aligned");
  relu_backward(y, gy, gx, count, reinterpret_cast<hipStream_t>(hip_stream));
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_head_bytes(int n, int C, size_t* out) {
  if (!out) return api_fail(D2IP_EINVAL, "null output");
  d2ip_status st = head_check(n, C);
  if (st != D2IP_OK) return st;
  *out = head_scratch_bytes((size_t)n * n * n, C) + 256;
  return D2IP_OK;
}

d2ip_status d2ip_op_head_forward(const float* x, const float* w, const float* b,
                                 const float* mask, float* out, int n, int C, int sigmoid_tail,
                                 void* hip_stream) {
  d2ip_status st = head_check(n, C);
  if (st != D2IP_OK) return st;
  if (!x || !w || !b || !out) return api_fail(D2IP_EINVAL, "null x, w, b or out");
  if (!aligned16(x) || !aligned16(w)) return api_fail(D2IP_EINVAL, "x and w must be 16-byte aligned");
  head_forward(x, w, b, mask, (size_t)n * n * n, C, sigmoid_tail ? 1 : 0, out,
               reinterpret_cast<hipStream_t>(hip_stream));
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_head_backward(const float* x, const float* w, const float* b,
                                  const float* mask, const float* gout, float* gx, float* gw,
                                  float* gb, int n, int C, int sigmoid_tail, void* workspace,
                                  size_t bytes, void* hip_stream) {
  d2ip_status st = head_check(n, C);
  if (st != D2IP_OK) return st;
  if (!x || !w || !b || !gout) return api_fail(D2IP_EINVAL, "null x, w, b or gout");
  if (!aligned16(x) || !aligned16(w) || (gx && !aligned16(gx)))
    return api_fail(D2IP_EINVAL, "x, w and gx must be 16-byte aligned");
  size_t need = 0;
  d2ip_op_head_bytes(n, C, &need);
  if ((st = ws_check(workspace, bytes, need)) != D2IP_OK) return st;
  head_backward(x, w, b, mask, gout, (size_t)n * n * n, C, sigmoid_tail ? 1 : 0, gx, gw, gb,
                workspace, reinterpret_cast<hipStream_t>(hip_stream));
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_attention_bytes(int n, int c, int cu, size_t* out) {
  if (!out) return api_fail(D2IP_EINVAL, "null output");
  d2ip_status st = att_check(n, c, cu);
  if (st != D2IP_OK) return st;
  *out = att_scratch_bytes(n, c, cu) + 256;
  return D2IP_OK;
}

d2ip_status d2ip_op_attention_forward(const float* x, const float* g, const float* wx,
                                      const float* wg, const float* b, const float* psi,
                                      const float* bpsi, float* y, float* alpha, int n, int c,
                                      int cu, void* workspace, size_t bytes, void* hip_stream) {
  d2ip_status st = att_check(n, c, cu);
  if (st != D2IP_OK) return st;
  size_t need = 0;
  d2ip_op_attention_bytes(n, c, cu, &need);
  if ((st = ws_check(workspace, bytes, need)) != D2IP_OK) return st;
  if (!x || !g || !wx || !wg || !b || !psi || !bpsi || !y)
    return api_fail(D2IP_EINVAL, "null tensor");
  if (!aligned16(x) || !aligned16(g) || !aligned16(y) || !aligned16(wx) || !aligned16(wg))
    return api_fail(D2IP_EINVAL, "x, g, y, wx and wg must be 16-byte aligned");
  att_forward(x, g, wx, wg, b, psi, bpsi, y, alpha, n, c, cu, workspace,
              reinterpret_cast<hipStream_t>(hip_stream));
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_attention_backward(const float* x, const float* g, const float* wx,
                                       const float* wg, const float* b, const float* psi,
                                       const float* bpsi, const float* gy, float* gx, float* gg,
                                       float* gwx, float* gwg, float* gb, float* gpsi,
                                       float* gbpsi, int n, int c, int cu, void* workspace,
                                       size_t bytes, void* hip_stream) {
  d2ip_status st = att_check(n, c, cu);
  if (st != D2IP_OK) return st;
  if (!x || !g || !wx || !wg || !b || !psi || !bpsi || !gy)
    return api_fail(D2IP_EINVAL, "null tensor");
  if (!aligned16(x) || !aligned16(g) || !aligned16(gy) || (gx && !aligned16(gx)) ||
      !aligned16(wx) || !aligned16(wg))
    return api_fail(D2IP_EINVAL, "x, g, gy, gx, wx and wg must be 16-byte aligned");
  size_t need = 0;
  d2ip_op_attention_bytes(n, c, cu, &need);
  if ((st = ws_check(workspace, bytes, need)) != D2IP_OK) return st;
  att_backward(x, g, wx, wg, b, psi, bpsi, gy, gx, gg, gwx, gwg, gb, gpsi, gbpsi, n, c, cu,
               workspace, reinterpret_cast<hipStream_t>(hip_stream));
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_mse_loss(const float* p, const float* dv, float* gp, double* loss, int M,
                             void* hip_stream) {
  if (!p || !dv || !loss) return api_fail(D2IP_EINVAL, "null p, dv or loss");
  if (M < 1) return api_fail(D2IP_EINVAL, "need M >= 1");
  mse_loss(p, dv, M, gp, loss, reinterpret_cast<hipStream_t>(hip_stream));
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_op_jt_noalloc(const float* J, const float* g, float* out, int M, int Q,
                               void* hip_stream) {
  if (!J || !g || !out) return api_fail(D2IP_EINVAL, "null J, g or out");
  if (M < 1 || Q < 4 || Q % 4 != 0) return api_fail(D2IP_EINVAL, "need M >= 1 and Q % 4 == 0");
  if (Q > kNoAllocMaxQ)
    return api_fail(D2IP_EINVAL, "Q = " + std::to_string(Q) + " exceeds the " +
                                     std::to_string(kNoAllocMaxQ) +
                                     " columns of the static scratch (use d2ip_op_jt)");
  if (jt_dense_scratch(Q) * sizeof(float) > kNoAllocScratchBytes)
    return api_fail(D2IP_EINVAL, "static scratch too small");
  if (!aligned16(J) || !aligned16(out)) return api_fail(D2IP_EINVAL, "J and out must be 16-byte aligned");
  void* part = nullptr;
  d2ip_status st = scratch_address(&part);
  if (st != D2IP_OK) return st;
  // every partial the sum reads is written first: nothing to clear
  jt_dense(J, M, Q, g, reinterpret_cast<float*>(part), out,
           reinterpret_cast<hipStream_t>(hip_stream));
  OPCHK(hipGetLastError());
  return D2IP_OK;
}

}  // extern "C"
