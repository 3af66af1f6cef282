// The fitting iteration of the 3D-FastResUNet variants (Sec. III-D) in one
// library call: forward from the fixed noise input, p = J sigma, the FP64
// data term and its gradient, J^T, the backward of every module, Adam.
//
// The network is the residual U-Net of the plain context with any mix of the
// paper's lightweight modules: depthwise-separable ResBlock convolutions, an
// SE unit after every encoder ResBlock, an ASPP module at the bottleneck,
// attention units on the decoder skips and the sigmoid output head.  Every
// step runs one of the library's standalone operators (the same kernels the
// d2ip_op_* entry points launch) on buffers carved from the caller's
// workspace, in the order the network defines; the backward is written out
// by hand in reverse order, with every tensor that feeds several consumers
// accumulating their gradients in a fixed order (deterministic).
//
// Parameters live on the device in a padded layout: every tensor of the
// canonical flat order starts at a multiple of four floats (16 bytes), the
// gaps hold zeros (their gradient is zero and Adam leaves them at zero).
// set_params / get_params / get_grad convert from and to the flat order.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "d2ip.h"
#include "kernels.h"

namespace d2ip {
d2ip_status api_fail(d2ip_status s, const std::string& m);
}
using namespace d2ip;

namespace {

#define MNCHK(expr)                                                                      \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return api_fail(D2IP_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)
#define MNOK(expr)                        \
  do {                                    \
    d2ip_status s_ = (expr);              \
    if (s_ != D2IP_OK) return s_;         \
  } while (0)

constexpr int kAsppRates[3] = {1, 2, 3};

// ---- small kernels ----------------------------------------------------------

// w8 [C][8][27] = stem weight [C][1][27] in input channel 0, zeros elsewhere.
__global__ void k_stem_pad(const float* __restrict__ w, int C, float* __restrict__ w8) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= C * 8 * 27) return;
  const int co = i / 216, r = i - co * 216, ci = r / 27, t = r - ci * 27;
  w8[i] = ci == 0 ? w[co * 27 + t] : 0.f;
}

// gw [C][27] = gw8 [C][0][27].
__global__ void k_stem_unpad(const float* __restrict__ gw8, int C, float* __restrict__ gw) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= C * 27) return;
  gw[i] = gw8[(i / 27) * 216 + (i % 27)];
}

// z8 [V][8] = (z[v], 0, ..., 0); maskf[v] = mask[v] != 0.
__global__ void k_prep_input(const float* __restrict__ z, const uint8_t* __restrict__ mask,
                             size_t V, float* __restrict__ z8, float* __restrict__ maskf) {
  for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < V;
       v += (size_t)gridDim.x * blockDim.x) {
    if (z) {
      float4* d = reinterpret_cast<float4*>(z8 + v * 8);
      d[0] = make_float4(z[v], 0.f, 0.f, 0.f);
      d[1] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (mask) maskf[v] = mask[v] ? 1.f : 0.f;
  }
}

// y += x over n4 float4s.
__global__ void k_acc(float4* __restrict__ y, const float4* __restrict__ x, size_t n4) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4;
       i += (size_t)gridDim.x * blockDim.x) {
    float4 a = y[i];
    const float4 b = x[i];
    a.x += b.x;
    a.y += b.y;
    a.z += b.z;
    a.w += b.w;
    y[i] = a;
  }
}

// End of an iteration: the data term becomes the iteration's loss, the step
// counter advances (Adam's bias correction of this step used t + 1).
__global__ void k_end_iter(IterState* it, const double* loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const double L = *loss;
    it->loss = L;
    if (!isfinite(L)) it->nonfinite |= 1;
    it->t = it->t + 1;
  }
}

// Flat-order <-> padded-layout copies: segment k holds flat [f0, f0 + len)
// at padded offset p0.
struct Seg {
  long long f0, p0, len;
};
__global__ void k_unflatten(const Seg* __restrict__ segs, int nseg, const float* __restrict__ flat,
                            float* __restrict__ pad) {
  const Seg s = segs[blockIdx.y];
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < s.len;
       i += (long long)gridDim.x * blockDim.x)
    pad[s.p0 + i] = flat[s.f0 + i];
}
__global__ void k_flatten(const Seg* __restrict__ segs, int nseg, const float* __restrict__ pad,
                          float* __restrict__ flat) {
  const Seg s = segs[blockIdx.y];
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < s.len;
       i += (long long)gridDim.x * blockDim.x)
    flat[s.f0 + i] = pad[s.p0 + i];
}

unsigned blocks_for(size_t work) {
  return (unsigned)std::max<size_t>(1, std::min<size_t>((work + 255) / 256, 8192));
}

// ---- layout -------------------------------------------------------------------

struct Layout {
  std::vector<Seg> segs;  // flat order
  size_t flat = 0, padded = 0;
  size_t add(size_t n) {
    const size_t p = padded;
    segs.push_back(Seg{(long long)flat, (long long)p, (long long)n});
    flat += n;
    padded += (n + 3) / 4 * 4;
    return p;
  }
};

struct ConvP {  // a ResBlock 3x3x3 conv: dense (w, b) or separable (dw, dwb, pw, pwb)
  size_t w = 0, b = 0, dw = 0, dwb = 0, pw = 0, pwb = 0;
};
struct BlockP {
  int n = 0, a = 0, c = 0;  // grid, input and output channels
  ConvP c1, c2;
  size_t g1 = 0, g2 = 0;    // gamma, beta follows at + c
  bool proj = false;
  size_t wp = 0, bp = 0;
};
struct SeP {
  int h = 0;
  size_t w1 = 0, b1 = 0, w2 = 0, b2 = 0;
};
struct AttP {
  size_t wx = 0, wg = 0, b = 0, psi = 0, bpsi = 0;
};
struct AsppP {
  size_t w0 = 0, b0 = 0, dw[3] = {0, 0, 0}, dwb[3] = {0, 0, 0}, pw[3] = {0, 0, 0},
         pwb[3] = {0, 0, 0}, wp = 0, bp = 0;
};

// Buffers of one ResBlock: its input x is owned by the caller.
struct BlockB {
  float *t1 = nullptr, *h1 = nullptr, *a1 = nullptr, *t2 = nullptr, *h2 = nullptr,
        *s = nullptr, *y = nullptr;
};

}  // namespace

struct d2ip_mnet {
  d2ip_mnet_desc d{};
  int L = 0, C = 0, n = 0, M = 0;
  size_t V0 = 0;
  std::vector<int> ch;  // channels per level
  Layout lay;
  size_t stem_w = 0, stem_b = 0, stem_g = 0, head_w = 0, head_b = 0;
  std::vector<BlockP> enc, dec;  // dec[l] for l = 0 .. L-2
  std::vector<SeP> se;
  std::vector<AttP> att;
  AsppP aspp;
  // device buffers
  float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  IterState* it = nullptr;
  double* loss = nullptr;
  Seg* segs = nullptr;
  float *J = nullptr, *maskf = nullptr, *z8 = nullptr, *dv = nullptr, *p = nullptr, *gp = nullptr;
  float *w8 = nullptr, *gw8 = nullptr, *hs = nullptr, *as = nullptr, *sigma = nullptr,
        *gsigma = nullptr;
  std::vector<float*> xin, seo, pooled;   // per encoder level: block input, SE output, pooled
  std::vector<BlockB> eb, db;             // encoder / decoder block buffers
  std::vector<float*> atto, cat;          // per decoder level: gated skip, concatenation
  float *abr[4] = {nullptr, nullptr, nullptr, nullptr}, *at[3] = {nullptr, nullptr, nullptr};
  float *acat = nullptr, *apr = nullptr, *aout = nullptr;
  // gradient buffers
  std::vector<float*> g_enc;  // dL/d(encoder level output)
  std::vector<float*> g_dec;  // dL/d(decoder level output); g_dec[L-1]: bottleneck output
  float *g_a = nullptr, *g_b = nullptr, *g_c = nullptr, *g_d = nullptr, *g_e = nullptr;
  float* flat = nullptr;    // parameters in the flat order (conversion staging)
  char* scratch = nullptr;  // operator workspace (256-byte aligned)
  size_t scratch_bytes = 0;
  float lr = 1e-3f, b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  bool has_problem = false, has_frame = false;
  hipStream_t stream = nullptr;
  // graph form: one iteration captured on `cap`, replayed on `stream`
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
};

namespace {

size_t vox(int n) { return (size_t)n * n * n; }

d2ip_status check_desc(const d2ip_mnet_desc* d) {
  if (!d) return api_fail(D2IP_EINVAL, "null network description");
  if (d->levels < 2 || d->levels > 5) return api_fail(D2IP_EINVAL, "levels must be in [2, 5]");
  if (d->base_ch != 8 && d->base_ch != 16 && d->base_ch != 32)
    return api_fail(D2IP_EINVAL, "base_ch must be 8, 16 or 32");
  if ((d->base_ch << (d->levels - 1)) > 256)
    return api_fail(D2IP_EINVAL, "base_ch * 2^(levels-1) must be <= 256");
  const int f = 1 << (d->levels - 1);
  if (d->n < 2 * f || d->n % f || d->n > 128)
    return api_fail(D2IP_EINVAL, "n must be a multiple of 2^(levels-1), n / 2^(levels-1) >= 2, n <= 128");
  if (d->M < 1) return api_fail(D2IP_EINVAL, "need M >= 1");
  if (d->se_ratio < 0) return api_fail(D2IP_EINVAL, "se_ratio must be >= 0");
  return D2IP_OK;
}

// Parameter layout in the canonical flat order (stem, encoder modules,
// ASPP, decoder modules, head; within a module conv1, norm1, conv2, norm2,
// projection, then its SE or attention unit).
void build_layout(d2ip_mnet& N) {
  const d2ip_mnet_desc& d = N.d;
  Layout& Y = N.lay;
  const int C = N.C, L = N.L;
  N.stem_w = Y.add((size_t)C * 27);
  N.stem_b = Y.add(C);
  N.stem_g = Y.add(C);
  Y.add(C);  // beta
  auto conv = [&](ConvP& c, int a, int b) {
    if (d.sep) {
      c.dw = Y.add((size_t)a * 27);
      c.dwb = Y.add(a);
      c.pw = Y.add((size_t)b * a);
      c.pwb = Y.add(b);
    } else {
      c.w = Y.add((size_t)b * a * 27);
      c.b = Y.add(b);
    }
  };
  auto block = [&](BlockP& B, int n, int a, int b) {
    B.n = n;
    B.a = a;
    B.c = b;
    conv(B.c1, a, b);
    B.g1 = Y.add(b);
    Y.add(b);
    conv(B.c2, b, b);
    B.g2 = Y.add(b);
    Y.add(b);
    B.proj = a != b;
    if (B.proj) {
      B.wp = Y.add((size_t)b * a);
      B.bp = Y.add(b);
    }
  };
  N.enc.assign(L, BlockP());
  N.se.assign(L, SeP());
  for (int l = 0; l < L; ++l) {
    block(N.enc[l], N.n >> l, l == 0 ? C : N.ch[l - 1], N.ch[l]);
    if (d.se_ratio > 0) {
      SeP& s = N.se[l];
      const int c = N.ch[l];
      s.h = std::max(1, c / d.se_ratio);
      s.w1 = Y.add((size_t)s.h * c);
      s.b1 = Y.add(s.h);
      s.w2 = Y.add((size_t)c * s.h);
      s.b2 = Y.add(c);
    }
  }
  if (d.aspp) {
    const int c = N.ch[L - 1];
    N.aspp.w0 = Y.add((size_t)c * c);
    N.aspp.b0 = Y.add(c);
    for (int r = 0; r < 3; ++r) {
      N.aspp.dw[r] = Y.add((size_t)c * 27);
      N.aspp.dwb[r] = Y.add(c);
      N.aspp.pw[r] = Y.add((size_t)c * c);
      N.aspp.pwb[r] = Y.add(c);
    }
    N.aspp.wp = Y.add((size_t)c * 4 * c);
    N.aspp.bp = Y.add(c);
  }
  N.dec.assign(std::max(0, L - 1), BlockP());
  N.att.assign(std::max(0, L - 1), AttP());
  for (int l = L - 2; l >= 0; --l) {
    block(N.dec[l], N.n >> l, N.ch[l + 1] + N.ch[l], N.ch[l]);
    if (d.att) {
      AttP& a = N.att[l];
      const int c = N.ch[l], cu = N.ch[l + 1];
      a.wx = Y.add((size_t)c * c);
      a.wg = Y.add((size_t)c * cu);
      a.b = Y.add(c);
      a.psi = Y.add(c);
      a.bpsi = Y.add(1);
    }
  }
  N.head_w = Y.add(C);
  N.head_b = Y.add(1);
}

// Largest operator workspace the iteration needs (0 and an error if a shape
// is outside an operator's limits).
d2ip_status scratch_need(const d2ip_mnet& N, size_t* out) {
  size_t need = 0, b = 0;
  auto take = [&](d2ip_status st) {
    if (st == D2IP_OK) need = std::max(need, b);
    return st;
  };
  const d2ip_mnet_desc& d = N.d;
  MNOK(take(d2ip_op_conv3d_bytes(N.n, 8, N.C, 27, D2IP_PLAIN_FP32, &b)));
  MNOK(take(d2ip_op_ln_relu_bytes(N.n, N.C, &b)));
  auto conv = [&](int n, int a, int c) -> d2ip_status {
    if (d.sep) {
      MNOK(take(d2ip_op_dwconv3d_bytes(n, a, &b)));
      return take(d2ip_op_pwconv3d_bytes(n, a, c, &b));
    }
    return take(d2ip_op_conv3d_bytes(n, a, c, 27, D2IP_PLAIN_FP32, &b));
  };
  auto block = [&](const BlockP& B) -> d2ip_status {
    MNOK(conv(B.n, B.a, B.c));
    MNOK(conv(B.n, B.c, B.c));
    MNOK(take(d2ip_op_ln_relu_bytes(B.n, B.c, &b)));
    if (B.proj) MNOK(take(d2ip_op_pwconv3d_bytes(B.n, B.a, B.c, &b)));
    return D2IP_OK;
  };
  for (int l = 0; l < N.L; ++l) {
    MNOK(block(N.enc[l]));
    if (d.se_ratio > 0) MNOK(take(d2ip_op_se_bytes(N.enc[l].n, N.ch[l], N.se[l].h, &b)));
  }
  if (d.aspp) {
    const int n = N.n >> (N.L - 1), c = N.ch[N.L - 1];
    MNOK(take(d2ip_op_pwconv3d_bytes(n, c, c, &b)));
    MNOK(take(d2ip_op_pwconv3d_bytes(n, 4 * c, c, &b)));
    for (int r = 0; r < 3; ++r) MNOK(take(d2ip_op_dwconv3d_dilated_bytes(n, c, kAsppRates[r], &b)));
  }
  for (int l = 0; l + 1 < N.L; ++l) {
    MNOK(block(N.dec[l]));
    if (d.att) MNOK(take(d2ip_op_attention_bytes(N.dec[l].n, N.ch[l], N.ch[l + 1], &b)));
  }
  MNOK(take(d2ip_op_head_bytes(N.n, N.C, &b)));
  MNOK(take(d2ip_op_jt_bytes(N.M, (int)N.V0, &b)));
  *out = need;
  return D2IP_OK;
}

// Carves 256-byte aligned pieces (sizes only when base is null).
struct Carve {
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

void carve(d2ip_mnet& N, Carve& cv) {
  const int L = N.L, C = N.C;
  const size_t P = N.lay.padded;
  N.theta = cv.take<float>(P);
  N.grad = cv.take<float>(P);
  N.m = cv.take<float>(P);
  N.v = cv.take<float>(P);
  N.it = cv.take<IterState>(1);
  N.loss = cv.take<double>(1);
  N.segs = cv.take<Seg>(N.lay.segs.size());
  N.J = cv.take<float>((size_t)N.M * N.V0);
  N.maskf = cv.take<float>(N.V0);
  N.z8 = cv.take<float>(N.V0 * 8);
  N.dv = cv.take<float>(N.M);
  N.p = cv.take<float>(N.M);
  N.gp = cv.take<float>(N.M);
  N.w8 = cv.take<float>((size_t)C * 8 * 27);
  N.gw8 = cv.take<float>((size_t)C * 8 * 27);
  N.hs = cv.take<float>(N.V0 * C);
  N.as = cv.take<float>(N.V0 * C);
  N.sigma = cv.take<float>(N.V0);
  N.gsigma = cv.take<float>(N.V0);
  auto block = [&](BlockB& B, const BlockP& P_) {
    const size_t V = vox(P_.n);
    if (N.d.sep) {
      B.t1 = cv.take<float>(V * P_.a);
      B.t2 = cv.take<float>(V * P_.c);
    }
    B.h1 = cv.take<float>(V * P_.c);
    B.a1 = cv.take<float>(V * P_.c);
    B.h2 = cv.take<float>(V * P_.c);
    if (P_.proj) B.s = cv.take<float>(V * P_.c);
    B.y = cv.take<float>(V * P_.c);
  };
  N.xin.assign(L, nullptr);
  N.seo.assign(L, nullptr);
  N.eb.assign(L, BlockB());
  for (int l = 0; l < L; ++l) {
    const size_t V = vox(N.enc[l].n);
    N.xin[l] = l == 0 ? N.as : cv.take<float>(V * N.ch[l - 1]);
    block(N.eb[l], N.enc[l]);
    if (N.d.se_ratio > 0) N.seo[l] = cv.take<float>(V * N.ch[l]);
  }
  if (N.d.aspp) {
    const size_t V = vox(N.n >> (L - 1));
    const int c = N.ch[L - 1];
    for (int r = 0; r < 4; ++r) N.abr[r] = cv.take<float>(V * c);
    for (int r = 0; r < 3; ++r) N.at[r] = cv.take<float>(V * c);
    N.acat = cv.take<float>(V * 4 * c);
    N.apr = cv.take<float>(V * c);
    N.aout = cv.take<float>(V * c);
  }
  N.db.assign(std::max(0, L - 1), BlockB());
  N.atto.assign(std::max(0, L - 1), nullptr);
  N.cat.assign(std::max(0, L - 1), nullptr);
  for (int l = L - 2; l >= 0; --l) {
    const size_t V = vox(N.dec[l].n);
    if (N.d.att) N.atto[l] = cv.take<float>(V * N.ch[l]);
    N.cat[l] = cv.take<float>(V * N.dec[l].a);
    block(N.db[l], N.dec[l]);
  }
  // gradients: one accumulator per encoder / decoder output, and five
  // transient buffers as large as the largest activation (4c at the
  // bottleneck for the ASPP concatenation, 3c for a decoder input)
  N.g_enc.assign(L, nullptr);
  N.g_dec.assign(L, nullptr);
  size_t big = N.V0 * 8;
  for (int l = 0; l < L; ++l) {
    const size_t V = vox(N.n >> l);
    N.g_enc[l] = cv.take<float>(V * N.ch[l]);
    N.g_dec[l] = cv.take<float>(V * N.ch[l]);
    big = std::max(big, V * N.ch[l] * 4);
  }
  N.g_a = cv.take<float>(big);
  N.g_b = cv.take<float>(big);
  N.g_c = cv.take<float>(big);
  N.g_d = cv.take<float>(big);
  N.g_e = cv.take<float>(big);
  N.flat = cv.take<float>(N.lay.flat);
  N.scratch = cv.take<char>(N.scratch_bytes);  // scratch_bytes comes from scratch_need
}

void acc(float* y, const float* x, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_acc, dim3(blocks_for(n / 4)), dim3(256), 0, s, reinterpret_cast<float4*>(y),
                     reinterpret_cast<const float4*>(x), n / 4);
}

// ---- forward ------------------------------------------------------------------

#define WS N.scratch, N.scratch_bytes, N.stream

d2ip_status conv_fwd(d2ip_mnet& N, const ConvP& c, const float* x, float* t, float* y, int n,
                     int a, int b) {
  const float* th = N.theta;
  if (N.d.sep) {
    MNOK(d2ip_op_dwconv3d_forward(x, th + c.dw, th + c.dwb, t, n, a, N.stream));
    return d2ip_op_pwconv3d_forward(t, th + c.pw, th + c.pwb, y, n, a, b, N.stream);
  }
  return d2ip_op_conv3d_forward(x, th + c.w, th + c.b, y, n, a, b, 27, D2IP_PLAIN_FP32, WS);
}

d2ip_status block_fwd(d2ip_mnet& N, const BlockP& P, BlockB& B, const float* x) {
  const float* th = N.theta;
  MNOK(conv_fwd(N, P.c1, x, B.t1, B.h1, P.n, P.a, P.c));
  MNOK(d2ip_op_ln_relu_forward(B.h1, th + P.g1, th + P.g1 + P.c, nullptr, B.a1, P.n, P.c, WS));
  MNOK(conv_fwd(N, P.c2, B.a1, B.t2, B.h2, P.n, P.c, P.c));
  const float* skip = x;
  if (P.proj) {
    MNOK(d2ip_op_pwconv3d_forward(x, th + P.wp, th + P.bp, B.s, P.n, P.a, P.c, N.stream));
    skip = B.s;
  }
  return d2ip_op_ln_relu_forward(B.h2, th + P.g2, th + P.g2 + P.c, skip, B.y, P.n, P.c, WS);
}

// Output of encoder level l (after its SE unit) and of the bottleneck.
float* enc_out(d2ip_mnet& N, int l) { return N.d.se_ratio > 0 ? N.seo[l] : N.eb[l].y; }
float* bottleneck(d2ip_mnet& N) { return N.d.aspp ? N.aout : enc_out(N, N.L - 1); }
float* dec_out(d2ip_mnet& N, int l) { return l == N.L - 1 ? bottleneck(N) : N.db[l].y; }

d2ip_status forward(d2ip_mnet& N) {
  const float* th = N.theta;
  const int L = N.L, C = N.C;
  hipLaunchKernelGGL(k_stem_pad, dim3((C * 216 + 255) / 256), dim3(256), 0, N.stream,
                     th + N.stem_w, C, N.w8);
  MNOK(d2ip_op_conv3d_forward(N.z8, N.w8, th + N.stem_b, N.hs, N.n, 8, C, 27, D2IP_PLAIN_FP32, WS));
  MNOK(d2ip_op_ln_relu_forward(N.hs, th + N.stem_g, th + N.stem_g + C, nullptr, N.as, N.n, C, WS));
  for (int l = 0; l < L; ++l) {
    const BlockP& P = N.enc[l];
    if (l > 0) MNOK(d2ip_op_pool2_forward(enc_out(N, l - 1), N.xin[l], N.n >> (l - 1), N.ch[l - 1],
                                          N.stream));
    MNOK(block_fwd(N, P, N.eb[l], N.xin[l]));
    if (N.d.se_ratio > 0) {
      const SeP& s = N.se[l];
      MNOK(d2ip_op_se_forward(N.eb[l].y, th + s.w1, th + s.b1, th + s.w2, th + s.b2, N.seo[l], P.n,
                              P.c, s.h, WS));
    }
  }
  if (N.d.aspp) {
    const AsppP& A = N.aspp;
    const int n = N.n >> (L - 1), c = N.ch[L - 1];
    const size_t V = vox(n);
    const float* x = enc_out(N, L - 1);
    MNOK(d2ip_op_pwconv3d_forward(x, th + A.w0, th + A.b0, N.abr[0], n, c, c, N.stream));
    for (int r = 0; r < 3; ++r) {
      MNOK(d2ip_op_dwconv3d_dilated_forward(x, th + A.dw[r], th + A.dwb[r], N.at[r], n, c,
                                            kAsppRates[r], N.stream));
      MNOK(d2ip_op_pwconv3d_forward(N.at[r], th + A.pw[r], th + A.pwb[r], N.abr[r + 1], n, c, c,
                                    N.stream));
    }
    for (int r = 0; r < 4; ++r)
      MNOK(d2ip_op_channel_copy(N.abr[r], c, 0, N.acat, 4 * c, r * c, c, V, N.stream));
    MNOK(d2ip_op_pwconv3d_forward(N.acat, th + A.wp, th + A.bp, N.apr, n, 4 * c, c, N.stream));
    MNOK(d2ip_op_relu_forward(N.apr, N.aout, V * c, N.stream));
  }
  for (int l = L - 2; l >= 0; --l) {
    const BlockP& P = N.dec[l];
    const float* s = enc_out(N, l);
    const float* g = dec_out(N, l + 1);
    if (N.d.att) {
      const AttP& a = N.att[l];
      MNOK(d2ip_op_attention_forward(s, g, th + a.wx, th + a.wg, th + a.b, th + a.psi, th + a.bpsi,
                                     N.atto[l], nullptr, P.n, N.ch[l], N.ch[l + 1], WS));
      s = N.atto[l];
    }
    MNOK(d2ip_op_up2_concat_forward(g, N.ch[l + 1], s, N.ch[l], P.n, N.cat[l], N.stream));
    MNOK(block_fwd(N, P, N.db[l], N.cat[l]));
  }
  return d2ip_op_head_forward(dec_out(N, 0), th + N.head_w, th + N.head_b, N.maskf, N.sigma, N.n,
                              C, N.d.sigmoid_tail ? 1 : 0, N.stream);
}

// ---- backward -----------------------------------------------------------------

// gx = dL/dx of one conv given gy (gx may be null); parameter gradients into grad.
d2ip_status conv_bwd(d2ip_mnet& N, const ConvP& c, const float* x, const float* t, const float* gy,
                     float* gx, float* gt, int n, int a, int b) {
  const float* th = N.theta;
  float* gr = N.grad;
  if (N.d.sep) {
    MNOK(d2ip_op_pwconv3d_backward(t, th + c.pw, gy, gt, gr + c.pw, gr + c.pwb, n, a, b, WS));
    return d2ip_op_dwconv3d_backward(x, th + c.dw, gt, gx, gr + c.dw, gr + c.dwb, n, a, WS);
  }
  return d2ip_op_conv3d_backward(x, th + c.w, gy, gx, gr + c.w, gr + c.b, n, a, b, 27,
                                 D2IP_PLAIN_FP32, WS);
}

// gx (written) = dL/dx of a ResBlock given gy = dL/dy.  Uses g_a .. g_d.
d2ip_status block_bwd(d2ip_mnet& N, const BlockP& P, const BlockB& B, const float* x,
                      const float* gy, float* gx) {
  const float* th = N.theta;
  float* gr = N.grad;
  const size_t V = vox(P.n);
  float *gh = N.g_a, *gs = N.g_b, *ga = N.g_c, *gt = N.g_d;
  MNOK(d2ip_op_ln_relu_backward(B.h2, B.y, th + P.g2, gy, gh, gs, gr + P.g2, P.n, P.c, WS));
  MNOK(conv_bwd(N, P.c2, B.a1, B.t2, gh, ga, gt, P.n, P.c, P.c));
  MNOK(d2ip_op_ln_relu_backward(B.h1, B.a1, th + P.g1, ga, gh, nullptr, gr + P.g1, P.n, P.c, WS));
  MNOK(conv_bwd(N, P.c1, x, B.t1, gh, gx, gt, P.n, P.a, P.c));
  if (P.proj) {
    MNOK(d2ip_op_pwconv3d_backward(x, th + P.wp, gs, ga, gr + P.wp, gr + P.bp, P.n, P.a, P.c,
                                   WS));
    acc(gx, ga, V * P.a, N.stream);
  } else {
    acc(gx, gs, V * P.c, N.stream);
  }
  return D2IP_OK;
}

d2ip_status backward(d2ip_mnet& N) {
  const float* th = N.theta;
  float* gr = N.grad;
  const int L = N.L, C = N.C;
  for (int l = 0; l < L; ++l) {
    const size_t V = vox(N.n >> l);
    zero_words(N.g_enc[l], V * N.ch[l], N.stream);
    zero_words(N.g_dec[l], V * N.ch[l], N.stream);
  }
  // data term -> image -> head
  MNOK(d2ip_op_jt(N.J, N.gp, N.gsigma, N.M, (int)N.V0, WS));
  MNOK(d2ip_op_head_backward(dec_out(N, 0), th + N.head_w, th + N.head_b, N.maskf, N.gsigma,
                             N.g_dec[0], gr + N.head_w, gr + N.head_b, N.n, C,
                             N.d.sigmoid_tail ? 1 : 0, WS));
  // decoder, finest first
  for (int l = 0; l <= L - 2; ++l) {
    const BlockP& P = N.dec[l];
    const size_t V = vox(P.n), Vc = vox(P.n / 2);
    float* gcat = N.g_e;
    MNOK(block_bwd(N, P, N.db[l], N.cat[l], N.g_dec[l], gcat));
    // concatenation [up2(g), s]: gd to the coarser output, ge to the (gated) skip
    float *gd = N.g_a, *ge = N.g_b;
    MNOK(d2ip_op_up2_concat_backward(gcat, N.ch[l + 1], N.ch[l], P.n, gd, ge, N.stream));
    acc(N.g_dec[l + 1], gd, Vc * N.ch[l + 1], N.stream);
    if (N.d.att) {
      const AttP& a = N.att[l];
      float *gsk = N.g_c, *gg = N.g_d;
      MNOK(d2ip_op_attention_backward(enc_out(N, l), dec_out(N, l + 1), th + a.wx, th + a.wg,
                                      th + a.b, th + a.psi, th + a.bpsi, ge, gsk, gg, gr + a.wx,
                                      gr + a.wg, gr + a.b, gr + a.psi, gr + a.bpsi, P.n, N.ch[l],
                                      N.ch[l + 1], WS));
      acc(N.g_dec[l + 1], gg, Vc * N.ch[l + 1], N.stream);
      acc(N.g_enc[l], gsk, V * N.ch[l], N.stream);
    } else {
      acc(N.g_enc[l], ge, V * N.ch[l], N.stream);
    }
  }
  // bottleneck
  {
    const int n = N.n >> (L - 1), c = N.ch[L - 1];
    const size_t V = vox(n);
    if (N.d.aspp) {
      const AsppP& A = N.aspp;
      const float* x = enc_out(N, L - 1);
      float *gpr = N.g_a, *gcat = N.g_b, *gbr = N.g_c, *gt = N.g_d, *gx = N.g_e;
      MNOK(d2ip_op_relu_backward(N.aout, N.g_dec[L - 1], gpr, V * c, N.stream));
      MNOK(d2ip_op_pwconv3d_backward(N.acat, th + A.wp, gpr, gcat, gr + A.wp, gr + A.bp, n, 4 * c,
                                     c, WS));
      MNOK(d2ip_op_channel_copy(gcat, 4 * c, 0, gbr, c, 0, c, V, N.stream));
      MNOK(d2ip_op_pwconv3d_backward(x, th + A.w0, gbr, gx, gr + A.w0, gr + A.b0, n, c, c, WS));
      acc(N.g_enc[L - 1], gx, V * c, N.stream);
      for (int r = 0; r < 3; ++r) {
        MNOK(d2ip_op_channel_copy(gcat, 4 * c, (r + 1) * c, gbr, c, 0, c, V, N.stream));
        MNOK(d2ip_op_pwconv3d_backward(N.at[r], th + A.pw[r], gbr, gt, gr + A.pw[r],
                                       gr + A.pwb[r], n, c, c, WS));
        MNOK(d2ip_op_dwconv3d_dilated_backward(x, th + A.dw[r], gt, gx, gr + A.dw[r],
                                               gr + A.dwb[r], n, c, kAsppRates[r], WS));
        acc(N.g_enc[L - 1], gx, V * c, N.stream);
      }
    } else {
      acc(N.g_enc[L - 1], N.g_dec[L - 1], V * c, N.stream);
    }
  }
  // encoder, coarsest first
  for (int l = L - 1; l >= 0; --l) {
    const BlockP& P = N.enc[l];
    const float* gy = N.g_enc[l];
    if (N.d.se_ratio > 0) {
      const SeP& s = N.se[l];
      MNOK(d2ip_op_se_backward(N.eb[l].y, th + s.w1, th + s.b1, th + s.w2, th + s.b2, gy, N.g_e,
                               gr + s.w1, gr + s.b1, gr + s.w2, gr + s.b2, P.n, P.c, s.h, WS));
      gy = N.g_e;
    }
    // g_e may hold gy: the block writes its input gradient elsewhere first
    float* gx = l > 0 ? N.g_dec[l] : N.g_dec[0];
    // g_dec[l] is free here (the decoder pass has consumed it); for l == 0
    // the block input is the stem output
    MNOK(block_bwd(N, P, N.eb[l], N.xin[l], gy, gx));
    if (l > 0) {
      float* gp_ = N.g_e;
      MNOK(d2ip_op_pool2_backward(gx, gp_, N.n >> (l - 1), N.ch[l - 1], N.stream));
      acc(N.g_enc[l - 1], gp_, vox(N.n >> (l - 1)) * N.ch[l - 1], N.stream);
    }
  }
  // stem: the encoder's input gradient is in g_dec[0]
  MNOK(d2ip_op_ln_relu_backward(N.hs, N.as, th + N.stem_g, N.g_dec[0], N.g_a, nullptr,
                                gr + N.stem_g, N.n, C, WS));
  MNOK(d2ip_op_conv3d_backward(N.z8, N.w8, N.g_a, nullptr, N.gw8, gr + N.stem_b, N.n, 8, C, 27,
                               D2IP_PLAIN_FP32, WS));
  hipLaunchKernelGGL(k_stem_unpad, dim3((C * 27 + 255) / 256), dim3(256), 0, N.stream, N.gw8, C,
                     gr + N.stem_w);
  return D2IP_OK;
}

d2ip_status iteration(d2ip_mnet& N) {
  MNOK(forward(N));
  MNOK(d2ip_op_j_forward(N.J, N.sigma, N.p, N.M, (int)N.V0, N.stream));
  MNOK(d2ip_op_mse_loss(N.p, N.dv, N.gp, N.loss, N.M, N.stream));
  MNOK(backward(N));
  adam(N.theta, N.grad, N.m, N.v, N.lay.padded, N.lr, N.b1, N.b2, N.eps, N.it, 1, 0, N.stream);
  hipLaunchKernelGGL(k_end_iter, dim3(1), dim3(64), 0, N.stream, N.it, N.loss);
  MNCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status copy_in(void* dst, const void* src, size_t bytes, int on_device, hipStream_t s) {
  MNCHK(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                       s));
  if (!on_device) MNCHK(hipStreamSynchronize(s));  // the host buffer may go once we return
  return D2IP_OK;
}

// padded <-> flat through the segment table (device side)
d2ip_status convert(d2ip_mnet& N, const float* src, float* dst, bool to_padded) {
  const dim3 grid(64, (unsigned)N.lay.segs.size());
  if (to_padded)
    hipLaunchKernelGGL(k_unflatten, grid, dim3(256), 0, N.stream, N.segs, (int)N.lay.segs.size(),
                       src, dst);
  else
    hipLaunchKernelGGL(k_flatten, grid, dim3(256), 0, N.stream, N.segs, (int)N.lay.segs.size(),
                       src, dst);
  MNCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status setup(const d2ip_mnet_desc* desc, d2ip_mnet& N) {
  MNOK(check_desc(desc));
  N.d = *desc;
  N.L = desc->levels;
  N.C = desc->base_ch;
  N.n = desc->n;
  N.M = desc->M;
  N.V0 = vox(N.n);
  N.ch.resize(N.L);
  for (int l = 0; l < N.L; ++l) N.ch[l] = N.C << l;
  build_layout(N);
  return scratch_need(N, &N.scratch_bytes);
}

d2ip_status total_bytes(d2ip_mnet& N, size_t* out) {
  Carve cv;
  carve(N, cv);
  *out = cv.off + 256;
  return D2IP_OK;
}

void drop_graph(d2ip_mnet& N) {
  if (N.gexec) (void)hipGraphExecDestroy(N.gexec);
  if (N.graph) (void)hipGraphDestroy(N.graph);
  N.gexec = nullptr;
  N.graph = nullptr;
}

// Records one iteration on the capture stream (every operator's launches and
// copies; none allocates, fills with memset or synchronises) and instantiates it.
d2ip_status capture(d2ip_mnet& N) {
  hipStream_t user = N.stream;
  N.stream = N.cap;
  hipError_t e = hipStreamBeginCapture(N.cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    N.stream = user;
    return api_fail(D2IP_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  }
  const d2ip_status st = iteration(N);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(N.cap, &g);
  N.stream = user;
  if (st != D2IP_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return api_fail(D2IP_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  N.graph = g;
  e = hipGraphInstantiate(&N.gexec, N.graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(N);
    return api_fail(D2IP_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
  }
  return D2IP_OK;
}

}  // namespace

extern "C" {

d2ip_status d2ip_mnet_param_count(const d2ip_mnet_desc* desc, size_t* out) {
  if (!out) return api_fail(D2IP_EINVAL, "null output");
  MNOK(check_desc(desc));
  d2ip_mnet N;
  N.d = *desc;
  N.L = desc->levels;
  N.C = desc->base_ch;
  N.n = desc->n;
  N.ch.resize(N.L);
  for (int l = 0; l < N.L; ++l) N.ch[l] = N.C << l;
  build_layout(N);
  *out = N.lay.flat;
  return D2IP_OK;
}

d2ip_status d2ip_mnet_workspace_bytes(const d2ip_mnet_desc* desc, size_t* out) {
  if (!out) return api_fail(D2IP_EINVAL, "null output");
  d2ip_mnet N;
  MNOK(setup(desc, N));
  return total_bytes(N, out);
}

d2ip_status d2ip_mnet_create(const d2ip_mnet_desc* desc, void* workspace, size_t bytes,
                             void* hip_stream, d2ip_mnet** out) {
  if (!out) return api_fail(D2IP_EINVAL, "null output");
  *out = nullptr;
  d2ip_mnet* N = new d2ip_mnet();
  d2ip_status st = setup(desc, *N);
  size_t need = 0;
  if (st == D2IP_OK) st = total_bytes(*N, &need);
  if (st == D2IP_OK && (!workspace || ((uintptr_t)workspace & 255)))
    st = api_fail(D2IP_EINVAL, "workspace must be non-null and 256-byte aligned");
  if (st == D2IP_OK && bytes < need)
    st = api_fail(D2IP_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  if (st != D2IP_OK) {
    delete N;
    return st;
  }
  N->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (desc->graph && hipStreamCreateWithFlags(&N->cap, hipStreamNonBlocking) != hipSuccess) {
    delete N;
    return api_fail(D2IP_EHIP, "capture stream");
  }
  Carve cv;
  cv.base = reinterpret_cast<char*>(workspace);
  carve(*N, cv);
  // zero parameters, gradients (their padding stays zero), moments and state
  zero_words(N->theta, N->lay.padded, N->stream);
  zero_words(N->grad, N->lay.padded, N->stream);
  zero_words(N->m, N->lay.padded, N->stream);
  zero_words(N->v, N->lay.padded, N->stream);
  zero_words(N->it, sizeof(IterState) / 4, N->stream);
  st = copy_in(N->segs, N->lay.segs.data(), N->lay.segs.size() * sizeof(Seg), 0, N->stream);
  if (st == D2IP_OK && hipGetLastError() != hipSuccess) st = api_fail(D2IP_EHIP, "setup launch");
  if (st != D2IP_OK) {
    if (N->cap) (void)hipStreamDestroy(N->cap);
    delete N;
    return st;
  }
  *out = N;
  return D2IP_OK;
}

d2ip_status d2ip_mnet_destroy(d2ip_mnet* N) {
  if (!N) return D2IP_OK;
  const hipError_t e = hipStreamSynchronize(N->stream);  // nothing may still use the workspace
  drop_graph(*N);
  if (N->cap) (void)hipStreamDestroy(N->cap);
  delete N;
  if (e != hipSuccess) return api_fail(D2IP_EHIP, std::string("destroy: ") + hipGetErrorString(e));
  return D2IP_OK;
}

d2ip_status d2ip_mnet_set_problem(d2ip_mnet* N, const float* J, const uint8_t* mask,
                                  const float* z, int on_device) {
  if (!N || !J || !mask || !z) return api_fail(D2IP_EINVAL, "null argument");
  MNOK(copy_in(N->J, J, (size_t)N->M * N->V0 * 4, on_device, N->stream));
  // mask and z staged through the gradient buffers (free between iterations)
  MNOK(copy_in(N->g_a, z, N->V0 * 4, on_device, N->stream));
  MNOK(copy_in(N->g_b, mask, N->V0, on_device, N->stream));
  hipLaunchKernelGGL(k_prep_input, dim3(blocks_for(N->V0)), dim3(256), 0, N->stream, N->g_a,
                     reinterpret_cast<const uint8_t*>(N->g_b), N->V0, N->z8, N->maskf);
  MNCHK(hipGetLastError());
  N->has_problem = true;
  return D2IP_OK;
}

d2ip_status d2ip_mnet_set_params(d2ip_mnet* N, const float* theta, size_t n, int on_device) {
  if (!N || !theta) return api_fail(D2IP_EINVAL, "null argument");
  if (n != N->lay.flat)
    return api_fail(D2IP_EINVAL, "theta must hold " + std::to_string(N->lay.flat) + " floats");
  MNOK(copy_in(N->flat, theta, n * 4, on_device, N->stream));
  MNOK(convert(*N, N->flat, N->theta, true));
  zero_words(N->grad, N->lay.padded, N->stream);
  zero_words(N->it, sizeof(IterState) / 4, N->stream);
  return d2ip_mnet_reset_optimizer(N);
}

d2ip_status d2ip_mnet_get_params(d2ip_mnet* N, float* theta, size_t n, int on_device) {
  if (!N || !theta) return api_fail(D2IP_EINVAL, "null argument");
  if (n != N->lay.flat)
    return api_fail(D2IP_EINVAL, "theta must hold " + std::to_string(N->lay.flat) + " floats");
  MNOK(convert(*N, N->theta, N->flat, false));
  MNCHK(hipMemcpyAsync(theta, N->flat, n * 4,
                       on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, N->stream));
  MNCHK(hipStreamSynchronize(N->stream));
  return D2IP_OK;
}

d2ip_status d2ip_mnet_get_grad(d2ip_mnet* N, float* grad, size_t n, int on_device) {
  if (!N || !grad) return api_fail(D2IP_EINVAL, "null argument");
  if (n != N->lay.flat)
    return api_fail(D2IP_EINVAL, "grad must hold " + std::to_string(N->lay.flat) + " floats");
  MNOK(convert(*N, N->grad, N->flat, false));
  MNCHK(hipMemcpyAsync(grad, N->flat, n * 4,
                       on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, N->stream));
  MNCHK(hipStreamSynchronize(N->stream));
  return D2IP_OK;
}

d2ip_status d2ip_mnet_set_frame(d2ip_mnet* N, const float* dv, int on_device) {
  if (!N || !dv) return api_fail(D2IP_EINVAL, "null argument");
  MNOK(copy_in(N->dv, dv, (size_t)N->M * 4, on_device, N->stream));
  N->has_frame = true;
  return D2IP_OK;
}

d2ip_status d2ip_mnet_set_adam(d2ip_mnet* N, const d2ip_adam_cfg* cfg) {
  if (!N || !cfg) return api_fail(D2IP_EINVAL, "null argument");
  if (!(cfg->lr > 0.f) || !(cfg->beta1 >= 0.f && cfg->beta1 < 1.f) ||
      !(cfg->beta2 >= 0.f && cfg->beta2 < 1.f) || !(cfg->eps > 0.f))
    return api_fail(D2IP_EINVAL, "need lr > 0, beta1 and beta2 in [0, 1), eps > 0");
  N->lr = cfg->lr;
  N->b1 = cfg->beta1;
  N->b2 = cfg->beta2;
  N->eps = cfg->eps;
  drop_graph(*N);  // the captured Adam step holds the old values
  return D2IP_OK;
}

d2ip_status d2ip_mnet_reset_optimizer(d2ip_mnet* N) {
  if (!N) return api_fail(D2IP_EINVAL, "null argument");
  zero_words(N->m, N->lay.padded, N->stream);
  zero_words(N->v, N->lay.padded, N->stream);
  zero_words(&N->it->t, 1, N->stream);
  MNCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_mnet_run(d2ip_mnet* N, int k, double* last_loss) {
  if (!N) return api_fail(D2IP_EINVAL, "null argument");
  if (k < 0) return api_fail(D2IP_EINVAL, "k must be >= 0");
  if (!N->has_problem) return api_fail(D2IP_ESTATE, "problem (J, mask, noise input) not set");
  if (!N->has_frame) return api_fail(D2IP_ESTATE, "frame not set");
  if (k > 0 && N->d.graph) {
    if (!N->gexec) MNOK(capture(*N));
    for (int i = 0; i < k; ++i) MNCHK(hipGraphLaunch(N->gexec, N->stream));
  } else {
    for (int i = 0; i < k; ++i) MNOK(iteration(*N));
  }
  if (last_loss) {
    IterState st{};
    MNCHK(hipMemcpyAsync(&st, N->it, sizeof(st), hipMemcpyDeviceToHost, N->stream));
    MNCHK(hipStreamSynchronize(N->stream));
    *last_loss = st.loss;
    if (st.nonfinite) return api_fail(D2IP_ENONFINITE, "a non-finite loss or parameter was produced");
  }
  return D2IP_OK;
}

d2ip_status d2ip_mnet_read_image(d2ip_mnet* N, float* sigma, int on_device) {
  if (!N || !sigma) return api_fail(D2IP_EINVAL, "null argument");
  if (!N->has_problem) return api_fail(D2IP_ESTATE, "problem (J, mask, noise input) not set");
  MNOK(forward(*N));
  MNCHK(hipMemcpyAsync(sigma, N->sigma, N->V0 * 4,
                       on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, N->stream));
  MNCHK(hipStreamSynchronize(N->stream));
  return D2IP_OK;
}

}  // extern "C"
