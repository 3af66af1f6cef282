// Drives every C-ABI entry point of the library through the host emulation
// of the HIP runtime (device memory = host memory, launches not executed), so
// that AddressSanitizer sees all host-side bookkeeping: workspace planning,
// uploads, graph capture and replay, state save/restore, kernel timing and
// teardown, for several instance layouts, precisions and both run modes.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <tuple>
#include <vector>

#include "d2ip.h"

extern "C" long g_launches;
extern "C" long g_captured_launches;
extern "C" long emu_errors(void);
extern "C" void emu_flush_all(void);

#define CK(x)                                                              \
  do {                                                                     \
    d2ip_status s_ = (x);                                                  \
    if (s_) {                                                              \
      printf("FAIL %s: %d %s\n", #x, (int)s_, d2ip_last_error());          \
      return 1;                                                            \
    }                                                                      \
  } while (0)
#define EXPECT_ERR(x, code)                                                \
  do {                                                                     \
    if ((x) != (code)) {                                                   \
      printf("FAIL %s: expected %d\n", #x, (int)(code));                   \
      return 1;                                                            \
    }                                                                      \
  } while (0)

static int run_case(const std::vector<d2ip_geometry_desc>& G,
                    const std::vector<d2ip_instance_desc>& I, int prec, unsigned flags) {
  size_t need = 0;
  CK(d2ip_workspace_bytes(G.data(), (int)G.size(), I.data(), (int)I.size(), prec, flags, &need));
  char* ws = (char*)aligned_alloc(256, (need + 255) / 256 * 256);
  d2ip_ctx* X = nullptr;
  EXPECT_ERR(d2ip_create(G.data(), (int)G.size(), I.data(), (int)I.size(), prec, flags, ws,
                         need - 1, nullptr, &X),
             D2IP_ENOMEM);
  CK(d2ip_create(G.data(), (int)G.size(), I.data(), (int)I.size(), prec, flags, ws, need,
                 nullptr, &X));
  std::vector<double> loss(I.size());
  EXPECT_ERR(d2ip_run(X, 1, loss.data()), D2IP_ESTATE);
  std::mt19937 rng(1);
  std::normal_distribution<float> nd;
  for (size_t g = 0; g < G.size(); ++g) {
    const size_t Q = (size_t)G[g].n * G[g].n * G[g].n;
    std::vector<float> J((size_t)G[g].M * Q);
    for (float& v : J) v = nd(rng);
    std::vector<uint8_t> mask(Q);
    for (size_t q = 0; q < Q; ++q) mask[q] = (q * 7 % 5) != 0;
    CK(d2ip_set_geometry(X, (int)g, J.data(), mask.data(), 0));
  }
  for (size_t i = 0; i < I.size(); ++i) {
    size_t P = 0;
    CK(d2ip_param_count(I[i].levels, I[i].base_ch, &P));
    std::vector<float> th(P);
    for (float& v : th) v = 0.1f * nd(rng);
    EXPECT_ERR(d2ip_set_params(X, (int)i, th.data(), P - 1, 0), D2IP_EINVAL);
    CK(d2ip_set_params(X, (int)i, th.data(), P, 0));
    const size_t V = (size_t)G[I[i].geometry].n * G[I[i].geometry].n * G[I[i].geometry].n;
    std::vector<float> z(V);
    for (float& v : z) v = nd(rng);
    CK(d2ip_set_noise_input(X, (int)i, z.data(), 0));
    std::vector<float> dv(G[I[i].geometry].M);
    for (float& v : dv) v = nd(rng);
    CK(d2ip_set_frame(X, (int)i, dv.data(), 0));
  }
  EXPECT_ERR(d2ip_set_frame(X, (int)I.size(), nullptr, 0), D2IP_EINVAL);
  CK(d2ip_run(X, 4, loss.data()));
  d2ip_tv_cfg tv = {0.002f, 1.f, 0.1f, 1e-8f};
  CK(d2ip_set_tv(X, &tv));
  for (int rep = 0; rep < 34; ++rep) CK(d2ip_commit_frame(X, rep % (int)I.size()));
  CK(d2ip_run(X, 2, loss.data()));
  CK(d2ip_clear_history(X, 0));
  tv.eps = 0.f;
  EXPECT_ERR(d2ip_set_tv(X, &tv), D2IP_EINVAL);
  d2ip_adam_cfg cfg = {2e-3f, 0.9f, 0.999f, 1e-8f};
  CK(d2ip_set_adam(X, &cfg));
  CK(d2ip_run(X, 2, nullptr));
  for (size_t i = 0; i < I.size(); ++i) {
    size_t P = 0;
    CK(d2ip_param_count(I[i].levels, I[i].base_ch, &P));
    std::vector<float> st(3 * P), g(P);
    int64_t t = 0;
    CK(d2ip_get_state(X, (int)i, st.data(), &t, 0));
    CK(d2ip_set_state(X, (int)i, st.data(), t, 0));
    CK(d2ip_reset_optimizer(X, (int)i));
    CK(d2ip_get_grad(X, (int)i, g.data(), P, 0));
    CK(d2ip_get_params(X, (int)i, g.data(), P, 0));
    const size_t V = (size_t)G[I[i].geometry].n * G[I[i].geometry].n * G[I[i].geometry].n;
    std::vector<float> img(V);
    CK(d2ip_read_image(X, (int)i, img.data(), 0));
    double ms = 0.0;
    for (int k = 0; k <= 5; ++k)
      for (int blk = 0; blk < 2; ++blk) {
        d2ip_status s = d2ip_time_kernel(X, (int)i, k, blk, 2, &ms);
        if (s != D2IP_OK && s != D2IP_EINVAL) {
          printf("FAIL time_kernel %d %d: %s\n", k, blk, d2ip_last_error());
          return 1;
        }
      }
  }
  CK(d2ip_run(X, 3, loss.data()));
  CK(d2ip_check_launches(G.data(), (int)G.size(), I.data(), (int)I.size(), prec, flags));
  CK(d2ip_destroy(X));
  emu_flush_all();  // the caller frees device memory after its stream has passed
  free(ws);
  printf("ok: %zu geometries, %zu instances, precision %d, flags %u\n", G.size(), I.size(), prec,
         flags);
  return 0;
}

// Standalone pass timing and the tuning table over every pass of one plan.
static int tuning_case() {
  const d2ip_geometry_desc G[1] = {{16, 208}};
  const d2ip_instance_desc I[1] = {{0, 3, 8}};
  int count = 0;
  CK(d2ip_plan_convs(G, 1, I, 1, D2IP_BF16X3_CONV, 0, 0, nullptr, 0, &count));
  std::vector<d2ip_tuning_entry> e(count);
  CK(d2ip_plan_convs(G, 1, I, 1, D2IP_BF16X3_CONV, 0, 0, e.data(), count, &count));
  for (const d2ip_tuning_entry& t : e) {
    size_t need = 0;
    CK(d2ip_time_conv_bytes(&t, &need));
    char* ws = (char*)aligned_alloc(256, (need + 255) / 256 * 256);
    double ms = 0.0;
    EXPECT_ERR(d2ip_time_conv(&t, ws, need - 1, nullptr, 2, &ms), D2IP_ENOMEM);
    CK(d2ip_time_conv(&t, ws, need, nullptr, 2, &ms));
    emu_flush_all();  // the caller frees device memory after its stream has passed
    free(ws);
  }
  CK(d2ip_set_tuning(e.data(), count));
  d2ip_tuning_entry bad = e[0];
  bad.shape.ck = 12;
  EXPECT_ERR(d2ip_set_tuning(&bad, 1), D2IP_EINVAL);
  CK(d2ip_check_launches(G, 1, I, 1, D2IP_BF16X3_CONV, 1));
  CK(d2ip_set_tuning(nullptr, 0));
  printf("ok: tuning, %d passes\n", count);
  return 0;
}

// The standalone operators on host-emulated buffers.
static int ops_case() {
  const int n = 8, cin = 16, cout = 24, C = 16, M = 40, Q = n * n * n;
  std::vector<float> x((size_t)Q * 32, 0.f), y((size_t)Q * 32), w((size_t)cout * cin * 27),
      b(cout), g((size_t)Q * 32), gx((size_t)Q * 32), gw(w.size()), gb(cout), gam(C, 1.f),
      bet(C), gs((size_t)Q * C), ggb(2 * C), J((size_t)M * Q), p(M), out(Q);
  for (int taps : {27, 1})
    for (int prec = 0; prec < 3; ++prec) {
      size_t need = 0;
      CK(d2ip_op_conv3d_bytes(n, cin, cout, taps, prec, &need));
      char* ws = (char*)aligned_alloc(256, (need + 255) / 256 * 256);
      std::vector<float> wt((size_t)cout * cin * taps);
      CK(d2ip_op_conv3d_forward(x.data(), wt.data(), b.data(), y.data(), n, cin, cout, taps, prec,
                                ws, need, nullptr));
      CK(d2ip_op_conv3d_backward(x.data(), wt.data(), g.data(), gx.data(), gw.data(), gb.data(), n,
                                 cin, cout, taps, prec, ws, need, nullptr));
      EXPECT_ERR(d2ip_op_conv3d_forward(x.data(), wt.data(), b.data(), y.data(), n, cin, cout,
                                        taps, prec, ws, need - 1, nullptr),
                 D2IP_ENOMEM);
      emu_flush_all();  // the caller frees device memory after its stream has passed
      free(ws);
    }
  size_t need = 0;
  EXPECT_ERR(d2ip_op_conv3d_bytes(n, 12, cout, 27, 0, &need), D2IP_EINVAL);
  CK(d2ip_op_ln_relu_bytes(n, C, &need));
  char* ws = (char*)aligned_alloc(256, (need + 255) / 256 * 256);
  CK(d2ip_op_ln_relu_forward(x.data(), gam.data(), bet.data(), nullptr, y.data(), n, C, ws, need,
                             nullptr));
  CK(d2ip_op_ln_relu_backward(x.data(), y.data(), gam.data(), g.data(), gx.data(), gs.data(),
                              ggb.data(), n, C, ws, need, nullptr));
  emu_flush_all();  // the caller frees device memory after its stream has passed
  free(ws);
  EXPECT_ERR(d2ip_op_ln_relu_bytes(n, 12, &need), D2IP_EINVAL);
  for (int Cd : {4, 8, 12, 16, 32}) {
    std::vector<float> wd((size_t)Cd * 27), bd(Cd), gwd(wd.size()), gbd(Cd);
    CK(d2ip_op_dwconv3d_bytes(n, Cd, &need));
    ws = (char*)aligned_alloc(256, (need + 255) / 256 * 256);
    CK(d2ip_op_dwconv3d_forward(x.data(), wd.data(), bd.data(), y.data(), n, Cd, nullptr));
    CK(d2ip_op_dwconv3d_backward(x.data(), wd.data(), g.data(), gx.data(), gwd.data(), gbd.data(),
                                 n, Cd, ws, need, nullptr));
    EXPECT_ERR(d2ip_op_dwconv3d_backward(x.data(), wd.data(), g.data(), gx.data(), gwd.data(),
                                         nullptr, n, Cd, ws, need - 1, nullptr),
               D2IP_ENOMEM);
    emu_flush_all();  // the caller frees device memory after its stream has passed
    free(ws);
  }
  EXPECT_ERR(d2ip_op_dwconv3d_bytes(n, 6, &need), D2IP_EINVAL);
  for (int dil : {1, 2, 5}) {
    std::vector<float> wd((size_t)16 * 27), bd(16), gwd(wd.size()), gbd(16);
    CK(d2ip_op_dwconv3d_dilated_bytes(n, 16, dil, &need));
    ws = (char*)aligned_alloc(256, (need + 255) / 256 * 256);
    CK(d2ip_op_dwconv3d_dilated_forward(x.data(), wd.data(), bd.data(), y.data(), n, 16, dil,
                                        nullptr));
    CK(d2ip_op_dwconv3d_dilated_backward(x.data(), wd.data(), g.data(), gx.data(), gwd.data(),
                                         gbd.data(), n, 16, dil, ws, need, nullptr));
    emu_flush_all();  // the caller frees device memory after its stream has passed
    free(ws);
  }
  EXPECT_ERR(d2ip_op_dwconv3d_dilated_bytes(n, 16, 0, &need), D2IP_EINVAL);
  for (int ci : {4, 16, 100})
    for (int co : {8, 64, 132}) {
      CK(d2ip_op_pwconv3d_bytes(n, ci, co, &need));
      ws = (char*)aligned_alloc(256, (need + 255) / 256 * 256);
      std::vector<float> wpw((size_t)ci * co), bpw(co), gwp(wpw.size()), gbp(co),
          ybig((size_t)Q * co), gbig((size_t)Q * co);
      CK(d2ip_op_pwconv3d_forward(x.data(), wpw.data(), bpw.data(), ybig.data(), n, ci, co,
                                  nullptr));
      CK(d2ip_op_pwconv3d_backward(x.data(), wpw.data(), gbig.data(), gx.data(), gwp.data(),
                                   gbp.data(), n, ci, co, ws, need, nullptr));
      EXPECT_ERR(d2ip_op_pwconv3d_backward(x.data(), wpw.data(), gbig.data(), nullptr,
                                           gwp.data(), nullptr, n, ci, co, ws, need - 1, nullptr),
                 D2IP_ENOMEM);
      emu_flush_all();  // the caller frees device memory after its stream has passed
      free(ws);
    }
  EXPECT_ERR(d2ip_op_pwconv3d_bytes(n, 6, 8, &need), D2IP_EINVAL);
  for (int Cs : {4, 12, 32})
    for (int Hs : {1, 3, 8}) {
      CK(d2ip_op_se_bytes(n, Cs, Hs, &need));
      ws = (char*)aligned_alloc(256, (need + 255) / 256 * 256);
      std::vector<float> a1((size_t)Hs * Cs), c1(Hs), a2((size_t)Cs * Hs), c2(Cs);
      std::vector<float> ga1(a1.size()), gc1(Hs), ga2(a2.size()), gc2(Cs);
      CK(d2ip_op_se_forward(x.data(), a1.data(), c1.data(), a2.data(), c2.data(), y.data(), n,
                            Cs, Hs, ws, need, nullptr));
      CK(d2ip_op_se_backward(x.data(), a1.data(), c1.data(), a2.data(), c2.data(), g.data(),
                             gx.data(), ga1.data(), gc1.data(), ga2.data(), gc2.data(), n, Cs, Hs,
                             ws, need, nullptr));
      EXPECT_ERR(d2ip_op_se_forward(x.data(), a1.data(), c1.data(), a2.data(), c2.data(),
                                    y.data(), n, Cs, Hs, ws, need - 1, nullptr),
                 D2IP_ENOMEM);
      emu_flush_all();  // the caller frees device memory after its stream has passed
      free(ws);
    }
  EXPECT_ERR(d2ip_op_se_bytes(n, 16, 0, &need), D2IP_EINVAL);
  // pooling, up-sampling + concatenation, channel copy, ReLU
  for (int Cp : {4, 16, 32}) {
    CK(d2ip_op_pool2_forward(x.data(), y.data(), n, Cp, nullptr));
    CK(d2ip_op_pool2_backward(g.data(), gx.data(), n, Cp, nullptr));
  }
  CK(d2ip_op_up2_concat_forward(x.data(), 16, g.data(), 16, n, y.data(), nullptr));
  CK(d2ip_op_up2_concat_backward(g.data(), 16, 16, n, gx.data(), y.data(), nullptr));
  CK(d2ip_op_channel_copy(x.data(), 32, 20, y.data(), 16, 4, 12, Q, nullptr));
  CK(d2ip_op_channel_copy(x.data(), 8, 0, y.data(), 32, 24, 8, Q, nullptr));
  CK(d2ip_op_relu_forward(x.data(), y.data(), (size_t)Q * 32, nullptr));
  CK(d2ip_op_relu_forward(y.data(), y.data(), (size_t)Q * 32, nullptr));
  CK(d2ip_op_relu_backward(y.data(), g.data(), gx.data(), (size_t)Q * 32, nullptr));
  // output head, linear and sigmoid, masked and not
  for (int Ch : {4, 16, 32})
    for (int sig : {0, 1}) {
      std::vector<float> wh(Ch), bh(1), gwh(Ch), gbh(1), mk(Q, 1.f);
      CK(d2ip_op_head_bytes(n, Ch, &need));
      ws = (char*)aligned_alloc(256, (need + 255) / 256 * 256);
      CK(d2ip_op_head_forward(x.data(), wh.data(), bh.data(), sig ? mk.data() : nullptr,
                              out.data(), n, Ch, sig, nullptr));
      CK(d2ip_op_head_backward(x.data(), wh.data(), bh.data(), sig ? nullptr : mk.data(),
                               out.data(), gx.data(), gwh.data(), gbh.data(), n, Ch, sig, ws,
                               need, nullptr));
      EXPECT_ERR(d2ip_op_head_backward(x.data(), wh.data(), bh.data(), nullptr, out.data(),
                                       nullptr, gwh.data(), nullptr, n, Ch, sig, ws, need - 1,
                                       nullptr),
                 D2IP_ENOMEM);
      emu_flush_all();  // the caller frees device memory after its stream has passed
      free(ws);
    }
  // attention unit: ragged last block at 6^3 and the widest channels
  for (auto [na, ca, cua] : {std::tuple{8, 8, 16}, std::tuple{6, 4, 8}, std::tuple{8, 64, 128},
                              std::tuple{4, 12, 4}, std::tuple{4, 128, 256},
                              std::tuple{6, 256, 512}}) {
    const size_t Va = (size_t)na * na * na, Vc = Va / 8;
    std::vector<float> xa(Va * ca), ga(Vc * cua), ya(Va * ca), al(Vc), gxa(Va * ca),
        gga(Vc * cua), wx((size_t)ca * ca), wg((size_t)ca * cua), ba(ca), ps(ca), bp(1),
        gwx(wx.size()), gwg(wg.size()), gba(ca), gps(ca), gbp(1);
    CK(d2ip_op_attention_bytes(na, ca, cua, &need));
    ws = (char*)aligned_alloc(256, (need + 255) / 256 * 256);
    CK(d2ip_op_attention_forward(xa.data(), ga.data(), wx.data(), wg.data(), ba.data(), ps.data(),
                                 bp.data(), ya.data(), al.data(), na, ca, cua, ws, need, nullptr));
    CK(d2ip_op_attention_backward(xa.data(), ga.data(), wx.data(), wg.data(), ba.data(),
                                  ps.data(), bp.data(), ya.data(), gxa.data(), gga.data(),
                                  gwx.data(), gwg.data(), gba.data(), gps.data(), gbp.data(), na,
                                  ca, cua, ws, need, nullptr));
    CK(d2ip_op_attention_backward(xa.data(), ga.data(), wx.data(), wg.data(), ba.data(),
                                  ps.data(), bp.data(), ya.data(), nullptr, nullptr, gwx.data(),
                                  nullptr, nullptr, nullptr, nullptr, na, ca, cua, ws, need,
                                  nullptr));
    EXPECT_ERR(d2ip_op_attention_backward(xa.data(), ga.data(), wx.data(), wg.data(), ba.data(),
                                          ps.data(), bp.data(), ya.data(), gxa.data(), nullptr,
                                          nullptr, nullptr, nullptr, nullptr, nullptr, na, ca, cua,
                                          ws, need - 1, nullptr),
               D2IP_ENOMEM);
    emu_flush_all();  // the caller frees device memory after its stream has passed
    free(ws);
  }
  EXPECT_ERR(d2ip_op_dwconv3d_forward(x.data() + 1, gam.data(), nullptr, y.data(), n, C, nullptr),
             D2IP_EINVAL);
  CK(d2ip_op_j_forward(J.data(), x.data(), p.data(), M, Q, nullptr));
  CK(d2ip_op_jt_bytes(M, Q, &need));
  ws = (char*)aligned_alloc(256, (need + 255) / 256 * 256);
  CK(d2ip_op_jt(J.data(), p.data(), out.data(), M, Q, ws, need, nullptr));
  CK(d2ip_op_jt_noalloc(J.data(), p.data(), out.data(), M, Q, nullptr));
  EXPECT_ERR(d2ip_op_jt_noalloc(J.data(), p.data(), out.data(), M, 64 * 64 * 64 + 4, nullptr),
             D2IP_EINVAL);
  emu_flush_all();  // the caller frees device memory after its stream has passed
  free(ws);
  printf("ok: standalone operators\n");
  return 0;
}


// ---------------------------------------------------------------------------
// The benchmark's C-ABI call sequence, replayed on the emulation: each
// workload's context created, loaded from host arrays, run (warm-up with a
// loss read, timed iterations without, a final loss read), its image read and
// the context destroyed, one context after another, in the order and with the
// shapes the benchmark uses; the kernel table of the chosen form; the
// multi-instance workloads.
// ---------------------------------------------------------------------------
struct Problem {
  int n, M;
  std::vector<float> J, z, dv;
  std::vector<uint8_t> mask;
};

static Problem make_problem(int n, int M, unsigned seed) {
  Problem p;
  p.n = n;
  p.M = M;
  const size_t Q = (size_t)n * n * n;
  std::mt19937 rng(seed);
  std::normal_distribution<float> nd;
  p.J.resize((size_t)M * Q);
  for (float& v : p.J) v = nd(rng);
  p.mask.resize(Q);
  for (int z = 0; z < n; ++z)
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        const double cx = -1.0 + (2.0 * x + 1.0) / n, cy = -1.0 + (2.0 * y + 1.0) / n;
        p.mask[((size_t)z * n + y) * n + x] = cx * cx + cy * cy <= 1.0;
      }
  p.z.resize(Q);
  for (float& v : p.z) v = nd(rng);
  p.dv.resize(M);
  for (float& v : p.dv) v = 0.01f * nd(rng);
  return p;
}

static int load_instance(d2ip_ctx* X, int inst, const Problem& p, int levels, int C, bool geo,
                         int geo_index, unsigned seed) {
  if (geo) CK(d2ip_set_geometry(X, geo_index, p.J.data(), p.mask.data(), 0));
  size_t P = 0;
  CK(d2ip_param_count(levels, C, &P));
  std::vector<float> th(P);
  std::mt19937 rng(seed);
  std::normal_distribution<float> nd;
  for (float& v : th) v = 0.05f * nd(rng);
  CK(d2ip_set_params(X, inst, th.data(), P, 0));
  CK(d2ip_set_noise_input(X, inst, p.z.data(), 0));
  CK(d2ip_set_frame(X, inst, p.dv.data(), 0));
  return 0;
}

// One single-instance workload as the benchmark times it.
static int single_form(const Problem& p, int levels, int C, int prec, unsigned flags, int steps,
                       int warmup, bool tv, bool kernels) {
  const d2ip_geometry_desc G[1] = {{p.n, p.M}};
  const d2ip_instance_desc I[1] = {{0, levels, C}};
  size_t need = 0;
  CK(d2ip_workspace_bytes(G, 1, I, 1, prec, flags, &need));
  char* ws = (char*)aligned_alloc(256, (need + 255) / 256 * 256);
  d2ip_ctx* X = nullptr;
  CK(d2ip_create(G, 1, I, 1, prec, flags, ws, need, nullptr, &X));
  if (load_instance(X, 0, p, levels, C, true, 0, 7)) return 1;
  d2ip_adam_cfg cfg = {1e-3f, 0.9f, 0.999f, 1e-8f};
  CK(d2ip_set_adam(X, &cfg));
  if (tv) {
    d2ip_tv_cfg t = {0.002f, 1.f, 0.1f, 1e-8f};
    CK(d2ip_set_tv(X, &t));
  }
  double loss = 0.0;
  CK(d2ip_run(X, warmup, &loss));
  CK(d2ip_run(X, steps, nullptr));
  CK(d2ip_run(X, 0, &loss));
  std::vector<float> img((size_t)p.n * p.n * p.n);
  CK(d2ip_read_image(X, 0, img.data(), 0));
  if (kernels) {
    double ms = 0.0;
    CK(d2ip_time_kernel(X, 0, D2IP_KERNEL_JVEC, 0, 50, &ms));
    CK(d2ip_time_kernel(X, 0, D2IP_KERNEL_JTVEC, 0, 50, &ms));
    const int nblocks = 2 * levels - 1;
    for (int b = 0; b < nblocks; ++b)
      for (int k = D2IP_KERNEL_CONV_FWD; k <= D2IP_KERNEL_CONV_WGRAD; ++k)
        CK(d2ip_time_kernel(X, 0, k, b, 20, &ms));
    CK(d2ip_time_kernel(X, 0, D2IP_KERNEL_ADAM, 0, 50, &ms));
  }
  CK(d2ip_destroy(X));
  emu_flush_all();  // the caller frees device memory after its stream has passed
  free(ws);
  return 0;
}

// Several instances in one context (sequences with frame transitions, or
// uneven instances), as the benchmark's multi-instance workloads run them.
static int multi(const std::vector<Problem*>& geos, const std::vector<d2ip_instance_desc>& I,
                 int prec, unsigned flags, int first, int later, int frames) {
  std::vector<d2ip_geometry_desc> G;
  for (const Problem* p : geos) G.push_back({p->n, p->M});
  size_t need = 0;
  CK(d2ip_workspace_bytes(G.data(), (int)G.size(), I.data(), (int)I.size(), prec, flags, &need));
  char* ws = (char*)aligned_alloc(256, (need + 255) / 256 * 256);
  d2ip_ctx* X = nullptr;
  CK(d2ip_create(G.data(), (int)G.size(), I.data(), (int)I.size(), prec, flags, ws, need, nullptr,
                 &X));
  std::vector<char> done(G.size(), 0);
  for (size_t i = 0; i < I.size(); ++i) {
    const int g = I[i].geometry;
    if (load_instance(X, (int)i, *geos[g], I[i].levels, I[i].base_ch, !done[g], g,
                      100 + (unsigned)i))
      return 1;
    done[g] = 1;
  }
  d2ip_adam_cfg cfg = {1e-3f, 0.9f, 0.999f, 1e-8f};
  CK(d2ip_set_adam(X, &cfg));
  CK(d2ip_run(X, first, nullptr));
  for (int f = 0; f < frames; ++f) {
    for (size_t i = 0; i < I.size(); ++i) {
      CK(d2ip_set_frame(X, (int)i, geos[I[i].geometry]->dv.data(), 0));
      CK(d2ip_reset_optimizer(X, (int)i));
    }
    CK(d2ip_run(X, later, nullptr));
  }
  std::vector<double> loss(I.size());
  CK(d2ip_run(X, 0, loss.data()));
  CK(d2ip_destroy(X));
  emu_flush_all();  // the caller frees device memory after its stream has passed
  free(ws);
  return 0;
}

static int bench_sequence(bool large) {
  Problem c1 = make_problem(32, 928, 1), c0 = make_problem(16, 208, 0);
  const int steps = 20, warmup = 5;
  for (int prec : {0, 2, 1})
    for (unsigned fl : {1u, 0u})
      if (single_form(c1, 3, 16, prec, fl, steps, warmup, false, false)) return 1;
  if (single_form(c1, 3, 16, 0, 0, steps, warmup, false, false)) return 1;  // plain
  if (single_form(c1, 3, 16, 0, 0, steps, warmup, true, false)) return 1;   // 4D-TV
  if (single_form(c1, 3, 16, 0, 0, 0, warmup, false, true)) return 1;       // kernel table
  for (int prec : {0, 1})
    for (unsigned fl : {1u, 0u})
      if (single_form(c0, 2, 8, prec, fl, 50, 0, false, false)) return 1;
  if (large) {
    Problem c2 = make_problem(64, 928, 2);
    for (int prec : {0, 1})
      for (unsigned fl : {1u, 0u})
        if (single_form(c2, 4, 32, prec, fl, 40, 3, false, fl == 0)) return 1;
  }
  // eight sequences of the 32^3 workload: first frame, then frames with TPP
  std::vector<d2ip_instance_desc> seq(8, d2ip_instance_desc{0, 3, 16});
  for (int prec : {0, 1})
    for (unsigned fl : {1u, 0u})
      if (multi({&c1}, seq, prec, fl, 20, 5, 3)) return 1;
  // sixteen uneven instances
  Problem g24a = make_problem(24, 208, 3), g32a = make_problem(32, 208, 4),
          g48a = make_problem(48, 208, 5), g24b = make_problem(24, 928, 6),
          g48b = make_problem(48, 928, 8);
  std::vector<Problem*> geos = {&g24a, &g32a, &g48a, &g24b, &c1, &g48b};
  std::vector<d2ip_instance_desc> un;
  for (int i = 0; i < 16; ++i) {
    const int g = (i % 3) + 3 * ((i / 3) % 2);
    un.push_back({g, 3, ((i / 6) % 2) ? 16 : 8});
  }
  for (int prec : {0, 1})
    for (unsigned fl : {1u, 0u})
      if (multi(geos, un, prec, fl, 2, 3, 1)) return 1;
  printf("ok: benchmark call sequence\n");
  return 0;
}

// The module-network context (every module mix) on host-emulated buffers.
static int mnet_case() {
  const int n = 8, M = 40;
  const size_t Q = (size_t)n * n * n;
  std::vector<float> J((size_t)M * Q, 0.01f), z(Q, 0.5f), dv(M, 0.1f), img(Q);
  std::vector<uint8_t> mask(Q, 1);
  int mixes[][5] = {{0, 0, 0, 0, 0}, {1, 0, 0, 0, 0}, {0, 4, 0, 0, 0}, {0, 0, 1, 1, 0},
                    {0, 0, 0, 0, 1}, {1, 4, 1, 1, 1}};
  for (auto& mx : mixes)
    for (int levels : {2, 3})
      for (int graph : {0, 1}) {
      d2ip_mnet_desc d{n, M, levels, 8, mx[0], mx[1], mx[2], mx[3], mx[4], graph};
      size_t bytes = 0, P = 0;
      CK(d2ip_mnet_workspace_bytes(&d, &bytes));
      CK(d2ip_mnet_param_count(&d, &P));
      char* ws = (char*)aligned_alloc(256, (bytes + 255) / 256 * 256);
      d2ip_mnet* net = nullptr;
      EXPECT_ERR(d2ip_mnet_create(&d, ws, bytes - 1, nullptr, &net), D2IP_ENOMEM);
      CK(d2ip_mnet_create(&d, ws, bytes, nullptr, &net));
      EXPECT_ERR(d2ip_mnet_run(net, 1, nullptr), D2IP_ESTATE);
      std::vector<float> th(P, 0.01f), g(P);
      CK(d2ip_mnet_set_problem(net, J.data(), mask.data(), z.data(), 0));
      CK(d2ip_mnet_set_params(net, th.data(), P, 0));
      EXPECT_ERR(d2ip_mnet_set_params(net, th.data(), P + 1, 0), D2IP_EINVAL);
      CK(d2ip_mnet_set_frame(net, dv.data(), 0));
      d2ip_adam_cfg cfg{1e-3f, 0.9f, 0.999f, 1e-8f};
      CK(d2ip_mnet_set_adam(net, &cfg));
      double loss = -1.0;
      CK(d2ip_mnet_run(net, 2, &loss));
      CK(d2ip_mnet_get_params(net, th.data(), P, 0));
      CK(d2ip_mnet_get_grad(net, g.data(), P, 0));
      CK(d2ip_mnet_read_image(net, img.data(), 0));
      CK(d2ip_mnet_set_frame(net, dv.data(), 0));
      CK(d2ip_mnet_reset_optimizer(net));
      CK(d2ip_mnet_run(net, 1, nullptr));
      CK(d2ip_mnet_set_adam(net, &cfg));  // discards a captured graph
      CK(d2ip_mnet_run(net, 2, &loss));
      CK(d2ip_mnet_destroy(net));
      emu_flush_all();
      free(ws);
      }
  printf("ok: module networks\n");
  return 0;
}

int main(int argc, char** argv) {
  if (argc > 1 && std::string(argv[1]) == "bench") {
    int bad = bench_sequence(argc > 2 && std::string(argv[2]) == "large");
    emu_flush_all();
    printf("launches: %ld (captured %ld), emulation errors: %ld\n", g_launches,
           g_captured_launches, emu_errors());
    return bad || emu_errors() != 0;
  }
  int bad = tuning_case() | ops_case() | mnet_case();
  for (int prec = 0; prec < 3; ++prec)
    for (unsigned fl = 0; fl < 2; ++fl) {
      bad |= run_case({{16, 928}}, {{0, 3, 8}, {0, 3, 8}, {0, 3, 8}}, prec, fl);
      bad |= run_case({{16, 208}, {24, 208}}, {{0, 2, 8}, {0, 2, 16}, {1, 3, 8}, {0, 2, 8}}, prec,
                      fl);
      bad |= run_case({{16, 208}}, {{0, 2, 8}}, prec, fl);
    }
  emu_flush_all();
  printf("launches: %ld (captured %ld), emulation errors: %ld\n", g_launches,
         g_captured_launches, emu_errors());
  return bad || emu_errors() != 0;
}
