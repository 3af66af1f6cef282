// Context, workspace plan, per-iteration launch schedule and the C-ABI of the
// D2IP fitting library.  One context holds geometries (compacted J, mask) and
// instances (network parameters, Adam state, activations); every launch goes
// to the context's stream, and with D2IP_FLAG_GRAPH one iteration of all
// instances is captured once into a hipGraph and replayed.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "d2ip.h"
#include "kernels.h"

using namespace d2ip;

namespace {

thread_local std::string g_err;

d2ip_status fail(d2ip_status s, const std::string& m) {
  g_err = m;
  return s;
}

#define HIPCHK(expr)                                                                 \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(D2IP_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)


// ---------------------------------------------------------------------------
// Launch-extent checker (host only).  With a checker active, the workspace is
// planned at a fake base address, every carved allocation is recorded, and the
// launch schedule is walked without launching: each pointer argument's byte
// extent, implied by the kernel's shapes, must lie inside one allocation for
// every member of its instance group.
// ---------------------------------------------------------------------------
struct Checker {
  struct Alloc {
    uintptr_t lo, hi;
  };
  std::vector<Alloc> allocs;
  std::vector<std::string> errors;
  const char* where = "";
  void add(const void* p, size_t bytes) {
    allocs.push_back({(uintptr_t)p, (uintptr_t)p + bytes});
  }
  bool inside(uintptr_t lo, uintptr_t hi) const {
    for (const Alloc& a : allocs)
      if (lo >= a.lo && hi <= a.hi) return true;
    return false;
  }
  // [p + b*istride, + bytes) for members b < B must each fit one allocation
  void range(const void* p, size_t bytes, const char* what, int B = 1, long long istride = 0) {
    if (!p || bytes == 0) return;
    for (int b = 0; b < B; ++b) {
      const uintptr_t lo = (uintptr_t)p + (uintptr_t)(b * istride);
      if (!inside(lo, lo + bytes) && errors.size() < 20)
        errors.push_back(std::string(where) + ": " + what + " (member " + std::to_string(b) +
                         ", " + std::to_string(bytes) + " bytes) outside every allocation");
    }
  }
  void require(bool ok, const std::string& what) {
    if (!ok && errors.size() < 20) errors.push_back(std::string(where) + ": " + what);
  }
};
thread_local Checker* g_chk = nullptr;

constexpr bool kGroupInstances = false;

struct Carver {
  char* base = nullptr;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    if (g_chk && p) g_chk->add(p, count * sizeof(T));
    return p;
  }
};

// Launch shape of one conv role (forward or input gradient).
struct Shape {
  int tile = TILE_2x4x16, bn = 16, ck = 8, ksplit = 1;
};

struct Conv {
  int th_w = -1, th_b = -1;
  int cin_real = 0, cin = 0, cout = 0, taps = 0;
  long long wf = 0, wd = 0;
  bool dgrad = false;
  int n = 0;
  Shape fwd, bwd;          // forward / input-gradient launch shapes
  int pro_fwd = PRO_NONE, pro_bwd = PRO_NONE, pro_wg = 0;  // fused operand transforms
  int wg_tile = 0, wg_ck = 8, wg_splits = 1;
  long long wg_off = 0, wgb_off = 0;  // partial regions of the weight gradient
};

struct Norm {
  int th_g = -1, th_b = -1;
};

struct Block {
  bool enc = true;
  int level = 0, n = 0, cin = 0, cout = 0;
  bool proj = false;
  Conv c1, c2, pj;
  Norm n1, n2;
  float *x = nullptr, *h1 = nullptr, *h2 = nullptr, *s = nullptr, *y = nullptr;
  float* pool_out = nullptr;        // encoder l < L-1: input of encoder l+1
  const float* up_src = nullptr;    // decoder: output of the level below
  const float* skip_src = nullptr;  // decoder: output of encoder l
  float *gz = nullptr, *ga = nullptr;  // this block's LayerNorm-backward gradients
  float* gpj = nullptr;  // input gradient of the 1x1 projection (side stream)
  PairRef st1{}, st2{};         // forward statistics partials of h1, h2
  PairRef cb1{}, cb2{};         // LayerNorm-backward coefficient partials
  double *lnc1 = nullptr, *lnc2 = nullptr;  // per-channel dgamma/dbeta partials
};

struct Level {
  int n = 0, c = 0;
  size_t V = 0;
  float *gy = nullptr, *gz = nullptr, *ga = nullptr, *gx = nullptr, *genc = nullptr;
};

struct Geometry {
  int n = 0, M = 0;
  size_t Q = 0;
  int qa = 0, qa_pad = 0, qa_cap = 0;
  float* Jc = nullptr;
  int* idx = nullptr;
  int* inv = nullptr;
  float* mask = nullptr;
  bool set = false;
};

struct Instance {
  int geo = 0, L = 0, C = 0, n = 0;
  size_t V0 = 0, P = 0;
  float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  float* wf32 = nullptr;
  uint16_t* wbf16 = nullptr;
  long long wtotal = 0;
  std::vector<ConvPack> packs;
  ConvPack* packs_dev = nullptr;
  int max_pack = 0;
  std::vector<GradSeg> segs;
  GradSeg* segs_dev = nullptr;
  int max_seg = 0;
  float *wg_part = nullptr, *wg_partb = nullptr;
  long long wg_total = 0, wgb_total = 0;
  float* zpad = nullptr;
  Conv stem;
  Norm stem_n;
  float *hs = nullptr, *as = nullptr;
  PairRef sts{}, cbs{};
  double* lncs = nullptr;
  std::vector<Block> blocks;
  int tail_w = -1, tail_b = -1;
  float *sigma = nullptr, *dv = nullptr;
  IterState* it = nullptr;
  std::vector<Level> lv;
  double* dpart = nullptr;   // FP64 partial arena (statistics, LN and head gradients)
  long long dtotal = 0;
  float *ppart = nullptr, *tpart = nullptr;
  double* tail_part = nullptr;
  double* rsum = nullptr;
  float* kpart = nullptr;   // split-K partial outputs
  // 4D-TV: gradient w.r.t. the image, per-block loss partials, image history
  float *gtv = nullptr, *hist = nullptr;
  double* tvsum = nullptr;
  TvState* tvs = nullptr;
  std::vector<int> tv_count, tv_head;  // host mirror per member
  // group: B members of identical shape; member b's data is b * istride
  // bytes after member 0's (every pointer above is member 0's)
  int B = 1;
  long long istride = 0;
  std::vector<int> member_inst;  // API instance index of each member
  std::vector<char> has_frame, has_z;
};

int conv_prec(int precision) {
  if (precision == D2IP_BF16_CONV) return PREC_BF16;
  if (precision == D2IP_BF16X3_CONV) return PREC_BF16X3;
  return PREC_F32;
}

int pick_tile(int n) {
  if (n % 16 == 0) return n >= 32 ? TILE_2x4x16 : TILE_1x4x16;
  return TILE_1x8x8;
}

int largest_ck(int cin) { return cin % 32 == 0 ? 32 : cin % 16 == 0 ? 16 : 8; }

constexpr int kTargetBlocks = 256;
constexpr size_t kLdsBudget = 60 * 1024;  // dynamic LDS per block (static use stays small)

// Enough blocks to cover the chip: narrow N tiles and channel split-K on
// coarse grids, wide N tiles and whole-channel chunks on fine ones; the halo
// plus weight slab must fit the LDS budget (two blocks per CU).
Shape choose_shape(int n, int cin, int cout, int taps, int prec) {
  Shape s;
  s.tile = pick_tile(n);
  s.bn = cout <= 16 ? 16 : cout <= 32 ? 32 : 64;
  if (s.tile == TILE_2x4x16 && s.bn > 32) s.bn = 32;  // <= 16 accumulator tiles per wave
  const int tiles = conv_tiles(n, s.tile);
  auto blocks = [&](int bn) { return tiles * ((cout + bn - 1) / bn); };
  if (blocks(s.bn) < kTargetBlocks) s.bn = 16;
  s.ck = largest_ck(cin);
  while (conv_fwd_lds_bytes(s.tile, taps, s.bn, s.ck, prec) > kLdsBudget) {
    if (s.ck > 8)
      s.ck >>= 1;
    else if (s.bn > 16)
      s.bn >>= 1;
    else
      break;
  }
  const int base = blocks(s.bn);
  if (base < kTargetBlocks) {
    const int want = (kTargetBlocks + base - 1) / base;
    while (s.ck > 8 && cin / s.ck < want) s.ck >>= 1;
    const int nch = cin / s.ck;
    int ks = std::min(want, nch);
    while (nch % ks != 0) --ks;
    s.ksplit = ks;
  }
  return s;
}

d2ip_status check_desc(const d2ip_geometry_desc* geos, int n_geo, const d2ip_instance_desc* insts,
                       int n_inst, int precision) {
  if (!geos || n_geo <= 0 || !insts || n_inst <= 0)
    return fail(D2IP_EINVAL, "empty geometry or instance list");
  if (precision != D2IP_PLAIN_FP32 && precision != D2IP_BF16_CONV &&
      precision != D2IP_BF16X3_CONV)
    return fail(D2IP_EINVAL, "unknown precision");
  for (int g = 0; g < n_geo; ++g) {
    if (geos[g].n < 4 || geos[g].n > 256 || geos[g].M <= 0 || geos[g].M > 65536)
      return fail(D2IP_EINVAL,
                  "geometry " + std::to_string(g) + ": n must be in [4, 256], M in [1, 65536]");
  }
  for (int i = 0; i < n_inst; ++i) {
    const d2ip_instance_desc& d = insts[i];
    if (d.geometry < 0 || d.geometry >= n_geo)
      return fail(D2IP_EINVAL, "instance " + std::to_string(i) + ": bad geometry index");
    if (d.levels < 2 || d.levels > 5)
      return fail(D2IP_EINVAL, "instance " + std::to_string(i) + ": levels must be 2..5");
    if (d.base_ch != 8 && d.base_ch != 16 && d.base_ch != 32)
      return fail(D2IP_EINVAL, "instance " + std::to_string(i) + ": base_ch must be 8, 16 or 32");
    if (d.base_ch << (d.levels - 1) > 256)
      return fail(D2IP_EINVAL, "instance " + std::to_string(i) + ": base_ch * 2^(levels-1) > 256");
    const int n = geos[d.geometry].n, f = 1 << (d.levels - 1);
    if (n % f != 0 || n / f < 2)
      return fail(D2IP_EINVAL,
                  "instance " + std::to_string(i) + ": grid not divisible by 2^(levels-1)");
  }
  return D2IP_OK;
}

// Parameter offsets of one network in the flat order.
struct LayoutBuilder {
  int off = 0;
  Conv conv(int cout, int cin, int k, int n) {
    Conv c;
    c.th_w = off;
    off += cout * cin * k * k * k;
    c.th_b = off;
    off += cout;
    c.cout = cout;
    c.cin_real = cin;
    c.cin = (cin + 7) / 8 * 8;
    c.taps = k * k * k;
    c.dgrad = true;
    c.n = n;
    return c;
  }
  Norm norm(int c) {
    Norm nm;
    nm.th_g = off;
    off += c;
    nm.th_b = off;
    off += c;
    return nm;
  }
};

void make_block(LayoutBuilder& lb, Block& b, int cin, int cout) {
  b.cin = cin;
  b.cout = cout;
  b.c1 = lb.conv(cout, cin, 3, b.n);
  b.n1 = lb.norm(cout);
  b.c2 = lb.conv(cout, cout, 3, b.n);
  b.n2 = lb.norm(cout);
  b.proj = cin != cout;
  if (b.proj) b.pj = lb.conv(cout, cin, 1, b.n);
}

size_t layout(Instance& I) {
  LayoutBuilder lb;
  const int C = I.C, L = I.L;
  I.stem = lb.conv(C, 1, 3, I.n);
  I.stem.dgrad = false;
  I.stem_n = lb.norm(C);
  I.blocks.clear();
  for (int l = 0; l < L; ++l) {
    Block b;
    b.enc = true;
    b.level = l;
    b.n = I.n >> l;
    make_block(lb, b, l == 0 ? C : (C << (l - 1)), C << l);
    I.blocks.push_back(b);
  }
  for (int l = L - 2; l >= 0; --l) {
    Block b;
    b.enc = false;
    b.level = l;
    b.n = I.n >> l;
    make_block(lb, b, (C << (l + 1)) + (C << l), C << l);
    I.blocks.push_back(b);
  }
  Conv t = lb.conv(1, C, 1, I.n);
  I.tail_w = t.th_w;
  I.tail_b = t.th_b;
  return (size_t)lb.off;
}

// Process-wide table of tuned launch shapes, consulted by every later plan.
std::vector<d2ip_tuning_entry> g_tuning;

// Whether `e` describes a launch the kernels support; the reason if not.
bool shape_ok(const d2ip_tuning_entry& e, std::string* why) {
  auto no = [&](const char* m) {
    if (why) *why = m;
    return false;
  };
  const d2ip_conv_shape& sh = e.shape;
  if (e.n < 1 || e.n > 256) return no("n must be in [1, 256]");
  if (e.taps != 27 && e.taps != 1) return no("taps must be 27 or 1");
  if (e.cin < 8 || e.cout < 1 || e.cin > 1024 || e.cout > 1024) return no("bad channel counts");
  if (e.precision < D2IP_PLAIN_FP32 || e.precision > D2IP_BF16X3_CONV) return no("bad precision");
  if (sh.tile < TILE_2x4x16 || sh.tile > TILE_1x8x8) return no("tile must be 0, 1 or 2");
  if (sh.ck != 8 && sh.ck != 16 && sh.ck != 32) return no("ck must be 8, 16 or 32");
  const int prec = conv_prec(e.precision);
  if (e.pass == 0 || e.pass == 1) {
    const int kin = e.pass == 0 ? e.cin : e.cout;
    if (kin % sh.ck != 0) return no("ck must divide the pass's input channels");
    if (sh.bn != 16 && sh.bn != 32 && sh.bn != 64) return no("bn must be 16, 32 or 64");
    if (sh.tile == TILE_2x4x16 && sh.bn == 64) return no("the 2x4x16 tile takes bn <= 32");
    if (sh.split < 1 || (kin / sh.ck) % sh.split != 0)
      return no("split must divide the number of channel chunks");
    if (e.taps == 1 && sh.split != 1)
      return no("1x1 convs run on the side stream without split-K");
    const bool pro_ok = e.pass == 0 ? (e.prologue == PRO_NONE || e.prologue == PRO_LN_RELU)
                                    : (e.prologue == PRO_NONE || e.prologue == PRO_LN_BWD);
    if (!pro_ok || (e.taps == 1 && e.prologue != PRO_NONE)) return no("bad prologue");
    if (conv_fwd_lds_bytes(sh.tile, e.taps, sh.bn, sh.ck, prec) > kLdsBudget)
      return no("LDS over budget");
    return true;
  }
  if (e.pass == 2) {
    if (e.cin % sh.ck != 0) return no("ck must divide the input channels");
    if (sh.split < 1 || sh.split > 256 || sh.split > conv_tiles(e.n, sh.tile))
      return no("split must be in [1, min(256, voxel tiles)]");
    const int xp = e.prologue / 3, gp = e.prologue % 3;
    if (e.prologue < 0 || xp > PRO_LN_RELU || (gp != PRO_NONE && gp != PRO_LN_BWD) ||
        (e.taps == 1 && e.prologue != 0))
      return no("bad prologue");
    if (conv_wgrad_lds_bytes(sh.tile, e.taps, sh.ck, prec) > kLdsBudget)
      return no("LDS over budget");
    return true;
  }
  return no("pass must be 0, 1 or 2");
}

const d2ip_tuning_entry* find_tuned(int n, int cin, int cout, int taps, int pass, int pro,
                                    int precision) {
  for (const d2ip_tuning_entry& e : g_tuning)
    if (e.n == n && e.cin == cin && e.cout == cout && e.taps == taps && e.pass == pass &&
        e.prologue == pro && e.precision == precision)
      return &e;
  return nullptr;
}

// Launch shapes, packing table and weight-gradient partial regions of a conv.
void add_conv(Instance& I, Conv& c, int precision, size_t& kpart_max) {
  const int prec = conv_prec(precision);
  c.wf = I.wtotal;
  I.wtotal += (long long)c.cout * c.taps * c.cin;
  if (c.dgrad) {
    c.wd = I.wtotal;
    I.wtotal += (long long)c.cin_real * c.taps * c.cout;
  }
  ConvPack p;
  p.th_off = c.th_w;
  p.cout = c.cout;
  p.cin_real = c.cin_real;
  p.cin = c.cin;
  p.taps = c.taps;
  p.need_dgrad = c.dgrad ? 1 : 0;
  p.wf_off = c.wf;
  p.wd_off = c.wd;
  I.packs.push_back(p);
  I.max_pack = std::max(I.max_pack, c.cout * c.cin_real * c.taps);

  const size_t V = (size_t)c.n * c.n * c.n;
  c.fwd = choose_shape(c.n, c.cin, c.cout, c.taps, prec);
  // 1x1 projections run forward on the side stream, concurrently with split-K
  // convs of the main stream: they must not share the split-K scratch
  if (c.taps == 1) c.fwd.ksplit = 1;
  if (const d2ip_tuning_entry* t = find_tuned(c.n, c.cin, c.cout, c.taps, 0, c.pro_fwd, precision)) {
    c.fwd.tile = t->shape.tile;
    c.fwd.bn = t->shape.bn;
    c.fwd.ck = t->shape.ck;
    c.fwd.ksplit = t->shape.split;
  }
  if (c.fwd.ksplit > 1) kpart_max = std::max(kpart_max, (size_t)c.fwd.ksplit * V * c.cout);
  if (c.dgrad) {
    c.bwd = choose_shape(c.n, c.cout, c.cin_real, c.taps, prec);
    // a 1x1 projection's input gradient runs on the side stream too
    if (c.taps == 1) c.bwd.ksplit = 1;
    if (const d2ip_tuning_entry* t =
            find_tuned(c.n, c.cin, c.cout, c.taps, 1, c.pro_bwd, precision)) {
      c.bwd.tile = t->shape.tile;
      c.bwd.bn = t->shape.bn;
      c.bwd.ck = t->shape.ck;
      c.bwd.ksplit = t->shape.split;
    }
    if (c.bwd.ksplit > 1) kpart_max = std::max(kpart_max, (size_t)c.bwd.ksplit * V * c.cin_real);
  }
  // weight gradient: voxel splits sized so that about 512 blocks run
  c.wg_tile = pick_tile(c.n);
  c.wg_ck = largest_ck(c.cin);
  while (c.wg_ck > 8 && conv_wgrad_lds_bytes(c.wg_tile, c.taps, c.wg_ck, prec) > kLdsBudget)
    c.wg_ck >>= 1;
  const int cout16 = (c.cout + 15) / 16 * 16;
  const int per = (c.cin / c.wg_ck) * conv_wgrad_groups(c.taps, c.wg_ck) * (cout16 / 16);
  const int tiles = conv_tiles(c.n, c.wg_tile);
  c.wg_splits = std::max(1, std::min(std::min(tiles, 64), (512 + per - 1) / per));  // ~512 blocks
  if (const d2ip_tuning_entry* t = find_tuned(c.n, c.cin, c.cout, c.taps, 2, c.pro_wg, precision)) {
    c.wg_tile = t->shape.tile;
    c.wg_ck = t->shape.ck;
    c.wg_splits = t->shape.split;
  }
  c.wg_off = I.wg_total;
  I.wg_total += (long long)c.wg_splits * cout16 * c.taps * c.cin;
  c.wgb_off = I.wgb_total;
  I.wgb_total += (long long)c.wg_splits * cout16;
  GradSeg sg;
  sg.kind = 0;
  sg.part_off = c.wg_off;
  sg.partb_off = c.wgb_off;
  sg.splits = c.wg_splits;
  sg.cout = c.cout;
  sg.taps = c.taps;
  sg.cin = c.cin;
  sg.cin_real = c.cin_real;
  sg.th_w = c.th_w;
  sg.th_b = c.th_b;
  I.segs.push_back(sg);
  I.max_seg = std::max(I.max_seg, c.cout * c.cin_real * c.taps);
}

}  // namespace

namespace d2ip {
d2ip_status api_fail(d2ip_status s, const std::string& m) { return fail(s, m); }

void default_conv_shape(int n, int cin, int cout, int taps, int prec, int* tile, int* bn, int* ck,
                        int* ksplit) {
  const Shape sh = choose_shape(n, cin, cout, taps, prec);
  *tile = sh.tile;
  *bn = sh.bn;
  *ck = sh.ck;
  *ksplit = sh.ksplit;
}

int default_wgrad_splits(int n, int cin, int cout, int taps, int tile, int ck) {
  const int cout16 = (cout + 15) / 16 * 16;
  const int per = (cin / ck) * conv_wgrad_groups(taps, ck) * (cout16 / 16);
  const int tiles = conv_tiles(n, tile);
  return std::max(1, std::min(std::min(tiles, 64), (512 + per - 1) / per));
}

int default_tile(int n) { return pick_tile(n); }
int default_ck(int cin) { return largest_ck(cin); }
}  // namespace d2ip

struct d2ip_ctx {
  int precision = D2IP_PLAIN_FP32;
  unsigned flags = 0;
  hipStream_t stream = nullptr;
  std::vector<Geometry> geos;
  std::vector<Instance> insts;              // instance groups
  std::vector<std::pair<int, int>> members;  // API instance -> (group, member)
  float lr = 1e-3f, b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  bool tv_on = false;
  TvCoef tv{0.002f, 1.f, 0.1f, 1e-8f};
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap = nullptr;  // capture stream (the caller's may be the legacy default stream)
  hipStream_t side = nullptr;  // branch for work off the critical path (weight gradients)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_pj = nullptr;  // a projection's input gradient, done on the side stream
  // instance groups run concurrently, each on one of a few lanes (a main and
  // a side stream) forked from and joined back into the context stream
  struct Lane {
    hipStream_t main = nullptr, side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr, done = nullptr, pj = nullptr;
  };
  std::vector<Lane> lanes;
  hipEvent_t ev_start = nullptr;
  size_t bytes = 0;
};

namespace {

// Carve the workspace (base == nullptr: only count bytes).
void plan(d2ip_ctx& X, const d2ip_geometry_desc* gd, int n_geo, const d2ip_instance_desc* id,
          int n_inst, Carver& cv) {
  X.geos.assign(n_geo, Geometry());
  for (int g = 0; g < n_geo; ++g) {
    Geometry& G = X.geos[g];
    G.n = gd[g].n;
    G.M = gd[g].M;
    G.Q = (size_t)G.n * G.n * G.n;
    G.qa_cap = (int)((G.Q + 63) / 64 * 64);
    G.Jc = cv.take<float>((size_t)G.M * G.qa_cap);
    G.idx = cv.take<int>(G.qa_cap);
    G.inv = cv.take<int>(G.Q);
    G.mask = cv.take<float>(G.Q);
  }
  // Instances of equal geometry, levels and channels can form one group
  // (batched launches).  Groups of more than one member are switched off
  // (kGroupInstances): their first GPU run ended in a host-side crash whose
  // cause has not been found, so every instance forms its own group.
  X.insts.clear();
  X.members.assign(n_inst, std::make_pair(0, 0));
  for (int i = 0; i < n_inst; ++i) {
    int g = -1;
    for (size_t k = 0; kGroupInstances && k < X.insts.size(); ++k) {
      const Instance& J = X.insts[k];
      if (J.geo == id[i].geometry && J.L == id[i].levels && J.C == id[i].base_ch) g = (int)k;
    }
    if (g < 0) {
      X.insts.push_back(Instance());
      g = (int)X.insts.size() - 1;
      X.insts[g].geo = id[i].geometry;
      X.insts[g].L = id[i].levels;
      X.insts[g].C = id[i].base_ch;
      X.insts[g].B = 0;
    }
    Instance& J = X.insts[g];
    X.members[i] = std::make_pair(g, J.B);
    J.member_inst.push_back(i);
    J.B += 1;
  }
  const int prec = conv_prec(X.precision);
  for (size_t gi = 0; gi < X.insts.size(); ++gi) {
    size_t kpart_max = 0;
    Instance& I = X.insts[gi];
    I.has_frame.assign(I.B, 0);
    I.has_z.assign(I.B, 0);
    cv.off = (cv.off + 255) & ~size_t(255);
    const size_t region0 = cv.off;
    const Geometry& G = X.geos[I.geo];
    I.n = G.n;
    I.V0 = G.Q;
    I.P = layout(I);
    I.packs.clear();
    I.segs.clear();
    I.wtotal = 0;
    I.max_pack = 0;
    I.wg_total = 0;
    I.wgb_total = 0;
    // operand transforms fused into each pass (fixed by the schedule)
    I.stem.pro_wg = PRO_LN_BWD;
    for (Block& b : I.blocks) {
      b.c2.pro_fwd = PRO_LN_RELU;
      b.c1.pro_bwd = b.c2.pro_bwd = PRO_LN_BWD;
      b.c1.pro_wg = PRO_LN_BWD;
      b.c2.pro_wg = 3 * PRO_LN_RELU + PRO_LN_BWD;
    }
    add_conv(I, I.stem, X.precision, kpart_max);
    for (Block& b : I.blocks) {
      add_conv(I, b.c1, X.precision, kpart_max);
      add_conv(I, b.c2, X.precision, kpart_max);
      if (b.proj) add_conv(I, b.pj, X.precision, kpart_max);
    }
    // FP64 partial arena: statistics of every LayerNorm input, LayerNorm
    // backward partials, head gradient and residual sums (offsets in doubles)
    auto dtake = [&](size_t nd) {
      const long long o = I.dtotal;
      I.dtotal += (long long)((nd + 31) / 32 * 32);
      return o;
    };
    auto fwd_tiles = [](const Conv& c) {
      return conv_tiles(c.n, c.fwd.tile) * ((c.cout + c.fwd.bn - 1) / c.fwd.bn);
    };
    auto ln_seg = [&](long long off, int nblk, int C2, int th_g) {
      GradSeg sg;
      std::memset(&sg, 0, sizeof(sg));
      sg.kind = 1;
      sg.part_off = off;
      sg.splits = nblk;
      sg.cout = C2;
      sg.th_w = th_g;
      I.segs.push_back(sg);
      I.max_seg = std::max(I.max_seg, C2);
    };
    const size_t V0 = I.V0;
    const int C = I.C;
    const int nb0 = ln_bwd_blocks(V0, C);
    const long long o_sts = dtake(2 * (size_t)fwd_tiles(I.stem));
    const long long o_cbs = dtake(2 * (size_t)nb0);
    const long long o_lncs = dtake((size_t)nb0 * 2 * C);
    ln_seg(o_lncs, nb0, 2 * C, I.stem_n.th_g);
    std::vector<long long> o_st1, o_st2, o_cb1, o_cb2, o_lnc1, o_lnc2;
    for (Block& b : I.blocks) {
      const size_t V = (size_t)b.n * b.n * b.n;
      const int nb = ln_bwd_blocks(V, b.cout);
      o_st1.push_back(dtake(2 * (size_t)fwd_tiles(b.c1)));
      o_st2.push_back(dtake(2 * (size_t)fwd_tiles(b.c2)));
      o_cb1.push_back(dtake(2 * (size_t)nb));
      o_cb2.push_back(dtake(2 * (size_t)nb));
      o_lnc1.push_back(dtake((size_t)nb * 2 * b.cout));
      o_lnc2.push_back(dtake((size_t)nb * 2 * b.cout));
      ln_seg(o_lnc1.back(), nb, 2 * b.cout, b.n1.th_g);
      ln_seg(o_lnc2.back(), nb, 2 * b.cout, b.n2.th_g);
    }
    const int ntb = tail_bwd_blocks(V0, C);
    const long long o_tail = dtake((size_t)ntb * (C + 1));
    ln_seg(o_tail, ntb, C + 1, I.tail_w);
    const long long o_rsum = dtake(jt_mblocks(G.M));
    const long long o_tv = dtake(tv_blocks(V0));

    I.theta = cv.take<float>(I.P);
    I.grad = cv.take<float>(I.P);
    I.m = cv.take<float>(I.P);
    I.v = cv.take<float>(I.P);
    if (X.precision == D2IP_BF16_CONV)
      I.wbf16 = cv.take<uint16_t>(I.wtotal);
    else if (X.precision == D2IP_BF16X3_CONV)
      I.wbf16 = cv.take<uint16_t>(2 * I.wtotal);  // hi parts, then lo parts
    else
      I.wf32 = cv.take<float>(I.wtotal);
    I.packs_dev = cv.take<ConvPack>(I.packs.size());
    I.segs_dev = cv.take<GradSeg>(I.segs.size());
    I.wg_part = cv.take<float>(I.wg_total);
    I.wg_partb = cv.take<float>(I.wgb_total);
    I.dpart = cv.take<double>(I.dtotal);
    auto dp = [&](long long off) { return I.dpart ? I.dpart + off : nullptr; };
    I.zpad = cv.take<float>(V0 * 8);
    I.hs = cv.take<float>(V0 * C);
    I.as = cv.take<float>(V0 * C);
    I.sts = PairRef{dp(o_sts), fwd_tiles(I.stem), (double)V0 * C};
    I.cbs = PairRef{dp(o_cbs), nb0, (double)V0 * C};
    I.lncs = dp(o_lncs);
    I.lv.assign(I.L, Level());
    for (int l = 0; l < I.L; ++l) {
      Level& Lv = I.lv[l];
      Lv.n = I.n >> l;
      Lv.c = C << l;
      Lv.V = (size_t)Lv.n * Lv.n * Lv.n;
      Lv.gy = cv.take<float>(Lv.V * Lv.c);
      Lv.gz = cv.take<float>(Lv.V * Lv.c);
      Lv.ga = cv.take<float>(Lv.V * Lv.c);
      Lv.gx = cv.take<float>(Lv.V * Lv.c * 3);
      Lv.genc = cv.take<float>(Lv.V * Lv.c);
    }
    const int L = I.L;
    for (size_t k = 0; k < I.blocks.size(); ++k) {
      Block& b = I.blocks[k];
      const size_t V = (size_t)b.n * b.n * b.n;
      if (b.enc && b.level == 0)
        b.x = I.as;
      else if (b.enc)
        b.x = I.blocks[b.level - 1].pool_out;
      else
        b.x = cv.take<float>(V * b.cin);
      b.h1 = cv.take<float>(V * b.cout);
      b.h2 = cv.take<float>(V * b.cout);
      b.y = cv.take<float>(V * b.cout);
      if (b.proj) b.s = cv.take<float>(V * b.cout);
      if (b.proj) b.gpj = cv.take<float>(V * b.cin);
      if (b.enc && b.level < L - 1) b.pool_out = cv.take<float>(V / 8 * b.cout);
      b.gz = cv.take<float>(V * b.cout);
      b.ga = cv.take<float>(V * b.cout);
      const int nb = ln_bwd_blocks(V, b.cout);
      const double cnt = (double)V * b.cout;
      b.st1 = PairRef{dp(o_st1[k]), fwd_tiles(b.c1), cnt};
      b.st2 = PairRef{dp(o_st2[k]), fwd_tiles(b.c2), cnt};
      b.cb1 = PairRef{dp(o_cb1[k]), nb, cnt};
      b.cb2 = PairRef{dp(o_cb2[k]), nb, cnt};
      b.lnc1 = dp(o_lnc1[k]);
      b.lnc2 = dp(o_lnc2[k]);
    }
    for (size_t k = L; k < I.blocks.size(); ++k) {
      Block& b = I.blocks[k];
      b.up_src = (b.level == L - 2) ? I.blocks[L - 1].y : I.blocks[k - 1].y;
      b.skip_src = I.blocks[b.level].y;
    }
    I.sigma = cv.take<float>(V0);
    I.dv = cv.take<float>(G.M);
    I.it = cv.take<IterState>(1);
    I.ppart = cv.take<float>((size_t)jvec_qblocks(G.qa_cap) * G.M);
    I.tpart = cv.take<float>((size_t)jt_mblocks(G.M) * G.qa_cap);
    I.tail_part = dp(o_tail);
    I.rsum = dp(o_rsum);
    I.tvsum = dp(o_tv);
    I.gtv = cv.take<float>(V0);
    I.hist = cv.take<float>((size_t)kTvHistory * V0);
    I.tvs = cv.take<TvState>(1);
    I.tv_count.assign(I.B, 0);
    I.tv_head.assign(I.B, kTvHistory - 1);
    I.kpart = cv.take<float>(std::max<size_t>(kpart_max, 1));
    // members 1.. follow member 0 at a fixed stride
    cv.off = (cv.off + 255) & ~size_t(255);
    I.istride = (long long)(cv.off - region0);
    cv.off = region0 + (size_t)I.istride * I.B;
    if (g_chk && cv.base) {
      // members 1.. hold the same allocations shifted by the member stride
      const uintptr_t lo0 = (uintptr_t)cv.base + region0, hi0 = lo0 + (uintptr_t)I.istride;
      std::vector<Checker::Alloc> mine;
      for (const Checker::Alloc& a : g_chk->allocs)
        if (a.lo >= lo0 && a.hi <= hi0) mine.push_back(a);
      for (int b = 1; b < I.B; ++b)
        for (const Checker::Alloc& a : mine)
          g_chk->allocs.push_back({a.lo + (uintptr_t)(b * I.istride), a.hi + (uintptr_t)(b * I.istride)});
    }
  }
}

// Launch wrappers: launch, or (checker active) verify argument extents.
void chk_src(Checker& c, const ConvSrc& s, size_t V, int ch, int B, long long is, const char* nm) {
  const std::string n = nm;
  c.require(s.stride >= ch, n + ": stride < channels read");
  c.range(s.x, ((V - 1) * s.stride + ch) * sizeof(float), (n + ".x").c_str(), B, is);
  if (s.prologue != PRO_NONE) {
    c.range(s.gamma, ch * sizeof(float), (n + ".gamma").c_str(), B, is);
    c.range(s.st.part, s.st.nparts * 2 * sizeof(double), (n + ".stats").c_str(), B, is);
    c.require(s.st.nparts > 0, n + ": no statistics partials");
  }
  if (s.prologue == PRO_LN_RELU) c.range(s.beta, ch * sizeof(float), (n + ".beta").c_str(), B, is);
  if (s.prologue == PRO_LN_BWD) {
    c.range(s.h, ((V - 1) * s.stride + ch) * sizeof(float), (n + ".h").c_str(), B, is);
    c.range(s.bw.part, s.bw.nparts * 2 * sizeof(double), (n + ".coef").c_str(), B, is);
  }
}

void L_conv_fwd(const ConvFwd& a, hipStream_t s) {
  if (!g_chk) return conv_fwd(a, s);
  Checker& c = *g_chk;
  c.where = "conv_fwd";
  const size_t V = (size_t)a.n * a.n * a.n;
  const int B = a.batch;
  const long long is = a.istride;
  c.require(B >= 1, "batch < 1");
  c.require(a.ck == 8 || a.ck == 16 || a.ck == 32, "bad channel chunk");
  c.require(a.cin % a.ck == 0, "cin not a multiple of the chunk");
  c.require(a.ksplit >= 1 && (a.cin / a.ck) % a.ksplit == 0, "ksplit does not divide the chunks");
  c.require(a.bn == 16 || a.bn == 32 || a.bn == 64, "bad N tile");
  c.require(!(a.tile == TILE_2x4x16 && a.bn == 64), "128-voxel tile with N tile 64");
  c.require(conv_fwd_lds_bytes(a.tile, a.taps, a.bn, a.ck, a.prec) <= 60 * 1024, "LDS over budget");
  chk_src(c, a.src, V, a.cin, B, is, "src");
  const size_t el = a.prec == PREC_F32 ? 4 : 2;
  const size_t wel = (size_t)a.w_rows * a.taps * a.cin;
  c.range(a.w, (a.prec == PREC_BF16X3 ? a.w_lo_off + wel : wel) * el, "weights", B, is);
  c.require(a.w_rows >= a.cout, "fewer weight rows than outputs");
  c.range(a.bias, a.cout * sizeof(float), "bias", B, is);
  c.range(a.add, V * a.cout * sizeof(float), "add", B, is);
  c.range(a.y, V * a.cout * sizeof(float), "y", B, is);
  const int tiles = conv_fwd_blocks(a);
  c.range(a.stat_part, (size_t)tiles * 2 * sizeof(double), "stat partials", B, is);
  if (a.ksplit > 1) {
    c.range(a.kpart, (size_t)a.ksplit * V * a.cout * sizeof(float), "split-K partials", B, is);
  }
}

void L_conv_wgrad(const ConvWgrad& a, hipStream_t s) {
  if (!g_chk) return conv_wgrad(a, s);
  Checker& c = *g_chk;
  c.where = "conv_wgrad";
  const size_t V = (size_t)a.n * a.n * a.n;
  const int B = a.batch;
  const long long is = a.istride;
  c.require(a.cin % a.ck == 0, "cin not a multiple of the chunk");
  c.require(conv_wgrad_lds_bytes(a.tile, a.taps, a.ck, a.prec) <= 60 * 1024, "LDS over budget");
  c.require(a.gsrc.stride == a.cout, "g stride != cout");
  chk_src(c, a.src, V, a.cin, B, is, "x");
  chk_src(c, a.gsrc, V, a.cout, B, is, "g");
  const size_t cout16 = (a.cout + 15) / 16 * 16;
  c.range(a.part, (size_t)a.splits * cout16 * a.taps * a.cin * sizeof(float), "partials", B, is);
  c.range(a.partb, (size_t)a.splits * cout16 * sizeof(float), "bias partials", B, is);
}

void L_ln_apply(const float* h, PairRef st, const float* g, const float* b, const float* skip,
                float* y, size_t V, int C, int B, long long is, hipStream_t s) {
  if (!g_chk) return ln_apply(h, st, g, b, skip, y, V, C, B, is, s);
  Checker& c = *g_chk;
  c.where = "ln_apply";
  c.range(h, V * C * 4, "h", B, is);
  c.range(st.part, st.nparts * 16, "stats", B, is);
  c.range(g, C * 4, "gamma", B, is);
  c.range(b, C * 4, "beta", B, is);
  c.range(skip, V * C * 4, "skip", B, is);
  c.range(y, V * C * 4, "y", B, is);
}

void L_ln_apply_pool(const float* h, PairRef st, const float* g, const float* b,
                     const float* skip, float* y, float* pooled, int n, int C, int B,
                     long long is, hipStream_t s) {
  if (!g_chk) return ln_apply_pool(h, st, g, b, skip, y, pooled, n, C, B, is, s);
  Checker& c = *g_chk;
  c.where = "ln_apply_pool";
  const size_t V = (size_t)n * n * n;
  c.require(n % 2 == 0, "odd grid");
  c.range(h, V * C * 4, "h", B, is);
  c.range(st.part, st.nparts * 16, "stats", B, is);
  c.range(g, C * 4, "gamma", B, is);
  c.range(b, C * 4, "beta", B, is);
  c.range(skip, V * C * 4, "skip", B, is);
  c.range(y, V * C * 4, "y", B, is);
  c.range(pooled, V / 8 * C * 4, "pooled", B, is);
}

void L_ln_bwd(const float* gy, int mm, const float* my, const float* mg, const float* mb,
              const float* h, PairRef st, float* gz, double* pc, double* pab, size_t V, int C,
              const float* gamma, int B, long long is, hipStream_t s) {
  if (!g_chk) return ln_bwd(gy, mm, my, mg, mb, h, st, gz, pc, pab, V, C, gamma, B, is, s);
  Checker& c = *g_chk;
  c.where = "ln_bwd";
  const size_t nb = ln_bwd_blocks(V, C);
  c.require(256 % C == 0, "channels do not divide 256");
  c.range(gy, V * C * 4, "gy", B, is);
  if (mm == LNMASK_Y) c.range(my, V * C * 4, "mask y", B, is);
  if (mm == LNMASK_LN) {
    c.range(mg, C * 4, "mask gamma", B, is);
    c.range(mb, C * 4, "mask beta", B, is);
  }
  c.range(h, V * C * 4, "h", B, is);
  c.range(st.part, st.nparts * 16, "stats", B, is);
  c.range(gz, V * C * 4, "gz", B, is);
  c.range(pc, nb * 2 * C * 8, "channel partials", B, is);
  c.range(pab, nb * 2 * 8, "coefficient partials", B, is);
  c.range(gamma, C * 4, "gamma", B, is);
}

void L_up_concat(const float* d, int Cu, const float* e, int Cs, int n, float* cat, int B,
                 long long is, hipStream_t s) {
  if (!g_chk) return up_concat(d, Cu, e, Cs, n, cat, B, is, s);
  Checker& c = *g_chk;
  c.where = "up_concat";
  const size_t V = (size_t)n * n * n;
  c.range(d, V / 8 * Cu * 4, "coarse", B, is);
  c.range(e, V * Cs * 4, "skip", B, is);
  c.range(cat, V * (Cu + Cs) * 4, "cat", B, is);
}

void L_up_concat_bwd(const float* gcat, int Cu, int Cs, int n, float* gu, float* gs, int B,
                     long long is, hipStream_t s) {
  if (!g_chk) return up_concat_bwd(gcat, Cu, Cs, n, gu, gs, B, is, s);
  Checker& c = *g_chk;
  c.where = "up_concat_bwd";
  const size_t V = (size_t)n * n * n;
  c.range(gcat, V * (Cu + Cs) * 4, "gcat", B, is);
  c.range(gu, V / 8 * Cu * 4, "gu", B, is);
  c.range(gs, V * Cs * 4, "gs", B, is);
}

void L_pool_bwd_add(const float* gx, const float* add, int n, int C, float* gy, int B,
                    long long is, hipStream_t s) {
  if (!g_chk) return pool_bwd_add(gx, add, n, C, gy, B, is, s);
  Checker& c = *g_chk;
  c.where = "pool_bwd_add";
  const size_t V = (size_t)n * n * n;
  c.range(gx, V / 8 * C * 4, "gx", B, is);
  c.range(add, V * C * 4, "add", B, is);
  c.range(gy, V * C * 4, "gy", B, is);
}

void L_tail_fwd(const float* d0, int C, const float* w, const float* b, const float* mask,
                size_t V, float* sigma, int B, long long is, hipStream_t s) {
  if (!g_chk) return tail_fwd(d0, C, w, b, mask, V, sigma, B, is, s);
  Checker& c = *g_chk;
  c.where = "tail_fwd";
  c.range(d0, V * C * 4, "d0", B, is);
  c.range(w, C * 4, "w", B, is);
  c.range(b, 4, "b", B, is);
  c.range(mask, V * 4, "mask");
  c.range(sigma, V * 4, "sigma", B, is);
}

void L_jvec(const float* Jc, int M, int qa_pad, const int* idx, const float* sigma, float* ppart,
            size_t V, int B, long long is, hipStream_t s) {
  if (!g_chk) return jvec(Jc, M, qa_pad, idx, sigma, ppart, B, is, s);
  Checker& c = *g_chk;
  c.where = "jvec";
  c.range(Jc, (size_t)M * qa_pad * 4, "J");
  c.range(idx, (size_t)qa_pad * 4, "idx");
  c.range(sigma, V * 4, "sigma", B, is);
  c.range(ppart, (size_t)jvec_qblocks(qa_pad) * M * 4, "ppart", B, is);
}

void L_jtvec(const float* Jc, int M, int qa_pad, const float* ppart, int nqb, const float* dv,
             double* rsum, float* tpart, int B, long long is, hipStream_t s) {
  if (!g_chk) return jtvec(Jc, M, qa_pad, ppart, nqb, dv, rsum, tpart, B, is, s);
  Checker& c = *g_chk;
  c.where = "jtvec";
  c.range(Jc, (size_t)M * qa_pad * 4, "J");
  c.range(ppart, (size_t)nqb * M * 4, "ppart", B, is);
  c.range(dv, (size_t)M * 4, "dv", B, is);
  c.range(rsum, (size_t)jt_mblocks(M) * 8, "rsum", B, is);
  c.require(jt_partials(M, qa_pad) <= jt_mblocks(M), "J^T g row groups beyond the partial buffer");
  c.range(tpart, (size_t)jt_partials(M, qa_pad) * qa_pad * 4, "tpart", B, is);
}

void L_tail_bwd(const float* tpart, int nmb, int qa_pad, const int* inv, const float* d0, int C,
                const float* w, size_t V, float* gd0, double* part, const float* gtv, int B,
                long long is, hipStream_t s) {
  if (!g_chk) return tail_bwd(tpart, nmb, qa_pad, inv, d0, C, w, V, gd0, part, gtv, B, is, s);
  Checker& c = *g_chk;
  c.where = "tail_bwd";
  c.range(tpart, (size_t)nmb * qa_pad * 4, "tpart", B, is);
  c.range(inv, V * 4, "inv");
  c.range(d0, V * C * 4, "d0", B, is);
  c.range(w, C * 4, "w", B, is);
  c.range(gd0, V * C * 4, "gd0", B, is);
  c.range(part, (size_t)tail_bwd_blocks(V, C) * (C + 1) * 8, "partials", B, is);
  c.range(gtv, V * 4, "gtv", B, is);
}

void L_tv(const float* sigma, int n, const float* hist, const TvState* ts, TvCoef k, float* gtv,
          double* tvsum, int B, long long is, hipStream_t s) {
  if (!g_chk) return tv_reg(sigma, n, hist, ts, k, gtv, tvsum, B, is, s);
  Checker& c = *g_chk;
  c.where = "tv";
  const size_t V = (size_t)n * n * n;
  c.range(sigma, V * 4, "sigma", B, is);
  c.range(hist, (size_t)kTvHistory * V * 4, "history", B, is);
  c.range(ts, sizeof(TvState), "tv state", B, is);
  c.range(gtv, V * 4, "gtv", B, is);
  c.range(tvsum, (size_t)tv_blocks(V) * 8, "tv partials", B, is);
}

void L_grad_reduce(const Instance& I, float* grad, hipStream_t s) {
  if (!g_chk)
    return grad_reduce(I.segs_dev, (int)I.segs.size(), I.max_seg, I.wg_part, I.wg_partb, I.dpart,
                       grad, I.B, I.istride, s);
  Checker& c = *g_chk;
  c.where = "grad_reduce";
  c.range(I.segs_dev, I.segs.size() * sizeof(GradSeg), "segments");
  for (const GradSeg& g : I.segs) {
    if (g.kind == 0) {
      const size_t cout16 = (g.cout + 15) / 16 * 16;
      c.range(I.wg_part + g.part_off, (size_t)g.splits * cout16 * g.taps * g.cin * 4, "conv partials",
              I.B, I.istride);
      c.range(I.wg_partb + g.partb_off, (size_t)g.splits * cout16 * 4, "bias partials", I.B,
              I.istride);
      c.range(grad + g.th_w, (size_t)g.cout * g.cin_real * g.taps * 4, "dW", I.B, I.istride);
      c.range(grad + g.th_b, (size_t)g.cout * 4, "db", I.B, I.istride);
      c.require(g.th_w + g.cout * g.cin_real * g.taps <= (long long)I.P, "dW beyond theta");
    } else {
      c.range(I.dpart + g.part_off, (size_t)g.splits * g.cout * 8, "column partials", I.B,
              I.istride);
      c.range(grad + g.th_w, (size_t)g.cout * 4, "columns", I.B, I.istride);
      c.require(g.th_w + g.cout <= (int)I.P, "columns beyond theta");
    }
  }
}

void L_adam(Instance& I, const d2ip_ctx& X, hipStream_t s);
void L_pack(Instance& I, int prec, bool end_iteration, int M, hipStream_t s,
            bool tv = false);

// ---------------------------------------------------------------------------
// launch schedule
// ---------------------------------------------------------------------------

ConvSrc src_plain(const float* x, int stride) {
  ConvSrc s;
  std::memset(&s, 0, sizeof(s));
  s.x = x;
  s.stride = stride;
  s.prologue = PRO_NONE;
  return s;
}

ConvSrc src_ln_relu(const float* h, int stride, const PairRef& st, const float* g,
                    const float* b) {
  ConvSrc s = src_plain(h, stride);
  s.prologue = PRO_LN_RELU;
  s.st = st;
  s.gamma = g;
  s.beta = b;
  return s;
}

ConvSrc src_ln_bwd(const float* gz, const float* h, int stride, const PairRef& st,
                   const float* g, const PairRef& cb) {
  ConvSrc s = src_plain(gz, stride);
  s.prologue = PRO_LN_BWD;
  s.h = h;
  s.st = st;
  s.gamma = g;
  s.bw = cb;
  return s;
}

// Forward conv: y = conv(src) + bias, with LayerNorm statistics into `st`.
ConvFwd fwd_args(const d2ip_ctx& X, const Instance& I, const Conv& c, ConvSrc src, float* y,
                 const PairRef* st) {
  const int prec = conv_prec(X.precision);
  ConvFwd a;
  std::memset(&a, 0, sizeof(a));
  a.src = src;
  a.n = c.n;
  a.cin = c.cin;
  a.w = prec != PREC_F32 ? (const void*)(I.wbf16 + c.wf) : (const void*)(I.wf32 + c.wf);
  a.w_lo_off = prec == PREC_BF16X3 ? I.wtotal : 0;
  a.w_rows = c.cout;
  a.bias = I.theta + c.th_b;
  a.cout = c.cout;
  a.y = y;
  a.taps = c.taps;
  a.stat_part = st ? const_cast<double*>(st->part) : nullptr;
  a.prec = prec;
  a.tile = c.fwd.tile;
  a.bn = c.fwd.bn;
  a.ck = c.fwd.ck;
  a.ksplit = c.fwd.ksplit;
  a.kpart = I.kpart;
  a.batch = I.B;
  a.istride = I.istride;
  return a;
}

// Input gradient: y (+)= conv^T(src) (+ add).
ConvFwd dgrad_args(const d2ip_ctx& X, const Instance& I, const Conv& c, ConvSrc src, float* y) {
  const int prec = conv_prec(X.precision);
  ConvFwd a;
  std::memset(&a, 0, sizeof(a));
  a.src = src;
  a.n = c.n;
  a.cin = c.cout;
  a.w = prec != PREC_F32 ? (const void*)(I.wbf16 + c.wd) : (const void*)(I.wf32 + c.wd);
  a.w_lo_off = prec == PREC_BF16X3 ? I.wtotal : 0;
  a.w_rows = c.cin_real;
  a.cout = c.cin_real;
  a.y = y;
  a.taps = c.taps;
  a.prec = prec;
  a.tile = c.bwd.tile;
  a.bn = c.bwd.bn;
  a.ck = c.bwd.ck;
  a.ksplit = c.bwd.ksplit;
  a.kpart = I.kpart;
  a.batch = I.B;
  a.istride = I.istride;
  return a;
}

void wgrad(const d2ip_ctx& X, const Instance& I, const Conv& c, ConvSrc xs, ConvSrc gsrc,
           hipStream_t stream) {
  ConvWgrad a;
  std::memset(&a, 0, sizeof(a));
  a.src = xs;
  a.gsrc = gsrc;
  a.n = c.n;
  a.cin = c.cin;
  a.cout = c.cout;
  a.taps = c.taps;
  a.part = I.wg_part + c.wg_off;
  a.partb = I.wg_partb + c.wgb_off;
  a.splits = c.wg_splits;
  a.prec = conv_prec(X.precision);
  a.tile = c.wg_tile;
  a.ck = c.wg_ck;
  a.batch = I.B;
  a.istride = I.istride;
  L_conv_wgrad(a, stream);
}

// Fork the side stream off the main stream at this point / join it back.
// Event calls made while an iteration is enqueued report errors through the
// hipGetLastError check after it (or through the end of a graph capture);
// teardown calls ignore theirs.
void fork(d2ip_ctx& X) {
  if (g_chk) return;
  (void)hipEventRecord(X.ev_fork, X.stream);
  (void)hipStreamWaitEvent(X.side, X.ev_fork, 0);
}
void join(d2ip_ctx& X) {
  if (g_chk) return;
  (void)hipEventRecord(X.ev_join, X.side);
  (void)hipStreamWaitEvent(X.stream, X.ev_join, 0);
}

void enqueue_forward(d2ip_ctx& X, Instance& I) {
  const Geometry& G = X.geos[I.geo];
  hipStream_t s = X.stream;
  float* th = I.theta;
  const int L = I.L;
  L_conv_fwd(fwd_args(X, I, I.stem, src_plain(I.zpad, 8), I.hs, &I.sts), s);
  L_ln_apply(I.hs, I.sts, th + I.stem_n.th_g, th + I.stem_n.th_b, nullptr, I.as, I.V0, I.C, I.B,
           I.istride, s);
  for (Block& b : I.blocks) {
    const size_t V = (size_t)b.n * b.n * b.n;
    if (!b.enc) L_up_concat(b.up_src, b.cout * 2, b.skip_src, b.cout, b.n, b.x, I.B, I.istride, s);
    if (b.proj) {
      // the 1x1 projection only needs x: overlap it with conv1 / conv2
      fork(X);
      L_conv_fwd(fwd_args(X, I, b.pj, src_plain(b.x, b.cin), b.s, nullptr), X.side);
    }
    L_conv_fwd(fwd_args(X, I, b.c1, src_plain(b.x, b.cin), b.h1, &b.st1), s);
    L_conv_fwd(fwd_args(X, I, b.c2,
                      src_ln_relu(b.h1, b.cout, b.st1, th + b.n1.th_g, th + b.n1.th_b), b.h2,
                      &b.st2),
             s);
    if (b.proj) join(X);
    const float* skip = b.proj ? b.s : b.x;
    if (b.enc && b.level < L - 1)
      L_ln_apply_pool(b.h2, b.st2, th + b.n2.th_g, th + b.n2.th_b, skip, b.y, b.pool_out, b.n,
                    b.cout, I.B, I.istride, s);
    else
      L_ln_apply(b.h2, b.st2, th + b.n2.th_g, th + b.n2.th_b, skip, b.y, V, b.cout, I.B, I.istride,
               s);
  }
  L_tail_fwd(I.blocks.back().y, I.C, th + I.tail_w, th + I.tail_b, G.mask, I.V0, I.sigma, I.B,
           I.istride, s);
}

void enqueue_iteration(d2ip_ctx& X, Instance& I) {
  const Geometry& G = X.geos[I.geo];
  hipStream_t s = X.stream;
  float* th = I.theta;
  float* gr = I.grad;
  enqueue_forward(X, I);
  // measurement operator, data term and its gradient w.r.t. the image
  const int nqb = jvec_qblocks(G.qa_pad);
  if (X.tv_on) {
    // the 4D-TV term only needs the image: beside the J products
    fork(X);
    L_tv(I.sigma, I.n, I.hist, I.tvs, X.tv, I.gtv, I.tvsum, I.B, I.istride, X.side);
  }
  L_jvec(G.Jc, G.M, G.qa_pad, G.idx, I.sigma, I.ppart, I.V0, I.B, I.istride, s);
  L_jtvec(G.Jc, G.M, G.qa_pad, I.ppart, nqb, I.dv, I.rsum, I.tpart, I.B, I.istride, s);
  if (X.tv_on) join(X);
  L_tail_bwd(I.tpart, jt_partials(G.M, G.qa_pad), G.qa_pad, G.inv, I.blocks.back().y, I.C, th + I.tail_w,
           I.V0, I.lv[0].gy, I.tail_part, X.tv_on ? I.gtv : nullptr, I.B, I.istride, s);
  // network backward, decoder first.  Weight gradients only feed the batched
  // reduction at the end: they run on the side stream, overlapping the
  // input-gradient chain, and join before the reduction.
  for (int k = (int)I.blocks.size() - 1; k >= 0; --k) {
    Block& b = I.blocks[k];
    Level& Lv = I.lv[b.level];
    const size_t V = (size_t)b.n * b.n * b.n;
    const float* g1 = th + b.n1.th_g;
    const float* b1 = th + b.n1.th_b;
    const float* g2 = th + b.n2.th_g;
    // LN2 backward (mask from y): gz and its partials
    L_ln_bwd(Lv.gy, LNMASK_Y, b.y, nullptr, nullptr, b.h2, b.st2, b.gz, b.lnc2,
           const_cast<double*>(b.cb2.part), V, b.cout, g2, I.B, I.istride, s);
    const ConvSrc gh2 = src_ln_bwd(b.gz, b.h2, b.cout, b.st2, g2, b.cb2);
    fork(X);
    if (b.proj) {
      // the projection's input gradient needs only gz: first on the side
      // stream, off the critical path; conv1's input gradient adds it
      L_conv_fwd(dgrad_args(X, I, b.pj, src_plain(b.gz, b.cout), b.gpj), X.side);
      if (!g_chk) (void)hipEventRecord(X.ev_pj, X.side);
    }
    wgrad(X, I, b.c2, src_ln_relu(b.h1, b.cout, b.st1, g1, b1), gh2, X.side);
    if (b.proj) wgrad(X, I, b.pj, src_plain(b.x, b.cin), src_plain(b.gz, b.cout), X.side);
    L_conv_fwd(dgrad_args(X, I, b.c2, gh2, b.ga), s);
    // LN1 backward (mask from LN1 output), in place on ga
    L_ln_bwd(b.ga, LNMASK_LN, nullptr, g1, b1, b.h1, b.st1, b.ga, b.lnc1,
           const_cast<double*>(b.cb1.part), V, b.cout, g1, I.B, I.istride, s);
    const ConvSrc gh1 = src_ln_bwd(b.ga, b.h1, b.cout, b.st1, g1, b.cb1);
    fork(X);
    wgrad(X, I, b.c1, src_plain(b.x, b.cin), gh1, X.side);
    {
      ConvFwd a = dgrad_args(X, I, b.c1, gh1, Lv.gx);
      a.add = b.proj ? b.gpj : b.gz;
      if (b.proj && !g_chk) (void)hipStreamWaitEvent(s, X.ev_pj, 0);
      L_conv_fwd(a, s);
    }
    if (!b.enc) {
      L_up_concat_bwd(Lv.gx, b.cout * 2, b.cout, b.n, I.lv[b.level + 1].gy, Lv.genc, I.B,
                    I.istride, s);
    } else if (b.level > 0) {
      Level& Lp = I.lv[b.level - 1];
      L_pool_bwd_add(Lv.gx, Lp.genc, Lp.n, Lp.c, Lp.gy, I.B, I.istride, s);
    }
  }
  // stem
  {
    Level& L0 = I.lv[0];
    const float* gs = th + I.stem_n.th_g;
    L_ln_bwd(L0.gx, LNMASK_Y, I.as, nullptr, nullptr, I.hs, I.sts, L0.gz, I.lncs,
           const_cast<double*>(I.cbs.part), I.V0, I.C, gs, I.B, I.istride, s);
    fork(X);
    wgrad(X, I, I.stem, src_plain(I.zpad, 8), src_ln_bwd(L0.gz, I.hs, I.C, I.sts, gs, I.cbs),
          X.side);
  }
  join(X);
  L_grad_reduce(I, gr, s);
  L_adam(I, X, s);
  L_pack(I, X.precision, true, G.M, s, X.tv_on);
}

// One iteration of every instance group: groups on different lanes run
// concurrently (their workspace regions are disjoint; geometries are read
// only).  Lanes are used for eager launches only: the first captured graph
// with lanes ended in a host-side crash whose cause has not been found, so a
// captured iteration runs the groups one after another.
void enqueue_all(d2ip_ctx& X, bool capturing) {
  if (X.lanes.empty() || capturing) {
    for (Instance& I : X.insts) enqueue_iteration(X, I);
    return;
  }
  const hipStream_t s0 = X.stream, side0 = X.side;
  const hipEvent_t f0 = X.ev_fork, j0 = X.ev_join, p0 = X.ev_pj;
  (void)hipEventRecord(X.ev_start, s0);
  for (d2ip_ctx::Lane& l : X.lanes) (void)hipStreamWaitEvent(l.main, X.ev_start, 0);
  for (size_t k = 0; k < X.insts.size(); ++k) {
    d2ip_ctx::Lane& l = X.lanes[k % X.lanes.size()];
    X.stream = l.main;
    X.side = l.side;
    X.ev_fork = l.fork;
    X.ev_join = l.join;
    X.ev_pj = l.pj;
    enqueue_iteration(X, X.insts[k]);
  }
  X.stream = s0;
  X.side = side0;
  X.ev_fork = f0;
  X.ev_join = j0;
  X.ev_pj = p0;
  for (d2ip_ctx::Lane& l : X.lanes) {
    (void)hipEventRecord(l.done, l.main);
    (void)hipStreamWaitEvent(s0, l.done, 0);
  }
}

void L_adam(Instance& I, const d2ip_ctx& X, hipStream_t s) {
  if (!g_chk)
    return adam(I.theta, I.grad, I.m, I.v, I.P, X.lr, X.b1, X.b2, X.eps, I.it, I.B, I.istride, s);
  Checker& c = *g_chk;
  c.where = "adam";
  for (const float* p : {(const float*)I.theta, (const float*)I.grad, (const float*)I.m,
                         (const float*)I.v})
    c.range(p, I.P * 4, "parameter vector", I.B, I.istride);
  c.range(I.it, sizeof(IterState), "iteration state", I.B, I.istride);
}

void L_pack(Instance& I, int precision, bool end_iteration, int M, hipStream_t s, bool tv) {
  const long long lo = precision == D2IP_BF16X3_CONV ? I.wtotal : 0;
  const int nrs = jt_mblocks(M);
  const int ntv = end_iteration && tv ? tv_blocks(I.V0) : 0;
  if (!g_chk)
    return pack_weights(I.packs_dev, (int)I.packs.size(), I.max_pack, I.theta, I.wf32, I.wbf16,
                        lo, end_iteration ? I.it : nullptr, end_iteration ? I.rsum : nullptr,
                        end_iteration ? nrs : 0, end_iteration ? M : 1, I.tvsum, ntv, I.B,
                        I.istride, s);
  Checker& c = *g_chk;
  c.where = "pack_weights";
  c.range(I.packs_dev, I.packs.size() * sizeof(ConvPack), "pack table");
  for (const ConvPack& p : I.packs) {
    c.range(I.theta + p.th_off, (size_t)p.cout * p.cin_real * p.taps * 4, "theta", I.B, I.istride);
    const size_t nf = (size_t)p.cout * p.taps * p.cin, nd = (size_t)p.cin_real * p.taps * p.cout;
    if (I.wf32) {
      c.range(I.wf32 + p.wf_off, nf * 4, "packed fwd", I.B, I.istride);
      if (p.need_dgrad) c.range(I.wf32 + p.wd_off, nd * 4, "packed dgrad", I.B, I.istride);
    }
    if (I.wbf16) {
      c.range(I.wbf16 + p.wf_off + lo, nf * 2, "packed fwd (lo)", I.B, I.istride);
      c.range(I.wbf16 + p.wf_off, nf * 2, "packed fwd", I.B, I.istride);
      if (p.need_dgrad) {
        c.range(I.wbf16 + p.wd_off, nd * 2, "packed dgrad", I.B, I.istride);
        c.range(I.wbf16 + p.wd_off + lo, nd * 2, "packed dgrad (lo)", I.B, I.istride);
      }
    }
  }
  if (ntv) c.range(I.tvsum, (size_t)ntv * 8, "tv partials", I.B, I.istride);
  if (end_iteration) {
    c.range(I.rsum, nrs * 8, "rsum", I.B, I.istride);
    c.range(I.it, sizeof(IterState), "iteration state", I.B, I.istride);
  }
}

// Waits for a stream when it goes out of scope: declared after the host
// buffers that asynchronous copies on that stream read or write, so that no
// return path frees them before the copies have run.
struct StreamDrain {
  hipStream_t s;
  ~StreamDrain() { (void)hipStreamSynchronize(s); }
};

d2ip_status check_inst(d2ip_ctx* X, int inst) {
  if (!X) return fail(D2IP_EINVAL, "null context");
  if (inst < 0 || inst >= (int)X->members.size()) return fail(D2IP_EINVAL, "bad instance index");
  return D2IP_OK;
}

hipMemcpyKind kind_to_dev(int on_device) {
  return on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
}
hipMemcpyKind kind_from_dev(int on_device) {
  return on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
}

d2ip_status copy_in(d2ip_ctx* X, void* dst, const void* src, size_t bytes, int on_device) {
  HIPCHK(hipMemcpyAsync(dst, src, bytes, kind_to_dev(on_device), X->stream));
  if (!on_device) HIPCHK(hipStreamSynchronize(X->stream));
  return D2IP_OK;
}

d2ip_status copy_out(d2ip_ctx* X, void* dst, const void* src, size_t bytes, int on_device) {
  HIPCHK(hipMemcpyAsync(dst, src, bytes, kind_from_dev(on_device), X->stream));
  if (!on_device) HIPCHK(hipStreamSynchronize(X->stream));
  return D2IP_OK;
}

d2ip_status repack(d2ip_ctx* X, Instance& I) {
  L_pack(I, X->precision, false, 1, X->stream);
  HIPCHK(hipGetLastError());
  return D2IP_OK;
}

// Operand buffers of one standalone conv pass (d2ip_time_conv).
struct TimeConvBufs {
  float *x = nullptr, *h = nullptr, *g = nullptr, *y = nullptr, *gamma = nullptr, *beta = nullptr;
  float *bias = nullptr, *kpart = nullptr, *part = nullptr, *partb = nullptr;
  void* w = nullptr;
  double *st = nullptr, *stat = nullptr;
};

void carve_time_conv(const d2ip_tuning_entry& e, Carver& cv, TimeConvBufs& b) {
  const size_t V = (size_t)e.n * e.n * e.n;
  const int kin = e.pass == 1 ? e.cout : e.cin, kout = e.pass == 1 ? e.cin : e.cout;
  const int cmax = std::max(e.cin, e.cout);
  b.x = cv.take<float>(V * kin);
  b.h = cv.take<float>(V * cmax);
  b.g = cv.take<float>(V * e.cout);
  b.y = cv.take<float>(V * kout);
  b.gamma = cv.take<float>(cmax);
  b.beta = cv.take<float>(cmax);
  b.bias = cv.take<float>(kout);
  b.st = cv.take<double>(2);
  const int prec = conv_prec(e.precision);
  const size_t wel = (size_t)kout * e.taps * kin;
  if (prec == PREC_F32)
    b.w = cv.take<float>(wel);
  else
    b.w = cv.take<uint16_t>((prec == PREC_BF16X3 ? 2 : 1) * wel);
  const int tiles = conv_tiles(e.n, e.shape.tile) * ((kout + std::max(e.shape.bn, 16) - 1) /
                                                     std::max(e.shape.bn, 16));
  b.stat = cv.take<double>(2 * (size_t)tiles);
  b.kpart = cv.take<float>(std::max<size_t>(1, (size_t)e.shape.split * V * kout));
  const size_t cout16 = (e.cout + 15) / 16 * 16;
  b.part = cv.take<float>((size_t)e.shape.split * cout16 * e.taps * e.cin);
  b.partb = cv.take<float>((size_t)e.shape.split * cout16);
}

constexpr size_t kMaxLanes = 4;  // concurrent instance groups (hardware queues per process)

void release_lanes(d2ip_ctx* X) {
  for (d2ip_ctx::Lane& l : X->lanes) {
    if (l.pj) (void)hipEventDestroy(l.pj);
    if (l.done) (void)hipEventDestroy(l.done);
    if (l.join) (void)hipEventDestroy(l.join);
    if (l.fork) (void)hipEventDestroy(l.fork);
    if (l.side) (void)hipStreamDestroy(l.side);
    if (l.main) (void)hipStreamDestroy(l.main);
  }
  X->lanes.clear();
  if (X->ev_start) (void)hipEventDestroy(X->ev_start);
  X->ev_start = nullptr;
}

void drop_graph(d2ip_ctx* X) {
  if (X->gexec) (void)hipGraphExecDestroy(X->gexec);
  if (X->graph) (void)hipGraphDestroy(X->graph);
  X->gexec = nullptr;
  X->graph = nullptr;
}

}  // namespace

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------

extern "C" {

const char* d2ip_last_error(void) { return g_err.c_str(); }

d2ip_status d2ip_param_count(int levels, int base_ch, size_t* out) {
  if (!out) return fail(D2IP_EINVAL, "null output");
  if (levels < 2 || levels > 5 || base_ch <= 0 || base_ch > 256)
    return fail(D2IP_EINVAL, "levels must be 2..5 and base_ch in 1..256");
  Instance I;
  I.L = levels;
  I.C = base_ch;
  *out = layout(I);
  return D2IP_OK;
}

d2ip_status d2ip_runtime_versions(int* compiled, int* loaded) {
  if (!compiled || !loaded) return fail(D2IP_EINVAL, "null output");
  *compiled = HIP_VERSION;
  *loaded = 0;
  HIPCHK(hipRuntimeGetVersion(loaded));
  return D2IP_OK;
}

d2ip_status d2ip_init_params_host(int levels, int base_ch, uint64_t seed, float* theta,
                                  size_t n) {
  size_t P = 0;
  d2ip_status st = d2ip_param_count(levels, base_ch, &P);
  if (st != D2IP_OK) return st;
  if (!theta || n != P) return fail(D2IP_EINVAL, "theta must hold " + std::to_string(P) + " floats");
  Instance I;
  I.L = levels;
  I.C = base_ch;
  I.n = 2 << levels;  // offsets do not depend on the grid
  layout(I);
  // Standard normals from a counter-based generator: value k of the flat
  // vector uses SplitMix64 outputs 2k and 2k + 1 (Box-Muller), so a draw
  // depends only on the seed and the parameter's index.
  auto mix = [](uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  auto normal = [&](size_t k) {
    const uint64_t base = seed * 0x100000001B3ull;
    const double u1 = ((mix(base + 2 * k) >> 11) + 1.0) * (1.0 / 9007199254740993.0);  // (0, 1]
    const double u2 = (mix(base + 2 * k + 1) >> 11) * (1.0 / 9007199254740992.0);      // [0, 1)
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  };
  // Kaiming (fan-in, ReLU gain): W ~ N(0, 2 / (cin * taps)), biases 0
  auto conv = [&](int th_w, int th_b, int cout, int cin, int taps) {
    const double sd = std::sqrt(2.0 / ((double)cin * taps));
    for (size_t k = 0; k < (size_t)cout * cin * taps; ++k)
      theta[th_w + k] = (float)(sd * normal(th_w + k));
    for (int k = 0; k < cout; ++k) theta[th_b + k] = 0.f;
  };
  auto norm = [&](const Norm& nm, int c) {  // gamma 1, beta 0
    for (int k = 0; k < c; ++k) {
      theta[nm.th_g + k] = 1.f;
      theta[nm.th_b + k] = 0.f;
    }
  };
  conv(I.stem.th_w, I.stem.th_b, I.stem.cout, I.stem.cin_real, I.stem.taps);
  norm(I.stem_n, I.C);
  for (const Block& b : I.blocks) {
    conv(b.c1.th_w, b.c1.th_b, b.cout, b.cin, 27);
    norm(b.n1, b.cout);
    conv(b.c2.th_w, b.c2.th_b, b.cout, b.cout, 27);
    norm(b.n2, b.cout);
    if (b.proj) conv(b.pj.th_w, b.pj.th_b, b.cout, b.cin, 1);
  }
  conv(I.tail_w, I.tail_b, 1, I.C, 1);
  return D2IP_OK;
}

d2ip_status d2ip_init_params(d2ip_ctx* X, int inst, uint64_t seed) {
  d2ip_status st = check_inst(X, inst);
  if (st != D2IP_OK) return st;
  const Instance& I = X->insts[X->members[inst].first];
  std::vector<float> th(I.P);
  st = d2ip_init_params_host(I.L, I.C, seed, th.data(), th.size());
  if (st != D2IP_OK) return st;
  return d2ip_set_params(X, inst, th.data(), th.size(), 0);
}

d2ip_status d2ip_check_launches(const d2ip_geometry_desc* geos, int n_geo,
                                const d2ip_instance_desc* insts, int n_inst, int precision,
                                unsigned flags) {
  d2ip_status st = check_desc(geos, n_geo, insts, n_inst, precision);
  if (st != D2IP_OK) return st;
  Checker c;
  d2ip_ctx X;
  X.precision = precision;
  X.flags = flags;
  X.tv_on = true;  // walk the optional 4D-TV launches too
  Carver cv;
  cv.base = reinterpret_cast<char*>((uintptr_t)1 << 40);  // never dereferenced
  g_chk = &c;
  plan(X, geos, n_geo, insts, n_inst, cv);
  for (Geometry& G : X.geos) {
    G.qa = (int)G.Q;
    G.qa_pad = G.qa_cap;  // every voxel active: the largest extents
    G.set = true;
  }
  for (Instance& I : X.insts) {
    enqueue_iteration(X, I);
    L_pack(I, X.precision, false, 1, X.stream);
  }
  g_chk = nullptr;
  if (!c.errors.empty()) {
    std::string m;
    for (const std::string& e : c.errors) m += e + "; ";
    return fail(D2IP_EINVAL, m);
  }
  return D2IP_OK;
}

d2ip_status d2ip_set_tuning(const d2ip_tuning_entry* table, int count) {
  if (count < 0 || (count > 0 && !table)) return fail(D2IP_EINVAL, "bad tuning table");
  for (int i = 0; i < count; ++i) {
    std::string why;
    if (!shape_ok(table[i], &why))
      return fail(D2IP_EINVAL, "tuning entry " + std::to_string(i) + ": " + why);
  }
  g_tuning.assign(table, table + count);
  return D2IP_OK;
}

d2ip_status d2ip_plan_convs(const d2ip_geometry_desc* geos, int n_geo,
                            const d2ip_instance_desc* insts, int n_inst, int precision,
                            unsigned flags, int inst, d2ip_tuning_entry* out, int cap,
                            int* count) {
  d2ip_status st = check_desc(geos, n_geo, insts, n_inst, precision);
  if (st != D2IP_OK) return st;
  if (!count || cap < 0 || (cap > 0 && !out)) return fail(D2IP_EINVAL, "bad output");
  if (inst < 0 || inst >= n_inst) return fail(D2IP_EINVAL, "bad instance index");
  d2ip_ctx X;
  X.precision = precision;
  X.flags = flags;
  Carver cv;
  plan(X, geos, n_geo, insts, n_inst, cv);
  const Instance& I = X.insts[X.members[inst].first];
  std::vector<d2ip_tuning_entry> v;
  auto put = [&](const Conv& c) {
    d2ip_tuning_entry e;
    e.n = c.n;
    e.cin = c.cin;
    e.cout = c.cout;
    e.taps = c.taps;
    e.precision = precision;
    e.pass = 0;
    e.prologue = c.pro_fwd;
    e.shape = d2ip_conv_shape{c.fwd.tile, c.fwd.bn, c.fwd.ck, c.fwd.ksplit};
    v.push_back(e);
    if (c.dgrad) {
      e.pass = 1;
      e.prologue = c.pro_bwd;
      e.shape = d2ip_conv_shape{c.bwd.tile, c.bwd.bn, c.bwd.ck, c.bwd.ksplit};
      v.push_back(e);
    }
    e.pass = 2;
    e.prologue = c.pro_wg;
    e.shape = d2ip_conv_shape{c.wg_tile, 0, c.wg_ck, c.wg_splits};
    v.push_back(e);
  };
  put(I.stem);
  for (const Block& b : I.blocks) {
    put(b.c1);
    put(b.c2);
    if (b.proj) put(b.pj);
  }
  *count = (int)v.size();
  for (int i = 0; i < cap && i < (int)v.size(); ++i) out[i] = v[i];
  return D2IP_OK;
}

d2ip_status d2ip_time_conv_bytes(const d2ip_tuning_entry* e, size_t* out) {
  if (!e || !out) return fail(D2IP_EINVAL, "null argument");
  std::string why;
  if (!shape_ok(*e, &why)) return fail(D2IP_EINVAL, why);
  Carver cv;
  TimeConvBufs b;
  carve_time_conv(*e, cv, b);
  *out = cv.off + 256;
  return D2IP_OK;
}

d2ip_status d2ip_time_conv(const d2ip_tuning_entry* e, void* workspace, size_t bytes,
                           void* hip_stream, int reps, double* avg_ms) {
  if (!e || !workspace || !avg_ms || reps <= 0) return fail(D2IP_EINVAL, "bad argument");
  if (((uintptr_t)workspace & 255) != 0) return fail(D2IP_EINVAL, "workspace not 256-byte aligned");
  size_t need = 0;
  d2ip_status st = d2ip_time_conv_bytes(e, &need);
  if (st != D2IP_OK) return st;
  if (bytes < need) return fail(D2IP_ENOMEM, "workspace too small: need " + std::to_string(need));
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  Carver cv;
  cv.base = reinterpret_cast<char*>(workspace);
  TimeConvBufs b;
  carve_time_conv(*e, cv, b);
  HIPCHK(hipMemsetAsync(workspace, 0, cv.off, s));
  const int prec = conv_prec(e->precision);
  const int n = e->n;
  const double cnt = (double)n * n * n;
  auto launch = [&]() {
    if (e->pass == 2) {
      ConvWgrad a;
      std::memset(&a, 0, sizeof(a));
      a.src = ConvSrc{b.x, e->cin, e->prologue / 3, PairRef{b.st, 1, cnt * e->cin}, b.gamma,
                      b.beta, nullptr, PairRef{}};
      a.gsrc = ConvSrc{b.g, e->cout, e->prologue % 3, PairRef{b.st, 1, cnt * e->cout}, b.gamma,
                       nullptr, b.h, PairRef{b.st, 1, cnt * e->cout}};
      a.n = n;
      a.cin = e->cin;
      a.cout = e->cout;
      a.taps = e->taps;
      a.part = b.part;
      a.partb = b.partb;
      a.splits = e->shape.split;
      a.prec = prec;
      a.tile = e->shape.tile;
      a.ck = e->shape.ck;
      a.batch = 1;
      conv_wgrad(a, s);
    } else {
      const int kin = e->pass == 0 ? e->cin : e->cout, kout = e->pass == 0 ? e->cout : e->cin;
      ConvFwd a;
      std::memset(&a, 0, sizeof(a));
      a.src = ConvSrc{b.x, kin, e->prologue, PairRef{b.st, 1, cnt * kin}, b.gamma, b.beta, b.h,
                      PairRef{b.st, 1, cnt * kin}};
      a.n = n;
      a.cin = kin;
      a.w = b.w;
      a.w_lo_off = prec == PREC_BF16X3 ? (long long)kout * e->taps * kin : 0;
      a.w_rows = kout;
      a.bias = e->pass == 0 ? b.bias : nullptr;
      a.cout = kout;
      a.y = b.y;
      a.taps = e->taps;
      a.stat_part = e->pass == 0 ? b.stat : nullptr;
      a.prec = prec;
      a.tile = e->shape.tile;
      a.bn = e->shape.bn;
      a.ck = e->shape.ck;
      a.ksplit = e->shape.split;
      a.kpart = b.kpart;
      a.batch = 1;
      conv_fwd(a, s);
    }
  };
  launch();
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r) launch();
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(hipGetLastError());
  *avg_ms = (double)ms / reps;
  return D2IP_OK;
}

d2ip_status d2ip_workspace_bytes(const d2ip_geometry_desc* geos, int n_geo,
                                 const d2ip_instance_desc* insts, int n_inst, int precision,
                                 unsigned flags, size_t* out) {
  if (!out) return fail(D2IP_EINVAL, "null output");
  d2ip_status st = check_desc(geos, n_geo, insts, n_inst, precision);
  if (st != D2IP_OK) return st;
  d2ip_ctx X;
  X.precision = precision;
  X.flags = flags;
  Carver cv;
  plan(X, geos, n_geo, insts, n_inst, cv);
  *out = (cv.off + 255) & ~size_t(255);
  return D2IP_OK;
}

d2ip_status d2ip_create(const d2ip_geometry_desc* geos, int n_geo, const d2ip_instance_desc* insts,
                        int n_inst, int precision, unsigned flags, void* workspace, size_t bytes,
                        void* hip_stream, d2ip_ctx** out) {
  if (!out) return fail(D2IP_EINVAL, "null output");
  *out = nullptr;
  size_t need = 0;
  d2ip_status st = d2ip_workspace_bytes(geos, n_geo, insts, n_inst, precision, flags, &need);
  if (st != D2IP_OK) return st;
  if (!workspace) return fail(D2IP_EINVAL, "null workspace");
  if (((uintptr_t)workspace & 255) != 0) return fail(D2IP_EINVAL, "workspace not 256-byte aligned");
  if (bytes < need)
    return fail(D2IP_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes, got " +
                                 std::to_string(bytes));
  d2ip_ctx* X = new d2ip_ctx();
  X->precision = precision;
  X->flags = flags;
  X->stream = reinterpret_cast<hipStream_t>(hip_stream);
  X->bytes = bytes;
  Carver cv;
  cv.base = reinterpret_cast<char*>(workspace);
  plan(*X, geos, n_geo, insts, n_inst, cv);
  auto cleanup = [&](d2ip_status s) {
    release_lanes(X);
    if (X->ev_pj) (void)hipEventDestroy(X->ev_pj);
    if (X->ev_join) (void)hipEventDestroy(X->ev_join);
    if (X->ev_fork) (void)hipEventDestroy(X->ev_fork);
    if (X->side) (void)hipStreamDestroy(X->side);
    if (X->cap) (void)hipStreamDestroy(X->cap);
    delete X;
    return s;
  };
  // zero everything once: padding of packed weights and J, state
  hipError_t e = hipMemsetAsync(workspace, 0, need, X->stream);
  if (e == hipSuccess) {
    for (Instance& I : X->insts) {
      e = hipMemcpyAsync(I.packs_dev, I.packs.data(), I.packs.size() * sizeof(ConvPack),
                         hipMemcpyHostToDevice, X->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(I.segs_dev, I.segs.data(), I.segs.size() * sizeof(GradSeg),
                           hipMemcpyHostToDevice, X->stream);
      if (e != hipSuccess) break;
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(X->stream);
  if (e == hipSuccess && (flags & D2IP_FLAG_GRAPH))
    e = hipStreamCreateWithFlags(&X->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&X->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&X->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&X->ev_join, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&X->ev_pj, hipEventDisableTiming);
  if (e == hipSuccess && X->insts.size() > 1) {
    e = hipEventCreateWithFlags(&X->ev_start, hipEventDisableTiming);
    X->lanes.resize(std::min<size_t>(X->insts.size(), kMaxLanes));
    for (d2ip_ctx::Lane& l : X->lanes) {
      if (e == hipSuccess) e = hipStreamCreateWithFlags(&l.main, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipStreamCreateWithFlags(&l.side, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&l.fork, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&l.join, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&l.done, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&l.pj, hipEventDisableTiming);
    }
  }
  if (e != hipSuccess)
    return cleanup(fail(D2IP_EHIP, std::string("workspace init: ") + hipGetErrorString(e)));
  *out = X;
  return D2IP_OK;
}

d2ip_status d2ip_destroy(d2ip_ctx* X) {
  if (!X) return D2IP_OK;
  (void)hipStreamSynchronize(X->stream);
  drop_graph(X);
  if (X->side) (void)hipStreamSynchronize(X->side);
  for (d2ip_ctx::Lane& l : X->lanes) {
    if (l.main) (void)hipStreamSynchronize(l.main);
    if (l.side) (void)hipStreamSynchronize(l.side);
  }
  release_lanes(X);
  if (X->ev_pj) (void)hipEventDestroy(X->ev_pj);
  if (X->ev_join) (void)hipEventDestroy(X->ev_join);
  if (X->ev_fork) (void)hipEventDestroy(X->ev_fork);
  if (X->side) (void)hipStreamDestroy(X->side);
  if (X->cap) (void)hipStreamDestroy(X->cap);
  delete X;
  return D2IP_OK;
}

d2ip_status d2ip_set_geometry(d2ip_ctx* X, int geo, const float* J, const uint8_t* mask,
                              int on_device) {
  if (!X) return fail(D2IP_EINVAL, "null context");
  if (geo < 0 || geo >= (int)X->geos.size()) return fail(D2IP_EINVAL, "bad geometry index");
  if (!J || !mask) return fail(D2IP_EINVAL, "null J or mask");
  Geometry& G = X->geos[geo];
  std::vector<uint8_t> hm(G.Q);
  StreamDrain drain_mask{X->stream};
  if (on_device) {
    HIPCHK(hipMemcpyAsync(hm.data(), mask, G.Q, hipMemcpyDeviceToHost, X->stream));
    HIPCHK(hipStreamSynchronize(X->stream));
  } else {
    std::memcpy(hm.data(), mask, G.Q);
  }
  std::vector<int> idx;
  std::vector<int> inv(G.Q, -1);
  std::vector<float> maskf(G.Q, 0.f);
  for (size_t q = 0; q < G.Q; ++q)
    if (hm[q]) {
      inv[q] = (int)idx.size();
      idx.push_back((int)q);
      maskf[q] = 1.f;
    }
  if (idx.empty()) return fail(D2IP_EINVAL, "mask selects no voxel");
  const int qa = (int)idx.size();
  const int qa_pad = (qa + 63) / 64 * 64;
  std::vector<int> idxp(qa_pad, idx[0]);
  std::copy(idx.begin(), idx.end(), idxp.begin());
  std::vector<float> jc;  // compacted J (host input)
  // the host buffers above are the sources of asynchronous copies: every
  // return below waits for the stream before they are freed
  StreamDrain drain{X->stream};
  HIPCHK(hipMemcpyAsync(G.idx, idxp.data(), qa_pad * sizeof(int), hipMemcpyHostToDevice, X->stream));
  HIPCHK(hipMemcpyAsync(G.inv, inv.data(), G.Q * sizeof(int), hipMemcpyHostToDevice, X->stream));
  HIPCHK(hipMemcpyAsync(G.mask, maskf.data(), G.Q * sizeof(float), hipMemcpyHostToDevice, X->stream));
  if (on_device) {
    gather_columns(J, G.M, (int)G.Q, G.idx, qa, qa_pad, G.Jc, X->stream);
    HIPCHK(hipGetLastError());
  } else {
    jc.assign((size_t)G.M * qa_pad, 0.f);
    for (int m = 0; m < G.M; ++m) {
      const float* row = J + (size_t)m * G.Q;
      float* dst = jc.data() + (size_t)m * qa_pad;
      for (int q = 0; q < qa; ++q) dst[q] = row[idx[q]];
    }
    HIPCHK(hipMemcpyAsync(G.Jc, jc.data(), jc.size() * sizeof(float), hipMemcpyHostToDevice,
                          X->stream));
  }
  HIPCHK(hipStreamSynchronize(X->stream));
  G.qa = qa;
  G.qa_pad = qa_pad;
  G.set = true;
  drop_graph(X);
  return D2IP_OK;
}

d2ip_status d2ip_set_params(d2ip_ctx* X, int inst, const float* theta, size_t n, int on_device) {
  d2ip_status st = check_inst(X, inst);
  if (st != D2IP_OK) return st;
  Instance& I = X->insts[X->members[inst].first];
  const int mb = X->members[inst].second;
  const long long mo = (long long)mb * I.istride;
  if (!theta || n != I.P)
    return fail(D2IP_EINVAL, "theta must hold " + std::to_string(I.P) + " floats");
  st = copy_in(X, ishift(I.theta, mo), theta, n * sizeof(float), on_device);
  if (st != D2IP_OK) return st;
  zero_words(&ishift(I.it, mo)->nonfinite, 1, X->stream);  // new parameters, no stale flag
  return repack(X, I);
}

d2ip_status d2ip_get_params(d2ip_ctx* X, int inst, float* theta, size_t n, int on_device) {
  d2ip_status st = check_inst(X, inst);
  if (st != D2IP_OK) return st;
  Instance& I = X->insts[X->members[inst].first];
  const int mb = X->members[inst].second;
  const long long mo = (long long)mb * I.istride;
  if (!theta || n != I.P)
    return fail(D2IP_EINVAL, "theta must hold " + std::to_string(I.P) + " floats");
  return copy_out(X, theta, ishift(I.theta, mo), n * sizeof(float), on_device);
}

d2ip_status d2ip_get_grad(d2ip_ctx* X, int inst, float* grad, size_t n, int on_device) {
  d2ip_status st = check_inst(X, inst);
  if (st != D2IP_OK) return st;
  Instance& I = X->insts[X->members[inst].first];
  const int mb = X->members[inst].second;
  const long long mo = (long long)mb * I.istride;
  if (!grad || n != I.P)
    return fail(D2IP_EINVAL, "grad must hold " + std::to_string(I.P) + " floats");
  return copy_out(X, grad, ishift(I.grad, mo), n * sizeof(float), on_device);
}

d2ip_status d2ip_set_noise_input(d2ip_ctx* X, int inst, const float* z, int on_device) {
  d2ip_status st = check_inst(X, inst);
  if (st != D2IP_OK) return st;
  if (!z) return fail(D2IP_EINVAL, "null Z");
  Instance& I = X->insts[X->members[inst].first];
  const int mb = X->members[inst].second;
  const long long mo = (long long)mb * I.istride;
  // stage Z in the sigma buffer, then spread it into the padded input
  st = copy_in(X, ishift(I.sigma, mo), z, I.V0 * sizeof(float), on_device);
  if (st != D2IP_OK) return st;
  pad_input(ishift(I.sigma, mo), I.V0, ishift(I.zpad, mo), X->stream);
  HIPCHK(hipGetLastError());
  I.has_z[mb] = 1;
  return D2IP_OK;
}

d2ip_status d2ip_set_frame(d2ip_ctx* X, int inst, const float* dv, int on_device) {
  d2ip_status st = check_inst(X, inst);
  if (st != D2IP_OK) return st;
  if (!dv) return fail(D2IP_EINVAL, "null dv");
  Instance& I = X->insts[X->members[inst].first];
  const int mb = X->members[inst].second;
  const long long mo = (long long)mb * I.istride;
  const int M = X->geos[I.geo].M;
  if (!on_device) {
    for (int m = 0; m < M; ++m)
      if (!std::isfinite(dv[m])) return fail(D2IP_ENONFINITE, "dv holds a non-finite value");
  }
  st = copy_in(X, ishift(I.dv, mo), dv, M * sizeof(float), on_device);
  if (st != D2IP_OK) return st;
  I.has_frame[mb] = 1;
  return D2IP_OK;
}

d2ip_status d2ip_set_adam(d2ip_ctx* X, const d2ip_adam_cfg* cfg) {
  if (!X || !cfg) return fail(D2IP_EINVAL, "null argument");
  if (!(cfg->lr > 0.f) || !(cfg->beta1 >= 0.f && cfg->beta1 < 1.f) ||
      !(cfg->beta2 >= 0.f && cfg->beta2 < 1.f) || !(cfg->eps > 0.f))
    return fail(D2IP_EINVAL, "Adam needs lr > 0, 0 <= beta < 1, eps > 0");
  X->lr = cfg->lr;
  X->b1 = cfg->beta1;
  X->b2 = cfg->beta2;
  X->eps = cfg->eps;
  drop_graph(X);
  return D2IP_OK;
}

d2ip_status d2ip_reset_optimizer(d2ip_ctx* X, int inst) {
  d2ip_status st = check_inst(X, inst);
  if (st != D2IP_OK) return st;
  Instance& I = X->insts[X->members[inst].first];
  const int mb = X->members[inst].second;
  const long long mo = (long long)mb * I.istride;
  zero_words(ishift(I.m, mo), I.P, X->stream);
  zero_words(ishift(I.v, mo), I.P, X->stream);
  zero_words(&ishift(I.it, mo)->t, 1, X->stream);
  HIPCHK(hipGetLastError());
  return D2IP_OK;
}

d2ip_status d2ip_get_state(d2ip_ctx* X, int inst, float* tmv, int64_t* t, int on_device) {
  d2ip_status st = check_inst(X, inst);
  if (st != D2IP_OK) return st;
  if (!tmv || !t) return fail(D2IP_EINVAL, "null argument");
  Instance& I = X->insts[X->members[inst].first];
  const int mb = X->members[inst].second;
  const long long mo = (long long)mb * I.istride;
  const size_t b = I.P * sizeof(float);
  const hipMemcpyKind k = kind_from_dev(on_device);
  HIPCHK(hipMemcpyAsync(tmv, ishift(I.theta, mo), b, k, X->stream));
  HIPCHK(hipMemcpyAsync(tmv + I.P, ishift(I.m, mo), b, k, X->stream));
  HIPCHK(hipMemcpyAsync(tmv + 2 * I.P, ishift(I.v, mo), b, k, X->stream));
  int tt = 0;
  StreamDrain drain{X->stream};
  HIPCHK(hipMemcpyAsync(&tt, &ishift(I.it, mo)->t, sizeof(int), hipMemcpyDeviceToHost, X->stream));
  HIPCHK(hipStreamSynchronize(X->stream));
  *t = tt;
  return D2IP_OK;
}

d2ip_status d2ip_set_state(d2ip_ctx* X, int inst, const float* tmv, int64_t t, int on_device) {
  d2ip_status st = check_inst(X, inst);
  if (st != D2IP_OK) return st;
  if (!tmv || t < 0 || t > (int64_t)1 << 30) return fail(D2IP_EINVAL, "bad state");
  Instance& I = X->insts[X->members[inst].first];
  const int mb = X->members[inst].second;
  const long long mo = (long long)mb * I.istride;
  const size_t b = I.P * sizeof(float);
  const hipMemcpyKind k = kind_to_dev(on_device);
  int tt = (int)t;
  StreamDrain drain{X->stream};
  HIPCHK(hipMemcpyAsync(ishift(I.theta, mo), tmv, b, k, X->stream));
  HIPCHK(hipMemcpyAsync(ishift(I.m, mo), tmv + I.P, b, k, X->stream));
  HIPCHK(hipMemcpyAsync(ishift(I.v, mo), tmv + 2 * I.P, b, k, X->stream));
  HIPCHK(hipMemcpyAsync(&ishift(I.it, mo)->t, &tt, sizeof(int), hipMemcpyHostToDevice, X->stream));
  zero_words(&ishift(I.it, mo)->nonfinite, 1, X->stream);
  HIPCHK(hipStreamSynchronize(X->stream));
  return repack(X, I);
}

d2ip_status d2ip_run(d2ip_ctx* X, int k, double* last_loss) {
  if (!X) return fail(D2IP_EINVAL, "null context");
  if (k < 0) return fail(D2IP_EINVAL, "k must be >= 0");
  for (size_t i = 0; i < X->members.size(); ++i) {
    const Instance& I = X->insts[X->members[i].first];
    const int mb = X->members[i].second;
    if (!X->geos[I.geo].set)
      return fail(D2IP_ESTATE, "geometry " + std::to_string(I.geo) + " not set");
    if (!I.has_z[mb])
      return fail(D2IP_ESTATE, "instance " + std::to_string(i) + ": noise input not set");
    if (!I.has_frame[mb])
      return fail(D2IP_ESTATE, "instance " + std::to_string(i) + ": frame not set");
  }
  if (k > 0) {
    if (X->flags & D2IP_FLAG_GRAPH) {
      if (!X->gexec) {
        // record one iteration of every instance on the capture stream; the
        // graph is then launched on the caller's stream
        hipStream_t user = X->stream;
        X->stream = X->cap;
        hipError_t e = hipStreamBeginCapture(X->cap, hipStreamCaptureModeThreadLocal);
        hipGraph_t g = nullptr;
        if (e == hipSuccess) {
          enqueue_all(*X, true);
          e = hipStreamEndCapture(X->cap, &g);
        }
        X->stream = user;
        if (e != hipSuccess) return fail(D2IP_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        X->graph = g;
        HIPCHK(hipGraphInstantiate(&X->gexec, X->graph, nullptr, nullptr, 0));
      }
      for (int i = 0; i < k; ++i) HIPCHK(hipGraphLaunch(X->gexec, X->stream));
    } else {
      for (int i = 0; i < k; ++i) enqueue_all(*X, false);
      HIPCHK(hipGetLastError());
    }
  }
  if (last_loss) {
    bool bad = false;
    for (size_t i = 0; i < X->members.size(); ++i) {
      const Instance& I = X->insts[X->members[i].first];
      const long long mo = (long long)X->members[i].second * I.istride;
      IterState h;
      StreamDrain drain{X->stream};
      HIPCHK(hipMemcpyAsync(&h, ishift(I.it, mo), sizeof(h), hipMemcpyDeviceToHost, X->stream));
      HIPCHK(hipStreamSynchronize(X->stream));
      last_loss[i] = h.loss;
      if (h.nonfinite) bad = true;
    }
    if (bad) return fail(D2IP_ENONFINITE, "a non-finite loss or parameter was produced");
  }
  return D2IP_OK;
}

d2ip_status d2ip_time_kernel(d2ip_ctx* X, int inst, int which, int block, int reps,
                             double* avg_ms) {
  d2ip_status st = check_inst(X, inst);
  if (st != D2IP_OK) return st;
  if (!avg_ms || reps <= 0) return fail(D2IP_EINVAL, "need reps > 0 and an output");
  Instance& I = X->insts[X->members[inst].first];
  const int mb = X->members[inst].second;
  const long long mo = (long long)mb * I.istride;
  const Geometry& G = X->geos[I.geo];
  for (int b = 0; b < I.B; ++b)
    if (!G.set || !I.has_frame[b] || !I.has_z[b])
      return fail(D2IP_ESTATE, "every instance of the group must be ready");
  (void)mo;
  hipStream_t s = X->stream;
  Block* b = nullptr;
  if (which >= D2IP_KERNEL_CONV_FWD) {
    if (block < 0 || block >= (int)I.blocks.size()) return fail(D2IP_EINVAL, "bad block index");
    b = &I.blocks[block];
  }
  Level* Lv = b ? &I.lv[b->level] : nullptr;
  auto launch = [&]() {
    switch (which) {
      case D2IP_KERNEL_JVEC:
        jvec(G.Jc, G.M, G.qa_pad, G.idx, I.sigma, I.ppart, I.B, I.istride, s);
        break;
      case D2IP_KERNEL_JTVEC:
        jtvec(G.Jc, G.M, G.qa_pad, I.ppart, jvec_qblocks(G.qa_pad), I.dv, I.rsum, I.tpart, I.B,
              I.istride, s);
        break;
      case D2IP_KERNEL_ADAM:
        adam(I.theta, I.grad, I.m, I.v, I.P, X->lr, X->b1, X->b2, X->eps, I.it, I.B, I.istride, s);
        break;
      case D2IP_KERNEL_CONV_FWD:
        conv_fwd(fwd_args(*X, I, b->c1, src_plain(b->x, b->cin), b->h1, &b->st1), s);
        break;
      case D2IP_KERNEL_CONV_DGRAD: {
        const float* th = I.theta;
        conv_fwd(dgrad_args(*X, I, b->c1,
                            src_ln_bwd(b->ga, b->h1, b->cout, b->st1, th + b->n1.th_g, b->cb1),
                            Lv->gx),
                 s);
        break;
      }
      default: {
        const float* th = I.theta;
        wgrad(*X, I, b->c1, src_plain(b->x, b->cin),
              src_ln_bwd(b->ga, b->h1, b->cout, b->st1, th + b->n1.th_g, b->cb1), s);
        break;
      }
    }
  };
  if (which < D2IP_KERNEL_JVEC || which > D2IP_KERNEL_CONV_WGRAD)
    return fail(D2IP_EINVAL, "unknown kernel id");
  launch();
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r) launch();
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(hipGetLastError());
  *avg_ms = (double)ms / reps;
  return D2IP_OK;
}

d2ip_status d2ip_set_tv(d2ip_ctx* X, const d2ip_tv_cfg* cfg) {
  if (!X || !cfg) return fail(D2IP_EINVAL, "null argument");
  if (!(cfg->lambda_tv >= 0.f) || !(cfg->lambda_s >= 0.f) || !(cfg->lambda_t >= 0.f) ||
      !(cfg->eps > 0.f))
    return fail(D2IP_EINVAL, "4D-TV needs lambda_tv, lambda_s, lambda_t >= 0 and eps > 0");
  X->tv_on = cfg->lambda_tv > 0.f;
  X->tv = TvCoef{cfg->lambda_tv, cfg->lambda_s, cfg->lambda_t, cfg->eps};
  drop_graph(X);
  return D2IP_OK;
}

namespace {
// Upload member mb's history ring state with weights exp(-k) / sum, k = 1..count.
d2ip_status put_tv_state(d2ip_ctx* X, Instance& I, int mb) {
  TvState t;
  std::memset(&t, 0, sizeof(t));
  t.count = I.tv_count[mb];
  t.head = I.tv_head[mb];
  double sum = 0.0;
  for (int k = 1; k <= t.count; ++k) sum += std::exp(-(double)k);
  for (int k = 1; k <= t.count; ++k) t.w[k - 1] = (float)(std::exp(-(double)k) / sum);
  StreamDrain drain{X->stream};
  HIPCHK(hipMemcpyAsync(ishift(I.tvs, (long long)mb * I.istride), &t, sizeof(t),
                        hipMemcpyHostToDevice, X->stream));
  HIPCHK(hipStreamSynchronize(X->stream));
  return D2IP_OK;
}
}  // namespace

d2ip_status d2ip_commit_frame(d2ip_ctx* X, int inst) {
  d2ip_status st = check_inst(X, inst);
  if (st != D2IP_OK) return st;
  Instance& I = X->insts[X->members[inst].first];
  const int mb = X->members[inst].second;
  const long long mo = (long long)mb * I.istride;
  if (!X->geos[I.geo].set) return fail(D2IP_ESTATE, "geometry not set");
  for (int b = 0; b < I.B; ++b)
    if (!I.has_z[b]) return fail(D2IP_ESTATE, "noise input not set");
  enqueue_forward(*X, I);  // the image at the current theta
  const int slot = (I.tv_head[mb] + 1) % kTvHistory;
  HIPCHK(hipMemcpyAsync(ishift(I.hist, mo) + (size_t)slot * I.V0, ishift(I.sigma, mo),
                        I.V0 * sizeof(float), hipMemcpyDeviceToDevice, X->stream));
  I.tv_head[mb] = slot;
  I.tv_count[mb] = std::min(I.tv_count[mb] + 1, kTvHistory);
  return put_tv_state(X, I, mb);
}

d2ip_status d2ip_clear_history(d2ip_ctx* X, int inst) {
  d2ip_status st = check_inst(X, inst);
  if (st != D2IP_OK) return st;
  Instance& I = X->insts[X->members[inst].first];
  const int mb = X->members[inst].second;
  I.tv_count[mb] = 0;
  I.tv_head[mb] = kTvHistory - 1;
  return put_tv_state(X, I, mb);
}

d2ip_status d2ip_read_image(d2ip_ctx* X, int inst, float* sigma, int on_device) {
  d2ip_status st = check_inst(X, inst);
  if (st != D2IP_OK) return st;
  if (!sigma) return fail(D2IP_EINVAL, "null output");
  Instance& I = X->insts[X->members[inst].first];
  const int mb = X->members[inst].second;
  const long long mo = (long long)mb * I.istride;
  if (!X->geos[I.geo].set) return fail(D2IP_ESTATE, "geometry not set");
  for (int b = 0; b < I.B; ++b)
    if (!I.has_z[b]) return fail(D2IP_ESTATE, "noise input not set");
  enqueue_forward(*X, I);
  HIPCHK(hipGetLastError());
  return copy_out(X, sigma, ishift(I.sigma, mo), I.V0 * sizeof(float), on_device);
}

}  // extern "C"
