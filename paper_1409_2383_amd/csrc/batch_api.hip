// C-ABI host layer of the batched solver: validation, workspace carving,
// tile choice (defaults, autotuner, caller-supplied), the work list and the
// captured graph of one outer iteration (a counter reset and the persistent
// kernel of batch.hip).
#include "../../include/ntf_admm.h"
#include "batch.h"
#include "ntf_launch.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

using namespace ntf;

namespace {

constexpr int kMaxSpi1 = 16;          // pass-1 slabs per item (LDS for the W1 partials)
constexpr int64_t kDefaultElems1 = 256 * 1024;
constexpr int64_t kDefaultElems3 = 1024 * 1024;
constexpr int kInnerRowsPerItem = 64;   // rows of one inner-sweep work item (at least one block; 32 measured 0.6% slower)
constexpr long long kSpinLimit = 1ll << 22;   // polls (>= 50 ns each) before a wait gives up
constexpr size_t kLdsMax = 156 * 1024;   // dynamic LDS; the kernel also has ~2 KB static

int rup(int x, int a) { return (x + a - 1) / a * a; }
size_t align256(size_t x) { return (x + 255) / 256 * 256; }

int qbucket(int q) { return q <= 128 ? 0 : q <= 256 ? 1 : q <= 512 ? 2 : 3; }

typedef std::tuple<int, int, int> TileKey;   // kind (1 or 3), ft, qbucket
struct TileVal {
  int mt;
  int64_t elems;
  double us;
};

int cus() {
  static int cached = 0;
  if (!cached) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      cached = n;
    else
      cached = 256;
  }
  return cached;
}

struct ProbLayout {
  size_t xr, xt, scale, T, W[3], W3p, gram[3], gpart, ginv, rho, end;
};

}  // namespace

struct ntf_batch_ctx {
  int n = 0;
  ntf_opts opts{};
  std::vector<ntf_problem> probs;
  std::vector<BProb> hp;
  std::vector<ProbLayout> lay;
  std::map<TileKey, TileVal> tiles;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  // global pieces of the workspace
  BProb* dprobs = nullptr;
  uint2* ditems = nullptr;      // main list
  uint2* dkind[3] = {nullptr, nullptr, nullptr};   // pass-1, mode-2, pass-3 lists
  int64_t cap_main = 0, cap_kind[3] = {0, 0, 0};
  int* ctr = nullptr;           // [n][kCtrPerProb] then the ticket counter
  int* flag = nullptr;
  double* fitpart = nullptr;
  double* fitout = nullptr;     // [n][2]
  unsigned long long* prof = nullptr;   // [BK_NKINDS][3] profile counters
  int n_items = 0, n_kind[3] = {0, 0, 0};
  int64_t by_kind[BK_NKINDS] = {};
  int grid = 0;
  size_t lds = 0;
  hipStream_t s0 = nullptr, sc = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::string err;
};

#define NTFB_HIP(ctx, call)                                                           \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      if (ctx) (ctx)->err = std::string(#call) + ": " + hipGetErrorString(e_);       \
      return NTF_E_HIP;                                                               \
    }                                                                                 \
  } while (0)

static thread_local std::string g_batch_err;

static int fl_of(int F) {
  int fl = 4;
  while (fl < F) fl *= 2;
  return fl;
}

// Sizes of one problem's descriptor that do not depend on the tiles.
static BProb base_prob(const ntf_problem& pr) {
  BProb b;
  std::memset(&b, 0, sizeof(b));
  b.I = (int)pr.dims[0];
  b.J = (int)pr.dims[1];
  b.K = (int)pr.dims[2];
  b.F = pr.F;
  b.FT = (pr.F + 15) / 16;
  b.FL = fl_of(pr.F);
  b.NB = (pr.F + 15) / 16;
  b.Kp = rup(b.K, 32);
  b.Jp = rup(b.J, 32);
  b.rpb = batch_inner_rows(b.FL);
  const int d[3] = {b.I, b.J, b.K};
  b.ipi = std::max(1, kInnerRowsPerItem / b.rpb);
  for (int m = 0; m < 3; ++m) {
    b.n_in[m] = (d[m] + b.rpb - 1) / b.rpb;
    b.ni[m] = (b.n_in[m] + b.ipi - 1) / b.ipi;
  }
  b.n_m2 = (b.J + 63) / 64;
  return b;
}

static TileVal default_tile(int kind, const BProb& b) {
  const int rows = (kind == 1) ? b.J : b.K;
  return TileVal{rows >= 64 ? 2 : 1, kind == 1 ? kDefaultElems1 : kDefaultElems3, 0.0};
}

static TileKey key_of(int kind, const BProb& b) {
  return TileKey(kind, b.FT, qbucket(kind == 1 ? b.K : b.J));
}

// Tile-dependent fields of a descriptor.
static void apply_tiles(BProb& b, const TileVal& t1, const TileVal& t3) {
  const int64_t slab = (int64_t)b.J * b.K;
  b.mt1 = t1.mt;
  b.spi1 = (int)std::max<int64_t>(1, std::min<int64_t>({t1.elems / slab, kMaxSpi1, (int64_t)b.I}));
  b.n_p1 = (b.I + b.spi1 - 1) / b.spi1;
  b.mt3 = t3.mt;
  b.spi3 = (int)std::max<int64_t>(1, std::min<int64_t>(t3.elems / slab, (int64_t)b.I));
  b.n_p3 = (b.I + b.spi3 - 1) / b.spi3;
}

// LDS of the largest item a problem can have under any tile choice.
static size_t max_lds(const BProb& b) {
  BProb t = b;
  t.spi1 = std::min(kMaxSpi1, b.I);
  return std::max({batch_lds_p1(t), batch_lds_p3(b), batch_lds_inner(b.FL), batch_lds_prep()});
}

static size_t lds_of(const BProb& b) {
  return std::max({batch_lds_p1(b), batch_lds_p3(b), batch_lds_inner(b.FL), batch_lds_prep()});
}

static ntf_status validate(const ntf_problem* probs, int32_t n, const ntf_opts* o, std::string* why) {
  auto fail = [&](const std::string& m, ntf_status s = NTF_E_INVAL) {
    if (why) *why = m;
    return s;
  };
  if (!probs || !o || n < 1) return fail("null problems/options or n < 1");
  if (n > 65536) return fail("at most 65536 problems");
  if (o->precision != NTF_PREC_BF16_MIXED)
    return fail("the batched solver implements NTF_PREC_BF16_MIXED only", NTF_E_UNSUPPORTED);
  if (o->inner_iters < 1) return fail("inner_iters must be >= 1");
  if (o->rho_policy != NTF_RHO_TRACE && o->rho_policy != NTF_RHO_FIXED)
    return fail("the batched solver supports rho_policy TRACE or FIXED", NTF_E_UNSUPPORTED);
  if (!(o->rho0 > 0.0)) return fail("rho0 must be > 0");
  if (o->inner_eps_abs < 0 || o->inner_eps_rel < 0) return fail("tolerances must be >= 0");
  if (o->factor_source != 0 || o->paper_init != 0 || o->warm_hidden != 0 || o->stop_eps_abs != 0 ||
      o->stop_eps_rel != 0)
    return fail("factor_source, paper_init, warm_hidden and stop_eps_* must be 0", NTF_E_UNSUPPORTED);
  for (int q = 0; q < 3; ++q)
    if (o->reserved[q] != 0) return fail("reserved fields must be zero");
  for (int32_t p = 0; p < n; ++p) {
    const ntf_problem& pr = probs[p];
    const std::string at = " (problem " + std::to_string(p) + ")";
    for (int m = 0; m < 3; ++m)
      if (pr.dims[m] < 1 || pr.dims[m] > 65535) return fail("dims must be in [1, 65535]" + at);
    if (pr.F < 1 || pr.F > 64) return fail("F must be in [1, 64]" + at);
    if (pr.x_dtype != 0) return fail("x_dtype must be 0 (float32)" + at);
    if (!pr.X || ((uintptr_t)pr.X & 15)) return fail("X null or not 16-byte aligned" + at);
    for (int m = 0; m < 3; ++m)
      if (!pr.H[m] || !pr.U[m] || ((((uintptr_t)pr.H[m]) | ((uintptr_t)pr.U[m])) & 15))
        return fail("factor/dual null or not 16-byte aligned" + at);
    if (pr.dims[0] * pr.dims[1] * pr.dims[2] > ((int64_t)1 << 40)) return fail("tensor too large" + at);
    const BProb b = base_prob(pr);
    // the work items address one slab, a factor or a partial of W3 through
    // 32-bit byte offsets (plus a tile of rows past the end)
    if ((int64_t)(b.J + 64) * b.Kp * 2 >= kBufferOOB || (int64_t)(b.K + 64) * b.Jp * 2 >= kBufferOOB ||
        (int64_t)(std::max({b.I, b.J, b.K}) + 64) * b.F * 4 >= kBufferOOB)
      return fail("the batched solver takes slabs J x K and factors under 1 GiB" + at, NTF_E_UNSUPPORTED);
    if (max_lds(b) > kLdsMax)
      return fail("work items of this shape exceed the LDS" + at, NTF_E_UNSUPPORTED);
  }
  return NTF_OK;
}

// Workspace: per-problem blocks, then the shared pieces.
struct BatchLayout {
  std::vector<ProbLayout> probs;
  size_t dprobs = 0, items = 0, kind[3] = {0, 0, 0}, ctr = 0, flag = 0, fitpart = 0, fitout = 0,
         prof = 0, total = 0;
  int64_t cap_main = 0, cap_kind[3] = {0, 0, 0};
};

static BatchLayout make_layout(const ntf_problem* probs, int32_t n) {
  BatchLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  int64_t maxfit = 1;
  for (int32_t p = 0; p < n; ++p) {
    const BProb b = base_prob(probs[p]);
    const int64_t I = b.I, J = b.J, K = b.K, F = b.F;
    ProbLayout pl;
    pl.xr = take((size_t)(I * J * b.Kp) * 2);
    pl.xt = take((size_t)(I * K * b.Jp) * 2);
    pl.scale = take((size_t)I * 4);
    pl.T = take((size_t)(I * J * F) * 4);
    const int64_t d[3] = {I, J, K};
    for (int m = 0; m < 3; ++m) pl.W[m] = take((size_t)(d[m] * F) * 8);
    pl.W3p = take((size_t)(I * K * F) * 4);     // up to one partial per slab
    for (int m = 0; m < 3; ++m) pl.gram[m] = take((size_t)(F * F) * 8);
    const int maxin = std::max({b.n_in[0], b.n_in[1], b.n_in[2]});
    pl.gpart = take((size_t)maxin * F * F * 8);
    pl.ginv = take((size_t)(F * F + F + 1) * 8);   // Ginv, Ginv 1, 1^T Ginv 1
    pl.rho = take(6 * 8);
    pl.end = off;
    L.probs.push_back(pl);
    L.cap_main += 2 * I + b.n_m2 + b.n_in[0] + b.n_in[1] + b.n_in[2] + 3;
    L.cap_kind[0] += I;
    L.cap_kind[1] += b.n_m2;
    L.cap_kind[2] += I;
    Plan fp;
    fp.I = I;
    fp.J = J;
    fp.K = K;
    maxfit = std::max<int64_t>(maxfit, fit_parts(fp));
  }
  L.dprobs = take((size_t)n * sizeof(BProb));
  L.items = take((size_t)L.cap_main * sizeof(uint2));
  for (int q = 0; q < 3; ++q) L.kind[q] = take((size_t)L.cap_kind[q] * sizeof(uint2));
  L.ctr = take(((size_t)n * kCtrPerProb + 1) * 4);
  L.flag = take(4);
  L.fitpart = take((size_t)maxfit * 2 * 8);
  L.fitout = take((size_t)n * 2 * 8);
  L.prof = take((size_t)kProfWords * 8);
  L.total = off;
  return L;
}

static inline uint2 item(int p, int kind, int idx) {
  return make_uint2((unsigned)p, ((unsigned)kind << 24) | (unsigned)idx);
}

// Descriptors from the tile table; work lists; upload; grid and LDS.
static ntf_status build_lists(ntf_batch_ctx* c) {
  for (int p = 0; p < c->n; ++p) {
    BProb& b = c->hp[p];
    auto k1 = key_of(1, b), k3 = key_of(3, b);
    if (!c->tiles.count(k1)) c->tiles[k1] = default_tile(1, b);
    if (!c->tiles.count(k3)) c->tiles[k3] = default_tile(3, b);
    apply_tiles(b, c->tiles[k1], c->tiles[k3]);
  }
  // problems by tensor size, largest first
  std::vector<int> order(c->n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const BProb &x = c->hp[a], &y = c->hp[b];
    return (int64_t)x.I * x.J * x.K > (int64_t)y.I * y.J * y.K;
  });
  std::vector<uint2> L, L1, L2, L3;
  std::fill(std::begin(c->by_kind), std::end(c->by_kind), 0);
  auto add = [&](std::vector<uint2>& v, int p, int kind, int count) {
    for (int q = 0; q < count; ++q) v.push_back(item(p, kind, q));
    c->by_kind[kind] += (&v == &L) ? count : 0;
  };
  // every item depends only on kinds of earlier groups
  for (int p : order) add(L, p, BK_PREP1, 1);
  for (int p : order) add(L, p, BK_P1, c->hp[p].n_p1);
  for (int p : order) add(L, p, BK_IN1, c->hp[p].ni[0]);
  for (int p : order) add(L, p, BK_PREP2, 1);
  for (int p : order) add(L, p, BK_M2, c->hp[p].n_m2);
  for (int p : order) add(L, p, BK_IN2, c->hp[p].ni[1]);
  for (int p : order) add(L, p, BK_PREP3, 1);
  for (int p : order) add(L, p, BK_P3, c->hp[p].n_p3);
  for (int p : order) add(L, p, BK_IN3, c->hp[p].ni[2]);
  for (int p : order) add(L1, p, BK_P1, c->hp[p].n_p1);
  for (int p : order) add(L2, p, BK_M2, c->hp[p].n_m2);
  for (int p : order) add(L3, p, BK_P3, c->hp[p].n_p3);
  if ((int64_t)L.size() > c->cap_main || (int64_t)L1.size() > c->cap_kind[0] ||
      (int64_t)L2.size() > c->cap_kind[1] || (int64_t)L3.size() > c->cap_kind[2]) {
    c->err = "work list exceeds its capacity";
    return NTF_E_HIP;
  }
  c->n_items = (int)L.size();
  c->n_kind[0] = (int)L1.size();
  c->n_kind[1] = (int)L2.size();
  c->n_kind[2] = (int)L3.size();
  c->lds = 0;
  for (const BProb& b : c->hp) c->lds = std::max(c->lds, lds_of(b));
  const int occ = batch_occupancy(c->lds);
  if (occ < 1) {
    c->err = "persistent kernel does not fit a compute unit";
    return NTF_E_UNSUPPORTED;
  }
  c->grid = std::max(1, std::min(occ * cus(), c->n_items));
  NTFB_HIP(c, hipMemcpy(c->dprobs, c->hp.data(), c->hp.size() * sizeof(BProb), hipMemcpyHostToDevice));
  NTFB_HIP(c, hipMemcpy(c->ditems, L.data(), L.size() * sizeof(uint2), hipMemcpyHostToDevice));
  if (!L1.empty())
    NTFB_HIP(c, hipMemcpy(c->dkind[0], L1.data(), L1.size() * sizeof(uint2), hipMemcpyHostToDevice));
  if (!L2.empty())
    NTFB_HIP(c, hipMemcpy(c->dkind[1], L2.data(), L2.size() * sizeof(uint2), hipMemcpyHostToDevice));
  if (!L3.empty())
    NTFB_HIP(c, hipMemcpy(c->dkind[2], L3.data(), L3.size() * sizeof(uint2), hipMemcpyHostToDevice));
  return NTF_OK;
}

static BatchK kargs(ntf_batch_ctx* c, const uint2* items, int n_items, int nodeps) {
  BatchK k;
  k.probs = c->dprobs;
  k.items = items;
  k.n_items = n_items;
  k.nodeps = nodeps;
  k.head = reinterpret_cast<unsigned*>(c->ctr + (size_t)c->n * kCtrPerProb);
  k.ctr = c->ctr;
  k.flag = c->flag;
  k.T = c->opts.inner_iters;
  k.eps_abs = c->opts.inner_eps_abs;
  k.eps_rel = c->opts.inner_eps_rel;
  k.rescale = c->opts.rescale_dual_on_rho_change ? 1 : 0;
  k.policy = c->opts.rho_policy;
  k.rho0 = c->opts.rho0;
  k.spin_limit = kSpinLimit;
  k.prof = nullptr;
  return k;
}

static ntf_status enqueue_iteration(ntf_batch_ctx* c, hipStream_t s) {
  NTFB_HIP(c, launch_zero_ints(c->ctr, (int64_t)c->n * kCtrPerProb + 1, s));
  NTFB_HIP(c, launch_batch(kargs(c, c->ditems, c->n_items, 0), c->grid, c->lds, s));
  return NTF_OK;
}

static void drop_graph(ntf_batch_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
}

static ntf_status capture(ntf_batch_ctx* c) {
  drop_graph(c);
  NTFB_HIP(c, hipStreamBeginCapture(c->sc, hipStreamCaptureModeThreadLocal));
  ntf_status st = enqueue_iteration(c, c->sc);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->sc, &g);
  if (st != NTF_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  NTFB_HIP(c, e);
  c->graph = g;
  NTFB_HIP(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
  return NTF_OK;
}

// Pass-only launch of one kind (0 = pass 1, 1 = mode 2, 2 = pass 3) without dependencies.
static ntf_status launch_kind_list(ntf_batch_ctx* c, int q, hipStream_t s) {
  if (c->n_kind[q] == 0) return NTF_OK;
  NTFB_HIP(c, launch_zero_ints(c->ctr, (int64_t)c->n * kCtrPerProb + 1, s));
  const int grid = std::max(1, std::min(c->grid, c->n_kind[q]));
  NTFB_HIP(c, launch_batch(kargs(c, c->dkind[q], c->n_kind[q], 1), grid, c->lds, s));
  return NTF_OK;
}

extern "C" {

size_t ntf_batch_workspace_bytes(const ntf_problem* probs, int32_t n, const ntf_opts* opts) {
  if (validate(probs, n, opts, nullptr) != NTF_OK) return 0;
  return make_layout(probs, n).total;
}

const char* ntf_batch_last_error(const ntf_batch_ctx* c) { return c ? c->err.c_str() : g_batch_err.c_str(); }

ntf_status ntf_batch_destroy(ntf_batch_ctx* c) {
  if (!c) return NTF_E_INVAL;
  if (c->s0) (void)hipStreamSynchronize(c->s0);
  drop_graph(c);
  if (c->sc) (void)hipStreamDestroy(c->sc);
  delete c;
  return NTF_OK;
}

ntf_status ntf_batch_init(ntf_batch_ctx** out, const ntf_problem* probs, int32_t n,
                          const ntf_opts* opts, void* workspace, size_t ws_bytes, void* stream) {
  if (!out) return NTF_E_INVAL;
  *out = nullptr;
  std::string why;
  ntf_status vs = validate(probs, n, opts, &why);
  g_batch_err = why;
  if (vs != NTF_OK) return vs;
  BatchLayout L = make_layout(probs, n);
  if (!workspace || ((uintptr_t)workspace & 255)) {
    g_batch_err = "workspace null or not 256-byte aligned";
    return NTF_E_INVAL;
  }
  if (ws_bytes < L.total) {
    g_batch_err = "workspace too small";
    return NTF_E_WORKSPACE;
  }
  ntf_batch_ctx* c = new (std::nothrow) ntf_batch_ctx();
  if (!c) return NTF_E_HIP;
  c->n = n;
  c->opts = *opts;
  c->probs.assign(probs, probs + n);
  c->lay = L.probs;
  c->ws = reinterpret_cast<char*>(workspace);
  c->ws_bytes = ws_bytes;
  c->s0 = reinterpret_cast<hipStream_t>(stream);
  c->dprobs = reinterpret_cast<BProb*>(c->ws + L.dprobs);
  c->ditems = reinterpret_cast<uint2*>(c->ws + L.items);
  c->cap_main = L.cap_main;
  for (int q = 0; q < 3; ++q) {
    c->dkind[q] = reinterpret_cast<uint2*>(c->ws + L.kind[q]);
    c->cap_kind[q] = L.cap_kind[q];
  }
  c->ctr = reinterpret_cast<int*>(c->ws + L.ctr);
  c->flag = reinterpret_cast<int*>(c->ws + L.flag);
  c->fitpart = reinterpret_cast<double*>(c->ws + L.fitpart);
  c->fitout = reinterpret_cast<double*>(c->ws + L.fitout);
  c->prof = reinterpret_cast<unsigned long long*>(c->ws + L.prof);
  ntf_status st = [&]() -> ntf_status {
    NTFB_HIP(c, hipStreamCreateWithFlags(&c->sc, hipStreamNonBlocking));
    c->hp.resize(n);
    for (int p = 0; p < n; ++p) {
      const ntf_problem& pr = probs[p];
      const ProbLayout& pl = c->lay[p];
      BProb b = base_prob(pr);
      b.Xr = reinterpret_cast<const __bf16*>(c->ws + pl.xr);
      b.Xt = reinterpret_cast<const __bf16*>(c->ws + pl.xt);
      b.scale = reinterpret_cast<const float*>(c->ws + pl.scale);
      for (int m = 0; m < 3; ++m) {
        b.H[m] = reinterpret_cast<float*>(pr.H[m]);
        b.U[m] = reinterpret_cast<float*>(pr.U[m]);
        b.W[m] = reinterpret_cast<double*>(c->ws + pl.W[m]);
        b.gram[m] = reinterpret_cast<double*>(c->ws + pl.gram[m]);
      }
      b.T = reinterpret_cast<float*>(c->ws + pl.T);
      b.W3p = reinterpret_cast<float*>(c->ws + pl.W3p);
      b.gpart = reinterpret_cast<double*>(c->ws + pl.gpart);
      b.Ginv = reinterpret_cast<double*>(c->ws + pl.ginv);
      b.rho = reinterpret_cast<double*>(c->ws + pl.rho);
      c->hp[p] = b;
      NTFB_HIP(c, launch_batch_quantize(reinterpret_cast<const float*>(pr.X), b.I, b.J, b.K, b.Kp,
                                        b.Jp, const_cast<__bf16*>(b.Xr), const_cast<__bf16*>(b.Xt),
                                        const_cast<float*>(b.scale), c->s0));
      NTFB_HIP(c, launch_fill(b.rho, 6, opts->rho0, c->s0));
      // Grams of the initial factors: FP32 per inner row block, summed in FP64
      // in block order (the inner sweep's own partition)
      const int d[3] = {b.I, b.J, b.K};
      for (int m = 0; m < 3; ++m) {
        NTFB_HIP(c, launch_gram_part(pr.H[m], 0, d[m], b.F, b.rpb, 1, b.gpart, c->s0));
        NTFB_HIP(c, launch_reduce_partials(b.gpart, 1, (int64_t)b.F * b.F, b.F, b.n_in[m], b.F,
                                           b.F, b.gram[m], c->s0, 4));
      }
    }
    NTFB_HIP(c, launch_zero_ints(c->flag, 1, c->s0));
    NTFB_HIP(c, hipStreamSynchronize(c->s0));
    ntf_status s2 = build_lists(c);
    if (s2 != NTF_OK) return s2;
    return capture(c);
  }();
  if (st != NTF_OK) {
    g_batch_err = c->err;
    ntf_batch_destroy(c);
    return st;
  }
  *out = c;
  return NTF_OK;
}

ntf_status ntf_batch_step(ntf_batch_ctx* c, int32_t n_outer) {
  if (!c || n_outer < 0) return NTF_E_INVAL;
  for (int32_t q = 0; q < n_outer; ++q) NTFB_HIP(c, hipGraphLaunch(c->gexec, c->s0));
  return NTF_OK;
}

ntf_status ntf_batch_sync(ntf_batch_ctx* c, int32_t* flags_out) {
  if (!c) return NTF_E_INVAL;
  int h = 0;
  NTFB_HIP(c, hipMemcpyAsync(&h, c->flag, 4, hipMemcpyDeviceToHost, c->s0));
  NTFB_HIP(c, hipStreamSynchronize(c->s0));
  if (flags_out) *flags_out = h;
  if (h) {
    c->err = (h & 8) ? "a dependency wait of the persistent kernel timed out"
                     : "non-PD system or NaN/Inf met on the device";
    return NTF_E_NUMERIC;
  }
  return NTF_OK;
}

ntf_status ntf_batch_fit(ntf_batch_ctx* c, double* rfe_host) {
  if (!c || !rfe_host) return NTF_E_INVAL;
  for (int p = 0; p < c->n; ++p) {
    const BProb& b = c->hp[p];
    Plan fp;
    fp.I = b.I;
    fp.J = b.J;
    fp.K = b.K;
    fp.F = b.F;
    NTFB_HIP(c, launch_fit(fp, c->probs[p].X, 0, b.H[0], b.H[1], b.H[2], 0, c->fitpart,
                           c->fitout + 2 * p, c->s0, nullptr));
  }
  std::vector<double> h((size_t)c->n * 2);
  NTFB_HIP(c, hipMemcpyAsync(h.data(), c->fitout, h.size() * 8, hipMemcpyDeviceToHost, c->s0));
  NTFB_HIP(c, hipStreamSynchronize(c->s0));
  for (int p = 0; p < c->n; ++p)
    rfe_host[p] = h[2 * p + 1] > 0 ? std::sqrt(std::max(h[2 * p], 0.0) / h[2 * p + 1]) : 0.0;
  return NTF_OK;
}

ntf_status ntf_batch_launch_kind(ntf_batch_ctx* c, int32_t kind) {
  if (!c) return NTF_E_INVAL;
  const int q = (kind == BK_P1) ? 0 : (kind == BK_M2) ? 1 : (kind == BK_P3) ? 2 : -1;
  if (q < 0) {
    c->err = "kind must be 0 (pass 1), 4 (mode 2) or 7 (pass 3)";
    return NTF_E_INVAL;
  }
  return launch_kind_list(c, q, c->s0);
}

ntf_status ntf_batch_mttkrp(ntf_batch_ctx* c, int32_t prob, int32_t mode, double* W_out) {
  if (!c || prob < 0 || prob >= c->n || mode < 0 || mode > 2 || !W_out) return NTF_E_INVAL;
  const BProb& b = c->hp[prob];
  if (mode == 2) {
    ntf_status st = launch_kind_list(c, 2, c->s0);
    if (st != NTF_OK) return st;
    NTFB_HIP(c, launch_reduce_partials(b.W3p, 0, (int64_t)b.K * b.F, b.F, b.n_p3, b.K, b.F, W_out,
                                       c->s0, 4));
    return NTF_OK;
  }
  ntf_status st = launch_kind_list(c, 0, c->s0);
  if (st == NTF_OK && mode == 1) st = launch_kind_list(c, 1, c->s0);
  if (st != NTF_OK) return st;
  const int64_t rows = mode == 0 ? b.I : b.J;
  NTFB_HIP(c, hipMemcpyAsync(W_out, b.W[mode], (size_t)(rows * b.F) * 8, hipMemcpyDeviceToDevice, c->s0));
  return NTF_OK;
}

ntf_status ntf_batch_get_tiles(ntf_batch_ctx* c, ntf_batch_tile* out, int32_t cap, int32_t* n_out) {
  if (!c || (cap > 0 && !out)) return NTF_E_INVAL;
  int32_t w = 0;
  for (const auto& kv : c->tiles) {
    if (w < cap) {
      ntf_batch_tile t;
      t.kind = std::get<0>(kv.first);
      t.ft = std::get<1>(kv.first);
      t.qbucket = std::get<2>(kv.first);
      t.mt = kv.second.mt;
      t.item_elems = kv.second.elems;
      t.us = kv.second.us;
      out[w] = t;
    }
    ++w;
  }
  if (n_out) *n_out = std::min(w, cap);
  return NTF_OK;
}

ntf_status ntf_batch_set_tiles(ntf_batch_ctx* c, const ntf_batch_tile* tiles, int32_t n) {
  if (!c || n < 0 || (n > 0 && !tiles)) return NTF_E_INVAL;
  for (int32_t q = 0; q < n; ++q) {
    const ntf_batch_tile& t = tiles[q];
    if ((t.kind != 1 && t.kind != 3) || (t.mt != 1 && t.mt != 2) || t.item_elems < 1) {
      c->err = "tile: kind must be 1 or 3, mt 1 or 2, item_elems >= 1";
      return NTF_E_INVAL;
    }
  }
  NTFB_HIP(c, hipStreamSynchronize(c->s0));
  for (int32_t q = 0; q < n; ++q) {
    const ntf_batch_tile& t = tiles[q];
    c->tiles[TileKey(t.kind, t.ft, t.qbucket)] = TileVal{t.mt, t.item_elems, t.us};
  }
  ntf_status st = build_lists(c);
  if (st != NTF_OK) return st;
  return capture(c);
}

ntf_status ntf_batch_autotune(ntf_batch_ctx* c, int32_t reps, ntf_batch_tile* out, int32_t cap,
                              int32_t* n_out) {
  if (!c || reps < 1 || (cap > 0 && !out)) return NTF_E_INVAL;
  NTFB_HIP(c, hipStreamSynchronize(c->s0));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  NTFB_HIP(c, hipEventCreate(&e0));
  NTFB_HIP(c, hipEventCreate(&e1));
  ntf_status result = [&]() -> ntf_status {
    ntf_status st = build_lists(c);   // make sure every bucket has an entry
    if (st != NTF_OK) return st;
    const std::vector<TileKey> keys = [&] {
      std::vector<TileKey> k;
      for (const auto& kv : c->tiles) k.push_back(kv.first);
      return k;
    }();
    std::vector<int> order(c->n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      const BProb &x = c->hp[a], &y = c->hp[b];
      return (int64_t)x.I * x.J * x.K > (int64_t)y.I * y.J * y.K;
    });
    for (const TileKey& key : keys) {
      const int kind = std::get<0>(key);
      std::vector<int> members;
      for (int p = 0; p < c->n; ++p)
        if (key_of(kind, c->hp[p]) == key) members.push_back(p);
      if (members.empty()) continue;
      const int64_t elems[3] = {kind == 1 ? 64 * 1024 : 256 * 1024, kind == 1 ? 256 * 1024 : 1024 * 1024,
                                kind == 1 ? 1024 * 1024 : 4096 * 1024};
      TileVal best = c->tiles[key];
      double best_us = 1e300;
      for (int mt = 1; mt <= 2; ++mt)
        for (int ei = 0; ei < 3; ++ei) {
          // the candidate for this bucket, every other problem at its current
          // tiles: the whole pass runs, so the time is the one that matters
          // (a bucket on its own may not fill the GPU)
          const TileVal cand{mt, elems[ei], 0.0};
          for (int p : members) {
            BProb& b = c->hp[p];
            if (kind == 1) apply_tiles(b, cand, c->tiles[key_of(3, b)]);
            else apply_tiles(b, c->tiles[key_of(1, b)], cand);
          }
          std::vector<uint2> L;
          size_t lds = 0;
          for (int p : order) {
            const BProb& b = c->hp[p];
            const int cnt = kind == 1 ? b.n_p1 : b.n_p3;
            for (int q = 0; q < cnt; ++q) L.push_back(item(p, kind == 1 ? BK_P1 : BK_P3, q));
            lds = std::max(lds, kind == 1 ? batch_lds_p1(b) : batch_lds_p3(b));
          }
          if ((int64_t)L.size() > c->cap_main) continue;
          const int occ = batch_occupancy(lds);
          if (occ < 1) continue;
          const int grid = std::max(1, std::min(occ * cus(), (int)L.size()));
          NTFB_HIP(c, hipMemcpy(c->dprobs, c->hp.data(), c->hp.size() * sizeof(BProb),
                                hipMemcpyHostToDevice));
          NTFB_HIP(c, hipMemcpy(c->ditems, L.data(), L.size() * sizeof(uint2), hipMemcpyHostToDevice));
          const BatchK k = kargs(c, c->ditems, (int)L.size(), 1);
          // one untimed launch, then reps timed ones
          for (int r = 0; r <= reps; ++r) {
            if (r == 1) NTFB_HIP(c, hipEventRecord(e0, c->s0));
            NTFB_HIP(c, launch_zero_ints(c->ctr, (int64_t)c->n * kCtrPerProb + 1, c->s0));
            NTFB_HIP(c, launch_batch(k, grid, lds, c->s0));
          }
          NTFB_HIP(c, hipEventRecord(e1, c->s0));
          NTFB_HIP(c, hipEventSynchronize(e1));
          float ms = 0.f;
          NTFB_HIP(c, hipEventElapsedTime(&ms, e0, e1));
          const double us = 1e3 * ms / reps;
          if (us < best_us) {
            best_us = us;
            best = TileVal{mt, elems[ei], us};
          }
        }
      c->tiles[key] = best;
      for (int p : members) {
        BProb& b = c->hp[p];
        apply_tiles(b, c->tiles[key_of(1, b)], c->tiles[key_of(3, b)]);
      }
    }
    st = build_lists(c);
    if (st != NTF_OK) return st;
    return capture(c);
  }();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (result != NTF_OK) return result;
  return ntf_batch_get_tiles(c, out, cap, n_out);
}

ntf_status ntf_batch_profile(ntf_batch_ctx* c, double* busy_us, double* wait_us, int64_t* items) {
  if (!c || !busy_us || !wait_us || !items) return NTF_E_INVAL;
  int dev = 0, khz = 0;
  NTFB_HIP(c, hipGetDevice(&dev));
  NTFB_HIP(c, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  if (khz <= 0) {
    c->err = "device reports no wall-clock rate";
    return NTF_E_UNSUPPORTED;
  }
  NTFB_HIP(c, launch_zero_ints(reinterpret_cast<int*>(c->prof), 2 * kProfWords, c->s0));
  NTFB_HIP(c, launch_zero_ints(c->ctr, (int64_t)c->n * kCtrPerProb + 1, c->s0));
  BatchK k = kargs(c, c->ditems, c->n_items, 0);
  k.prof = c->prof;
  NTFB_HIP(c, launch_batch(k, c->grid, c->lds, c->s0));
  unsigned long long h[kProfWords];
  NTFB_HIP(c, hipMemcpyAsync(h, c->prof, sizeof(h), hipMemcpyDeviceToHost, c->s0));
  NTFB_HIP(c, hipStreamSynchronize(c->s0));
  for (int q = 0; q < BK_NKINDS; ++q) {
    busy_us[q] = 1e3 * (double)h[3 * q] / khz;
    wait_us[q] = 1e3 * (double)h[3 * q + 1] / khz;
    items[q] = (int64_t)h[3 * q + 2];
  }
  return NTF_OK;
}

ntf_status ntf_batch_info_get(ntf_batch_ctx* c, ntf_batch_info* out) {
  if (!c || !out) return NTF_E_INVAL;
  std::memset(out, 0, sizeof(*out));
  out->n_problems = c->n;
  out->grid = c->grid;
  out->lds_bytes = (int32_t)c->lds;
  out->n_items = c->n_items;
  for (int k = 0; k < BK_NKINDS; ++k) out->items_by_kind[k] = c->by_kind[k];
  for (const BProb& b : c->hp) {
    out->x_bytes += (int64_t)b.I * b.J * b.K * 2;
    out->t_bytes += (int64_t)b.I * b.J * b.F * 4;
  }
  return NTF_OK;
}

}  // extern "C"
