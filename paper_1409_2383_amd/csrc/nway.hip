// C-ABI host layer for tensors of order N = 3..8 (Appendix A): the mode-n
// MTTKRP contracts X^(n) with the Khatri-Rao matrix of the N - 1 other
// factors, the system matrix is the Hadamard product of their N - 1 Grams,
// and the inner sweep is unchanged.
//
// Every mode-n MTTKRP runs the three-way kernels on a three-way view of the
// same C-order tensor (no copy): the modes before n fold into one index, the
// modes after n into another, and the factor of a folded group is the
// Khatri-Rao product of its factors (formed per outer iteration, rows in C
// order).  Mode 1 views X as (I_1, prod I_2..I_{N-1}, I_N) and takes the
// pass-1 MTTKRP; a middle mode n views it as (prod before, I_n, prod after)
// and takes pass 1 (contraction over the trailing group) then the mode-2
// reduction over the leading group; mode N views it as (I_1, prod I_2..I_{N-1},
// I_N) and takes pass 3.  FP32 and FP64 only.
//
// Two consecutive middle modes n, n+1 share one pass inside an outer
// iteration.  Mode n+1's view (prod up to n, I_{n+1}, prod after n+1) has
// pass 1 contract the trailing group into T and, in its epilogue, weight T by
// H_{n+1} and sum over I_{n+1}: that is X contracted with every factor after
// n, indexed by (modes up to n).  Mode n's MTTKRP is then a reduction of
// those rows over the modes before n, and mode n+1's is the mode-2 reduction
// of the same T (T holds no factor of modes up to n+1, so it is still valid
// after mode n's update).  One pass over X instead of two, and the pass that
// remains contracts a short trailing group whose factor fits in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "ntf_admm.h"
#include "ntf_launch.h"

using namespace ntf;

namespace ntf {
ntf_status validate_opts(const ntf_opts* o, std::string* why);
int cu_count();
}

namespace {

constexpr int kMax = NTF_MAX_ORDER;
// rows of the leading group per partial of the pair reduction (k_pair_reduce)
constexpr int kPairRows = 4;

struct NwState {
  double rho[kMax][2];
  double resid[kMax][8];
  double fin[10];
  double xnorm2;
  double fit[2];
  int fresh[kMax];
  int flag;
  unsigned counter[kMax];
  int taken[kMax];
  int pad_;
};

// A folded group of consecutive modes [lo, hi): its factor is the Khatri-Rao
// product of theirs (a single mode: the factor itself).
struct Group {
  int lo = 0, hi = 0;
  int64_t rows = 1;
};

struct ModeView {
  int kind = 0;        // 0: pass 1 (mode 1 of the view); 1: pass 1 + mode 2; 2: pass 3
  int pair = 0;        // kind 1 only: 1 = first of a pair (from mode n+1's pass), 2 = second
  Group g[3];          // the three view modes
  Plan plan;
};

struct NwLayout {
  size_t state = 0, T = 0, P1 = 0, P2 = 0, P3 = 0, W = 0, krA = 0, krB = 0, prim[kMax] = {},
         gram[kMax] = {}, ginv[kMax] = {}, hrest = 0, gpart = 0, rpart = 0, sumsq = 0, fitpart = 0,
         total = 0;
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  }
};

struct Setup {
  int N = 0, F = 0, prec = 0, FL = 0, rpb = 0, nprep = 1;
  int64_t d[kMax] = {};
  int nblk[kMax] = {};
  ModeView v[kMax];
};

Group group(const Setup& s, int lo, int hi) {
  Group g;
  g.lo = lo;
  g.hi = hi;
  g.rows = 1;
  for (int m = lo; m < hi; ++m) g.rows *= s.d[m];
  return g;
}

bool make_setup(Setup& s, const ntf_nway_problem* pr, const ntf_opts* o, int cus, std::string* why) {
  s = Setup();
  s.N = pr->order;
  s.F = pr->F;
  s.prec = o->precision == NTF_PREC_F64 ? PREC_F64 : PREC_F32;
  for (int m = 0; m < s.N; ++m) s.d[m] = pr->dims[m];
  int FL = 4;
  while (FL < s.F) FL <<= 1;
  s.FL = FL;
  s.rpb = inner_rows_per_block(FL);
  for (int m = 0; m < s.N; ++m) s.nblk[m] = (int)((s.d[m] + s.rpb - 1) / s.rpb);
  s.nprep = (int)std::max<int64_t>(1, ((int64_t)s.F * s.F + 63) / 64);
  const int N = s.N;
  for (int n = 0; n < N; ++n) {
    ModeView& mv = s.v[n];
    if (n == 0) {
      mv.kind = 0;
      mv.g[0] = group(s, 0, 1);
      mv.g[1] = group(s, 1, N - 1);
      mv.g[2] = group(s, N - 1, N);
    } else if (n == N - 1) {
      mv.kind = 2;
      mv.g[0] = group(s, 0, 1);
      mv.g[1] = group(s, 1, N - 1);
      mv.g[2] = group(s, N - 1, N);
    } else {
      mv.kind = 1;
      mv.g[0] = group(s, 0, n);
      mv.g[1] = group(s, n, n + 1);
      mv.g[2] = group(s, n + 1, N);
    }
    const int64_t vd[3] = {mv.g[0].rows, mv.g[1].rows, mv.g[2].rows};
    for (int q = 0; q < 3; ++q)
      if (vd[q] >= ((int64_t)1 << 31)) {
        if (why) *why = "a folded group of modes has 2^31 rows or more";
        return false;
      }
    if (!make_plan(mv.plan, s.prec, vd, s.F, cus)) {
      if (why) *why = "no MTTKRP plan for a three-way view of the tensor";
      return false;
    }
  }
  // middle modes paired from the second mode on: (1, 2), (3, 4), ...
  // (a pair's reduction takes one grid row per kPairRows rows of the leading
  // group: at most 65535)
  for (int n = 1; n + 1 <= N - 2; n += 2) {
    if ((s.v[n].g[0].rows + kPairRows - 1) / kPairRows > 65535) continue;
    s.v[n].pair = 1;
    s.v[n + 1].pair = 2;
  }
  return true;
}

NwLayout make_layout(const Setup& s, const ntf_opts& o) {
  NwLayout L;
  Carver c;
  const size_t es = elem_size(s.prec);
  const int64_t F = s.F;
  size_t t = 0, p1 = 0, p2 = 0, p3 = 0, kr = 1;
  int64_t maxd = 1;
  int maxblk = 1;
  for (int n = 0; n < s.N; ++n) {
    const Plan& p = s.v[n].plan;
    if (s.v[n].kind == 1) t = std::max(t, (size_t)(p.I * p.J * F) * es);
    if (s.v[n].kind != 2) {
      p1 = std::max(p1, (size_t)(p.I * p.nch1 * F) * es);
    }
    if (s.v[n].kind == 1) p2 = std::max(p2, (size_t)((int64_t)p.nich2 * p.J * F) * es);
    // (FP64 partials of kPairRows rows each for the first mode of a pair)
    if (s.v[n].pair == 1) p2 = std::max(p2, (size_t)(((p.I + kPairRows - 1) / kPairRows) * p.J * F) * 8);
    if (s.v[n].kind == 2) p3 = std::max(p3, (size_t)((int64_t)p.nrc3 * p.K * F) * es);
    for (int q = 0; q < 3; ++q)
      if (s.v[n].g[q].hi - s.v[n].g[q].lo > 1) kr = std::max(kr, (size_t)s.v[n].g[q].rows);
    maxd = std::max(maxd, s.d[n]);
    maxblk = std::max(maxblk, s.nblk[n]);
  }
  L.state = c.take(sizeof(NwState));
  L.T = c.take(t);
  L.P1 = c.take(p1);
  L.P2 = c.take(p2);
  L.P3 = c.take(p3);
  L.W = c.take((size_t)(maxd * F) * 8);
  L.krA = c.take(kr * F * es);
  L.krB = c.take(kr * F * es);
  for (int m = 0; m < s.N; ++m) {
    L.prim[m] = (o.factor_source == 1) ? c.take((size_t)(s.d[m] * F) * es) : 0;
    L.gram[m] = c.take((size_t)(F * F) * 8);
    L.ginv[m] = c.take((size_t)(F * F + F + 1) * 8);
  }
  L.hrest = c.take((size_t)(F * F) * 8);
  L.gpart = c.take((size_t)maxblk * F * F * 8);
  L.rpart = c.take((size_t)maxblk * 8 * 8);
  L.sumsq = c.take(1024 * 8);
  L.fitpart = c.take((size_t)fit_parts(s.v[0].plan) * 2 * 8);
  L.total = c.off;
  return L;
}

// ---------------------------------------------------------------- kernels

struct KrK {
  const void* f[kMax];
  int64_t d[kMax];
  int k;          // factors in the group
  int F;
  int64_t rows;
  void* out;      // [rows][F]
};

// Row p of the Khatri-Rao product of the group's factors, C order (the last
// factor's index fastest): the Hadamard product of one row of each.
template <typename T>
__global__ __launch_bounds__(256) void k_kr(KrK a) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= a.rows * a.F) return;
  const int64_t p = e / a.F;
  const int f = (int)(e - p * a.F);
  int64_t r = p;
  T v = T(1);
  for (int q = a.k - 1; q >= 0; --q) {
    const int64_t i = r % a.d[q];
    r /= a.d[q];
    v *= reinterpret_cast<const T*>(a.f[q])[i * a.F + f];
  }
  reinterpret_cast<T*>(a.out)[e] = v;
}

// The first mode n of a pair, from the pass of mode n+1's view: P1 holds, for
// row r = a * In + j of that view (a over the modes before n, j over I_n) and
// chunk c of I_{n+1}, the chunk's sum over l of H_{n+1}[l,:] T[r,l,:].  Partial
// ac of the result takes rows a = kPairRows * ac + q, q = 0 .. kPairRows-1:
//   out[ac][j][f] = sum_q G0[a][f] * (sum_c P1[r][c][f])     (FP64, q and c
// increasing; the kPairRows rows' loads of one c are issued together).
template <typename T>
__global__ __launch_bounds__(256) void k_pair_reduce(const T* __restrict__ P1, int nch,
                                                     const T* __restrict__ G0, int64_t A,
                                                     int64_t In, int F, double* __restrict__ out) {
  const int64_t JF = In * F;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= JF) return;
  const int64_t j = idx / F;
  const int f = (int)(idx - j * F);
  const int64_t a0 = (int64_t)blockIdx.y * kPairRows;
  const T* p[kPairRows];
  bool ok[kPairRows];
  double w[kPairRows];
#pragma unroll
  for (int q = 0; q < kPairRows; ++q) {
    ok[q] = a0 + q < A;
    p[q] = P1 + (((ok[q] ? a0 + q : a0) * In + j) * nch) * F + f;
    w[q] = 0.0;
  }
  for (int c = 0; c < nch; ++c) {
    T v[kPairRows];
#pragma unroll
    for (int q = 0; q < kPairRows; ++q) v[q] = p[q][(int64_t)c * F];
#pragma unroll
    for (int q = 0; q < kPairRows; ++q) w[q] += (double)v[q];
  }
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < kPairRows; ++q)
    if (ok[q]) acc += (double)G0[(a0 + q) * F + f] * w[q];
  out[(int64_t)blockIdx.y * JF + idx] = acc;
}

struct HprodK {
  const double* g[kMax];
  int k;
  int FF;
  double* out;
};

// Hadamard product of k Grams, in the order given.
__global__ __launch_bounds__(256) void k_gram_hprod(HprodK a) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= a.FF) return;
  double v = a.g[0][e];
  for (int q = 1; q < a.k; ++q) v *= a.g[q][e];
  a.out[e] = v;
}

}  // namespace

struct ntf_nway_ctx {
  ntf_nway_problem prob;
  ntf_opts opts;
  Setup su;
  NwLayout lay;
  char* ws = nullptr;
  hipStream_t s0 = nullptr, s1 = nullptr, sc = nullptr;
  hipEvent_t ev_fork = nullptr, ev_inner[kMax] = {}, ev_prep[kMax] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool use_graph = true;
  int64_t outer = 0;
  NwState* host_state = nullptr;
  std::string err;

  template <typename T> T* at(size_t off) { return reinterpret_cast<T*>(ws + off); }
  NwState* dstate() { return at<NwState>(lay.state); }
  int hf64() const { return su.prec == PREC_F64 ? 1 : 0; }
  const void* feed(int m) const {
    return (opts.factor_source == 1) ? (const void*)(ws + lay.prim[m]) : (const void*)prob.H[m];
  }
};

#define NW_HIP(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      if (ctx) (ctx)->err = std::string(#call) + ": " + hipGetErrorString(e_);        \
      return NTF_E_HIP;                                                                \
    }                                                                                  \
  } while (0)

namespace {

thread_local std::string g_nw_init_err;

ntf_status validate_nway(const ntf_nway_problem* pr, const ntf_opts* o, std::string* why) {
  auto fail = [&](const char* m, ntf_status st = NTF_E_INVAL) {
    if (why) *why = m;
    return st;
  };
  if (!pr || !o) return fail("null problem or options");
  if (pr->order < 3 || pr->order > kMax) return fail("order must be in [3, NTF_MAX_ORDER]");
  int64_t total = 1;
  for (int m = 0; m < pr->order; ++m) {
    if (pr->dims[m] < 1 || pr->dims[m] > (int64_t)1 << 31) return fail("dims must be in [1, 2^31]");
    if (total > ((int64_t)1 << 46) / pr->dims[m]) return fail("tensor too large");
    total *= pr->dims[m];
  }
  if (pr->F < 1 || pr->F > 64) return fail("F must be in [1, 64]");
  if (o->precision == NTF_PREC_BF16_MIXED)
    return fail("order-N tensors run in NTF_PREC_F32 or NTF_PREC_F64", NTF_E_UNSUPPORTED);
  if (o->precision != NTF_PREC_F32 && o->precision != NTF_PREC_F64) return fail("unknown precision");
  if (pr->x_dtype != 0 && pr->x_dtype != 1) return fail("x_dtype must be 0 or 1");
  if ((o->precision == NTF_PREC_F64) != (pr->x_dtype == 1)) return fail("x_dtype does not match precision");
  if (pr->reserved != 0) return fail("reserved field must be zero");
  if (!pr->X || (((uintptr_t)pr->X) & 15)) return fail("X null or not 16-byte aligned");
  for (int m = 0; m < pr->order; ++m) {
    if (!pr->H[m] || !pr->U[m]) return fail("null factor or dual");
    if ((((uintptr_t)pr->H[m]) | ((uintptr_t)pr->U[m])) & 15) return fail("factor/dual not 16-byte aligned");
  }
  if (o->warm_hidden != 0) return fail("the learned warm start is not offered for order-N tensors", NTF_E_UNSUPPORTED);
  return validate_opts(o, why);
}

// Khatri-Rao factor of view mode q of mode n's view, from the given factors.
ntf_status group_factor(ntf_nway_ctx* c, const Group& g, const void* const* fac, void* buf, hipStream_t s,
                        const void** out) {
  if (g.hi - g.lo == 1) {
    *out = fac[g.lo];
    return NTF_OK;
  }
  KrK k;
  std::memset(&k, 0, sizeof(k));
  k.k = g.hi - g.lo;
  for (int q = 0; q < k.k; ++q) {
    k.f[q] = fac[g.lo + q];
    k.d[q] = c->su.d[g.lo + q];
  }
  k.F = c->su.F;
  k.rows = g.rows;
  k.out = buf;
  const unsigned grid = (unsigned)((g.rows * k.F + 255) / 256);
  if (c->hf64())
    hipLaunchKernelGGL(k_kr<double>, dim3(grid), dim3(256), 0, s, k);
  else
    hipLaunchKernelGGL(k_kr<float>, dim3(grid), dim3(256), 0, s, k);
  NW_HIP(c, hipGetLastError());
  *out = buf;
  return NTF_OK;
}

// W (FP64, [d_n][F]) = mode-n MTTKRP with the feed factors.  In an outer
// iteration (`paired`) the second mode of a pair takes T from the first
// mode's pass; called alone it runs its own pass.
ntf_status enqueue_mttkrp(ntf_nway_ctx* c, int n, double* W, hipStream_t s, bool paired) {
  const ModeView& mv = c->su.v[n];
  const Plan& p = mv.plan;
  const void* fac[kMax];
  for (int m = 0; m < c->su.N; ++m) fac[m] = c->feed(m);
  void* T = c->ws + c->lay.T;
  const int pf64 = c->hf64();
  const void* g0 = nullptr;
  const void* g1 = nullptr;
  const void* g2 = nullptr;
  ntf_status st;
  if (mv.kind == 0) {
    if ((st = group_factor(c, mv.g[1], fac, c->ws + c->lay.krA, s, &g1)) != NTF_OK) return st;
    g2 = fac[c->su.N - 1];
    // (only the mode-1 partials are wanted: no T)
    NW_HIP(c, launch_pass1(p, c->prob.X, nullptr, nullptr, g1, g2, nullptr, c->ws + c->lay.P1, s));
    NW_HIP(c, launch_reduce_partials(c->ws + c->lay.P1, pf64, p.F, (int64_t)p.nch1 * p.F, p.nch1, p.I, p.F,
                                     W, s, 16));
  } else if (mv.kind == 1 && mv.pair == 1) {
    // the pass of mode n+1's view (its mode-1 partials weight T by H_{n+1}),
    // then the reduction over the modes before n
    const ModeView& nv = c->su.v[n + 1];
    const Plan& q = nv.plan;
    if ((st = group_factor(c, nv.g[2], fac, c->ws + c->lay.krB, s, &g2)) != NTF_OK) return st;
    NW_HIP(c, launch_pass1(q, c->prob.X, nullptr, nullptr, fac[n + 1], g2, T, c->ws + c->lay.P1, s));
    if ((st = group_factor(c, mv.g[0], fac, c->ws + c->lay.krA, s, &g0)) != NTF_OK) return st;
    double* P2 = c->at<double>(c->lay.P2);
    const int nparts = (int)((p.I + kPairRows - 1) / kPairRows);
    const dim3 grid((unsigned)((p.J * p.F + 255) / 256), (unsigned)nparts);
    if (pf64)
      hipLaunchKernelGGL(k_pair_reduce<double>, grid, dim3(256), 0, s, c->at<const double>(c->lay.P1),
                         q.nch1, (const double*)g0, p.I, p.J, p.F, P2);
    else
      hipLaunchKernelGGL(k_pair_reduce<float>, grid, dim3(256), 0, s, c->at<const float>(c->lay.P1),
                         q.nch1, (const float*)g0, p.I, p.J, p.F, P2);
    NW_HIP(c, hipGetLastError());
    NW_HIP(c, launch_reduce_partials(P2, 1, p.J * p.F, p.F, nparts, p.J, p.F, W, s, 16));
  } else if (mv.kind == 1) {
    if ((st = group_factor(c, mv.g[0], fac, c->ws + c->lay.krA, s, &g0)) != NTF_OK) return st;
    if (!(paired && mv.pair == 2)) {
      if ((st = group_factor(c, mv.g[2], fac, c->ws + c->lay.krB, s, &g2)) != NTF_OK) return st;
      // pass 1 forms T = X x_3 (trailing group); its mode-1 partials (against
      // this mode's own factor) are not used
      NW_HIP(c, launch_pass1(p, c->prob.X, nullptr, nullptr, fac[n], g2, T, c->ws + c->lay.P1, s));
    }
    NW_HIP(c, launch_mode2(p, T, g0, c->ws + c->lay.P2, s));
    NW_HIP(c, launch_reduce_partials(c->ws + c->lay.P2, pf64, p.J * p.F, p.F, p.nich2, p.J, p.F, W, s, 16));
  } else {
    g0 = fac[0];
    if ((st = group_factor(c, mv.g[1], fac, c->ws + c->lay.krA, s, &g1)) != NTF_OK) return st;
    NW_HIP(c, launch_pass3(p, c->prob.X, nullptr, nullptr, g0, g1, c->ws + c->lay.P3, s));
    NW_HIP(c, launch_reduce_partials(c->ws + c->lay.P3, pf64, p.K * p.F, p.F, p.nrc3, p.K, p.F, W, s, 16));
  }
  return NTF_OK;
}

ntf_status enqueue_outer(ntf_nway_ctx* c, hipStream_t ms) {
  const Setup& su = c->su;
  const int N = su.N;
  NwState* ds = c->dstate();
  double* W = c->at<double>(c->lay.W);
  for (int n = 0; n < N; ++n) {
    hipEvent_t ev = (n == 0) ? c->ev_fork : c->ev_inner[n - 1];
    NW_HIP(c, hipEventRecord(ev, ms));
    NW_HIP(c, hipStreamWaitEvent(c->s1, ev, 0));
    // prepare mode n on the side: the Grams of the other modes, the one
    // updated last reduced from its partials
    const int src = (n + N - 1) % N;
    const double* gb;
    if (N == 3) {
      gb = c->at<double>(c->lay.gram[(n + 1) % N]);
    } else {
      HprodK h;
      std::memset(&h, 0, sizeof(h));
      for (int m = 0; m < N; ++m)
        if (m != n && m != src) h.g[h.k++] = c->at<double>(c->lay.gram[m]);
      h.FF = su.F * su.F;
      h.out = c->at<double>(c->lay.hrest);
      hipLaunchKernelGGL(k_gram_hprod, dim3((unsigned)((h.FF + 255) / 256)), dim3(256), 0, c->s1, h);
      NW_HIP(c, hipGetLastError());
      gb = h.out;
    }
    PrepArgs pa;
    pa.F = su.F;
    pa.gram_part = c->at<double>(c->lay.gpart);
    pa.nparts = su.nblk[src];
    pa.gram_dst = c->at<double>(c->lay.gram[src]);
    pa.resid_part = c->at<double>(c->lay.rpart);
    pa.resid_dst = ds->resid[src];
    pa.fresh_dst = &ds->fresh[src];
    pa.gram_a = c->at<double>(c->lay.gram[src]);
    pa.gram_b = gb;
    pa.policy = c->opts.rho_policy;
    pa.rho0 = c->opts.rho0;
    pa.mu = c->opts.mu;
    pa.tau_incr = c->opts.tau_incr;
    pa.tau_decr = c->opts.tau_decr;
    pa.rho_state = ds->rho[n];
    pa.resid_mode = ds->resid[n];
    pa.fresh_mode = &ds->fresh[n];
    pa.Ginv = c->at<double>(c->lay.ginv[n]);
    pa.taken = &ds->taken[n];
    pa.flag = &ds->flag;
    pa.counter = &ds->counter[n];
    NW_HIP(c, launch_prep(pa, su.nprep, c->s1));
    NW_HIP(c, hipEventRecord(c->ev_prep[n], c->s1));
    ntf_status st = enqueue_mttkrp(c, n, W, ms, true);
    if (st != NTF_OK) return st;
    NW_HIP(c, hipStreamWaitEvent(ms, c->ev_prep[n], 0));
    InnerArgs ia;
    ia.part = W;
    ia.part_f64 = 1;
    ia.pstride = 0;
    ia.rowstride = su.F;
    ia.nparts = 1;
    ia.H = c->prob.H[n];
    ia.U = c->prob.U[n];
    ia.Pout = (c->opts.factor_source == 1) ? (void*)(c->ws + c->lay.prim[n]) : nullptr;
    ia.h_f64 = c->hf64();
    ia.rows = su.d[n];
    ia.F = su.F;
    ia.FL = su.FL;
    ia.Ginv = c->at<double>(c->lay.ginv[n]);
    ia.rho = ds->rho[n];
    ia.rescale = (c->opts.rescale_dual_on_rho_change || c->opts.rho_policy == NTF_RHO_ADAPTIVE) ? 1 : 0;
    ia.T = c->opts.inner_iters;
    ia.eps_abs = c->opts.inner_eps_abs;
    ia.eps_rel = c->opts.inner_eps_rel;
    ia.gram_from_primal = (c->opts.factor_source == 1) ? 1 : 0;
    ia.gram_f32 = 0;
    ia.gram_part = c->at<double>(c->lay.gpart);
    ia.resid_part = c->at<double>(c->lay.rpart);
    ia.flag = &ds->flag;
    NW_HIP(c, launch_inner(ia, su.nblk[n], ms));
  }
  return NTF_OK;
}

ntf_status launch_outer(ntf_nway_ctx* c) {
  if (!c->use_graph) {
    ntf_status st = enqueue_outer(c, c->s0);
    if (st == NTF_OK) c->outer++;
    return st;
  }
  if (!c->gexec) {
    NW_HIP(c, hipStreamBeginCapture(c->sc, hipStreamCaptureModeThreadLocal));
    ntf_status st = enqueue_outer(c, c->sc);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->sc, &g);
    if (st != NTF_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    NW_HIP(c, e);
    c->graph = g;
    NW_HIP(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
  }
  NW_HIP(c, hipGraphLaunch(c->gexec, c->s0));
  c->outer++;
  return NTF_OK;
}

ntf_status fill_stats(ntf_nway_ctx* c, ntf_nway_stats* st) {
  const Setup& su = c->su;
  const int N = su.N;
  NwState* ds = c->dstate();
  // the last mode's residual partials are still unreduced: total them apart
  NW_HIP(c, launch_finish(su.F, c->at<double>(c->lay.gpart), su.nblk[N - 1], c->at<double>(c->lay.rpart), su.nblk[N - 1],
                          c->at<double>(c->lay.gram[0]), c->at<double>(c->lay.gram[1]), c->at<double>(c->lay.W),
                          c->prob.H[N - 1], c->hf64(), su.d[N - 1], ds->fin, c->s0));
  NW_HIP(c, hipMemcpyAsync(c->host_state, ds, sizeof(NwState), hipMemcpyDeviceToHost, c->s0));
  NW_HIP(c, hipStreamSynchronize(c->s0));
  const NwState& h = *c->host_state;
  std::memset(st, 0, sizeof(*st));
  st->outer = c->outer;
  bool conv = true;
  for (int m = 0; m < N; ++m) {
    const double* r = (m == N - 1) ? h.fin : h.resid[m];
    const double rho = h.rho[m][0];
    st->rho[m] = rho;
    st->prim[m] = std::sqrt(r[0]);
    st->dual[m] = rho * std::sqrt(r[1]);
    st->norm_h[m] = std::sqrt(r[2]);
    st->norm_p[m] = std::sqrt(r[3]);
    st->norm_y[m] = rho * std::sqrt(r[4]);
    st->inner_iters_mean[m] = r[5] / (double)su.d[m];
    const double sq = std::sqrt((double)su.d[m] * su.F) * c->opts.stop_eps_abs;
    if (st->prim[m] > sq + c->opts.stop_eps_rel * std::fmax(st->norm_p[m], st->norm_h[m])) conv = false;
    if (st->dual[m] > sq + c->opts.stop_eps_rel * st->norm_y[m]) conv = false;
  }
  st->numeric_error = h.flag;
  st->converged = (c->opts.stop_eps_abs > 0 || c->opts.stop_eps_rel > 0) && conv && c->outer > 0 ? 1 : 0;
  return h.flag ? NTF_E_NUMERIC : NTF_OK;
}

}  // namespace

extern "C" {

size_t ntf_nway_workspace_bytes(const ntf_nway_problem* prob, const ntf_opts* opts) {
  if (validate_nway(prob, opts, nullptr) != NTF_OK) return 0;
  Setup su;
  if (!make_setup(su, prob, opts, 256, nullptr)) return 0;
  return make_layout(su, *opts).total;
}

const char* ntf_nway_last_error(const ntf_nway_ctx* c) { return c ? c->err.c_str() : g_nw_init_err.c_str(); }

ntf_status ntf_nway_destroy(ntf_nway_ctx* c) {
  if (!c) return NTF_E_INVAL;
  if (c->s0 || c->s1) {
    (void)hipStreamSynchronize(c->s0);
    if (c->s1) (void)hipStreamSynchronize(c->s1);
  }
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  for (int m = 0; m < kMax; ++m) {
    if (c->ev_inner[m]) (void)hipEventDestroy(c->ev_inner[m]);
    if (c->ev_prep[m]) (void)hipEventDestroy(c->ev_prep[m]);
  }
  if (c->s1) (void)hipStreamDestroy(c->s1);
  if (c->sc) (void)hipStreamDestroy(c->sc);
  if (c->host_state) (void)hipHostFree(c->host_state);
  delete c;
  return NTF_OK;
}

ntf_status ntf_nway_init(ntf_nway_ctx** out, const ntf_nway_problem* prob, const ntf_opts* opts,
                         void* workspace, size_t ws_bytes, void* stream) {
  if (!out) return NTF_E_INVAL;
  *out = nullptr;
  std::string why;
  ntf_status vs = validate_nway(prob, opts, &why);
  g_nw_init_err = why;
  if (vs != NTF_OK) return vs;
  ntf_nway_ctx* c = new (std::nothrow) ntf_nway_ctx();
  if (!c) return NTF_E_HIP;
  c->prob = *prob;
  c->opts = *opts;
  if (!make_setup(c->su, prob, opts, cu_count(), &why)) {
    g_nw_init_err = why;
    delete c;
    return NTF_E_UNSUPPORTED;
  }
  c->lay = make_layout(c->su, c->opts);
  if (!workspace || ((uintptr_t)workspace & 255)) {
    delete c;
    return NTF_E_INVAL;
  }
  if (ws_bytes < c->lay.total) {
    delete c;
    return NTF_E_WORKSPACE;
  }
  c->ws = reinterpret_cast<char*>(workspace);
  c->s0 = reinterpret_cast<hipStream_t>(stream);
  const char* ng = std::getenv("NTF_NO_GRAPH");
  c->use_graph = !(ng && ng[0] == '1');
  ntf_status st = [&]() -> ntf_status {
    const Setup& su = c->su;
    const int N = su.N;
    NW_HIP(c, hipStreamCreateWithFlags(&c->s1, hipStreamNonBlocking));
    NW_HIP(c, hipStreamCreateWithFlags(&c->sc, hipStreamNonBlocking));
    NW_HIP(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    for (int m = 0; m < N; ++m) {
      NW_HIP(c, hipEventCreateWithFlags(&c->ev_inner[m], hipEventDisableTiming));
      NW_HIP(c, hipEventCreateWithFlags(&c->ev_prep[m], hipEventDisableTiming));
    }
    NW_HIP(c, hipHostMalloc((void**)&c->host_state, sizeof(NwState), hipHostMallocDefault));
    NwState init;
    std::memset(&init, 0, sizeof(init));
    for (int m = 0; m < kMax; ++m) init.rho[m][0] = init.rho[m][1] = c->opts.rho0;
    *c->host_state = init;
    NW_HIP(c, hipMemcpyAsync(c->dstate(), c->host_state, sizeof(NwState), hipMemcpyHostToDevice, c->s0));
    int64_t total = 1;
    for (int m = 0; m < N; ++m) total *= su.d[m];
    NW_HIP(c, launch_sumsq(prob->X, prob->x_dtype, total, c->at<double>(c->lay.sumsq), 1024,
                           &c->dstate()->xnorm2, c->s0));
    const size_t es = elem_size(su.prec);
    if (c->opts.factor_source == 1) {
      for (int m = 0; m < N; ++m) {
        NW_HIP(c, hipMemcpyAsync(c->ws + c->lay.prim[m], prob->H[m], (size_t)(su.d[m] * su.F) * es,
                                 hipMemcpyDeviceToDevice, c->s0));
        if (c->opts.paper_init) {
          NW_HIP(c, hipMemsetAsync(prob->H[m], 0, (size_t)(su.d[m] * su.F) * es, c->s0));
          NW_HIP(c, hipMemsetAsync(prob->U[m], 0, (size_t)(su.d[m] * su.F) * es, c->s0));
        }
      }
    }
    // Grams of the starting factors; the last mode's partials stay for the
    // first prepare step, its residual partials start at zero
    double* gpart = c->at<double>(c->lay.gpart);
    for (int m = 0; m < N; ++m) {
      NW_HIP(c, launch_gram_part(c->feed(m), c->hf64(), su.d[m], su.F, su.rpb, 0, gpart, c->s0));
      NW_HIP(c, launch_reduce_partials(gpart, 1, (int64_t)su.F * su.F, su.F, su.nblk[m], su.F, su.F,
                                       c->at<double>(c->lay.gram[m]), c->s0, 4));
    }
    NW_HIP(c, launch_fill(c->at<double>(c->lay.rpart), (int64_t)su.nblk[N - 1] * 8, 0.0, c->s0));
    NW_HIP(c, hipStreamSynchronize(c->s0));
    return NTF_OK;
  }();
  if (st != NTF_OK) {
    g_nw_init_err = c->err;
    ntf_nway_destroy(c);
    return st;
  }
  *out = c;
  return NTF_OK;
}

ntf_status ntf_nway_step(ntf_nway_ctx* c, ntf_nway_stats* stats) {
  if (!c) return NTF_E_INVAL;
  ntf_status st = launch_outer(c);
  if (st != NTF_OK) return st;
  if (stats) return fill_stats(c, stats);
  return NTF_OK;
}

ntf_status ntf_nway_run(ntf_nway_ctx* c, int32_t max_outer, int32_t check_every, ntf_nway_stats* stats) {
  if (!c || max_outer < 0) return NTF_E_INVAL;
  const bool test = c->opts.stop_eps_abs > 0 || c->opts.stop_eps_rel > 0;
  if (test && check_every < 1) return NTF_E_INVAL;
  ntf_nway_stats local;
  for (int32_t it = 0; it < max_outer; ++it) {
    ntf_status st = launch_outer(c);
    if (st != NTF_OK) return st;
    if (test && ((it + 1) % check_every == 0 || it + 1 == max_outer)) {
      st = fill_stats(c, stats ? stats : &local);
      if (st != NTF_OK) return st;
      if ((stats ? stats : &local)->converged) return NTF_OK;
    }
  }
  if (stats && !test) {
    ntf_status st = fill_stats(c, stats);
    if (st != NTF_OK) return st;
  }
  return test ? NTF_NOT_CONVERGED : NTF_OK;
}

ntf_status ntf_nway_mttkrp(ntf_nway_ctx* c, int32_t mode, double* W_out) {
  if (!c || !W_out || mode < 0 || mode >= c->su.N) return NTF_E_INVAL;
  return enqueue_mttkrp(c, mode, W_out, c->s0, false);
}

ntf_status ntf_nway_fit(ntf_nway_ctx* c, double* rfe) {
  if (!c || !rfe) return NTF_E_INVAL;
  const Setup& su = c->su;
  const int N = su.N;
  NwState* ds = c->dstate();
  // the model on mode 1's view: H_1, the Khatri-Rao of H_2 .. H_{N-1}, H_N
  const void* H[kMax];
  for (int m = 0; m < N; ++m) H[m] = c->prob.H[m];
  const void* mid = nullptr;
  ntf_status st = group_factor(c, su.v[0].g[1], H, c->ws + c->lay.krA, c->s0, &mid);
  if (st != NTF_OK) return st;
  NW_HIP(c, launch_fit(su.v[0].plan, c->prob.X, c->prob.x_dtype, H[0], mid, H[N - 1], c->hf64(),
                       c->at<double>(c->lay.fitpart), ds->fit, c->s0, nullptr));
  double h[2];
  NW_HIP(c, hipMemcpyAsync(h, ds->fit, sizeof(h), hipMemcpyDeviceToHost, c->s0));
  NW_HIP(c, hipStreamSynchronize(c->s0));
  *rfe = h[1] > 0 ? std::sqrt(h[0] / h[1]) : 0.0;
  return NTF_OK;
}

}  // extern "C"
