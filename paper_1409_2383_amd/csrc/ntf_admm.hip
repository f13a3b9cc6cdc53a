// C-ABI host layer of libntf_admm.so: validation, workspace carving, the
// per-outer-iteration launch sequence (captured once into a HIP graph with a
// side branch for the small F x F work), statistics, fit and checkpointing.
//
// One outer iteration (eq. ADMoM_NTF; modes in the Gauss-Seidel order of
// eq. ADMM_NTF_ALS_C) is enqueued as
//
//   main stream                          side stream
//   pass 1  (W1 partials + T)            prep 1: Gram_3 of C; (G1 + rho I)^{-1}
//   inner 1  <------------------------- (join)
//   mode 2 from T                        prep 2: Gram_1 of A; (G2 + rho I)^{-1}
//   inner 2  <------------------------- (join)
//   pass 3  (W3 partials)                prep 3: Gram_2 of B; (G3 + rho I)^{-1}
//   inner 3  <------------------------- (join)
//
// so every factorisation overlaps an MTTKRP pass.  The fused inner kernel of mode n
// leaves the Gram partials of its new factor for the next prepare step.
#include "../../include/ntf_admm.h"
#include "ntf_launch.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

using namespace ntf;

namespace ntf {
ntf_status validate_opts(const ntf_opts* o, std::string* why);
int cu_count();
}

namespace {

struct DevState {
  double rho[3][2];      // [mode][0] rho of the last update, [1] rho of the update before
  double resid[3][8];    // residual totals of the last update of each mode
  double fin[10];        // statistics scratch (mode-3 residual totals, cheap fit terms)
  double xnorm2;         // ||X||_F^2
  double fit[2];         // direct fit: squared error, squared norm
  int fresh[3];          // resid[m] not yet used by the penalty rule
  int flag;              // numeric error bits
  unsigned counter[4];   // last-block tickets of the prepare kernels
  int warm_taken[3];     // rows started from the network in the last update of each mode
  int pad_;
};

struct Layout {
  size_t state = 0, T = 0, P1 = 0, P2 = 0, P3 = 0, W[3] = {0, 0, 0}, prim[3] = {0, 0, 0},
         gram[3] = {0, 0, 0}, ginv[3] = {0, 0, 0}, gpart = 0, rpart = 0, sumsq = 0, fitpart = 0,
         xr = 0, xj8 = 0, scale = 0, wx = 0, wy = 0, wact = 0, wscale = 0, wG[3] = {0, 0, 0},
         card = 0, order = 0, total = 0;
  // sparse tensors: per-mode sorted copies, MTTKRP segment carries, set-up sort scratch
  size_t sp_rec[3] = {0, 0, 0}, sp_val[3] = {0, 0, 0}, sp_tail[3] = {0, 0, 0}, sp_len[3] = {0, 0, 0},
         sp_heavy[3] = {0, 0, 0}, sp_nheavy = 0, sp_ch = 0, sp_ct = 0, sp_k0 = 0, sp_k1 = 0, sp_p0 = 0,
         sp_p1 = 0, sp_hist = 0, sp_offs = 0, sp_tot = 0;
  int64_t sp_nseg = 0;
  int sp_S = 0;
};

const int kSumsqParts = 1024;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  }
};

}  // namespace

// Compute units of the current device (256 if the query fails); shared with
// the order-N host layer.
int ntf::cu_count() {
  static int cached = 0;
  if (cached == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      cached = n;
    else
      cached = 256;
  }
  return cached;
}

namespace {

// nnz >= 0: a sparse tensor of nnz non-zeros (no dense buffers)
Layout make_layout(const Plan& p, const ntf_opts& o, int64_t nnz = -1) {
  Layout L;
  Carver c;
  const size_t es = elem_size(p.prec);
  const int64_t F = p.F;
  const bool sparse = nnz >= 0;
  L.state = c.take(sizeof(DevState));
  if (!sparse) {
    L.T = c.take((size_t)(p.I * p.J * F) * es);
    L.P1 = c.take((size_t)(p.I * p.nch1 * F) * es);
    L.P2 = c.take((size_t)((int64_t)p.nich2 * p.J * F) * es);
    L.P3 = c.take((size_t)((int64_t)p.nrc3 * p.K * F) * es);
  } else {
    const size_t n = (size_t)nnz;
    L.sp_S = sp_segment_len(p.F, p.prec == PREC_F64 ? 1 : 0);
    L.sp_nseg = (nnz + L.sp_S - 1) / L.sp_S;
    const size_t ns = (size_t)L.sp_nseg;
    for (int m = 0; m < 3; ++m) {
      L.sp_rec[m] = c.take(n * 16);
      if (p.prec == PREC_F64) L.sp_val[m] = c.take(n * 8);
      L.sp_tail[m] = c.take(ns * 4);
      L.sp_len[m] = c.take(ns * 4);
      L.sp_heavy[m] = c.take(ns * 4);
    }
    L.sp_nheavy = c.take(3 * 4);
    L.sp_ch = c.take(ns * (size_t)F * es);
    L.sp_ct = c.take(ns * (size_t)F * es);
    L.sp_k0 = c.take(n * 8);
    L.sp_k1 = c.take(n * 8);
    L.sp_p0 = c.take(n * 4);
    L.sp_p1 = c.take(n * 4);
    L.sp_hist = c.take(sp_scan_len(nnz) * 4);
    L.sp_offs = c.take(sp_scan_len(nnz) * 4);
    L.sp_tot = c.take(sp_scan_chunks(nnz) * 4);
  }
  const int64_t d[3] = {p.I, p.J, p.K};
  int maxblk = 1;
  for (int m = 0; m < 3; ++m) {
    L.W[m] = c.take((size_t)(d[m] * F) * 8);
    L.prim[m] = (o.factor_source == 1) ? c.take((size_t)(d[m] * F) * es) : 0;
    L.gram[m] = c.take((size_t)(F * F) * 8);
    L.ginv[m] = c.take((size_t)(F * F + F + 1) * 8);   // Ginv, Ginv 1, 1^T Ginv 1
    if (p.nblk_inner[m] > maxblk) maxblk = p.nblk_inner[m];
  }
  // Gram partials: the direct Gram of the prepare step (at most 16), the
  // standalone Gram partials of the statistics, and the inner sweep's own
  L.gpart = c.take((size_t)std::max<int64_t>(maxblk, 16) * F * F * 8);
  L.rpart = c.take((size_t)maxblk * 8 * 8);
  L.sumsq = c.take((size_t)kSumsqParts * 8);
  L.order = c.take(8);   // target of the one-element kernel that orders mode 2's launches
  // whole-factor projection (cardinality constraint): V, Ht^T and the factor
  // before the update, FP64 [rows][F] each, for the largest mode
  L.card = c.take((size_t)(3 * std::max(p.I, std::max(p.J, p.K)) * F) * 8);
  // fit partials; also scratch for ntf_admm_mode_problem (two Grams + partials)
  // and for the sparse fit (three Grams + partials, then the non-zero partials)
  if (!sparse)
    L.fitpart = c.take(std::max<size_t>((size_t)fit_parts(p) * 2, (size_t)(2 + maxblk) * F * F) * 8);
  else
    L.fitpart = c.take(((size_t)(3 + maxblk) * F * F + 2 * (size_t)sp_fit_parts()) * 8);
  if (p.prec == PREC_BF16 && !sparse) {
    L.xr = c.take((size_t)(p.I * p.J * p.Kp) * 2);
    L.xj8 = c.take((size_t)(p.I * p.JG * p.Kp3 * 8) * 2);
    L.scale = c.take((size_t)p.I * 4);
  }
  if (o.warm_hidden > 0) {
    const int64_t rmax = std::max(p.I, std::max(p.J, p.K));
    const int64_t D = F * (F + 1) / 2 + F;
    L.wx = c.take((size_t)(rmax * D) * 4);
    L.wy = c.take((size_t)(rmax * F) * 4);
    L.wact = c.take((size_t)(2 * rmax * o.warm_hidden) * 4);
    L.wscale = c.take((size_t)rmax * 4);
    for (int m = 0; m < 3; ++m) L.wG[m] = c.take((size_t)(F * F) * 8);
  }
  L.total = c.off;
  return L;
}

}  // namespace

struct ntf_admm_ctx {
  ntf_problem prob;
  ntf_opts opts;
  Plan plan;
  Layout lay;
  char* ws = nullptr;
  hipStream_t s0 = nullptr, s1 = nullptr;  // caller's stream, side stream
  hipStream_t sc = nullptr;                 // internal stream the graph is captured on
  hipEvent_t ev_fork = nullptr, ev_inner[3] = {nullptr, nullptr, nullptr},
             ev_prep[3] = {nullptr, nullptr, nullptr};
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool use_graph = true;
  int64_t outer = 0;
  DevState* host_state = nullptr;  // pinned
  bool warm_on = false;
  ntf_mlp warm{};
  ntf_constraints cons{};   // all zero: every factor non-negative
  bool sparse = false;      // tensor given by its non-zeros (ntf_admm_init_sparse)
  int64_t nnz = 0;
  int nheavy[3] = {0, 0, 0};  // rows cut into more than kLightPieces segment pieces, per mode
  std::string err;

  template <typename T> T* at(size_t off) { return reinterpret_cast<T*>(ws + off); }
  DevState* dstate() { return at<DevState>(lay.state); }
  int hf64() const { return plan.prec == PREC_F64 ? 1 : 0; }
  const void* feed(int m) const {
    return (opts.factor_source == 1) ? (const void*)(ws + lay.prim[m]) : (const void*)prob.H[m];
  }
};

#define NTF_HIP(ctx, call)                                                             \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      if (ctx) (ctx)->err = std::string(#call) + ": " + hipGetErrorString(e_);        \
      return NTF_E_HIP;                                                                \
    }                                                                                  \
  } while (0)

static ntf_status validate(const ntf_problem* pr, const ntf_opts* o, std::string* why) {
  auto fail = [&](const char* m) {
    if (why) *why = m;
    return NTF_E_INVAL;
  };
  if (!pr || !o) return fail("null problem or options");
  for (int m = 0; m < 3; ++m)
    if (pr->dims[m] < 1 || pr->dims[m] > (int64_t)1 << 31) return fail("dims must be in [1, 2^31]");
  if (pr->F < 1 || pr->F > 64) return fail("F must be in [1, 64]");
  if (o->precision != NTF_PREC_F32 && o->precision != NTF_PREC_BF16_MIXED &&
      o->precision != NTF_PREC_F64)
    return fail("unknown precision");
  if ((o->precision == NTF_PREC_F64) != (pr->x_dtype == 1)) return fail("x_dtype does not match precision");
  if (pr->x_dtype != 0 && pr->x_dtype != 1) return fail("x_dtype must be 0 or 1");
  if (!pr->X) return fail("null X");
  if (((uintptr_t)pr->X) & 15) return fail("X not 16-byte aligned");
  for (int m = 0; m < 3; ++m) {
    if (!pr->H[m] || !pr->U[m]) return fail("null factor or dual");
    if ((((uintptr_t)pr->H[m]) | ((uintptr_t)pr->U[m])) & 15) return fail("factor/dual not 16-byte aligned");
  }
  {
    const ntf_status vo = validate_opts(o, why);
    if (vo != NTF_OK) return vo;
  }
  const int64_t I = pr->dims[0], J = pr->dims[1], K = pr->dims[2];
  if (I * J > ((int64_t)1 << 40) || I * J * K > ((int64_t)1 << 46)) return fail("tensor too large");
  return NTF_OK;
}

// Option checks shared by every entry point that takes ntf_opts.
ntf_status ntf::validate_opts(const ntf_opts* o, std::string* why) {
  auto fail = [&](const char* m) {
    if (why) *why = m;
    return NTF_E_INVAL;
  };
  if (o->inner_iters < 1) return fail("inner_iters must be >= 1");
  if (o->rho_policy < 0 || o->rho_policy > 2) return fail("unknown rho_policy");
  if (!(o->rho0 > 0.0)) return fail("rho0 must be > 0");
  if (o->rho_policy == NTF_RHO_ADAPTIVE && !(o->mu > 1.0 && o->tau_incr > 1.0 && o->tau_decr > 1.0))
    return fail("mu, tau_incr, tau_decr must be > 1");
  if (o->inner_eps_abs < 0 || o->inner_eps_rel < 0 || o->stop_eps_abs < 0 || o->stop_eps_rel < 0)
    return fail("tolerances must be >= 0");
  if (o->factor_source != 0 && o->factor_source != 1) return fail("factor_source must be 0 or 1");
  if (o->paper_init && o->factor_source != 1) return fail("paper_init needs factor_source 1");
  for (int q = 0; q < 3; ++q)
    if (o->reserved[q] != 0) return fail("reserved fields must be zero");
  if (o->warm_hidden < 0 || o->warm_hidden > 1024) return fail("warm_hidden must be in [0, 1024]");
  return NTF_OK;
}

static ntf_status validate_sparse(const ntf_sparse_problem* pr, const ntf_opts* o, std::string* why) {
  auto fail = [&](const char* m, ntf_status st = NTF_E_INVAL) {
    if (why) *why = m;
    return st;
  };
  if (!pr || !o) return fail("null problem or options");
  for (int m = 0; m < 3; ++m)
    if (pr->dims[m] < 1 || pr->dims[m] > (int64_t)1 << 31) return fail("dims must be in [1, 2^31]");
  if (pr->F < 1 || pr->F > 64) return fail("F must be in [1, 64]");
  if (o->precision == NTF_PREC_BF16_MIXED)
    return fail("sparse tensors run in NTF_PREC_F32 or NTF_PREC_F64", NTF_E_UNSUPPORTED);
  if (o->precision != NTF_PREC_F32 && o->precision != NTF_PREC_F64) return fail("unknown precision");
  if (pr->x_dtype != 0 && pr->x_dtype != 1) return fail("x_dtype must be 0 or 1");
  if ((o->precision == NTF_PREC_F64) != (pr->x_dtype == 1)) return fail("x_dtype does not match precision");
  if (pr->nnz < 0 || pr->nnz >= ((int64_t)1 << 31)) return fail("nnz must be in [0, 2^31)");
  if (pr->nnz > 0 && (!pr->idx || !pr->val)) return fail("null coordinates or values");
  if ((((uintptr_t)pr->idx) | ((uintptr_t)pr->val)) & 15) return fail("coordinates/values not 16-byte aligned");
  if (sp_key_bits(pr->dims) > 64)
    return fail("dims too large for the 64-bit sort key of the sparse set-up", NTF_E_UNSUPPORTED);
  for (int m = 0; m < 3; ++m) {
    if (!pr->H[m] || !pr->U[m]) return fail("null factor or dual");
    if ((((uintptr_t)pr->H[m]) | ((uintptr_t)pr->U[m])) & 15) return fail("factor/dual not 16-byte aligned");
  }
  if (o->warm_hidden != 0) return fail("the learned warm start is not offered for sparse tensors", NTF_E_UNSUPPORTED);
  return validate_opts(o, why);
}

// Plan of a sparse problem: only the inner-sweep and prepare geometry.
static void make_plan_sparse(Plan& p, int prec, const int64_t dims[3], int F) {
  p = Plan();
  p.prec = prec;
  p.I = dims[0];
  p.J = dims[1];
  p.K = dims[2];
  p.F = F;
  int FL = 4;
  while (FL < F) FL <<= 1;
  p.FL = FL;
  p.rpb = inner_rows_per_block(FL);
  for (int m = 0; m < 3; ++m) p.nblk_inner[m] = (int)((dims[m] + p.rpb - 1) / p.rpb);
  p.nprep = (int)std::max<int64_t>(1, ((int64_t)F * F + 63) / 64);
}

extern "C" {

const char* ntf_status_str(ntf_status s) {
  switch (s) {
    case NTF_OK: return "ok";
    case NTF_NOT_CONVERGED: return "not converged";
    case NTF_E_INVAL: return "invalid argument";
    case NTF_E_WORKSPACE: return "workspace too small";
    case NTF_E_HIP: return "HIP runtime error";
    case NTF_E_NUMERIC: return "numeric failure (non-PD system or NaN/Inf)";
    case NTF_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

static thread_local std::string g_init_err;  // why the last failed init on this thread failed

const char* ntf_admm_last_error(const ntf_admm_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_init_err.c_str();
}

size_t ntf_admm_workspace_bytes(const ntf_problem* prob, const ntf_opts* opts) {
  if (validate(prob, opts, nullptr) != NTF_OK) return 0;
  Plan p;
  if (!make_plan(p, opts->precision, prob->dims, prob->F, 256)) return 0;
  return make_layout(p, *opts).total;
}

size_t ntf_admm_sparse_workspace_bytes(const ntf_sparse_problem* prob, const ntf_opts* opts) {
  if (validate_sparse(prob, opts, nullptr) != NTF_OK) return 0;
  Plan p;
  make_plan_sparse(p, opts->precision, prob->dims, prob->F);
  return make_layout(p, *opts, prob->nnz).total;
}

}  // extern "C"

// Gram of one factor (as fed to the updates) by the partition and order of
// the prepare step's direct Gram: FP64 partials of whole 64-row chunks,
// reduced in 4 fixed groups, so both give bitwise identical Grams.
static hipError_t direct_gram(ntf_admm_ctx* c, int m, double* out, hipStream_t s) {
  const Plan& p = c->plan;
  const int64_t d[3] = {p.I, p.J, p.K};
  int64_t rpp;
  int nb;
  gram_split(d[m], &rpp, &nb);
  double* gpart = c->at<double>(c->lay.gpart);
  hipError_t e = launch_gram_direct(c->feed(m), c->hf64(), d[m], p.F, rpp, gpart, s);
  if (e != hipSuccess) return e;
  return launch_reduce_partials(gpart, 1, (int64_t)p.F * p.F, p.F, nb, p.F, p.F, out, s, 4);
}

// Grams of the three current factors, and zero residual partials for the
// first prepare step.
static ntf_status compute_grams(ntf_admm_ctx* c) {
  const Plan& p = c->plan;
  for (int m = 0; m < 3; ++m) NTF_HIP(c, direct_gram(c, m, c->at<double>(c->lay.gram[m]), c->s0));
  NTF_HIP(c, launch_fill(c->at<double>(c->lay.rpart), (int64_t)p.nblk_inner[2] * 8, 0.0, c->s0));
  return NTF_OK;
}

static void prep_args(ntf_admm_ctx* c, int m, PrepArgs& a) {
  // prepare mode m: reduce the partials of mode (m+2)%3 (the one updated last)
  const Plan& p = c->plan;
  const int src = (m + 2) % 3;
  const int oth = (m + 1) % 3;  // the other Gram in G_m besides gram[src]
  DevState* ds = c->dstate();
  a = PrepArgs();
  a.F = p.F;
  // the Gram of the mode updated last, directly from that factor
  const int64_t d[3] = {p.I, p.J, p.K};
  a.gram_h = c->feed(src);
  a.h_f64 = c->hf64();
  a.gram_rows = d[src];
  gram_split(d[src], &a.gram_rpp, &a.gram_nb);
  a.gram_scratch = c->at<double>(c->lay.gpart);
  a.nparts = p.nblk_inner[src];   // its residual partials
  a.gram_dst = c->at<double>(c->lay.gram[src]);
  a.resid_part = c->at<double>(c->lay.rpart);
  a.resid_dst = ds->resid[src];
  a.fresh_dst = &ds->fresh[src];
  a.gram_a = c->at<double>(c->lay.gram[src]);
  a.gram_b = c->at<double>(c->lay.gram[oth]);
  a.policy = c->opts.rho_policy;
  a.rho0 = c->opts.rho0;
  a.mu = c->opts.mu;
  a.tau_incr = c->opts.tau_incr;
  a.tau_decr = c->opts.tau_decr;
  a.rho_state = ds->rho[m];
  a.resid_mode = ds->resid[m];
  a.fresh_mode = &ds->fresh[m];
  a.Ginv = c->at<double>(c->lay.ginv[m]);
  a.G_out = c->warm_on ? c->at<double>(c->lay.wG[m]) : nullptr;
  a.taken = &ds->warm_taken[m];
  a.flag = &ds->flag;
  a.counter = &ds->counter[m];
}

static void inner_args(ntf_admm_ctx* c, int m, InnerArgs& a, bool from_p1 = false) {
  const Plan& p = c->plan;
  const int64_t d[3] = {p.I, p.J, p.K};
  DevState* ds = c->dstate();
  a = InnerArgs();
  if (from_p1) {
    // W_1 summed by the inner sweep itself from pass 1's partials [I][nch][F]
    // (in chunk order), and written out for the statistics
    a.part = c->ws + c->lay.P1;
    a.part_f64 = c->hf64();
    a.pstride = p.F;
    a.rowstride = (int64_t)p.nch1 * p.F;
    a.nparts = p.nch1;
  } else {
    // W_m was reduced from the MTTKRP partials by the grouped reduction
    a.part = c->ws + c->lay.W[m];
    a.part_f64 = 1;
    a.pstride = 0;
    a.rowstride = p.F;
    a.nparts = 1;
  }
  a.Wout = from_p1 ? c->at<double>(c->lay.W[0]) : nullptr;
  a.H = c->prob.H[m];
  a.U = c->prob.U[m];
  a.Pout = (c->opts.factor_source == 1) ? (void*)(c->ws + c->lay.prim[m]) : nullptr;
  a.h_f64 = c->hf64();
  a.rows = d[m];
  a.F = p.F;
  a.FL = p.FL;
  a.Ginv = c->at<double>(c->lay.ginv[m]);
  a.proj = (c->cons.kind[m] == NTF_CONS_BOX) ? 1 : (c->cons.kind[m] == NTF_CONS_PMF_ROWS) ? 2 : 0;
  a.lo = c->cons.lo[m];
  a.hi = c->cons.hi[m];
  a.rho = ds->rho[m];
  a.rescale = (c->opts.rescale_dual_on_rho_change || c->opts.rho_policy == NTF_RHO_ADAPTIVE) ? 1 : 0;
  a.T = c->opts.inner_iters;
  a.eps_abs = c->opts.inner_eps_abs;
  a.eps_rel = c->opts.inner_eps_rel;
  a.gram_from_primal = (c->opts.factor_source == 1) ? 1 : 0;
  a.gram_f32 = (p.prec == PREC_BF16) ? 1 : 0;
  a.gram_part = nullptr;   // the prepare step forms the Gram from the factor itself
  a.resid_part = c->at<double>(c->lay.rpart);
  a.flag = &ds->flag;
}

// Inner sweep of mode m.  A factor under the cardinality constraint couples
// every row in its projection: each inner iteration is the row-wise solve
// (projection deferred) followed by the whole-factor projection, then the
// Gram partials of the updated factor.
static ntf_status enqueue_inner(ntf_admm_ctx* c, int m, hipStream_t ms, bool from_p1 = false) {
  const Plan& p = c->plan;
  InnerArgs ia;
  inner_args(c, m, ia, from_p1);
  if (c->cons.kind[m] != NTF_CONS_CARDINALITY) {
    NTF_HIP(c, launch_inner(ia, p.nblk_inner[m], ms));
    return NTF_OK;
  }
  const int64_t d[3] = {p.I, p.J, p.K};
  const int64_t n = d[m] * p.F;
  double* V = c->at<double>(c->lay.card);
  double* Xt = V + n;
  double* H0 = Xt + n;
  const int T = ia.T;
  ia.T = 1;
  ia.proj = 3;
  ia.dv = V;
  ia.dx = Xt;
  for (int t = 0; t < T; ++t) {
    ia.dh0 = (t == 0) ? H0 : nullptr;
    if (t > 0) ia.rescale = 0;   // U is already in the scale of this update's rho
    NTF_HIP(c, launch_inner(ia, p.nblk_inner[m], ms));
    NTF_HIP(c, launch_card_project(V, Xt, H0, ia.H, ia.U, ia.Pout, ia.h_f64, n, c->cons.card[m],
                                   (double)T * (double)d[m], ia.resid_part, p.nblk_inner[m], ms));
  }
  return NTF_OK;
}

// Learned warm start of mode m (after its W and its prepare step): row
// inputs, network forward, and the per-row KKT judge that writes the chosen
// starting point into H_m, U_m.
static ntf_status enqueue_warm(ntf_admm_ctx* c, int m, hipStream_t ms) {
  const Plan& p = c->plan;
  const int64_t d[3] = {p.I, p.J, p.K};
  DevState* ds = c->dstate();
  float* X = c->at<float>(c->lay.wx);
  float* Y = c->at<float>(c->lay.wy);
  float* sc = c->at<float>(c->lay.wscale);
  const double* G = c->at<double>(c->lay.wG[m]);
  const double* W = c->at<double>(c->lay.W[m]);
  NTF_HIP(c, mlp_features(G, W, d[m], p.F, ds->rho[m], 0.0, X, sc, ms));
  NTF_HIP(c, mlp_forward(c->warm.params, c->warm.dtype, p.F, c->warm.hidden, X, d[m], Y,
                         c->at<float>(c->lay.wact), ms));
  const int rescale = (c->opts.rescale_dual_on_rho_change || c->opts.rho_policy == NTF_RHO_ADAPTIVE) ? 1 : 0;
  NTF_HIP(c, mlp_judge(Y, sc, G, W, c->prob.H[m], c->prob.U[m], c->hf64(), d[m], p.F, p.FL,
                       ds->rho[m], rescale, &ds->warm_taken[m], ms));
  return NTF_OK;
}

// Sparse MTTKRP of mode m into W (the other factors as the feed holds them).
static hipError_t sparse_mttkrp(ntf_admm_ctx* c, int m, double* W, hipStream_t ms) {
  const Plan& p = c->plan;
  const int64_t d[3] = {p.I, p.J, p.K};
  const int ma = (m == 0) ? 1 : 0, mb = (m == 2) ? 1 : 2;
  SpModeArgs a;
  a.rec = c->at<int4>(c->lay.sp_rec[m]);
  a.val = c->hf64() ? (const void*)(c->ws + c->lay.sp_val[m]) : nullptr;
  a.Fa = c->feed(ma);
  a.Fb = c->feed(mb);
  a.f64 = c->hf64();
  a.F = p.F;
  a.S = c->lay.sp_S;
  a.n = c->nnz;
  a.nseg = c->lay.sp_nseg;
  a.rows = d[m];
  a.W = W;
  a.tail = c->at<int32_t>(c->lay.sp_tail[m]);
  a.len = c->at<int32_t>(c->lay.sp_len[m]);
  a.heavy = c->at<int32_t>(c->lay.sp_heavy[m]);
  a.nheavy = c->nheavy[m];
  a.carry_h = c->ws + c->lay.sp_ch;
  a.carry_t = c->ws + c->lay.sp_ct;
  return sp_mttkrp(a, ms);
}

// One outer iteration of a sparse tensor: per mode, the prepare step on s1
// beside the sparse MTTKRP, then the inner sweep.
static ntf_status enqueue_outer_sparse(ntf_admm_ctx* c, hipStream_t ms) {
  const Plan& p = c->plan;
  PrepArgs pa;
  for (int m = 0; m < 3; ++m) {
    NTF_HIP(c, hipEventRecord(m == 0 ? c->ev_fork : c->ev_inner[m - 1], ms));
    NTF_HIP(c, hipStreamWaitEvent(c->s1, m == 0 ? c->ev_fork : c->ev_inner[m - 1], 0));
    prep_args(c, m, pa);
    NTF_HIP(c, launch_prep(pa, p.nprep, c->s1));
    NTF_HIP(c, hipEventRecord(c->ev_prep[m], c->s1));
    NTF_HIP(c, sparse_mttkrp(c, m, c->at<double>(c->lay.W[m]), ms));
    NTF_HIP(c, hipStreamWaitEvent(ms, c->ev_prep[m], 0));
    ntf_status st = enqueue_inner(c, m, ms);
    if (st != NTF_OK) return st;
  }
  return NTF_OK;
}

// Whether a mode's MTTKRP pass is captured before its prepare step.  The
// graph runs the node captured first on the launching queue, next to the
// inner sweeps around it: the handoffs inner -> pass -> inner then take 5-6
// us instead of 10-14 across queues.  The prepare step captured second must
// still find CUs the pass leaves free (each pass block takes a CU: 512
// threads and, in pass 3, most of the LDS); otherwise it would wait for the
// whole pass, so the order stays prepare first.
static bool pass_first(const ntf_admm_ctx* c, int m) {
  const Plan& p = c->plan;
  if (m == 1) return false;
  const int64_t d[3] = {p.I, p.J, p.K};
  int64_t rpp;
  int nb;
  gram_split(d[(m + 2) % 3], &rpp, &nb);
  const int64_t pass = (m == 0) ? p.grid1
                                : (p.prec == PREC_BF16 ? (int64_t)p.nch3 * p.bpc3 : (int64_t)p.nb3 * p.nkg3);
  return pass + nb + 1 <= cu_count();
}

// Enqueue one outer iteration on `ms` with the prepare kernels on s1.
static ntf_status enqueue_outer(ntf_admm_ctx* c, hipStream_t ms) {
  if (c->sparse) return enqueue_outer_sparse(c, ms);
  const Plan& p = c->plan;
  const __bf16* xr = p.prec == PREC_BF16 ? c->at<__bf16>(c->lay.xr) : nullptr;
  const __bf16* xj8 = p.prec == PREC_BF16 ? c->at<__bf16>(c->lay.xj8) : nullptr;
  const float* scale = p.prec == PREC_BF16 ? c->at<float>(c->lay.scale) : nullptr;
  void* T = c->ws + c->lay.T;
  PrepArgs pa;
  // mode 1 (A): prepare on the side while pass 1 streams X
  NTF_HIP(c, hipEventRecord(c->ev_fork, ms));
  NTF_HIP(c, hipStreamWaitEvent(c->s1, c->ev_fork, 0));
  const bool pf1 = pass_first(c, 0);
  if (pf1)
    NTF_HIP(c, launch_pass1(p, c->prob.X, xr, scale, c->feed(1), c->feed(2), T, c->ws + c->lay.P1, ms));
  prep_args(c, 0, pa);
  NTF_HIP(c, launch_prep(pa, p.nprep, c->s1));
  NTF_HIP(c, hipEventRecord(c->ev_prep[0], c->s1));
  if (!pf1)
    NTF_HIP(c, launch_pass1(p, c->prob.X, xr, scale, c->feed(1), c->feed(2), T, c->ws + c->lay.P1, ms));
  // The warm start reads W_1 before the inner sweep: reduce it first.  Without
  // it the inner sweep sums pass 1's (few, per row-chunk) partials itself.
  const bool w1_in_inner = !c->warm_on;
  if (!w1_in_inner)
    NTF_HIP(c, launch_reduce_partials(c->ws + c->lay.P1, c->hf64(), p.F, (int64_t)p.nch1 * p.F,
                                      p.nch1, p.I, p.F, c->at<double>(c->lay.W[0]), ms, 16));
  NTF_HIP(c, hipStreamWaitEvent(ms, c->ev_prep[0], 0));
  if (c->warm_on) {
    ntf_status w = enqueue_warm(c, 0, ms);
    if (w != NTF_OK) return w;
  }
  {
    ntf_status st = enqueue_inner(c, 0, ms, w1_in_inner);
    if (st != NTF_OK) return st;
  }
  // mode 2 (B)
  NTF_HIP(c, hipEventRecord(c->ev_inner[0], ms));
  NTF_HIP(c, hipStreamWaitEvent(c->s1, c->ev_inner[0], 0));
  prep_args(c, 1, pa);
  NTF_HIP(c, launch_prep(pa, p.nprep, c->s1));
  NTF_HIP(c, hipEventRecord(c->ev_prep[1], c->s1));
  // The mode-2 prepare step is the longer branch here.  A one-element kernel
  // ahead of the mode-2 MTTKRP lets the prepare step's blocks be dispatched
  // first, on CUs of their own: when the MTTKRP's blocks come first, the
  // prepare step shares their CUs and takes 72 us instead of 55.
  NTF_HIP(c, launch_fill(c->at<double>(c->lay.order), 1, 0.0, ms));
  NTF_HIP(c, launch_mode2(p, T, c->feed(0), c->ws + c->lay.P2, ms));
  NTF_HIP(c, launch_reduce_partials(c->ws + c->lay.P2, c->hf64(), p.J * p.F, p.F, p.nich2, p.J, p.F,
                                    c->at<double>(c->lay.W[1]), ms, 16));
  NTF_HIP(c, hipStreamWaitEvent(ms, c->ev_prep[1], 0));
  if (c->warm_on) {
    ntf_status w = enqueue_warm(c, 1, ms);
    if (w != NTF_OK) return w;
  }
  {
    ntf_status st = enqueue_inner(c, 1, ms);
    if (st != NTF_OK) return st;
  }
  // mode 3 (C)
  NTF_HIP(c, hipEventRecord(c->ev_inner[1], ms));
  NTF_HIP(c, hipStreamWaitEvent(c->s1, c->ev_inner[1], 0));
  const bool pf3 = pass_first(c, 2);
  if (pf3) NTF_HIP(c, launch_pass3(p, c->prob.X, xj8, scale, c->feed(0), c->feed(1), c->ws + c->lay.P3, ms));
  prep_args(c, 2, pa);
  NTF_HIP(c, launch_prep(pa, p.nprep, c->s1));
  NTF_HIP(c, hipEventRecord(c->ev_prep[2], c->s1));
  if (!pf3) NTF_HIP(c, launch_pass3(p, c->prob.X, xj8, scale, c->feed(0), c->feed(1), c->ws + c->lay.P3, ms));
  NTF_HIP(c, launch_reduce_partials(c->ws + c->lay.P3, c->hf64(), p.K * p.F, p.F, p.nrc3, p.K, p.F,
                                    c->at<double>(c->lay.W[2]), ms, 16));
  NTF_HIP(c, hipStreamWaitEvent(ms, c->ev_prep[2], 0));
  if (c->warm_on) {
    ntf_status w = enqueue_warm(c, 2, ms);
    if (w != NTF_OK) return w;
  }
  {
    ntf_status st = enqueue_inner(c, 2, ms);
    if (st != NTF_OK) return st;
  }
  return NTF_OK;
}

static ntf_status launch_outer(ntf_admm_ctx* c) {
  if (!c->use_graph) {
    ntf_status st = enqueue_outer(c, c->s0);
    if (st == NTF_OK) c->outer++;
    return st;
  }
  if (!c->gexec) {
    NTF_HIP(c, hipStreamBeginCapture(c->sc, hipStreamCaptureModeThreadLocal));
    ntf_status st = enqueue_outer(c, c->sc);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->sc, &g);
    if (st != NTF_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    NTF_HIP(c, e);
    c->graph = g;
    NTF_HIP(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
  }
  NTF_HIP(c, hipGraphLaunch(c->gexec, c->s0));
  c->outer++;
  return NTF_OK;
}

// Residual totals of the last mode and the fit terms, into out[0..9]: the
// Gram of mode 3 is formed from the factor (partials in the Gram scratch).
static hipError_t finish_stats(ntf_admm_ctx* c, double* out) {
  const Plan& p = c->plan;
  int64_t rpp;
  int nb;
  gram_split(p.K, &rpp, &nb);
  double* gpart = c->at<double>(c->lay.gpart);
  hipError_t e = launch_gram_direct(c->feed(2), c->hf64(), p.K, p.F, rpp, gpart, c->s0);
  if (e != hipSuccess) return e;
  return launch_finish(p.F, gpart, nb, c->at<double>(c->lay.rpart), p.nblk_inner[2],
                       c->at<double>(c->lay.gram[0]), c->at<double>(c->lay.gram[1]),
                       c->at<double>(c->lay.W[2]), c->prob.H[2], c->hf64(), p.K, out, c->s0);
}

static ntf_status fill_stats(ntf_admm_ctx* c, ntf_stats* st) {
  const Plan& p = c->plan;
  DevState* ds = c->dstate();
  NTF_HIP(c, finish_stats(c, ds->fin));
  NTF_HIP(c, hipMemcpyAsync(c->host_state, ds, sizeof(DevState), hipMemcpyDeviceToHost, c->s0));
  NTF_HIP(c, hipStreamSynchronize(c->s0));
  const DevState& h = *c->host_state;
  std::memset(st, 0, sizeof(*st));
  st->outer = c->outer;
  const int64_t d[3] = {p.I, p.J, p.K};
  bool conv = true;
  for (int m = 0; m < 3; ++m) {
    const double* r = (m == 2) ? h.fin : h.resid[m];
    const double rho = h.rho[m][0];
    st->rho[m] = rho;
    st->prim[m] = std::sqrt(r[0]);
    st->dual[m] = rho * std::sqrt(r[1]);
    st->norm_h[m] = std::sqrt(r[2]);
    st->norm_p[m] = std::sqrt(r[3]);
    st->norm_y[m] = rho * std::sqrt(r[4]);
    st->inner_iters_mean[m] = r[5] / (double)d[m];
    const double sq = std::sqrt((double)d[m] * p.F) * c->opts.stop_eps_abs;
    if (st->prim[m] > sq + c->opts.stop_eps_rel * std::fmax(st->norm_p[m], st->norm_h[m])) conv = false;
    if (st->dual[m] > sq + c->opts.stop_eps_rel * st->norm_y[m]) conv = false;
  }
  const double e2 = h.xnorm2 - 2.0 * h.fin[8] + h.fin[9];
  st->rfe_cheap = h.xnorm2 > 0 ? std::sqrt(std::fmax(e2, 0.0) / h.xnorm2) : 0.0;
  st->numeric_error = h.flag;
  for (int m = 0; m < 3; ++m) st->warm_taken[m] = h.warm_taken[m];
  st->converged = (c->opts.stop_eps_abs > 0 || c->opts.stop_eps_rel > 0) && conv ? 1 : 0;
  if (c->outer == 0) st->converged = 0;
  return h.flag ? NTF_E_NUMERIC : NTF_OK;
}

extern "C" {

// Streams, events, the pinned state mirror and the device state block.
static ntf_status ctx_setup(ntf_admm_ctx* c) {
  NTF_HIP(c, hipStreamCreateWithFlags(&c->s1, hipStreamNonBlocking));
  NTF_HIP(c, hipStreamCreateWithFlags(&c->sc, hipStreamNonBlocking));
  NTF_HIP(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  for (int m = 0; m < 3; ++m) {
    NTF_HIP(c, hipEventCreateWithFlags(&c->ev_inner[m], hipEventDisableTiming));
    NTF_HIP(c, hipEventCreateWithFlags(&c->ev_prep[m], hipEventDisableTiming));
  }
  NTF_HIP(c, hipHostMalloc((void**)&c->host_state, sizeof(DevState), hipHostMallocDefault));
  DevState init;
  std::memset(&init, 0, sizeof(init));
  for (int m = 0; m < 3; ++m) init.rho[m][0] = init.rho[m][1] = c->opts.rho0;
  *c->host_state = init;
  NTF_HIP(c, hipMemcpyAsync(c->dstate(), c->host_state, sizeof(DevState), hipMemcpyHostToDevice, c->s0));
  return NTF_OK;
}

// Paper initialisation (the given factors seed the primal; auxiliary and
// duals start at zero) and the Grams of the starting factors.
static ntf_status ctx_seed(ntf_admm_ctx* c) {
  const Plan& p = c->plan;
  const int64_t d[3] = {p.I, p.J, p.K};
  const size_t es = elem_size(p.prec);
  if (c->opts.factor_source == 1) {
    for (int m = 0; m < 3; ++m) {
      NTF_HIP(c, hipMemcpyAsync(c->ws + c->lay.prim[m], c->prob.H[m], (size_t)(d[m] * p.F) * es,
                                hipMemcpyDeviceToDevice, c->s0));
      if (c->opts.paper_init) {
        NTF_HIP(c, hipMemsetAsync(c->prob.H[m], 0, (size_t)(d[m] * p.F) * es, c->s0));
        NTF_HIP(c, hipMemsetAsync(c->prob.U[m], 0, (size_t)(d[m] * p.F) * es, c->s0));
      }
    }
  }
  return compute_grams(c);
}

static ntf_status ctx_attach(ntf_admm_ctx* c, void* workspace, size_t ws_bytes, void* stream) {
  if (!workspace || ((uintptr_t)workspace & 255)) return NTF_E_INVAL;
  if (ws_bytes < c->lay.total) return NTF_E_WORKSPACE;
  c->ws = reinterpret_cast<char*>(workspace);
  c->s0 = reinterpret_cast<hipStream_t>(stream);
  const char* ng = std::getenv("NTF_NO_GRAPH");
  c->use_graph = !(ng && ng[0] == '1');
  return NTF_OK;
}

ntf_status ntf_admm_init(ntf_admm_ctx** out, const ntf_problem* prob, const ntf_opts* opts,
                         void* workspace, size_t ws_bytes, void* stream) {
  if (!out) return NTF_E_INVAL;
  *out = nullptr;
  std::string why;
  ntf_status vs = validate(prob, opts, &why);
  g_init_err = why;
  if (vs != NTF_OK) return vs;
  ntf_admm_ctx* c = new (std::nothrow) ntf_admm_ctx();
  if (!c) return NTF_E_HIP;
  c->prob = *prob;
  c->opts = *opts;
  if (!make_plan(c->plan, opts->precision, prob->dims, prob->F, cu_count())) {
    delete c;
    return NTF_E_UNSUPPORTED;
  }
  c->lay = make_layout(c->plan, c->opts);
  {
    const ntf_status a = ctx_attach(c, workspace, ws_bytes, stream);
    if (a != NTF_OK) {
      delete c;
      return a;
    }
  }
  ntf_status st = [&]() -> ntf_status {
    ntf_status q = ctx_setup(c);
    if (q != NTF_OK) return q;
    const Plan& p = c->plan;
    // bfloat16 copies
    if (p.prec == PREC_BF16)
      NTF_HIP(c, launch_quantize((const float*)prob->X, p, c->at<__bf16>(c->lay.xr),
                                 c->at<__bf16>(c->lay.xj8), c->at<float>(c->lay.scale), c->s0));
    NTF_HIP(c, launch_sumsq(prob->X, prob->x_dtype, p.I * p.J * p.K, c->at<double>(c->lay.sumsq),
                            kSumsqParts, &c->dstate()->xnorm2, c->s0));
    q = ctx_seed(c);
    if (q != NTF_OK) return q;
    NTF_HIP(c, hipStreamSynchronize(c->s0));
    return NTF_OK;
  }();
  if (st != NTF_OK) {
    g_init_err = c->err;
    ntf_admm_destroy(c);
    return st;
  }
  *out = c;
  return NTF_OK;
}

ntf_status ntf_admm_init_sparse(ntf_admm_ctx** out, const ntf_sparse_problem* prob,
                                const ntf_opts* opts, void* workspace, size_t ws_bytes,
                                void* stream) {
  if (!out) return NTF_E_INVAL;
  *out = nullptr;
  std::string why;
  ntf_status vs = validate_sparse(prob, opts, &why);
  g_init_err = why;
  if (vs != NTF_OK) return vs;
  ntf_admm_ctx* c = new (std::nothrow) ntf_admm_ctx();
  if (!c) return NTF_E_HIP;
  c->sparse = true;
  c->nnz = prob->nnz;
  std::memset(&c->prob, 0, sizeof(c->prob));
  for (int m = 0; m < 3; ++m) {
    c->prob.dims[m] = prob->dims[m];
    c->prob.H[m] = prob->H[m];
    c->prob.U[m] = prob->U[m];
  }
  c->prob.F = prob->F;
  c->prob.x_dtype = prob->x_dtype;
  c->opts = *opts;
  make_plan_sparse(c->plan, opts->precision, prob->dims, prob->F);
  c->lay = make_layout(c->plan, c->opts, prob->nnz);
  {
    const ntf_status a = ctx_attach(c, workspace, ws_bytes, stream);
    if (a != NTF_OK) {
      delete c;
      return a;
    }
  }
  ntf_status st = [&]() -> ntf_status {
    ntf_status q = ctx_setup(c);
    if (q != NTF_OK) return q;
    DevState* ds = c->dstate();
    const int64_t n = prob->nnz;
    // coordinates in range before anything is built from them
    NTF_HIP(c, sp_check(prob->idx, n, prob->dims, &ds->flag, c->s0));
    int flag = 0;
    NTF_HIP(c, hipMemcpyAsync(&c->host_state->flag, &ds->flag, sizeof(int), hipMemcpyDeviceToHost, c->s0));
    NTF_HIP(c, hipStreamSynchronize(c->s0));
    flag = c->host_state->flag;
    if (flag & kSparseFlagRange) {
      c->err = "a coordinate lies outside the tensor";
      return NTF_E_INVAL;
    }
    for (int m = 0; m < 3; ++m) {
      SpBuildArgs b;
      b.idx = prob->idx;
      b.val = prob->val;
      b.val_f64 = prob->x_dtype;
      b.n = n;
      for (int q2 = 0; q2 < 3; ++q2) b.dims[q2] = prob->dims[q2];
      b.mode = m;
      b.k0 = c->at<uint64_t>(c->lay.sp_k0);
      b.k1 = c->at<uint64_t>(c->lay.sp_k1);
      b.p0 = c->at<uint32_t>(c->lay.sp_p0);
      b.p1 = c->at<uint32_t>(c->lay.sp_p1);
      b.hist = c->at<uint32_t>(c->lay.sp_hist);
      b.offs = c->at<uint32_t>(c->lay.sp_offs);
      b.tot = c->at<uint32_t>(c->lay.sp_tot);
      b.rec = c->at<int4>(c->lay.sp_rec[m]);
      b.val_out = prob->x_dtype ? (void*)(c->ws + c->lay.sp_val[m]) : nullptr;
      b.S = c->lay.sp_S;
      b.nseg = c->lay.sp_nseg;
      b.tail = c->at<int32_t>(c->lay.sp_tail[m]);
      b.len = c->at<int32_t>(c->lay.sp_len[m]);
      b.heavy = c->at<int32_t>(c->lay.sp_heavy[m]);
      b.nheavy = c->at<uint32_t>(c->lay.sp_nheavy) + m;
      b.flag = &ds->flag;
      NTF_HIP(c, sp_build_mode(b, c->s0));
    }
    uint32_t nh[3] = {0, 0, 0};
    if (n > 0)
      NTF_HIP(c, hipMemcpyAsync(nh, c->at<uint32_t>(c->lay.sp_nheavy), sizeof(nh), hipMemcpyDeviceToHost, c->s0));
    NTF_HIP(c, hipMemcpyAsync(&c->host_state->flag, &ds->flag, sizeof(int), hipMemcpyDeviceToHost, c->s0));
    NTF_HIP(c, hipStreamSynchronize(c->s0));
    if (c->host_state->flag & kSparseFlagDuplicate) {
      c->err = "a coordinate is given more than once";
      return NTF_E_INVAL;
    }
    for (int m = 0; m < 3; ++m) c->nheavy[m] = (int)nh[m];
    NTF_HIP(c, launch_sumsq(prob->val, prob->x_dtype, n, c->at<double>(c->lay.sumsq), kSumsqParts,
                            &ds->xnorm2, c->s0));
    q = ctx_seed(c);
    if (q != NTF_OK) return q;
    NTF_HIP(c, hipStreamSynchronize(c->s0));
    return NTF_OK;
  }();
  if (st != NTF_OK) {
    g_init_err = c->err;
    ntf_admm_destroy(c);
    return st;
  }
  *out = c;
  return NTF_OK;
}

ntf_status ntf_admm_step(ntf_admm_ctx* c, ntf_stats* stats) {
  if (!c) return NTF_E_INVAL;
  ntf_status st = launch_outer(c);
  if (st != NTF_OK) return st;
  if (stats) return fill_stats(c, stats);
  return NTF_OK;
}

ntf_status ntf_admm_run(ntf_admm_ctx* c, int32_t max_outer, int32_t check_every, ntf_stats* stats) {
  if (!c || max_outer < 0) return NTF_E_INVAL;
  const bool test = c->opts.stop_eps_abs > 0 || c->opts.stop_eps_rel > 0;
  if (test && check_every < 1) return NTF_E_INVAL;
  ntf_stats local;
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

ntf_status ntf_admm_fit(ntf_admm_ctx* c, double* rfe) {
  if (!c || !rfe) return NTF_E_INVAL;
  const Plan& p = c->plan;
  DevState* ds = c->dstate();
  if (c->sparse) {
    // Grams of the factors (FP64), then the non-zero terms
    const int64_t d[3] = {p.I, p.J, p.K};
    double* g = c->at<double>(c->lay.fitpart);
    const int64_t FF = (int64_t)p.F * p.F;
    double* gp = g + 3 * FF;
    for (int m = 0; m < 3; ++m) {
      NTF_HIP(c, launch_gram_part(c->prob.H[m], c->hf64(), d[m], p.F, p.rpb, 0, gp, c->s0));
      NTF_HIP(c, launch_reduce_partials(gp, 1, FF, p.F, p.nblk_inner[m], p.F, p.F, g + m * FF, c->s0, 4));
    }
    double* fp = gp + (int64_t)std::max(p.nblk_inner[0], std::max(p.nblk_inner[1], p.nblk_inner[2])) * FF;
    NTF_HIP(c, sp_fit(c->at<int4>(c->lay.sp_rec[0]), c->hf64() ? (const void*)(c->ws + c->lay.sp_val[0]) : nullptr,
                      c->hf64(), c->prob.H[0], c->prob.H[1], c->prob.H[2], p.F, c->nnz, g, g + FF, g + 2 * FF,
                      &ds->xnorm2, fp, ds->fit, c->s0));
  } else {
    NTF_HIP(c, launch_fit(p, c->prob.X, c->prob.x_dtype, c->prob.H[0], c->prob.H[1], c->prob.H[2],
                          c->hf64(), c->at<double>(c->lay.fitpart), ds->fit, c->s0, nullptr));
  }
  double h[2];
  NTF_HIP(c, hipMemcpyAsync(h, ds->fit, sizeof(h), hipMemcpyDeviceToHost, c->s0));
  NTF_HIP(c, hipStreamSynchronize(c->s0));
  *rfe = h[1] > 0 ? std::sqrt(std::fmax(h[0], 0.0) / h[1]) : 0.0;
  return NTF_OK;
}

size_t ntf_admm_state_bytes(const ntf_admm_ctx* c) {
  if (!c) return 0;
  size_t b = sizeof(DevState) + sizeof(int64_t);
  if (c->opts.factor_source == 1) {
    const int64_t d[3] = {c->plan.I, c->plan.J, c->plan.K};
    for (int m = 0; m < 3; ++m) b += (size_t)(d[m] * c->plan.F) * elem_size(c->plan.prec);
  }
  return b;
}

ntf_status ntf_admm_get_state(ntf_admm_ctx* c, void* buf, size_t bytes) {
  if (!c || !buf || bytes != ntf_admm_state_bytes(c)) return NTF_E_INVAL;
  char* o = reinterpret_cast<char*>(buf);
  // The last mode's residuals are still partials; fold their totals into the
  // snapshot (fin[0..7]) so it is self-contained (the penalty rule reads them).
  const Plan& p = c->plan;
  NTF_HIP(c, finish_stats(c, c->dstate()->fin));
  NTF_HIP(c, hipStreamSynchronize(c->s0));
  NTF_HIP(c, hipMemcpy(o, c->dstate(), sizeof(DevState), hipMemcpyDeviceToHost));
  std::memcpy(o + sizeof(DevState), &c->outer, sizeof(int64_t));
  size_t off = sizeof(DevState) + sizeof(int64_t);
  if (c->opts.factor_source == 1) {
    const int64_t d[3] = {c->plan.I, c->plan.J, c->plan.K};
    for (int m = 0; m < 3; ++m) {
      const size_t nb = (size_t)(d[m] * c->plan.F) * elem_size(c->plan.prec);
      NTF_HIP(c, hipMemcpy(o + off, c->ws + c->lay.prim[m], nb, hipMemcpyDeviceToHost));
      off += nb;
    }
  }
  return NTF_OK;
}

ntf_status ntf_admm_set_state(ntf_admm_ctx* c, const void* buf, size_t bytes) {
  if (!c || !buf || bytes != ntf_admm_state_bytes(c)) return NTF_E_INVAL;
  const char* in = reinterpret_cast<const char*>(buf);
  DevState s;
  std::memcpy(&s, in, sizeof(DevState));
  std::memcpy(&c->outer, in + sizeof(DevState), sizeof(int64_t));
  for (int q = 0; q < 4; ++q) s.counter[q] = 0;
  s.flag = 0;
  *c->host_state = s;
  NTF_HIP(c, hipMemcpyAsync(c->dstate(), c->host_state, sizeof(DevState), hipMemcpyHostToDevice, c->s0));
  size_t off = sizeof(DevState) + sizeof(int64_t);
  if (c->opts.factor_source == 1) {
    const int64_t d[3] = {c->plan.I, c->plan.J, c->plan.K};
    for (int m = 0; m < 3; ++m) {
      const size_t nb = (size_t)(d[m] * c->plan.F) * elem_size(c->plan.prec);
      NTF_HIP(c, hipMemcpyAsync(c->ws + c->lay.prim[m], in + off, nb, hipMemcpyHostToDevice, c->s0));
      off += nb;
    }
  }
  ntf_status g = compute_grams(c);
  if (g != NTF_OK) return g;
  // the last mode's residual totals become its first partial (the rest are zero)
  NTF_HIP(c, hipMemcpyAsync(c->at<double>(c->lay.rpart), c->host_state->fin, 8 * sizeof(double),
                            hipMemcpyHostToDevice, c->s0));
  NTF_HIP(c, hipStreamSynchronize(c->s0));
  return NTF_OK;
}

ntf_status ntf_admm_mttkrp(ntf_admm_ctx* c, int32_t mode, double* W_out) {
  if (!c || !W_out || mode < 0 || mode > 2) return NTF_E_INVAL;
  if (c->sparse) {
    NTF_HIP(c, sparse_mttkrp(c, mode, W_out, c->s0));
    return NTF_OK;
  }
  const Plan& p = c->plan;
  const __bf16* xr = p.prec == PREC_BF16 ? c->at<__bf16>(c->lay.xr) : nullptr;
  const __bf16* xj8 = p.prec == PREC_BF16 ? c->at<__bf16>(c->lay.xj8) : nullptr;
  const float* scale = p.prec == PREC_BF16 ? c->at<float>(c->lay.scale) : nullptr;
  void* T = c->ws + c->lay.T;
  const int pf64 = c->hf64();
  if (mode == 0 || mode == 1)
    NTF_HIP(c, launch_pass1(p, c->prob.X, xr, scale, c->feed(1), c->feed(2), T, c->ws + c->lay.P1, c->s0));
  if (mode == 0)
    NTF_HIP(c, launch_reduce_partials(c->ws + c->lay.P1, pf64, p.F, (int64_t)p.nch1 * p.F, p.nch1,
                                      p.I, p.F, W_out, c->s0, 16));
  if (mode == 1) {
    NTF_HIP(c, launch_mode2(p, T, c->feed(0), c->ws + c->lay.P2, c->s0));
    NTF_HIP(c, launch_reduce_partials(c->ws + c->lay.P2, pf64, p.J * p.F, p.F, p.nich2, p.J, p.F,
                                      W_out, c->s0, 16));
  }
  if (mode == 2) {
    NTF_HIP(c, launch_pass3(p, c->prob.X, xj8, scale, c->feed(0), c->feed(1), c->ws + c->lay.P3, c->s0));
    NTF_HIP(c, launch_reduce_partials(c->ws + c->lay.P3, pf64, p.K * p.F, p.F, p.nrc3, p.K, p.F,
                                      W_out, c->s0, 16));
  }
  return NTF_OK;
}

ntf_status ntf_admm_launch_pass(ntf_admm_ctx* c, int32_t pass) {
  if (!c || pass < 0 || pass > 2) return NTF_E_INVAL;
  if (c->sparse) {
    NTF_HIP(c, sparse_mttkrp(c, pass, c->at<double>(c->lay.W[pass]), c->s0));
    return NTF_OK;
  }
  const Plan& p = c->plan;
  const __bf16* xr = p.prec == PREC_BF16 ? c->at<__bf16>(c->lay.xr) : nullptr;
  const __bf16* xj8 = p.prec == PREC_BF16 ? c->at<__bf16>(c->lay.xj8) : nullptr;
  const float* scale = p.prec == PREC_BF16 ? c->at<float>(c->lay.scale) : nullptr;
  void* T = c->ws + c->lay.T;
  if (pass == 0)
    NTF_HIP(c, launch_pass1(p, c->prob.X, xr, scale, c->feed(1), c->feed(2), T, c->ws + c->lay.P1, c->s0));
  else if (pass == 1)
    NTF_HIP(c, launch_mode2(p, T, c->feed(0), c->ws + c->lay.P2, c->s0));
  else
    NTF_HIP(c, launch_pass3(p, c->prob.X, xj8, scale, c->feed(0), c->feed(1), c->ws + c->lay.P3, c->s0));
  return NTF_OK;
}

ntf_status ntf_admm_destroy(ntf_admm_ctx* c) {
  if (!c) return NTF_E_INVAL;
  if (c->s0 || c->s1) {
    (void)hipStreamSynchronize(c->s0);
    if (c->s1) (void)hipStreamSynchronize(c->s1);
  }
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  for (int m = 0; m < 3; ++m) {
    if (c->ev_inner[m]) (void)hipEventDestroy(c->ev_inner[m]);
    if (c->ev_prep[m]) (void)hipEventDestroy(c->ev_prep[m]);
  }
  if (c->s1) (void)hipStreamDestroy(c->s1);
  if (c->sc) (void)hipStreamDestroy(c->sc);
  if (c->host_state) (void)hipHostFree(c->host_state);
  delete c;
  return NTF_OK;
}

ntf_status ntf_admm_mode_problem(ntf_admm_ctx* c, int32_t mode, double* W_out, double* G_out,
                                 double* rho_out) {
  if (!c || mode < 0 || mode > 2 || !W_out || !G_out || !rho_out) return NTF_E_INVAL;
  const Plan& p = c->plan;
  const int64_t d[3] = {p.I, p.J, p.K};
  ntf_status st = ntf_admm_mttkrp(c, mode, W_out);
  if (st != NTF_OK) return st;
  // Grams of the two other factors, in the fit-partial scratch buffer
  double* tmp = c->at<double>(c->lay.fitpart);
  double* Ga = tmp;
  double* Gb = tmp + (size_t)p.F * p.F;
  double* part = tmp + 2 * (size_t)p.F * p.F;
  const int a = (mode + 1) % 3, b = (mode + 2) % 3;
  const int gf32 = (p.prec == PREC_BF16) ? 1 : 0;
  NTF_HIP(c, launch_gram_part(c->feed(a), c->hf64(), d[a], p.F, p.rpb, gf32, part, c->s0));
  NTF_HIP(c, launch_reduce_partials(part, 1, (int64_t)p.F * p.F, p.F, p.nblk_inner[a], p.F, p.F, Ga,
                                    c->s0, 4));
  NTF_HIP(c, launch_gram_part(c->feed(b), c->hf64(), d[b], p.F, p.rpb, gf32, part, c->s0));
  NTF_HIP(c, launch_reduce_partials(part, 1, (int64_t)p.F * p.F, p.F, p.nblk_inner[b], p.F, p.F, Gb,
                                    c->s0, 4));
  NTF_HIP(c, hadamard_rho(Ga, Gb, p.F, c->opts.rho0, G_out, rho_out, c->s0));
  return NTF_OK;
}

ntf_status ntf_mlp_targets(const double* Hstar, const float* scale, int64_t rows, int32_t F,
                           float* T_out, void* stream) {
  if (!Hstar || !scale || !T_out || rows < 1 || F < 1 || F > 64) return NTF_E_INVAL;
  return mlp_targets(Hstar, scale, rows, F, T_out, (hipStream_t)stream) == hipSuccess ? NTF_OK
                                                                                       : NTF_E_HIP;
}

ntf_status ntf_admm_set_constraints(ntf_admm_ctx* c, const ntf_constraints* cons) {
  if (!c) return NTF_E_INVAL;
  ntf_constraints z{};
  const ntf_constraints& k = cons ? *cons : z;
  if (k.reserved != 0) {
    c->err = "reserved field must be zero";
    return NTF_E_INVAL;
  }
  bool any = false;
  for (int m = 0; m < 3; ++m) {
    switch (k.kind[m]) {
      case NTF_CONS_NONNEG: break;
      case NTF_CONS_BOX:
        if (!std::isfinite(k.lo[m]) || std::isnan(k.hi[m]) || !(k.lo[m] <= k.hi[m])) {
          c->err = "box constraint needs finite lo <= hi";
          return NTF_E_INVAL;
        }
        any = true;
        break;
      case NTF_CONS_PMF_ROWS: any = true; break;
      case NTF_CONS_CARDINALITY: {
        const int64_t d[3] = {c->plan.I, c->plan.J, c->plan.K};
        if (k.card[m] < 0) {
          c->err = "cardinality constraint needs card >= 0";
          return NTF_E_INVAL;
        }
        if (d[m] * c->plan.F >= ((int64_t)1 << 31)) {
          c->err = "cardinality constraint: factor has 2^31 entries or more";
          return NTF_E_UNSUPPORTED;
        }
        if (c->opts.inner_eps_abs > 0.0 || c->opts.inner_eps_rel > 0.0) {
          c->err = "cardinality constraint couples all rows: inner early stop must be off";
          return NTF_E_UNSUPPORTED;
        }
        any = true;
        break;
      }
      default:
        c->err = "unknown constraint kind";
        return NTF_E_INVAL;
    }
  }
  if (any && c->warm_on) {
    c->err = "constraints and the learned warm start do not combine";
    return NTF_E_UNSUPPORTED;
  }
  if (c->gexec || c->graph) {
    NTF_HIP(c, hipStreamSynchronize(c->s0));
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
  }
  c->cons = k;
  return NTF_OK;
}

ntf_status ntf_admm_set_warmstart(ntf_admm_ctx* c, const ntf_mlp* net) {
  if (!c) return NTF_E_INVAL;
  if (net) {
    if (net->F != c->plan.F || net->hidden < 1 || net->hidden > c->opts.warm_hidden ||
        (net->dtype != 0 && net->dtype != 1) || !net->params || net->reserved != 0) {
      c->err = "warm start network does not match the context (rank, hidden <= warm_hidden, dtype)";
      return NTF_E_INVAL;
    }
    for (int m = 0; m < 3; ++m)
      if (c->cons.kind[m] != NTF_CONS_NONNEG) {
        c->err = "constraints and the learned warm start do not combine";
        return NTF_E_UNSUPPORTED;
      }
    c->warm = *net;
    c->warm_on = true;
  } else {
    c->warm_on = false;
  }
  // the iteration graph changes: capture it again on the next step
  if (c->gexec) {
    NTF_HIP(c, hipStreamSynchronize(c->s0));
    (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
  if (c->graph) {
    (void)hipGraphDestroy(c->graph);
    c->graph = nullptr;
  }
  return NTF_OK;
}

size_t ntf_mlp_param_count(int32_t F, int32_t hidden) {
  if (F < 1 || F > 64 || hidden < 1 || hidden > 1024) return 0;
  return mlp_param_count(F, hidden);
}

static bool mlp_ok(const ntf_mlp* n) {
  return n && n->F >= 1 && n->F <= 64 && n->hidden >= 1 && n->hidden <= 1024 &&
         (n->dtype == 0 || n->dtype == 1) && n->params && n->reserved == 0;
}

ntf_status ntf_mlp_features(const double* G, const double* W, int64_t rows, int32_t F, double rho,
                            float* X_out, float* scale_out, void* stream) {
  if (!G || !W || !X_out || !scale_out || rows < 1 || F < 1 || F > 64 || !(rho > 0)) return NTF_E_INVAL;
  return mlp_features(G, W, rows, F, nullptr, rho, X_out, scale_out, (hipStream_t)stream) == hipSuccess
             ? NTF_OK : NTF_E_HIP;
}

ntf_status ntf_mlp_forward(const ntf_mlp* net, const float* X, int64_t batch, float* Y, float* act,
                           void* stream) {
  if (!mlp_ok(net) || !X || !Y || !act || batch < 1) return NTF_E_INVAL;
  return mlp_forward(net->params, net->dtype, net->F, net->hidden, X, batch, Y, act,
                     (hipStream_t)stream) == hipSuccess ? NTF_OK : NTF_E_HIP;
}

ntf_status ntf_mlp_backward(const ntf_mlp* net, const float* X, const float* act, const float* Y,
                            const float* dY, int64_t batch, float* grad, float* work, void* stream) {
  if (!mlp_ok(net) || net->dtype != 0 || !X || !act || !Y || !dY || !grad || !work || batch < 1)
    return NTF_E_INVAL;
  return mlp_backward((const float*)net->params, net->F, net->hidden, X, act, Y, dY, batch, grad,
                      work, (hipStream_t)stream) == hipSuccess ? NTF_OK : NTF_E_HIP;
}

ntf_status ntf_mlp_mse(const float* Y, const float* T, int64_t batch, int32_t F, float* dY,
                       double* loss_dev, double* part_dev, void* stream) {
  if (!Y || !T || !dY || !loss_dev || !part_dev || batch < 1 || F < 1) return NTF_E_INVAL;
  return mlp_mse(Y, T, batch, F, dY, part_dev, loss_dev, (hipStream_t)stream) == hipSuccess
             ? NTF_OK : NTF_E_HIP;
}

ntf_status ntf_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t n, float lr,
                        float beta1, float beta2, float eps, int32_t step, void* params_f16,
                        void* stream) {
  if (!params || !grad || !m || !v || n < 1 || step < 1 || !(lr > 0)) return NTF_E_INVAL;
  return mlp_adam(params, grad, m, v, n, lr, beta1, beta2, eps, step, params_f16,
                  (hipStream_t)stream) == hipSuccess ? NTF_OK : NTF_E_HIP;
}

ntf_status ntf_gather_rows(const float* src, const int64_t* idx, int64_t n, int32_t cols,
                           float* dst, void* stream) {
  if (!src || !idx || !dst || n < 1 || cols < 1) return NTF_E_INVAL;
  return gather_rows(src, idx, n, cols, dst, (hipStream_t)stream) == hipSuccess ? NTF_OK : NTF_E_HIP;
}

// ---------------------------------------------------------------- kernel-level calls

size_t ntf_gram_workspace_bytes(int64_t rows, int32_t F) {
  if (rows < 1 || F < 1 || F > 64) return 0;
  const int64_t nparts = (rows + 63) / 64;
  return align_up((size_t)nparts * F * F * 8, 256);
}

ntf_status ntf_gram(const void* H, int64_t rows, int32_t F, int32_t dtype, double* G_out,
                    void* workspace, size_t ws_bytes, void* stream) {
  if (!H || !G_out || rows < 1 || F < 1 || F > 64 || (dtype != 0 && dtype != 1) || !workspace)
    return NTF_E_INVAL;
  if (ws_bytes < ntf_gram_workspace_bytes(rows, F)) return NTF_E_WORKSPACE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t nparts = (rows + 63) / 64;
  double* part = reinterpret_cast<double*>(workspace);
  if (launch_gram_part(H, dtype, rows, F, 64, 0, part, s) != hipSuccess) return NTF_E_HIP;
  if (launch_reduce_partials(part, 1, (int64_t)F * F, F, (int)nparts, F, F, G_out, s, 4) != hipSuccess)
    return NTF_E_HIP;
  return NTF_OK;
}

namespace {
struct InnerWs {
  size_t state, ones, ginv, gpart, rpart, total;
};
InnerWs inner_ws(int64_t rows, int F) {
  int FL = 4;
  while (FL < F) FL <<= 1;
  const int rpb = inner_rows_per_block(FL);
  const int64_t nblk = (rows + rpb - 1) / rpb;
  Carver c;
  InnerWs w;
  w.state = c.take(sizeof(DevState));
  w.ones = c.take((size_t)F * F * 8);
  w.ginv = c.take((size_t)(F * F + F + 1) * 8);
  w.gpart = c.take((size_t)nblk * F * F * 8);
  w.rpart = c.take((size_t)nblk * 8 * 8);
  w.total = c.off;
  return w;
}
}  // namespace

size_t ntf_inner_workspace_bytes(int64_t rows, int32_t F) {
  if (rows < 1 || F < 1 || F > 64) return 0;
  return inner_ws(rows, F).total;
}

ntf_status ntf_inner_update(const double* W, void* H, void* U, int64_t rows, int32_t F,
                            int32_t dtype, const double* G, double rho, int32_t T, double eps_abs,
                            double eps_rel, int32_t* iters_out, void* Ht_out, void* workspace,
                            size_t ws_bytes, void* stream) {
  if (!W || !H || !U || !G || rows < 1 || F < 1 || F > 64 || (dtype != 0 && dtype != 1) || T < 1 ||
      !workspace || eps_abs < 0 || eps_rel < 0)
    return NTF_E_INVAL;
  const InnerWs w = inner_ws(rows, F);
  if (ws_bytes < w.total) return NTF_E_WORKSPACE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* base = reinterpret_cast<char*>(workspace);
  DevState* ds = reinterpret_cast<DevState*>(base + w.state);
  // zeroed state (rho/prev = given rho or 0 for trace), ones for the Hadamard partner
  if (launch_fill(reinterpret_cast<double*>(ds), sizeof(DevState) / 8, 0.0, s) != hipSuccess) return NTF_E_HIP;
  if (launch_fill(reinterpret_cast<double*>(base + w.ones), (int64_t)F * F, 1.0, s) != hipSuccess) return NTF_E_HIP;
  PrepArgs pa;
  pa.F = F;
  pa.gram_a = G;
  pa.gram_b = reinterpret_cast<double*>(base + w.ones);
  pa.policy = rho > 0 ? 1 : 0;
  pa.rho0 = rho > 0 ? rho : 1.0;
  pa.rho_state = ds->rho[0];
  pa.Ginv = reinterpret_cast<double*>(base + w.ginv);
  pa.flag = &ds->flag;
  pa.counter = &ds->counter[0];
  if (launch_prep(pa, 1, s) != hipSuccess) return NTF_E_HIP;
  int FL = 4;
  while (FL < F) FL <<= 1;
  InnerArgs ia;
  ia.part = W;
  ia.part_f64 = 1;
  ia.pstride = 0;
  ia.rowstride = F;
  ia.nparts = 1;
  ia.H = H;
  ia.U = U;
  ia.Pout = Ht_out;
  ia.h_f64 = dtype;
  ia.rows = rows;
  ia.F = F;
  ia.FL = FL;
  ia.Ginv = pa.Ginv;
  ia.rho = ds->rho[0];
  ia.T = T;
  ia.eps_abs = eps_abs;
  ia.eps_rel = eps_rel;
  ia.iters_out = iters_out;
  // (the Gram and residual partials are not outputs of this call: no fused
  // Gram partial, so both this call and ntf_inner_update_noalloc take the
  // same kernel)
  ia.gram_part = nullptr;
  ia.resid_part = reinterpret_cast<double*>(base + w.rpart);
  ia.flag = &ds->flag;
  const int rpb = inner_rows_per_block(FL);
  if (launch_inner(ia, (int)((rows + rpb - 1) / rpb), s) != hipSuccess) return NTF_E_HIP;
  return NTF_OK;
}

}  // extern "C"

// ------------------------------------------------- mode update without allocation
//
// ntf_inner_update_noalloc runs the kernels of ntf_inner_update with their
// scratch (device state, the all-ones Hadamard partner, the factored system)
// in the file-scope array below instead of a caller workspace.  The Gram and
// residual partials that ntf_inner_update also leaves in its workspace are
// outputs nobody reads there, so this variant skips them; H, U, the
// iteration counts and Ht are bitwise the same.  Host code never passes
// `scratch` itself to a kernel: its device address comes from
// hipGetSymbolAddress, taken once per device with that device current.

namespace {
constexpr size_t kStaticScratchBytes = 128 * 1024;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

struct StaticInnerLayout {
  size_t state, ones, ginv, total;
};
StaticInnerLayout static_inner_layout(int F) {
  Carver c;
  StaticInnerLayout l;
  l.state = c.take(sizeof(DevState));
  l.ones = c.take((size_t)F * F * 8);
  l.ginv = c.take((size_t)(F * F + F + 1) * 8);
  l.total = c.off;
  return l;
}

// Device address of this device's copy of `scratch` (looked up once per device).
hipError_t static_scratch(char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = reinterpret_cast<char*>(g_scratch_ptr[dev]);
  return hipSuccess;
}
}  // namespace

extern "C" {

size_t ntf_inner_static_scratch_bytes(int32_t F) {
  if (F < 1 || F > 64) return 0;
  return static_inner_layout(F).total;
}

ntf_status ntf_inner_update_noalloc(const double* W, void* H, void* U, int64_t rows, int32_t F,
                                    int32_t dtype, const double* G, double rho, int32_t T,
                                    double eps_abs, double eps_rel, int32_t* iters_out,
                                    void* Ht_out, void* stream) {
  if (!W || !H || !U || !G || rows < 1 || F < 1 || F > 64 || (dtype != 0 && dtype != 1) || T < 1 ||
      eps_abs < 0 || eps_rel < 0)
    return NTF_E_INVAL;
  const StaticInnerLayout l = static_inner_layout(F);
  if (l.total > kStaticScratchBytes) return NTF_E_WORKSPACE;
  char* base = nullptr;
  if (static_scratch(&base) != hipSuccess) return NTF_E_HIP;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  DevState* ds = reinterpret_cast<DevState*>(base + l.state);
  // the array keeps the previous call's contents: state restarts at zero
  if (launch_fill(reinterpret_cast<double*>(ds), sizeof(DevState) / 8, 0.0, s) != hipSuccess) return NTF_E_HIP;
  if (launch_fill(reinterpret_cast<double*>(base + l.ones), (int64_t)F * F, 1.0, s) != hipSuccess)
    return NTF_E_HIP;
  PrepArgs pa;
  pa.F = F;
  pa.gram_a = G;
  pa.gram_b = reinterpret_cast<double*>(base + l.ones);
  pa.policy = rho > 0 ? 1 : 0;
  pa.rho0 = rho > 0 ? rho : 1.0;
  pa.rho_state = ds->rho[0];
  pa.Ginv = reinterpret_cast<double*>(base + l.ginv);
  pa.flag = &ds->flag;
  pa.counter = &ds->counter[0];
  if (launch_prep(pa, 1, s) != hipSuccess) return NTF_E_HIP;
  int FL = 4;
  while (FL < F) FL <<= 1;
  InnerArgs ia;
  ia.part = W;
  ia.part_f64 = 1;
  ia.pstride = 0;
  ia.rowstride = F;
  ia.nparts = 1;
  ia.H = H;
  ia.U = U;
  ia.Pout = Ht_out;
  ia.h_f64 = dtype;
  ia.rows = rows;
  ia.F = F;
  ia.FL = FL;
  ia.Ginv = pa.Ginv;
  ia.rho = ds->rho[0];
  ia.T = T;
  ia.eps_abs = eps_abs;
  ia.eps_rel = eps_rel;
  ia.iters_out = iters_out;
  ia.gram_part = nullptr;
  ia.resid_part = nullptr;
  ia.flag = &ds->flag;
  const int rpb = inner_rows_per_block(FL);
  if (launch_inner(ia, (int)((rows + rpb - 1) / rpb), s) != hipSuccess) return NTF_E_HIP;
  return NTF_OK;
}

}  // extern "C"
