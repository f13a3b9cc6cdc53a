/*
 * ntf_admm.h -- C ABI of the gfx950 (MI355X) ADMoM non-negative CP
 * factorisation library, libntf_admm.so.
 *
 * Method: Liavas & Sidiropoulos, "Parallel algorithms for constrained tensor
 * factorization via the alternating direction method of multipliers".
 * The problem is eq. Problem_NTF (Section II): given a dense 3-way tensor X
 * and a rank F, find A, B, C >= 0 minimising 1/2 ||X - [A,B,C]||_F^2.  One
 * outer iteration is one ADMoM iteration (eq. ADMoM_NTF): the three factors
 * are updated in Gauss-Seidel order A, B, C (eq. ADMM_NTF_ALS_C), each by
 *
 *   W   = X^(n) (Khatri-Rao of the other two factors)            (MTTKRP)
 *   G   = Hadamard product of the other factors' Grams          (Section IV-A)
 *   Ginv = (G + rho I)^{-1}  (block Gauss-Jordan, FP64, once per mode update)
 *   T times:  Ht^T = (W + rho (H + U)) (G + rho I)^{-1}
 *             H    = max(0, Ht^T - U),   U += H - Ht^T            (eq. ADMoM_NTF)
 *
 * with H the non-negative auxiliary factor (the paper's A-tilde) and U the
 * scaled dual, U = -Y / rho.  The paper runs T = 1 (footnote to eq.
 * ADMM_NTF_ALS_C); T is a parameter here.
 *
 * Conventions for every entry point:
 *  - All array arguments are DEVICE pointers unless stated otherwise; the
 *    caller allocates and owns them.  The library allocates no device memory:
 *    every temporary lives in a caller-provided workspace whose size the
 *    matching *_workspace_bytes function returns.
 *  - Tensors are dense, C order [I][J][K] (k fastest).  Factor matrices are
 *    row-major [d_n][F].
 *  - `stream` is a hipStream_t (NULL = the default stream); all device work is
 *    enqueued on it in order.  Functions documented as synchronising wait for
 *    the stream before returning.
 *  - Errors are returned as ntf_status codes; nothing is printed and nothing
 *    aborts.  On error nothing has been enqueued unless stated otherwise.
 *  - Device pointers must be 16-byte aligned.
 */
#ifndef NTF_ADMM_H
#define NTF_ADMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NTF_OK = 0,
  NTF_NOT_CONVERGED = 1,   /* informational: run() hit its cap before the stop test held */
  NTF_E_INVAL = -1,        /* bad sizes, null/misaligned pointers, inconsistent options */
  NTF_E_WORKSPACE = -2,    /* workspace smaller than *_workspace_bytes */
  NTF_E_HIP = -3,          /* a HIP runtime call failed; see ntf_admm_last_error */
  NTF_E_NUMERIC = -4,      /* G + rho I not positive definite, or NaN/Inf met on device */
  NTF_E_UNSUPPORTED = -5   /* valid request outside what this library implements */
} ntf_status;

typedef enum {
  NTF_PREC_F32 = 0,         /* X float32; MTTKRP on FP32 MFMA; Gram, (G + rho I)^{-1}, solves FP64; H,U float32 */
  NTF_PREC_BF16_MIXED = 1,  /* X float32 + bfloat16 copy with a power-of-two scale per mode-1 slab;
                               MTTKRP on BF16 MFMA with FP32 accumulation against
                               bfloat16(H_3) (modes 1, 2) or H_2 as two bfloat16 terms
                               hi + lo (mode 3, each slab's result scaled by the slab's
                               row of H_1 in FP32);
                               Gram, (G + rho I)^{-1} and solves FP64; H,U float32 */
  NTF_PREC_F64 = 3          /* X float64; everything FP64 (MFMA f64); H,U float64 */
} ntf_precision;

typedef enum {
  NTF_RHO_TRACE = 0,        /* rho_n = trace(G_n)/F at every update of mode n */
  NTF_RHO_FIXED = 1,        /* rho_n = rho0 */
  NTF_RHO_ADAPTIVE = 2      /* residual balancing, Section IV-D (eq. varying_penalty_rule),
                               applied after every outer iteration, starting from rho0 */
} ntf_rho_policy;

/* The problem, as Section II states it. */
typedef struct {
  int64_t dims[3];          /* I, J, K >= 1 */
  int32_t F;                /* rank, 1..64 */
  int32_t x_dtype;          /* 0 = float32 (F32, BF16_MIXED), 1 = float64 (F64) */
  const void *X;            /* device, [I][J][K]; BORROWED read-only, must outlive the context */
  void *H[3];               /* device in/out, [d_n][F]: initial factors in, factors out.
                               float32, or float64 for NTF_PREC_F64 */
  void *U[3];               /* device in/out, [d_n][F], same dtype: scaled duals (zero = cold start) */
} ntf_problem;

typedef struct {
  int32_t inner_iters;      /* T >= 1: inner ADMoM iterations per mode update (row-wise cap) */
  int32_t rho_policy;       /* ntf_rho_policy */
  double rho0;              /* initial / fixed penalty, > 0 (Section VI-A uses 1) */
  double mu, tau_incr, tau_decr;   /* residual balancing (Section VI-A: 8, 4, 2) */
  double inner_eps_abs, inner_eps_rel; /* row-wise inner early stop: the Section IV-C test
                               written for one row (sqrt(F) in place of sqrt(I F));
                               both 0 = always run T iterations */
  double stop_eps_abs, stop_eps_rel;   /* outer stop test of Section IV-C on every mode,
                               used by ntf_admm_run; both 0 = no outer test */
  int32_t precision;        /* ntf_precision */
  int32_t factor_source;    /* 0: later modes use the projected H (default);
                               1: they use the unconstrained primal Ht^T, as the paper does */
  int32_t rescale_dual_on_rho_change; /* 1: U *= rho_old/rho_new when rho changes (keeps the
                               unscaled dual Y fixed); forced on for NTF_RHO_ADAPTIVE */
  int32_t paper_init;       /* 1: auxiliary and dual variables start at zero and the given
                               factors seed the primal (Section VI-A); needs factor_source 1 */
  int32_t warm_hidden;      /* > 0: reserve workspace for a learned warm start with this many
                               hidden units (see ntf_admm_set_warmstart); 0 = none */
  int32_t reserved[3];      /* must be zero */
} ntf_opts;

/* Statistics of the most recent outer iteration (Section IV-C quantities). */
typedef struct {
  int64_t outer;            /* outer iterations completed since init */
  double rho[3];            /* penalty used by the last update of each mode */
  double prim[3];           /* ||H_n - Ht_n^T||_F after the last inner iteration */
  double dual[3];           /* rho_n ||H_n^new - H_n^old||_F over the whole mode update */
  double norm_h[3];         /* ||H_n||_F */
  double norm_p[3];         /* ||Ht_n^T||_F */
  double norm_y[3];         /* rho_n ||U_n||_F = ||Y_n||_F */
  double inner_iters_mean[3]; /* mean inner iterations per row in the last update */
  double rfe_cheap;         /* RFE from ||X||^2 - 2<W_3,H_3> + sum(G1*G2*G3); monitoring only */
  int64_t warm_taken[3];    /* rows whose inner sweep started from the network's prediction */
  int32_t numeric_error;    /* non-zero if a non-PD system or NaN/Inf was met */
  int32_t converged;        /* Section IV-C stop test held for all modes (needs stop_eps_* > 0) */
} ntf_stats;

typedef struct ntf_admm_ctx ntf_admm_ctx;

/* ------------------------------------------------------------------ solver */

/* Workspace bytes ntf_admm_init needs for this problem and options; 0 if the
 * arguments are invalid.  Host-only, no device work. */
size_t ntf_admm_workspace_bytes(const ntf_problem *prob, const ntf_opts *opts);

/* Validate, carve the workspace, build the bfloat16 copy of X if the
 * precision asks for it (Section II data, stored as two bf16 layouts), compute
 * ||X||^2 and the initial Grams, and factor G_1 + rho I.  The context keeps
 * the pointers in `prob`; `workspace` (device, >= ntf_admm_workspace_bytes)
 * is borrowed for the life of the context.  Synchronises the stream. */
ntf_status ntf_admm_init(ntf_admm_ctx **out, const ntf_problem *prob, const ntf_opts *opts,
                         void *workspace, size_t ws_bytes, void *stream);

/* ------------------------------------------------------ order-N tensors */

#define NTF_MAX_ORDER 8

/* A dense tensor of order N = 3 .. NTF_MAX_ORDER (Appendix A: the mode-n
 * unfolding is A_n times the transposed Khatri-Rao product of the other N - 1
 * factors, and the method carries over with N - 1 Grams in the Hadamard
 * product). */
typedef struct {
  int32_t order;                   /* N */
  int32_t F;                       /* rank, 1..64 */
  int64_t dims[NTF_MAX_ORDER];     /* I_1 .. I_N >= 1 (entries past N ignored); prod <= 2^46 */
  int32_t x_dtype;                 /* 0 = float32 (NTF_PREC_F32), 1 = float64 (NTF_PREC_F64) */
  int32_t reserved;                /* must be zero */
  const void *X;                   /* device, C order [I_1]..[I_N]; BORROWED read-only */
  void *H[NTF_MAX_ORDER];          /* device in/out [I_n][F] factors, as in ntf_problem */
  void *U[NTF_MAX_ORDER];          /* device in/out [I_n][F] scaled duals */
} ntf_nway_problem;

typedef struct {                   /* as ntf_stats, per mode of the N */
  int64_t outer;
  double rho[NTF_MAX_ORDER];
  double prim[NTF_MAX_ORDER];
  double dual[NTF_MAX_ORDER];
  double norm_h[NTF_MAX_ORDER];
  double norm_p[NTF_MAX_ORDER];
  double norm_y[NTF_MAX_ORDER];
  double inner_iters_mean[NTF_MAX_ORDER];
  int32_t numeric_error;
  int32_t converged;
} ntf_nway_stats;

typedef struct ntf_nway_ctx ntf_nway_ctx;

/* Workspace bytes for ntf_nway_init; 0 if the arguments are invalid. */
size_t ntf_nway_workspace_bytes(const ntf_nway_problem *prob, const ntf_opts *opts);

/* Solver context for an order-N tensor.  One outer iteration updates the N
 * factors in order 1..N (Gauss-Seidel, as eq. ADMM_NTF_ALS_C for three).  The
 * mode-n MTTKRP runs on a three-way view of X with the modes before n and
 * after n folded (their factor the Khatri-Rao product of the folded factors,
 * formed per iteration); the prepare step takes the Hadamard product of the
 * N - 1 other Grams; the inner sweep is the three-way one.  Options as in
 * ntf_opts: precision NTF_PREC_F32 or NTF_PREC_F64 (NTF_PREC_BF16_MIXED and
 * warm_hidden > 0 are NTF_E_UNSUPPORTED); factor_source, paper_init, the
 * penalty policies, the inner and outer stop tests apply as for three modes.
 * With N = 3 the iterates are those of ntf_admm_init up to rounding order.
 * Synchronises the stream. */
ntf_status ntf_nway_init(ntf_nway_ctx **out, const ntf_nway_problem *prob, const ntf_opts *opts,
                         void *workspace, size_t ws_bytes, void *stream);
ntf_status ntf_nway_step(ntf_nway_ctx *ctx, ntf_nway_stats *stats);          /* as ntf_admm_step */
ntf_status ntf_nway_run(ntf_nway_ctx *ctx, int32_t max_outer, int32_t check_every,
                        ntf_nway_stats *stats);                              /* as ntf_admm_run */
/* Direct RFE ||X - [H_1, .., H_N]|| / ||X|| in FP64 over every entry;
 * synchronises. */
ntf_status ntf_nway_fit(ntf_nway_ctx *ctx, double *rfe);
/* W_out (device, FP64 [I_mode][F]) = X^(mode) times the Khatri-Rao product of
 * the other factors as the next update would see them; enqueued only. */
ntf_status ntf_nway_mttkrp(ntf_nway_ctx *ctx, int32_t mode, double *W_out);
const char *ntf_nway_last_error(const ntf_nway_ctx *ctx);   /* NULL ctx: last failed init */
ntf_status ntf_nway_destroy(ntf_nway_ctx *ctx);

/* ------------------------------------------------------- sparse tensors */

/* A sparse 3-way tensor given by its non-zeros (Section IV-A, item 1: n
 * non-zeros, n << IJK; every other entry is zero). */
typedef struct {
  int64_t dims[3];          /* I, J, K >= 1; the packed sort key needs
                               ceil(log2 I) + ceil(log2 J) + ceil(log2 K) <= 64 */
  int32_t F;                /* rank, 1..64 */
  int32_t x_dtype;          /* 0 = float32 values (NTF_PREC_F32), 1 = float64 (NTF_PREC_F64) */
  int64_t nnz;              /* number of non-zeros, 0 .. 2^31 - 1 */
  const int32_t *idx;       /* device [nnz][3] coordinates (i, j, k), all distinct, any order;
                               read during ntf_admm_init_sparse only */
  const void *val;          /* device [nnz] values; read during ntf_admm_init_sparse only */
  void *H[3];               /* as in ntf_problem */
  void *U[3];
} ntf_sparse_problem;

/* Workspace bytes ntf_admm_init_sparse needs: three sorted copies of the
 * non-zeros ((12 + value bytes) per non-zero each), the sort scratch of the
 * set-up (24 bytes per non-zero), the MTTKRP segment carries and the
 * per-mode buffers of the dense solver; 0 if the arguments are invalid. */
size_t ntf_admm_sparse_workspace_bytes(const ntf_sparse_problem *prob, const ntf_opts *opts);

/* Create a solver context for a sparse tensor.  Set-up builds, per mode, a
 * copy of the non-zeros sorted by (that mode's index, then the other two in
 * mode order) with the library's radix sort; the caller's coordinate and value
 * arrays are not used afterwards.  Every MTTKRP of the outer iteration then
 * takes 3 nnz F flops from the sorted copy (one product of the other two
 * factor rows per non-zero, Section IV-A, item 1); the Gram, penalty,
 * factorisation and inner sweep are those of the dense tensor.  All other
 * ntf_admm_* calls apply unchanged; ntf_admm_fit evaluates
 * ||X - M||^2 = sum over non-zeros (x - m)^2 + ||M||^2 - sum over non-zeros m^2,
 * ||M||^2 from the Grams of the factors, in FP64; ntf_admm_launch_pass(p)
 * runs the MTTKRP of mode p.  Precision NTF_PREC_F32 (FP32 products and
 * segment sums, FP64 across segments) or NTF_PREC_F64; NTF_PREC_BF16_MIXED
 * and a learned warm start (warm_hidden > 0) are NTF_E_UNSUPPORTED.  Errors:
 * a coordinate outside the tensor or repeated is NTF_E_INVAL (found on the
 * device during set-up; nothing is built from an out-of-range coordinate).
 * Synchronises the stream. */
ntf_status ntf_admm_init_sparse(ntf_admm_ctx **out, const ntf_sparse_problem *prob,
                                const ntf_opts *opts, void *workspace, size_t ws_bytes,
                                void *stream);

/* One outer iteration (modes 1, 2, 3 in Gauss-Seidel order, eqs. ADMoM_NTF and
 * ADMM_NTF_ALS_C).  The first call captures the iteration into a HIP graph;
 * later calls replay it.  If `stats` is non-NULL the call synchronises and
 * fills it; otherwise it only enqueues. */
ntf_status ntf_admm_step(ntf_admm_ctx *ctx, ntf_stats *stats);

/* Up to `max_outer` outer iterations.  With opts.stop_eps_abs or stop_eps_rel > 0 the
 * run stops early once the Section IV-C test holds on every mode (checked
 * every `check_every` iterations, >= 1; each check synchronises) and returns
 * NTF_OK, else NTF_NOT_CONVERGED.  With both eps zero it enqueues all
 * iterations and returns NTF_OK.  `stats` as in ntf_admm_step. */
ntf_status ntf_admm_run(ntf_admm_ctx *ctx, int32_t max_outer, int32_t check_every, ntf_stats *stats);

/* Direct relative fit error ||X - [H1,H2,H3]||_F / ||X||_F (Section VI-A),
 * the model formed and the error accumulated in FP64 over the original X.
 * Synchronises; result to host *rfe. */
ntf_status ntf_admm_fit(ntf_admm_ctx *ctx, double *rfe);

/* Checkpoint support.  The complete solver state (eq. ADMoM_NTF's Z plus the
 * penalties, Section IV-C/D) is H and U, which live in the caller's buffers,
 * and a context-internal part: per-mode penalties and residual totals, the
 * outer count and, with factor_source 1, the primal factors.
 * ntf_admm_state_bytes gives the size of that internal part; get_state
 * synchronises and copies it to host memory `buf`; set_state loads it into a
 * context created for the same problem and options and recomputes the Grams
 * from the current H buffers exactly as the solver forms them, so that
 * run(a+b) and run(a); get_state; set_state; run(b) give bitwise identical
 * results.  Both return NTF_E_INVAL if `bytes` is not the state size. */
size_t ntf_admm_state_bytes(const ntf_admm_ctx *ctx);
ntf_status ntf_admm_get_state(ntf_admm_ctx *ctx, void *buf, size_t bytes);
ntf_status ntf_admm_set_state(ntf_admm_ctx *ctx, const void *buf, size_t bytes);

/* W_n (the MTTKRP of mode n, 0-based) with the context's precision and
 * kernels, from the current factors, into `W_out` (device, float64 [d_n][F]).
 * Stream-ordered, does not change the solver state. */
ntf_status ntf_admm_mttkrp(ntf_admm_ctx *ctx, int32_t mode, double *W_out);

/* Measurement hook: enqueue exactly one MTTKRP kernel with the current
 * factors and nothing else -- pass 0: mode-1 partials plus the k-contracted
 * intermediate T = X x_3 C (streams X); pass 1: mode-2 partials from T;
 * pass 2: mode-3 partials (streams X).  Stream-ordered; writes only scratch
 * (T and the partials), never the solver state. */
ntf_status ntf_admm_launch_pass(ntf_admm_ctx *ctx, int32_t pass);

ntf_status ntf_admm_destroy(ntf_admm_ctx *ctx);
const char *ntf_admm_last_error(const ntf_admm_ctx *ctx);
const char *ntf_status_str(ntf_status s);

/* ------------------------------------------- learned warm start (not in the paper)
 *
 * A 3-layer MLP (ReLU after the two hidden layers, linear output) maps one row's NNLS problem
 * min_{h>=0} 1/2 h^T G h - w^T h (the fixed point of the inner sweep for that
 * row, Section IV) to a starting point.  Row inputs (D = F(F+1)/2 + F floats):
 * the upper triangle of G/rho, row by row, then w/||w||; the network predicts
 * h rho/||w||.  Parameters are one flat vector
 *   [W1 hidden*D, b1 hidden, W2 hidden*hidden, b2 hidden, W3 F*hidden, b3 F]
 * with a = relu(W x + b) for the hidden layers and y = W3 a2 + b3 (weights
 * row-major [out][in]); the judge projects y onto h >= 0. */
typedef struct {
  int32_t F;                /* rank the network serves, 1..64 */
  int32_t hidden;           /* hidden units per layer, 1..1024 */
  int32_t dtype;            /* 0 = float32 parameters, 1 = float16 */
  int32_t reserved;         /* must be zero */
  const void *params;       /* device, flat parameter vector (borrowed) */
} ntf_mlp;

/* Number of parameters of the network for rank F and `hidden` units. */
size_t ntf_mlp_param_count(int32_t F, int32_t hidden);

/* Row inputs X_out [rows][D] (float32) and output scales scale_out [rows]
 * (||w_i||/rho) from G [F][F] and W [rows][F] (float64, device). */
ntf_status ntf_mlp_features(const double *G, const double *W, int64_t rows, int32_t F, double rho,
                            float *X_out, float *scale_out, void *stream);

/* Forward pass on `batch` rows: Y [batch][F]; `act` [2][batch][hidden]
 * float32 receives the two hidden activations (needed by the backward pass). */
ntf_status ntf_mlp_forward(const ntf_mlp *net, const float *X, int64_t batch, float *Y, float *act,
                           void *stream);

/* Gradient of sum(dY * Y) with respect to the parameters of a float32
 * network, into grad (flat, overwritten).  `work` holds (2*hidden + F)*batch
 * floats of scratch.  FP32 throughout; every sum has a fixed order. */
ntf_status ntf_mlp_backward(const ntf_mlp *net, const float *X, const float *act, const float *Y,
                            const float *dY, int64_t batch, float *grad, float *work, void *stream);

/* dY = (Y - T)/batch and the loss 1/(2 batch) sum (Y - T)^2 into loss_dev[0]
 * (device double); part_dev holds 64 doubles of scratch. */
ntf_status ntf_mlp_mse(const float *Y, const float *T, int64_t batch, int32_t F, float *dY,
                       double *loss_dev, double *part_dev, void *stream);

/* One Adam step (bias-corrected, `step` >= 1) on n parameters; if params_f16
 * is non-NULL it receives the updated parameters as float16. */
ntf_status ntf_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t n, float lr,
                        float beta1, float beta2, float eps, int32_t step, void *params_f16,
                        void *stream);

/* dst[r][:] = src[idx[r]][:] for r < n (minibatch gather; idx device int64). */
ntf_status ntf_gather_rows(const float *src, const int64_t *idx, int64_t n, int32_t cols,
                           float *dst, void *stream);

/* Training targets T_out [rows][F] = h* / scale for converged rows h*
 * (float64) and the scales of ntf_mlp_features. */
ntf_status ntf_mlp_targets(const double *Hstar, const float *scale, int64_t rows, int32_t F,
                           float *T_out, void *stream);

/* The NNLS problems mode `mode` would solve from the current factors: W_out
 * [d_n][F] (its MTTKRP), G_out [F][F] (the Gram Hadamard product) and
 * rho_out[0] = trace(G)/F, all float64 device buffers.  Stream-ordered; does
 * not change the solver state.  Used to generate warm-start training pairs. */
ntf_status ntf_admm_mode_problem(ntf_admm_ctx *ctx, int32_t mode, double *W_out, double *G_out,
                                 double *rho_out);

/* Use `net` (rank ctx's F, hidden <= opts.warm_hidden) to warm-start every
 * mode update: after G and W are formed, each row starts from the network's
 * candidate if its NNLS KKT violation ||min(h, hG - w)|| is smaller than the
 * previous iterate's, otherwise from the previous iterate (the fallback).
 * NULL disables.  The next step re-captures the iteration graph. */
ntf_status ntf_admm_set_warmstart(ntf_admm_ctx *ctx, const ntf_mlp *net);

/* ------------------------------------------------------ kernel-level calls */

/* One mode update on its own (Section IV, one line of eq. ADMM_NTF_ALS_C with
 * the projection and dual update): given W [rows][F] (float64) and G [F][F]
 * (float64, symmetric PSD), factor G + rho I in FP64 on the device, then run
 * up to T inner iterations per row on H, U (in/out, [rows][F], dtype 0 =
 * float32, 1 = float64).  rho <= 0 selects trace(G)/F.  Row-wise early stop
 * as in ntf_opts.eps_*.  `iters_out` (device int32 [rows], may be NULL)
 * receives the iterations each row ran; `Ht_out` (device, same dtype as H,
 * may be NULL) the last Ht^T.  Stream-ordered. */
size_t ntf_inner_workspace_bytes(int64_t rows, int32_t F);
ntf_status ntf_inner_update(const double *W, void *H, void *U, int64_t rows, int32_t F, int32_t dtype,
                            const double *G, double rho, int32_t T, double eps_abs, double eps_rel,
                            int32_t *iters_out, void *Ht_out, void *workspace, size_t ws_bytes,
                            void *stream);

/* ntf_inner_update for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments and results (H, U, iters_out, Ht_out bitwise those of
 * ntf_inner_update) but no workspace.  Its scratch (device state, the system
 * G + rho I in factored form) lives in a fixed 128 KiB array in the library's
 * device memory, one copy per GPU, held until the process ends; a call needs
 * ntf_inner_static_scratch_bytes(F) of it (at most ~67 KB, for F = 64) and
 * returns NTF_E_WORKSPACE if that exceeded the array.  The call allocates
 * nothing and issues no memset (fill kernels only).  Every call on one GPU
 * shares that array: calls that overlap on one GPU (different streams, or
 * host threads without ordering) race and give undefined results; calls
 * ordered on one stream are safe.  Errors: NTF_E_INVAL as ntf_inner_update,
 * NTF_E_HIP if the array's address cannot be obtained or a launch fails. */
size_t ntf_inner_static_scratch_bytes(int32_t F);
ntf_status ntf_inner_update_noalloc(const double *W, void *H, void *U, int64_t rows, int32_t F,
                                    int32_t dtype, const double *G, double rho, int32_t T,
                                    double eps_abs, double eps_rel, int32_t *iters_out,
                                    void *Ht_out, void *stream);

/* Gram matrix H^T H of a [rows][F] factor (dtype 0 = float32, 1 = float64),
 * accumulated in FP64, into G_out (device float64 [F][F]).  Stream-ordered. */
size_t ntf_gram_workspace_bytes(int64_t rows, int32_t F);
ntf_status ntf_gram(const void *H, int64_t rows, int32_t F, int32_t dtype, double *G_out,
                    void *workspace, size_t ws_bytes, void *stream);

/* ---------------------------------------------------- structural constraints */

/* Set constraint of each factor (Section IV-E: a set constraint changes only
 * the projection of the auxiliary factor; Section VI-D: rows that are
 * probability mass functions change the least-squares step instead). */
typedef enum {
  NTF_CONS_NONNEG = 0,      /* H >= 0 (the default, eq. g_M_def) */
  NTF_CONS_BOX = 1,         /* lo <= H <= hi elementwise: the auxiliary update projects onto the box */
  NTF_CONS_PMF_ROWS = 2,    /* every row non-negative and summing to one: the least-squares step of
                               each row is solved with the constraint 1^T h = 1 (closed form from
                               (G + rho I)^{-1}), the auxiliary update stays the non-negative one */
  NTF_CONS_CARDINALITY = 3  /* H >= 0 with at most card non-zeros in the whole factor (eq.
                               g_new_def): the auxiliary update keeps the card largest positive
                               entries of Ht^T - U (ties by row-major index).  The projection
                               couples every row, so each inner iteration is a row-wise solve
                               plus one whole-factor select pass; needs inner early stop off
                               (inner_eps_abs = inner_eps_rel = 0) and rows * F < 2^31, else
                               NTF_E_UNSUPPORTED; card < 0 is NTF_E_INVAL */
} ntf_constraint_kind;

typedef struct {
  int32_t kind[3];          /* ntf_constraint_kind per mode */
  int32_t reserved;         /* must be zero */
  double lo[3], hi[3];      /* NTF_CONS_BOX: finite lo <= hi (hi may be +inf); otherwise ignored */
  int64_t card[3];          /* NTF_CONS_CARDINALITY: maximum number of non-zeros of the factor */
} ntf_constraints;

/* Constrain the factors from the next outer iteration on (NULL = all
 * non-negative).  Not combinable with a learned warm start.  The next step
 * re-captures the iteration graph (an existing one is dropped after the
 * stream is synchronised). */
ntf_status ntf_admm_set_constraints(ntf_admm_ctx *ctx, const ntf_constraints *cons);

/* ------------------------------------------------------------- batched */

/* Many independent problems of uneven shapes factorised together: one
 * persistent kernel per outer iteration runs every problem's three mode
 * updates (eq. ADMoM_NTF, Gauss-Seidel order of eq. ADMM_NTF_ALS_C) from one
 * global work list, and each outer iteration is one replay of a captured HIP
 * graph.  Every problem is the single-problem method of Section IV with its
 * own F, G, rho and (G + rho I)^{-1}; problems share nothing but the launch.
 *
 * Precision is NTF_PREC_BF16_MIXED only: at init the library writes two
 * bfloat16 copies of each X with a power-of-two scale per mode-1 slab
 * ([I][J][Kp], k fastest, and [I][K][Jp], j fastest; Kp, Jp = K, J rounded
 * up to 32), then the MTTKRPs run on BF16 MFMA with FP32 accumulation (as
 * in the single-problem solver, the mode-3 product takes H_2 as two bfloat16
 * terms and scales each slab's result by the row of H_1), Grams in FP32 per
 * row block summed in FP64, and
 * (G + rho I)^{-1} and solves in FP64.  Options used: inner_iters, rho_policy
 * (TRACE or FIXED), rho0, inner_eps_abs/rel, rescale_dual_on_rho_change;
 * factor_source, paper_init, warm_hidden and the outer stop test must be 0.
 * Every problem: x_dtype 0, float32 H and U, F in 1..64, and its work items
 * must fit the LDS (contraction lengths up to about 1000 at F = 64, larger at
 * smaller F); otherwise init returns NTF_E_UNSUPPORTED. */
typedef struct ntf_batch_ctx ntf_batch_ctx;

/* Tile choice of one bucket of MTTKRP work items, as the autotuner reports
 * and accepts it. */
typedef struct {
  int32_t kind;            /* 1 = the pass for modes 1 and 2 (contraction over k),
                              3 = the pass for mode 3 (contraction over j) */
  int32_t ft;              /* ceil(F / 16): 16-column MFMA tiles of the rank */
  int32_t qbucket;         /* contraction length: 0 <= 128, 1 <= 256, 2 <= 512, 3 larger */
  int32_t mt;              /* 16-row MFMA tiles per wave step, 1 or 2 */
  int64_t item_elems;      /* target tensor elements per work item (whole slabs, >= 1 slab) */
  double us;               /* autotuner: measured microseconds of the bucket's items, else 0 */
} ntf_batch_tile;

typedef struct {
  int32_t n_problems;
  int32_t grid;            /* persistent blocks (resident blocks per CU x CUs) */
  int32_t lds_bytes;       /* dynamic LDS per block */
  int32_t n_items;         /* work items per outer iteration */
  int64_t items_by_kind[9];/* pass 1, prep 1, inner 1, prep 2, mode 2, inner 2, prep 3, pass 3, inner 3 */
  int64_t x_bytes;         /* bytes of one BF16 copy of all tensors (unpadded) */
  int64_t t_bytes;         /* bytes of all I x J x F intermediates */
} ntf_batch_info;

/* Workspace bytes for these problems and options (0 and *why on error). */
size_t ntf_batch_workspace_bytes(const ntf_problem *probs, int32_t n, const ntf_opts *opts);

/* Validates, carves the workspace (device, 256-byte aligned, caller-owned),
 * writes the BF16 copies and the initial Grams, picks default tiles and
 * captures the iteration graph.  `probs` is host memory [n], copied; every X
 * is borrowed and must outlive the context.  Synchronising. */
ntf_status ntf_batch_init(ntf_batch_ctx **out, const ntf_problem *probs, int32_t n,
                          const ntf_opts *opts, void *workspace, size_t ws_bytes, void *stream);

/* n_outer outer iterations of every problem (graph replays on the stream).
 * Stream-ordered; errors found on the device are reported by ntf_batch_sync. */
ntf_status ntf_batch_step(ntf_batch_ctx *ctx, int32_t n_outer);

/* Waits for the stream; returns NTF_E_NUMERIC if a non-PD system or NaN/Inf
 * was met (bits 1, 2) or a dependency wait timed out (bit 8) since init.
 * `flags_out` (host, may be NULL) receives the bits. */
ntf_status ntf_batch_sync(ntf_batch_ctx *ctx, int32_t *flags_out);

/* Relative fit error ||X - [H1,H2,H3]||_F / ||X||_F of every problem from the
 * FP32 tensors and current factors, FP64 accumulation; rfe_host is host
 * memory [n].  Synchronising. */
ntf_status ntf_batch_fit(ntf_batch_ctx *ctx, double *rfe_host);

/* MTTKRP of mode `mode` (0..2) of problem `prob` from the current factors
 * (the batched kernels' BF16 arithmetic, no factor update) into W_out
 * (device float64 [d_mode][F]).  Runs the pass work of all problems.
 * Stream-ordered. */
ntf_status ntf_batch_mttkrp(ntf_batch_ctx *ctx, int32_t prob, int32_t mode, double *W_out);

/* Launches the work items of one kind for all problems on their own, without
 * dependencies: kind 0 = pass for modes 1 and 2, 4 = mode 2 from T, 7 = pass
 * for mode 3.  Leaves the factors unchanged.  For timing.  Stream-ordered. */
ntf_status ntf_batch_launch_kind(ntf_batch_ctx *ctx, int32_t kind);

/* Autotuner: for each bucket present in the batch, in turn, times six tile
 * choices (mt 1 or 2 x three item sizes) by launching the whole pass of that
 * kind (all problems, the other buckets at their current tiles; one untimed
 * and `reps` timed launches, HIP events), keeps the fastest, then rebuilds
 * the work list and re-captures the graph.  The `us` of a tile is the whole
 * pass time it was chosen with.  Writes the chosen tiles to out (host, up to
 * cap entries; *n_out = entries written).  Factors are unchanged.
 * Synchronising. */
ntf_status ntf_batch_autotune(ntf_batch_ctx *ctx, int32_t reps, ntf_batch_tile *out, int32_t cap,
                              int32_t *n_out);

/* Applies tile choices (e.g. from an autotuner cache) to the matching
 * buckets; others keep theirs.  Rebuilds the work list and re-captures the
 * graph.  Synchronising. */
ntf_status ntf_batch_set_tiles(ntf_batch_ctx *ctx, const ntf_batch_tile *tiles, int32_t n);

/* The current tile choices (host out, up to cap entries). */
ntf_status ntf_batch_get_tiles(ntf_batch_ctx *ctx, ntf_batch_tile *out, int32_t cap, int32_t *n_out);

/* Runs one outer iteration (not from the graph) with per-item wall-clock
 * timing and returns, per work-item kind (the order of items_by_kind), the
 * summed microseconds blocks spent running items (busy_us), waiting for their
 * dependencies (wait_us), and the item count; host arrays [9].  The
 * iteration updates the factors like ntf_batch_step.  Synchronising. */
ntf_status ntf_batch_profile(ntf_batch_ctx *ctx, double *busy_us, double *wait_us, int64_t *items);

ntf_status ntf_batch_info_get(ntf_batch_ctx *ctx, ntf_batch_info *out);
const char *ntf_batch_last_error(const ntf_batch_ctx *ctx);
ntf_status ntf_batch_destroy(ntf_batch_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* NTF_ADMM_H */
