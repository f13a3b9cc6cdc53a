// Host-side launch interface between the NTF kernels and the C-ABI layer.
// Internal to libntf_admm.so; not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ntf {

// A byte offset past every buffer resource the kernels build (their sizes
// stay below it; the host checks that before choosing such a kernel).
constexpr int kBufferOOB = 0x7ffffff0;

enum Prec { PREC_F32 = 0, PREC_BF16 = 1, PREC_F64 = 3 };

// Launch geometry of the three MTTKRP kernels and the inner sweep for one
// problem shape; fixed at context creation.
struct Plan {
  int prec = 0;
  int64_t I = 0, J = 0, K = 0;
  int F = 0, FT = 0, FP = 0;      // rank, 16-column MFMA tiles, padded rank
  int vec = 4;                    // row loads of the FP32/FP64 tensor: 4 (K % 4 == 0), 2 (K even), 1
  // bfloat16 copies: row-major [I][J][Kp] and j-interleaved [I][JG][Kp3][8]
  int64_t Kp = 0, JG = 0, Kp3 = 0;
  // pass 1 (mode-1 MTTKRP plus the k-contracted intermediate T = X x_3 C)
  int MT1 = 1, R1 = 16, nch1 = 0, KC1 = 0, grid1 = 0;  // 16*MT1 rows per wave item
  int64_t ntiles1 = 0;
  size_t lds1 = 0;
  bool ts1 = false;
  int spg1 = 0, G1 = 0;           // BF16 streaming pass 1: slabs per run, runs per row tile               // BF16 streaming pass 1: T rows staged in LDS, 16-byte stores
  // mode 2 from T
  int ich2 = 16, nich2 = 0;
  // pass 3 (mode-3 MTTKRP): waves per block, k-groups, row chunks
  int nw3 = 0, nkg3 = 0, nrc3 = 0;  // nrc3: partials of P3
  int64_t rpc3 = 0;               // rows (FP32/FP64) or slabs (BF16) per block
  int nb3 = 0, rg3 = 1;           // FP32/FP64: row blocks; row groups per block (one partial each)
  bool s3 = false;                // FP32 streaming form
  int jcg3 = 0;                   // BF16: 8-row groups of j per chunk staged in LDS
  int nkt3 = 0, nch3 = 0, ngr3 = 0, bpc3 = 0;   // BF16: k tiles, j chunks, slab groups, blocks per chunk
  size_t lds3 = 0;
  // inner sweep: lanes per row, rows per block, blocks per mode
  int FL = 0, rpb = 0;
  int nblk_inner[3] = {0, 0, 0};
  int nprep = 1;                  // blocks of the prepare kernel
};

size_t elem_size(int prec);       // bytes of an X / factor element for a precision

// Fill `p` for a problem; returns false if unsupported.
bool make_plan(Plan& p, int prec, const int64_t dims[3], int F, int cu_count);

// ---- set-up
hipError_t launch_quantize(const float* X, const Plan& p, __bf16* Xr, __bf16* Xj8, float* scale,
                           hipStream_t s);
hipError_t launch_sumsq(const void* X, int x_is_f64, int64_t n, double* partial, int nparts,
                        double* out, hipStream_t s);

// ---- MTTKRP
// pass 1: Tout [I*J][F] (T elem = float, or double for F64) and P1 [I][nch1][F];
// FP32 and FP64 take Tout = nullptr when only P1 is wanted
hipError_t launch_pass1(const Plan& p, const void* X, const __bf16* Xr, const float* scale,
                        const void* Hb, const void* Hc, void* Tout, void* P1, hipStream_t s);
// mode 2 from T: P2 [nich2][J][F]
hipError_t launch_mode2(const Plan& p, const void* Tin, const void* Ha, void* P2, hipStream_t s);
// pass 3: P3 [nrc3][K][F]
hipError_t launch_pass3(const Plan& p, const void* X, const __bf16* Xj8, const float* scale,
                        const void* Ha, const void* Hb, void* P3, hipStream_t s);
// W[rows][F] (double) = sum over partials, fixed order
// (fixed grouped order: partial p to group p % groups, groups = 4 or 16)
hipError_t launch_reduce_partials(const void* part, int part_is_f64, int64_t pstride,
                                  int64_t rowstride, int nparts, int64_t rows, int F, double* W,
                                  hipStream_t s, int groups);

// ---- ADMM
struct InnerArgs {
  const void* part = nullptr;     // MTTKRP partials (float or double)
  int part_f64 = 0;
  int64_t pstride = 0, rowstride = 0;
  int nparts = 0;
  double* Wout = nullptr;         // may be null
  void* H = nullptr;
  void* U = nullptr;
  void* Pout = nullptr;           // last Ht^T (may be null)
  int h_f64 = 0;
  int64_t rows = 0;
  int F = 0, FL = 0;
  const double* Ginv = nullptr;   // [F][F] (G + rho I)^{-1}, then Ginv 1 [F], 1^T Ginv 1
  int proj = 0;                   // constraint of the factor: 0 non-negative, 1 box, 2 pmf rows,
                                  // 3 deferred to launch_card_project
  double lo = 0.0, hi = 0.0;      // box bounds
  const double* rho = nullptr;    // device: [0] rho for this update, [1] rho of the previous update
  int rescale = 0;
  int T = 1;
  double eps_abs = 0.0, eps_rel = 0.0;
  int32_t* iters_out = nullptr;   // may be null
  int gram_from_primal = 0;       // Gram partial of Ht^T instead of H
  int gram_f32 = 0;               // accumulate the Gram partial in FP32 (mixed precision)
  double* gram_part = nullptr;    // [nblk][F][F]
  double* resid_part = nullptr;   // [nblk][8]
  int* flag = nullptr;
  double* dv = nullptr;           // proj == 3: V, Ht^T and the factor before the update,
  double* dx = nullptr;           // FP64 [rows][F] (dh0 may be null)
  double* dh0 = nullptr;
};
hipError_t launch_inner(const InnerArgs& a, int nblk, hipStream_t s);
int inner_rows_per_block(int FL);     // rows one inner-sweep block handles

struct PrepArgs {
  int F = 0;
  const double* gram_part = nullptr;  // partials of the mode just updated (nullptr: none)
  int nparts = 0;
  double* gram_dst = nullptr;         // its reduced Gram [F][F]
  const double* resid_part = nullptr; // its residual partials [nparts][8]
  double* resid_dst = nullptr;        // its residual totals [8]
  int* fresh_dst = nullptr;           // set to 1 when resid_dst is written
  const double* gram_a = nullptr;     // G = gram_a (*) gram_b for the mode being prepared
  const double* gram_b = nullptr;
  int policy = 0;
  double rho0 = 1, mu = 8, tau_incr = 4, tau_decr = 2;
  double* rho_state = nullptr;        // [0] rho (in/out), [1] previous rho (out)
  const double* resid_mode = nullptr; // residual totals of the mode being prepared
  int* fresh_mode = nullptr;
  double* Ginv = nullptr;             // out [F][F]: (G + rho I)^{-1}; then [F]
                                      // its row sums and [1] their total
  double* G_out = nullptr;            // optional out: G of the mode being prepared [F][F]
  int* taken = nullptr;               // warm-start counter of the mode being prepared (zeroed)
  int* flag = nullptr;
  unsigned* counter = nullptr;        // last-block ticket, zero on entry, left zero
  // optional cheap fit (after the third mode): <W3,H3> and sum(G1*G2*G3)
  const double* W3 = nullptr;
  const void* H3 = nullptr;
  int h_f64 = 0;
  int64_t K = 0;
  const double* gram_c = nullptr;     // third Gram for sum(G1*G2*G3)
  double* fit_out = nullptr;          // [2]
  // direct Gram of the mode just updated (used instead of gram_part when set):
  // gram_nb blocks each sum gram_rpp rows of gram_h (h_f64 dtype) in FP64
  // into gram_scratch[b], and the last block reduces them (4 fixed groups)
  const void* gram_h = nullptr;
  int64_t gram_rows = 0, gram_rpp = 0;
  int gram_nb = 0;
  double* gram_scratch = nullptr;
};
hipError_t launch_prep(const PrepArgs& a, int nblk, hipStream_t s);

// Gram partials: ceil(rows/rpp) partials [p][F][F] of rows [p*rpp, (p+1)*rpp)
hipError_t launch_gram_part(const void* H, int h_f64, int64_t rows, int F, int64_t rpp,
                            int gram_f32, double* part, hipStream_t s);
hipError_t launch_fit(const Plan& p, const void* X, int x_f64, const void* H1, const void* H2,
                      const void* H3, int h_f64, double* part, double* out, hipStream_t s,
                      int* nparts_out);
int fit_parts(const Plan& p);
hipError_t launch_finish(int F, const double* gram_part, int gram_nparts, const double* resid_part,
                         int nparts, const double* g0, const double* g1, const double* W3,
                         const void* H3, int h_f64, int64_t K, double* out, hipStream_t s);
// Gram of a factor by rows: the partition (rows per partial, partials) the
// prepare step's direct Gram uses for `rows` rows
void gram_split(int64_t rows, int64_t* rpp, int* nb);
// FP64 Gram partials by the matrix cores, the partition of gram_split (the
// prepare step's direct Gram forms the same partials)
hipError_t launch_gram_direct(const void* H, int h_f64, int64_t rows, int F, int64_t rpp,
                              double* part, hipStream_t s);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s);

// Cardinality constraint (card.hip): from V, Ht^T and the factor before the
// update (FP64 [n]), keep the card largest positive entries of V in H (ties
// by index), U = H - V, Pout = Ht^T (Pout may be null); residual partial 0
// gets the totals with `iters_total` iterations, partials 1 .. nparts-1 zero.
// One block; n < 2^31.
hipError_t launch_card_project(const double* V, const double* X, const double* H0, void* H,
                               void* U, void* Pout, int h_f64, int64_t n, int64_t card,
                               double iters_total, double* resid_part, int nparts, hipStream_t s);

// ---- sparse tensors (sparse.hip)
constexpr int kSparseFlagRange = 16;      // a coordinate outside the tensor
constexpr int kSparseFlagDuplicate = 32;  // a coordinate given twice
constexpr int kLightPieces = 16;          // cut rows of more pieces are reduced by a block each

int sp_key_bits(const int64_t dims[3]);   // bits of the packed (i_m, i_a, i_b) sort key
int64_t sp_tiles(int64_t n);              // radix-sort tiles of n keys
size_t sp_scan_len(int64_t n);            // digit-count entries per sort pass
size_t sp_scan_chunks(int64_t n);         // scan chunk totals per sort pass
int sp_segment_len(int F, int f64);       // non-zeros per MTTKRP segment
int sp_fit_parts();

// Set-up of one mode: sort, records, segment structure.  Records are
// (row, a, b, value bits) with a, b the other two indices in mode order; FP64
// values go to val_out.  tail/len/heavy describe the rows cut by segment
// boundaries (see sparse.hip); *nheavy gets the number of heavy cut rows.
struct SpBuildArgs {
  const int32_t* idx = nullptr;   // [n][3]
  const void* val = nullptr;      // [n]
  int val_f64 = 0;
  int64_t n = 0;
  int64_t dims[3] = {0, 0, 0};
  int mode = 0;
  uint64_t* k0 = nullptr;         // sort scratch: keys x2, permutations x2 [n]
  uint64_t* k1 = nullptr;
  uint32_t* p0 = nullptr;
  uint32_t* p1 = nullptr;
  uint32_t* hist = nullptr;       // [sp_scan_len]
  uint32_t* offs = nullptr;       // [sp_scan_len]
  uint32_t* tot = nullptr;        // [sp_scan_chunks]
  int4* rec = nullptr;            // outputs [n]
  void* val_out = nullptr;        // FP64 only
  int S = 0;
  int64_t nseg = 0;
  int32_t* tail = nullptr;        // [nseg]
  int32_t* len = nullptr;         // [nseg]
  int32_t* heavy = nullptr;       // [nseg]
  uint32_t* nheavy = nullptr;     // device, one value
  int* flag = nullptr;
};
hipError_t sp_check(const int32_t* idx, int64_t n, const int64_t dims[3], int* flag, hipStream_t s);
hipError_t sp_build_mode(const SpBuildArgs& a, hipStream_t s);

struct SpModeArgs {
  const int4* rec = nullptr;
  const void* val = nullptr;      // FP64 values (null for FP32: in the records)
  const void* Fa = nullptr;       // factor of the slower other mode
  const void* Fb = nullptr;       // factor of the faster other mode
  int f64 = 0;
  int F = 0, S = 0;
  int64_t n = 0, nseg = 0, rows = 0;
  double* W = nullptr;            // [rows][F]
  const int32_t* tail = nullptr;  // segment structure of this mode
  const int32_t* len = nullptr;
  const int32_t* heavy = nullptr;
  int nheavy = 0;
  void* carry_h = nullptr;        // [nseg][F] float (double for f64)
  void* carry_t = nullptr;
};
hipError_t sp_mttkrp(const SpModeArgs& a, hipStream_t s);
hipError_t sp_fit(const int4* rec, const void* val, int f64, const void* A, const void* B, const void* C,
                  int F, int64_t n, const double* g0, const double* g1, const double* g2,
                  const double* xnorm2, double* part, double* out, hipStream_t s);

// ---- learned warm start (mlp.hip)
size_t mlp_param_count(int F, int Hd);
hipError_t mlp_forward(const void* params, int f16, int F, int Hd, const float* X, int64_t B,
                       float* Y, float* act, hipStream_t s);
hipError_t mlp_backward(const float* P, int F, int Hd, const float* X, const float* act,
                        const float* Y, const float* dY, int64_t B, float* grad, float* work,
                        hipStream_t s);
hipError_t mlp_mse(const float* Y, const float* T, int64_t B, int F, float* dY, double* part,
                   double* loss, hipStream_t s);
hipError_t mlp_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                    float b2, float eps, int step, void* p16, hipStream_t s);
hipError_t mlp_features(const double* G, const double* W, int64_t rows, int F,
                        const double* rho_p, double rho_v, float* X, float* scale, hipStream_t s);
hipError_t gather_rows(const float* src, const int64_t* idx, int64_t n, int cols, float* dst,
                       hipStream_t s);
hipError_t mlp_targets(const double* Hs, const float* scale, int64_t rows, int F, float* T,
                       hipStream_t s);
hipError_t hadamard_rho(const double* Ga, const double* Gb, int F, double rho0, double* G,
                        double* rho, hipStream_t s);
hipError_t mlp_judge(const float* Y, const float* scale, const double* G, const double* W, void* H,
                     void* U, int h_f64, int64_t rows, int F, int FL, const double* rho_p,
                     int rescale, int* taken, hipStream_t s);

}  // namespace ntf
