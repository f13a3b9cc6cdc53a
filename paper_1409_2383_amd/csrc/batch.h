// Batched ADMoM NTF: host/device interface of the persistent kernel that runs
// one outer iteration (eq. ADMoM_NTF, modes in the order of eq.
// ADMM_NTF_ALS_C) of many independent problems of uneven shapes.  Internal
// to libntf_admm.so; not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ntf {

// Work-item kinds, also the per-problem phase ids of the completion counters.
// The global work list is sorted so that every item depends only on items
// with smaller tickets (see batch.hip).
enum BKind {
  BK_P1 = 0,     // slab group: T = X x_3 H3 (BF16 MFMA) and W1 rows
  BK_PREP1 = 1,  // G1 = Gram2 (*) Gram3, rho, (G1 + rho I)^{-1}
  BK_IN1 = 2,    // row block of the mode-1 inner sweep (last block: Gram1)
  BK_PREP2 = 3,
  BK_M2 = 4,     // 64 rows of W2 = sum_i H1[i] * T[i]
  BK_IN2 = 5,
  BK_PREP3 = 6,
  BK_P3 = 7,     // slab group: W3 partial from the transposed BF16 copy
  BK_IN3 = 8,
  BK_NKINDS = 9
};
constexpr int kCtrPerProb = 16;   // [0..8] done counts, [9..12] last-block tickets
constexpr int kArriveIn = 9;      // + mode: tickets of the inner phases
constexpr int kArriveP3 = 12;

// One problem of the batch, as the kernel sees it (device pointers).
struct BProb {
  int I, J, K, F;
  int FT, FL, NB;        // 16-column MFMA tiles, inner lanes per row, 16x16 prepare tiles
  int Kp, Jp;            // row lengths of the BF16 copies (multiples of 32)
  int spi1, spi3;        // slabs per pass-1 / pass-3 item
  int mt1, mt3;          // 16-row MFMA tiles per wave step in the two passes
  int n_p1, n_m2, n_p3;  // items per kind
  int n_in[3];           // inner row blocks per mode (Gram partials)
  int ni[3];             // inner items per mode (ipi row blocks each)
  int rpb;               // inner rows per row block
  int ipi;               // inner row blocks per item
  const __bf16* Xr;      // [I][Kp/8][J][8]  (eight consecutive k innermost, zero padded)
  const __bf16* Xt;      // [I][Jp/8][K][8]  (eight consecutive j innermost, zero padded)
  const float* scale;    // [I] power-of-two slab scales
  float* H[3];
  float* U[3];
  float* T;              // [I][J][F]
  double* W[3];          // [d_n][F]
  float* W3p;            // [n_p3][K][F] pass-3 partials
  double* gram[3];       // [F][F] Grams of the current factors
  double* gpart;         // [max n_in][F][F] inner-sweep Gram partials
  double* Ginv;          // [F][F]
  double* rho;           // [3][2]: rho of the last update of each mode, and the one before
};

struct BatchK {
  const BProb* probs;
  const uint2* items;    // x = problem, y = kind << 24 | index
  int n_items;
  int nodeps;            // 1: items run without waiting (pass-only lists)
  unsigned* head;        // ticket counter, zero on entry
  int* ctr;              // [n_probs][kCtrPerProb], zero on entry
  int* flag;             // numeric / wait-timeout bits
  int T;                 // inner iterations
  double eps_abs, eps_rel;
  int rescale;           // scale U by rho_old / rho_new
  int policy;            // 0 trace, 1 fixed
  double rho0;
  long long spin_limit;  // polls before a wait gives up (flag bit 8)
  unsigned long long* prof;  // null, or [BK_NKINDS][3]: wall-clock ticks busy, waiting, items
};

// LDS bytes a problem's items need.
size_t batch_lds_p1(const BProb& p);
size_t batch_lds_p3(const BProb& p);
size_t batch_lds_inner(int FL);
int batch_inner_rows(int FL);      // inner-sweep rows per work item
size_t batch_lds_prep();

hipError_t launch_batch(const BatchK& k, int grid, size_t lds, hipStream_t s);
constexpr int kProfWords = BK_NKINDS * 3;
int batch_occupancy(size_t lds);   // resident blocks per CU at this LDS size (0 on error)
hipError_t launch_zero_ints(int* p, int64_t n, hipStream_t s);
// BF16 copies [I][J][Kp] and [I][K][Jp] of one FP32 problem with slab scales
hipError_t launch_batch_quantize(const float* X, int I, int J, int K, int Kp, int Jp, __bf16* Xr,
                                 __bf16* Xt, float* scale, hipStream_t s);

}  // namespace ntf
