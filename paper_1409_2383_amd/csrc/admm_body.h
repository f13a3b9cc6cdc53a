// Device bodies of the ADMoM mode update shared by the per-problem kernels
// (admm.hip) and the batched persistent kernel (batch.hip): the fused
// row-wise inner sweep and the F x F prepare step (Gram Hadamard product,
// penalty, FP64 inverse of G + rho I).  Internal header.
#pragma once

#include "ntf_device.h"

namespace ntf {

// Block of 256 threads.  A row of the factor lives on FL consecutive lanes
// (FL = next power of two >= F, so a row never straddles a wave), and every
// lane group carries RPL rows at once: lane f holds h_f, u_f, w_f of RPL rows
// in FP64 registers for the whole sweep.  The solve with G + rho I is one
// lane-parallel mat-vec against Ginv = (G + rho I)^{-1}
// (formed once per mode update by the prepare step, symmetric, zero
// padded to FL x FL) in LDS; each Ginv element read serves the RPL rows of
// the lane.  The right-hand sides are exchanged through two alternating LDS
// buffers (broadcast reads): one barrier per inner iteration.
struct InnerK {
  const void* part;
  int part_f64;
  int64_t pstride, rowstride;
  int nparts;
  double* Wout;
  void* H;
  void* U;
  void* Pout;
  int64_t rows;
  int F;
  const double* Ginv;          // (G + rho I)^{-1}, [F][F], then Ginv 1 [F] and 1^T Ginv 1
  int proj;                    // 0 non-negative, 1 box [lo, hi], 2 rows summing to one,
                               // 3 projection deferred to a whole-factor pass (dv, dx, dh0)
  double lo, hi;
  const double* rho;
  int rescale, T;
  double eps_abs, eps_rel;
  int32_t* iters_out;
  int gram_from_primal, gram_f32;
  double* gram_part;
  double* resid_part;
  int* flag;
  // proj == 3 (one inner iteration per launch): V = Ht^T - U, Ht^T and, when
  // dh0 is set, the factor before the update go to these FP64 [rows][F]
  // buffers; H, U, the partials and the statistics are left to the
  // whole-factor projection that follows
  double* dv;
  double* dx;
  double* dh0;
};

// Rows per lane group: two at FL = 32 (each LDS read of Ginv serves both);
// one at FL = 64, where twice the blocks fill more of the chip (measured
// faster at F = 64, 1000 rows)
template <int FL>
static constexpr int inner_rpl() { return FL == 32 ? 2 : 1; }

// out[q] = sum_g M[g*FL + f] * V[q*BS + g] for the RPL rows of a lane, with
// the LDS reads of chunk c+1 issued before the FMAs of chunk c (register
// double buffering), so LDS latency overlaps arithmetic.
template <int FL, int RPL, int BS, int CH = 8>
static __device__ __forceinline__ void lane_matvec(const double* __restrict__ M,
                                                   const double* __restrict__ V, int f,
                                                   double (&out)[RPL]) {
  constexpr int C = FL < CH ? FL : CH;
  constexpr int NC = FL / C;
  double ma[C], va[RPL][C], mb[C], vb[RPL][C];
#pragma unroll
  for (int q = 0; q < RPL; ++q) out[q] = 0.0;
  auto ld = [&](int c, double (&m)[C], double (&v)[RPL][C]) {
#pragma unroll
    for (int t = 0; t < C; ++t) {
      m[t] = M[(c * C + t) * FL + f];
#pragma unroll
      for (int q = 0; q < RPL; ++q) v[q][t] = V[q * BS + c * C + t];
    }
  };
  auto fm = [&](const double (&m)[C], const double (&v)[RPL][C]) {
#pragma unroll
    for (int t = 0; t < C; ++t)
#pragma unroll
      for (int q = 0; q < RPL; ++q) out[q] += m[t] * v[q][t];
  };
  ld(0, ma, va);
  if constexpr (NC == 1) {
    fm(ma, va);
  } else {
    // NC is even here; a rolled loop keeps the compiler from hoisting every
    // chunk's loads (which would blow the register budget)
#pragma unroll 1
    for (int c = 0; c < NC; c += 2) {
      ld(c + 1, mb, vb);
      fm(ma, va);
      if (c + 2 < NC) ld(c + 2, ma, va);
      fm(mb, vb);
    }
  }
}
template <int FL>
static constexpr int inner_rows_per_block() { return (256 / FL) * inner_rpl<FL>(); }

// The body of one inner-sweep block (rows bid*RPB ..), with its dynamic LDS at
// smem_raw; also called per work item by the batched persistent kernel, with
// a smaller register footprint: CH = mat-vec chunk, GF = 1 fixes the Gram
// partial to FP32 (-1: a.gram_f32 decides at run time).
template <typename HT, int FL, int RPL = inner_rpl<FL>(), int CH = 8, int GF = -1>
__device__ __forceinline__ void inner_body(const InnerK& a, int64_t bid, unsigned char* smem_raw,
                                           const int tid, const bool load_ginv = true) {
  constexpr int NG = 256 / FL;             // lane groups per block
  constexpr int RPB = NG * RPL;            // rows per block
  constexpr int BS = FL + 1;               // padded row stride of the exchange buffers
  const int F = a.F;
  double* Ms = reinterpret_cast<double*>(smem_raw);   // Ms[g][f] = Ginv[g][f] = Ginv[f][g]
  double* xb = Ms + FL * FL;                          // [2][RPB][BS] right-hand sides
  __shared__ double red[4][8];

  const int grp = tid / FL, f = tid - grp * FL;
  const int64_t row0 = bid * RPB;

  // (a caller that runs several row blocks in turn with the same Ginv loads
  // it for the first only: nothing below writes that LDS region)
  if (load_ginv) {
    // all loads first, then the LDS writes (no serialised load-wait chain)
    constexpr int PER = (FL * FL + 255) / 256;
    double lv[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q;
      const int r = e / FL, c = e - r * FL;
      lv[q] = (e < FL * FL && r < F && c < F) ? a.Ginv[r * F + c] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q;
      if (e < FL * FL) Ms[e] = lv[q];
    }
  }
  const double rho = a.rho[0];
  const double uscale = (a.rescale && a.rho[1] > 0.0) ? a.rho[1] / rho : 1.0;
  // pmf rows: this lane's entry of Ginv 1 and 1 / (1^T Ginv 1)
  const double g1f = (a.proj == 2 && f < F) ? a.Ginv[F * F + f] : 0.0;
  const double inv_1g1 = (a.proj == 2) ? 1.0 / a.Ginv[F * F + F] : 0.0;

  // row q of this lane group is block row grp*RPL + q
  double w[RPL], h[RPL], u[RPL], x[RPL], h0[RPL];
  bool act[RPL], done[RPL];
  int iters[RPL];
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int64_t row = row0 + grp * RPL + q;
    act[q] = (row < a.rows) && (f < F);
    done[q] = row >= a.rows;
    iters[q] = 0;
    w[q] = h[q] = u[q] = x[q] = 0.0;
    if (act[q]) {
      const int64_t off = row * a.rowstride + f;
      double sw = 0.0;
      if (a.part_f64) {
        const double* p = reinterpret_cast<const double*>(a.part) + off;
#pragma unroll 8
        for (int t = 0; t < a.nparts; ++t) sw += p[t * a.pstride];
      } else {
        const float* p = reinterpret_cast<const float*>(a.part) + off;
#pragma unroll 8
        for (int t = 0; t < a.nparts; ++t) sw += (double)p[t * a.pstride];
      }
      w[q] = sw;
      if (a.Wout) a.Wout[row * F + f] = sw;
      h[q] = (double)reinterpret_cast<const HT*>(a.H)[row * F + f];
      u[q] = (double)reinterpret_cast<const HT*>(a.U)[row * F + f] * uscale;
    }
    h0[q] = h[q];
  }
  const bool early = (a.eps_abs > 0.0) || (a.eps_rel > 0.0);
  const double sqF = sqrt((double)F);
  __shared__ int any_active;

  for (int t = 0; t < a.T; ++t) {
    if (early) {
      if (tid == 0) any_active = 0;
      __syncthreads();
      bool mine = false;
#pragma unroll
      for (int q = 0; q < RPL; ++q) mine |= !done[q];
      if (mine) any_active = 1;
      __syncthreads();
      if (!any_active) break;
    }
    // iteration t writes buffer t & 1: a wave still reading the other one
    // (iteration t - 1) is past the barrier before it is written again
    double* bb = xb + (t & 1) * RPB * BS;
#pragma unroll
    for (int q = 0; q < RPL; ++q) bb[(grp * RPL + q) * BS + f] = act[q] ? w[q] + rho * (h[q] + u[q]) : 0.0;
    __syncthreads();
    double xn[RPL];
    lane_matvec<FL, RPL, BS, CH>(Ms, bb + grp * RPL * BS, f, xn);  // x = (G + rho I)^{-1} b
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      if (done[q]) continue;
      if (a.proj == 2) {
        // rows summing to one: x -= Ginv 1 (1^T x - 1) / (1^T Ginv 1)
        const double sx = group_sum(xn[q], FL);
        xn[q] -= g1f * ((sx - 1.0) * inv_1g1);
      }
      const double v = xn[q] - u[q];
      const double hn = (a.proj == 1) ? fmin(fmax(v, a.lo), a.hi)
                        : (a.proj == 3) ? v : ((v > 0.0) ? v : 0.0);
      const double un = hn - v;
      const double dh = hn - h[q];
      h[q] = act[q] ? hn : 0.0;
      u[q] = act[q] ? un : 0.0;
      x[q] = act[q] ? xn[q] : 0.0;
      ++iters[q];
      if (early) {
        const double sp = group_sum((h[q] - x[q]) * (h[q] - x[q]), FL);
        const double sx = group_sum(x[q] * x[q], FL);
        const double sh = group_sum(h[q] * h[q], FL);
        const double sd = group_sum(act[q] ? dh * dh : 0.0, FL);
        const double su = group_sum(u[q] * u[q], FL);
        const double tol_p = sqF * a.eps_abs + a.eps_rel * fmax(sqrt(sx), sqrt(sh));
        const double tol_d = sqF * a.eps_abs + a.eps_rel * rho * sqrt(su);
        if (sqrt(sp) <= tol_p && rho * sqrt(sd) <= tol_d) done[q] = true;
      }
    }
  }
  __syncthreads();

  if (a.proj == 3) {   // uniform over the block
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int64_t row = row0 + grp * RPL + q;
      if (act[q]) {
        if (!isfinite(x[q]) || !isfinite(w[q])) atomicOr(a.flag, 1);
        a.dv[row * F + f] = h[q];
        a.dx[row * F + f] = x[q];
        if (a.dh0) a.dh0[row * F + f] = h0[q];
      }
    }
    return;
  }

  double qs[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int64_t row = row0 + grp * RPL + q;
    if (act[q]) {
      if (!isfinite(x[q]) || !isfinite(w[q])) atomicOr(a.flag, 1);
      reinterpret_cast<HT*>(a.H)[row * F + f] = (HT)h[q];
      reinterpret_cast<HT*>(a.U)[row * F + f] = (HT)u[q];
      if (a.Pout) reinterpret_cast<HT*>(a.Pout)[row * F + f] = (HT)x[q];
      if (a.iters_out && f == 0) a.iters_out[row] = iters[q];
      const double hv = (double)(HT)h[q], xv = (double)(HT)x[q], uv = (double)(HT)u[q];
      qs[0] += (hv - xv) * (hv - xv);
      qs[1] += (hv - h0[q]) * (hv - h0[q]);
      qs[2] += hv * hv;
      qs[3] += xv * xv;
      qs[4] += uv * uv;
      if (f == 0) qs[5] += (double)iters[q];
    }
  }
  // residual partials of this block: ||h-x||^2, ||h-h0||^2, ||h||^2, ||x||^2, ||u||^2, iterations
  {
    const int wave = tid >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double sum = group_sum(qs[k], 64);
      if ((tid & 63) == 0) red[wave][k] = sum;
    }
    __syncthreads();
    if (a.resid_part) {
      if (tid < 6) {
        const double sum = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
        a.resid_part[bid * 8 + tid] = sum;
      }
      if (tid == 6 || tid == 7) a.resid_part[bid * 8 + tid] = 0.0;
    }
  }
  // Gram partial of this block's rows (of the stored factor values), rows in
  // order (skipped when the caller forms the Gram from the factor itself)
  if (a.gram_part) {
    double* hs = xb;  // [RPB][BS]; the barrier after the sweep ends every read of xb
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const double src = a.gram_from_primal ? x[q] : h[q];
      hs[(grp * RPL + q) * BS + f] = act[q] ? (double)(HT)src : 0.0;
    }
    __syncthreads();
    const int nrow = (int)min((int64_t)RPB, a.rows - row0);
    // thread (ti,tj) owns entries (ti+16p, tj+16q); each entry is summed over
    // the block's rows in row order (the order the standalone Gram partials use)
    constexpr int NBT = (FL + 15) / 16;
    const int ti = tid >> 4, tj = tid & 15;
    const bool gf32 = (GF < 0) ? (a.gram_f32 != 0) : (GF == 1);
    constexpr int NBD = (GF == 1) ? 1 : NBT;   // FP64 accumulators (unused when GF == 1)
    double acc[NBD][NBD];
    float accf[NBT][NBT];
#pragma unroll
    for (int p = 0; p < NBT; ++p)
#pragma unroll
      for (int q = 0; q < NBT; ++q) accf[p][q] = 0.f;
#pragma unroll
    for (int p = 0; p < NBD; ++p)
#pragma unroll
      for (int q = 0; q < NBD; ++q) acc[p][q] = 0.0;
    for (int r2 = 0; r2 < nrow; ++r2) {
      double vi[NBT], vj[NBT];
#pragma unroll
      for (int p = 0; p < NBT; ++p) {
        vi[p] = (ti + 16 * p < FL) ? hs[r2 * BS + ti + 16 * p] : 0.0;
        vj[p] = (tj + 16 * p < FL) ? hs[r2 * BS + tj + 16 * p] : 0.0;
      }
      if (gf32) {
#pragma unroll
        for (int p = 0; p < NBT; ++p)
#pragma unroll
          for (int q = 0; q < NBT; ++q) accf[p][q] += (float)vi[p] * (float)vj[q];
      } else if constexpr (GF != 1) {
#pragma unroll
        for (int p = 0; p < NBD; ++p)
#pragma unroll
          for (int q = 0; q < NBD; ++q) acc[p][q] += vi[p] * vj[q];
      }
    }
#pragma unroll
    for (int p = 0; p < NBT; ++p)
#pragma unroll
      for (int q = 0; q < NBT; ++q) {
        const int r = ti + 16 * p, c = tj + 16 * q;
        if (r < F && c < F) {
          double v = (double)accf[p][q];
          if constexpr (GF != 1) {
            if (!gf32) v = acc[p][q];
          }
          a.gram_part[bid * F * F + r * F + c] = v;
        }
      }
  }
}

struct PrepK {
  int F;
  const double* gram_part;
  int nparts;
  double* gram_dst;
  const double* resid_part;
  double* resid_dst;
  int* fresh_dst;
  const double* gram_a;
  const double* gram_b;
  int policy;
  double rho0, mu, tau_incr, tau_decr;
  double* rho_state;
  const double* resid_mode;
  int* fresh_mode;
  double* Ginv;
  double* G_out;
  int* taken;
  int* flag;
  unsigned* counter;
  const double* W3;
  const void* H3;
  int h_f64;
  int64_t K;
  const double* gram_c;
  double* fit_out;
  // direct Gram of the mode just updated (instead of gram_part): blocks
  // 0 .. gram_nb-1 each sum gram_rpp rows of gram_h into gram_scratch[b]
  const void* gram_h;
  int64_t gram_rows, gram_rpp;
  int gram_nb;
  double* gram_scratch;
};

// LDS of prep_body: S [64][65] (the inverse, for the symmetrised write-out;
// during the elimination it holds the broadcast rows [2][16][64]; the Gram
// stage of the prepare kernel borrows it too), the diagonal of G [64], a
// reduction buffer [256], rho.
constexpr int kPrepLdsDoubles = 64 * 65 + 64 + 256 + 1;
// LDS of the matrix-core Gram partial (gram_rows_mfma): 4 waves x 4 tiles of
// 16 x 16 doubles
constexpr int kGramLdsDoubles = 4 * 4 * 4 * 64;

// Global inputs of prep_body, loaded into registers ahead of it (the
// per-problem prepare kernel issues these loads before its Gram phase, so
// their latency overlaps that work): this thread's tile of gram_a and gram_b
// (prep_entry) and (thread 0) the penalty state.
template <int NB>
struct PrepIn {
  double ga[NB * NB], gb[NB * NB];
  double rho_prev, res0, res1;
  int fresh;
};

// Entry q of a thread's tile: thread (ti, tj) = (tid / 16, tid % 16) holds
// the entries (ti + 16 a, tj + 16 b), a, b < NB, q = a NB + b.  Returns the
// row-major index in an F x F matrix, or -1 past F.
template <int NB>
__device__ __forceinline__ int prep_entry(int F, int tid, int q) {
  const int r = (tid >> 4) + 16 * (q / NB), c = (tid & 15) + 16 * (q % NB);
  return (r < F && c < F) ? r * F + c : -1;
}

template <int NB>
__device__ __forceinline__ void prep_load_b(const PrepK& a, const int tid, PrepIn<NB>& in) {
  const int F = a.F;
#pragma unroll
  for (int q = 0; q < NB * NB; ++q) {
    const int e = prep_entry<NB>(F, tid, q);
    in.gb[q] = (e >= 0) ? a.gram_b[e] : 0.0;
  }
  in.rho_prev = 0.0;
  in.res0 = in.res1 = 0.0;
  in.fresh = 0;
  if (tid == 0) {
    in.rho_prev = a.rho_state[0];
    if (a.policy == 2 && a.fresh_mode) {
      in.fresh = *a.fresh_mode;
      in.res0 = a.resid_mode[0];
      in.res1 = a.resid_mode[1];
    }
  }
}

template <int NB>
__device__ __forceinline__ void prep_load_a(const PrepK& a, const int tid, PrepIn<NB>& in) {
  const int F = a.F;
#pragma unroll
  for (int q = 0; q < NB * NB; ++q) {
    const int e = prep_entry<NB>(F, tid, q);
    in.ga[q] = (e >= 0) ? a.gram_a[e] : 0.0;
  }
}

// 1 / x by the hardware reciprocal and two Newton steps (x positive and
// normal: the pivots of an SPD matrix); within an ulp or two of 1.0 / x.
static __device__ __forceinline__ double recip_pos(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  return r;
}

// Factors of one Gauss-Jordan step on a thread's tile (below) with the pivot
// p in tile row and column slot 0.  rowc[u] / rowr[s] hold row p as it
// stands before the step at the thread's columns of slot u and at its rows of
// slot s (the column p entries of those rows, by symmetry up to sign); sg[s]
// is -1 for slots of tile rows before p's, +1 after; inv = 1 / pivot; own_r /
// own_c: the thread holds row p / column p in slot 0, before_r: its slot-0
// row precedes p.  Every entry becomes fma(-cv[s], rs[u], M[s][u]); row p and
// column p go through the same form with their old value multiplied by 0
// (kr, kc) and the factors replaced: cv = -1 on row p, rs = 1 / pivot on
// column p.
template <int NB>
struct GjStep {
  double cv[NB], rs[NB], kr, kc;
};

template <int NB>
__device__ __forceinline__ GjStep<NB> gj_factors(double inv, const double (&rowc)[NB],
                                                 const double (&rowr)[NB], const double (&sg)[NB],
                                                 bool own_r, bool own_c, bool before_r) {
  GjStep<NB> g;
  g.kr = own_r ? 0.0 : 1.0;
  g.kc = own_c ? 0.0 : 1.0;
  g.cv[0] = own_r ? -1.0 : (before_r ? -rowr[0] : rowr[0]);
  g.rs[0] = own_c ? inv : rowc[0] * inv;
#pragma unroll
  for (int s = 1; s < NB; ++s) g.cv[s] = rowr[s] * sg[s];
#pragma unroll
  for (int u = 1; u < NB; ++u) g.rs[u] = rowc[u] * inv;   // row p over the pivot
  return g;
}

// the step on tile row slot 0 (the row that is broadcast next)
template <int NB>
__device__ __forceinline__ void gj_row0(double (&M)[NB][NB], const GjStep<NB>& g) {
  M[0][0] = __builtin_fma(-g.cv[0], g.rs[0], M[0][0] * (g.kr * g.kc));
#pragma unroll
  for (int u = 1; u < NB; ++u) M[0][u] = __builtin_fma(-g.cv[0], g.rs[u], M[0][u] * g.kr);
}

// the step on tile row slots 1 .. NB-1
template <int NB>
__device__ __forceinline__ void gj_rest(double (&M)[NB][NB], const GjStep<NB>& g) {
#pragma unroll
  for (int s = 1; s < NB; ++s) {
    M[s][0] = __builtin_fma(-g.cv[s], g.rs[0], M[s][0] * g.kc);
#pragma unroll
    for (int u = 1; u < NB; ++u) M[s][u] = __builtin_fma(-g.cv[s], g.rs[u], M[s][u]);
  }
}

// (a pivot that is not positive and finite only sets the flag: the result is
// discarded then, so what it does to the rest of the elimination is moot)
static __device__ __forceinline__ double pivot_recip(double piv, bool& bad) {
  bad |= !(piv > 0.0) || !isfinite(piv);
  return recip_pos(piv);
}

// Second half of the prepare step, run by one block of 256 threads: G =
// gram_a (*) gram_b, the penalty, and Ginv = (G + rho I)^{-1} by Gauss-Jordan
// elimination on the matrix held in registers, a tile of NB x NB entries per
// thread (prep_entry).  `lds` holds kPrepLdsDoubles doubles; `in` holds the
// global inputs (prep_load_a, prep_load_b).  Also called per work item by the
// batched persistent kernel.
//
// Step p = 0 .. F-1 on M (initially S = G + rho I):
//   M[p][p] <- 1 / M[p][p],   M[p][j] <- M[p][j] / M[p][p],
//   M[i][p] <- -M[i][p] / M[p][p],   M[i][j] <- M[i][j] - M[i][p] M[p][j] / M[p][p]
// leaves S^{-1}.  Before step p, with A the leading p x p block of the
// symmetric S = [A B; B^T D], M = [A^{-1}, A^{-1} B; -B^T A^{-1}, D - B^T A^{-1} B],
// so column p is row p with the sign changed above row p: only rows are
// broadcast.  Steps go in pairs: every thread writes its slot-0 tile row to
// LDS (rows p and p + 1 among them, as they stand before step p), one
// barrier, then each thread forms row p + 1 after step p itself where it
// reads it (the same operations its owners apply) and applies both steps.
// The tile slots rotate by one after each tile row, so the pivot's tile row
// and column are always slot 0.  No pivoting: the pivots are diagonal
// entries of successive Schur complements of the SPD S, so a pivot that is
// not positive and finite means S is not (numerically) positive definite:
// the failure flag is set and Ginv is zero.
template <int NB>
__device__ __forceinline__ void prep_body(const PrepK& a, double* lds, const int tid,
                                          const PrepIn<NB>& in) {
  constexpr int LD = 65;
  const int F = a.F;
  const int ti = tid >> 4, tj = tid & 15;
  double* S = lds;                 // [64][65]
  double* Rall = lds;              // [2][16][64] during the elimination
  double* Dg = lds + 64 * LD;      // [64]
  double* sred = Dg + 64;          // [256]
  double& rho_sh = sred[256];

  double M[NB][NB];
#pragma unroll
  for (int ia = 0; ia < NB; ++ia)
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) {
      const int q = ia * NB + ib;
      const int e = prep_entry<NB>(F, tid, q);
      const double gv = (e >= 0) ? in.ga[q] * in.gb[q] : 0.0;
      M[ia][ib] = gv;
      if (e >= 0) {
        if (a.G_out) a.G_out[e] = gv;
        if (ia == ib && ti == tj) Dg[ti + 16 * ia] = gv;
      }
    }
  if (tid == 0 && a.taken) *a.taken = 0;
  __syncthreads();

  // penalty (the trace summed by one wave)
  if (tid < 64) {
    double tr = 0.0;
    if (a.policy == 0) tr = group_sum(tid < F ? Dg[tid] : 0.0, 64);
    if (tid == 0) {
      const double rho_prev = in.rho_prev;
      double rho;
      if (a.policy == 0) {
        rho = tr / F;
        if (!(rho > 0.0) || !isfinite(rho)) rho = a.rho0;
      } else if (a.policy == 1) {
        rho = a.rho0;
      } else {
        rho = rho_prev > 0.0 ? rho_prev : a.rho0;
        if (in.fresh) {
          const double prim = sqrt(in.res0);
          const double dual = rho * sqrt(in.res1);
          if (prim > a.mu * dual) rho = rho * a.tau_incr;
          else if (dual > a.mu * prim) rho = rho / a.tau_decr;
          *a.fresh_mode = 0;
        }
      }
      a.rho_state[1] = (rho_prev > 0.0) ? rho_prev : rho;
      a.rho_state[0] = rho;
      rho_sh = rho;
    }
  }
  __syncthreads();
  {
    const double rho = rho_sh;
    if (ti == tj) {
#pragma unroll
      for (int ia = 0; ia < NB; ++ia)
        if (ti + 16 * ia < F) M[ia][ia] += rho;
    }
  }

  // slot u of the tile holds tile row / column (u + PA) mod NB while tile
  // row PA is eliminated
  double sg[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) sg[u] = 1.0;
  // a broadcast row is stored in slot order (slot u of column group tj at
  // tj + 16 u), so every read below is a fixed offset from a lane base
  auto put_rows = [&](int buf) {
    double* W = Rall + (buf * 16 + ti) * 64 + tj;
#pragma unroll
    for (int u = 0; u < NB; ++u) W[16 * u] = M[0][u];
  };
  put_rows(0);
  int buf = 0;
  bool bad = false;   // (every thread sees the same pivots)
#pragma unroll 1
  for (int PA = 0; PA < NB; ++PA) {
    const int n = min(16, F - 16 * PA);   // pivots in this tile row (>= 1)
    // Steps p and p + 1 together, as one step with the 2 x 2 pivot block
    // P = [a b; b d] of rows and columns K = {p, p + 1}:
    //   M_KK <- P^{-1},  M_Kj <- P^{-1} M_Kj,  M_iK <- -M_iK P^{-1},
    //   M_ij <- M_ij - M_iK P^{-1} M_Kj
    // (one reciprocal, of det P = a d - b^2 = a times the second pivot)
#pragma unroll 1
    for (int pt = 0; pt + 1 < n; pt += 2) {
      __syncthreads();
      const double* R0 = Rall + (buf * 16 + pt) * 64;
      const double* R1 = R0 + 64;
      double rowc0[NB], rowr0[NB], rowc1[NB], rowr1[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        rowc0[u] = R0[tj + 16 * u];
        rowc1[u] = R1[tj + 16 * u];
        rowr0[u] = R0[ti + 16 * u];
        rowr1[u] = R1[ti + 16 * u];
      }
      const double pa = R0[pt], pb = R0[pt + 1], pd = R1[pt + 1];
      const double det = __builtin_fma(pa, pd, -(pb * pb));
      bad |= !(pa > 0.0) || !isfinite(pa) || !(det > 0.0) || !isfinite(det);
      const double rd = recip_pos(det);
      const double q00 = pd * rd, q01 = -pb * rd, q11 = pa * rd;   // P^{-1}
      const bool or0 = (ti == pt), or1 = (ti == pt + 1), oc0 = (tj == pt), oc1 = (tj == pt + 1);
      // P^{-1} M_Kc at the thread's columns, -M_rK (signed rows p, p + 1 at
      // its rows), with the substitutions that give rows and columns K
      double w0[NB], w1[NB], c0[NB], c1[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        w0[u] = __builtin_fma(q00, rowc0[u], q01 * rowc1[u]);
        w1[u] = __builtin_fma(q01, rowc0[u], q11 * rowc1[u]);
      }
      w0[0] = oc0 ? q00 : oc1 ? q01 : w0[0];
      w1[0] = oc0 ? q01 : oc1 ? q11 : w1[0];
      {
        const double s0 = (ti < pt) ? -1.0 : 1.0;
        c0[0] = or0 ? -1.0 : or1 ? 0.0 : rowr0[0] * s0;
        c1[0] = or0 ? 0.0 : or1 ? -1.0 : rowr1[0] * s0;
      }
#pragma unroll
      for (int u = 1; u < NB; ++u) {
        c0[u] = rowr0[u] * sg[u];
        c1[u] = rowr1[u] * sg[u];
      }
      const double kr = (or0 || or1) ? 0.0 : 1.0, kc = (oc0 || oc1) ? 0.0 : 1.0;
#pragma unroll
      for (int sl = 0; sl < NB; ++sl)
#pragma unroll
        for (int u = 0; u < NB; ++u) {
          double m = M[sl][u];
          if (sl == 0 && u == 0) m *= kr * kc;
          else if (sl == 0) m *= kr;
          else if (u == 0) m *= kc;
          M[sl][u] = __builtin_fma(-c0[sl], w0[u], __builtin_fma(-c1[sl], w1[u], m));
        }
      buf ^= 1;
      if (pt + 2 < n) put_rows(buf);
    }
    if (n & 1) {   // the last pivot of an odd tile row on its own
      const int pt = n - 1;
      __syncthreads();
      const double* R0 = Rall + (buf * 16 + pt) * 64;
      double rowc0[NB], rowr0[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        rowc0[u] = R0[tj + 16 * u];
        rowr0[u] = R0[ti + 16 * u];
      }
      const double inv0 = pivot_recip(R0[pt], bad);
      const GjStep<NB> g = gj_factors<NB>(inv0, rowc0, rowr0, sg, ti == pt, tj == pt, ti < pt);
      gj_row0<NB>(M, g);
      gj_rest<NB>(M, g);
      buf ^= 1;
    }
    // rotate the slots: tile row / column PA + 1 into slot 0
    if (NB > 1) {
      double t0[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) t0[u] = M[0][u];
#pragma unroll
      for (int s = 0; s + 1 < NB; ++s)
#pragma unroll
        for (int u = 0; u < NB; ++u) M[s][u] = M[s + 1][u];
#pragma unroll
      for (int u = 0; u < NB; ++u) M[NB - 1][u] = t0[u];
#pragma unroll
      for (int s = 0; s < NB; ++s) {
        const double c0 = M[s][0];
#pragma unroll
        for (int u = 0; u + 1 < NB; ++u) M[s][u] = M[s][u + 1];
        M[s][NB - 1] = c0;
      }
#pragma unroll
      for (int u = 0; u + 1 < NB; ++u) sg[u] = sg[u + 1];
      sg[NB - 1] = -1.0;   // tile row PA, now eliminated
    }
    if (PA + 1 < NB) put_rows(buf);
  }
  __syncthreads();   // (S overlays the broadcast rows)
#pragma unroll
  for (int ia = 0; ia < NB; ++ia)
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) {
      const int r = ti + 16 * ia, c = tj + 16 * ib;
      if (r < F && c < F) S[r * LD + c] = M[ia][ib];
    }
  __syncthreads();
  // Ginv (symmetrised), Ginv 1 and 1^T Ginv 1 (the sum-to-one least-squares
  // step uses them): thread t sums a quarter of row t / 4
  {
    const int i = tid >> 2, c0 = (tid & 3) * 16;
    double rs = 0.0;
    if (i < F) {
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const int j = c0 + c;
        if (j < F) {
          const double v = bad ? 0.0 : 0.5 * (S[i * LD + j] + S[j * LD + i]);
          a.Ginv[i * F + j] = v;
          rs += v;
        }
      }
    }
    rs = group_sum(rs, 4);
    if ((tid & 3) == 0) {
      if (i < F) a.Ginv[F * F + i] = rs;
      sred[i] = (i < F) ? rs : 0.0;
    }
    __syncthreads();
    if (tid < 64) {
      const double tot = group_sum(sred[tid], 64);
      if (tid == 0) a.Ginv[F * F + F] = tot;
    }
    __syncthreads();   // sred is reused below
  }
  if (bad && tid == 0) atomicOr(a.flag, 2);

  // optional cheap fit terms: <W3, H3> and sum(G1 * G2 * G3)
  if (a.fit_out) {
    double s1 = 0.0, s2 = 0.0;
    const int64_t nkf = a.K * F;
    for (int64_t e = tid; e < nkf; e += 256) {
      const double hv = a.h_f64 ? reinterpret_cast<const double*>(a.H3)[e]
                                : (double)reinterpret_cast<const float*>(a.H3)[e];
      s1 += a.W3[e] * hv;
    }
    for (int e = tid; e < F * F; e += 256) s2 += a.gram_a[e] * a.gram_b[e] * a.gram_c[e];
    sred[tid] = s1;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) sred[tid] += sred[tid + w];
      __syncthreads();
    }
    if (tid == 0) a.fit_out[0] = sred[0];
    __syncthreads();
    sred[tid] = s2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) sred[tid] += sred[tid + w];
      __syncthreads();
    }
    if (tid == 0) a.fit_out[1] = sred[0];
  }
}

}  // namespace ntf
