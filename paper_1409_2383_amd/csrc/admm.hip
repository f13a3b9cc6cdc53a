// ADMoM kernels for gfx950: the F x F system (Gram Hadamard product, penalty,
// FP64 Cholesky and triangular inverse) and the fused row-wise inner sweep
// (two triangular solves, projection, dual update, residuals, Gram partial),
// plus the standalone Gram and direct-fit kernels.
//
// One mode update (Section IV, eq. ADMM_NTF_ALS_C with eq. ADMoM_NTF) is
//   prep:  G = Gram_a (*) Gram_b,  rho,  L = chol(G + rho I),  Linv = L^{-1}
//   inner: per row, T times:  b = w + rho (h + u);  ht = Linv^T (Linv b);
//                             v = ht - u;  h = max(0, v);  u = h - v.
// The system matrix is common to all rows (Appendix B), so it is factored
// once per mode update; the rows are then independent.
#include "ntf_device.h"
#include "ntf_launch.h"

namespace ntf {

// ---------------------------------------------------------------- inner sweep

// Block of 256 threads.  A row of the factor lives on FL consecutive lanes
// (FL = next power of two >= F, so a row never straddles a wave), and every
// lane group carries RPL rows at once: lane f holds h_f, u_f, w_f of RPL rows
// in FP64 registers for the whole sweep.  Both triangular applications are
// lane-parallel mat-vecs against Linv (zero padded to FL x FL) in LDS, held
// row-major and transposed so every step reads consecutive banks; each Linv
// element read from LDS serves the RPL rows of the lane.  The right-hand
// sides are exchanged through LDS (broadcast reads), two barriers per
// inner iteration.
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
  const double* Linv;
  const double* rho;
  int rescale, T;
  double eps_abs, eps_rel;
  int32_t* iters_out;
  int gram_from_primal, gram_f32;
  double* gram_part;
  double* resid_part;
  int* flag;
};

template <int FL>
static constexpr int inner_rpl() { return FL >= 32 ? 2 : 1; }

// out[q] = sum_g M[g*FL + f] * V[q*BS + g] for the RPL rows of a lane, with
// the LDS reads of chunk c+1 issued before the FMAs of chunk c (register
// double buffering), so LDS latency overlaps arithmetic.
template <int FL, int RPL, int BS>
static __device__ __forceinline__ void lane_matvec(const double* __restrict__ M,
                                                   const double* __restrict__ V, int f,
                                                   double (&out)[RPL]) {
  constexpr int C = FL < 8 ? FL : 8;
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

template <typename HT, int FL>
__global__ __launch_bounds__(256) void k_inner(InnerK a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int RPL = inner_rpl<FL>();
  constexpr int NG = 256 / FL;             // lane groups per block
  constexpr int RPB = NG * RPL;            // rows per block
  constexpr int BS = FL + 1;               // padded row stride of the exchange buffers
  const int F = a.F;
  double* Ls = reinterpret_cast<double*>(smem_raw);   // Ls[g][f]  = Linv[g][f]
  double* LTs = Ls + FL * FL;                         // LTs[g][f] = Linv[f][g]
  double* xb = LTs + FL * FL;                         // [RPB][BS] exchange (b, then y)
  __shared__ double red[4][8];

  const int tid = threadIdx.x;
  const int grp = tid / FL, f = tid - grp * FL;
  const int64_t row0 = (int64_t)blockIdx.x * RPB;

  {
    // all loads first, then the LDS writes (no serialised load-wait chain)
    constexpr int PER = (FL * FL + 255) / 256;
    double lv[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q;
      const int r = e / FL, c = e - r * FL;
      lv[q] = (e < FL * FL && r < F && c < F) ? a.Linv[r * F + c] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q;
      if (e < FL * FL) {
        const int r = e / FL, c = e - r * FL;
        Ls[e] = lv[q];
        LTs[c * FL + r] = lv[q];
      }
    }
  }
  const double rho = a.rho[0];
  const double uscale = (a.rescale && a.rho[1] > 0.0) ? a.rho[1] / rho : 1.0;

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
  double* yb = xb + RPB * BS;   // second exchange buffer: b and y never share one

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
#pragma unroll
    for (int q = 0; q < RPL; ++q) xb[(grp * RPL + q) * BS + f] = act[q] ? w[q] + rho * (h[q] + u[q]) : 0.0;
    __syncthreads();
    double y[RPL];
    lane_matvec<FL, RPL, BS>(LTs, xb + grp * RPL * BS, f, y);      // y = L^{-1} b
#pragma unroll
    for (int q = 0; q < RPL; ++q) yb[(grp * RPL + q) * BS + f] = y[q];
    __syncthreads();
    double xn[RPL];
    lane_matvec<FL, RPL, BS>(Ls, yb + grp * RPL * BS, f, xn);      // x = L^{-T} y
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      if (done[q]) continue;
      const double v = xn[q] - u[q];
      const double hn = (v > 0.0) ? v : 0.0;
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
    if (tid < 6) {
      const double sum = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
      a.resid_part[(int64_t)blockIdx.x * 8 + tid] = sum;
    }
    if (tid == 6 || tid == 7) a.resid_part[(int64_t)blockIdx.x * 8 + tid] = 0.0;
  }
  // Gram partial of this block's rows (of the stored factor values), rows in order
  {
    double* hs = xb;  // [RPB][BS]
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
    double acc[NBT][NBT];
    float accf[NBT][NBT];
#pragma unroll
    for (int p = 0; p < NBT; ++p)
#pragma unroll
      for (int q = 0; q < NBT; ++q) {
        acc[p][q] = 0.0;
        accf[p][q] = 0.f;
      }
    for (int r2 = 0; r2 < nrow; ++r2) {
      double vi[NBT], vj[NBT];
#pragma unroll
      for (int p = 0; p < NBT; ++p) {
        vi[p] = (ti + 16 * p < FL) ? hs[r2 * BS + ti + 16 * p] : 0.0;
        vj[p] = (tj + 16 * p < FL) ? hs[r2 * BS + tj + 16 * p] : 0.0;
      }
      if (a.gram_f32) {
#pragma unroll
        for (int p = 0; p < NBT; ++p)
#pragma unroll
          for (int q = 0; q < NBT; ++q) accf[p][q] += (float)vi[p] * (float)vj[q];
      } else {
#pragma unroll
        for (int p = 0; p < NBT; ++p)
#pragma unroll
          for (int q = 0; q < NBT; ++q) acc[p][q] += vi[p] * vj[q];
      }
    }
#pragma unroll
    for (int p = 0; p < NBT; ++p)
#pragma unroll
      for (int q = 0; q < NBT; ++q) {
        const int r = ti + 16 * p, c = tj + 16 * q;
        if (r < F && c < F)
          a.gram_part[(int64_t)blockIdx.x * F * F + r * F + c] = a.gram_f32 ? (double)accf[p][q] : acc[p][q];
      }
  }
}

template <typename HT, int FL>
static hipError_t inner_launch(const InnerK& k, int nblk, hipStream_t s) {
  const size_t lds = (size_t)(2 * FL * FL + 2 * inner_rows_per_block<FL>() * (FL + 1)) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_inner<HT, FL>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_inner<HT, FL>), dim3(nblk), dim3(256), lds, s, k);
  return hipGetLastError();
}

int inner_rows_per_block(int FL) {
  switch (FL) {
    case 4: return inner_rows_per_block<4>();
    case 8: return inner_rows_per_block<8>();
    case 16: return inner_rows_per_block<16>();
    case 32: return inner_rows_per_block<32>();
    default: return inner_rows_per_block<64>();
  }
}

template <typename HT>
static hipError_t inner_dispatch(const InnerK& k, int FL, int nblk, hipStream_t s) {
  switch (FL) {
    case 4: return inner_launch<HT, 4>(k, nblk, s);
    case 8: return inner_launch<HT, 8>(k, nblk, s);
    case 16: return inner_launch<HT, 16>(k, nblk, s);
    case 32: return inner_launch<HT, 32>(k, nblk, s);
    default: return inner_launch<HT, 64>(k, nblk, s);
  }
}

hipError_t launch_inner(const InnerArgs& ia, int nblk, hipStream_t s) {
  InnerK k;
  k.part = ia.part;
  k.part_f64 = ia.part_f64;
  k.pstride = ia.pstride;
  k.rowstride = ia.rowstride;
  k.nparts = ia.nparts;
  k.Wout = ia.Wout;
  k.H = ia.H;
  k.U = ia.U;
  k.Pout = ia.Pout;
  k.rows = ia.rows;
  k.F = ia.F;
  k.Linv = ia.Linv;
  k.rho = ia.rho;
  k.rescale = ia.rescale;
  k.T = ia.T;
  k.eps_abs = ia.eps_abs;
  k.eps_rel = ia.eps_rel;
  k.iters_out = ia.iters_out;
  k.gram_from_primal = ia.gram_from_primal;
  k.gram_f32 = ia.gram_f32;
  k.gram_part = ia.gram_part;
  k.resid_part = ia.resid_part;
  k.flag = ia.flag;
  if (ia.h_f64) return inner_dispatch<double>(k, ia.FL, nblk, s);
  return inner_dispatch<float>(k, ia.FL, nblk, s);
}

// ---------------------------------------------------------------- prepare

// Every block reduces a slice of the Gram partials of the mode just updated
// (fixed order over partials); the last block to finish (atomic ticket) forms
// G = Gram_a (*) Gram_b, picks rho, and factors G + rho I.
//
// Cholesky and the triangular inverse use 256 threads on a 16 x 16 grid, thread
// (ti,tj) owning elements (ti+16a, tj+16b) in registers; each elimination step
// broadcasts one column (or row) through LDS, one barrier per step.
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
  double* Linv;
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
};

// Totals of the 8 residual partial columns over nparts partials, grouped
// fixed order (32 groups of 256 threads); used by the prepare and statistics
// kernels so both give bitwise identical totals.
static __device__ void resid_totals(const double* __restrict__ part, int nparts,
                                    double* __restrict__ out) {
  __shared__ double rr[32][8];
  const int c = threadIdx.x & 7, pg = threadIdx.x >> 3;
  rr[pg][c] = group_partial(part + c, 8, nparts, pg, 32);
  __syncthreads();
  if (threadIdx.x < 8) {
    double t = rr[0][threadIdx.x];
    for (int q = 1; q < 32; ++q) t += rr[q][threadIdx.x];
    out[threadIdx.x] = t;
  }
  __syncthreads();
}

template <int NB>
__global__ __launch_bounds__(256) void k_prep(PrepK a) {
  const int F = a.F;
  const int tid = threadIdx.x;
  __shared__ int is_last;
  if (a.gram_part) {
    // grouped fixed-order reduction (the same order as launch_reduce_partials
    // with 4 groups): block b reduces entries b*64 .. b*64+63
    __shared__ double gred[4][64];
    const int nent = F * F;
    const int el = tid & 63, pg = tid >> 6;
    for (int e0 = blockIdx.x * 64; e0 < nent; e0 += gridDim.x * 64) {
      const int e = e0 + el;
      gred[pg][el] = (e < nent) ? group_partial(a.gram_part + e, nent, a.nparts, pg, 4) : 0.0;
      __syncthreads();
      if (pg == 0 && e < nent) a.gram_dst[e] = ((gred[0][el] + gred[1][el]) + gred[2][el]) + gred[3][el];
      __syncthreads();
    }
    if (blockIdx.x == 0) resid_totals(a.resid_part, a.nparts, a.resid_dst);
    __threadfence();
    __syncthreads();
    if (tid == 0) {
      const unsigned ticket = atomicAdd(a.counter, 1u);
      is_last = (ticket == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    if (tid == 0) {
      *a.counter = 0u;
      if (a.fresh_dst) *a.fresh_dst = 1;
    }
  } else if (blockIdx.x != 0) {
    return;
  }

  __shared__ double Gs[64 * 65];
  __shared__ double rowbuf[2][128];
  __shared__ double colbuf[2][64];
  __shared__ double sred[256];
  __shared__ double rho_sh;
  __shared__ int bad_sh;

  {
    double ga[NB * NB], gb[NB * NB];
#pragma unroll
    for (int q = 0; q < NB * NB; ++q) {
      const int e = tid + 256 * q;
      ga[q] = (e < F * F) ? a.gram_a[e] : 0.0;
      gb[q] = (e < F * F) ? a.gram_b[e] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NB * NB; ++q) {
      const int e = tid + 256 * q;
      if (e < F * F) {
        const int r = e / F, c = e - r * F;
        const double gv = ga[q] * gb[q];
        Gs[r * 65 + c] = gv;
        if (a.G_out) a.G_out[e] = gv;
      }
    }
  }
  if (tid == 0) {
    bad_sh = 0;
    if (a.taken) *a.taken = 0;
  }
  __syncthreads();

  // penalty
  if (tid == 0) {
    const double rho_prev = a.rho_state[0];
    double rho;
    if (a.policy == 0) {
      double tr = 0.0;
#pragma unroll 8
      for (int f = 0; f < F; ++f) tr += Gs[f * 65 + f];
      rho = tr / F;
      if (!(rho > 0.0) || !isfinite(rho)) rho = a.rho0;
    } else if (a.policy == 1) {
      rho = a.rho0;
    } else {
      rho = rho_prev > 0.0 ? rho_prev : a.rho0;
      if (a.fresh_mode && *a.fresh_mode) {
        const double prim = sqrt(a.resid_mode[0]);
        const double dual = rho * sqrt(a.resid_mode[1]);
        if (prim > a.mu * dual) rho = rho * a.tau_incr;
        else if (dual > a.mu * prim) rho = rho / a.tau_decr;
        *a.fresh_mode = 0;
      }
    }
    a.rho_state[1] = (rho_prev > 0.0) ? rho_prev : rho;
    a.rho_state[0] = rho;
    rho_sh = rho;
  }
  __syncthreads();
  const double rho = rho_sh;

  // One elimination sweep over the augmented matrix [G + rho I | I]: row k is
  // divided by sqrt(a_kk) and a_ik / a_kk times the unscaled row k is
  // subtracted from every row i > k.  The left block becomes L^T and the
  // right block L^{-1} (L the Cholesky factor), i.e. the factorisation and
  // the triangular inverse in F steps.  Thread (ti,tj) owns rows ti+16a and
  // columns tj+16b of both blocks; row k and column k are broadcast through
  // LDS (double buffered, one barrier per step).
  const int ti = tid >> 4, tj = tid & 15;
  double rl[NB][NB], rr[NB][NB];
#pragma unroll
  for (int ia = 0; ia < NB; ++ia)
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) {
      const int i = ti + 16 * ia, j = tj + 16 * ib;
      double v;
      if (i < F && j < F) v = Gs[i * 65 + j] + ((i == j) ? rho : 0.0);
      else v = (i == j) ? 1.0 : 0.0;
      rl[ia][ib] = v;
      rr[ia][ib] = (i == j) ? 1.0 : 0.0;
    }
#pragma unroll
  for (int kb = 0; kb < NB; ++kb) {
    for (int kk = 0; kk < 16; ++kk) {
      const int k = 16 * kb + kk;
      if (k >= F) break;
      const int buf = k & 1;
      if (ti == kk) {
#pragma unroll
        for (int ib = 0; ib < NB; ++ib) {
          rowbuf[buf][tj + 16 * ib] = rl[kb][ib];
          rowbuf[buf][64 + tj + 16 * ib] = rr[kb][ib];
        }
      }
      if (tj == kk) {
#pragma unroll
        for (int ia = 0; ia < NB; ++ia) colbuf[buf][ti + 16 * ia] = rl[ia][kb];
      }
      __syncthreads();
      double akk = rowbuf[buf][k];
      if (!(akk > 0.0) || !isfinite(akk)) {
        if (tid == 0) bad_sh = 1;
        akk = 1.0;
      }
      const double inv = 1.0 / akk;
      const double sc = 1.0 / sqrt(akk);
      double rkl[NB], rkr[NB];
#pragma unroll
      for (int ib = 0; ib < NB; ++ib) {
        rkl[ib] = rowbuf[buf][tj + 16 * ib];
        rkr[ib] = rowbuf[buf][64 + tj + 16 * ib];
      }
#pragma unroll
      for (int ia = 0; ia < NB; ++ia) {
        const int i = ti + 16 * ia;
        if (i == k) {
#pragma unroll
          for (int ib = 0; ib < NB; ++ib) {
            rl[ia][ib] = rkl[ib] * sc;
            rr[ia][ib] = rkr[ib] * sc;
          }
        } else if (i > k && i < F) {
          const double m = colbuf[buf][i] * inv;
#pragma unroll
          for (int ib = 0; ib < NB; ++ib) {
            rl[ia][ib] -= m * rkl[ib];
            rr[ia][ib] -= m * rkr[ib];
          }
        }
      }
    }
  }
  __syncthreads();
  const bool bad = bad_sh != 0;
#pragma unroll
  for (int ia = 0; ia < NB; ++ia)
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) {
      const int i = ti + 16 * ia, j = tj + 16 * ib;
      if (i < F && j < F) a.Linv[i * F + j] = bad ? 0.0 : (j <= i ? rr[ia][ib] : 0.0);
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

hipError_t launch_prep(const PrepArgs& pa, int nblk, hipStream_t s) {
  PrepK k;
  k.F = pa.F;
  k.gram_part = pa.gram_part;
  k.nparts = pa.nparts;
  k.gram_dst = pa.gram_dst;
  k.resid_part = pa.resid_part;
  k.resid_dst = pa.resid_dst;
  k.fresh_dst = pa.fresh_dst;
  k.gram_a = pa.gram_a;
  k.gram_b = pa.gram_b;
  k.policy = pa.policy;
  k.rho0 = pa.rho0;
  k.mu = pa.mu;
  k.tau_incr = pa.tau_incr;
  k.tau_decr = pa.tau_decr;
  k.rho_state = pa.rho_state;
  k.resid_mode = pa.resid_mode;
  k.fresh_mode = pa.fresh_mode;
  k.Linv = pa.Linv;
  k.G_out = pa.G_out;
  k.taken = pa.taken;
  k.flag = pa.flag;
  k.counter = pa.counter;
  k.W3 = pa.W3;
  k.H3 = pa.H3;
  k.h_f64 = pa.h_f64;
  k.K = pa.K;
  k.gram_c = pa.gram_c;
  k.fit_out = pa.fit_out;
  const int grid = pa.gram_part ? nblk : 1;
  switch ((pa.F + 15) / 16) {
    case 1: hipLaunchKernelGGL(k_prep<1>, dim3(grid), dim3(256), 0, s, k); break;
    case 2: hipLaunchKernelGGL(k_prep<2>, dim3(grid), dim3(256), 0, s, k); break;
    case 3: hipLaunchKernelGGL(k_prep<3>, dim3(grid), dim3(256), 0, s, k); break;
    default: hipLaunchKernelGGL(k_prep<4>, dim3(grid), dim3(256), 0, s, k); break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- statistics

// Totals of the last mode's residual partials and Gram partials (without
// touching the solver state) and the cheap fit terms <W3,H3> and
// sum(G1 * G2 * G3): out[0..7] residual totals, out[8], out[9] fit terms.
__global__ __launch_bounds__(256) void k_finish(int F, const double* __restrict__ gram_part,
                                                const double* __restrict__ resid_part, int nparts,
                                                const double* __restrict__ g0,
                                                const double* __restrict__ g1,
                                                const double* __restrict__ W3, const void* H3,
                                                int h_f64, int64_t K, double* __restrict__ out) {
  __shared__ double sred[256];
  __shared__ double gred[4][64];
  const int tid = threadIdx.x;
  resid_totals(resid_part, nparts, out);
  double s1 = 0.0, s2 = 0.0;
  for (int64_t e = tid; e < K * F; e += 256) {
    const double hv = h_f64 ? reinterpret_cast<const double*>(H3)[e]
                            : (double)reinterpret_cast<const float*>(H3)[e];
    s1 += W3[e] * hv;
  }
  {
    const int el = tid & 63, pg = tid >> 6;
    for (int e0 = 0; e0 < F * F; e0 += 64) {
      const int e = e0 + el;
      gred[pg][el] = (e < F * F) ? group_partial(gram_part + e, (int64_t)F * F, nparts, pg, 4) : 0.0;
      __syncthreads();
      if (pg == 0 && e < F * F) {
        const double g2 = ((gred[0][el] + gred[1][el]) + gred[2][el]) + gred[3][el];
        s2 += g0[e] * g1[e] * g2;
      }
      __syncthreads();
    }
  }
  sred[tid] = s1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) sred[tid] += sred[tid + w];
    __syncthreads();
  }
  if (tid == 0) out[8] = sred[0];
  __syncthreads();
  sred[tid] = s2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) sred[tid] += sred[tid + w];
    __syncthreads();
  }
  if (tid == 0) out[9] = sred[0];
}

hipError_t launch_finish(int F, const double* gram_part, const double* resid_part, int nparts,
                         const double* g0, const double* g1, const double* W3, const void* H3,
                         int h_f64, int64_t K, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, F, gram_part, resid_part, nparts, g0, g1,
                     W3, H3, h_f64, K, out);
  return hipGetLastError();
}

// Fill n doubles with a value (used instead of memset nodes inside graphs).
__global__ __launch_bounds__(256) void k_fill(double* __restrict__ p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------- standalone Gram

// Partial p covers rows [p*rpp, (p+1)*rpp) and sums them in row order, the
// same partition and order the inner sweep uses for its fused Gram partials
// when rpp equals its rows per block, so both give bitwise identical Grams.
template <typename HT>
__global__ __launch_bounds__(256) void k_gram_part(const HT* __restrict__ H, int64_t rows, int F,
                                                   int64_t rpp, int gram_f32,
                                                   double* __restrict__ part) {
  __shared__ double hs[64 * 64];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * rpp, r1 = min(rows, r0 + rpp);
  double acc[16];
  float accf[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    acc[q] = 0.0;
    accf[q] = 0.f;
  }
  for (int64_t rb = r0; rb < r1; rb += 64) {
    const int nr = (int)min((int64_t)64, r1 - rb);
    __syncthreads();
    for (int e = tid; e < nr * F; e += 256) hs[e] = (double)H[rb * F + e];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + 256 * q;
      if (e < F * F) {
        const int r = e / F, c = e - r * F;
        if (gram_f32) {
          float sf = accf[q];
          for (int t = 0; t < nr; ++t) sf += (float)hs[t * F + r] * (float)hs[t * F + c];
          accf[q] = sf;
        } else {
          double sd = acc[q];
          for (int t = 0; t < nr; ++t) sd += hs[t * F + r] * hs[t * F + c];
          acc[q] = sd;
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q;
    if (e < F * F) part[(int64_t)blockIdx.x * F * F + e] = gram_f32 ? (double)accf[q] : acc[q];
  }
}

hipError_t launch_gram_part(const void* H, int h_f64, int64_t rows, int F, int64_t rpp,
                            int gram_f32, double* part, hipStream_t s) {
  const int nparts = (int)((rows + rpp - 1) / rpp);
  if (h_f64)
    hipLaunchKernelGGL(k_gram_part<double>, dim3(nparts), dim3(256), 0, s, (const double*)H, rows,
                       F, rpp, gram_f32, part);
  else
    hipLaunchKernelGGL(k_gram_part<float>, dim3(nparts), dim3(256), 0, s, (const float*)H, rows,
                       F, rpp, gram_f32, part);
  return hipGetLastError();
}

// ---------------------------------------------------------------- direct fit

// ||X - [H1,H2,H3]||^2 and ||X||^2 in FP64.  Block tile: 64 rows (i,j) x 64 k;
// thread (tr,tk) forms the model for rows tr+16a and columns tk+16b from
// Khatri-Rao rows and H3 rows staged in LDS.
template <typename XT, typename HT>
__global__ __launch_bounds__(256) void k_fit(const XT* __restrict__ X, int64_t IJ, int J, int K,
                                             int F, const HT* __restrict__ H1,
                                             const HT* __restrict__ H2, const HT* __restrict__ H3,
                                             double* __restrict__ part) {
  __shared__ double KRs[64 * 65];
  __shared__ double H3s[64 * 65];
  __shared__ double red[2][256];
  const int tid = threadIdx.x, tr = tid >> 4, tk = tid & 15;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int k0 = blockIdx.y * 64;
  double se = 0.0, sx = 0.0;
  // F <= 64: one staging round holds the whole rank
  for (int e = tid; e < 64 * 64; e += 256) {
    const int rr = e >> 6, f = e & 63;
    const int64_t r = r0 + rr;
    double v = 0.0, w = 0.0;
    if (f < F) {
      if (r < IJ) {
        const int64_t i = r / J, j = r - i * J;
        v = (double)H1[i * F + f] * (double)H2[j * F + f];
      }
      if (k0 + rr < K) w = (double)H3[(int64_t)(k0 + rr) * F + f];
    }
    KRs[rr * 65 + f] = v;
    H3s[rr * 65 + f] = w;
  }
  __syncthreads();
  double m[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) m[a][b] = 0.0;
  for (int f = 0; f < F; ++f) {
    double ka[4], hb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) ka[a] = KRs[(tr + 16 * a) * 65 + f];
#pragma unroll
    for (int b = 0; b < 4; ++b) hb[b] = H3s[(tk + 16 * b) * 65 + f];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) m[a][b] += ka[a] * hb[b];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t r = r0 + tr + 16 * a;
      const int k = k0 + tk + 16 * b;
      if (r < IJ && k < K) {
        const double xv = (double)X[r * K + k];
        const double e = xv - m[a][b];
        se += e * e;
        sx += xv * xv;
      }
    }
  red[0][tid] = se;
  red[1][tid] = sx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      red[0][tid] += red[0][tid + w];
      red[1][tid] += red[1][tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    part[2 * b] = red[0][0];
    part[2 * b + 1] = red[1][0];
  }
}

__global__ __launch_bounds__(256) void k_fit_sum(const double* __restrict__ part, int64_t nparts,
                                                 double* __restrict__ out) {
  __shared__ double red[2][256];
  double a = 0.0, b = 0.0;
  for (int64_t p = threadIdx.x; p < nparts; p += 256) {
    a += part[2 * p];
    b += part[2 * p + 1];
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0][0];
    out[1] = red[1][0];
  }
}

int fit_parts(const Plan& p) {
  const int64_t gx = (p.I * p.J + 63) / 64, gy = (p.K + 63) / 64;
  return (int)(gx * gy);
}

hipError_t launch_fit(const Plan& p, const void* X, int x_f64, const void* H1, const void* H2,
                      const void* H3, int h_f64, double* part, double* out, hipStream_t s,
                      int* nparts_out) {
  const int64_t gx = (p.I * p.J + 63) / 64, gy = (p.K + 63) / 64;
  dim3 grid((unsigned)gx, (unsigned)gy);
  const int64_t IJ = p.I * p.J;
  if (x_f64 && h_f64)
    hipLaunchKernelGGL((k_fit<double, double>), grid, dim3(256), 0, s, (const double*)X, IJ,
                       (int)p.J, (int)p.K, p.F, (const double*)H1, (const double*)H2,
                       (const double*)H3, part);
  else if (!x_f64 && !h_f64)
    hipLaunchKernelGGL((k_fit<float, float>), grid, dim3(256), 0, s, (const float*)X, IJ, (int)p.J,
                       (int)p.K, p.F, (const float*)H1, (const float*)H2, (const float*)H3, part);
  else
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fit_sum, dim3(1), dim3(256), 0, s, part, gx * gy, out);
  if (nparts_out) *nparts_out = (int)(gx * gy);
  return hipGetLastError();
}

}  // namespace ntf
