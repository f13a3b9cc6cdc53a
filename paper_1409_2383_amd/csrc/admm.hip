// ADMoM kernels for gfx950: the F x F system (Gram Hadamard product, penalty,
// FP64 inverse of G + rho I) and the fused row-wise inner sweep (the solve as
// a mat-vec with that inverse, projection, dual update, residuals, Gram partial),
// plus the standalone Gram and direct-fit kernels.
//
// One mode update (Section IV, eq. ADMM_NTF_ALS_C with eq. ADMoM_NTF) is
//   prep:  G = Gram_a (*) Gram_b,  rho,  Ginv = (G + rho I)^{-1} (block Gauss-Jordan)
//   inner: per row, T times:  b = w + rho (h + u);  ht = Ginv b;
//                             v = ht - u;  h = max(0, v);  u = h - v.
// The system matrix is common to all rows (Appendix B), so it is factored
// once per mode update; the rows are then independent.
#include "admm_body.h"
#include "ntf_launch.h"

namespace ntf {

// ---------------------------------------------------------------- inner sweep

template <typename HT, int FL>
__global__ __launch_bounds__(256) void k_inner(InnerK a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  inner_body<HT, FL>(a, (int64_t)blockIdx.x, smem_raw, (int)threadIdx.x);
}

// Register form of the inner sweep for 33 <= F <= 64 (FL = 64), used when
// no Gram partial is fused and the projection is row-wise: one row per wave
// (the same rows per block, 4, as k_inner at FL = 64), lane f holding column f
// of Ginv (= row f, Ginv is symmetric) in 64 FP64 registers.  The right-hand
// side of the row is read from its lanes with lane reads, so an inner
// iteration touches neither LDS nor a barrier; the mat-vec keeps four
// interleaved partial sums (g = 0 mod 4, 1 mod 4, ...) to shorten the
// dependent FMA chain.  Loads, projections, stop test, stores and residual
// partials are those of inner_body.
template <typename HT>
__global__ __launch_bounds__(256) void k_inner_reg64(InnerK a) {
  const int tid = threadIdx.x, f = tid & 63, wave = tid >> 6;
  const int F = a.F;
  const int64_t bid = blockIdx.x;
  const int64_t row = bid * 4 + wave;
  const bool act = (row < a.rows) && (f < F);
  __shared__ double red[4][8];
  double gc[64];
#pragma unroll
  for (int r = 0; r < 64; ++r) gc[r] = (r < F && f < F) ? a.Ginv[r * F + f] : 0.0;
  const double rho = a.rho[0];
  const double uscale = (a.rescale && a.rho[1] > 0.0) ? a.rho[1] / rho : 1.0;
  const double g1f = (a.proj == 2 && f < F) ? a.Ginv[F * F + f] : 0.0;
  const double inv_1g1 = (a.proj == 2) ? 1.0 / a.Ginv[F * F + F] : 0.0;
  double w = 0.0, h = 0.0, u = 0.0, x = 0.0;
  if (act) {
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
    w = sw;
    if (a.Wout) a.Wout[row * F + f] = sw;
    h = (double)reinterpret_cast<const HT*>(a.H)[row * F + f];
    u = (double)reinterpret_cast<const HT*>(a.U)[row * F + f] * uscale;
  }
  const double h0 = h;
  bool done = row >= a.rows;
  int iters = 0;
  const bool early = (a.eps_abs > 0.0) || (a.eps_rel > 0.0);
  const double sqF = sqrt((double)F);
  for (int t = 0; t < a.T && !done; ++t) {   // (done is uniform over the wave)
    const double b = act ? w + rho * (h + u) : 0.0;
    // (lane reads in batches of 16 into distinct scalar registers: one pair
    // reused for every lane read serialises each FMA behind its read)
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r0 = 0; r0 < 64; r0 += 16) {
      double bb[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) bb[k] = lane_value_d(b, r0 + k);
#pragma unroll
      for (int k = 0; k < 16; ++k) s4[k & 3] += gc[r0 + k] * bb[k];
    }
    double xn = (s4[0] + s4[1]) + (s4[2] + s4[3]);   // x = (G + rho I)^{-1} b
    if (a.proj == 2) {
      const double sx = group_sum(xn, 64);
      xn -= g1f * ((sx - 1.0) * inv_1g1);
    }
    const double v = xn - u;
    const double hn = (a.proj == 1) ? fmin(fmax(v, a.lo), a.hi) : ((v > 0.0) ? v : 0.0);
    const double un = hn - v;
    const double dh = hn - h;
    h = act ? hn : 0.0;
    u = act ? un : 0.0;
    x = act ? xn : 0.0;
    ++iters;
    if (early) {
      const double sp = group_sum((h - x) * (h - x), 64);
      const double sx = group_sum(x * x, 64);
      const double sh = group_sum(h * h, 64);
      const double sd = group_sum(act ? dh * dh : 0.0, 64);
      const double su = group_sum(u * u, 64);
      const double tol_p = sqF * a.eps_abs + a.eps_rel * fmax(sqrt(sx), sqrt(sh));
      const double tol_d = sqF * a.eps_abs + a.eps_rel * rho * sqrt(su);
      if (sqrt(sp) <= tol_p && rho * sqrt(sd) <= tol_d) done = true;
    }
  }
  double qs[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (act) {
    if (!isfinite(x) || !isfinite(w)) atomicOr(a.flag, 1);
    reinterpret_cast<HT*>(a.H)[row * F + f] = (HT)h;
    reinterpret_cast<HT*>(a.U)[row * F + f] = (HT)u;
    if (a.Pout) reinterpret_cast<HT*>(a.Pout)[row * F + f] = (HT)x;
    if (a.iters_out && f == 0) a.iters_out[row] = iters;
    const double hv = (double)(HT)h, xv = (double)(HT)x, uv = (double)(HT)u;
    qs[0] = (hv - xv) * (hv - xv);
    qs[1] = (hv - h0) * (hv - h0);
    qs[2] = hv * hv;
    qs[3] = xv * xv;
    qs[4] = uv * uv;
    if (f == 0) qs[5] = (double)iters;
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double sum = group_sum(qs[k], 64);
    if (f == 0) red[wave][k] = sum;
  }
  __syncthreads();
  if (a.resid_part) {
    if (tid < 6) a.resid_part[bid * 8 + tid] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
    if (tid == 6 || tid == 7) a.resid_part[bid * 8 + tid] = 0.0;
  }
}

template <typename HT, int FL>
static hipError_t inner_launch(const InnerK& k, int nblk, hipStream_t s) {
  if constexpr (FL == 64) {
    if (!k.gram_part && (k.proj == 0 || k.proj == 1 || k.proj == 2)) {
      hipLaunchKernelGGL((k_inner_reg64<HT>), dim3(nblk), dim3(256), 0, s, k);
      return hipGetLastError();
    }
  }
  const size_t lds = (size_t)(FL * FL + 2 * inner_rows_per_block<FL>() * (FL + 1)) * sizeof(double);
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
  k.Ginv = ia.Ginv;
  k.proj = ia.proj;
  k.lo = ia.lo;
  k.hi = ia.hi;
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
  k.dv = ia.dv;
  k.dx = ia.dx;
  k.dh0 = ia.dh0;
  if (ia.h_f64) return inner_dispatch<double>(k, ia.FL, nblk, s);
  return inner_dispatch<float>(k, ia.FL, nblk, s);
}

// ---------------------------------------------------------------- prepare

// Every block forms (or reduces) a slice of the Gram of the mode just updated
// (fixed order); the last block to finish (atomic ticket) forms G = Gram_a (*)
// Gram_b, picks rho, and inverts G + rho I (prep_body).
//
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

template <typename HT, int NB>
__device__ __forceinline__ void gram_rows_mfma(const HT* __restrict__ H, int64_t r0, int64_t r1, int F,
                               double* __restrict__ part, double* lds);

template <int NB>
__global__ __launch_bounds__(256) void k_prep(PrepK a) {
  const int F = a.F;
  const int tid = threadIdx.x;
  __shared__ int is_last;
  __shared__ double prep_lds[kPrepLdsDoubles];
  static_assert(kPrepLdsDoubles >= kGramLdsDoubles, "the Gram stage borrows the prepare LDS");
  // the inputs that do not depend on this kernel's Gram, loaded before it
  PrepIn<NB> in;
  prep_load_b(a, tid, in);
  bool have_a = false;
  if (a.gram_h) {
    // direct Gram: block b sums rows [b rpp, (b+1) rpp) of the updated factor
    // in FP64 on the matrix cores; the last block to finish reduces the
    // partials (4 fixed groups)
    const int64_t r0 = (int64_t)blockIdx.x * a.gram_rpp;
    const int64_t r1 = min(a.gram_rows, r0 + a.gram_rpp);
    double* part = a.gram_scratch + (int64_t)blockIdx.x * F * F;
    // (the block past the partials sums the residual partials meanwhile)
    if (blockIdx.x == a.gram_nb)
      resid_totals(a.resid_part, a.nparts, a.resid_dst);
    else if (a.h_f64)
      gram_rows_mfma<double, NB>(reinterpret_cast<const double*>(a.gram_h), r0, r1, F, part, prep_lds);
    else
      gram_rows_mfma<float, NB>(reinterpret_cast<const float*>(a.gram_h), r0, r1, F, part, prep_lds);
    // release before the ticket, acquire by the last block after it: the
    // partials written here are visible to that block's loads (a full fence
    // on both sides also wrote back the last block's L2 and invalidated the
    // others': 3-4 us more on the mode-2 prepare step)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) {
      const unsigned ticket = atomicAdd(a.counter, 1u);
      is_last = (ticket == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (!is_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (tid == 0) {
      *a.counter = 0u;
      if (a.fresh_dst) *a.fresh_dst = 1;
    }
    // group g sums partials g, g+4, ... in order, the four group sums are
    // added in order (the order of the 4-group reduction kernel); each thread
    // reduces the entries of its prep_body tile, the loads of four partials
    // for all of them going out together
    const int nent = F * F;
    double gs[4][NB * NB];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int k = 0; k < NB * NB; ++k) gs[g][k] = 0.0;
    for (int p0 = 0; p0 < a.gram_nb; p0 += 4) {
      double v[4][NB * NB];
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int k = 0; k < NB * NB; ++k) {
          const int e = prep_entry<NB>(F, tid, k);
          v[g][k] = (p0 + g < a.gram_nb && e >= 0) ? a.gram_scratch[(int64_t)(p0 + g) * nent + e] : 0.0;
        }
#pragma unroll
      for (int g = 0; g < 4; ++g)
        if (p0 + g < a.gram_nb) {
#pragma unroll
          for (int k = 0; k < NB * NB; ++k) gs[g][k] += v[g][k];
        }
    }
#pragma unroll
    for (int k = 0; k < NB * NB; ++k) {
      const int e = prep_entry<NB>(F, tid, k);
      const double v = ((gs[0][k] + gs[1][k]) + gs[2][k]) + gs[3][k];
      if (e >= 0) a.gram_dst[e] = v;
      in.ga[k] = (e >= 0) ? v : 0.0;
    }
    have_a = (a.gram_a == a.gram_dst);
    __threadfence_block();
    __syncthreads();
  } else if (a.gram_part) {
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
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // (as above)
    __syncthreads();
    if (tid == 0) {
      const unsigned ticket = atomicAdd(a.counter, 1u);
      is_last = (ticket == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (!is_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (tid == 0) {
      *a.counter = 0u;
      if (a.fresh_dst) *a.fresh_dst = 1;
    }
  } else if (blockIdx.x != 0) {
    return;
  }
  if (!have_a) prep_load_a(a, tid, in);
  prep_body<NB>(a, prep_lds, tid, in);
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
  k.Ginv = pa.Ginv;
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
  k.gram_h = pa.gram_h;
  k.gram_rows = pa.gram_rows;
  k.gram_rpp = pa.gram_rpp;
  k.gram_nb = pa.gram_nb;
  k.gram_scratch = pa.gram_scratch;
  const int grid = pa.gram_h ? pa.gram_nb + 1 : pa.gram_part ? nblk : 1;
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
                                                int gram_nparts,
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
      gred[pg][el] = (e < F * F) ? group_partial(gram_part + e, (int64_t)F * F, gram_nparts, pg, 4) : 0.0;
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

hipError_t launch_finish(int F, const double* gram_part, int gram_nparts, const double* resid_part,
                         int nparts, const double* g0, const double* g1, const double* W3,
                         const void* H3, int h_f64, int64_t K, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, F, gram_part, gram_nparts, resid_part, nparts,
                     g0, g1, W3, H3, h_f64, K, out);
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
// One partial: rows [r0, r1) of H into part[0 .. F*F), each entry summed in
// row order (256 threads; hs holds 64*64 doubles of LDS).  Thread (ti,tj)
// owns entries (ti+16a, tj+16b): per row eight LDS reads feed sixteen
// independent products.
template <typename HT>
__device__ void gram_rows(const HT* __restrict__ H, int64_t r0, int64_t r1, int F, int gram_f32,
                          double* __restrict__ part, double* hs) {
  const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  double acc[4][4];
  float accf[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc[p][q] = 0.0;
      accf[p][q] = 0.f;
    }
  // the next 64-row chunk is loaded into registers (16 values per thread,
  // all in flight at once) while the current one is summed: the factor was
  // just written on other XCDs, so each load is a full memory round trip
  double nx[16];
  auto load_chunk = [&](int64_t rb) {
    const int n = (int)min((int64_t)64, r1 - rb) * F;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + 256 * q;
      nx[q] = (e < n) ? (double)H[rb * F + e] : 0.0;
    }
  };
  if (r0 < r1) load_chunk(r0);
  for (int64_t rb = r0; rb < r1; rb += 64) {
    const int nr = (int)min((int64_t)64, r1 - rb);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + 256 * q;
      if (e < nr * F) hs[e] = nx[q];
    }
    __syncthreads();
    // (issued after the barrier, which would otherwise wait for them: they
    // arrive during the sums below)
    if (rb + 64 < r1) load_chunk(rb + 64);
    // (columns past F read other rows' values into entries that are never
    // stored; every index stays inside the 64 x 64 buffer)
    if (gram_f32) {
#pragma unroll 4
      for (int t = 0; t < nr; ++t) {
        float vi[4], vj[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          vi[p] = (float)hs[t * F + ti + 16 * p];
          vj[p] = (float)hs[t * F + tj + 16 * p];
        }
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int q = 0; q < 4; ++q) accf[p][q] += vi[p] * vj[q];
      }
    } else {
#pragma unroll 4
      for (int t = 0; t < nr; ++t) {
        double vi[4], vj[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          vi[p] = hs[t * F + ti + 16 * p];
          vj[p] = hs[t * F + tj + 16 * p];
        }
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[p][q] += vi[p] * vj[q];
      }
    }
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = ti + 16 * p, c = tj + 16 * q;
      if (r < F && c < F) part[r * F + c] = gram_f32 ? (double)accf[p][q] : acc[p][q];
    }
}

template <typename HT>
__global__ __launch_bounds__(256) void k_gram_part(const HT* __restrict__ H, int64_t rows, int F,
                                                   int64_t rpp, int gram_f32,
                                                   double* __restrict__ part) {
  __shared__ double hs[64 * 64];
  const int64_t r0 = (int64_t)blockIdx.x * rpp, r1 = min(rows, r0 + rpp);
  gram_rows<HT>(H, r0, r1, F, gram_f32, part + (int64_t)blockIdx.x * F * F, hs);
}

// One partial by the FP64 matrix cores: rows [r0, r1) of H into part[0 ..
// F*F), NB = ceil(F / 16).  Wave w sums a quarter of the rows (in steps of 4
// rows, 16 steps of loads in flight) into every 16 x 16 tile (I, J), I <= J,
// one v_mfma_f64_16x16x4 per tile and step with operands read straight from H
// (lane l: row l / 16 of the step, column 16 X + l % 16 of tile row / column
// X; products of FP32 factors are exact in FP64); the four waves' tiles are
// then added in wave order through LDS (kGramLdsDoubles) and written to both
// triangles (the diagonal tiles from their upper half), so the partial is
// exactly symmetric.  Used by the prepare step's direct Gram and by every
// Gram of the dense path that must match it bitwise.
template <typename HT, int NB>
__device__ __forceinline__ void gram_rows_mfma(const HT* __restrict__ H, int64_t r0, int64_t r1, int F,
                               double* __restrict__ part, double* lds) {
  constexpr int NT = NB * (NB + 1) / 2;   // tiles I <= J, row-major
  constexpr int es = (int)sizeof(HT);
  constexpr int U = 16;                   // steps of loads in flight
  constexpr int G = 4;                    // tiles per round of the wave sum
  static_assert(4 * G * 4 * 64 <= kGramLdsDoubles, "LDS of the wave sum");
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int64_t nsteps = (r1 > r0) ? (r1 - r0 + 3) / 4 : 0;
  const int64_t per = (nsteps + 3) / 4;
  const int64_t ws0 = min(nsteps, wave * per), ws1 = min(nsteps, ws0 + per);
  int off[NB];
#pragma unroll
  for (int X = 0; X < NB; ++X) {
    const int c = 16 * X + li;
    off[X] = (c < F) ? (lk * F + c) * es : kBufferOOB;
  }
  f64x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int64_t sb = ws0; sb < ws1; sb += U) {
    const int ns = (int)min((int64_t)U, ws1 - sb);
    const int64_t rb = r0 + 4 * sb;
    const int nr = (int)min((int64_t)(4 * ns), r1 - rb);
    const __amdgpu_buffer_rsrc_t rs = uniform_rsrc(H + rb * F, nr * F * es);
    HT v[U][NB];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int X = 0; X < NB; ++X) {
        if constexpr (sizeof(HT) == 8)
          v[u][X] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off[X], u * 4 * F * es, 0));
        else
          v[u][X] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, off[X], u * 4 * F * es, 0));
      }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (u < ns) {
#pragma unroll
        for (int I = 0; I < NB; ++I)
#pragma unroll
          for (int J = I; J < NB; ++J) {
            const int t = I * NB - I * (I - 1) / 2 + (J - I);
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)v[u][I], (double)v[u][J], acc[t], 0, 0, 0);
          }
      }
    }
  }
  // ((w0 + w1) + w2) + w3 per entry, G tiles per round: every wave stores its
  // tiles, then wave w adds up tile g0 + w.  D[i][j] of a tile sits in lane
  // j + 16 (i % 4), register i / 4.
#pragma unroll
  for (int g0 = 0; g0 < NT; g0 += G) {
    __syncthreads();
#pragma unroll
    for (int t = g0; t < g0 + G && t < NT; ++t)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) lds[((wave * G + (t - g0)) * 4 + rr) * 64 + lane] = acc[t][rr];
    __syncthreads();
    const int t = g0 + wave;
    if (t < NT) {
      int I = 0, rem = t;
      while (rem >= NB - I) {
        rem -= NB - I;
        ++I;
      }
      const int J = I + rem;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const double* L = lds + ((t - g0) * 4 + rr) * 64 + lane;
        const double vsum = ((L[0] + L[G * 4 * 64]) + L[2 * G * 4 * 64]) + L[3 * G * 4 * 64];
        const int i = 4 * rr + lk, j = li;
        const int gi = 16 * I + i, gj = 16 * J + j;
        if (gi < F && gj < F && (I != J || i <= j)) {
          part[gi * F + gj] = vsum;
          part[gj * F + gi] = vsum;
        }
      }
    }
  }
  __syncthreads();   // (the caller reuses the LDS)
}

template <typename HT, int NB>
__global__ __launch_bounds__(256) void k_gram_mfma(const HT* __restrict__ H, int64_t rows, int F,
                                                   int64_t rpp, double* __restrict__ part) {
  __shared__ double lds[kGramLdsDoubles];
  const int64_t r0 = (int64_t)blockIdx.x * rpp, r1 = min(rows, r0 + rpp);
  gram_rows_mfma<HT, NB>(H, r0, r1, F, part + (int64_t)blockIdx.x * F * F, lds);
}

template <typename HT>
static void launch_gram_mfma_t(const HT* H, int64_t rows, int F, int64_t rpp, double* part, int nparts,
                               hipStream_t s) {
  switch ((F + 15) / 16) {
    case 1: hipLaunchKernelGGL((k_gram_mfma<HT, 1>), dim3(nparts), dim3(256), 0, s, H, rows, F, rpp, part); break;
    case 2: hipLaunchKernelGGL((k_gram_mfma<HT, 2>), dim3(nparts), dim3(256), 0, s, H, rows, F, rpp, part); break;
    case 3: hipLaunchKernelGGL((k_gram_mfma<HT, 3>), dim3(nparts), dim3(256), 0, s, H, rows, F, rpp, part); break;
    default: hipLaunchKernelGGL((k_gram_mfma<HT, 4>), dim3(nparts), dim3(256), 0, s, H, rows, F, rpp, part); break;
  }
}

hipError_t launch_gram_direct(const void* H, int h_f64, int64_t rows, int F, int64_t rpp,
                              double* part, hipStream_t s) {
  const int nparts = (int)((rows + rpp - 1) / rpp);
  if (h_f64) launch_gram_mfma_t((const double*)H, rows, F, rpp, part, nparts, s);
  else launch_gram_mfma_t((const float*)H, rows, F, rpp, part, nparts, s);
  return hipGetLastError();
}

void gram_split(int64_t rows, int64_t* rpp, int* nb) {
  // partials of whole 64-row chunks: at most 4 chunks (256 rows, one round of
  // loads per wave) each while that gives at most 16 partials, then more.
  // Up to 4 partials the last block of the prepare step reads them back in
  // one round of loads (they were written on other XCDs: every load is a
  // memory round trip)
  const int64_t chunks = (rows + 63) / 64;
  const int64_t per = std::max<int64_t>((chunks + 15) / 16, std::min<int64_t>(4, (chunks + 3) / 4));
  *rpp = per * 64;
  *nb = (int)((rows + *rpp - 1) / *rpp);
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
