// Batched ADMoM NTF for gfx950: one persistent kernel runs one outer
// iteration (eq. ADMoM_NTF, modes in the Gauss-Seidel order of eq.
// ADMM_NTF_ALS_C) of every problem of a batch of independent tensors of
// uneven shapes.
//
// Work items (problem, kind, index) sit in one global list; blocks take
// tickets from an atomic counter and run the item of their ticket.  Per
// problem and outer iteration the kinds depend on each other as
//
//   P1 (slab groups) --------------+--> IN1 (row blocks) --+--> M2 --> IN2 --+--> P3 --> IN3
//   PREP1 -------------------------+                       +--> PREP2 ---^   +--> PREP3 --^
//
// (PREPn: G_n = Gram (*) Gram of the other two modes, rho, (G_n + rho I)^{-1}; INn: the
// fused inner sweep of mode n; P1: T = X x_3 H3 and the W1 rows; M2: W2
// from T and the new H1; P3: W3 partials from the new H1 and H2).  The list
// is sorted so that every item depends only on items with smaller tickets,
// and a block waits (thread 0 polls the problem's completion counters) only
// on such items.  A waiting block's dependencies are therefore held by
// running blocks or already done, and the lowest held ticket never waits:
// the kernel cannot deadlock, whatever the number of resident blocks.  Every
// wait is also bounded (flag bit 8 when a bound is hit).
//
// MTTKRP arithmetic: BF16 operands, FP32 MFMA accumulation, the power-of-two
// slab scale of X applied to each slab's FP32 result.
//   P1: T[i,j,:] = s_i sum_k Xq[i,j,k] bf16(H3[k,:]);  W1[i,:] = sum_j H2[j,:] * T[i,j,:]
//   M2: W2[j,:]  = sum_i H1[i,:] * T[i,j,:]                      (FP64 accumulation)
//   P3: W3[k,:]  = sum_i s_i H1[i,:] * (sum_j Xq[i,j,k] bf16(H2[j,:]))
// P3 reads a second BF16 copy with j fastest ([I][K][Jp]), so that its
// contraction is contiguous like P1's; the Khatri-Rao factor of mode 3 is
// applied in factored form (the H1 row scales each slab's result), so no
// Khatri-Rao row is formed at all.
#include "admm_body.h"
#include "batch.h"
#include "ntf_launch.h"

#include <algorithm>

namespace ntf {

static __host__ __device__ __forceinline__ int rup_i(int x, int a) { return (x + a - 1) / a * a; }

// Columns of j per chunk of the pass-3 item's H2 tiles (a multiple of 64).
constexpr int kP3ChunkCols = 256;

// Problem descriptors are read-only for a whole launch: the kernel reads them
// through the constant address space (scalar loads into scalar registers),
// by reference, never as a local copy (a copy indexed at run time would live
// in scratch memory).
typedef __attribute__((address_space(4))) const BProb ConstProb;

size_t batch_lds_p1(const BProb& p) {
  const int FP = p.FT * 16, KCS = rup_i(p.Kp, 64) + 8;
  return (size_t)FP * KCS * 2 + (size_t)4 * p.spi1 * FP * 4;
}
size_t batch_lds_p3(const BProb& p) {
  // hi and lo tiles of a chunk of at most kP3Chunk columns of j
  const int FP = p.FT * 16, JCS = std::min(rup_i(p.Jp, 64), kP3ChunkCols) + 8;
  return (size_t)2 * FP * JCS * 2;
}
// The batched kernel runs the inner sweep with one row per lane group
// (256 / FL rows per block), which keeps its register budget within two
// resident blocks per compute unit; latency is hidden by the other items.
// At FL = 32 and 64 a lane group takes two rows (each LDS read of Ginv serves
// both, and a block step loads Ginv for twice the rows): the sweep is bound by
// LDS reads there (256-tensor batch 8.23 -> 7.87 ms per iteration with two
// rows at FL = 64, 7.75 ms with two at FL = 32 as well).
template <int FL>
static constexpr int batch_inner_rpl() { return FL >= 32 ? 2 : 1; }
int batch_inner_rows(int FL) { return (256 / FL) * (FL >= 32 ? 2 : 1); }
size_t batch_lds_inner(int FL) {
  return (size_t)(FL * FL + 2 * batch_inner_rows(FL) * (FL + 1)) * sizeof(double);
}
size_t batch_lds_prep() { return (size_t)kPrepLdsDoubles * sizeof(double); }

// ---------------------------------------------------------------- pass 1 item

// Slabs s0 .. s0+ns-1 of one problem.  H3^T (BF16) sits in LDS; each wave
// walks its 16*MT-row tiles (slab-major, tiles wave, wave+4, ...) as one
// continuous sequence of 64-element super steps with U steps of loads in
// flight, so its pipeline does not drain between tiles.  The two MFMAs of a
// super step contract its elements 0-31 and 32-63 (lane group g: 8g .. 8g+7
// of each half), so each 16-byte load instruction reads 64 contiguous bytes
// of 16 rows.
template <int FT, int MT>
__device__ __forceinline__ void p1_item(const ConstProb& P, int idx, unsigned char* lds, const int tid) {
  constexpr int FP = FT * 16;
  constexpr int R = 16 * MT;
  constexpr int U = 4;
  const int lane = tid & 63, wave = tid >> 6, n = lane & 15, g = lane >> 4;
  const int J = P.J, K = P.K, F = P.F, Kp = P.Kp;
  const int KC = rup_i(Kp, 64), KCS = KC + 8;
  __bf16* Cs = reinterpret_cast<__bf16*>(lds);
  const int s0 = idx * P.spi1;
  const int ns = min(P.I, s0 + P.spi1) - s0;
  float* w1p = reinterpret_cast<float*>(lds + (size_t)FP * KCS * 2);   // [4][ns][FP]
  const float* __restrict__ Hb = P.H[1];
  const float* __restrict__ Hc = P.H[2];
  const int nrg = (J + R - 1) / R;
  const int ntiles = ns * nrg;
  const int myt = ntiles > wave ? (ntiles - wave + 3) / 4 : 0;
  const int nsteps = KC / 64;
  const int total = myt * nsteps;
  // Loads go through a buffer resource per slab: rows j >= J lie past its
  // num_records and k >= Kp gets an offset past it, so both read as zeros,
  // and every path issues the same loads (the cursor stays on its last tile
  // past the wave's end and re-reads in-bounds data nothing consumes): the
  // wait before a step then covers that step's loads only.
  // The copy is k-grouped, Xr[i][Kp/8][J][8] (eight consecutive k innermost,
  // then j): lane (n, g) reads the 8 values k = kk .. kk+7 (kk = step column
  // + 8g) of row j as one 16-byte piece and the 16 rows of a tile lie
  // together, so a load instruction reads four runs of 256 bytes.  Rows
  // j >= J and columns k >= Kp take offsets with bit 31 set (past the
  // resource: zeros).
  int l_t = wave, l_kb = 0, l_sl = 0;
  const __bf16* l_slab = P.Xr;
  int l_j[MT];
  auto set_rows = [&](int t) {
    const int sl = t / nrg, rg = t - sl * nrg;
    l_sl = sl;
    l_slab = P.Xr + (int64_t)(s0 + sl) * J * Kp;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) l_j[mt] = rg * R + mt * 16 + n;
  };
  // each step's loads also bring its slab's scale (the tile epilogue then
  // reads it from a register instead of waiting on a load of its own)
  const __amdgpu_buffer_rsrc_t srs = uniform_rsrc(P.scale, P.I * 4);
  bf16x8 xv[U][2][MT];
  float as[U];
  auto load_next = [&](bf16x8 (&dst)[2][MT], float& sdst) {
    sdst = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(srs, (s0 + l_sl) * 4, 0, 0));
    const __amdgpu_buffer_rsrc_t rs = uniform_rsrc(l_slab, J * Kp * 2);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int kk = l_kb + 32 * h + 8 * g;
        const unsigned past = ((unsigned)(J - 1 - l_j[mt]) | (unsigned)(Kp - 1 - kk)) & 0x80000000u;
        const int off = (int)(((unsigned)((kk >> 3) * J + l_j[mt]) * 16u) | past);
        dst[h][mt] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
      }
    l_kb += 64;
    if (l_kb >= Kp) {
      l_kb = 0;
      l_t += 4;
      if (l_t < ntiles) set_rows(l_t);
    }
  };
  // the first U steps of tensor loads go out before H3^T is staged, so the
  // staging overlaps them
  if (total > 0) {
    set_rows(l_t);
#pragma unroll
    for (int u = 0; u < U; ++u) load_next(xv[u], as[u]);
  }
  for (int e = tid; e < KC * FP; e += 256) {
    const int kk = e / FP, f = e - kk * FP;
    const float v = (kk < K && f < F) ? Hc[(int64_t)kk * F + f] : 0.f;
    Cs[f * KCS + kk] = (__bf16)v;
  }
  for (int e = tid; e < 4 * ns * FP; e += 256) w1p[e] = 0.f;
  __syncthreads();

  if (total > 0) {
    f32x4 acc[MT][FT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int ft = 0; ft < FT; ++ft) acc[mt][ft] = f32x4{0.f, 0.f, 0.f, 0.f};
    float wrun[FT];
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) wrun[ft] = 0.f;
    int cur_sl = -1;
    auto flush = [&]() {
      if (cur_sl >= 0 && g == 0) {
#pragma unroll
        for (int ft = 0; ft < FT; ++ft) w1p[(wave * ns + cur_sl) * FP + ft * 16 + n] = wrun[ft];
      }
    };
    int c_t = wave, c_step = 0;
    const __bf16* cb = Cs + n * KCS + 8 * g;
    // H2 values of the current tile's epilogue, loaded when the tile starts
    // so that their latency hides behind the tile's MFMA steps
    // H2 values and T stores through resources too (rows past J, columns
    // past F: offsets past them, zeros in, stores dropped)
    float hbv[MT][FT][4];
    const __amdgpu_buffer_rsrc_t hrs = uniform_rsrc(Hb, J * F * 4);
    auto eoff = [&](int rg, int mt, int ft, int ii) {
      const int j = rg * R + mt * 16 + 4 * g + ii, f = ft * 16 + n;
      return (j < J && f < F) ? (j * F + f) * 4 : kBufferOOB;
    };
    auto load_hb = [&](int t) {
      const int rg = t - (t / nrg) * nrg;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int ft = 0; ft < FT; ++ft)
#pragma unroll
          for (int ii = 0; ii < 4; ++ii)
            hbv[mt][ft][ii] = __builtin_bit_cast(
                float, __builtin_amdgcn_raw_buffer_load_b32(hrs, eoff(rg, mt, ft, ii), 0, 0));
    };
    auto step = [&](int u, bool reload) {
          if (c_step == 0) load_hb(c_t);
#pragma unroll
          for (int ft = 0; ft < FT; ++ft) {
            const __bf16* cp = cb + ft * 16 * KCS + c_step * 64;
            const bf16x8 c0 = *reinterpret_cast<const bf16x8*>(cp);
            const bf16x8 c1 = *reinterpret_cast<const bf16x8*>(cp + 32);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt][ft] = mma_bf16(xv[u][0][mt], c0, acc[mt][ft]);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt][ft] = mma_bf16(xv[u][1][mt], c1, acc[mt][ft]);
          }
          const float sc = as[u];   // (read before the reload rewrites it)
          if (reload) load_next(xv[u], as[u]);
          if (++c_step == nsteps) {
            const int sl = c_t / nrg, rg = c_t - sl * nrg;
            const int i = s0 + sl;
            if (sl != cur_sl) {
              flush();
              cur_sl = sl;
#pragma unroll
              for (int ft = 0; ft < FT; ++ft) wrun[ft] = 0.f;
            }
            const __amdgpu_buffer_rsrc_t trs = uniform_rsrc(P.T + (int64_t)i * J * F, J * F * 4);
            float part[FT];
#pragma unroll
            for (int ft = 0; ft < FT; ++ft) part[ft] = 0.f;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
              for (int ft = 0; ft < FT; ++ft) {
#pragma unroll
                for (int ii = 0; ii < 4; ++ii) {
                  const float v = sc * acc[mt][ft][ii];
                  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), trs,
                                                        eoff(rg, mt, ft, ii), 0, 0);
                  part[ft] += hbv[mt][ft][ii] * v;
                }
                acc[mt][ft] = f32x4{0.f, 0.f, 0.f, 0.f};
              }
#pragma unroll
            for (int ft = 0; ft < FT; ++ft) {
              part[ft] += __shfl_xor(part[ft], 16);
              part[ft] += __shfl_xor(part[ft], 32);
              wrun[ft] += part[ft];
            }
            c_step = 0;
            c_t += 4;
          }
    };
    const int full = total - total % U;
    for (int s = 0; s < full; s += U) {
#pragma unroll
      for (int u = 0; u < U; ++u) step(u, true);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (full + u < total) step(u, false);
    flush();
  }
  __syncthreads();
  // W1 rows of this item's slabs: the four waves' partials in wave order
  for (int e = tid; e < ns * F; e += 256) {
    const int sl = e / F, f = e - sl * F;
    double w = 0.0;
#pragma unroll
    for (int wv = 0; wv < 4; ++wv) w += (double)w1p[(wv * ns + sl) * FP + f];
    P.W[0][(int64_t)(s0 + sl) * F + f] = w;
  }
}

// ---------------------------------------------------------------- pass 3 item

// Slabs s0 .. s0+ns-1 of one problem, from the j-fastest copy.  H2^T sits in
// LDS as two bfloat16 tiles, hi = bf16(B) and lo = bf16(B - hi) (one rounding
// of B shared by every slab would bias all slabs alike), for a chunk of
// kP3Chunk columns of j at a time.  Per chunk, each wave owns 16*MT-row groups
// of k (rg = wave, wave+4, ..) and, for each, streams the slabs of the item:
// the FP32 result of a slab is scaled by s_i * H1[i,:] and added to the
// group's total, which the first chunk stores into this item's partial of W3
// and every later chunk adds to it (same block, in chunk order).
constexpr int kP3Chunk = kP3ChunkCols;

template <int FT, int MT>
__device__ __forceinline__ void p3_item(const ConstProb& P, int idx, unsigned char* lds, const int tid) {
  constexpr int FP = FT * 16;
  constexpr int R = 16 * MT;
  constexpr int U = 4;
  const int lane = tid & 63, wave = tid >> 6, n = lane & 15, g = lane >> 4;
  const int J = P.J, K = P.K, F = P.F, Jp = P.Jp;
  const int JC = rup_i(Jp, 64);
  const int JCH = min(JC, kP3Chunk), JCS = JCH + 8;
  __bf16* Bs = reinterpret_cast<__bf16*>(lds);   // hi tile [FP][JCS], then the lo tile
  __bf16* Bl = Bs + FP * JCS;
  const float* __restrict__ Ha = P.H[0];
  const float* __restrict__ Hb = P.H[1];
  const int s0 = idx * P.spi3;
  const int ns = min(P.I, s0 + P.spi3) - s0;
  const int nrg = (K + R - 1) / R;
  const int myrg = nrg > wave ? (nrg - wave + 3) / 4 : 0;
  const int nchunk = (JC + JCH - 1) / JCH;
  const __amdgpu_buffer_rsrc_t ars = uniform_rsrc(Ha, P.I * F * 4);
  const __amdgpu_buffer_rsrc_t srs = uniform_rsrc(P.scale, P.I * 4);
  const int aof = lane < F ? lane * 4 : kBufferOOB;
  const __amdgpu_buffer_rsrc_t wrs = uniform_rsrc(P.W3p + (int64_t)idx * K * F, K * F * 4);

  for (int chk = 0; chk < nchunk; ++chk) {
    const int j0 = chk * JCH, jw = min(JCH, JC - j0);
    const int nsteps = jw / 64;
    const int total = myrg * ns * nsteps;

    // Loads through a buffer resource per slab of the j-grouped copy
    // Xg[i][Jp/8][K][8]: lane (n, g) reads the 8 values j = jj .. jj+7 (jj =
    // step column + 8g) of row k as one 16-byte piece, and the 16 rows of a
    // tile lie together, so a load instruction reads four runs of 256 bytes.
    // Rows k >= K and columns j >= Jp take offsets with bit 31 set (past the
    // resource: zeros), and past the wave's last step the cursor keeps
    // re-reading its last (in-bounds) row group.
    int l_rgc = 0, l_sl = 0, l_kb = j0;
    int l_k[MT];
    auto set_rows = [&]() {
      const int rg = wave + 4 * l_rgc;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) l_k[mt] = rg * R + mt * 16 + n;
    };
    // Each step's loads also bring the slab's row of H1 (lane l: H1[i, l]) and
    // its scale, so the end of a slab takes its coefficients from registers
    // instead of waiting on loads issued behind U steps of tensor loads.
    bf16x8 xv[U][2][MT];
    float ar[U], as[U];
    auto load_next = [&](bf16x8 (&dst)[2][MT], float& adst, float& sdst) {
      const int li = s0 + l_sl;
      adst = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ars, li * F * 4 + aof, 0, 0));
      sdst = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(srs, li * 4, 0, 0));
      const __amdgpu_buffer_rsrc_t rs = uniform_rsrc(P.Xt + (int64_t)(s0 + l_sl) * K * Jp, K * Jp * 2);
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int jj = l_kb + 32 * h + 8 * g;
          const unsigned past = ((unsigned)(K - 1 - l_k[mt]) | (unsigned)(Jp - 1 - jj)) & 0x80000000u;
          const int off = (int)(((unsigned)((jj >> 3) * K + l_k[mt]) * 16u) | past);
          dst[h][mt] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
        }
      l_kb += 64;
      if (l_kb >= j0 + jw) {
        l_kb = j0;
        if (++l_sl == ns) {
          l_sl = 0;
          if (l_rgc + 1 < myrg) {
            ++l_rgc;
            set_rows();
          }
        }
      }
    };
    // the first U steps of tensor loads go out before the chunk is staged
    if (total > 0) {
      set_rows();
#pragma unroll
      for (int u = 0; u < U; ++u) load_next(xv[u], ar[u], as[u]);
    }
    __syncthreads();   // the previous chunk's MFMAs are done with the tiles
    for (int e = tid; e < jw * FP; e += 256) {
      const int jj = e / FP, f = e - jj * FP;
      const int j = j0 + jj;
      const float v = (j < J && f < F) ? Hb[(int64_t)j * F + f] : 0.f;
      const __bf16 hi = (__bf16)v;
      Bs[f * JCS + jj] = hi;
      Bl[f * JCS + jj] = (__bf16)(v - (float)hi);   // (the difference is exact in FP32)
    }
    __syncthreads();
    if (total > 0) {   // (wave-uniform; waves without rows still take every barrier)
      f32x4 acc[MT][FT], tot[MT][FT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int ft = 0; ft < FT; ++ft) {
          acc[mt][ft] = f32x4{0.f, 0.f, 0.f, 0.f};
          tot[mt][ft] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
      int c_step = 0, c_sl = 0, c_rgc = 0;
      const __bf16* bb = Bs + n * JCS + 8 * g;
      auto step = [&](int u, bool reload) {
#pragma unroll
        for (int ft = 0; ft < FT; ++ft) {
          const __bf16* bp = bb + ft * 16 * JCS + c_step * 64;
          const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(bp);
          const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(bp + 32);
          const bf16x8 l0 = *reinterpret_cast<const bf16x8*>(bp + FP * JCS);
          const bf16x8 l1 = *reinterpret_cast<const bf16x8*>(bp + FP * JCS + 32);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) acc[mt][ft] = mma_bf16(xv[u][0][mt], b0, acc[mt][ft]);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) acc[mt][ft] = mma_bf16(xv[u][0][mt], l0, acc[mt][ft]);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) acc[mt][ft] = mma_bf16(xv[u][1][mt], b1, acc[mt][ft]);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) acc[mt][ft] = mma_bf16(xv[u][1][mt], l1, acc[mt][ft]);
        }
        // (the coefficients are read out of ar[u], as[u] before the reload
        // writes the next step's values into the same registers)
        const bool last = c_step + 1 == nsteps;
        float coefs[FT];
        if (last) {
#pragma unroll
          for (int ft = 0; ft < FT; ++ft) coefs[ft] = as[u] * __shfl(ar[u], ft * 16 + n);
        }
        if (reload) load_next(xv[u], ar[u], as[u]);
        if (++c_step == nsteps) {
          // end of a slab: scale by s_i * H1[i, f] and accumulate
#pragma unroll
          for (int ft = 0; ft < FT; ++ft) {
            const float coef = coefs[ft];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
              for (int ii = 0; ii < 4; ++ii) tot[mt][ft][ii] += coef * acc[mt][ft][ii];
              acc[mt][ft] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
          }
          c_step = 0;
          if (++c_sl == ns) {
            // end of a row group: its rows of this item's partial (rows past
            // K and columns past F get offsets past the resource: dropped);
            // a later chunk adds to what the earlier ones stored
            const int rg = wave + 4 * c_rgc;
            int offs[MT][FT][4];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
              for (int ft = 0; ft < FT; ++ft)
#pragma unroll
                for (int ii = 0; ii < 4; ++ii) {
                  const int k = rg * R + mt * 16 + 4 * g + ii;
                  const int f = ft * 16 + n;
                  offs[mt][ft][ii] = (k < K && f < F) ? (k * F + f) * 4 : kBufferOOB;
                }
            // a later chunk reads all of the earlier chunks' sums first (one
            // wait for the lot, not one round trip per element)
            float prev[MT][FT][4];
            if (chk > 0) {
#pragma unroll
              for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int ft = 0; ft < FT; ++ft)
#pragma unroll
                  for (int ii = 0; ii < 4; ++ii)
                    prev[mt][ft][ii] = __builtin_bit_cast(
                        float, __builtin_amdgcn_raw_buffer_load_b32(wrs, offs[mt][ft][ii], 0, 0));
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
              for (int ft = 0; ft < FT; ++ft) {
#pragma unroll
                for (int ii = 0; ii < 4; ++ii) {
                  // (the element is copied out first: a bit cast of a vector
                  // element lvalue reads element 0 with this compiler)
                  float t = tot[mt][ft][ii];
                  if (chk > 0) t = prev[mt][ft][ii] + t;
                  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, t), wrs,
                                                        offs[mt][ft][ii], 0, 0);
                }
                tot[mt][ft] = f32x4{0.f, 0.f, 0.f, 0.f};
              }
            c_sl = 0;
            ++c_rgc;
          }
        }
      };
      const int full = total - total % U;
      for (int s = 0; s < full; s += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) step(u, true);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (full + u < total) step(u, false);
    }
  }
}

// ---------------------------------------------------------------- mode-2 item

// W2 rows j0 .. j0+63: one thread per (j, f), summing over all slabs i in
// order (FP64), reads of T coalesced over the contiguous (j, f) index.
__device__ __forceinline__ void m2_item(const ConstProb& P, int idx, const int tid) {
  const int I = P.I, J = P.J, F = P.F;
  const int j0 = idx * 64;
  const int E = min(64, J - j0) * F;
  const int64_t JF = (int64_t)J * F;
  const float* __restrict__ A = P.H[0];
  const float* __restrict__ Tb = P.T + (int64_t)j0 * F;
  // (sixteen slabs of loads in flight per thread: one item streams I rows of
  // T through one block, so its rate is the loads in flight over the latency)
  for (int e = tid; e < E; e += 256) {
    const int f = e % F;
    double s = 0.0;
    int i = 0;
    for (; i + 16 <= I; i += 16) {
      float t[16], a[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        t[q] = Tb[(int64_t)(i + q) * JF + e];
        a[q] = A[(int64_t)(i + q) * F + f];
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) s += (double)a[q] * (double)t[q];
    }
    for (; i < I; ++i) s += (double)A[(int64_t)i * F + f] * (double)Tb[(int64_t)i * JF + e];
    P.W[1][(int64_t)j0 * F + e] = s;
  }
}

// ---------------------------------------------------------------- ADMM items

template <int FL>
__device__ __forceinline__ void inner_item(const ConstProb& P, const BatchK& a, int m, int idx,
                                           unsigned char* lds, const int tid) {
  InnerK k;
  if (m == 2) {   // W3 = the pass-3 partials, summed in item order per element
    k.part = P.W3p;
    k.part_f64 = 0;
    k.pstride = (int64_t)P.K * P.F;
    k.nparts = P.n_p3;
  } else {
    k.part = (m == 0) ? P.W[0] : P.W[1];
    k.part_f64 = 1;
    k.pstride = 0;
    k.nparts = 1;
  }
  k.rowstride = P.F;
  k.Wout = nullptr;
  // (selects, not P.H[m]: a run-time index would put the descriptor in scratch)
  k.H = (m == 0) ? P.H[0] : (m == 1) ? P.H[1] : P.H[2];
  k.U = (m == 0) ? P.U[0] : (m == 1) ? P.U[1] : P.U[2];
  k.Pout = nullptr;
  k.rows = (m == 0) ? P.I : (m == 1) ? P.J : P.K;
  k.F = P.F;
  k.Ginv = P.Ginv;
  k.proj = 0;
  k.lo = 0.0;
  k.hi = 0.0;
  k.rho = P.rho + 2 * m;
  k.rescale = a.rescale;
  k.T = a.T;
  k.eps_abs = a.eps_abs;
  k.eps_rel = a.eps_rel;
  k.iters_out = nullptr;
  k.gram_from_primal = 0;
  k.gram_f32 = 1;
  k.gram_part = P.gpart;
  k.resid_part = nullptr;
  k.flag = a.flag;
  k.dv = k.dx = k.dh0 = nullptr;
  // ipi row blocks of batch_inner_rows(FL) rows; the barrier keeps one block's last LDS
  // reads apart from the next block's first writes
  const int nb = (m == 0) ? P.n_in[0] : (m == 1) ? P.n_in[1] : P.n_in[2];
  const int b0 = idx * P.ipi, b1 = min(nb, b0 + P.ipi);
  for (int bid = b0; bid < b1; ++bid) {
    if (bid > b0) __syncthreads();
    inner_body<float, FL, batch_inner_rpl<FL>(), 4, 1>(k, bid, lds, tid, bid == b0);
  }
}

template <int NB>
__device__ __forceinline__ void prep_item(const ConstProb& P, const BatchK& a, int m,
                                          unsigned char* lds, const int tid) {
  PrepK k{};
  k.F = P.F;
  k.gram_part = nullptr;
  k.gram_a = (m == 0) ? P.gram[1] : P.gram[0];
  k.gram_b = (m == 2) ? P.gram[1] : P.gram[2];
  k.policy = a.policy;
  k.rho0 = a.rho0;
  k.rho_state = P.rho + 2 * m;
  k.Ginv = P.Ginv;
  k.flag = a.flag;
  PrepIn<NB> in;
  prep_load_b(k, tid, in);
  prep_load_a(k, tid, in);
  prep_body<NB>(k, reinterpret_cast<double*>(lds), tid, in);
}

// One function per item family, each loading the fields of the problem's
// descriptor it uses (read-only for the launch: through the constant address
// space, into scalar registers), so no descriptor field stays live across
// the families.
static __device__ __forceinline__ const ConstProb& load_prob(const BProb* probs, int p) {
  return ((const ConstProb*)probs)[p];
}

__device__ __forceinline__ void run_p1(const BProb* probs, int p, int idx,
                                                 unsigned char* lds, const int tid) {
  const ConstProb& P = load_prob(probs, p);
  switch (P.FT * 4 + P.mt1) {
    case 1 * 4 + 1: p1_item<1, 1>(P, idx, lds, tid); break;
    case 1 * 4 + 2: p1_item<1, 2>(P, idx, lds, tid); break;
    case 2 * 4 + 1: p1_item<2, 1>(P, idx, lds, tid); break;
    case 2 * 4 + 2: p1_item<2, 2>(P, idx, lds, tid); break;
    case 3 * 4 + 1: p1_item<3, 1>(P, idx, lds, tid); break;
    case 3 * 4 + 2: p1_item<3, 2>(P, idx, lds, tid); break;
    case 4 * 4 + 1: p1_item<4, 1>(P, idx, lds, tid); break;
    default: p1_item<4, 2>(P, idx, lds, tid); break;
  }
}

__device__ __forceinline__ void run_p3(const BProb* probs, int p, int idx,
                                                 unsigned char* lds, const int tid) {
  const ConstProb& P = load_prob(probs, p);
  switch (P.FT * 4 + P.mt3) {
    case 1 * 4 + 1: p3_item<1, 1>(P, idx, lds, tid); break;
    case 1 * 4 + 2: p3_item<1, 2>(P, idx, lds, tid); break;
    case 2 * 4 + 1: p3_item<2, 1>(P, idx, lds, tid); break;
    case 2 * 4 + 2: p3_item<2, 2>(P, idx, lds, tid); break;
    case 3 * 4 + 1: p3_item<3, 1>(P, idx, lds, tid); break;
    case 3 * 4 + 2: p3_item<3, 2>(P, idx, lds, tid); break;
    case 4 * 4 + 1: p3_item<4, 1>(P, idx, lds, tid); break;
    default: p3_item<4, 2>(P, idx, lds, tid); break;
  }
}

__device__ __forceinline__ void run_m2(const BProb* probs, int p, int idx, const int tid) {
  const ConstProb& P = load_prob(probs, p);
  m2_item(P, idx, tid);
}

__device__ __forceinline__ void run_inner(const BProb* probs, int p, const BatchK& a,
                                                    int m, int idx, unsigned char* lds, const int tid) {
  const ConstProb& P = load_prob(probs, p);
  switch (P.FL) {
    case 4: inner_item<4>(P, a, m, idx, lds, tid); break;
    case 8: inner_item<8>(P, a, m, idx, lds, tid); break;
    case 16: inner_item<16>(P, a, m, idx, lds, tid); break;
    case 32: inner_item<32>(P, a, m, idx, lds, tid); break;
    default: inner_item<64>(P, a, m, idx, lds, tid); break;
  }
}

__device__ __forceinline__ void run_prep(const BProb* probs, int p, const BatchK& a,
                                                   int m, unsigned char* lds, const int tid) {
  const ConstProb& P = load_prob(probs, p);
  switch (P.NB) {
    case 1: prep_item<1>(P, a, m, lds, tid); break;
    case 2: prep_item<2>(P, a, m, lds, tid); break;
    case 3: prep_item<3>(P, a, m, lds, tid); break;
    default: prep_item<4>(P, a, m, lds, tid); break;
  }
}

// Dependencies of an item kind: (kind, count that must be done) pairs.
__device__ __forceinline__ int item_deps(int kind, const ConstProb* P, int (&dk)[2], int (&need)[2]) {
  switch (kind) {
    case BK_IN1: dk[0] = BK_P1; need[0] = P->n_p1; dk[1] = BK_PREP1; need[1] = 1; return 2;
    case BK_PREP2: dk[0] = BK_IN1; need[0] = P->ni[0]; return 1;
    case BK_M2: dk[0] = BK_P1; need[0] = P->n_p1; dk[1] = BK_IN1; need[1] = P->ni[0]; return 2;
    case BK_IN2: dk[0] = BK_M2; need[0] = P->n_m2; dk[1] = BK_PREP2; need[1] = 1; return 2;
    case BK_PREP3: dk[0] = BK_IN2; need[0] = P->ni[1]; return 1;
    case BK_P3: dk[0] = BK_IN2; need[0] = P->ni[1]; return 1;
    case BK_IN3: dk[0] = BK_P3; need[0] = P->n_p3; dk[1] = BK_PREP3; need[1] = 1; return 2;
    default: return 0;
  }
}

// Bounded wait: gives up (flag bit 8) after spin_limit polls, and at once
// when an earlier wait of the launch has given up.
__device__ __forceinline__ void wait_count(int* c, int need, const BatchK& a) {
  long long spins = 0;
  while (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
    __builtin_amdgcn_s_sleep(2);
    if (++spins > a.spin_limit ||
        (__hip_atomic_load(a.flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 8)) {
      atomicOr(a.flag, 8);
      break;
    }
  }
}

__global__ __launch_bounds__(256, 2) void k_batch(BatchK a) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ unsigned s_ticket;
  __shared__ int s_last;
  const int tid0 = threadIdx.x;
  for (;;) {
    // The thread index, made opaque to the compiler once per item: it cannot
    // hoist each item family's thread-index arithmetic out of this loop,
    // where it would stay live across all the families.
    int tid = tid0;
    asm volatile("" : "+v"(tid));
    if (tid == 0) s_ticket = atomicAdd(a.head, 1u);
    __syncthreads();
    // (readfirstlane: the ticket is block-uniform, so the item, the problem
    // descriptor and everything derived from them live in scalar registers)
    const unsigned t = __builtin_amdgcn_readfirstlane(s_ticket);
    __syncthreads();
    if (t >= (unsigned)a.n_items) break;
    const uint2 it = a.items[t];
    const int p = __builtin_amdgcn_readfirstlane((int)it.x);
    const int kind = __builtin_amdgcn_readfirstlane((int)(it.y >> 24));
    const int idx = __builtin_amdgcn_readfirstlane((int)(it.y & 0xffffffu));
    const ConstProb* P = (const ConstProb*)(a.probs) + p;
    int* ctr = a.ctr + (int64_t)p * kCtrPerProb;
    const unsigned long long t_take = a.prof ? wall_clock64() : 0ull;
    if (!a.nodeps) {
      int dk[2], need[2];
      const int nd = item_deps(kind, P, dk, need);   // block-uniform
      if (nd > 0) {
        if (tid == 0) {
          wait_count(&ctr[dk[0]], need[0], a);
          if (nd > 1) wait_count(&ctr[dk[1]], need[1], a);
          // acquire at agent scope, by one wave: invalidates this CU's L1 and
          // the XCD's L2, so every wave of the block then reads the
          // producers' data from memory
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
      }
    }
    const unsigned long long t_ready = a.prof ? wall_clock64() : 0ull;
    switch (kind) {
      case BK_P1: run_p1(a.probs, p, idx, lds, tid); break;
      case BK_P3: run_p3(a.probs, p, idx, lds, tid); break;
      case BK_M2: run_m2(a.probs, p, idx, tid); break;
      case BK_PREP1: run_prep(a.probs, p, a, 0, lds, tid); break;
      case BK_PREP2: run_prep(a.probs, p, a, 1, lds, tid); break;
      case BK_PREP3: run_prep(a.probs, p, a, 2, lds, tid); break;
      default: {   // inner sweep of mode m; the last block of the mode forms its Gram
        const int m = (kind == BK_IN1) ? 0 : (kind == BK_IN2) ? 1 : 2;
        run_inner(a.probs, p, a, m, idx, lds, tid);
        __builtin_amdgcn_s_waitcnt(0);   // this wave's stores have reached the L2
        __syncthreads();
        if (tid == 0) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // L2 written back
          const int tk = atomicAdd(&ctr[kArriveIn + m], 1);
          s_last = (tk == ((m == 0) ? P->ni[0] : (m == 1) ? P->ni[1] : P->ni[2]) - 1) ? 1 : 0;
          if (s_last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (s_last) {
          const int F = P->F, nb = (m == 0) ? P->n_in[0] : (m == 1) ? P->n_in[1] : P->n_in[2];
          const double* gp = P->gpart;
          double* gm = (m == 0) ? P->gram[0] : (m == 1) ? P->gram[1] : P->gram[2];
          for (int e = tid; e < F * F; e += 256) {
            double s = 0.0;
            for (int b = 0; b < nb; ++b) s += gp[(int64_t)b * F * F + e];
            gm[e] = s;
          }
        }
        break;
      }
    }
    // release: every wave waits for its own stores to reach the L2, then one
    // wave writes the L2 back (agent scope) before the count moves
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      atomicAdd(&ctr[kind], 1);
      if (a.prof) {
        const unsigned long long t_done = wall_clock64();
        atomicAdd(&a.prof[kind * 3 + 0], t_done - t_ready);
        atomicAdd(&a.prof[kind * 3 + 1], t_ready - t_take);
        atomicAdd(&a.prof[kind * 3 + 2], 1ull);
      }
    }
  }
}

hipError_t launch_batch(const BatchK& k, int grid, size_t lds, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute((const void*)k_batch,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batch, dim3(grid), dim3(256), lds, s, k);
  return hipGetLastError();
}

int batch_occupancy(size_t lds) {
  if (hipFuncSetAttribute((const void*)k_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds) != hipSuccess)
    return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch, 256, lds) != hipSuccess) return 0;
  return nb;
}

__global__ __launch_bounds__(256) void k_zero_ints(int* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = 0;
}

hipError_t launch_zero_ints(int* p, int64_t n, hipStream_t s) {
  const int64_t nb = std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_zero_ints, dim3((unsigned)std::max<int64_t>(nb, 1)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- set-up

// One block per slab: the power-of-two scale (max|X[i]|/s_i in [1,2)), the
// k-grouped copy [Kp/8][J][8] and, through 32 x 32 LDS tiles, the j-grouped copy
// [Jp/8][K][8] (eight consecutive j innermost, then k); padding is zero.
__global__ __launch_bounds__(256) void k_bquant(const float* __restrict__ X, int J, int K, int Kp,
                                                int Jp, __bf16* __restrict__ Xr,
                                                __bf16* __restrict__ Xt, float* __restrict__ scale) {
  const int64_t i = blockIdx.x;
  const int tid = threadIdx.x;
  const float* Xi = X + i * J * K;
  const int64_t n = (int64_t)J * K;
  float m = 0.f;
  for (int64_t t = tid; t < n; t += 256) m = fmaxf(m, fabsf(Xi[t]));
  __shared__ float red[256];
  __shared__ float tile[32][33];
  red[tid] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmaxf(red[tid], red[tid + w]);
    __syncthreads();
  }
  m = red[0];
  float s = 1.f;
  if (m > 0.f && isfinite(m)) {
    int e;
    (void)frexpf(m, &e);
    s = ldexpf(1.f, e - 1);
  }
  if (tid == 0) scale[i] = s;
  const float inv = 1.f / s;   // exact: s is a power of two
  __bf16* Xri = Xr + i * J * Kp;
  for (int64_t t = tid; t < (int64_t)J * Kp; t += 256) {
    const int64_t j = t / Kp, k = t - j * Kp;
    Xri[((k >> 3) * J + j) * 8 + (k & 7)] = (__bf16)((k < K) ? Xi[j * K + k] * inv : 0.f);
  }
  __bf16* Xti = Xt + i * K * Jp;
  const int tr = tid >> 5, tc = tid & 31;
  for (int j0 = 0; j0 < Jp; j0 += 32)
    for (int k0 = 0; k0 < K; k0 += 32) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = j0 + tr + 8 * q, k = k0 + tc;
        tile[tr + 8 * q][tc] = (j < J && k < K) ? Xi[(int64_t)j * K + k] * inv : 0.f;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = k0 + tr + 8 * q, j = j0 + tc;
        if (k < K) Xti[((int64_t)(j >> 3) * K + k) * 8 + (j & 7)] = (__bf16)tile[tc][tr + 8 * q];
      }
    }
}

hipError_t launch_batch_quantize(const float* X, int I, int J, int K, int Kp, int Jp, __bf16* Xr,
                                 __bf16* Xt, float* scale, hipStream_t s) {
  hipLaunchKernelGGL(k_bquant, dim3(I), dim3(256), 0, s, X, J, K, Kp, Jp, Xr, Xt, scale);
  return hipGetLastError();
}

}  // namespace ntf
