// MTTKRP kernels for gfx950: the three matricised-tensor-times-Khatri-Rao
// products of one ADMoM iteration (eq. ADMM_NTF_ALS_C), computed from one copy
// of the dense tensor X [I][J][K] (k fastest) in two streaming passes.
//
//   pass 1:  T[i,j,:] = sum_k X[i,j,k] C[k,:]         (MFMA, contraction over k)
//            W1[i,:]  = sum_j B[j,:] * T[i,j,:]       (fused epilogue, per-tile partials)
//   mode 2:  W2[j,:]  = sum_i A_new[i,:] * T[i,j,:]   (T re-read; X is not)
//   pass 3:  W3[k,:]  = sum_{i,j} X[i,j,k] A_new[i,:] * B_new[j,:]
//                                                    (MFMA, contraction over (i,j);
//                                                     FP32/FP64: Khatri-Rao rows built
//                                                     per tile in LDS; BF16: B_new in
//                                                     LDS, A_new applied per slab)
//
// Modes 1 and 2 both contract C^k over k (the update of B uses A^{k+1} and C^k),
// so the k-contraction T is shared by them: two passes over X per outer
// iteration instead of three.  The Khatri-Rao matrix is never materialised:
// pass 1 keeps C in LDS; pass 3 builds 64 Khatri-Rao rows at a time in LDS
// (FP32/FP64) or contracts each slab against B and scales the result by the
// slab's row of A (BF16).
//
// All partial sums are written to fixed slots and reduced later in a fixed
// order, so results are bitwise reproducible.
#include "ntf_device.h"
#include "ntf_launch.h"

#include <algorithm>

namespace ntf {

// zeroed bfloat16 elements after H3^T in the streaming pass-1 LDS (a super
// step of the last row may read up to 32 past it)
constexpr int kPass1Tail = 64;

// Waves per SIMD the streaming pass-1 kernel is compiled for: four (two
// blocks of 512 threads per CU, 128 VGPRs) while F <= 32, two at larger F
// (its accumulators and prefetched epilogue values need more registers).
template <int FT>
static constexpr int kPass1Waves() { return FT <= 2 ? 4 : 2; }

// ---------------------------------------------------------------- set-up

// bfloat16 copies of X with a power-of-two scale per mode-1 slab:
//   s_i = 2^(e-1) where max|X[i]| = m * 2^e, m in [0.5, 1)  (so max|X[i]|/s_i in [1,2));
//   Xr  [I][Kp/8][J][8] groups of 8 consecutive k innermost, then j, k padded
//                       with zeros to Kp (multiple of 32);
//   Xj8 [I][JG][Kp3][8] groups of 8 consecutive j interleaved innermost, zero padded.
// (A wave's 16 rows of one 8-column group are 256 contiguous bytes in either
// copy, so a pass-1 or pass-3 load instruction reads four such runs.)
__global__ __launch_bounds__(256) void k_quantize(const float* __restrict__ X, int64_t J, int64_t K,
                                                  int64_t Kp, int64_t JG, int64_t Kp3,
                                                  __bf16* __restrict__ Xr, __bf16* __restrict__ Xj8,
                                                  float* __restrict__ scale) {
  const int64_t i = blockIdx.x;
  const float* Xi = X + i * J * K;
  const int64_t n = J * K;
  float m = 0.f;
  for (int64_t t = threadIdx.x; t < n; t += 256) m = fmaxf(m, fabsf(Xi[t]));
  __shared__ float red[256];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  m = red[0];
  float s = 1.f;
  if (m > 0.f && isfinite(m)) {
    int e;
    (void)frexpf(m, &e);
    s = ldexpf(1.f, e - 1);
  }
  if (threadIdx.x == 0) scale[i] = s;
  const float inv = 1.f / s;  // exact: s is a power of two
  __bf16* Xri = Xr + i * J * Kp;
  for (int64_t t = threadIdx.x; t < J * Kp; t += 256) {
    const int64_t j = t / Kp, k = t - j * Kp;
    const float v = (k < K) ? Xi[j * K + k] * inv : 0.f;
    Xri[((k >> 3) * J + j) * 8 + (k & 7)] = (__bf16)v;
  }
  __bf16* Xji = Xj8 + i * JG * Kp3 * 8;
  for (int64_t t = threadIdx.x; t < JG * Kp3 * 8; t += 256) {
    const int64_t e = t & 7, rest = t >> 3;
    const int64_t jg = rest / Kp3, k = rest - jg * Kp3;
    const int64_t j = jg * 8 + e;
    const float v = (j < J && k < K) ? Xi[j * K + k] * inv : 0.f;
    Xji[t] = (__bf16)v;
  }
}

// The same scales and the j-grouped copy for K a multiple of 4, one slab per
// block: the slab's maximum from 16-byte loads, then one pass in which 32
// lanes walk the 4-column groups of 8 consecutive rows j (16-byte loads of
// each row): every value is read once more and written to Xj8 with 16-byte
// stores (the 8 rows of one column).  k_xr_from_xj8 then forms the k-grouped
// copy from it.  The bfloat16 values are those of k_quantize (round to
// nearest even of X * (1/s), the same FP32 product).
__global__ __launch_bounds__(256) void k_quantize4(const float* __restrict__ X, int J, int K, int Kp,
                                                   int JG, int Kp3, __bf16* __restrict__ Xr,
                                                   __bf16* __restrict__ Xj8,
                                                   float* __restrict__ scale) {
  const int64_t i = blockIdx.x;
  const float4* Xi4 = reinterpret_cast<const float4*>(X + i * (int64_t)J * K);
  const int n4 = J * K / 4;
  float m = 0.f;
  {
    int t = threadIdx.x;
    for (; t + 768 < n4; t += 1024) {
      const float4 a = Xi4[t], b = Xi4[t + 256], c = Xi4[t + 512], d = Xi4[t + 768];
      m = fmaxf(m, fmaxf(fmaxf(fabsf(a.x), fabsf(a.y)), fmaxf(fabsf(a.z), fabsf(a.w))));
      m = fmaxf(m, fmaxf(fmaxf(fabsf(b.x), fabsf(b.y)), fmaxf(fabsf(b.z), fabsf(b.w))));
      m = fmaxf(m, fmaxf(fmaxf(fabsf(c.x), fabsf(c.y)), fmaxf(fabsf(c.z), fabsf(c.w))));
      m = fmaxf(m, fmaxf(fmaxf(fabsf(d.x), fabsf(d.y)), fmaxf(fabsf(d.z), fabsf(d.w))));
    }
    for (; t < n4; t += 256) {
      const float4 a = Xi4[t];
      m = fmaxf(m, fmaxf(fmaxf(fabsf(a.x), fabsf(a.y)), fmaxf(fabsf(a.z), fabsf(a.w))));
    }
  }
  __shared__ float red[256];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  m = red[0];
  float s = 1.f;
  if (m > 0.f && isfinite(m)) {
    int e;
    (void)frexpf(m, &e);
    s = ldexpf(1.f, e - 1);
  }
  if (threadIdx.x == 0) scale[i] = s;
  const float inv = 1.f / s;  // exact: s is a power of two
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int K4 = K / 4, C4 = Kp3 / 4;
  __bf16* Xji = Xj8 + i * (int64_t)JG * Kp3 * 8;
  for (int jg = ty; jg < JG; jg += 8) {
    for (int c4 = tx; c4 < C4; c4 += 32) {
      float4 v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int j = 8 * jg + e;
        v[e] = (j < J && c4 < K4) ? Xi4[(int64_t)j * K4 + c4] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
      if (4 * c4 < Kp3) {
        bf16x8 o[4];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          o[0][e] = (__bf16)(v[e].x * inv);
          o[1][e] = (__bf16)(v[e].y * inv);
          o[2][e] = (__bf16)(v[e].z * inv);
          o[3][e] = (__bf16)(v[e].w * inv);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
          *reinterpret_cast<bf16x8*>(Xji + ((int64_t)jg * Kp3 + 4 * c4 + c) * 8) = o[c];
      }
    }
  }
}

// sum of squares, FP64 accumulation, fixed-order two-level reduction
template <typename XT>
__global__ __launch_bounds__(256) void k_sumsq_part(const XT* __restrict__ X, int64_t n,
                                                    double* __restrict__ part) {
  // eight interleaved sums per thread (eight loads in flight; one sum had
  // each load wait for the previous add), added in a fixed order
  constexpr int V = 8;
  double acc[V];
#pragma unroll
  for (int q = 0; q < V; ++q) acc[q] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (; t + (V - 1) * stride < n; t += V * stride) {
    double v[V];
#pragma unroll
    for (int q = 0; q < V; ++q) v[q] = (double)X[t + q * stride];
#pragma unroll
    for (int q = 0; q < V; ++q) acc[q] += v[q] * v[q];
  }
  for (; t < n; t += stride) {
    const double v = (double)X[t];
    acc[0] += v * v;
  }
  const double a = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __shared__ double red[256];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// (lane l sums partials l, l + 64, .. in order, then the lanes' sums are
// added by a fixed butterfly; one lane walking all partials took 60 us)
__global__ __launch_bounds__(64) void k_sum_parts(const double* __restrict__ part, int nparts,
                                                  double* __restrict__ out) {
  double s = 0.0;
  for (int p = threadIdx.x; p < nparts; p += 64) s += part[p];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (threadIdx.x == 0) *out = s;
}

// ---------------------------------------------------------------- pass 1

// Work item = (slab i, chunk of 16*MT consecutive j), all of k, owned by ONE
// wave; the four waves of a block take four items at a time and share C in
// LDS (loaded once per block when it fits, which it does for K*F up to
// 600*64 in FP32 and 1200*64 in bf16).  Each wave streams its rows of X with
// 16-byte loads that are the MFMA A operands, keeping U k-steps of loads in
// flight, and contracts them against all FT 16-column tiles of the rank.
// The epilogue stores T and reduces this item's share of
// W1[i,:] = sum_j B[j,:] * T[i,j,:] across the wave into P1[i][chunk][:].
//
// FP32/FP64: C in LDS as [k/4][FP][4] so one 16-byte read gives the B
// operands of the four MFMAs whose contraction slots match the 16-byte X load
// (lane group g holds k = kb + 4g + c in element c).
template <typename T, int FT, int MT>
__global__ __launch_bounds__(512) void k_pass1(const T* __restrict__ X, int I, int J, int K, int F,
                                               const T* __restrict__ Hb, const T* __restrict__ Hc,
                                               T* __restrict__ Tout, T* __restrict__ P1, int nch,
                                               int KC, int vec) {
  typedef Mfma<T> M;
  typedef typename M::acc_t acc_t;
  constexpr int FP = FT * 16;
  constexpr int R = 16 * MT;
  constexpr int U = 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Cs = reinterpret_cast<T*>(smem_raw);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n = lane & 15, g = lane >> 4;
  const int64_t nitems = (int64_t)I * nch;
  const int nkc = (K + KC - 1) / KC;
  const int nwb = blockDim.x >> 6;
  const int64_t nblock_iters = (nitems + (int64_t)nwb * gridDim.x - 1) / ((int64_t)nwb * gridDim.x);
  for (int64_t bi = 0; bi < nblock_iters; ++bi) {
    const int64_t item = (bi * gridDim.x + blockIdx.x) * nwb + wave;
    const bool has = item < nitems;
    const int i = has ? (int)(item / nch) : 0;
    const int ch = has ? (int)(item - (int64_t)i * nch) : 0;
    const int j0 = ch * R;
    acc_t acc[MT][FT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int ft = 0; ft < FT; ++ft) acc[mt][ft] = M::zero();
    for (int kc = 0; kc < nkc; ++kc) {
      const int kbeg = kc * KC, kend = min(K, kbeg + KC);
      if (nkc > 1 || bi == 0) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < KC * FP; idx += blockDim.x) {
          const int kk = idx / FP, f = idx - kk * FP, k = kbeg + kk;
          const T v = (k < kend && f < F) ? Hc[(int64_t)k * F + f] : T(0);
          Cs[((kk >> 2) * FP + f) * 4 + (kk & 3)] = v;
        }
        __syncthreads();
      }
      if (!has) continue;
      const T* xrow[MT];
      bool rowok[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int j = j0 + mt * 16 + n;
        rowok[mt] = j < J;
        xrow[mt] = X + ((int64_t)i * J + (rowok[mt] ? j : 0)) * K + 8 * g;
      }
      // super step = 32 k: lane group g loads k = kb+8g .. kb+8g+7 of each of
      // its rows (two 16-byte loads, h = 0, 1); MFMA (h,c) contracts slot g
      // at k = kb + 8g + 4h + c
      T xv[U][2][MT][4];
      auto load_step = [&](int kb, T (&dst)[2][MT][4]) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int valid = kend - (kb + 8 * g + 4 * h);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            if (rowok[mt] && valid > 0) {
              load4<T>(xrow[mt] + kb + 4 * h, valid, vec, dst[h][mt]);
            } else {
#pragma unroll
              for (int c = 0; c < 4; ++c) dst[h][mt][c] = T(0);
            }
          }
        }
      };
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (kbeg + 32 * u < kend) load_step(kbeg + 32 * u, xv[u]);
      for (int kb = kbeg; kb < kend; kb += 32 * U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int kbu = kb + 32 * u;
          if (kbu < kend) {
            // every MFMA of the super step runs: slots past K hold zeros in X and C
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const T* cbase = Cs + ((((kbu - kbeg) >> 2) + 2 * g + h) * FP + n) * 4;
#pragma unroll
              for (int ft = 0; ft < FT; ++ft) {
                T cv[4];
                Vec4Load<T>::load(cbase + ft * 64, cv);
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                  for (int mt = 0; mt < MT; ++mt)
                    acc[mt][ft] = M::mma(xv[u][h][mt][c], cv[c], acc[mt][ft]);
              }
            }
            if (kbu + 32 * U < kend) load_step(kbu + 32 * U, xv[u]);
          }
        }
      }
    }
    if (!has) continue;
    // epilogue: store T, reduce this item's share of W1[i,:]
    T part[FT];
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) part[ft] = T(0);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int ft = 0; ft < FT; ++ft)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const int j = j0 + mt * 16 + M::row(g, ii);
          const int f = ft * 16 + n;
          if (j < J && f < F) {
            const T v = acc[mt][ft][ii];
            if (Tout) Tout[((int64_t)i * J + j) * F + f] = v;
            part[ft] += Hb[(int64_t)j * F + f] * v;
          }
        }
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) {
      part[ft] += __shfl_xor(part[ft], 16);
      part[ft] += __shfl_xor(part[ft], 32);
      const int f = ft * 16 + n;
      if (g == 0 && f < F) P1[((int64_t)i * nch + ch) * F + f] = part[ft];
    }
  }
}

// BF16: X from the k-grouped bfloat16 copy (Kp a multiple of 32, zero
// padded); C transposed in LDS as bf16 [FP][KC+8].  A super step covers 64 k:
// lane (n,g) loads columns k = kb+16g .. kb+16g+15 of its row (two 16-byte
// pieces, one from each of two 8-column groups) and feeds them to two MFMAs,
// h = 0, 1, whose contraction slot of lane group g holds k = kb+16g+8h+e; the
// matching B operands are one 32-byte LDS read per rank tile.  The slab scale
// s_i is applied to the FP32 accumulator in the epilogue (exact).
template <int FT, int MT>
__global__ __launch_bounds__(512) void k_pass1_bf16(const __bf16* __restrict__ Xr,
                                                    const float* __restrict__ scale, int I, int J,
                                                    int K, int Kp, int F, const float* __restrict__ Hb,
                                                    const float* __restrict__ Hc,
                                                    float* __restrict__ Tout, float* __restrict__ P1,
                                                    int nch, int KC) {
  constexpr int FP = FT * 16;
  constexpr int R = 16 * MT;
  constexpr int U = 2;
  const int KCS = KC + 8;  // LDS row stride (elements); 16-byte multiple since KC % 32 == 0
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __bf16* Cs = reinterpret_cast<__bf16*>(smem_raw);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n = lane & 15, g = lane >> 4;
  const int64_t nitems = (int64_t)I * nch;
  const int nkc = (Kp + KC - 1) / KC;
  const int nwb = blockDim.x >> 6;
  const int64_t nblock_iters = (nitems + (int64_t)nwb * gridDim.x - 1) / ((int64_t)nwb * gridDim.x);
  for (int64_t bi = 0; bi < nblock_iters; ++bi) {
    const int64_t item = (bi * gridDim.x + blockIdx.x) * nwb + wave;
    const bool has = item < nitems;
    const int i = has ? (int)(item / nch) : 0;
    const int ch = has ? (int)(item - (int64_t)i * nch) : 0;
    const int j0 = ch * R;
    f32x4 acc[MT][FT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int ft = 0; ft < FT; ++ft) acc[mt][ft] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < nkc; ++kc) {
      // KC is a multiple of 64 (whole super steps, zero filled past K in LDS);
      // X rows end at Kp (a multiple of 32), so loads are masked per lane
      const int kbeg = kc * KC, kend = min(Kp, kbeg + KC);
      if (nkc > 1 || bi == 0) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < KC * FP; idx += blockDim.x) {
          const int kk = idx / FP, f = idx - kk * FP, k = kbeg + kk;
          const float v = (k < K && f < F) ? Hc[(int64_t)k * F + f] : 0.f;
          Cs[f * KCS + kk] = (__bf16)v;
        }
        __syncthreads();
      }
      if (!has) continue;
      // (row j's 8-column group q of slab i starts at Xr + ((i Kp/8 + q) J + j) 8)
      const __bf16* xrow[MT];
      bool rowok[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int j = j0 + mt * 16 + n;
        rowok[mt] = j < J;
        xrow[mt] = Xr + ((int64_t)i * (Kp / 8) * J + (rowok[mt] ? j : 0)) * 8;
      }
      bf16x8 xv[U][2][MT];
      auto load_step = [&](int kb, bf16x8 (&dst)[2][MT]) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            if (rowok[mt] && kb + 16 * g + 8 * h < kend) {
              const int q = (kb + 16 * g + 8 * h) >> 3;
              dst[h][mt] = *reinterpret_cast<const bf16x8*>(xrow[mt] + (int64_t)q * J * 8);
            } else {
#pragma unroll
              for (int e = 0; e < 8; ++e) dst[h][mt][e] = (__bf16)0.f;
            }
          }
      };
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (kbeg + 64 * u < kend) load_step(kbeg + 64 * u, xv[u]);
      const __bf16* cb = Cs + n * KCS + 16 * g;
      for (int kb = kbeg; kb < kend; kb += 64 * U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int kbu = kb + 64 * u;
          if (kbu < kend) {
#pragma unroll
            for (int ft = 0; ft < FT; ++ft) {
              const __bf16* cp = cb + ft * 16 * KCS + (kbu - kbeg);
              const bf16x8 c0 = *reinterpret_cast<const bf16x8*>(cp);
              const bf16x8 c1 = *reinterpret_cast<const bf16x8*>(cp + 8);
#pragma unroll
              for (int mt = 0; mt < MT; ++mt) acc[mt][ft] = mma_bf16(xv[u][0][mt], c0, acc[mt][ft]);
#pragma unroll
              for (int mt = 0; mt < MT; ++mt) acc[mt][ft] = mma_bf16(xv[u][1][mt], c1, acc[mt][ft]);
            }
            if (kbu + 64 * U < kend) load_step(kbu + 64 * U, xv[u]);
          }
        }
      }
    }
    if (!has) continue;
    const float s = scale[i];
    float part[FT];
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) part[ft] = 0.f;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int ft = 0; ft < FT; ++ft)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const int j = j0 + mt * 16 + 4 * g + ii;
          const int f = ft * 16 + n;
          if (j < J && f < F) {
            const float v = s * acc[mt][ft][ii];
            Tout[((int64_t)i * J + j) * F + f] = v;
            part[ft] += Hb[(int64_t)j * F + f] * v;
          }
        }
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) {
      part[ft] += __shfl_xor(part[ft], 16);
      part[ft] += __shfl_xor(part[ft], 32);
      const int f = ft * 16 + n;
      if (g == 0 && f < F) P1[((int64_t)i * nch + ch) * F + f] = part[ft];
    }
  }
}

// BF16 pass 1, streaming form (C fits in LDS, loaded once per block).  Work
// is split into (row tile ch of j, run of consecutive slabs) pairs, tiles
// fastest, so a wave keeps one tile for a long run: its H2 values (the
// epilogue's W1 weights, 32 per lane) load once per run, and the X loads of
// the run go through a per-slab buffer resource at lane offsets fixed for the
// run.  The wave walks (slab, 64-k super step) as one continuous sequence with
// U steps of loads in flight; every step issues the same loads (rows j >= J
// and columns past Kp in the last super step get offsets past the resource),
// so the wait before a step covers that step only.  The two MFMAs of a super
// step contract its columns 0-31 and 32-63 (lane group g: columns 8g .. 8g+7
// of a half), so with the k-grouped copy each load instruction reads four
// runs of 256 bytes, the 16 rows of four 8-column groups (with the row-major
// copy it read 64-byte pieces of 16 rows: 0.277 -> 0.267 ms).  The epilogue of a slab
// (T rows and the W1 partial of (i, ch)) stores through resources at offsets
// that drop rows past J, columns past F and the lanes that hold no partial.
// TS (F a multiple of 4, LDS to spare): the T rows of a slab go through a
// per-wave LDS area (row stride FP + 4 floats: the column writes of the lane
// groups then fall in distinct banks) and leave as 16-byte stores, four
// whole 64-column rows per instruction, instead of 64-byte pieces.
template <int FT, int MT, bool TS>
__global__ __launch_bounds__(512, kPass1Waves<FT>()) void k_pass1_bf16s(const __bf16* __restrict__ Xr,
                                                     const float* __restrict__ scale, int I, int J,
                                                     int K, int Kp, int F,
                                                     const float* __restrict__ Hb,
                                                     const float* __restrict__ Hc,
                                                     float* __restrict__ Tout,
                                                     float* __restrict__ P1, int nch, int spg,
                                                     int G) {
  constexpr int FP = FT * 16;
  constexpr int R = 16 * MT;
  // (four waves per SIMD at FT <= 2, two at FT > 2: the same 128 KB of
  // tensor loads in flight per CU either way)
  constexpr int U = (FT <= 2) ? 2 : 4;
  // Rows of H3^T are Kp + 8 long (not KC + 8): two blocks then fit a CU at
  // F = 64, K = 600.  A super step past Kp reads the start of the next row (or
  // the zeroed tail after the last row) against tensor operands that are zero
  // there, so those products vanish.
  const int KCS = Kp + 8;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __bf16* Cs = reinterpret_cast<__bf16*>(smem_raw);
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n = lane & 15, g = lane >> 4;
  for (int idx = threadIdx.x; idx < Kp * FP; idx += blockDim.x) {
    const int kk = idx / FP, f = idx - kk * FP;
    const float v = (kk < K && f < F) ? Hc[(int64_t)kk * F + f] : 0.f;
    Cs[f * KCS + kk] = (__bf16)v;
  }
  for (int idx = threadIdx.x; idx < FP * 8 + kPass1Tail; idx += blockDim.x) {
    // the 8 padding elements of every row, then the tail
    const int e = (idx < FP * 8) ? (idx >> 3) * KCS + Kp + (idx & 7) : FP * KCS + (idx - FP * 8);
    Cs[e] = (__bf16)0.f;
  }
  __syncthreads();
  const int nwb = blockDim.x >> 6;
  const int W = gridDim.x * nwb;
  const int gw = blockIdx.x * nwb + wave;
  // G slab groups of spg slabs per tile (the host's split)
  const int64_t npairs = (int64_t)nch * G;
  const int nsteps = (Kp + 63) / 64;
  const __bf16* cb = Cs + n * KCS + 8 * g;
  // per-wave T staging area (TS), after H3^T and its tail
  constexpr int TSS = FP + 4;
  float* Ts = reinterpret_cast<float*>(smem_raw + ((size_t)FP * KCS + kPass1Tail) * 2) + wave * R * TSS;
  const __amdgpu_buffer_rsrc_t hrs = uniform_rsrc(Hb, J * F * 4);
  // byte offset of column f = 16 ft + n in a row of T (past F: kBufferOOB);
  // OR-ed with gmask it is the offset in the W1 partial, which lane group 0
  // stores (for the others it is at least kBufferOOB)
  int fo[FT];
#pragma unroll
  for (int ft = 0; ft < FT; ++ft) fo[ft] = ft * 16 + n < F ? (ft * 16 + n) * 4 : kBufferOOB;
  const int gmask = g == 0 ? 0 : kBufferOOB;

  for (int64_t pr = gw; pr < npairs; pr += W) {
    // (said to be wave-uniform: slab indices then live in scalar registers
    // and the slab scale is a scalar load, outside the vector-load count)
    const int ch = __builtin_amdgcn_readfirstlane((int)(pr % nch));
    const int i0 = __builtin_amdgcn_readfirstlane((int)(pr / nch) * spg);
    const int ns = min(I, i0 + spg) - i0;
    const int total = ns * nsteps;   // >= 1

    // H2 values of the tile (zeros past J and F), loaded before the run's
    // first tensor loads: the wait before the first step covers them
    float hbv[MT][FT][4];
    // byte offset of the tile row (mt, ii) of this lane in a [J][F] slab
    const int tb = (ch * R + 4 * g) * F * 4;
    auto trow = [&](int mt, int ii) { return tb + (mt * 16 + ii) * F * 4; };
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int ii = 0; ii < 4; ++ii)
#pragma unroll
        for (int ft = 0; ft < FT; ++ft)
          hbv[mt][ft][ii] = __builtin_bit_cast(
              float, __builtin_amdgcn_raw_buffer_load_b32(
                         hrs, (int)((unsigned)trow(mt, ii) + (unsigned)fo[ft]), 0, 0));

    // load cursor: (slab l_sl of the run, super step at column l_kb); lane
    // (n, g) reads the 8 columns kk = l_kb + 32h + 8g .. of its row as one
    // 16-byte piece of the k-grouped copy; rows past J and columns past Kp
    // take offsets with bit 31 set (past the resource: zeros)
    int l_off[MT];
    unsigned l_past[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int j = ch * R + mt * 16 + n;
      l_off[mt] = (g * J + j) * 16;
      l_past[mt] = (unsigned)(J - 1 - j) & 0x80000000u;
    }
    int l_sl = 0, l_kb = 0;
    bf16x8 xv[U][2][MT];
    auto load_next = [&](bf16x8 (&dst)[2][MT]) {
      const bool tail = l_kb + 64 > Kp;   // wave-uniform
      const __amdgpu_buffer_rsrc_t l_rs = uniform_rsrc(Xr + (int64_t)(i0 + l_sl) * J * Kp, J * Kp * 2);
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          unsigned off = ((unsigned)l_off[mt] + (unsigned)(((l_kb + 32 * h) >> 3) * J * 16)) | l_past[mt];
          if (tail && l_kb + 8 * g + 32 * h >= Kp) off = kBufferOOB;
          dst[h][mt] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(l_rs, (int)off, 0, 0));
        }
      l_kb += 64;
      const bool wrap = l_kb >= Kp;
      l_kb = wrap ? 0 : l_kb;
      l_sl += (wrap && l_sl + 1 < ns) ? 1 : 0;   // past the run's end: stay on its last slab
    };
#pragma unroll
    for (int u = 0; u < U; ++u) load_next(xv[u]);

    f32x4 acc[MT][FT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int ft = 0; ft < FT; ++ft) acc[mt][ft] = f32x4{0.f, 0.f, 0.f, 0.f};
    int c_sl = 0, c_step = 0;
    auto step = [&](int u, bool reload) {
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
      if (reload) load_next(xv[u]);
      const bool last = c_step + 1 == nsteps;
      if (last) {
        // epilogue of slab i: T rows (scale folded in) and the W1 partial of
        // (i, ch), reduced over the 4 lane groups and stored by group 0
        const int i = __builtin_amdgcn_readfirstlane(i0 + c_sl);
        const float sc = scale[i];
        const __amdgpu_buffer_rsrc_t trs = uniform_rsrc(Tout + (int64_t)i * J * F, J * F * 4);
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
              if constexpr (TS) {
                Ts[(mt * 16 + 4 * g + ii) * TSS + ft * 16 + n] = v;
              } else {
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), trs,
                                                      (int)((unsigned)trow(mt, ii) + (unsigned)fo[ft]), 0, 0);
              }
              part[ft] += hbv[mt][ft][ii] * v;
            }
            acc[mt][ft] = f32x4{0.f, 0.f, 0.f, 0.f};
          }
        if constexpr (TS) {
          // lane l stores columns 4(l % 16) .. +3 of row 4q + l / 16 of the
          // tile (rows of one wave's LDS area: its own writes, in order)
          const int cq = 4 * (lane & 15), rq = lane >> 4;
          const int co = cq < F ? cq * 4 : kBufferOOB;
#pragma unroll
          for (int q = 0; q < R / 4; ++q) {
            const int r = 4 * q + rq;
            const f32x4 v = *reinterpret_cast<const f32x4*>(Ts + r * TSS + cq);
            // (non-temporal: T is written once here and read once by the
            // mode-2 pass; measured 2% faster than ordinary stores)
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), trs,
                                                   (int)((unsigned)((ch * R + r) * F * 4) + (unsigned)co), 0,
                                                   kAuxNonTemporal);
          }
        }
        const __amdgpu_buffer_rsrc_t prs = uniform_rsrc(P1 + ((int64_t)i * nch + ch) * F, F * 4);
#pragma unroll
        for (int ft = 0; ft < FT; ++ft) {
          part[ft] += __shfl_xor(part[ft], 16);
          part[ft] += __shfl_xor(part[ft], 32);
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, part[ft]), prs, fo[ft] | gmask, 0, 0);
        }
      }
      // (both counters assigned on every path, so they stay in registers)
      c_sl += last ? 1 : 0;
      c_step = last ? 0 : c_step + 1;
    };
    const int full = total - total % U;
    for (int s0 = 0; s0 < full; s0 += U) {
#pragma unroll
      for (int u = 0; u < U; ++u) step(u, true);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (full + u < total) step(u, false);
  }
}

// Streaming form of the FP32 pass 1 (all of H3 in LDS, rows of a length
// divisible by V = 4 or 2): items as in k_pass1, one load cursor per wave
// running U super steps (32 k) ahead across its items through a buffer
// resource per slab; rows j >= J and k >= K read as zeros, so every path
// issues the same loads and the wait before a step covers that step only.
// Lane group g of half h of a super step holds k = 16h + 4g .. 16h + 4g + 3,
// so each load instruction reads 64 contiguous bytes of 16 rows (with
// k = 8g + 4h it read 16-byte pieces spread over 128 bytes: 0.687 -> 0.669
// ms per outer iteration of the 120x110x100x90 workload, 1.426 -> 1.412 ms
// at 1000x800x600 F = 64).
// Offsets past the data carry bit 31 (an offset no resource reaches), taken
// from the sign of (limit - 1 - index) by plain integer arithmetic: a
// select against a constant offset, or a comparison, lets the compiler split
// the lanes into two loads into one register on divergent paths, each
// followed by a wait for every load in flight.  The item cursors (slab, row
// chunk) step by the grid stride in 32-bit scalar arithmetic.
template <int FT, int MT, int V>
__global__ __launch_bounds__(512, 2) void k_pass1s(const float* __restrict__ X, int I, int J, int K,
                                                   int F, const float* __restrict__ Hb,
                                                   const float* __restrict__ Hc,
                                                   float* __restrict__ Tout, float* __restrict__ P1,
                                                   int nch, int KC) {
  typedef Mfma<float> M;
  typedef typename M::acc_t acc_t;
  constexpr int FP = FT * 16;
  constexpr int R = 16 * MT;
  constexpr int U = 4;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* Cs = reinterpret_cast<float*>(smem_raw);
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n = lane & 15, g = lane >> 4;
  for (int idx = threadIdx.x; idx < KC * FP; idx += blockDim.x) {
    const int kk = idx / FP, f = idx - kk * FP;
    const float v = (kk < K && f < F) ? Hc[(int64_t)kk * F + f] : 0.f;
    Cs[((kk >> 2) * FP + f) * 4 + (kk & 3)] = v;
  }
  __syncthreads();
  const int64_t nitems = (int64_t)I * nch;
  const int nwb = blockDim.x >> 6;
  const int64_t stride = (int64_t)gridDim.x * nwb;
  const int64_t first = (int64_t)blockIdx.x * nwb + wave;
  if (first >= nitems) return;
  const int64_t myitems = (nitems - first + stride - 1) / stride;
  const int nsteps = (K + 31) / 32;
  const int total = __builtin_amdgcn_readfirstlane((int)(myitems * nsteps));
  // item = slab * nch + chunk; the grid stride as (slabs, chunks)
  const int sd = __builtin_amdgcn_readfirstlane((int)(stride / nch));
  const int sr = __builtin_amdgcn_readfirstlane((int)(stride - (int64_t)sd * nch));
  const int i_first = __builtin_amdgcn_readfirstlane((int)(first / nch));
  const int ch_first = __builtin_amdgcn_readfirstlane((int)(first - (int64_t)i_first * nch));
  auto advance = [&](int& i, int& ch) {
    ch += sr;
    i += sd;
    if (ch >= nch) {
      ch -= nch;
      ++i;
    }
  };
  constexpr unsigned kPast = 0x80000000u;   // bit 31: past every resource
  // kPast when idx >= lim (both non-negative and below 2^31), else 0
  auto past = [](int idx, int lim) { return (unsigned)(lim - 1 - idx) & kPast; };

  // load cursor (the cursor stays on the last item past the wave's end and
  // re-reads in-bounds data that nothing consumes)
  int l_i = i_first, l_ch = ch_first;
  int l_kb = 0;
  const float* l_slab = X + (int64_t)l_i * J * K;
  float xv[U][2][MT][4];
  auto load_next = [&](float (&dst)[2][MT][4]) {
    const __amdgpu_buffer_rsrc_t rs = uniform_rsrc(l_slab, J * K * 4);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int k = l_kb + 16 * h + 4 * g;   // (16 rows x 64 contiguous bytes per instruction)
        const int row = l_ch * R + mt * 16 + n;
        const unsigned base = (unsigned)(row * K + k) * 4u;
        const unsigned rmask = past(row, J);
        if constexpr (V == 4) {
          const int off = (int)(base | rmask | past(k, K));
          const f32x4 v = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
#pragma unroll
          for (int c = 0; c < 4; ++c) dst[h][mt][c] = v[c];
        } else {
          typedef float f2 __attribute__((ext_vector_type(2)));
          const int o0 = (int)(base | rmask | past(k, K));
          const int o1 = (int)((base + 8u) | rmask | past(k + 2, K));
          const f2 a = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(rs, o0, 0, 0));
          const f2 b = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(rs, o1, 0, 0));
          dst[h][mt][0] = a[0];
          dst[h][mt][1] = a[1];
          dst[h][mt][2] = b[0];
          dst[h][mt][3] = b[1];
        }
      }
    l_kb += 32;
    if (l_kb >= K) {
      l_kb = 0;
      int ni = l_i, nc = l_ch;
      advance(ni, nc);
      if (ni < I) {
        l_i = ni;
        l_ch = nc;
        l_slab = X + (int64_t)l_i * J * K;
      }
    }
  };
#pragma unroll
  for (int u = 0; u < U; ++u) load_next(xv[u]);

  acc_t acc[MT][FT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) acc[mt][ft] = M::zero();
  int c_i = i_first, c_ch = ch_first;
  int c_step = 0;
  const __amdgpu_buffer_rsrc_t hrs = uniform_rsrc(Hb, J * F * 4);
  float hbv[MT][FT][4];
  auto eoff = [&](int ch, int mt, int ft, int ii) {   // offset of (row, column) in a [J][F] slab
    const int j = ch * R + mt * 16 + M::row(g, ii), f = ft * 16 + n;
    return (int)(((unsigned)(j * F + f) * 4u) | past(f, F) | past(j, J));
  };
  auto item_start = [&](int ch) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int ft = 0; ft < FT; ++ft)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii)
          hbv[mt][ft][ii] = __builtin_bit_cast(
              float, __builtin_amdgcn_raw_buffer_load_b32(hrs, eoff(ch, mt, ft, ii), 0, 0));
  };
  auto step = [&](int u, bool reload) {
    if (c_step == 0) item_start(c_ch);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const float* cbase = Cs + (((c_step * 32) >> 2) + 4 * h + g) * FP * 4 + n * 4;
#pragma unroll
      for (int ft = 0; ft < FT; ++ft) {
        float cv[4];
        Vec4Load<float>::load(cbase + ft * 64, cv);
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) acc[mt][ft] = M::mma(xv[u][h][mt][c], cv[c], acc[mt][ft]);
      }
    }
    if (reload) load_next(xv[u]);
    if (++c_step == nsteps) {
      // epilogue of item c_item: T rows (rows past J and columns past F get
      // an offset past the slab: the hardware drops those stores; with no T
      // output the resource is empty and drops them all) and this item's
      // share of W1 against H2
      const int i = c_i, ch = c_ch;
      const __amdgpu_buffer_rsrc_t trs =
          Tout ? uniform_rsrc(Tout + (int64_t)i * J * F, J * F * 4) : uniform_rsrc(P1, 0);
      float part[FT];
#pragma unroll
      for (int ft = 0; ft < FT; ++ft) part[ft] = 0.f;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int ft = 0; ft < FT; ++ft) {
#pragma unroll
          for (int ii = 0; ii < 4; ++ii) {
            const float v = acc[mt][ft][ii];
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), trs,
                                                  eoff(ch, mt, ft, ii), 0, 0);
            part[ft] += hbv[mt][ft][ii] * v;
          }
          acc[mt][ft] = M::zero();
        }
#pragma unroll
      for (int ft = 0; ft < FT; ++ft) {
        part[ft] += __shfl_xor(part[ft], 16);
        part[ft] += __shfl_xor(part[ft], 32);
        const int f = ft * 16 + n;
        if (g == 0 && f < F) P1[((int64_t)i * nch + ch) * F + f] = part[ft];
      }
      c_step = 0;
      advance(c_i, c_ch);
    }
  };
  const int full = total - total % U;
  for (int s0 = 0; s0 < full; s0 += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) step(u, true);
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (full + u < total) step(u, false);
}

// ---------------------------------------------------------------- mode 2 from T

// P2[ic][j][f] = sum_{i in chunk ic} A[i][f] * T[i][j][f]; one thread per (j,f),
// coalesced over the contiguous (j,f) index of each slab of T.
// FP32 with F a multiple of 4: four consecutive columns per thread (16-byte
// loads of T and of the A row), the slabs of the partial loaded eight at a
// time before their products are added in slab order, one fused multiply-add
// per slab and column as in k_mode2 (so the partials are bitwise the same).
__global__ __launch_bounds__(256) void k_mode2v(const float4* __restrict__ Tin,
                                                const float4* __restrict__ Ha, int I, int64_t JF4,
                                                int F4, int ich, float4* __restrict__ P2) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= JF4) return;
  const int f4 = (int)(idx % F4);
  const int ic = blockIdx.y;
  const int i0 = ic * ich, i1 = min(I, i0 + ich);
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int ib = i0; ib < i1; ib += 8) {
    float4 tv[8], av[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = min(ib + q, i1 - 1);   // (past the partial's end: loaded, not used)
      tv[q] = Tin[(int64_t)i * JF4 + idx];
      av[q] = Ha[(int64_t)i * F4 + f4];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (ib + q < i1) {
        acc.x = __builtin_fmaf(av[q].x, tv[q].x, acc.x);
        acc.y = __builtin_fmaf(av[q].y, tv[q].y, acc.y);
        acc.z = __builtin_fmaf(av[q].z, tv[q].z, acc.z);
        acc.w = __builtin_fmaf(av[q].w, tv[q].w, acc.w);
      }
    }
  }
  P2[(int64_t)ic * JF4 + idx] = acc;
}

template <typename T>
__global__ __launch_bounds__(256) void k_mode2(const T* __restrict__ Tin, const T* __restrict__ Ha,
                                               int I, int64_t JF, int F, int ich,
                                               T* __restrict__ P2) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= JF) return;
  const int f = (int)(idx % F);
  const int ic = blockIdx.y;
  const int i0 = ic * ich, i1 = min(I, i0 + ich);
  T acc = T(0);
  for (int i = i0; i < i1; ++i) acc += Ha[(int64_t)i * F + f] * Tin[(int64_t)i * JF + idx];
  P2[(int64_t)ic * JF + idx] = acc;
}

// ---------------------------------------------------------------- pass 3, FP32 / FP64

// Block = nw waves; wave w covers k in [kw0, kw0+64) with four MFMA instances
// c = 0..3 whose result row m holds k = kw0 + 4m + c (the 16-byte X load of
// lane (n,g) covers k = kw0 + 4n .. +3 of row r0 + g).  Rows r = i*J + j of the
// block's chunk are contracted 64 at a time; their Khatri-Rao rows
// KR[r][f] = A[i][f] * B[j][f] are built in LDS (double buffered: the next
// 64 rows are built while the current ones are contracted, one barrier per
// 64 rows) and shared by all waves.  X loads run two steps ahead.
template <typename T, int FT>
__global__ __launch_bounds__(512) void k_pass3(const T* __restrict__ X, int64_t IJ, int J, int K,
                                               int F, const T* __restrict__ Ha,
                                               const T* __restrict__ Hb, T* __restrict__ P3,
                                               int64_t rpc, int vec) {
  typedef Mfma<T> M;
  typedef typename M::acc_t acc_t;
  constexpr int FP = FT * 16;
  constexpr int KRS = FP + ((FT % 2 == 0) ? 16 : 0);  // LDS row stride: 4 lane groups on distinct banks
  __shared__ __align__(16) T KRs[2][64 * KRS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n = lane & 15, g = lane >> 4;
  const int nw = blockDim.x >> 6;
  const int kw0 = (blockIdx.y * nw + wave) * 64;
  const int64_t rbeg = (int64_t)blockIdx.x * rpc;
  const int64_t rend = min(IJ, rbeg + rpc);
  const int nep = (int)((rend - rbeg + 63) >> 6);
  acc_t acc[4][FT];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) acc[c][ft] = M::zero();
  const int kl = kw0 + 4 * n;           // first k of this lane's 16-byte load
  const int valid = K - kl;
  const bool kact = kw0 < K;
  auto build = [&](int e, int buf) {
    const int64_t r0 = rbeg + 64LL * e;
    for (int idx = threadIdx.x; idx < 64 * FP; idx += blockDim.x) {
      const int rr = idx / FP, f = idx - rr * FP;
      const int64_t r = r0 + rr;
      T v = T(0);
      if (r < rend && f < F) {
        const int64_t i = r / J, j = r - i * J;
        v = Ha[i * F + f] * Hb[j * F + f];
      }
      KRs[buf][rr * KRS + f] = v;
    }
  };
  auto load = [&](int64_t r, T (&dst)[4]) {
    if (kact && r < rend && valid > 0) {
      load4<T>(X + r * K + kl, valid, vec, dst);
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) dst[c] = T(0);
    }
  };
  if (nep > 0) build(0, 0);
  __syncthreads();
  for (int e = 0; e < nep; ++e) {
    const int64_t r0 = rbeg + 64LL * e;
    if (e + 1 < nep) build(e + 1, (e + 1) & 1);
    if (kact) {
      const T* kbuf = KRs[e & 1];
      T xv[2][4];
      load(r0 + g, xv[0]);
      load(r0 + 4 + g, xv[1]);
#pragma unroll
      for (int st = 0; st < 16; ++st) {
        const T* kb = kbuf + (4 * st + g) * KRS + n;
#pragma unroll
        for (int ft = 0; ft < FT; ++ft) {
          const T b = kb[ft * 16];
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[c][ft] = M::mma(xv[st & 1][c], b, acc[c][ft]);
        }
        if (st + 2 < 16) load(r0 + 4 * (st + 2) + g, xv[st & 1]);
      }
    }
    __syncthreads();
  }
  if (!kact) return;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int ft = 0; ft < FT; ++ft)
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int k = kw0 + 4 * M::row(g, ii) + c;
        const int f = ft * 16 + n;
        if (k < K && f < F) P3[((int64_t)blockIdx.x * K + k) * F + f] = acc[c][ft][ii];
      }
}

// Streaming form of pass 3 (FP32, rows of a length divisible by V = 4 or 2;
// eight waves per block): each wave's load cursor runs U steps ahead over
// the block's rows, across the 64-row epochs, through a buffer resource over
// those rows, and rows past the block's end or columns past K read as zeros,
// so every path issues the same loads (the compiler's wait before a step
// then covers that step only).  The Khatri-Rao values of epoch e + 2 are
// loaded during epoch e + 1's predecessor and stored to the free LDS buffer
// after the epoch's MFMAs; each step's B operands are read one step ahead.
// With few 64-column k tiles (K <= 256) the waves also split the rows: RG row
// groups of 8 / RG waves each (wave -> k tile wave % (8 / RG), row group
// wave / (8 / RG)), group rg taking steps rg * 16/RG .. of every epoch, and
// each group writes a partial of its own (P3 partial blockIdx.x * RG + rg),
// so every wave streams X instead of two of eight.
template <typename T, int FT, int V, int RG>
__global__ __launch_bounds__(512, 2) void k_pass3s(const T* __restrict__ X, int64_t IJ, int J, int K,
                                                int F, const T* __restrict__ Ha,
                                                const T* __restrict__ Hb, T* __restrict__ P3,
                                                int64_t rpc, int I) {
  static_assert(sizeof(T) == 4, "FP32 only");
  typedef Mfma<T> M;
  typedef typename M::acc_t acc_t;
  constexpr int FP = FT * 16;
  constexpr int KRS = FP + ((FT % 2 == 0) ? 16 : 0);
  constexpr int U = 4;
  constexpr int PER = 64 * FP / 512;     // Khatri-Rao entries per thread and epoch (512 threads)
  __shared__ __align__(16) T KRs[2][64 * KRS];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, n = lane & 15, g = lane >> 4;
  constexpr int KT = 8 / RG;            // k tiles per block (eight waves)
  constexpr int SPW = 16 / RG;          // steps of an epoch per wave
  constexpr int UU = SPW < U ? SPW : U;
  constexpr int EPG = U / UU;           // epochs per loop turn (the load ring stays compile-time)
  const int kt = wave % KT, rg = wave / KT;
  const int kw0 = (blockIdx.y * KT + kt) * 64;
  const bool kact = kw0 < K;
  const int64_t rbeg = (int64_t)blockIdx.x * rpc;
  const int nrows = (int)(min(IJ, rbeg + rpc) - rbeg);
  // (epochs past the block's rows read zeros: their products add exact zeros)
  const int nep = (((nrows + 63) >> 6) + EPG - 1) / EPG * EPG;
  const int kl = kw0 + 4 * n;
  const __amdgpu_buffer_rsrc_t xrs = uniform_rsrc(X + rbeg * K, nrows * K * (int)sizeof(T));
  const __amdgpu_buffer_rsrc_t ars = uniform_rsrc(Ha, I * F * (int)sizeof(T));
  const __amdgpu_buffer_rsrc_t brs = uniform_rsrc(Hb, J * F * (int)sizeof(T));
  acc_t acc[4][FT];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) acc[c][ft] = M::zero();

  T xv[U][4];
  auto xload = [&](int st, T (&dst)[4]) {
    const int row = 4 * st + g;
    const bool rok = row < nrows;
    if constexpr (sizeof(T) == 4 && V == 4) {
      const int off = (rok && kl < K) ? (row * K + kl) * 4 : kBufferOOB;
      const f32x4 v = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(xrs, off, 0, 0));
#pragma unroll
      for (int c = 0; c < 4; ++c) dst[c] = v[c];
    } else {
      typedef float f2 __attribute__((ext_vector_type(2)));
      const int o0 = (rok && kl < K) ? (row * K + kl) * 4 : kBufferOOB;
      const int o1 = (rok && kl + 2 < K) ? (row * K + kl + 2) * 4 : kBufferOOB;
      const f2 a = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(xrs, o0, 0, 0));
      const f2 b = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(xrs, o1, 0, 0));
      dst[0] = a[0];
      dst[1] = a[1];
      dst[2] = b[0];
      dst[3] = b[1];
    }
  };
  T ha[PER], hb[PER];
  auto hload = [&](int e) {   // factor values of epoch e (zeros past the block's rows)
    // (i, j) of the epoch's first row once per epoch (uniform), then 32-bit
    // steps: rows of one epoch advance j by at most 63
    const int64_t re = rbeg + 64LL * e;
    const int ie = (int)(re / J), je = (int)(re - (int64_t)ie * J);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + nthr * q;
      const int rr = idx / FP, f = idx - rr * FP;
      const bool ok = idx < 64 * FP && (64 * e + rr < nrows) && f < F;
      int i = ie, j = je + rr;
      while (j >= J) {   // (at most 63 / J + 1 times)
        j -= J;
        ++i;
      }
      const int oa = ok ? (i * F + f) * (int)sizeof(T) : kBufferOOB;
      const int ob = ok ? (j * F + f) * (int)sizeof(T) : kBufferOOB;
      ha[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ars, oa, 0, 0));
      hb[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(brs, ob, 0, 0));
    }
  };
  auto hstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + nthr * q;
      const int rr = idx / FP, f = idx - rr * FP;
      if (idx < 64 * FP) KRs[buf][rr * KRS + f] = ha[q] * hb[q];
    }
  };
  // the wave's w-th step is step rg * SPW + w % SPW of epoch w / SPW
  auto sabs = [&](int w) { return 16 * (w / SPW) + rg * SPW + (w % SPW); };
  hload(0);
  hstore(0);
  hload(1);
#pragma unroll
  for (int u = 0; u < U; ++u) xload(sabs(u), xv[u]);
  __syncthreads();
  for (int e0 = 0; e0 < nep; e0 += EPG) {
#pragma unroll
    for (int ee = 0; ee < EPG; ++ee) {
      const int e = e0 + ee;
      const T* kb0 = KRs[e & 1] + g * KRS + n + (4 * rg * SPW) * KRS;
      T bc[FT], bn[FT];
#pragma unroll
      for (int ft = 0; ft < FT; ++ft) bc[ft] = kb0[ft * 16];
#pragma unroll 1
      for (int st0 = 0; st0 < SPW; st0 += UU) {
#pragma unroll
        for (int u = 0; u < UU; ++u) {
          const int st = st0 + u;
          const int slot = ee * UU + u;          // = (e * SPW + st) % U
          const int sn = min(st + 1, SPW - 1);   // the last step re-reads its own operands
#pragma unroll
          for (int ft = 0; ft < FT; ++ft) bn[ft] = kb0[(4 * sn) * KRS + ft * 16];
          if (kact) {
#pragma unroll
            for (int ft = 0; ft < FT; ++ft)
#pragma unroll
              for (int c = 0; c < 4; ++c) acc[c][ft] = M::mma(xv[slot][c], bc[ft], acc[c][ft]);
          }
          xload(sabs(e * SPW + st + U), xv[slot]);
#pragma unroll
          for (int ft = 0; ft < FT; ++ft) bc[ft] = bn[ft];
        }
      }
      if (e + 1 < nep) hstore((e + 1) & 1);
      hload(e + 2);
      __syncthreads();
    }
  }
  if (!kact) return;
  const int64_t part = (int64_t)blockIdx.x * RG + rg;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int ft = 0; ft < FT; ++ft)
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int k = kw0 + 4 * M::row(g, ii) + c;
        const int f = ft * 16 + n;
        if (k < K && f < F) P3[(part * K + k) * F + f] = acc[c][ft][ii];
      }
}

// ---------------------------------------------------------------- pass 3, BF16

// Mode-3 MTTKRP in split factored form: W3[k,:] = sum_i s_i A[i,:] *
// (sum_j Xq[i,j,k] (hi[j,:] + lo[j,:])), with H2 carried as two bfloat16
// terms hi = bf16(B), lo = bf16(B - hi) (one rounding of B shared by every
// slab would bias all slabs alike).  The inner sum is an MFMA contraction
// over j whose B operands do not depend on the slab, so a block stages hi^T
// and lo^T for one chunk of 8-row groups of j in LDS once ([FP][JCS] each,
// zero past J and past the chunk), and every step issues two MFMAs per
// operand pair.  X comes from the j-interleaved copy
// Xj8[q][k][e] (q = i*JG + jg, row j = 8jg + e): lane (n,g) of a 32-row step
// loads the 8 rows of group 4*step + g at row k with one 16-byte read, which
// is exactly the A operand of v_mfma_f32_16x16x32_bf16.  Each wave owns 64
// rows of k (four 16-row tiles) and a run of slabs, walked as one continuous
// sequence of (slab, step) with U steps of loads in flight through a buffer
// resource per (slab, chunk): groups past the chunk and rows past Kp3 read
// as zeros, so every path issues the same loads.  At the end of a slab the
// FP32 products are scaled by s_i A[i,f] (loaded when the slab starts) and
// added to the wave's running sums, which go to the partial of its (chunk,
// slab group): P3[chunk * ngroups + group][K][F].
template <int FT>
__global__ __launch_bounds__(512) void k_pass3_bf16s(const __bf16* __restrict__ Xj8,
                                                     const float* __restrict__ scale, int I, int J,
                                                     int JG, int K, int Kp3, int F,
                                                     const float* __restrict__ Ha,
                                                     const float* __restrict__ Hb,
                                                     float* __restrict__ P3, int nkt, int spg,
                                                     int ngroups, int jcg, int bpc) {
  constexpr int FP = FT * 16;
  constexpr int MT = 4;
  // (two steps in flight: measured 204 us against 209 with four, 242 with six)
  constexpr int U = 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __bf16* Bs = reinterpret_cast<__bf16*>(smem_raw);
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n = lane & 15, g = lane >> 4;
  const int c = blockIdx.x / bpc, lb = blockIdx.x - c * bpc;
  const int jg0 = c * jcg, ng = min(jcg, JG - jg0);
  const int nsteps = (ng + 3) >> 2;
  const int JL = 32 * nsteps;                  // staged rows of this chunk (whole steps)
  const int JCS = 32 * ((jcg + 3) >> 2) + 8;   // LDS row stride, a 16-byte multiple
  const int gw = lb * (int)(blockDim.x >> 6) + wave;
  const int grp = gw / nkt, kt = gw - grp * nkt;
  const int i0 = grp * spg;
  const int ns = grp < ngroups ? min(I, i0 + spg) - i0 : 0;
  const int total = __builtin_amdgcn_readfirstlane(ns * nsteps);

  // load cursor: (slab l_sl of the run, step l_st of the chunk); past the
  // end it stays on the run's last slab (in-bounds reads nothing consumes).
  // Rows k >= Kp3 get a byte offset of at least kBufferOOB, groups past the
  // chunk an offset past the (slab, chunk) resource: both read as zeros, and
  // every step issues the same loads, so the wait before a step covers that
  // step's loads only.  Each step also loads the A row of its slab (lane l:
  // A[i, l]); the slab's last step takes its coefficients from it.
  int kof[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int k = kt * 64 + mt * 16 + n;
    kof[mt] = k < Kp3 ? k * 16 : kBufferOOB;
  }
  const int aof = lane < F ? lane * 4 : kBufferOOB;
  const int chunk_bytes = ng * Kp3 * 16, gstride = Kp3 * 16;
  int l_sl = 0, l_st = 0;
  bf16x8 xv[U][MT];
  float ar[U];
  auto load_next = [&](bf16x8 (&dst)[MT], float& adst) {
    const int i = i0 + l_sl;
    const __amdgpu_buffer_rsrc_t ars = uniform_rsrc(Ha + (int64_t)i * F, F * 4);
    adst = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ars, aof, 0, 0));
    const __amdgpu_buffer_rsrc_t rs =
        uniform_rsrc(Xj8 + ((int64_t)i * JG + jg0) * Kp3 * 8, chunk_bytes);
    const int qoff = (4 * l_st + g) * gstride;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
      dst[mt] = __builtin_bit_cast(
          bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)((unsigned)qoff + (unsigned)kof[mt]), 0, 0));
    if (++l_st == nsteps) {
      l_st = 0;
      if (l_sl + 1 < ns) ++l_sl;
    }
  };
  // the first U steps go out before the chunk of H2^T is staged
  if (total > 0) {
#pragma unroll
    for (int u = 0; u < U; ++u) load_next(xv[u], ar[u]);
  }
  __bf16* Bl = Bs + FP * JCS;   // the lo tile after the hi tile
  for (int idx = threadIdx.x; idx < JL * FP; idx += blockDim.x) {
    const int jj = idx / FP, f = idx - jj * FP;
    const int j = jg0 * 8 + jj;
    const float v = (jj < 8 * ng && j < J && f < F) ? Hb[(int64_t)j * F + f] : 0.f;
    const __bf16 hi = (__bf16)v;
    Bs[f * JCS + jj] = hi;
    Bl[f * JCS + jj] = (__bf16)(v - (float)hi);   // (the difference is exact in FP32)
  }
  __syncthreads();
  if (total == 0) return;

  f32x4 acc[MT][FT], tot[MT][FT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) {
      acc[mt][ft] = f32x4{0.f, 0.f, 0.f, 0.f};
      tot[mt][ft] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  int c_sl = 0, c_st = 0;
  const __bf16* bb = Bs + n * JCS + 8 * g;
  auto step = [&](int u, bool reload) {
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) {
      const bf16x8 bh = *reinterpret_cast<const bf16x8*>(bb + ft * 16 * JCS + c_st * 32);
      const bf16x8 bl = *reinterpret_cast<const bf16x8*>(bb + FP * JCS + ft * 16 * JCS + c_st * 32);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt][ft] = mma_bf16(xv[u][mt], bh, acc[mt][ft]);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt][ft] = mma_bf16(xv[u][mt], bl, acc[mt][ft]);
    }
    // (the coefficients are read out of ar[u] before its reload, so the
    // reload can write the same registers: no copy, no wait, at the loop end)
    const bool last = c_st + 1 == nsteps;
    float coef[FT];
    if (last) {
      const float sc = scale[i0 + c_sl];
#pragma unroll
      for (int ft = 0; ft < FT; ++ft) coef[ft] = sc * __shfl(ar[u], ft * 16 + n);
    }
    if (reload) load_next(xv[u], ar[u]);
    if (last) {
#pragma unroll
      for (int ft = 0; ft < FT; ++ft)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
          for (int ii = 0; ii < 4; ++ii) tot[mt][ft][ii] += coef[ft] * acc[mt][ft][ii];
          acc[mt][ft] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    }
    // (both counters assigned on every path: an increment of one or the
    // other in two branches becomes a store through a pointer select, and
    // the counters then live in scratch memory)
    c_sl += last ? 1 : 0;
    c_st = last ? 0 : c_st + 1;
  };
  const int full = total - total % U;
  for (int s0 = 0; s0 < full; s0 += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) step(u, true);
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (full + u < total) step(u, false);

  // the wave's 64 rows of the partial (rows past K, columns past F: dropped)
  const int krows = min(64, K - kt * 64);
  const __amdgpu_buffer_rsrc_t wrs =
      uniform_rsrc(P3 + ((int64_t)(c * ngroups + grp) * K + kt * 64) * F, krows * F * 4);
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int ft = 0; ft < FT; ++ft)
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int r = mt * 16 + 4 * g + ii;
        const int f = ft * 16 + n;
        // (the element is copied to a scalar first: a bit cast of a vector
        // element lvalue reads element 0 with this compiler)
        const float t = tot[mt][ft][ii];
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, t), wrs,
                                              (r < krows && f < F) ? (r * F + f) * 4 : kBufferOOB, 0, 0);
      }
}

// ---------------------------------------------------------------- partial reduction

// Fixed-order grouped reduction: partial p goes to group p % G, each group
// sums its partials in increasing p, and the G group sums are added in
// increasing group order.  Block = 64 elements x G groups.
template <typename PT, int G>
__global__ __launch_bounds__(64 * G) void k_reduce_grouped(const PT* __restrict__ part,
                                                           int64_t pstride, int64_t rowstride,
                                                           int nparts, int64_t rows, int F,
                                                           double* __restrict__ W) {
  __shared__ double red[G][64];
  const int el = threadIdx.x & 63, pg = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + el;
  double s = 0.0;
  if (e < rows * F) {
    const int64_t r = e / F, f = e - r * F;
    s = group_partial(part + r * rowstride + f, pstride, nparts, pg, G);
  }
  red[pg][el] = s;
  __syncthreads();
  if (pg == 0 && e < rows * F) {
    double t = red[0][el];
#pragma unroll
    for (int q = 1; q < G; ++q) t += red[q][el];
    W[e] = t;
  }
}

// ---------------------------------------------------------------- planning and launchers

size_t elem_size(int prec) { return prec == PREC_F64 ? 8 : 4; }

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
static int64_t rup(int64_t a, int64_t b) { return cdiv(a, b) * b; }

static const size_t kLdsBudget = 158 * 1024;

// The BF16 streaming pass 1 applies: H3^T fits LDS whole, and slabs of the
// copy and of T are addressable by one buffer resource each.
static bool stream1_ok(const Plan& p) {
  return p.KC1 >= p.Kp && p.J * p.Kp * 2 < (int64_t)kBufferOOB &&
         (p.J + 32) * p.F * 4 < (int64_t)kBufferOOB;
}

// FP32 pass 1 in the streaming form (k_pass1s): all of H3 in LDS, even rows,
// a slab addressable by one buffer resource
static bool stream1f_ok(const Plan& p) {
  return p.KC1 >= p.K && p.vec >= 2 && p.J * p.K * 4 < (int64_t)kBufferOOB &&
         p.J * p.F * 4 < (int64_t)kBufferOOB;
}

bool make_plan(Plan& p, int prec, const int64_t dims[3], int F, int cu_count) {
  if (F < 1 || F > 64) return false;
  p = Plan();
  p.prec = prec;
  p.I = dims[0];
  p.J = dims[1];
  p.K = dims[2];
  p.F = F;
  p.FT = (F + 15) / 16;
  p.FP = p.FT * 16;
  p.vec = (p.K % 4) == 0 ? 4 : (p.K % 2) == 0 ? 2 : 1;
  const int cus = cu_count > 0 ? cu_count : 256;
  // pass 1: one wave per (slab, 16*MT rows) item, four waves per block
  if (prec == PREC_BF16) {
    p.MT1 = 2;
  } else {
    // MFMA-bound in FP32 at large F: pick the row tile with the least padding
    const int64_t pad1 = cdiv(p.J, 16) * 16, pad2 = cdiv(p.J, 32) * 32;
    p.MT1 = (pad2 - p.J) <= (pad1 - p.J) + p.J / 16 ? 2 : 1;
  }
  p.R1 = 16 * p.MT1;
  p.nch1 = (int)cdiv(p.J, p.R1);
  p.ntiles1 = p.I * p.nch1;
  if (prec == PREC_BF16) {
    p.Kp = rup(p.K, 32);
    p.JG = cdiv(p.J, 8);
    p.Kp3 = rup(p.K, 16);
    const size_t stream_lds = (size_t)p.FP * (p.Kp + 8) * 2 + kPass1Tail * 2;
    // T staging of the streaming form: 8 waves x 32 rows x (FP + 4) floats
    const size_t ts_lds = (size_t)8 * 32 * (p.FP + 4) * 4;
    const int blocks = p.FT <= 2 ? 2 : 1;   // per CU (kPass1Waves)
    if (stream_lds <= kLdsBudget) {
      // streaming form: all of H3^T in LDS, rows Kp + 8 long
      p.KC1 = (int)rup(p.Kp, 64);
      // (not at FT = 2: four waves per SIMD leave no registers for it)
      p.ts1 = (p.F % 4 == 0) && p.FT != 2 && stream_lds + ts_lds <= kLdsBudget &&
              blocks * (stream_lds + ts_lds) <= 160 * 1024;
      p.lds1 = stream_lds + (p.ts1 ? ts_lds : 0);
    } else {
      int64_t kc = rup(p.Kp, 64);
      while ((size_t)p.FP * (kc + 8) * 2 > kLdsBudget) kc = rup(kc / 2, 64);
      p.KC1 = (int)kc;
      p.lds1 = (size_t)p.FP * (kc + 8) * 2;
    }
  } else {
    const size_t es = elem_size(prec);
    int64_t kc = rup(p.K, 32);
    while ((size_t)p.FP * kc * es > kLdsBudget) kc = rup(kc / 2, 32);
    p.KC1 = (int)kc;
    p.lds1 = (size_t)p.FP * kc * es;
  }
  int occ = (int)std::min<size_t>(8, (160 * 1024) / std::max<size_t>(p.lds1 + 512, 1));
  if (prec == PREC_BF16) occ = std::min(occ, p.FT <= 2 ? 2 : 1);   // register-bound (kPass1Waves)
  // the FP32 streaming form is register-bound at two blocks per CU: a larger
  // grid only adds rounds of blocks that each stage H3 and stream a few items
  if (prec == PREC_F32 && stream1f_ok(p)) occ = std::min(occ, 2);
  if (occ < 1) occ = 1;
  p.grid1 = (int)std::min<int64_t>(cdiv(p.ntiles1, 8), (int64_t)cus * occ);
  if (prec == PREC_BF16 && stream1_ok(p)) {
    // streaming form: (row tile, run of spg1 slabs) pairs, G1 runs per tile,
    // about one pair per wave of a full grid; the grid is just large enough
    // for the pairs, so the CUs left over take the prepare step that runs
    // beside the pass instead of delaying one of its blocks
    const int64_t W0 = (int64_t)p.grid1 * 8;
    const int64_t g0 = std::max<int64_t>(1, W0 / p.nch1);
    p.spg1 = (int)cdiv(p.I, g0);
    p.G1 = (int)cdiv(p.I, p.spg1);
    const int64_t pairs = (int64_t)p.nch1 * p.G1;
    p.grid1 = (int)std::max<int64_t>(1, std::min<int64_t>(p.grid1, cdiv(pairs, 8)));
  }
  // mode 2 from T
  p.ich2 = 16;
  p.nich2 = (int)cdiv(p.I, p.ich2);
  // pass 3: k split into 64-column wave tiles.  FP32/FP64: at most 8 waves per
  // block, balanced over ceil(tiles/8) k-groups, row chunks for about two
  // blocks per CU.  BF16: see below.
  const int64_t kspan = (prec == PREC_BF16) ? p.Kp3 : p.K;
  const int ktiles = (int)cdiv(kspan, 64);
  if (prec == PREC_BF16) {
    // one block of 8 waves per CU; a wave owns 64 rows of k and a run of
    // slabs of one chunk of j, the chunk's bf16 hi and lo tiles of H2^T in LDS
    p.nkt3 = ktiles;
    // (two bfloat16 tiles, hi and lo of H2^T)
    auto lds_of = [&](int64_t q) { return (size_t)2 * p.FP * (32 * cdiv(q, 4) + 8) * 2; };
    int64_t jcg = p.JG;
    // (a chunk's byte offsets, three groups past its end included, stay
    // below 2^31, so an offset plus kBufferOOB does not wrap)
    auto fits = [&](int64_t q) {
      return lds_of(q) <= kLdsBudget && (q + 4) * p.Kp3 * 16 < (int64_t)kBufferOOB;
    };
    while (jcg > 4 && !fits(jcg)) jcg = rup(cdiv(jcg, 2), 4);
    if (!fits(jcg)) return false;
    p.jcg3 = (int)jcg;
    p.lds3 = lds_of(jcg);
    p.nch3 = (int)cdiv(p.JG, jcg);
    const int64_t waves = (int64_t)cus * 8;
    const int64_t ng = std::max<int64_t>(1, std::min<int64_t>(p.I, waves / ((int64_t)ktiles * p.nch3)));
    p.rpc3 = cdiv(p.I, ng);                 // slabs per group
    p.ngr3 = (int)cdiv(p.I, p.rpc3);
    p.bpc3 = (int)cdiv((int64_t)p.ngr3 * ktiles, 8);
    p.nrc3 = p.nch3 * p.ngr3;               // partials: one per (chunk, group)
  } else {
    p.nkg3 = (int)cdiv(ktiles, 8);
    p.nw3 = (int)cdiv(ktiles, p.nkg3);
    const int64_t units = p.I * p.J;
    int64_t nrc = std::max<int64_t>(1, 2LL * cus / p.nkg3);
    nrc = std::min<int64_t>(nrc, cdiv(units, 64));
    p.rpc3 = rup(cdiv(units, nrc), 64);
    p.nb3 = (int)cdiv(units, p.rpc3);
    // FP32 rows of even length whose block range fits 32-bit buffer offsets
    // take the streaming form, whose waves also split the rows when there
    // are at most four k tiles; one partial per row group of a block
    p.s3 = prec == PREC_F32 && p.vec >= 2 && p.rpc3 * p.K * 4 < kBufferOOB &&
           p.I * p.F * 4 < kBufferOOB && p.J * p.F * 4 < kBufferOOB;
    p.rg3 = !p.s3 ? 1 : ktiles == 1 ? 8 : ktiles == 2 ? 4 : ktiles <= 4 ? 2 : 1;
    p.nrc3 = p.nb3 * p.rg3;
  }
  // inner sweep
  int FL = 4;
  while (FL < F) FL <<= 1;
  p.FL = FL;
  p.rpb = inner_rows_per_block(FL);
  for (int m = 0; m < 3; ++m) p.nblk_inner[m] = (int)cdiv(dims[m], p.rpb);
  p.nprep = (int)std::max<int64_t>(1, cdiv((int64_t)F * F, 64));
  return true;
}

// The k-grouped copy Xr[i][Kp/8][J][8] from the j-grouped one
// Xj8[i][JG][Kp3][8]: both hold an 8 x 8 block (rows 8jg .. 8jg+7, columns
// 8q .. 8q+7) as 128 contiguous bytes, transposed.  A group of 8 lanes takes
// one block: lane l reads column 8q + l (16 bytes), the block goes through
// LDS, and lane e writes row 8jg + e; blocks are numbered ((i, q), jg) with
// jg fastest, so the 32 groups of a workgroup write 4 KB of one plane q in
// order.  Columns past Kp3 are zeros, rows past J are not stored.
__global__ __launch_bounds__(256) void k_xr_from_xj8(const __bf16* __restrict__ Xj8, int J, int JG,
                                                     int Kp, int Kp3, int64_t nblocks,
                                                     __bf16* __restrict__ Xr) {
  __shared__ bf16x8 tile[32][8];
  const int grp = threadIdx.x >> 3, l = threadIdx.x & 7;
  const int64_t t = (int64_t)blockIdx.x * 32 + grp;
  const bool ok = t < nblocks;
  const int NQ = Kp / 8;
  const int64_t iq = ok ? t / JG : 0;                  // slab * NQ + q
  const int jg = ok ? (int)(t - iq * JG) : 0;
  const int64_t slab = iq / NQ;
  const int q = (int)(iq - slab * NQ);
  const bf16x8 z = {};
  const int k = 8 * q + l;
  tile[grp][l] = (ok && k < Kp3)
                     ? *reinterpret_cast<const bf16x8*>(Xj8 + ((slab * JG + jg) * (int64_t)Kp3 + k) * 8)
                     : z;
  __syncthreads();
  const int j = 8 * jg + l;
  if (ok && j < J) {
    bf16x8 o;
#pragma unroll
    for (int r = 0; r < 8; ++r) o[r] = tile[grp][r][l];
    *reinterpret_cast<bf16x8*>(Xr + (iq * (int64_t)J + j) * 8) = o;
  }
}

hipError_t launch_quantize(const float* X, const Plan& p, __bf16* Xr, __bf16* Xj8, float* scale,
                           hipStream_t s) {
  if (p.K % 4 == 0 && p.J * p.K < (int64_t)1 << 31 && p.Kp % 4 == 0 && p.Kp3 % 4 == 0) {
    hipLaunchKernelGGL(k_quantize4, dim3((unsigned)p.I), dim3(256), 0, s, X, (int)p.J, (int)p.K,
                       (int)p.Kp, (int)p.JG, (int)p.Kp3, Xr, Xj8, scale);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nb = p.I * p.JG * (p.Kp / 8);   // 8 x 8 blocks, 32 per workgroup
    hipLaunchKernelGGL(k_xr_from_xj8, dim3((unsigned)cdiv(nb, 32)), dim3(256), 0, s, Xj8, (int)p.J,
                       (int)p.JG, (int)p.Kp, (int)p.Kp3, nb, Xr);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_quantize, dim3((unsigned)p.I), dim3(256), 0, s, X, p.J, p.K, p.Kp, p.JG,
                     p.Kp3, Xr, Xj8, scale);
  return hipGetLastError();
}

hipError_t launch_sumsq(const void* X, int x_is_f64, int64_t n, double* partial, int nparts,
                        double* out, hipStream_t s) {
  if (x_is_f64)
    hipLaunchKernelGGL(k_sumsq_part<double>, dim3(nparts), dim3(256), 0, s, (const double*)X, n,
                       partial);
  else
    hipLaunchKernelGGL(k_sumsq_part<float>, dim3(nparts), dim3(256), 0, s, (const float*)X, n,
                       partial);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, partial, nparts, out);
  return hipGetLastError();
}

template <typename T, int FT, int MT>
static hipError_t pass1_t(const Plan& p, const void* X, const void* Hb, const void* Hc, void* Tout,
                          void* P1, hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    if (stream1f_ok(p)) {
      auto kern = (p.vec == 4) ? k_pass1s<FT, MT, 4> : k_pass1s<FT, MT, 2>;
      hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)p.lds1);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(kern, dim3(p.grid1), dim3(512), p.lds1, s, (const float*)X, (int)p.I,
                         (int)p.J, (int)p.K, p.F, (const float*)Hb, (const float*)Hc, (float*)Tout,
                         (float*)P1, p.nch1, p.KC1);
      return hipGetLastError();
    }
  }
  auto kern = k_pass1<T, FT, MT>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)p.lds1);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(p.grid1), dim3(512), p.lds1, s, (const T*)X, (int)p.I, (int)p.J,
                     (int)p.K, p.F, (const T*)Hb, (const T*)Hc, (T*)Tout, (T*)P1, p.nch1, p.KC1,
                     p.vec);
  return hipGetLastError();
}

template <typename T, int FT>
static hipError_t pass1_mt(const Plan& p, const void* X, const void* Hb, const void* Hc, void* Tout,
                           void* P1, hipStream_t s) {
  if (p.MT1 == 2) return pass1_t<T, FT, 2>(p, X, Hb, Hc, Tout, P1, s);
  return pass1_t<T, FT, 1>(p, X, Hb, Hc, Tout, P1, s);
}

template <int FT>
static hipError_t pass1_bf16(const Plan& p, const __bf16* Xr, const float* scale, const void* Hb,
                             const void* Hc, void* Tout, void* P1, hipStream_t s) {
  if (stream1_ok(p)) {
    auto kern = k_pass1_bf16s<FT, 2, false>;
    if constexpr (FT != 2) {
      if (p.ts1) kern = k_pass1_bf16s<FT, 2, true>;
    }
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds1);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(p.grid1), dim3(512), p.lds1, s, Xr, scale, (int)p.I, (int)p.J,
                       (int)p.K, (int)p.Kp, p.F, (const float*)Hb, (const float*)Hc, (float*)Tout,
                       (float*)P1, p.nch1, p.spg1, p.G1);
    return hipGetLastError();
  }
  auto kern = k_pass1_bf16<FT, 2>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)p.lds1);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(p.grid1), dim3(512), p.lds1, s, Xr, scale, (int)p.I, (int)p.J,
                     (int)p.K, (int)p.Kp, p.F, (const float*)Hb, (const float*)Hc, (float*)Tout,
                     (float*)P1, p.nch1, p.KC1);
  return hipGetLastError();
}

hipError_t launch_pass1(const Plan& p, const void* X, const __bf16* Xr, const float* scale,
                        const void* Hb, const void* Hc, void* Tout, void* P1, hipStream_t s) {
  if (p.prec == PREC_BF16) {
    switch (p.FT) {
      case 1: return pass1_bf16<1>(p, Xr, scale, Hb, Hc, Tout, P1, s);
      case 2: return pass1_bf16<2>(p, Xr, scale, Hb, Hc, Tout, P1, s);
      case 3: return pass1_bf16<3>(p, Xr, scale, Hb, Hc, Tout, P1, s);
      default: return pass1_bf16<4>(p, Xr, scale, Hb, Hc, Tout, P1, s);
    }
  }
  if (p.prec == PREC_F64) {
    switch (p.FT) {
      case 1: return pass1_mt<double, 1>(p, X, Hb, Hc, Tout, P1, s);
      case 2: return pass1_mt<double, 2>(p, X, Hb, Hc, Tout, P1, s);
      case 3: return pass1_mt<double, 3>(p, X, Hb, Hc, Tout, P1, s);
      default: return pass1_mt<double, 4>(p, X, Hb, Hc, Tout, P1, s);
    }
  }
  switch (p.FT) {
    case 1: return pass1_mt<float, 1>(p, X, Hb, Hc, Tout, P1, s);
    case 2: return pass1_mt<float, 2>(p, X, Hb, Hc, Tout, P1, s);
    case 3: return pass1_mt<float, 3>(p, X, Hb, Hc, Tout, P1, s);
    default: return pass1_mt<float, 4>(p, X, Hb, Hc, Tout, P1, s);
  }
}

hipError_t launch_mode2(const Plan& p, const void* Tin, const void* Ha, void* P2, hipStream_t s) {
  const int64_t JF = p.J * p.F;
  if (p.prec != PREC_F64 && p.F % 4 == 0) {
    const int64_t JF4 = JF / 4;
    dim3 grid4((unsigned)cdiv(JF4, 256), (unsigned)p.nich2);
    hipLaunchKernelGGL(k_mode2v, grid4, dim3(256), 0, s, (const float4*)Tin, (const float4*)Ha,
                       (int)p.I, JF4, p.F / 4, p.ich2, (float4*)P2);
    return hipGetLastError();
  }
  dim3 grid((unsigned)cdiv(JF, 256), (unsigned)p.nich2);
  if (p.prec == PREC_F64)
    hipLaunchKernelGGL(k_mode2<double>, grid, dim3(256), 0, s, (const double*)Tin,
                       (const double*)Ha, (int)p.I, JF, p.F, p.ich2, (double*)P2);
  else
    hipLaunchKernelGGL(k_mode2<float>, grid, dim3(256), 0, s, (const float*)Tin, (const float*)Ha,
                       (int)p.I, JF, p.F, p.ich2, (float*)P2);
  return hipGetLastError();
}

template <typename T, int FT, int RG>
static void pass3_s(const Plan& p, const void* X, const void* Ha, const void* Hb, void* P3,
                    hipStream_t s) {
  const dim3 grid((unsigned)p.nb3, (unsigned)p.nkg3);
  if (p.vec == 4)
    hipLaunchKernelGGL((k_pass3s<float, FT, 4, RG>), grid, dim3(512), 0, s, (const float*)X,
                       p.I * p.J, (int)p.J, (int)p.K, p.F, (const float*)Ha, (const float*)Hb,
                       (float*)P3, p.rpc3, (int)p.I);
  else
    hipLaunchKernelGGL((k_pass3s<float, FT, 2, RG>), grid, dim3(512), 0, s, (const float*)X,
                       p.I * p.J, (int)p.J, (int)p.K, p.F, (const float*)Ha, (const float*)Hb,
                       (float*)P3, p.rpc3, (int)p.I);
}

template <typename T, int FT>
static void pass3_t(const Plan& p, const void* X, const void* Ha, const void* Hb, void* P3,
                    hipStream_t s) {
  // FP32 rows of even length whose block range fits 32-bit buffer offsets:
  // the streaming form (eight waves per block, rg3 row groups)
  if constexpr (sizeof(T) == 4) {
    if (p.s3) {
      switch (p.rg3) {
        case 8: pass3_s<T, FT, 8>(p, X, Ha, Hb, P3, s); break;
        case 4: pass3_s<T, FT, 4>(p, X, Ha, Hb, P3, s); break;
        case 2: pass3_s<T, FT, 2>(p, X, Ha, Hb, P3, s); break;
        default: pass3_s<T, FT, 1>(p, X, Ha, Hb, P3, s); break;
      }
      return;
    }
  }
  hipLaunchKernelGGL((k_pass3<T, FT>), dim3(p.nb3, p.nkg3), dim3(64 * p.nw3), 0, s, (const T*)X,
                     p.I * p.J, (int)p.J, (int)p.K, p.F, (const T*)Ha, (const T*)Hb, (T*)P3,
                     p.rpc3, p.vec);
}

template <int FT>
static hipError_t pass3_bf16(const Plan& p, const __bf16* Xj8, const float* scale, const void* Ha,
                             const void* Hb, void* P3, hipStream_t s) {
  auto kern = k_pass3_bf16s<FT>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)p.lds3);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)(p.nch3 * p.bpc3)), dim3(512), p.lds3, s, Xj8, scale,
                     (int)p.I, (int)p.J, (int)p.JG, (int)p.K, (int)p.Kp3, p.F, (const float*)Ha,
                     (const float*)Hb, (float*)P3, p.nkt3, (int)p.rpc3, p.ngr3, p.jcg3, p.bpc3);
  return hipGetLastError();
}

hipError_t launch_pass3(const Plan& p, const void* X, const __bf16* Xj8, const float* scale,
                        const void* Ha, const void* Hb, void* P3, hipStream_t s) {
  if (p.prec == PREC_BF16) {
    switch (p.FT) {
      case 1: return pass3_bf16<1>(p, Xj8, scale, Ha, Hb, P3, s);
      case 2: return pass3_bf16<2>(p, Xj8, scale, Ha, Hb, P3, s);
      case 3: return pass3_bf16<3>(p, Xj8, scale, Ha, Hb, P3, s);
      default: return pass3_bf16<4>(p, Xj8, scale, Ha, Hb, P3, s);
    }
  } else if (p.prec == PREC_F64) {
    switch (p.FT) {
      case 1: pass3_t<double, 1>(p, X, Ha, Hb, P3, s); break;
      case 2: pass3_t<double, 2>(p, X, Ha, Hb, P3, s); break;
      case 3: pass3_t<double, 3>(p, X, Ha, Hb, P3, s); break;
      default: pass3_t<double, 4>(p, X, Ha, Hb, P3, s); break;
    }
  } else {
    switch (p.FT) {
      case 1: pass3_t<float, 1>(p, X, Ha, Hb, P3, s); break;
      case 2: pass3_t<float, 2>(p, X, Ha, Hb, P3, s); break;
      case 3: pass3_t<float, 3>(p, X, Ha, Hb, P3, s); break;
      default: pass3_t<float, 4>(p, X, Ha, Hb, P3, s); break;
    }
  }
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const void* part, int part_is_f64, int64_t pstride,
                                  int64_t rowstride, int nparts, int64_t rows, int F, double* W,
                                  hipStream_t s, int groups) {
  const unsigned grid = (unsigned)cdiv(rows * F, 64);
  if (groups == 4) {
    if (part_is_f64)
      hipLaunchKernelGGL((k_reduce_grouped<double, 4>), dim3(grid), dim3(256), 0, s,
                         (const double*)part, pstride, rowstride, nparts, rows, F, W);
    else
      hipLaunchKernelGGL((k_reduce_grouped<float, 4>), dim3(grid), dim3(256), 0, s,
                         (const float*)part, pstride, rowstride, nparts, rows, F, W);
  } else {
    if (part_is_f64)
      hipLaunchKernelGGL((k_reduce_grouped<double, 16>), dim3(grid), dim3(1024), 0, s,
                         (const double*)part, pstride, rowstride, nparts, rows, F, W);
    else
      hipLaunchKernelGGL((k_reduce_grouped<float, 16>), dim3(grid), dim3(1024), 0, s,
                         (const float*)part, pstride, rowstride, nparts, rows, F, W);
  }
  return hipGetLastError();
}

}  // namespace ntf
