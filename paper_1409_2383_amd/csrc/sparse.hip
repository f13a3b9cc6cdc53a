// Sparse tensors (Section IV-A, item 1): the MTTKRP of a tensor given by its
// n non-zeros costs 3nF flops, one product of two factor rows per non-zero,
// without the Khatri-Rao matrix.
//
// Set-up builds, per mode m, a copy of the non-zeros sorted by (i_m, then the
// other two indices in mode order): a stable LSD radix sort of packed 64-bit
// keys (own kernels: digit histograms per 4096-key tile, a three-kernel
// exclusive scan, a stable scatter that ranks equal digits in tile order by
// wave ballots).  Each copy is four arrays: output row, the two other
// indices, the value.
//
// MTTKRP of mode m: the sorted non-zeros are cut into segments of S; a group
// of FL lanes (FL = next power of two >= F, lane f owns column f) walks one
// segment, gathering the two factor rows of each non-zero (coalesced F-wide
// reads) and accumulating v * a_f * b_f into the current output row.  A row
// that lies inside the segment is written once; a row cut by a segment
// boundary leaves its piece in a carry slot, and a fix-up kernel adds the
// pieces of each cut row in segment order.  No atomics: the result is
// deterministic.
#include <utility>

#include "ntf_device.h"
#include "ntf_launch.h"

namespace ntf {
namespace {

constexpr int kTileThreads = 256;
constexpr int kTileItems = 16;
constexpr int kTile = kTileThreads * kTileItems;   // keys per sort tile

int bits_for(int64_t d) {
  int b = 0;
  while (((int64_t)1 << b) < d) ++b;
  return b;
}

// ---------------------------------------------------------------- set-up

__global__ __launch_bounds__(256) void k_sp_check(const int32_t* __restrict__ idx, int64_t n,
                                                  int64_t d0, int64_t d1, int64_t d2,
                                                  int* __restrict__ flag) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const int32_t i = idx[3 * e], j = idx[3 * e + 1], k = idx[3 * e + 2];
  if (i < 0 || i >= d0 || j < 0 || j >= d1 || k < 0 || k >= d2) atomicOr(flag, kSparseFlagRange);
}

__global__ __launch_bounds__(256) void k_sp_keys(const int32_t* __restrict__ idx, int64_t n, int m,
                                                 int ma, int mb, int sa, int sb,
                                                 uint64_t* __restrict__ key, uint32_t* __restrict__ perm) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const uint64_t r = (uint32_t)idx[3 * e + m], a = (uint32_t)idx[3 * e + ma],
                 b = (uint32_t)idx[3 * e + mb];
  key[e] = (r << sa) | (a << sb) | b;
  perm[e] = (uint32_t)e;
}

// digit counts of one tile, stored digit-major: hist[d * ntile + tile]
__global__ __launch_bounds__(kTileThreads) void k_rs_hist(const uint64_t* __restrict__ key, int64_t n,
                                                          int shift, int ntile,
                                                          uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x;
  h[tid] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll 4
  for (int q = 0; q < kTileItems; ++q) {
    const int64_t e = base + q * kTileThreads + tid;
    if (e < n) atomicAdd(&h[(key[e] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)tid * ntile + blockIdx.x] = h[tid];
}

// exclusive scan of 256 per-thread values over the block; returns the block total
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t& excl) {
  __shared__ uint32_t wsum[kTileThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t before = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kTileThreads / 64; ++w) {
    before += (w < wave) ? wsum[w] : 0u;
    total += wsum[w];
  }
  __syncthreads();
  excl = before + incl - v;
  return total;
}

// chunk-local exclusive scan of kTile values; chunk totals to tot[]
__global__ __launch_bounds__(kTileThreads) void k_scan_chunk(const uint32_t* __restrict__ in, int64_t len,
                                                             uint32_t* __restrict__ out,
                                                             uint32_t* __restrict__ tot) {
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)tid * kTileItems;
  uint32_t v[kTileItems];
  uint32_t s = 0;
#pragma unroll
  for (int q = 0; q < kTileItems; ++q) {
    v[q] = (base + q < len) ? in[base + q] : 0u;
    s += v[q];
  }
  uint32_t excl;
  const uint32_t total = block_excl_scan(s, excl);
#pragma unroll
  for (int q = 0; q < kTileItems; ++q) {
    if (base + q < len) out[base + q] = excl;
    excl += v[q];
  }
  if (tid == 0) tot[blockIdx.x] = total;
}

// one block: exclusive scan of the chunk totals, in place
__global__ __launch_bounds__(kTileThreads) void k_scan_totals(uint32_t* __restrict__ tot, int64_t len) {
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0u;
  __syncthreads();
  for (int64_t b0 = 0; b0 < len; b0 += kTileThreads) {
    const int64_t e = b0 + threadIdx.x;
    const uint32_t v = (e < len) ? tot[e] : 0u;
    uint32_t excl;
    const uint32_t total = block_excl_scan(v, excl);
    const uint32_t c = carry;
    if (e < len) tot[e] = c + excl;
    __syncthreads();
    if (threadIdx.x == 0) carry = c + total;
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_scan_add(uint32_t* __restrict__ out, int64_t len,
                                                  const uint32_t* __restrict__ tot) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < len) out[e] += tot[e / kTile];
}

// stable scatter of one tile: keys ranked among equal digits in tile order
// (round q covers keys q*256 .. q*256+255 of the tile, thread order inside)
__global__ __launch_bounds__(kTileThreads) void k_rs_scatter(const uint64_t* __restrict__ kin,
                                                             const uint32_t* __restrict__ pin,
                                                             uint64_t* __restrict__ kout,
                                                             uint32_t* __restrict__ pout, int64_t n,
                                                             int shift, int ntile,
                                                             const uint32_t* __restrict__ offs) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wc[kTileThreads / 64][256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  base[tid] = offs[(int64_t)tid * ntile + blockIdx.x];
  const uint64_t lt = (1ull << lane) - 1ull;
  const int64_t t0 = (int64_t)blockIdx.x * kTile;
  for (int q = 0; q < kTileItems; ++q) {
    const int64_t e = t0 + q * kTileThreads + tid;
    const bool valid = e < n;
    const uint64_t k = valid ? kin[e] : 0ull;
    const uint32_t p = valid ? pin[e] : 0u;
    const uint32_t d = (uint32_t)(k >> shift) & 255u;
#pragma unroll
    for (int w = 0; w < kTileThreads / 64; ++w) wc[w][tid] = 0u;
    __syncthreads();
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t set = __ballot(valid && bit);
      peers &= bit ? set : ~set;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && lane == 63 - __clzll(peers)) wc[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t dst = base[d] + rank;
      for (int w = 0; w < wave; ++w) dst += wc[w][d];
      kout[dst] = k;
      pout[dst] = p;
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int w = 0; w < kTileThreads / 64; ++w) add += wc[w][tid];
    base[tid] += add;
    __syncthreads();
  }
}

// Sorted keys -> records (row, a, b, value bits) of one mode; FP64 values go
// to their own array.  A repeated key is a repeated coordinate.
template <typename T>
__global__ __launch_bounds__(256) void k_sp_unpack(const uint64_t* __restrict__ key,
                                                   const uint32_t* __restrict__ perm,
                                                   const T* __restrict__ vin, int64_t n, int sa, int sb,
                                                   int4* __restrict__ rec, T* __restrict__ vout,
                                                   int* __restrict__ flag) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const uint64_t k = key[e];
  const T v = vin[perm[e]];
  int4 r;
  r.x = (int32_t)(k >> sa);
  r.y = (int32_t)((k >> sb) & ((1ull << (sa - sb)) - 1ull));
  r.z = (int32_t)(k & ((1ull << sb) - 1ull));
  if constexpr (sizeof(T) == 4) {
    r.w = __float_as_int((float)v);
  } else {
    r.w = 0;
    vout[e] = v;
  }
  rec[e] = r;
  if (e > 0 && key[e - 1] == k) atomicOr(flag, kSparseFlagDuplicate);
}

// Segment structure of one mode (depends on the sparsity pattern only):
// tail[s] = the row that starts its cut in segment s (its last row goes on
// into s + 1 and did not come from s - 1 as the whole segment), else -1;
// whole[s] = 1 if segment s is one row that began earlier and goes on.
__global__ __launch_bounds__(256) void k_sp_segmeta(const int4* __restrict__ rec, int64_t n, int S,
                                                    int64_t nseg, int32_t* __restrict__ tail,
                                                    int32_t* __restrict__ whole) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= nseg) return;
  const int64_t e0 = s * S, e1 = min(n, e0 + (int64_t)S);
  const int32_t first = rec[e0].x, last = rec[e1 - 1].x;
  const bool head = e0 > 0 && rec[e0 - 1].x == first;
  const bool goes_on = e1 < n && rec[e1].x == last;
  const bool w = head && goes_on && first == last;
  whole[s] = w ? 1 : 0;
  tail[s] = (goes_on && !w) ? last : -1;
}

// Pieces of each cut row: its tail piece in segment s and the head pieces of
// s+1 .. t, t the first segment after s that is not whole.  len[s] = t - s + 1
// (0 where no cut row starts); heavy[s] = 1 if len[s] > kLightPieces.
__global__ __launch_bounds__(256) void k_sp_chain(const int32_t* __restrict__ tail,
                                                  const int32_t* __restrict__ whole, int64_t nseg,
                                                  int32_t* __restrict__ len, uint32_t* __restrict__ heavy) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= nseg) return;
  int32_t L = 0;
  if (tail[s] >= 0) {
    int64_t t = s + 1;
    while (t < nseg - 1 && whole[t]) ++t;
    L = (int32_t)(t - s + 1);
  }
  len[s] = L;
  heavy[s] = (L > kLightPieces) ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_sp_compact(const uint32_t* __restrict__ flag,
                                                    const uint32_t* __restrict__ pos, int64_t nseg,
                                                    int32_t* __restrict__ list,
                                                    uint32_t* __restrict__ count) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= nseg) return;
  if (flag[s]) list[pos[s]] = (int32_t)s;
  if (s == nseg - 1) *count = pos[s] + flag[s];
}

// ---------------------------------------------------------------- MTTKRP

template <typename T>
struct SpAcc { typedef float type; };
template <>
struct SpAcc<double> { typedef double type; };

// CPL consecutive columns of a row as one 16-byte load (CPL = 1: scalar)
template <typename T, int CPL>
__device__ __forceinline__ void load_cols(const T* __restrict__ p, T (&x)[CPL]) {
  if constexpr (CPL == 1) {
    x[0] = *p;
  } else {
    typedef T V __attribute__((ext_vector_type(CPL)));
    const V v = *reinterpret_cast<const V*>(p);
#pragma unroll
    for (int c = 0; c < CPL; ++c) x[c] = v[c];
  }
}

template <typename T, int CPL>
__device__ __forceinline__ void store_cols(T* __restrict__ p, const T (&x)[CPL]) {
  if constexpr (CPL == 1) {
    *p = x[0];
  } else {
    typedef T V __attribute__((ext_vector_type(CPL)));
    V v;
#pragma unroll
    for (int c = 0; c < CPL; ++c) v[c] = x[c];
    *reinterpret_cast<V*>(p) = v;
  }
}

template <int CPL>
__device__ __forceinline__ void store_w(double* __restrict__ p, const float (&x)[CPL]) {
  double d[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) d[c] = (double)x[c];
  if constexpr (CPL == 4) {
    typedef double V2 __attribute__((ext_vector_type(2)));
    *reinterpret_cast<V2*>(p) = V2{d[0], d[1]};
    *reinterpret_cast<V2*>(p + 2) = V2{d[2], d[3]};
  } else {
#pragma unroll
    for (int c = 0; c < CPL; ++c) p[c] = d[c];
  }
}
template <int CPL>
__device__ __forceinline__ void store_w(double* __restrict__ p, const double (&x)[CPL]) {
  store_cols<double, CPL>(p, x);
}

// Segment seg = blockIdx.x * (256 / VL) + group; a group of VL lanes, lane j
// owning columns j*CPL .. j*CPL + CPL - 1, walks the segment in batches of VL
// records (lane j loads record b0 + j, the group reads them back by
// shuffles).  Rows inside the segment go to W; the first row, when it began
// in an earlier segment, to carry_h[seg]; the last row, when it goes on into
// the next segment (and is not that first row), to carry_t[seg].
template <typename T, int VL, int CPL>
__global__ __launch_bounds__(256) void k_sp_mttkrp(const int4* __restrict__ rec, const T* __restrict__ val,
                                                   const T* __restrict__ Fa, const T* __restrict__ Fb, int F,
                                                   int64_t n, int S, int64_t nseg, double* __restrict__ W,
                                                   typename SpAcc<T>::type* __restrict__ carry_h,
                                                   typename SpAcc<T>::type* __restrict__ carry_t) {
  typedef typename SpAcc<T>::type A;
  constexpr int NG = 256 / VL;
  constexpr int U = VL < 8 ? VL : 8;
  const int grp = threadIdx.x / VL, j = threadIdx.x - grp * VL;
  const int64_t seg = (int64_t)blockIdx.x * NG + grp;
  if (seg >= nseg) return;   // no block barriers below
  const int c0 = j * CPL;
  const bool col = c0 < F;
  const int64_t e0 = seg * S, e1 = min(n, e0 + (int64_t)S);
  const int32_t prev_row = e0 > 0 ? rec[e0 - 1].x : -1;
  const int32_t next_row = e1 < n ? rec[e1].x : -1;
  int32_t cur = rec[e0].x;
  const bool head = cur == prev_row;
  bool first = true;
  A acc[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) acc[c] = 0;
  for (int64_t b0 = e0; b0 < e1; b0 += VL) {
    const int64_t e = b0 + j;
    const bool ok = e < e1;
    const int4 r = ok ? rec[e] : int4{0, 0, 0, 0};
    T vl;
    if constexpr (sizeof(T) == 4) vl = __int_as_float(r.w);
    else vl = ok ? val[e] : T(0);
    const int cnt = (int)min((int64_t)VL, e1 - b0);
    for (int u0 = 0; u0 < cnt; u0 += U) {
      int32_t rr[U];
      A pv[U][CPL];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int u = u0 + q;
        rr[q] = __shfl(r.x, u, VL);
        const int32_t a = __shfl(r.y, u, VL), b = __shfl(r.z, u, VL);
        const T v = __shfl(vl, u, VL);
        T xa[CPL], xb[CPL];
        if ((u < cnt) && col) {
          load_cols<T, CPL>(Fa + (int64_t)a * F + c0, xa);
          load_cols<T, CPL>(Fb + (int64_t)b * F + c0, xb);
        } else {
#pragma unroll
          for (int c = 0; c < CPL; ++c) xa[c] = xb[c] = T(0);
        }
#pragma unroll
        for (int c = 0; c < CPL; ++c) pv[q][c] = (A)v * (A)xa[c] * (A)xb[c];
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        if (u0 + q >= cnt) break;
        if (rr[q] != cur) {
          if (col) {
            if (first && head) store_cols<A, CPL>(carry_h + seg * F + c0, acc);
            else store_w<CPL>(W + (int64_t)cur * F + c0, acc);
          }
          first = false;
#pragma unroll
          for (int c = 0; c < CPL; ++c) acc[c] = 0;
          cur = rr[q];
        }
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[c] += pv[q][c];
      }
    }
  }
  if (col) {
    if (first && head) store_cols<A, CPL>(carry_h + seg * F + c0, acc);
    else if (cur == next_row) store_cols<A, CPL>(carry_t + seg * F + c0, acc);
    else store_w<CPL>(W + (int64_t)cur * F + c0, acc);
  }
}

// Cut rows of at most kLightPieces pieces: one group per segment, the pieces
// summed in segment order.
template <typename A, int VL, int CPL>
__global__ __launch_bounds__(256) void k_sp_fixup(const int32_t* __restrict__ tail,
                                                  const int32_t* __restrict__ len,
                                                  const A* __restrict__ carry_h,
                                                  const A* __restrict__ carry_t, int F, int64_t nseg,
                                                  double* __restrict__ W) {
  constexpr int NG = 256 / VL;
  const int grp = threadIdx.x / VL, j = threadIdx.x - grp * VL;
  const int64_t seg = (int64_t)blockIdx.x * NG + grp;
  const int c0 = j * CPL;
  if (seg >= nseg || c0 >= F) return;
  const int32_t L = len[seg];
  if (L == 0 || L > kLightPieces) return;
  A x[CPL];
  load_cols<A, CPL>(carry_t + seg * F + c0, x);
  double acc[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) acc[c] = (double)x[c];
  for (int p = 1; p < L; ++p) {
    load_cols<A, CPL>(carry_h + (seg + p) * F + c0, x);
#pragma unroll
    for (int c = 0; c < CPL; ++c) acc[c] += (double)x[c];
  }
  store_w<CPL>(W + (int64_t)tail[seg] * F + c0, acc);
}

// Cut rows of more pieces: one block per row; group g of VL lanes sums the
// pieces p = g, g + NG, ... in order, then the group sums are added in group
// order.
template <typename A, int VL, int CPL>
__global__ __launch_bounds__(256) void k_sp_fixup_heavy(const int32_t* __restrict__ list,
                                                        const int32_t* __restrict__ tail,
                                                        const int32_t* __restrict__ len,
                                                        const A* __restrict__ carry_h,
                                                        const A* __restrict__ carry_t, int F,
                                                        double* __restrict__ W) {
  constexpr int NG = 256 / VL;
  __shared__ double part[NG][VL * CPL];
  const int grp = threadIdx.x / VL, j = threadIdx.x - grp * VL;
  const int c0 = j * CPL;
  const int64_t s = list[blockIdx.x];
  const int32_t L = len[s];
  double acc[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) acc[c] = 0.0;
  if (c0 < F) {
    for (int p = grp; p < L; p += NG) {
      A x[CPL];
      load_cols<A, CPL>((p == 0 ? carry_t + s * F : carry_h + (s + p) * F) + c0, x);
#pragma unroll
      for (int c = 0; c < CPL; ++c) acc[c] += (double)x[c];
    }
  }
#pragma unroll
  for (int c = 0; c < CPL; ++c) part[grp][c0 + c] = acc[c];
  __syncthreads();
  if (grp == 0 && c0 < F) {
    double t[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      t[c] = part[0][c0 + c];
      for (int g = 1; g < NG; ++g) t[c] += part[g][c0 + c];
    }
    store_w<CPL>(W + (int64_t)tail[s] * F + c0, t);
  }
}

// ---------------------------------------------------------------- fit

// Per block: sum over its non-zeros of (x - m)^2 and m^2, m the model value
// sum_f A[i,f] B[j,f] C[k,f]; one thread per non-zero (mode-1 records).
template <typename T>
__global__ __launch_bounds__(256) void k_sp_fit(const int4* __restrict__ rec, const T* __restrict__ val,
                                                const T* __restrict__ A, const T* __restrict__ B,
                                                const T* __restrict__ C, int F, int64_t n,
                                                double* __restrict__ part) {
  __shared__ double red[4][2];
  double s0 = 0.0, s1 = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const int4 r = rec[e];
    const T* a = A + (int64_t)r.x * F;
    const T* b = B + (int64_t)r.y * F;
    const T* c = C + (int64_t)r.z * F;
    double m = 0.0;
    for (int q = 0; q < F; ++q) m += (double)a[q] * (double)b[q] * (double)c[q];
    double x;
    if constexpr (sizeof(T) == 4) x = (double)__int_as_float(r.w);
    else x = (double)val[e];
    const double d = x - m;
    s0 += d * d;
    s1 += m * m;
  }
  s0 = group_sum(s0, 64);
  s1 = group_sum(s1, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[wave][0] = s0;
    red[wave][1] = s1;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int c = threadIdx.x;
    part[2 * blockIdx.x + c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
  }
}

// out[0] = ||X - M||^2 = sum (x - m)^2 + sum(G1 * G2 * G3) - sum m^2, out[1] = ||X||^2
__global__ __launch_bounds__(256) void k_sp_fit_final(const double* __restrict__ part, int nparts,
                                                      const double* __restrict__ g0,
                                                      const double* __restrict__ g1,
                                                      const double* __restrict__ g2, int F,
                                                      const double* __restrict__ xnorm2,
                                                      double* __restrict__ out) {
  __shared__ double red[4][3];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int p = threadIdx.x; p < nparts; p += 256) {
    s0 += part[2 * p];
    s1 += part[2 * p + 1];
  }
  for (int e = threadIdx.x; e < F * F; e += 256) s2 += g0[e] * g1[e] * g2[e];
  s0 = group_sum(s0, 64);
  s1 = group_sum(s1, 64);
  s2 = group_sum(s2, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[wave][0] = s0;
    red[wave][1] = s1;
    red[wave][2] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[3];
    for (int c = 0; c < 3; ++c) t[c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
    out[0] = t[0] + t[2] - t[1];
    out[1] = *xnorm2;
  }
}

template <typename T, int VL, int CPL>
hipError_t sp_mttkrp_v(const SpModeArgs& a, hipStream_t s) {
  typedef typename SpAcc<T>::type A;
  constexpr int NG = 256 / VL;
  const unsigned grid = (unsigned)((a.nseg + NG - 1) / NG);
  hipLaunchKernelGGL((k_sp_mttkrp<T, VL, CPL>), dim3(grid), dim3(256), 0, s, a.rec, (const T*)a.val,
                     (const T*)a.Fa, (const T*)a.Fb, a.F, a.n, a.S, a.nseg, a.W, (A*)a.carry_h,
                     (A*)a.carry_t);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_sp_fixup<A, VL, CPL>), dim3(grid), dim3(256), 0, s, a.tail, a.len,
                     (const A*)a.carry_h, (const A*)a.carry_t, a.F, a.nseg, a.W);
  e = hipGetLastError();
  if (e != hipSuccess || a.nheavy == 0) return e;
  hipLaunchKernelGGL((k_sp_fixup_heavy<A, VL, CPL>), dim3((unsigned)a.nheavy), dim3(256), 0, s, a.heavy,
                     a.tail, a.len, (const A*)a.carry_h, (const A*)a.carry_t, a.F, a.W);
  return hipGetLastError();
}

// lanes per non-zero for a rank and a column width
int lanes_for(int F, int cpl) {
  int v = 1;
  while (v * cpl < F) v <<= 1;
  return v < 4 ? 4 : v;
}

template <typename T, int CPL>
hipError_t sp_mttkrp_c(const SpModeArgs& a, hipStream_t s) {
  switch (lanes_for(a.F, CPL)) {
    case 4: return sp_mttkrp_v<T, 4, CPL>(a, s);
    case 8: return sp_mttkrp_v<T, 8, CPL>(a, s);
    case 16: return sp_mttkrp_v<T, 16, CPL>(a, s);
    case 32: return sp_mttkrp_v<T, 32, CPL>(a, s);
    default: return sp_mttkrp_v<T, 64, CPL>(a, s);
  }
}

}  // namespace

int sp_key_bits(const int64_t dims[3]) { return bits_for(dims[0]) + bits_for(dims[1]) + bits_for(dims[2]); }

int64_t sp_tiles(int64_t n) { return (n + kTile - 1) / kTile; }

size_t sp_scan_len(int64_t n) { return (size_t)256 * (size_t)sp_tiles(n); }

size_t sp_scan_chunks(int64_t n) { return (sp_scan_len(n) + kTile - 1) / kTile; }

int sp_cols_per_lane(int F, int f64) {
  const int v = f64 ? 2 : 4;   // 16-byte loads of a factor row need F * elem % 16 == 0
  return (F % v == 0) ? v : 1;
}

int sp_segment_len(int F, int f64) { return 64 * lanes_for(F, sp_cols_per_lane(F, f64)); }

hipError_t sp_check(const int32_t* idx, int64_t n, const int64_t dims[3], int* flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sp_check, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, idx, n, dims[0],
                     dims[1], dims[2], flag);
  return hipGetLastError();
}

hipError_t sp_build_mode(const SpBuildArgs& a, hipStream_t s) {
  const int64_t n = a.n;
  if (n <= 0) return hipSuccess;
  const int m = a.mode;
  const int ma = (m == 0) ? 1 : 0, mb = (m == 2) ? 1 : 2;
  const int bb = bits_for(a.dims[mb]), ba = bits_for(a.dims[ma]), br = bits_for(a.dims[m]);
  const int sb = bb, sa = ba + bb;
  const unsigned g256 = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_sp_keys, dim3(g256), dim3(256), 0, s, a.idx, n, m, ma, mb, sa, sb, a.k0, a.p0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nbits = br + ba + bb;
  const int ntile = (int)sp_tiles(n);
  const int64_t len = (int64_t)256 * ntile;
  const unsigned nchunk = (unsigned)((len + kTile - 1) / kTile);
  uint64_t* kin = a.k0;
  uint64_t* kout = a.k1;
  uint32_t* pin = a.p0;
  uint32_t* pout = a.p1;
  for (int shift = 0; shift < nbits; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist, dim3(ntile), dim3(kTileThreads), 0, s, kin, n, shift, ntile, a.hist);
    hipLaunchKernelGGL(k_scan_chunk, dim3(nchunk), dim3(kTileThreads), 0, s, a.hist, len, a.offs, a.tot);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kTileThreads), 0, s, a.tot, (int64_t)nchunk);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, a.offs, len, a.tot);
    hipLaunchKernelGGL(k_rs_scatter, dim3(ntile), dim3(kTileThreads), 0, s, kin, pin, kout, pout, n, shift,
                       ntile, a.offs);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    std::swap(kin, kout);
    std::swap(pin, pout);
  }
  if (a.val_f64)
    hipLaunchKernelGGL(k_sp_unpack<double>, dim3(g256), dim3(256), 0, s, kin, pin, (const double*)a.val, n,
                       sa, sb, a.rec, (double*)a.val_out, a.flag);
  else
    hipLaunchKernelGGL(k_sp_unpack<float>, dim3(g256), dim3(256), 0, s, kin, pin, (const float*)a.val, n, sa,
                       sb, a.rec, (float*)nullptr, a.flag);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // segment structure and the list of heavy cut rows
  const int64_t nseg = a.nseg;
  const unsigned gs = (unsigned)((nseg + 255) / 256);
  int32_t* whole = reinterpret_cast<int32_t*>(a.p1 == pin ? a.p0 : a.p1);   // free permutation buffer
  uint32_t* flags = reinterpret_cast<uint32_t*>(a.k0 == kin ? a.k1 : a.k0);  // free key buffer
  hipLaunchKernelGGL(k_sp_segmeta, dim3(gs), dim3(256), 0, s, a.rec, n, a.S, nseg, a.tail, whole);
  hipLaunchKernelGGL(k_sp_chain, dim3(gs), dim3(256), 0, s, a.tail, whole, nseg, a.len, flags);
  const unsigned nch = (unsigned)((nseg + kTile - 1) / kTile);
  hipLaunchKernelGGL(k_scan_chunk, dim3(nch), dim3(kTileThreads), 0, s, flags, nseg, a.offs, a.tot);
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kTileThreads), 0, s, a.tot, (int64_t)nch);
  hipLaunchKernelGGL(k_scan_add, dim3(gs), dim3(256), 0, s, a.offs, nseg, a.tot);
  hipLaunchKernelGGL(k_sp_compact, dim3(gs), dim3(256), 0, s, flags, a.offs, nseg, a.heavy, a.nheavy);
  return hipGetLastError();
}

hipError_t sp_mttkrp(const SpModeArgs& a, hipStream_t s) {
  hipError_t e = launch_fill(a.W, a.rows * a.F, 0.0, s);
  if (e != hipSuccess || a.n <= 0) return e;
  const int cpl = sp_cols_per_lane(a.F, a.f64);
  if (a.f64) return cpl == 2 ? sp_mttkrp_c<double, 2>(a, s) : sp_mttkrp_c<double, 1>(a, s);
  return cpl == 4 ? sp_mttkrp_c<float, 4>(a, s) : sp_mttkrp_c<float, 1>(a, s);
}

int sp_fit_parts() { return 1024; }

hipError_t sp_fit(const int4* rec, const void* val, int f64, const void* A, const void* B, const void* C,
                  int F, int64_t n, const double* g0, const double* g1, const double* g2,
                  const double* xnorm2, double* part, double* out, hipStream_t s) {
  const int nparts = sp_fit_parts();
  if (f64)
    hipLaunchKernelGGL(k_sp_fit<double>, dim3(nparts), dim3(256), 0, s, rec, (const double*)val,
                       (const double*)A, (const double*)B, (const double*)C, F, n, part);
  else
    hipLaunchKernelGGL(k_sp_fit<float>, dim3(nparts), dim3(256), 0, s, rec, (const float*)nullptr,
                       (const float*)A, (const float*)B, (const float*)C, F, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sp_fit_final, dim3(1), dim3(256), 0, s, part, nparts, g0, g1, g2, F, xnorm2, out);
  return hipGetLastError();
}

}  // namespace ntf
