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

template <typename T>
__global__ __launch_bounds__(256) void k_sp_unpack(const uint64_t* __restrict__ key,
                                                   const uint32_t* __restrict__ perm,
                                                   const T* __restrict__ vin, int64_t n, int sa, int sb,
                                                   int32_t* __restrict__ row, int32_t* __restrict__ ia,
                                                   int32_t* __restrict__ ib, T* __restrict__ vout,
                                                   int* __restrict__ flag) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const uint64_t k = key[e];
  row[e] = (int32_t)(k >> sa);
  ia[e] = (int32_t)((k >> sb) & ((1ull << (sa - sb)) - 1ull));
  ib[e] = (int32_t)(k & ((1ull << sb) - 1ull));
  vout[e] = vin[perm[e]];
  if (e > 0 && key[e - 1] == k) atomicOr(flag, kSparseFlagDuplicate);
}

// ---------------------------------------------------------------- MTTKRP

template <typename T>
struct SpAcc { typedef float type; };
template <>
struct SpAcc<double> { typedef double type; };

// Segment seg = blockIdx.x * (256 / FL) + group.  Per segment: head_row (the
// first row, if it began in an earlier segment, else -1), tail_row (the last
// row, if it goes on into the next segment and is not the head, else -1) and
// whole (1 if the segment is one row that began earlier and goes on).
template <typename T, int FL>
__global__ __launch_bounds__(256) void k_sp_mttkrp(const int32_t* __restrict__ row,
                                                   const int32_t* __restrict__ ia,
                                                   const int32_t* __restrict__ ib,
                                                   const T* __restrict__ val, const T* __restrict__ Fa,
                                                   const T* __restrict__ Fb, int F, int64_t n, int S,
                                                   int64_t nseg, double* __restrict__ W,
                                                   int32_t* __restrict__ meta,
                                                   typename SpAcc<T>::type* __restrict__ carry_h,
                                                   typename SpAcc<T>::type* __restrict__ carry_t) {
  typedef typename SpAcc<T>::type A;
  constexpr int NG = 256 / FL;
  constexpr int U = 8;
  const int grp = threadIdx.x / FL, f = threadIdx.x - grp * FL;
  const int64_t seg = (int64_t)blockIdx.x * NG + grp;
  if (seg >= nseg) return;   // no block barriers below
  const bool col = f < F;
  const int64_t e0 = seg * S, e1 = min(n, e0 + (int64_t)S);
  const int32_t prev_row = e0 > 0 ? row[e0 - 1] : -1;
  const int32_t next_row = e1 < n ? row[e1] : -1;
  int32_t cur = row[e0];
  const bool head = cur == prev_row;
  bool first = true;
  A acc = 0;
  for (int64_t b0 = e0; b0 < e1; b0 += FL) {
    const int64_t e = b0 + f;
    const bool ok = e < e1;
    const int32_t rl = ok ? row[e] : 0, al = ok ? ia[e] : 0, bl = ok ? ib[e] : 0;
    const T vl = ok ? val[e] : T(0);
    const int cnt = (int)min((int64_t)FL, e1 - b0);
    for (int u0 = 0; u0 < cnt; u0 += U) {
      int32_t rr[U];
      A pv[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int u = u0 + q;
        rr[q] = __shfl(rl, u, FL);
        const int32_t a = __shfl(al, u, FL), b = __shfl(bl, u, FL);
        const T v = __shfl(vl, u, FL);
        const bool live = (u < cnt) && col;
        const T xa = live ? Fa[(int64_t)a * F + f] : T(0);
        const T xb = live ? Fb[(int64_t)b * F + f] : T(0);
        pv[q] = (A)v * (A)xa * (A)xb;
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        if (u0 + q >= cnt) break;
        if (rr[q] != cur) {
          if (col) {
            if (first && head) carry_h[seg * F + f] = acc;
            else W[(int64_t)cur * F + f] = (double)acc;
          }
          first = false;
          acc = 0;
          cur = rr[q];
        }
        acc += pv[q];
      }
    }
  }
  const bool tail = cur == next_row;
  const bool whole = first && head && tail;
  if (col) {
    if (first && head) carry_h[seg * F + f] = acc;
    else if (tail) carry_t[seg * F + f] = acc;
    else W[(int64_t)cur * F + f] = (double)acc;
  }
  if (f == 0) {
    meta[3 * seg] = head ? prev_row : -1;
    meta[3 * seg + 1] = (tail && !(first && head)) ? cur : -1;
    meta[3 * seg + 2] = whole ? 1 : 0;
  }
}

// Rows cut by segment boundaries: the tail piece of the segment where the row
// began, then the head pieces of the following segments in order.
template <typename A, int FL>
__global__ __launch_bounds__(256) void k_sp_fixup(const int32_t* __restrict__ meta,
                                                  const A* __restrict__ carry_h,
                                                  const A* __restrict__ carry_t, int F, int64_t nseg,
                                                  double* __restrict__ W) {
  constexpr int NG = 256 / FL;
  const int grp = threadIdx.x / FL, f = threadIdx.x - grp * FL;
  const int64_t seg = (int64_t)blockIdx.x * NG + grp;
  if (seg >= nseg || f >= F) return;
  const int32_t R = meta[3 * seg + 1];
  if (R < 0) return;
  double acc = (double)carry_t[seg * F + f];
  for (int64_t t = seg + 1; t < nseg; ++t) {
    acc += (double)carry_h[t * F + f];
    if (!meta[3 * t + 2]) break;
  }
  W[(int64_t)R * F + f] = acc;
}

// ---------------------------------------------------------------- fit

// Per block: sum over its non-zeros of (x - m)^2 and m^2, m the model value
// sum_f A[i,f] B[j,f] C[k,f]; one thread per non-zero.
template <typename T>
__global__ __launch_bounds__(256) void k_sp_fit(const int32_t* __restrict__ row,
                                                const int32_t* __restrict__ ia,
                                                const int32_t* __restrict__ ib,
                                                const T* __restrict__ val, const T* __restrict__ A,
                                                const T* __restrict__ B, const T* __restrict__ C, int F,
                                                int64_t n, double* __restrict__ part) {
  __shared__ double red[4][2];
  double s0 = 0.0, s1 = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const T* a = A + (int64_t)row[e] * F;
    const T* b = B + (int64_t)ia[e] * F;
    const T* c = C + (int64_t)ib[e] * F;
    double m = 0.0;
    for (int q = 0; q < F; ++q) m += (double)a[q] * (double)b[q] * (double)c[q];
    const double r = (double)val[e] - m;
    s0 += r * r;
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

template <typename T, int FL>
hipError_t sp_mttkrp_fl(const SpModeArgs& a, hipStream_t s) {
  typedef typename SpAcc<T>::type A;
  constexpr int NG = 256 / FL;
  const unsigned grid = (unsigned)((a.nseg + NG - 1) / NG);
  hipLaunchKernelGGL((k_sp_mttkrp<T, FL>), dim3(grid), dim3(256), 0, s, a.row, a.ia, a.ib,
                     (const T*)a.val, (const T*)a.Fa, (const T*)a.Fb, a.F, a.n, a.S, a.nseg, a.W,
                     a.meta, (A*)a.carry_h, (A*)a.carry_t);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_sp_fixup<A, FL>), dim3(grid), dim3(256), 0, s, a.meta, (const A*)a.carry_h,
                     (const A*)a.carry_t, a.F, a.nseg, a.W);
  return hipGetLastError();
}

template <typename T>
hipError_t sp_mttkrp_t(const SpModeArgs& a, int FL, hipStream_t s) {
  switch (FL) {
    case 4: return sp_mttkrp_fl<T, 4>(a, s);
    case 8: return sp_mttkrp_fl<T, 8>(a, s);
    case 16: return sp_mttkrp_fl<T, 16>(a, s);
    case 32: return sp_mttkrp_fl<T, 32>(a, s);
    default: return sp_mttkrp_fl<T, 64>(a, s);
  }
}

}  // namespace

int sp_key_bits(const int64_t dims[3]) { return bits_for(dims[0]) + bits_for(dims[1]) + bits_for(dims[2]); }

int64_t sp_tiles(int64_t n) { return (n + kTile - 1) / kTile; }

size_t sp_scan_len(int64_t n) { return (size_t)256 * (size_t)sp_tiles(n); }

size_t sp_scan_chunks(int64_t n) { return (sp_scan_len(n) + kTile - 1) / kTile; }

int sp_segment_len(int FL) { return 16 * FL; }

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
                       sa, sb, a.row, a.ia, a.ib, (double*)a.val_out, a.flag);
  else
    hipLaunchKernelGGL(k_sp_unpack<float>, dim3(g256), dim3(256), 0, s, kin, pin, (const float*)a.val, n, sa,
                       sb, a.row, a.ia, a.ib, (float*)a.val_out, a.flag);
  return hipGetLastError();
}

hipError_t sp_mttkrp(const SpModeArgs& a, hipStream_t s) {
  hipError_t e = launch_fill(a.W, a.rows * a.F, 0.0, s);
  if (e != hipSuccess || a.n <= 0) return e;
  return a.f64 ? sp_mttkrp_t<double>(a, a.FL, s) : sp_mttkrp_t<float>(a, a.FL, s);
}

int sp_fit_parts() { return 1024; }

hipError_t sp_fit(const int32_t* row, const int32_t* ia, const int32_t* ib, const void* val, int f64,
                  const void* A, const void* B, const void* C, int F, int64_t n, const double* g0,
                  const double* g1, const double* g2, const double* xnorm2, double* part, double* out,
                  hipStream_t s) {
  const int nparts = sp_fit_parts();
  if (f64)
    hipLaunchKernelGGL(k_sp_fit<double>, dim3(nparts), dim3(256), 0, s, row, ia, ib, (const double*)val,
                       (const double*)A, (const double*)B, (const double*)C, F, n, part);
  else
    hipLaunchKernelGGL(k_sp_fit<float>, dim3(nparts), dim3(256), 0, s, row, ia, ib, (const float*)val,
                       (const float*)A, (const float*)B, (const float*)C, F, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sp_fit_final, dim3(1), dim3(256), 0, s, part, nparts, g0, g1, g2, F, xnorm2, out);
  return hipGetLastError();
}

}  // namespace ntf
