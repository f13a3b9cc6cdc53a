// Whole-factor projection for the cardinality constraint (Section IV-E, eq.
// g_new_def): the auxiliary factor becomes the non-negative part of
// V = Ht^T - U kept on its `card` largest entries (ties by row-major index),
// the scaled dual becomes H - V.  The inner sweep (proj == 3) has written V,
// Ht^T and the factor before the update in FP64; one block of 1024 threads
// finds the card-th largest positive entry by an MSB-first radix select over
// the IEEE-754 bit patterns (positive doubles order as their patterns), then
// writes H, U, the primal copy and the residual partials of the mode update.
#include "ntf_device.h"
#include "ntf_launch.h"

namespace ntf {
namespace {

constexpr int kCardThreads = 1024;
constexpr int kCardWaves = kCardThreads / 64;

struct CardK {
  const double* V;
  const double* X;
  const double* H0;
  void* H;
  void* U;
  void* Pout;      // may be null
  int64_t n;       // rows * F
  int64_t card;
  double iters_total;
  double* resid_part;   // [nparts][8]: partial 0 gets the totals, the rest zero
  int nparts;
};

// Sort key of an entry: its bit pattern when positive; zero, negative and
// NaN entries map to 0 and are never kept.
__device__ __forceinline__ uint64_t card_key(double v) {
  return v > 0.0 ? (uint64_t)__double_as_longlong(v) : 0ull;
}

// Number of threads before this one (thread order) whose `pred` holds, and
// the block total.
__device__ __forceinline__ unsigned block_excl_count(bool pred, unsigned* wtot, unsigned& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t m = __ballot(pred);
  if (lane == 0) wtot[wave] = (unsigned)__popcll(m);
  __syncthreads();
  unsigned before = 0;
  total = 0;
  for (int w = 0; w < kCardWaves; ++w) {
    const unsigned c = wtot[w];
    before += (w < wave) ? c : 0u;
    total += c;
  }
  __syncthreads();   // wtot is rewritten by the next call
  return before + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
}

template <typename HT>
__global__ __launch_bounds__(kCardThreads) void k_card_project(CardK a) {
  __shared__ unsigned hist[256];
  __shared__ unsigned wtot[kCardWaves];
  __shared__ unsigned long long s_pos;
  __shared__ long long s_r;
  __shared__ int s_bin;
  __shared__ unsigned s_cnt;
  __shared__ double red[kCardWaves][5];
  const int tid = threadIdx.x;
  const int64_t n = a.n;

  if (tid == 0) s_pos = 0ull;
  __syncthreads();
  {
    unsigned pos = 0;
    for (int64_t e = tid; e < n; e += kCardThreads) pos += card_key(a.V[e]) != 0ull ? 1u : 0u;
    atomicAdd(&s_pos, (unsigned long long)pos);
  }
  __syncthreads();

  // keep: key > thr, plus the first take_eq (row-major) entries whose key is thr
  uint64_t thr;
  int64_t take_eq;
  unsigned cnt_eq;
  if (a.card == 0) {
    thr = ~0ull;
    take_eq = 0;
    cnt_eq = 0;
  } else if ((int64_t)s_pos <= a.card) {
    thr = 0ull;   // every positive entry
    take_eq = 0;
    cnt_eq = 0;
  } else {
    uint64_t prefix = 0ull, mask = 0ull;
    int64_t r = a.card;   // rank from the top among the keys matching the prefix
    cnt_eq = 0;
    for (int shift = 56; shift >= 0; shift -= 8) {
      for (int b = tid; b < 256; b += kCardThreads) hist[b] = 0u;
      __syncthreads();
      for (int64_t e = tid; e < n; e += kCardThreads) {
        const uint64_t k = card_key(a.V[e]);
        if (k != 0ull && (k & mask) == prefix) atomicAdd(&hist[(k >> shift) & 255ull], 1u);
      }
      __syncthreads();
      if (tid == 0) {
        // 1 <= r <= (keys matching the prefix): some bin b >= 0 holds rank r
        int64_t cum = 0;
        int b = 255;
        for (; b > 0; --b) {
          if (cum + (int64_t)hist[b] >= r) break;
          cum += hist[b];
        }
        s_bin = b;
        s_r = r - cum;
        s_cnt = hist[b];
      }
      __syncthreads();
      prefix |= (uint64_t)s_bin << shift;
      mask |= 255ull << shift;
      r = s_r;
      cnt_eq = s_cnt;
      __syncthreads();
    }
    thr = prefix;
    take_eq = r;
  }

  // projection, dual update, primal copy and residual terms; when some keys
  // equal to the threshold are dropped, the kept ones are the first take_eq
  // in row-major order (block-ordered count, chunk by chunk)
  const bool ordered = take_eq < (int64_t)cnt_eq;
  int64_t seen = 0;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  HT* H = reinterpret_cast<HT*>(a.H);
  HT* U = reinterpret_cast<HT*>(a.U);
  HT* P = reinterpret_cast<HT*>(a.Pout);
  for (int64_t base = 0; base < n; base += kCardThreads) {
    const int64_t e = base + tid;
    const bool in = e < n;
    const double v = in ? a.V[e] : 0.0;
    const uint64_t k = card_key(v);
    const bool eq = in && k != 0ull && k == thr;
    bool keep = k > thr;
    if (ordered) {
      unsigned tot;
      const unsigned before = block_excl_count(eq, wtot, tot);
      keep = keep || (eq && seen + (int64_t)before < take_eq);
      seen += tot;
    } else {
      keep = keep || eq;
    }
    if (in) {
      const double x = a.X[e], h0 = a.H0[e];
      const double hn = keep ? v : 0.0;
      const double un = hn - v;
      H[e] = (HT)hn;
      U[e] = (HT)un;
      if (P) P[e] = (HT)x;
      const double hv = (double)(HT)hn, xv = (double)(HT)x, uv = (double)(HT)un;
      acc[0] += (hv - xv) * (hv - xv);
      acc[1] += (hv - h0) * (hv - h0);
      acc[2] += hv * hv;
      acc[3] += xv * xv;
      acc[4] += uv * uv;
    }
  }
  // residual partials: ||h-x||^2, ||h-h0||^2, ||h||^2, ||x||^2, ||u||^2, iterations
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const double s = group_sum(acc[q], 64);
    if (lane == 0) red[wave][q] = s;
  }
  __syncthreads();
  if (tid < 5) {
    double t = red[0][tid];
    for (int w = 1; w < kCardWaves; ++w) t += red[w][tid];
    a.resid_part[tid] = t;
  }
  if (tid == 5) a.resid_part[5] = a.iters_total;
  if (tid == 6 || tid == 7) a.resid_part[tid] = 0.0;
  for (int64_t i = 8 + tid; i < (int64_t)a.nparts * 8; i += kCardThreads) a.resid_part[i] = 0.0;
}

}  // namespace

hipError_t launch_card_project(const double* V, const double* X, const double* H0, void* H,
                               void* U, void* Pout, int h_f64, int64_t n, int64_t card,
                               double iters_total, double* resid_part, int nparts, hipStream_t s) {
  CardK k;
  k.V = V;
  k.X = X;
  k.H0 = H0;
  k.H = H;
  k.U = U;
  k.Pout = Pout;
  k.n = n;
  k.card = card;
  k.iters_total = iters_total;
  k.resid_part = resid_part;
  k.nparts = nparts;
  if (h_f64)
    hipLaunchKernelGGL(k_card_project<double>, dim3(1), dim3(kCardThreads), 0, s, k);
  else
    hipLaunchKernelGGL(k_card_project<float>, dim3(1), dim3(kCardThreads), 0, s, k);
  return hipGetLastError();
}

}  // namespace ntf
