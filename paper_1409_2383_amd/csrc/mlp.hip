// Learned warm start for the inner sweep: a 3-layer MLP (ReLU after the two
// hidden layers, linear output) that maps one row's NNLS problem
// min_{h>=0} 1/2 h^T G h - w^T h  to an approximate solution (projected onto
// h >= 0 by the judge), trained on the GPU by the kernels below (forward,
// backward, Adam), and a per-row KKT judge that keeps the previous iterate
// whenever it is the better start.  Not part of the paper: an extension of
// the inner ADMoM sweep of Section IV whose fixed point is unchanged.
//
// Parameters are one flat vector [W1 Hd*D, b1 Hd, W2 Hd*Hd, b2 Hd, W3 F*Hd,
// b3 F], float32 for training and float16 for inference.  Row inputs: the
// upper triangle of G/rho (row by row) followed by w/||w||; the network
// predicts h*rho/||w||.
#include "ntf_device.h"
#include "ntf_launch.h"

#include <hip/hip_fp16.h>

namespace ntf {

// ---------------------------------------------------------------- GEMM

// C[m][n] = alpha * sum_k A(m,k) B(k,n) + beta * C[m][n], FP32 accumulation,
// A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn], C row-major [M][ldc].
// 64 x 64 block tile, 16-deep k slices staged in LDS, 4 x 4 outputs per
// thread; every output is one thread's sequential k sum (deterministic).
template <typename TB>
__global__ __launch_bounds__(256) void k_gemm(const float* __restrict__ A, int64_t sam,
                                              int64_t sak, const TB* __restrict__ B, int64_t sbk,
                                              int64_t sbn, float* __restrict__ C, int64_t ldc, int M,
                                              int N, int K, float alpha, float beta) {
  __shared__ float As[16][65];
  __shared__ float Bs[16][65];
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  float acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.f;
  for (int k0 = 0; k0 < K; k0 += 16) {
    __syncthreads();
    for (int e = tid; e < 16 * 64; e += 256) {
      const int kk = e >> 6, mm = e & 63;
      const int m = m0 + mm, k = k0 + kk;
      As[kk][mm] = (m < M && k < K) ? A[(int64_t)m * sam + (int64_t)k * sak] : 0.f;
      const int n = n0 + mm;
      Bs[kk][mm] = (n < N && k < K) ? (float)B[(int64_t)k * sbk + (int64_t)n * sbn] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[kk][tr + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[kk][tc + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] += av[a] * bv[b];
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int m = m0 + tr + 16 * a, n = n0 + tc + 16 * b;
      if (m < M && n < N) {
        float* c = C + (int64_t)m * ldc + n;
        *c = alpha * acc[a][b] + (beta != 0.f ? beta * *c : 0.f);
      }
    }
}

template <typename TB>
static hipError_t gemm(const float* A, int64_t sam, int64_t sak, const TB* B, int64_t sbk,
                       int64_t sbn, float* C, int64_t ldc, int M, int N, int K, float alpha,
                       float beta, hipStream_t s) {
  dim3 grid((N + 63) / 64, (M + 63) / 64);
  hipLaunchKernelGGL(k_gemm<TB>, grid, dim3(256), 0, s, A, sam, sak, B, sbk, sbn, C, ldc, M, N, K,
                     alpha, beta);
  return hipGetLastError();
}

// Z[b][n] = act(Z[b][n] + bias[n] + shared[n]) (shared may be null)
template <typename TB>
__global__ __launch_bounds__(256) void k_bias_act(float* __restrict__ Z, const TB* __restrict__ bias,
                                                  const float* __restrict__ shared, int64_t rows,
                                                  int N, int relu) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * N) return;
  const int n = (int)(e % N);
  float v = Z[e] + (float)bias[n] + (shared ? shared[n] : 0.f);
  if (relu) v = fmaxf(v, 0.f);
  Z[e] = v;
}

// dZ = dY * (Y > 0)
__global__ __launch_bounds__(256) void k_relu_back(const float* __restrict__ dY,
                                                   const float* __restrict__ Y,
                                                   float* __restrict__ dZ, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) dZ[e] = Y[e] > 0.f ? dY[e] : 0.f;
}

// db[n] = sum_b dZ[b][n], 16 fixed-order row groups
__global__ __launch_bounds__(1024) void k_colsum(const float* __restrict__ dZ, int64_t rows, int N,
                                                 float* __restrict__ db) {
  __shared__ float red[16][64];
  const int el = threadIdx.x & 63, pg = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + el;
  float s = 0.f;
  if (n < N)
    for (int64_t b = pg; b < rows; b += 16) s += dZ[b * N + n];
  red[pg][el] = s;
  __syncthreads();
  if (pg == 0 && n < N) {
    float t = red[0][el];
    for (int q = 1; q < 16; ++q) t += red[q][el];
    db[n] = t;
  }
}

// dY = (Y - T) / rows;  loss partials of 1/(2 rows) sum (Y - T)^2
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ Y, const float* __restrict__ T,
                                             int64_t n, float inv_rows, float* __restrict__ dY,
                                             double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const float d = Y[e] - T[e];
    dY[e] = d * inv_rows;
    acc += (double)d * d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] * 0.5 * inv_rows;
}

__global__ __launch_bounds__(64) void k_sum_small(const double* __restrict__ part, int n,
                                                  double* __restrict__ out) {
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < n; ++q) s += part[q];
    *out = s;
  }
}

// Adam with bias correction; optional float16 copy of the updated parameters
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              int64_t n, float lr, float b1, float b2, float eps,
                                              float c1, float c2, __half* __restrict__ p16) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.f - b1) * gi;
  const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  const float pi = p[e] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[e] = pi;
  if (p16) p16[e] = __float2half(pi);
}

// Row inputs: [upper(G/rho) | w/||w||] and scale ||w||/rho.  One block per
// 64 rows; rho comes from device memory (the solver's penalty of the mode).
__global__ __launch_bounds__(256) void k_features(const double* __restrict__ G,
                                                  const double* __restrict__ W, int64_t rows,
                                                  int F, const double* __restrict__ rho_p,
                                                  double rho_v, float* __restrict__ X,
                                                  float* __restrict__ scale) {
  const int D = F * (F + 1) / 2 + F;
  const double rho = rho_p ? rho_p[0] : rho_v;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  __shared__ double nrm[64];
  if (threadIdx.x < 64) {
    const int64_t r = r0 + threadIdx.x;
    double s = 0.0;
    if (r < rows)
      for (int f = 0; f < F; ++f) s += W[r * F + f] * W[r * F + f];
    nrm[threadIdx.x] = sqrt(s);
    if (r < rows) scale[r] = (float)(sqrt(s) / rho);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * D; e += 256) {
    const int rr = e / D, c = e - rr * D;
    const int64_t r = r0 + rr;
    if (r >= rows) continue;
    float v;
    if (c < D - F) {
      // upper-triangle index c -> (i, j), j >= i, row by row
      int i = 0, rem = c;
      while (rem >= F - i) {
        rem -= F - i;
        ++i;
      }
      v = (float)(G[i * F + i + rem] / rho);
    } else {
      const double n2 = nrm[rr];
      v = (float)(n2 > 0.0 ? W[r * F + (c - (D - F))] / n2 : 0.0);
    }
    X[r * D + c] = v;
  }
}

__global__ __launch_bounds__(256) void k_gather_rows(const float* __restrict__ src,
                                                     const int64_t* __restrict__ idx, int64_t n,
                                                     int cols, float* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * cols) return;
  const int64_t r = e / cols, c = e - r * cols;
  dst[e] = src[idx[r] * cols + c];
}

// Judge: per row, candidate h = y * scale (y the network output), u = 0 where
// h > 0 and max(0, (hG - w)/rho) where h = 0; keep it if its NNLS KKT
// violation in the units of h, ||min(h, (hG - w)/rho)|| (the change one
// projected-gradient step of length 1/rho would make; zero exactly at the
// solution), is smaller than the previous iterate's, otherwise keep (H, U).  One lane group of FL lanes per row.  `uback`
// converts a written u to the scale the inner kernel expects on load.
template <typename HT, int FL>
__global__ __launch_bounds__(256) void k_judge(const float* __restrict__ Y,
                                               const float* __restrict__ scale,
                                               const double* __restrict__ G,
                                               const double* __restrict__ W, HT* __restrict__ H,
                                               HT* __restrict__ U, int64_t rows, int F,
                                               const double* __restrict__ rho_p, int rescale,
                                               int* __restrict__ taken) {
  __shared__ double Gs[64 * 64];
  __shared__ double hs[256];
  __shared__ double ho[256];
  const int tid = threadIdx.x;
  for (int e = tid; e < F * F; e += 256) Gs[e] = G[e];
  const int rl = tid / FL, f = tid - rl * FL;
  const int64_t row = (int64_t)blockIdx.x * (256 / FL) + rl;
  const bool act = row < rows && f < F;
  const double rho = rho_p[0];
  const double uback = (rescale && rho_p[1] > 0.0) ? rho / rho_p[1] : 1.0;
  double hn = 0.0, hp = 0.0, w = 0.0, up = 0.0;
  if (act) {
    hn = fmax((double)Y[row * F + f] * (double)scale[row], 0.0);
    hp = (double)H[row * F + f];
    up = (double)U[row * F + f];
    w = W[row * F + f];
  }
  hs[tid] = hn;
  ho[tid] = hp;
  __syncthreads();
  double gn = 0.0, go = 0.0;
  if (f < F) {
    for (int q = 0; q < F; ++q) {
      gn += hs[rl * FL + q] * Gs[q * F + f];
      go += ho[rl * FL + q] * Gs[q * F + f];
    }
  }
  gn -= w;
  go -= w;
  // KKT violation in the units of h: min(h, (hG - w) / rho)
  const double kn = act ? fmin(hn, gn / rho) : 0.0;
  const double ko = act ? fmin(hp, go / rho) : 0.0;
  const double sn = group_sum(kn * kn, FL);
  const double so = group_sum(ko * ko, FL);
  if (act && sn < so) {
    const double un = (hn > 0.0) ? 0.0 : fmax(gn / rho, 0.0);
    H[row * F + f] = (HT)hn;
    U[row * F + f] = (HT)(un * uback);
    if (f == 0) atomicAdd(taken, 1);
  }
  (void)up;
}

// Training targets: t = h* / scale (scale = ||w||/rho), i.e. h* rho / ||w||.
__global__ __launch_bounds__(256) void k_targets(const double* __restrict__ Hs,
                                                 const float* __restrict__ scale, int64_t rows,
                                                 int F, float* __restrict__ T) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * F) return;
  const float sc = scale[e / F];
  T[e] = sc > 0.f ? (float)(Hs[e] / (double)sc) : 0.f;
}

// G = Ga * Gb (Hadamard) and rho = trace(G)/F (rho0 if not positive/finite).
__global__ __launch_bounds__(256) void k_hadamard_rho(const double* __restrict__ Ga,
                                                      const double* __restrict__ Gb, int F,
                                                      double rho0, double* __restrict__ G,
                                                      double* __restrict__ rho) {
  for (int e = threadIdx.x; e < F * F; e += 256) G[e] = Ga[e] * Gb[e];
  __syncthreads();
  if (threadIdx.x == 0) {
    double tr = 0.0;
    for (int f = 0; f < F; ++f) tr += G[f * F + f];
    double r = tr / F;
    if (!(r > 0.0) || !isfinite(r)) r = rho0;
    *rho = r;
  }
}

hipError_t mlp_targets(const double* Hs, const float* scale, int64_t rows, int F, float* T,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_targets, dim3((unsigned)((rows * F + 255) / 256)), dim3(256), 0, s, Hs,
                     scale, rows, F, T);
  return hipGetLastError();
}

hipError_t hadamard_rho(const double* Ga, const double* Gb, int F, double rho0, double* G,
                        double* rho, hipStream_t s) {
  hipLaunchKernelGGL(k_hadamard_rho, dim3(1), dim3(256), 0, s, Ga, Gb, F, rho0, G, rho);
  return hipGetLastError();
}

// ---------------------------------------------------------------- launchers

size_t mlp_param_count(int F, int Hd) {
  const int64_t D = (int64_t)F * (F + 1) / 2 + F;
  return (size_t)(Hd * D + Hd + (int64_t)Hd * Hd + Hd + (int64_t)F * Hd + F);
}

struct MlpOffsets {
  int64_t W1, b1, W2, b2, W3, b3;
};
static MlpOffsets mlp_offsets(int F, int Hd) {
  const int64_t D = (int64_t)F * (F + 1) / 2 + F;
  MlpOffsets o;
  o.W1 = 0;
  o.b1 = o.W1 + Hd * D;
  o.W2 = o.b1 + Hd;
  o.b2 = o.W2 + (int64_t)Hd * Hd;
  o.W3 = o.b2 + Hd;
  o.b3 = o.W3 + (int64_t)F * Hd;
  return o;
}

static unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// forward: act = [a1 | a2] per row (each Hd), Y [batch][F]
template <typename TP>
static hipError_t mlp_forward_t(const TP* P, int F, int Hd, const float* X, int64_t B, float* Y,
                                float* a1, float* a2, hipStream_t s) {
  const int D = F * (F + 1) / 2 + F;
  const MlpOffsets o = mlp_offsets(F, Hd);
  hipError_t e;
  // z1 = X W1^T  (B(k,n) = W1[n][k])
  if ((e = gemm<TP>(X, D, 1, P + o.W1, 1, D, a1, Hd, (int)B, Hd, D, 1.f, 0.f, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bias_act<TP>, dim3(blocks_for(B * Hd)), dim3(256), 0, s, a1, P + o.b1,
                     (const float*)nullptr, B, Hd, 1);
  if ((e = gemm<TP>(a1, Hd, 1, P + o.W2, 1, Hd, a2, Hd, (int)B, Hd, Hd, 1.f, 0.f, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bias_act<TP>, dim3(blocks_for(B * Hd)), dim3(256), 0, s, a2, P + o.b2,
                     (const float*)nullptr, B, Hd, 1);
  if ((e = gemm<TP>(a2, Hd, 1, P + o.W3, 1, Hd, Y, F, (int)B, F, Hd, 1.f, 0.f, s)) != hipSuccess) return e;
  // (linear output layer: a ReLU there can leave every output at zero for good)
  hipLaunchKernelGGL(k_bias_act<TP>, dim3(blocks_for(B * F)), dim3(256), 0, s, Y, P + o.b3,
                     (const float*)nullptr, B, F, 0);
  return hipGetLastError();
}

hipError_t mlp_forward(const void* params, int f16, int F, int Hd, const float* X, int64_t B,
                       float* Y, float* act, hipStream_t s) {
  float* a1 = act;
  float* a2 = act + B * Hd;
  if (f16) return mlp_forward_t<__half>((const __half*)params, F, Hd, X, B, Y, a1, a2, s);
  return mlp_forward_t<float>((const float*)params, F, Hd, X, B, Y, a1, a2, s);
}

// backward of sum(dY * Y): grad (flat, overwritten); work = 2*B*Hd + B*F floats
hipError_t mlp_backward(const float* P, int F, int Hd, const float* X, const float* act,
                        const float* Y, const float* dY, int64_t B, float* grad, float* work,
                        hipStream_t s) {
  const int D = F * (F + 1) / 2 + F;
  const MlpOffsets o = mlp_offsets(F, Hd);
  const float* a1 = act;
  const float* a2 = act + B * Hd;
  const float* d3 = dY;           // (linear output layer)
  float* dA = work + B * F;       // [B][Hd]
  float* dZ = dA + B * Hd;        // [B][Hd]
  hipError_t e;
  (void)Y;
  // dW3 = d3^T a2  [F][Hd]: A(m,k) = d3[k][m], B(k,n) = a2[k][n]
  if ((e = gemm<float>(d3, 1, F, a2, Hd, 1, grad + o.W3, Hd, F, Hd, (int)B, 1.f, 0.f, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum, dim3((F + 63) / 64), dim3(1024), 0, s, d3, B, F, grad + o.b3);
  // dA2 = d3 W3  [B][Hd]
  if ((e = gemm<float>(d3, F, 1, P + o.W3, Hd, 1, dA, Hd, (int)B, Hd, F, 1.f, 0.f, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_relu_back, dim3(blocks_for(B * Hd)), dim3(256), 0, s, dA, a2, dZ, B * Hd);
  if ((e = gemm<float>(dZ, 1, Hd, a1, Hd, 1, grad + o.W2, Hd, Hd, Hd, (int)B, 1.f, 0.f, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum, dim3((Hd + 63) / 64), dim3(1024), 0, s, dZ, B, Hd, grad + o.b2);
  // dA1 = dZ2 W2
  if ((e = gemm<float>(dZ, Hd, 1, P + o.W2, Hd, 1, dA, Hd, (int)B, Hd, Hd, 1.f, 0.f, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_relu_back, dim3(blocks_for(B * Hd)), dim3(256), 0, s, dA, a1, dZ, B * Hd);
  if ((e = gemm<float>(dZ, 1, Hd, X, D, 1, grad + o.W1, D, Hd, D, (int)B, 1.f, 0.f, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum, dim3((Hd + 63) / 64), dim3(1024), 0, s, dZ, B, Hd, grad + o.b1);
  return hipGetLastError();
}

hipError_t mlp_mse(const float* Y, const float* T, int64_t B, int F, float* dY, double* part,
                   double* loss, hipStream_t s) {
  const int nb = 64;
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, Y, T, B * F, 1.f / (float)B, dY, part);
  hipLaunchKernelGGL(k_sum_small, dim3(1), dim3(64), 0, s, part, nb, loss);
  return hipGetLastError();
}

hipError_t mlp_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                    float b2, float eps, int step, void* p16, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps,
                     c1, c2, (__half*)p16);
  return hipGetLastError();
}

hipError_t mlp_features(const double* G, const double* W, int64_t rows, int F,
                        const double* rho_p, double rho_v, float* X, float* scale, hipStream_t s) {
  hipLaunchKernelGGL(k_features, dim3((unsigned)((rows + 63) / 64)), dim3(256), 0, s, G, W, rows,
                     F, rho_p, rho_v, X, scale);
  return hipGetLastError();
}

hipError_t gather_rows(const float* src, const int64_t* idx, int64_t n, int cols, float* dst,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_gather_rows, dim3(blocks_for(n * cols)), dim3(256), 0, s, src, idx, n, cols,
                     dst);
  return hipGetLastError();
}

template <typename HT>
static hipError_t judge_t(const float* Y, const float* scale, const double* G, const double* W,
                          HT* H, HT* U, int64_t rows, int F, int FL, const double* rho_p,
                          int rescale, int* taken, hipStream_t s) {
  const unsigned nb = (unsigned)((rows + (256 / FL) - 1) / (256 / FL));
  switch (FL) {
    case 4: hipLaunchKernelGGL((k_judge<HT, 4>), dim3(nb), dim3(256), 0, s, Y, scale, G, W, H, U, rows, F, rho_p, rescale, taken); break;
    case 8: hipLaunchKernelGGL((k_judge<HT, 8>), dim3(nb), dim3(256), 0, s, Y, scale, G, W, H, U, rows, F, rho_p, rescale, taken); break;
    case 16: hipLaunchKernelGGL((k_judge<HT, 16>), dim3(nb), dim3(256), 0, s, Y, scale, G, W, H, U, rows, F, rho_p, rescale, taken); break;
    case 32: hipLaunchKernelGGL((k_judge<HT, 32>), dim3(nb), dim3(256), 0, s, Y, scale, G, W, H, U, rows, F, rho_p, rescale, taken); break;
    default: hipLaunchKernelGGL((k_judge<HT, 64>), dim3(nb), dim3(256), 0, s, Y, scale, G, W, H, U, rows, F, rho_p, rescale, taken); break;
  }
  return hipGetLastError();
}

hipError_t mlp_judge(const float* Y, const float* scale, const double* G, const double* W, void* H,
                     void* U, int h_f64, int64_t rows, int F, int FL, const double* rho_p,
                     int rescale, int* taken, hipStream_t s) {
  if (h_f64)
    return judge_t<double>(Y, scale, G, W, (double*)H, (double*)U, rows, F, FL, rho_p, rescale,
                           taken, s);
  return judge_t<float>(Y, scale, G, W, (float*)H, (float*)U, rows, F, FL, rho_p, rescale, taken, s);
}

}  // namespace ntf
