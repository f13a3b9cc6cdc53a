// Device-side helpers shared by the gfx950 kernels of libntf_admm.
//
// MFMA operand/result layouts (one wave of 64 lanes, lane l, n = l % 16,
// g = l / 16), as used by every contraction kernel here:
//   v_mfma_f32_16x16x4_f32 / v_mfma_f64_16x16x4_f64 (D = A[16x4] B[4x16] + C):
//     lane supplies A[n][g] and B[g][n];
//     f32 result: element i of the lane's 4 holds D[4g + i][n];
//     f64 result: element i holds D[g + 4i][n].
//   v_mfma_f32_16x16x32_bf16 (A 16x32, B 32x16, 8 bf16 per lane):
//     lane supplies A[n][8g .. 8g+7] and B[8g .. 8g+7][n];
//     result element i holds D[4g + i][n].
// The contraction index of one instruction may be permuted freely as long as
// A and B use the same permutation; the kernels use that to turn 16-byte
// vector loads into operands.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ntf {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;

template <> struct Mfma<float> {
  typedef f32x4 acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of the 16x16 result held in accumulator element i by lane group g
  static __device__ __forceinline__ int row(int g, int i) { return 4 * g + i; }
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
};

template <> struct Mfma<double> {
  typedef f64x4 acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int i) { return g + 4 * i; }
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
};

static __device__ __forceinline__ f32x4 mma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Four consecutive elements starting at p (p + 3 must be in bounds when full).
template <typename T> struct Vec4Load;
template <> struct Vec4Load<float> {
  static __device__ __forceinline__ void load(const float* p, float (&v)[4]) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
  }
};
template <> struct Vec4Load<double> {
  static __device__ __forceinline__ void load(const double* p, double (&v)[4]) {
    const double2 a = reinterpret_cast<const double2*>(p)[0];
    const double2 b = reinterpret_cast<const double2*>(p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  }
};

template <typename T> struct Vec2Load;
template <> struct Vec2Load<float> {
  static __device__ __forceinline__ void load(const float* p, float (&v)[4]) {
    const float2 a = reinterpret_cast<const float2*>(p)[0];
    const float2 b = reinterpret_cast<const float2*>(p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  }
};
template <> struct Vec2Load<double> {
  static __device__ __forceinline__ void load(const double* p, double (&v)[4]) {
    Vec4Load<double>::load(p, v);
  }
};

// Four consecutive row elements.  vec = 4: p is 16-byte aligned (row length
// a multiple of 4); vec = 2: p is aligned to two elements (even row length);
// otherwise element loads.  `valid` < 4 at a row's end: the rest read as 0.
template <typename T>
static __device__ __forceinline__ void load4(const T* p, int valid, int vec, T (&v)[4]) {
  if (vec == 4 && valid >= 4) {
    Vec4Load<T>::load(p, v);
  } else if (vec == 2 && valid >= 4) {
    Vec2Load<T>::load(p, v);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = (c < valid) ? p[c] : T(0);
  }
}

// Raw buffer resources (stride 0, num_records in bytes): the fourth word for
// gfx9-family parts.  kBufferOOB (the launch header) is a byte offset past
// any resource used here: a load past num_records returns zeros, a store
// there is dropped.
constexpr int kBufferWord3 = 0x00020000;
// Cache-policy bits of a buffer access (gfx9-family encoding of the aux
// operand): non-temporal.
constexpr int kAuxNonTemporal = 2;

// A raw buffer resource over [p, p + bytes) whose words are read from the
// first lane: the resource sits in scalar registers even where the compiler
// cannot prove p wave-uniform (p must be wave-uniform).
static __device__ __forceinline__ __amdgpu_buffer_rsrc_t uniform_rsrc(const void* p, int bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  void* q = reinterpret_cast<void*>(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(q, (short)0, __builtin_amdgcn_readfirstlane(bytes),
                                           kBufferWord3);
}

// Reduce across the `width` lanes of an aligned lane group (width a power of 2, <= 64).
template <typename T>
static __device__ __forceinline__ T group_sum(T v, int width) {
  for (int off = width >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, width);
  return v;
}

// Value of lane l's v (wave-uniform l) in every lane.
static __device__ __forceinline__ double lane_value_d(double v, int l) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum of the partials p = g, g+G, g+2G, ... < nparts of one element, in
// increasing p (one group of the fixed-order grouped reductions).
template <typename PT>
static __device__ __forceinline__ double group_partial(const PT* __restrict__ base, int64_t pstride,
                                                       int nparts, int g, int G) {
  double s = 0.0;
#pragma unroll 4
  for (int p = g; p < nparts; p += G) s += (double)base[(int64_t)p * pstride];
  return s;
}

}  // namespace ntf
