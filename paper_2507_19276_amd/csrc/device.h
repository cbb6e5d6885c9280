// Device helpers shared by the amplitude kernels (forward FP64/FP32 and BF16).
#pragma once
#include "internal.h"
#include <cmath>

namespace nqs {
namespace {


typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct V4;
template <> struct V4<double> { typedef d4 type; };
template <> struct V4<float> { typedef f4 type; };

__device__ inline d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int site_state(uint64_t lo, uint64_t hi, int i) {
  const int P = 2 * i;
  const uint64_t w = P < 64 ? (lo >> P) : (hi >> (P - 64));
  return int(w & 3ull);
}

__device__ inline bool allowed(int a_prev, int b_prev, int s, int rest, int na, int nb) {
  const int a = a_prev + (s & 1), b = b_prev + (s >> 1);
  return a <= na && a + rest >= na && b <= nb && b + rest >= nb;
}

// mask of the n lowest bits (n <= 0: none, n >= 64: all)
__device__ inline uint64_t low_bits(int n) { return n <= 0 ? 0ull : (n >= 64 ? ~0ull : ((1ull << n) - 1ull)); }

__device__ inline double tlog(double x) { return log(x); }
__device__ inline float tlog(float x) { return logf(x); }

// ---------------------------------------------------------------------------
// Multi-tile forward: one wavefront owns NTL tiles of 16 rows.  Every A operand
// fetched from memory feeds NTL MFMAs; after the per-tile partial sums in the
// MFMA output layout, a reduce-scatter across the four lane groups
// (permlane32_swap / permlane16_swap, plain VALU) leaves each lane group with
// the full sums of one tile, so the per-row work (mask, normalisation, sign)
// runs once per row instead of once per lane group.  log|Phi| is accumulated
// as a renormalised product of the conditionals P^{s_i} / Z_i (mantissa in T,
// exponent as an integer) and converted with one log at the end.
// ---------------------------------------------------------------------------
__device__ inline void pl16(float a, float b, float& na, float& nb) {
  auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  na = __uint_as_float(r[0]);
  nb = __uint_as_float(r[1]);
}
__device__ inline void pl32(float a, float b, float& na, float& nb) {
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  na = __uint_as_float(r[0]);
  nb = __uint_as_float(r[1]);
}
__device__ inline void pl16(double a, double b, double& na, double& nb) {
  const uint64_t ua = __double_as_longlong(a), ub = __double_as_longlong(b);
  auto lo = __builtin_amdgcn_permlane16_swap(uint32_t(ua), uint32_t(ub), false, false);
  auto hi = __builtin_amdgcn_permlane16_swap(uint32_t(ua >> 32), uint32_t(ub >> 32), false, false);
  na = __longlong_as_double(int64_t(uint64_t(lo[0]) | (uint64_t(hi[0]) << 32)));
  nb = __longlong_as_double(int64_t(uint64_t(lo[1]) | (uint64_t(hi[1]) << 32)));
}
__device__ inline void pl32(double a, double b, double& na, double& nb) {
  const uint64_t ua = __double_as_longlong(a), ub = __double_as_longlong(b);
  auto lo = __builtin_amdgcn_permlane32_swap(uint32_t(ua), uint32_t(ub), false, false);
  auto hi = __builtin_amdgcn_permlane32_swap(uint32_t(ua >> 32), uint32_t(ub >> 32), false, false);
  na = __longlong_as_double(int64_t(uint64_t(lo[0]) | (uint64_t(hi[0]) << 32)));
  nb = __longlong_as_double(int64_t(uint64_t(lo[1]) | (uint64_t(hi[1]) << 32)));
}

// x[t] is lane group g's partial of tile t; returns the sum over the four lane
// groups of tile own(g): own = g (4 tiles), g/2 (2 tiles), 0 (1 tile).
// permlane32_swap(a, b) exchanges the upper half of a with the lower half of
// b; permlane16_swap(a, b) exchanges the odd 16-lane rows of a with the even
// rows of b.
template <typename T, int NTL> struct ReduceOwn;
template <typename T> struct ReduceOwn<T, 4> {
  __device__ static T run(const T (&x)[4]) {
    T a, b, c, d;
    pl32(x[0], x[2], a, b);
    const T y02 = a + b;      // lanes 0-31: tile 0, lanes 32-63: tile 2
    pl32(x[1], x[3], c, d);
    const T y13 = c + d;      // lanes 0-31: tile 1, lanes 32-63: tile 3
    pl16(y02, y13, a, b);
    return a + b;             // lane group g: tile g
  }
};
template <typename T> struct ReduceOwn<T, 2> {
  __device__ static T run(const T (&x)[2]) {
    T a, b;
    pl32(x[0], x[1], a, b);
    const T y = a + b;        // lanes 0-31: tile 0, lanes 32-63: tile 1 (pair sums)
    pl16(y, y, a, b);
    return a + b;
  }
};
template <typename T> struct ReduceOwn<T, 1> {
  __device__ static T run(const T (&x)[1]) {
    T a, b;
    pl32(x[0], x[0], a, b);
    const T y = a + b;
    pl16(y, y, a, b);
    return a + b;
  }
};

__device__ inline float tfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double tfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float tfrexp(float x, int* e) { return frexpf(x, e); }
__device__ inline double tfrexp(double x, int* e) { return frexp(x, e); }

// read-only uniform tables in the constant address space: the compiler reads
// them with scalar loads
typedef const __attribute__((address_space(4))) int CInt;
template <typename T> using CT = const __attribute__((address_space(4))) T;

#ifndef NQS_MFMA_PRIO
#define NQS_MFMA_PRIO 2
#endif
constexpr int PRIO = NQS_MFMA_PRIO;

}  // namespace
}  // namespace nqs
