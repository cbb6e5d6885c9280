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

__device__ inline double tlog(double x) { return log(x); }
__device__ inline float tlog(float x) { return logf(x); }

}  // namespace
}  // namespace nqs
