// Merging sampled ONVs into unique ONVs with counts: a stable LSD radix sort of
// the two 64-bit words (low word, then high word when 2K > 64), head flags,
// an exclusive scan of the flags and a scatter of the heads; with weights, a
// unique ONV's count is the sum of its entries' weights (an inclusive scan of
// the weights in sorted order).  The sorts and scans are the hipCUB device
// primitives; the output is in ascending (high, low) order.
#include "internal.h"
#include <hipcub/hipcub.hpp>
#include <algorithm>

namespace nqs {
namespace {

__global__ void k_words(const uint64_t* __restrict__ m, int64_t N, int word, const uint32_t* __restrict__ idx,
                        uint64_t* __restrict__ key, uint32_t* __restrict__ ord) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const uint32_t src = idx ? idx[i] : uint32_t(i);
  key[i] = m[2 * size_t(src) + word];
  ord[i] = src;
}

__global__ void k_heads(const uint64_t* __restrict__ m, int64_t N, const uint32_t* __restrict__ ord,
                        int32_t* __restrict__ flag) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  bool head = i == 0;
  if (!head) {
    const uint32_t a = ord[i], b = ord[i - 1];
    head = m[2 * size_t(a)] != m[2 * size_t(b)] || m[2 * size_t(a) + 1] != m[2 * size_t(b) + 1];
  }
  flag[i] = head ? 1 : 0;
}

// heads write their unique ONV, amplitude and start; nu = number of unique
__global__ void k_scatter_heads(const uint64_t* __restrict__ m, const double* __restrict__ lphi,
                                const int8_t* __restrict__ sphi, int64_t N, const uint32_t* __restrict__ ord,
                                const int32_t* __restrict__ flag, const int32_t* __restrict__ pos, int64_t cap,
                                uint64_t* __restrict__ um, double* __restrict__ ul, int8_t* __restrict__ us,
                                int64_t* __restrict__ start, int64_t* __restrict__ nu) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  if (i == N - 1) *nu = int64_t(pos[i]) + flag[i];
  if (!flag[i]) return;
  const int64_t u = pos[i];
  start[u] = i;
  if (u >= cap) return;
  const uint32_t a = ord[i];
  um[2 * u] = m[2 * size_t(a)];
  um[2 * u + 1] = m[2 * size_t(a) + 1];
  if (ul) ul[u] = lphi[a];
  if (us) us[u] = sphi[a];
}

// count of unique ONV u: the number of its entries, or with weights the sum of
// their weights (difference of the inclusive prefix sums wsum in sorted order)
__global__ void k_counts(int64_t N, const int64_t* __restrict__ start, const int64_t* __restrict__ nu, int64_t cap,
                         const int64_t* __restrict__ wsum, int64_t* __restrict__ cnt) {
  const int64_t u = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t n = *nu;
  if (u >= n || u >= cap) return;
  const int64_t a = start[u], b = u + 1 < n ? start[u + 1] : N;
  cnt[u] = wsum ? wsum[b - 1] - (a > 0 ? wsum[a - 1] : 0) : b - a;
}

__global__ void k_gather_weights(int64_t N, const uint32_t* __restrict__ ord, const int64_t* __restrict__ wt,
                                 int64_t* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < N) out[i] = wt[ord[i]];
}

__global__ void k_fill_i64(int64_t* __restrict__ p, int64_t n, int64_t v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline unsigned blocks_for(int64_t n) { return unsigned((n + 255) / 256); }

}  // namespace

hipError_t unique_temp_bytes(int64_t N, size_t* bytes) {
  size_t a = 0, b = 0;
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, a, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                                    (const uint32_t*)nullptr, (uint32_t*)nullptr, int(N), 0, 64);
  if (e != hipSuccess) return e;
  e = hipcub::DeviceScan::ExclusiveSum(nullptr, b, (const int32_t*)nullptr, (int32_t*)nullptr, int(N));
  if (e != hipSuccess) return e;
  size_t c = 0;
  e = hipcub::DeviceScan::InclusiveSum(nullptr, c, (const int64_t*)nullptr, (int64_t*)nullptr, int(N));
  if (e != hipSuccess) return e;
  *bytes = std::max(a, std::max(b, c));
  return hipSuccess;
}

hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i64, dim3(blocks_for(n)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_unique(const uint64_t* m, const double* lphi, const int8_t* sphi, const int64_t* weights,
                         int64_t N, bool two_words, const UniqueScratch& w, int64_t cap, uint64_t* um, int64_t* ucnt,
                         double* ul, int8_t* us, int64_t* nu, hipStream_t st) {
  if (N <= 0) return hipMemsetAsync(nu, 0, sizeof(int64_t), st);
  if (N >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  size_t tb = w.temp_bytes;
  hipLaunchKernelGGL(k_words, dim3(blocks_for(N)), dim3(256), 0, st, m, N, 0, nullptr, w.key_a, w.ord_a);
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(w.temp, tb, w.key_a, w.key_b, w.ord_a, w.ord_b, int(N), 0, 64, st);
  if (e != hipSuccess) return e;
  const uint32_t* ord = w.ord_b;
  if (two_words) {
    hipLaunchKernelGGL(k_words, dim3(blocks_for(N)), dim3(256), 0, st, m, N, 1, w.ord_b, w.key_a, w.ord_a);
    tb = w.temp_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(w.temp, tb, w.key_a, w.key_b, w.ord_a, w.ord_b, int(N), 0, 64, st);
    if (e != hipSuccess) return e;
    ord = w.ord_b;
  }
  hipLaunchKernelGGL(k_heads, dim3(blocks_for(N)), dim3(256), 0, st, m, N, ord, w.flag);
  tb = w.temp_bytes;
  e = hipcub::DeviceScan::ExclusiveSum(w.temp, tb, w.flag, w.pos, int(N), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scatter_heads, dim3(blocks_for(N)), dim3(256), 0, st, m, lphi, sphi, N, ord, w.flag, w.pos,
                     cap, um, ul, us, w.start, nu);
  if (weights) {
    hipLaunchKernelGGL(k_gather_weights, dim3(blocks_for(N)), dim3(256), 0, st, N, ord, weights, w.wsum);
    tb = w.temp_bytes;
    e = hipcub::DeviceScan::InclusiveSum(w.temp, tb, w.wsum, w.wsum, int(N), st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_counts, dim3(blocks_for(N)), dim3(256), 0, st, N, w.start, nu, cap,
                     weights ? w.wsum : nullptr, ucnt);
  return hipGetLastError();
}

}  // namespace nqs
