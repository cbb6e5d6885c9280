// Row order for the resumed amplitude pass: a stable counting sort of the
// amplitude rows by their first changed site t0, the lowest site at which a
// row's ONV differs from its sample's (K when they are equal; the fill kernel
// writes it with the row).  The autoregressive conditionals of Eqs. (9)-(10)
// at sites below t0 depend only on the occupations below t0, which the row
// shares with its sample, so a row can resume at t0 from its sample's carried
// state; grouping rows by t0 lets a whole wavefront skip the shared prefix.
//
// Three launches, all deterministic:
//   count:   per block of kOrderChunk rows, a histogram of t0 (LDS atomics;
//            counts do not depend on their order);
//   scan:    one block per bucket: exclusive offsets of the bucket over the
//            blocks, and the bucket total;
//   scatter: each block walks its rows in order, 256 at a time; a row's
//            position is the bucket's base (sum of the lower totals) plus its
//            block offset, the rows of the bucket in earlier rounds, the rows
//            of the bucket in lower wavefronts of the round and the rows of the
//            bucket in lower lanes (one ballot per key bit), so equal keys
//            keep row order.
#include "internal.h"

namespace nqs {
namespace {

__global__ __launch_bounds__(256) void k_t0_count(const uint8_t* __restrict__ t0, int64_t R, int K,
                                                  int32_t* __restrict__ cnt) {
  __shared__ int h[65];
  for (int k = threadIdx.x; k <= K; k += 256) h[k] = 0;
  __syncthreads();
  const int64_t r0 = int64_t(blockIdx.x) * kOrderChunk;
  const int64_t r1 = r0 + kOrderChunk < R ? r0 + kOrderChunk : R;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) atomicAdd(&h[t0[r]], 1);
  __syncthreads();
  for (int k = threadIdx.x; k <= K; k += 256) cnt[int64_t(blockIdx.x) * (K + 1) + k] = h[k];
}

// block k scans column k of cnt[nb][K+1] in place (exclusive) and writes tot[k]
__global__ __launch_bounds__(256) void k_t0_scan(int32_t* __restrict__ cnt, int64_t nb, int K,
                                                 int64_t* __restrict__ tot) {
  __shared__ int64_t part[256];
  const int k = blockIdx.x, tid = threadIdx.x;
  const int64_t per = (nb + 255) / 256;
  const int64_t b0 = tid * per;
  const int64_t b1 = b0 + per < nb ? b0 + per : nb;
  int64_t s = 0;
  for (int64_t b = b0; b < b1; ++b) s += cnt[b * (K + 1) + k];
  part[tid] = s;
  __syncthreads();
  // inclusive scan of the 256 partial sums (Hillis-Steele)
  for (int d = 1; d < 256; d <<= 1) {
    const int64_t v = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int64_t run = tid > 0 ? part[tid - 1] : 0;
  for (int64_t b = b0; b < b1; ++b) {
    const int c = cnt[b * (K + 1) + k];
    cnt[b * (K + 1) + k] = int(run);
    run += c;
  }
  if (tid == 255) tot[k] = part[255];
}

__global__ __launch_bounds__(256) void k_t0_scatter(const uint8_t* __restrict__ t0, int64_t R, int K,
                                                    const int32_t* __restrict__ off,
                                                    const int64_t* __restrict__ tot, int32_t* __restrict__ perm,
                                                    uint8_t* __restrict__ t0s) {
  __shared__ int run[65];
  __shared__ int wc[4][65];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (threadIdx.x == 0) {
    int64_t acc = 0;
    for (int k = 0; k <= K; ++k) {
      run[k] = int(acc);
      acc += tot[k];
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k <= K; k += 256) {
    run[k] += off[int64_t(blockIdx.x) * (K + 1) + k];
    for (int w = 0; w < 4; ++w) wc[w][k] = 0;
  }
  __syncthreads();
  const int64_t r0 = int64_t(blockIdx.x) * kOrderChunk;
  const int64_t r1 = r0 + kOrderChunk < R ? r0 + kOrderChunk : R;
  const uint64_t below = (1ull << lane) - 1ull;
  for (int64_t rb = r0; rb < r1; rb += 256) {
    const int64_t r = rb + threadIdx.x;
    const bool valid = r < r1;
    const int t = valid ? int(t0[r]) : K;
    // the lanes of this wavefront with the same key (keys <= 64: one ballot per
    // key bit), and the rank among the lower ones
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 7; ++b) {
      const bool bit = (t >> b) & 1;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const int rank = __popcll(peers & below);
    if (valid && (peers & below) == 0) wc[wv][t] = __popcll(peers);
    __syncthreads();
    int pos = 0;
    if (valid) {
      pos = run[t] + rank;
      for (int w = 0; w < wv; ++w) pos += wc[w][t];
    }
    __syncthreads();
    for (int k = threadIdx.x; k <= K; k += 256) {
      int sum = 0;
      for (int w = 0; w < 4; ++w) {
        sum += wc[w][k];
        wc[w][k] = 0;
      }
      run[k] += sum;
    }
    __syncthreads();
    if (valid) {
      perm[pos] = int32_t(r);
      t0s[pos] = uint8_t(t);
    }
  }
}

// dst[p] = src[perm[p]]
__global__ __launch_bounds__(256) void k_gather_u8(const uint8_t* __restrict__ src, const int32_t* __restrict__ perm,
                                                   int64_t n, uint8_t* __restrict__ dst) {
  const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (p < n) dst[p] = src[perm[p]];
}

// out[p] = a[b[p]]
__global__ __launch_bounds__(256) void k_compose(const int32_t* __restrict__ a, const int32_t* __restrict__ b,
                                                 int64_t n, int32_t* __restrict__ out) {
  const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (p < n) out[p] = a[b[p]];
}

}  // namespace

hipError_t launch_order_t0(const uint8_t* t0, int64_t R, int K, int32_t* cnt, int64_t* tot, int32_t* perm,
                           uint8_t* t0s, hipStream_t st) {
  if (R <= 0) return hipSuccess;
  if (K < 1 || K > 64 || R >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  const int64_t nb = order_blocks(R);
  hipLaunchKernelGGL(k_t0_count, dim3(unsigned(nb)), dim3(256), 0, st, t0, R, K, cnt);
  hipLaunchKernelGGL(k_t0_scan, dim3(unsigned(K + 1)), dim3(256), 0, st, cnt, nb, K, tot);
  hipLaunchKernelGGL(k_t0_scatter, dim3(unsigned(nb)), dim3(256), 0, st, t0, R, K, cnt, tot, perm, t0s);
  return hipGetLastError();
}

// order by (t0, t1) ascending: a stable sort by t1, then a stable sort of
// the result by t0 (least significant key first); tmp: 2 R int32 and 2 R bytes
hipError_t launch_order_t0_t1(const uint8_t* t0, const uint8_t* t1, int64_t R, int K, int32_t* cnt, int64_t* tot,
                              int32_t* tmp_perm, uint8_t* tmp_key, int32_t* perm, uint8_t* t0s, hipStream_t st) {
  if (R <= 0) return hipSuccess;
  if (K < 1 || K > 64 || R >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  int32_t* p1 = tmp_perm;       // position -> row, sorted by t1
  int32_t* p2 = tmp_perm + R;   // position -> position of the first sort, sorted by t0
  uint8_t* k1 = tmp_key;        // t1 in the first order (not used further)
  uint8_t* g0 = tmp_key + R;    // t0 in the first order
  hipError_t e = launch_order_t0(t1, R, K, cnt, tot, p1, k1, st);
  if (e != hipSuccess) return e;
  const unsigned blocks = unsigned((R + 255) / 256);
  hipLaunchKernelGGL(k_gather_u8, dim3(blocks), dim3(256), 0, st, t0, p1, R, g0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_order_t0(g0, R, K, cnt, tot, p2, t0s, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_compose, dim3(blocks), dim3(256), 0, st, p1, p2, R, perm);
  return hipGetLastError();
}

}  // namespace nqs
