// Shared prefixes of the amplitude rows.  A row m of sample n differs from n at
// the sites c1 < c2 < c3 < ...; every row with the same first two changes
// (c1, state of m at c1, c2, state at c2) runs through the same hidden states
// up to its third changed site c3 (the conditionals of Eqs. (9)-(10) at a site
// see only the occupations below it).  Such a group is a node: the ONV of n
// with sites c1 and c2 set to the rows' states there (a row with a single
// change has c2 = K and shares a node with the rows of the same first change
// and no second one).  The node is evaluated from c1 (resumed from its sample)
// and stores its carried states and log-product states for the sites
// c1 .. e, e = the largest c3 of its rows; each row then resumes at c3 from the
// node.  Rows with fewer than three changed sites resume at K.
//
// With `pair` false (chosen by the caller, and always for K > 30, where the
// table of pair keys does not fit the LDS) nodes are keyed by the first change
// alone and rows resume at their second changed site.
//
// Three launches per pass of rows, all deterministic:
//   count:  one workgroup per sample marks the keys present among its rows in
//           an LDS table holding the set of resume sites per key (a bit mask,
//           whose highest site is e); writes the sample's node count and
//           storage entries (sum of e - c1 + 1);
//   scan:   one workgroup: exclusive offsets over the samples; a sample's
//           nodes are kept only if all of them fit the storage capacity
//           (whole samples in order, so the choice is deterministic);
//   assign: one workgroup per sample rebuilds the table, numbers its nodes in
//           key order, writes the node list and, per row, the node and the
//           site it resumes at (rows of samples without nodes resume at c1).
// The assign launch also marks, per node, the sites whose carried states its
// rows read when they resume at their own resume sites (need); after the rows
// are sorted by resume site, a fourth launch adds the sites read by rows whose
// wavefront starts below their own site.  The node pass stores only those
// carried states (and every log-product state); the tensor-term kernels store
// all of them.
#include "internal.h"

namespace nqs {
namespace {

constexpr int kNodeThreads = 256;

// key of a row and the site its row resumes at (pair keys when `pair`)
struct RowKey {
  int key, c1, res;
};

__device__ inline RowKey row_key(uint8_t t0, uint32_t v, int K, bool pair) {
  RowKey k;
  k.c1 = t0;
  const int c2 = int(v & 0xFF), s1 = int((v >> 8) & 3), c3 = int((v >> 16) & 0xFF), s2 = int((v >> 24) & 3);
  if (pair) {
    k.key = ((k.c1 * 4 + s1) * (K + 1) + c2) * 4 + (c2 < K ? s2 : 0);
    k.res = c3;
  } else {
    k.key = k.c1 * 4 + s1;
    k.res = c2;
  }
  return k;
}

__device__ inline int key_c1(int key, int K, bool pair) { return pair ? key / (16 * (K + 1)) : key / 4; }

// table of one sample: e[key] = the set of its rows' resume sites, bit res - 1
// (0 = key absent; res > c1 >= 0); the sample's own row (t0 = K) has no key.
// M = unsigned int for pair keys (K <= 30), unsigned long long for first-change
// keys.
template <typename M>
__device__ void build_table(const uint8_t* t0, const uint32_t* sec, int64_t r0, int64_t r1, int K, bool pair,
                            int T, M* e) {
  for (int k = threadIdx.x; k < T; k += blockDim.x) e[k] = 0;
  __syncthreads();
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    if (t0[r] >= K) continue;
    const RowKey k = row_key(t0[r], sec[r], K, pair);
    atomicOr(&e[k.key], M(1) << (k.res - 1));
  }
  __syncthreads();
}

// the largest resume site in a table entry
template <typename M> __device__ inline int last_res(M m) {
  return sizeof(M) == 4 ? 32 - __clz(uint32_t(m)) : 64 - __clzll((unsigned long long)m);
}

// the sites (bit s) whose carried states rows resuming at the sites of m read
// from a node with changed site c1: s in [res - W + 1, res - 1], s >= c1
template <typename M> __device__ inline uint64_t need_of(M m, int W, int c1) {
  const uint64_t b = uint64_t(m);   // bit res - 1
  uint64_t need = 0;
  for (int w = 0; w < W - 1; ++w) need |= b >> w;
  return need & ~((1ull << c1) - 1ull);
}

// block-wide exclusive scan of (count, entries) pairs held one per thread
__device__ void block_scan(int& cnt, int64_t& ent, int* sc, int64_t* se, int& tot_cnt, int64_t& tot_ent) {
  const int tid = threadIdx.x;
  sc[tid] = cnt;
  se[tid] = ent;
  __syncthreads();
  for (int d = 1; d < kNodeThreads; d <<= 1) {
    const int vc = tid >= d ? sc[tid - d] : 0;
    const int64_t ve = tid >= d ? se[tid - d] : 0;
    __syncthreads();
    sc[tid] += vc;
    se[tid] += ve;
    __syncthreads();
  }
  tot_cnt = sc[kNodeThreads - 1];
  tot_ent = se[kNodeThreads - 1];
  cnt = tid > 0 ? sc[tid - 1] : 0;
  ent = tid > 0 ? se[tid - 1] : 0;
  __syncthreads();
}

template <typename M>
__global__ __launch_bounds__(kNodeThreads) void k_node_count(const uint8_t* __restrict__ t0,
                                                             const uint32_t* __restrict__ sec, const int64_t* rowptr,
                                                             int64_t n0, int64_t row_base, int K, int32_t* ncnt,
                                                             int64_t* nent) {
  extern __shared__ unsigned long long lds_table[];
  M* e = reinterpret_cast<M*>(lds_table);
  __shared__ int sc[kNodeThreads];
  __shared__ int64_t se[kNodeThreads];
  constexpr bool pair = sizeof(M) == 4;
  const int T = pair ? 16 * K * (K + 1) : 4 * K;
  const int64_t n = n0 + blockIdx.x;
  build_table(t0, sec, rowptr[n] - row_base, rowptr[n + 1] - row_base, K, pair, T, e);
  int cnt = 0;
  int64_t ent = 0;
  for (int k = threadIdx.x; k < T; k += blockDim.x)
    if (e[k]) {
      ++cnt;
      ent += last_res(e[k]) - key_c1(k, K, pair) + 1;
    }
  int tc;
  int64_t te;
  block_scan(cnt, ent, sc, se, tc, te);
  if (threadIdx.x == 0) {
    ncnt[blockIdx.x] = tc;
    nent[blockIdx.x] = te;
  }
}

// one workgroup of 1024 threads over the ns samples of the pass: exclusive
// offsets; samples whose entries end beyond cap get no nodes (count 0)
__global__ __launch_bounds__(1024) void k_node_scan(int64_t ns, int64_t cap, int32_t* ncnt, int64_t* nent,
                                                    int64_t* nbase, int64_t* ebase, int64_t* totals) {
  __shared__ int64_t pc[1024], pe[1024];
  const int tid = threadIdx.x;
  const int64_t per = (ns + 1023) / 1024;
  const int64_t a = tid * per, b = a + per < ns ? a + per : ns;
  int64_t sc = 0, se = 0;
  for (int64_t i = a; i < b; ++i) {
    sc += ncnt[i];
    se += nent[i];
  }
  pc[tid] = sc;
  pe[tid] = se;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int64_t vc = tid >= d ? pc[tid - d] : 0, ve = tid >= d ? pe[tid - d] : 0;
    __syncthreads();
    pc[tid] += vc;
    pe[tid] += ve;
    __syncthreads();
  }
  // entries in sample order decide acceptance; once a sample does not fit,
  // no later one does (the running sum only grows), so the accepted samples
  // are a prefix and their nodes and entries are numbered contiguously
  int64_t rc = tid > 0 ? pc[tid - 1] : 0, re = tid > 0 ? pe[tid - 1] : 0;
  for (int64_t i = a; i < b; ++i) {
    const bool ok = re + nent[i] <= cap;
    nbase[i] = ok ? rc : -1;
    ebase[i] = re;
    rc += ncnt[i];
    re += nent[i];
  }
  __syncthreads();
  // totals: the end of the last accepted sample
  for (int64_t i = a; i < b; ++i)
    if (nbase[i] >= 0 && (i + 1 == ns || nbase[i + 1] < 0)) {
      totals[0] = nbase[i] + ncnt[i];
      totals[1] = ebase[i] + nent[i];
    }
  if (tid == 0 && nbase[0] < 0) {
    totals[0] = 0;
    totals[1] = 0;
  }
}

template <typename M>
__global__ __launch_bounds__(kNodeThreads) void k_node_assign(const uint8_t* __restrict__ t0,
                                                              const uint32_t* __restrict__ sec,
                                                              const uint64_t* __restrict__ samples,
                                                              const int64_t* rowptr, int64_t n0, int64_t row_base,
                                                              int K, int W, const int64_t* nbase,
                                                              const int64_t* ebase, NodeList nl, int32_t* row_node,
                                                              uint8_t* row_site) {
  extern __shared__ unsigned long long lds_table[];
  M* e = reinterpret_cast<M*>(lds_table);
  __shared__ int sc[kNodeThreads];
  __shared__ int64_t se[kNodeThreads];
  constexpr bool pair = sizeof(M) == 4;
  const int T = pair ? 16 * K * (K + 1) : 4 * K;
  const int64_t n = n0 + blockIdx.x;
  const int64_t r0 = rowptr[n] - row_base, r1 = rowptr[n + 1] - row_base;
  build_table(t0, sec, r0, r1, K, pair, T, e);
  const int64_t nb = nbase[blockIdx.x];
  const bool keep = nb >= 0;
  const uint64_t nlo = samples[2 * n], nhi = samples[2 * n + 1];
  // each thread numbers the keys of one contiguous chunk, in key order
  const int chunk = (T + kNodeThreads - 1) / kNodeThreads;
  const int k0 = threadIdx.x * chunk, k1 = k0 + chunk < T ? k0 + chunk : T;
  int cnt = 0;
  int64_t ent = 0;
  for (int k = k0; k < k1; ++k)
    if (e[k]) {
      ++cnt;
      ent += last_res(e[k]) - key_c1(k, K, pair) + 1;
    }
  int tc;
  int64_t te;
  block_scan(cnt, ent, sc, se, tc, te);
  int j = cnt;
  int64_t off = ebase[blockIdx.x] + ent;
  // after numbering, e[k] holds the key's node (all ones: none)
  for (int k = k0; k < k1; ++k) {
    const M ek = e[k];
    if (!ek) {
      e[k] = M(~M(0));
      continue;
    }
    const int c1 = key_c1(k, K, pair), last = last_res(ek);
    if (keep) {
      const int64_t node = nb + j;
      uint64_t lo = nlo, hi = nhi;
      const int s1 = pair ? (k / (4 * (K + 1))) % 4 : k % 4;
      int P = 2 * c1;
      if (P < 64) lo = (lo & ~(3ull << P)) | (uint64_t(s1) << P);
      else hi = (hi & ~(3ull << (P - 64))) | (uint64_t(s1) << (P - 64));
      if (pair) {
        const int c2 = (k / 4) % (K + 1), s2 = k % 4;
        if (c2 < K) {
          P = 2 * c2;
          if (P < 64) lo = (lo & ~(3ull << P)) | (uint64_t(s2) << P);
          else hi = (hi & ~(3ull << (P - 64))) | (uint64_t(s2) << (P - 64));
        }
      }
      nl.m[2 * node] = lo;
      nl.m[2 * node + 1] = hi;
      nl.owner[node] = int32_t(n);
      nl.c1[node] = uint8_t(c1);
      nl.e1[node] = uint8_t(last);
      nl.off[node] = off;
      nl.need[node] = need_of(ek, W, c1);
      e[k] = M(node);
    } else {
      e[k] = M(~M(0));
    }
    ++j;
    off += last - c1 + 1;
  }
  __syncthreads();
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    if (t0[r] >= K) {
      row_node[r] = -1;
      row_site[r] = uint8_t(K);
      continue;
    }
    const RowKey k = row_key(t0[r], sec[r], K, pair);
    const M ek = e[k.key];
    const int node = ek == M(~M(0)) ? -1 : int(ek);
    row_node[r] = node;
    row_site[r] = uint8_t(node >= 0 ? k.res : k.c1);
  }
}

// thread per sorted row position p: a wavefront of the row pass starts at the
// resume site of its first position, a multiple of its row count (16, 32 or
// 64), and reads the carried states of the W - 1 sites below that start; the
// positions are sorted by resume site, so that start lies between the site at
// the 64-aligned position at or below p and p's own site.  Where the two are
// equal the assign launch has marked the sites already (from the row's own
// resume site); otherwise the range marked covers both ends (and only sites
// from the node's changed site on: below it the row reads its sample's
// states).
__global__ __launch_bounds__(256) void k_node_need(const int32_t* __restrict__ perm, const uint8_t* __restrict__ t0s,
                                                   int64_t R, int W, const int32_t* __restrict__ row_node,
                                                   const uint8_t* __restrict__ nc1, uint64_t* __restrict__ need) {
  const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (p >= R) return;
  const int s0 = t0s[p & ~int64_t(63)];
  if (s0 == int(t0s[p])) return;
  const int nd = row_node[perm[p]];
  if (nd < 0) return;
  const int start = s0 - W + 1;
  const int lo = start > int(nc1[nd]) ? start : int(nc1[nd]);
  const int hi = int(t0s[p]) - 1;   // <= 63
  if (hi < lo) return;
  const uint64_t upto = hi >= 63 ? ~0ull : (1ull << (hi + 1)) - 1ull;
  atomicOr(reinterpret_cast<unsigned long long*>(need + nd), (unsigned long long)(upto & ~((1ull << lo) - 1ull)));
}

}  // namespace

bool node_pairs(int K) { return 16 * K * (K + 1) * int(sizeof(int)) <= 60 * 1024; }

hipError_t launch_node_count(const uint8_t* t0, const uint32_t* sec, const int64_t* rowptr, int64_t n0, int64_t n1,
                             int64_t row_base, int K, bool pair, int32_t* ncnt, int64_t* nent, hipStream_t st) {
  if (n1 <= n0) return hipSuccess;
  if (K < 1 || K > 64 || (pair && !node_pairs(K))) return hipErrorInvalidValue;
  if (pair)
    hipLaunchKernelGGL(k_node_count<unsigned int>, dim3(unsigned(n1 - n0)), dim3(kNodeThreads),
                       size_t(16 * K * (K + 1)) * 4, st, t0, sec, rowptr, n0, row_base, K, ncnt, nent);
  else
    hipLaunchKernelGGL(k_node_count<unsigned long long>, dim3(unsigned(n1 - n0)), dim3(kNodeThreads),
                       size_t(4 * K) * 8, st, t0, sec, rowptr, n0, row_base, K, ncnt, nent);
  return hipGetLastError();
}

hipError_t launch_node_scan(int64_t ns, int64_t cap, int32_t* ncnt, int64_t* nent, int64_t* nbase, int64_t* ebase,
                            int64_t* totals, hipStream_t st) {
  if (ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_node_scan, dim3(1), dim3(1024), 0, st, ns, cap, ncnt, nent, nbase, ebase, totals);
  return hipGetLastError();
}

hipError_t launch_node_assign(const uint8_t* t0, const uint32_t* sec, const uint64_t* samples,
                              const int64_t* rowptr, int64_t n0, int64_t n1, int64_t row_base, int K, int W,
                              bool pair, const int64_t* nbase, const int64_t* ebase, const NodeList& nl,
                              int32_t* row_node, uint8_t* row_site, hipStream_t st) {
  if (n1 <= n0) return hipSuccess;
  if (K < 1 || K > 64 || W < 1 || W > 64 || (pair && !node_pairs(K))) return hipErrorInvalidValue;
  if (pair)
    hipLaunchKernelGGL(k_node_assign<unsigned int>, dim3(unsigned(n1 - n0)), dim3(kNodeThreads),
                       size_t(16 * K * (K + 1)) * 4, st, t0, sec, samples, rowptr, n0, row_base, K, W, nbase, ebase,
                       nl, row_node, row_site);
  else
    hipLaunchKernelGGL(k_node_assign<unsigned long long>, dim3(unsigned(n1 - n0)), dim3(kNodeThreads),
                       size_t(4 * K) * 8, st, t0, sec, samples, rowptr, n0, row_base, K, W, nbase, ebase, nl,
                       row_node, row_site);
  return hipGetLastError();
}

hipError_t launch_node_need(const int32_t* perm, const uint8_t* t0s, int64_t R, int W, const int32_t* row_node,
                            const uint8_t* nc1, uint64_t* need, hipStream_t st) {
  if (R <= 0) return hipSuccess;
  if (W < 1 || W > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_node_need, dim3(unsigned((R + 255) / 256)), dim3(256), 0, st, perm, t0s, R, W, row_node, nc1,
                     need);
  return hipGetLastError();
}

}  // namespace nqs
