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
//           an LDS table with the largest resume site per key; writes the
//           sample's node count and storage entries (sum of e - c1 + 1);
//   scan:   one workgroup: exclusive offsets over the samples; a sample's
//           nodes are kept only if all of them fit the storage capacity
//           (whole samples in order, so the choice is deterministic);
//   assign: one workgroup per sample rebuilds the table, numbers its nodes in
//           key order, writes the node list and, per row, the node and the
//           site it resumes at (rows of samples without nodes resume at c1).
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

// table of one sample: e[key] = largest resume site + 1 (0 = key absent); the
// sample's own row (t0 = K) has no key
__device__ void build_table(const uint8_t* t0, const uint32_t* sec, int64_t r0, int64_t r1, int K, bool pair,
                            int T, int* e) {
  for (int k = threadIdx.x; k < T; k += blockDim.x) e[k] = 0;
  __syncthreads();
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    if (t0[r] >= K) continue;
    const RowKey k = row_key(t0[r], sec[r], K, pair);
    atomicMax(&e[k.key], k.res + 1);
  }
  __syncthreads();
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

__global__ __launch_bounds__(kNodeThreads) void k_node_count(const uint8_t* __restrict__ t0,
                                                             const uint32_t* __restrict__ sec, const int64_t* rowptr,
                                                             int64_t n0, int64_t row_base, int K, int pair_i,
                                                             int32_t* ncnt, int64_t* nent) {
  extern __shared__ int e[];
  __shared__ int sc[kNodeThreads];
  __shared__ int64_t se[kNodeThreads];
  const bool pair = pair_i != 0;
  const int T = pair ? 16 * K * (K + 1) : 4 * K;
  const int64_t n = n0 + blockIdx.x;
  build_table(t0, sec, rowptr[n] - row_base, rowptr[n + 1] - row_base, K, pair, T, e);
  int cnt = 0;
  int64_t ent = 0;
  for (int k = threadIdx.x; k < T; k += blockDim.x)
    if (e[k]) {
      ++cnt;
      ent += (e[k] - 1) - key_c1(k, K, pair) + 1;
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

__global__ __launch_bounds__(kNodeThreads) void k_node_assign(const uint8_t* __restrict__ t0,
                                                              const uint32_t* __restrict__ sec,
                                                              const uint64_t* __restrict__ samples,
                                                              const int64_t* rowptr, int64_t n0, int64_t row_base,
                                                              int K, int pair_i, const int64_t* nbase,
                                                              const int64_t* ebase, NodeList nl, int32_t* row_node,
                                                              uint8_t* row_site) {
  extern __shared__ int e[];
  __shared__ int sc[kNodeThreads];
  __shared__ int64_t se[kNodeThreads];
  const bool pair = pair_i != 0;
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
      ent += (e[k] - 1) - key_c1(k, K, pair) + 1;
    }
  int tc;
  int64_t te;
  block_scan(cnt, ent, sc, se, tc, te);
  int j = cnt;
  int64_t off = ebase[blockIdx.x] + ent;
  for (int k = k0; k < k1; ++k) {
    const int ek = e[k];
    if (!ek) {
      e[k] = -1;
      continue;
    }
    const int c1 = key_c1(k, K, pair), last = ek - 1;
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
      e[k] = int(node);
    } else {
      e[k] = -1;
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
    const int node = e[k.key];
    row_node[r] = node;
    row_site[r] = uint8_t(node >= 0 ? k.res : k.c1);
  }
}

}  // namespace

bool node_pairs(int K) { return 16 * K * (K + 1) * int(sizeof(int)) <= 60 * 1024; }

hipError_t launch_node_count(const uint8_t* t0, const uint32_t* sec, const int64_t* rowptr, int64_t n0, int64_t n1,
                             int64_t row_base, int K, bool pair, int32_t* ncnt, int64_t* nent, hipStream_t st) {
  if (n1 <= n0) return hipSuccess;
  if (K < 1 || K > 64 || (pair && !node_pairs(K))) return hipErrorInvalidValue;
  const size_t lds = size_t(pair ? 16 * K * (K + 1) : 4 * K) * sizeof(int);
  hipLaunchKernelGGL(k_node_count, dim3(unsigned(n1 - n0)), dim3(kNodeThreads), lds, st, t0, sec, rowptr, n0,
                     row_base, K, pair ? 1 : 0, ncnt, nent);
  return hipGetLastError();
}

hipError_t launch_node_scan(int64_t ns, int64_t cap, int32_t* ncnt, int64_t* nent, int64_t* nbase, int64_t* ebase,
                            int64_t* totals, hipStream_t st) {
  if (ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_node_scan, dim3(1), dim3(1024), 0, st, ns, cap, ncnt, nent, nbase, ebase, totals);
  return hipGetLastError();
}

hipError_t launch_node_assign(const uint8_t* t0, const uint32_t* sec, const uint64_t* samples,
                              const int64_t* rowptr, int64_t n0, int64_t n1, int64_t row_base, int K, bool pair,
                              const int64_t* nbase, const int64_t* ebase, const NodeList& nl, int32_t* row_node,
                              uint8_t* row_site, hipStream_t st) {
  if (n1 <= n0) return hipSuccess;
  if (pair && !node_pairs(K)) return hipErrorInvalidValue;
  const size_t lds = size_t(pair ? 16 * K * (K + 1) : 4 * K) * sizeof(int);
  hipLaunchKernelGGL(k_node_assign, dim3(unsigned(n1 - n0)), dim3(kNodeThreads), lds, st, t0, sec, samples, rowptr,
                     n0, row_base, K, pair ? 1 : 0, nbase, ebase, nl, row_node, row_site);
  return hipGetLastError();
}

}  // namespace nqs
