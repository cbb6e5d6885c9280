// Shared prefixes of the amplitude rows, one level deep.  A row m of sample n
// differs from n at the sites c1 < c2 < ...; every row with the same first
// change (c1, state of m at c1) runs through the same hidden states up to
// its second changed site c2 (the conditionals of Eqs. (9)-(10) at a site
// see only the occupations below it).  Such a group is a node: the ONV of n
// with site c1 set to the row's state there.  The node is evaluated once from
// c1 (resumed from its sample) and stores its carried states and log-product
// states for sites c1 .. e1, e1 = the largest c2 of its rows; each row then
// resumes at c2 from the node.  Rows with a single changed site resume at K.
//
// Three launches per pass of rows, all deterministic:
//   count:  one workgroup per sample marks the keys (c1, state) present among
//           its rows in an LDS table and the largest c2 per key; writes the
//           sample's node count and storage entries (sum of e1 - c1 + 1);
//   scan:   one workgroup: exclusive offsets over the samples; a sample's
//           nodes are kept only if all of them fit the storage capacity
//           (whole samples in order, so the choice is deterministic);
//   assign: one workgroup per sample rebuilds the table, numbers its nodes in
//           key order, writes the node list and, per row, the node and the
//           site it resumes at (rows of samples without nodes resume at c1).
#include "internal.h"

namespace nqs {
namespace {

// table of one sample: e[key] = largest c2 + 1 (0 = key absent), key =
// c1 * 4 + state at c1, from the bytes the fill kernel wrote per row (the
// sample's own row has c1 = K)
__device__ void build_table(const uint8_t* t0, const uint16_t* sec, int64_t r0, int64_t r1, int K, int* e) {
  for (int k = threadIdx.x; k < 4 * K; k += blockDim.x) e[k] = 0;
  __syncthreads();
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    const int c1 = t0[r];
    if (c1 >= K) continue;
    const int v = sec[r];
    atomicMax(&e[c1 * 4 + (v >> 8)], (v & 0xFF) + 1);
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_node_count(const uint8_t* __restrict__ t0, const uint16_t* __restrict__ sec,
                                                    const int64_t* rowptr, int64_t n0, int64_t row_base, int K,
                                                    int32_t* ncnt, int64_t* nent) {
  __shared__ int e[256];
  const int64_t n = n0 + blockIdx.x;
  build_table(t0, sec, rowptr[n] - row_base, rowptr[n + 1] - row_base, K, e);
  if (threadIdx.x == 0) {
    int cnt = 0;
    int64_t ent = 0;
    for (int k = 0; k < 4 * K; ++k)
      if (e[k]) {
        ++cnt;
        ent += (e[k] - 1) - k / 4 + 1;
      }
    ncnt[blockIdx.x] = cnt;
    nent[blockIdx.x] = ent;
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

__global__ __launch_bounds__(256) void k_node_assign(const uint8_t* __restrict__ t0, const uint16_t* __restrict__ sec,
                                                     const uint64_t* __restrict__ samples, const int64_t* rowptr,
                                                     int64_t n0, int64_t row_base, int K, const int64_t* nbase,
                                                     const int64_t* ebase, NodeList nl,
                                                     int32_t* row_node, uint8_t* row_site) {
  __shared__ int e[256];
  __shared__ int id[256];
  const int64_t n = n0 + blockIdx.x;
  const int64_t r0 = rowptr[n] - row_base, r1 = rowptr[n + 1] - row_base;
  build_table(t0, sec, r0, r1, K, e);
  const int64_t nb = nbase[blockIdx.x];
  const bool keep = nb >= 0;
  const uint64_t nlo = samples[2 * n], nhi = samples[2 * n + 1];
  if (threadIdx.x == 0) {
    int j = 0;
    int64_t off = ebase[blockIdx.x];
    for (int k = 0; k < 4 * K; ++k) {
      id[k] = -1;
      if (!e[k]) continue;
      const int c1 = k / 4, e1 = e[k] - 1;
      if (keep) {
        const int64_t node = nb + j;
        id[k] = int(node);
        const int P = 2 * c1;
        uint64_t lo = nlo, hi = nhi;
        if (P < 64) lo = (lo & ~(3ull << P)) | (uint64_t(k & 3) << P);
        else hi = (hi & ~(3ull << (P - 64))) | (uint64_t(k & 3) << (P - 64));
        nl.m[2 * node] = lo;
        nl.m[2 * node + 1] = hi;
        nl.owner[node] = int32_t(n);
        nl.c1[node] = uint8_t(c1);
        nl.e1[node] = uint8_t(e1);
        nl.off[node] = off;
      }
      ++j;
      off += e1 - c1 + 1;
    }
  }
  __syncthreads();
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    const int c1 = int(t0[r]);
    const int v = sec[r];
    const int node = c1 < K ? id[c1 * 4 + (v >> 8)] : -1;
    row_node[r] = node;
    row_site[r] = uint8_t(c1 >= K ? K : (node >= 0 ? (v & 0xFF) : c1));
  }
}

}  // namespace

hipError_t launch_node_count(const uint8_t* t0, const uint16_t* sec, const int64_t* rowptr, int64_t n0, int64_t n1,
                             int64_t row_base, int K, int32_t* ncnt, int64_t* nent, hipStream_t st) {
  if (n1 <= n0) return hipSuccess;
  if (K < 1 || K > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_node_count, dim3(unsigned(n1 - n0)), dim3(256), 0, st, t0, sec, rowptr, n0, row_base, K,
                     ncnt, nent);
  return hipGetLastError();
}

hipError_t launch_node_scan(int64_t ns, int64_t cap, int32_t* ncnt, int64_t* nent, int64_t* nbase, int64_t* ebase,
                            int64_t* totals, hipStream_t st) {
  if (ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_node_scan, dim3(1), dim3(1024), 0, st, ns, cap, ncnt, nent, nbase, ebase, totals);
  return hipGetLastError();
}

hipError_t launch_node_assign(const uint8_t* t0, const uint16_t* sec, const uint64_t* samples,
                              const int64_t* rowptr, int64_t n0, int64_t n1, int64_t row_base, int K,
                              const int64_t* nbase, const int64_t* ebase, const NodeList& nl, int32_t* row_node,
                              uint8_t* row_site, hipStream_t st) {
  if (n1 <= n0) return hipSuccess;
  hipLaunchKernelGGL(k_node_assign, dim3(unsigned(n1 - n0)), dim3(256), 0, st, t0, sec, samples, rowptr, n0,
                     row_base, K, nbase, ebase, nl, row_node, row_site);
  return hipGetLastError();
}

}  // namespace nqs
