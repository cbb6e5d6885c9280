// Shared prefixes of the amplitude rows.  A row m of sample n differs from n at
// the sites c1 < c2 < c3 < ...; every row with the same first two changes
// (c1, state of m at c1, c2, state at c2) runs through the same hidden states
// up to its third changed site c3 (the conditionals of Eqs. (9)-(10) at a site
// see only the occupations below it).  Such a group is a node: the ONV of n
// with sites c1 and c2 set to the rows' states there (a row with a single
// change has c2 = K and shares a node with the rows of the same first change
// and no second one).  The node is evaluated from c1 (resumed from its sample)
// up to e = the largest c3 of its rows; each row then resumes at c3 from the
// node.  Rows with fewer than three changed sites resume at K.
//
// With `pair` false (chosen by the caller where the pair table does not fit
// the LDS) nodes are keyed by the first change alone and rows resume at their
// second changed site.
//
// Storage of a node u: the log-product state before every site c1 .. e
// (entries off[u] + (i - c1)), and the carried state after site i only where
// need[u] has bit i (slots coff[u] + popcount(need[u] & bits below i)).
//
// Pair keys are compact: a changed site's state is numbered among the three
// states other than the sample's there (s' = s - (s > sample's state)); the
// first change (c1, s1') has the sub-keys j = 0 (no second change) and
// j = 1 + 3 (c2 - c1 - 1) + s2' (c1 < c2 < K), L(c1) = 3 (K - 1 - c1) + 1 of
// them, and the keys of c1 start at pair_base(c1) = 3 sum_{c < c1} L(c).
// K = 50 has 11175 pair keys (87 KiB of 64-bit resume-site masks).
//
// Launches per pass of rows, all deterministic:
//   count:  one workgroup per sample marks the keys present among its rows in
//           an LDS table holding the set of resume sites per key (a bit mask,
//           whose highest site is e); writes the sample's node count, storage
//           entries (sum of e - c1 + 1) and carried-state slots its own rows
//           read;
//   scan:   one workgroup: exclusive offsets over the samples; a sample's
//           nodes are kept only if all of them fit the three capacities
//           (whole samples in order, so the choice is deterministic);
//   assign: one workgroup per sample rebuilds the table, numbers its nodes in
//           key order, writes the node list and, per row, the node and the
//           site it resumes at (rows of samples without nodes resume at c1).
// The assign launch also marks, per node, the sites whose carried states its
// rows read when they resume at their own resume sites (need); after the rows
// are sorted by resume site, a further launch adds the sites read by rows
// whose wavefront starts below their own site (at most 63 rows in each of the
// at most K 64-row blocks that straddle two resume sites, each adding fewer
// than K sites: the slot capacity keeps 64 K^2 for them), and three launches
// write each node's record with its first slot (an exclusive scan of
// popcount(need) over the nodes).  The node pass stores only those carried
// states (and every log-product state); the tensor-term kernels store all of
// them (need = every site from c1 on, coff = off).
#include "internal.h"

namespace nqs {
namespace {

constexpr int kNodeThreads = 512;

__host__ __device__ inline int pair_len(int c, int K) { return 3 * (K - 1 - c) + 1; }
__host__ __device__ inline int pair_base(int c, int K) { return 3 * (3 * (c * (K - 1) - c * (c - 1) / 2) + c); }
__host__ __device__ inline int table_keys(int K, bool pair) { return pair ? pair_base(K, K) : 4 * K; }

// the 2-bit state of site c in an ONV
__device__ inline int site_state(uint64_t lo, uint64_t hi, int c) {
  return c < 32 ? int((lo >> (2 * c)) & 3ull) : int((hi >> (2 * c - 64)) & 3ull);
}

// key of a row and the site its row resumes at (pair keys when `pair`); the
// sample's ONV numbers the changed sites' states
struct RowKey {
  int key, c1, res;
};

__device__ inline RowKey row_key(uint8_t t0, uint32_t v, int K, bool pair, uint64_t nlo, uint64_t nhi) {
  RowKey k;
  k.c1 = t0;
  const int c2 = int(v & 0xFF), s1 = int((v >> 8) & 3), c3 = int((v >> 16) & 0xFF), s2 = int((v >> 24) & 3);
  if (pair) {
    const int a1 = s1 - (s1 > site_state(nlo, nhi, k.c1) ? 1 : 0);
    const int j = c2 < K ? 1 + 3 * (c2 - k.c1 - 1) + s2 - (s2 > site_state(nlo, nhi, c2) ? 1 : 0) : 0;
    k.key = pair_base(k.c1, K) + a1 * pair_len(k.c1, K) + j;
    k.res = c3;
  } else {
    k.key = k.c1 * 4 + s1;
    k.res = c2;
  }
  return k;
}

// the first changed site of a key: the largest c with pair_base(c) <= key
__device__ inline int key_c1(int key, int K, bool pair) {
  if (!pair) return key / 4;
  int lo = 0, hi = K - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pair_base(mid, K) <= key) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// table of one sample: e[key] = the set of its rows' resume sites, bit res - 1
// (0 = key absent; res > c1 >= 0, res <= K <= 64); the sample's own row (t0 =
// K) has no key
__device__ void build_table(const uint8_t* t0, const uint32_t* sec, int64_t r0, int64_t r1, int K, bool pair,
                            uint64_t nlo, uint64_t nhi, int T, unsigned long long* e) {
  for (int k = threadIdx.x; k < T; k += blockDim.x) e[k] = 0ull;
  __syncthreads();
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    if (t0[r] >= K) continue;
    const RowKey k = row_key(t0[r], sec[r], K, pair, nlo, nhi);
    atomicOr(&e[k.key], 1ull << (k.res - 1));
  }
  __syncthreads();
}

// the largest resume site in a table entry
__device__ inline int last_res(uint64_t m) { return 64 - __clzll((unsigned long long)m); }

// the sites (bit s) whose carried states rows resuming at the sites of m read
// from a node with changed site c1: s in [res - W + 1, res - 1], s >= c1
__device__ inline uint64_t need_of(uint64_t b, int W, int c1) {
  uint64_t need = 0;
  for (int w = 0; w < W - 1; ++w) need |= b >> w;
  return need & ~((1ull << c1) - 1ull);
}

// block-wide exclusive scan of (count, entries, slots) held one set per thread
__device__ void block_scan(int& cnt, int64_t& ent, int64_t& slt, int* sc, int64_t* se, int64_t* ss, int& tot_cnt,
                           int64_t& tot_ent, int64_t& tot_slt) {
  const int tid = threadIdx.x;
  sc[tid] = cnt;
  se[tid] = ent;
  ss[tid] = slt;
  __syncthreads();
  for (int d = 1; d < kNodeThreads; d <<= 1) {
    const int vc = tid >= d ? sc[tid - d] : 0;
    const int64_t ve = tid >= d ? se[tid - d] : 0;
    const int64_t vs = tid >= d ? ss[tid - d] : 0;
    __syncthreads();
    sc[tid] += vc;
    se[tid] += ve;
    ss[tid] += vs;
    __syncthreads();
  }
  tot_cnt = sc[kNodeThreads - 1];
  tot_ent = se[kNodeThreads - 1];
  tot_slt = ss[kNodeThreads - 1];
  cnt = tid > 0 ? sc[tid - 1] : 0;
  ent = tid > 0 ? se[tid - 1] : 0;
  slt = tid > 0 ? ss[tid - 1] : 0;
  __syncthreads();
}

__global__ __launch_bounds__(kNodeThreads) void k_node_count(const uint8_t* __restrict__ t0,
                                                             const uint32_t* __restrict__ sec,
                                                             const uint64_t* __restrict__ samples,
                                                             const int64_t* rowptr, int64_t n0, int64_t row_base,
                                                             int K, int W, bool pair, int32_t* ncnt, int64_t* nent,
                                                             int64_t* nslt) {
  extern __shared__ unsigned long long lds_table[];
  unsigned long long* e = lds_table;
  __shared__ int sc[kNodeThreads];
  __shared__ int64_t se[kNodeThreads], ss[kNodeThreads];
  const int T = table_keys(K, pair);
  const int64_t n = n0 + blockIdx.x;
  build_table(t0, sec, rowptr[n] - row_base, rowptr[n + 1] - row_base, K, pair, samples[2 * n], samples[2 * n + 1],
              T, e);
  int cnt = 0;
  int64_t ent = 0, slt = 0;
  for (int k = threadIdx.x; k < T; k += blockDim.x)
    if (e[k]) {
      const int c1 = key_c1(k, K, pair);
      ++cnt;
      ent += last_res(e[k]) - c1 + 1;
      slt += __popcll(need_of(e[k], W, c1));
    }
  int tc;
  int64_t te, ts;
  block_scan(cnt, ent, slt, sc, se, ss, tc, te, ts);
  if (threadIdx.x == 0) {
    ncnt[blockIdx.x] = tc;
    nent[blockIdx.x] = te;
    nslt[blockIdx.x] = ts;
  }
}

// one workgroup of 1024 threads over the ns samples of the pass: exclusive
// offsets; a sample is accepted while the nodes, entries and slots of it and
// all before it fit their capacities (samples not accepted get no nodes)
__global__ __launch_bounds__(1024) void k_node_scan(int64_t ns, NodeCaps cap, const int32_t* ncnt,
                                                    const int64_t* nent, const int64_t* nslt, int64_t* nbase,
                                                    int64_t* ebase, int64_t* totals) {
  __shared__ int64_t pc[1024], pe[1024], ps[1024];
  const int tid = threadIdx.x;
  const int64_t per = (ns + 1023) / 1024;
  const int64_t a = tid * per, b = a + per < ns ? a + per : ns;
  int64_t sc = 0, se = 0, sl = 0;
  for (int64_t i = a; i < b; ++i) {
    sc += ncnt[i];
    se += nent[i];
    sl += nslt[i];
  }
  pc[tid] = sc;
  pe[tid] = se;
  ps[tid] = sl;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int64_t vc = tid >= d ? pc[tid - d] : 0, ve = tid >= d ? pe[tid - d] : 0, vs = tid >= d ? ps[tid - d] : 0;
    __syncthreads();
    pc[tid] += vc;
    pe[tid] += ve;
    ps[tid] += vs;
    __syncthreads();
  }
  // the running sums only grow, so once a sample does not fit no later one
  // does: the accepted samples are a prefix, numbered contiguously
  int64_t rc = tid > 0 ? pc[tid - 1] : 0, re = tid > 0 ? pe[tid - 1] : 0, rs = tid > 0 ? ps[tid - 1] : 0;
  for (int64_t i = a; i < b; ++i) {
    const bool ok = rc + ncnt[i] <= cap.nodes && re + nent[i] <= cap.entries && rs + nslt[i] <= cap.own_slots;
    nbase[i] = ok ? rc : -1;
    ebase[i] = re;
    rc += ncnt[i];
    re += nent[i];
    rs += nslt[i];
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
                                                              int K, int W, bool pair, const int64_t* nbase,
                                                              const int64_t* ebase, NodeList nl, int32_t* row_node,
                                                              uint8_t* row_site) {
  extern __shared__ unsigned long long lds_table[];
  unsigned long long* e = lds_table;
  __shared__ int sc[kNodeThreads];
  __shared__ int64_t se[kNodeThreads], ss[kNodeThreads];
  const int T = table_keys(K, pair);
  const int64_t n = n0 + blockIdx.x;
  const int64_t r0 = rowptr[n] - row_base, r1 = rowptr[n + 1] - row_base;
  const uint64_t nlo = samples[2 * n], nhi = samples[2 * n + 1];
  build_table(t0, sec, r0, r1, K, pair, nlo, nhi, T, e);
  const int64_t nb = nbase[blockIdx.x];
  const bool keep = nb >= 0;
  // each thread numbers the keys of one contiguous chunk, in key order
  const int chunk = (T + kNodeThreads - 1) / kNodeThreads;
  const int k0 = threadIdx.x * chunk, k1 = k0 + chunk < T ? k0 + chunk : T;
  int cnt = 0;
  int64_t ent = 0, slt = 0;
  for (int k = k0; k < k1; ++k)
    if (e[k]) {
      ++cnt;
      ent += last_res(e[k]) - key_c1(k, K, pair) + 1;
    }
  int tc;
  int64_t te, ts;
  block_scan(cnt, ent, slt, sc, se, ss, tc, te, ts);
  int j = cnt;
  int64_t off = ebase[blockIdx.x] + ent;
  // after numbering, e[k] holds the key's node (all ones: none)
  for (int k = k0; k < k1; ++k) {
    const uint64_t ek = e[k];
    if (!ek) {
      e[k] = ~0ull;
      continue;
    }
    const int c1 = key_c1(k, K, pair), last = last_res(ek);
    if (keep) {
      const int64_t node = nb + j;
      uint64_t lo = nlo, hi = nhi;
      int s1, c2 = K, s2 = 0;
      if (pair) {
        const int r = k - pair_base(c1, K), L = pair_len(c1, K);
        const int a1 = r / L, jj = r % L;
        s1 = a1 + (a1 >= site_state(nlo, nhi, c1) ? 1 : 0);
        if (jj > 0) {
          c2 = c1 + 1 + (jj - 1) / 3;
          const int a2 = (jj - 1) % 3;
          s2 = a2 + (a2 >= site_state(nlo, nhi, c2) ? 1 : 0);
        }
      } else {
        s1 = k % 4;
      }
      int P = 2 * c1;
      if (P < 64) lo = (lo & ~(3ull << P)) | (uint64_t(s1) << P);
      else hi = (hi & ~(3ull << (P - 64))) | (uint64_t(s1) << (P - 64));
      if (c2 < K) {
        P = 2 * c2;
        if (P < 64) lo = (lo & ~(3ull << P)) | (uint64_t(s2) << P);
        else hi = (hi & ~(3ull << (P - 64))) | (uint64_t(s2) << (P - 64));
      }
      nl.m[2 * node] = lo;
      nl.m[2 * node + 1] = hi;
      nl.owner[node] = int32_t(n);
      nl.c1[node] = uint8_t(c1);
      nl.e1[node] = uint8_t(last);
      nl.off[node] = off;
      nl.need[node] = need_of(ek, W, c1);
      e[k] = node;
    } else {
      e[k] = ~0ull;
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
    const RowKey k = row_key(t0[r], sec[r], K, pair, nlo, nhi);
    const uint64_t ek = e[k.key];
    const int node = ek == ~0ull ? -1 : int(ek);
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

// slot numbering: coff[u] = sum over v < u of popcount(need[v]).  Block b
// covers the kSlotBlock nodes from b kSlotBlock on, in kSlotPer rounds of
// kSlotThreads consecutive nodes (coalesced loads and stores).
constexpr int kSlotThreads = 1024, kSlotPer = 16, kSlotBlock = kSlotThreads * kSlotPer;

__global__ __launch_bounds__(kSlotThreads) void k_slot_sums(const uint64_t* __restrict__ need, int64_t nn,
                                                            int64_t* bsum) {
  __shared__ int64_t red[kSlotThreads];
  const int64_t base = int64_t(blockIdx.x) * kSlotBlock + threadIdx.x;
  int64_t s = 0;
  for (int q = 0; q < kSlotPer; ++q) {
    const int64_t u = base + int64_t(q) * kSlotThreads;
    if (u < nn) s += __popcll(need[u]);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int d = kSlotThreads / 2; d > 0; d >>= 1) {
    if (int(threadIdx.x) < d) red[threadIdx.x] += red[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

// one workgroup: exclusive scan of the nb block sums in place; the total
// goes to *total
__global__ __launch_bounds__(kSlotThreads) void k_slot_scan(int64_t nb, int64_t* bsum, int64_t* total) {
  __shared__ int64_t pc[kSlotThreads];
  const int tid = threadIdx.x;
  const int64_t per = (nb + kSlotThreads - 1) / kSlotThreads;
  const int64_t a = tid * per, b = a + per < nb ? a + per : nb;
  int64_t s = 0;
  for (int64_t i = a; i < b; ++i) s += bsum[i];
  pc[tid] = s;
  __syncthreads();
  for (int d = 1; d < kSlotThreads; d <<= 1) {
    const int64_t v = tid >= d ? pc[tid - d] : 0;
    __syncthreads();
    pc[tid] += v;
    __syncthreads();
  }
  int64_t r = tid > 0 ? pc[tid - 1] : 0;
  for (int64_t i = a; i < b; ++i) {
    const int64_t v = bsum[i];
    bsum[i] = r;
    r += v;
  }
  if (tid == kSlotThreads - 1) *total = pc[kSlotThreads - 1];
}

// the record of every node (compact slots); where the slots would exceed
// the capacity (excluded by the capacities the scan applies; a safeguard)
// every node gets need = 0 and coff = 0, nothing is stored and *overflow is
// set, which the caller reports
__global__ __launch_bounds__(kSlotThreads) void k_slot_assign(NodeList nl, int64_t nn,
                                                              const int64_t* __restrict__ bsum,
                                                              const int64_t* total, int64_t cap,
                                                              NodeRec* __restrict__ rec, int* overflow) {
  constexpr int kWaves = kSlotThreads / 64;
  __shared__ int wsum[kWaves];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const bool over = *total > cap;
  if (over && blockIdx.x == 0 && tid == 0) *overflow = 1;
  int64_t run = bsum[blockIdx.x];
  for (int q = 0; q < kSlotPer; ++q) {
    const int64_t u = int64_t(blockIdx.x) * kSlotBlock + int64_t(q) * kSlotThreads + tid;
    const uint64_t need = u < nn ? nl.need[u] : 0ull;
    const int c = __popcll(need);
    // inclusive scan over the wavefront, then over the wavefronts' totals
    int x = c;
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o);
      x += lane >= o ? y : 0;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int pre = 0, tot = 0;
    for (int w = 0; w < kWaves; ++w) {
      pre += w < wv ? wsum[w] : 0;
      tot += wsum[w];
    }
    if (u < nn) {
      NodeRec r;
      r.off = nl.off[u];
      r.coff = over ? 0 : run + pre + x - c;
      r.need = over ? 0ull : need;
      r.c1 = nl.c1[u];
      r.e1 = nl.e1[u];
      rec[u] = r;
    }
    run += tot;
    __syncthreads();
  }
}

// the tensor-term kernels' records: a slot per entry
__global__ __launch_bounds__(256) void k_rec_full(NodeList nl, int64_t nn, NodeRec* __restrict__ rec) {
  const int64_t u = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (u >= nn) return;
  NodeRec x;
  x.off = nl.off[u];
  x.coff = x.off;
  x.c1 = nl.c1[u];
  x.e1 = nl.e1[u];
  x.need = ~((1ull << x.c1) - 1ull);
  rec[u] = x;
}

int lds_per_block_limit() {
  static int lim[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 64 * 1024;
  if (!lim[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
      v = 64 * 1024;
    lim[dev] = v;
  }
  return lim[dev];
}

size_t table_bytes(int K, bool pair) { return size_t(table_keys(K, pair)) * 8; }

// static LDS of the count and assign kernels
constexpr size_t kNodeStaticLds = kNodeThreads * (4 + 8 + 8);

}  // namespace

bool node_pairs(int K) {
  return K >= 1 && K <= 64 && table_bytes(K, true) + kNodeStaticLds <= size_t(lds_per_block_limit());
}

int64_t slot_reserve(int K) { return int64_t(64) * K * K; }

hipError_t launch_node_count(const uint8_t* t0, const uint32_t* sec, const uint64_t* samples, const int64_t* rowptr,
                             int64_t n0, int64_t n1, int64_t row_base, int K, int W, bool pair, int32_t* ncnt,
                             int64_t* nent, int64_t* nslt, hipStream_t st) {
  if (n1 <= n0) return hipSuccess;
  if (K < 1 || K > 64 || W < 1 || W > 64 || (pair && !node_pairs(K))) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_node_count, dim3(unsigned(n1 - n0)), dim3(kNodeThreads), table_bytes(K, pair), st, t0, sec,
                     samples, rowptr, n0, row_base, K, W, pair, ncnt, nent, nslt);
  return hipGetLastError();
}

hipError_t launch_node_scan(int64_t ns, const NodeCaps& cap, const int32_t* ncnt, const int64_t* nent,
                            const int64_t* nslt, int64_t* nbase, int64_t* ebase, int64_t* totals, hipStream_t st) {
  if (ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_node_scan, dim3(1), dim3(1024), 0, st, ns, cap, ncnt, nent, nslt, nbase, ebase, totals);
  return hipGetLastError();
}

hipError_t launch_node_assign(const uint8_t* t0, const uint32_t* sec, const uint64_t* samples,
                              const int64_t* rowptr, int64_t n0, int64_t n1, int64_t row_base, int K, int W,
                              bool pair, const int64_t* nbase, const int64_t* ebase, const NodeList& nl,
                              int32_t* row_node, uint8_t* row_site, hipStream_t st) {
  if (n1 <= n0) return hipSuccess;
  if (K < 1 || K > 64 || W < 1 || W > 64 || (pair && !node_pairs(K))) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_node_assign, dim3(unsigned(n1 - n0)), dim3(kNodeThreads), table_bytes(K, pair), st, t0, sec,
                     samples, rowptr, n0, row_base, K, W, pair, nbase, ebase, nl, row_node, row_site);
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

int64_t slot_blocks(int64_t nn) { return (nn + kSlotBlock - 1) / kSlotBlock; }

hipError_t launch_node_records(const NodeList& nl, int64_t nn, bool compact, int64_t cap, int64_t* bsum,
                               int64_t* total, NodeRec* rec, int* overflow, hipStream_t st) {
  if (nn <= 0) return hipSuccess;
  if (!compact) {
    hipLaunchKernelGGL(k_rec_full, dim3(unsigned((nn + 255) / 256)), dim3(256), 0, st, nl, nn, rec);
    return hipGetLastError();
  }
  const int64_t nb = slot_blocks(nn);
  if (nb > (int64_t(1) << 31) - 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_slot_sums, dim3(unsigned(nb)), dim3(kSlotThreads), 0, st, nl.need, nn, bsum);
  hipLaunchKernelGGL(k_slot_scan, dim3(1), dim3(kSlotThreads), 0, st, nb, bsum, total);
  hipLaunchKernelGGL(k_slot_assign, dim3(unsigned(nb)), dim3(kSlotThreads), 0, st, nl, nn, bsum, total, cap, rec,
                     overflow);
  return hipGetLastError();
}

}  // namespace nqs
