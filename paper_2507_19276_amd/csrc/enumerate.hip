// Hamiltonian side of the semi-stochastic local energy on gfx950:
// Slater-Condon matrix elements of every connected determinant (Sec. 2.4 and
// Sec. 3 of arXiv:2507.19276), screening into the deterministic set
// |H_nm| >= eps (Eq. (20)), integer proposal weights over the remainder,
// Philox draws from P(m) = q_m / Q (Eq. (21)) and the amplitude row list.
//
// Work layout: one wavefront owns a chunk of 64 consecutive ranks of one
// sample, each lane one rank; the occupied/virtual orbital lists of the
// sample are built once per wavefront in LDS with ballot + popcount.
// Fermionic signs come from masked popcounts of the 128-bit occupation.
//
// This file is compiled without floating-point contraction: the matrix
// elements are meant to equal a plain sequential evaluation bit for bit.
#include "internal.h"
#include <algorithm>
#include "philox.h"

#pragma clang fp contract(off)

namespace nqs {
namespace {

__device__ inline int lane_id() { return threadIdx.x & 63; }

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline uint32_t mdiv(uint32_t x, uint64_t m) {
  return uint32_t((uint64_t(x) * m) >> 32);
}

// number of occupied spin orbitals with index < P in the 128-bit (lo, hi)
__device__ inline int occ_below(uint64_t lo, uint64_t hi, int P) {
  return P < 64 ? __popcll(lo & ((1ull << P) - 1ull))
                : __popcll(lo) + __popcll(hi & ((1ull << (P - 64)) - 1ull));
}

// by selects: a branch on the word would let the compiler treat (lo, hi) as a
// two-element array indexed by P / 64 and move it to scratch
__device__ inline void flip(uint64_t& lo, uint64_t& hi, int P) {
  const uint64_t bit = 1ull << (P & 63);
  lo ^= P < 64 ? bit : 0ull;
  hi ^= P < 64 ? 0ull : bit;
}

// site (spatial orbital) of the lowest set spin-orbital bit of a nonzero XOR
// of two ONVs, with P = 2 p + sigma
__device__ inline int first_changed_site(uint64_t xlo, uint64_t xhi) {
  if (xlo) return (__ffsll((unsigned long long)xlo) - 1) >> 1;
  return (64 + __ffsll((unsigned long long)xhi) - 1) >> 1;
}

// first changed site c1 of row m against its sample n, and the row's second
// changed site c2 (K if none) with its local state at c1 packed as
// c2 | state << 8
// first changed site of the row (t0) and, packed in sec, the second changed
// site c2 (bits 0-7), the row's state at c1 (bits 8-9), the third changed site
// c3 (bits 16-23) and the row's state at c2 (bits 24-25); absent sites are K
__device__ inline void row_sites(uint64_t mlo, uint64_t mhi, uint64_t nlo, uint64_t nhi, int K, uint8_t* t0,
                                 uint32_t* sec) {
  uint64_t xl = mlo ^ nlo, xh = mhi ^ nhi;
  const int c1 = first_changed_site(xl, xh);
  *t0 = uint8_t(c1);
  if (!sec) return;
  auto take = [&](int c) {   // the row's state at site c; clears the site from the difference (by selects)
    const int P = 2 * c;
    const bool low = P < 64;
    const int sh = P & 63;
    const int st = int(((low ? mlo : mhi) >> sh) & 3ull);
    const uint64_t keep = ~(3ull << sh);
    xl &= low ? keep : ~0ull;
    xh &= low ? ~0ull : keep;
    return st;
  };
  const int s1 = take(c1);
  const int c2 = (xl | xh) ? first_changed_site(xl, xh) : K;
  const int s2 = c2 < K ? take(c2) : 0;
  const int c3 = (xl | xh) ? first_changed_site(xl, xh) : K;
  *sec = uint32_t(c2) | (uint32_t(s1) << 8) | (uint32_t(c3) << 16) | (uint32_t(s2) << 24);
}

__device__ inline bool bit_at(uint64_t lo, uint64_t hi, int P) {
  return P < 64 ? ((lo >> P) & 1ull) : ((hi >> (P - 64)) & 1ull);
}

struct Lists {
  uint8_t oa[64], va[64], ob[64], vb[64];
  uint8_t occ[128];   // occupied spin orbitals, ascending
};

// Build the orbital lists of one ONV with the whole wavefront (lane p looks at
// spatial orbital p).  Returns true when the ONV has exactly (na, nb)
// electrons and no bit beyond 2K.
__device__ bool decode_lists(const HamDev& H, uint64_t lo, uint64_t hi, Lists& L) {
  const int p = lane_id();
  const bool in = p < H.K;
  L.oa[p] = 0; L.va[p] = 0; L.ob[p] = 0; L.vb[p] = 0;
  L.occ[p] = 0; L.occ[p + 64] = 0;
  wave_sync();
  const bool xa = in && bit_at(lo, hi, 2 * p);
  const bool xb = in && bit_at(lo, hi, 2 * p + 1);
  const uint64_t ma = __ballot(xa), mb = __ballot(xb);
  const uint64_t lt = __lanemask_lt();
  const int ra = __popcll(ma & lt), rb = __popcll(mb & lt);
  if (in) {
    if (xa) L.oa[ra] = p; else L.va[p - ra] = p;
    if (xb) L.ob[rb] = p; else L.vb[p - rb] = p;
    const int base = ra + rb;
    if (xa) L.occ[base] = 2 * p;
    if (xb) L.occ[base + (xa ? 1 : 0)] = 2 * p + 1;
  }
  wave_sync();
  const int K2 = 2 * H.K;
  uint64_t stray_lo = K2 >= 64 ? 0ull : (lo >> K2);
  uint64_t stray_hi = K2 >= 128 ? 0ull : (K2 >= 64 ? (hi >> (K2 - 64)) : hi);
  return __popcll(ma) == H.na && __popcll(mb) == H.nb && stray_lo == 0 && stray_hi == 0;
}

// (32-bit arithmetic: K <= 64, so K^4 < 2^32)
__device__ inline uint32_t eidx(int K, int p, int q, int r, int s) {
  return ((uint32_t(p) * K + q) * K + r) * K + s;
}

// S(i) = number of pairs (i', j') with i' < i in lexicographic order of i<j<n
__device__ inline int pair_start(int i, int n) { return i * n - (i * (i + 1)) / 2; }

// pair p -> (i, j): i = max{i : S(i) <= p}, the floor of the smaller root of
// S(x) = p with b = 2n - 1.  For n <= 64 the FP32 estimate is within one of
// it (b^2 - 8p < 2^24 is exact in FP32 and the square root carries an ulp or
// two), so one correction step each way gives i exactly (checked for every
// n <= 64 and p, with the square root off by up to two ulps either way).
__device__ inline void unpair(uint32_t p, int n, int& i, int& j) {
  const float b = 2.0f * n - 1.0f;
  int ii = int((b - sqrtf(fmaxf(b * b - 8.0f * float(p), 0.0f))) * 0.5f);
  ii = max(0, min(ii, n - 2));
  ii += (ii + 1 <= n - 2 && pair_start(ii + 1, n) <= int(p)) ? 1 : 0;
  ii -= (ii > 0 && pair_start(ii, n) > int(p)) ? 1 : 0;
  i = ii;
  j = int(p) - pair_start(ii, n) + ii + 1;
}

struct Elem {
  double H;
  uint64_t mlo, mhi;
};

// apply a_I a_J a+_B a+_A in the order a_I, a_J, a+_B, a+_A (I<J, A<B) and
// return the parity of the sign
__device__ inline int apply_double(uint64_t& lo, uint64_t& hi, int I, int J, int A, int B) {
  int g = occ_below(lo, hi, I);
  flip(lo, hi, I);
  g += occ_below(lo, hi, J);
  flip(lo, hi, J);
  g += occ_below(lo, hi, B);
  flip(lo, hi, B);
  g += occ_below(lo, hi, A);
  flip(lo, hi, A);
  return g & 1;
}

// Matrix element H_mn and m for canonical rank r of the sample (lo, hi).
// FULL = false: |H_mn| only (the screening and the proposal weights need no
// sign and no m), in e.H.  KIND: 0 any rank; 2 (3) the caller knows r is a
// same-spin (opposite-spin) double and the other kinds' code is left out.
template <bool FULL = true, int KIND = 0>
__device__ Elem element(const HamDev& H, const Lists& L, uint64_t lo, uint64_t hi, uint32_t r) {
  const int K = H.K;
  Elem e;
  if (KIND == 0 && r < H.off_daa) {
    // single excitation I -> A of spin sigma: |m> = g a+_A a_I |n>,
    // H_mn = g (h_AI + sum_{J occ} <AJ||IJ>), J ascending
    const int sg = r >= H.off_sb ? 1 : 0;
    const uint32_t t = sg ? r - H.off_sb : r;
    const int v = sg ? H.vb : H.va;
    const uint32_t ii = mdiv(t, sg ? H.mg_vb : H.mg_va);
    const uint32_t aa = t - ii * uint32_t(v);
    const int i = sg ? L.ob[ii] : L.oa[ii];
    const int a = sg ? L.vb[aa] : L.va[aa];
    double acc = H.h[a * K + i];
    const int ne = H.na + H.nb;
    const double2* s3 = reinterpret_cast<const double2*>(H.s3) + (a * K + i) * K;   // ((ai|jj), (aj|ji)) over j
    for (int k = 0; k < ne; ++k) {
      const int J = L.occ[k];
      const double2 g = s3[J >> 1];
      const double g2 = ((J & 1) == sg) ? g.y : 0.0;
      acc += (g.x - g2);
    }
    if constexpr (!FULL) {
      e.H = fabs(acc);
      return e;
    }
    const int I = 2 * i + sg, A = 2 * a + sg;
    uint64_t ml = lo, mh = hi;
    int g = occ_below(ml, mh, I);
    flip(ml, mh, I);
    g += occ_below(ml, mh, A);
    flip(ml, mh, A);
    e.H = (g & 1) ? -acc : acc;
    e.mlo = ml; e.mhi = mh;
    return e;
  }
  if (KIND == 2 || (KIND == 0 && r < H.off_dab)) {
    // same-spin double (i<j) -> (a<b): H_mn = g ((ai|bj) - (aj|bi))
    const int sg = r >= H.off_dbb ? 1 : 0;
    const uint32_t t = sg ? r - H.off_dbb : r - H.off_daa;
    const uint32_t npv = sg ? H.npb_v : H.npa_v;
    const uint32_t pij = mdiv(t, sg ? H.mg_npb_v : H.mg_npa_v);
    const uint32_t pab = t - pij * npv;
    int ii, jj, aa, bb;
    unpair(pij, sg ? H.nb : H.na, ii, jj);
    unpair(pab, sg ? H.vb : H.va, aa, bb);
    const int i = sg ? L.ob[ii] : L.oa[ii];
    const int j = sg ? L.ob[jj] : L.oa[jj];
    const int a = sg ? L.vb[aa] : L.va[aa];
    const int b = sg ? L.vb[bb] : L.va[bb];
    const double val = H.eri[eidx(K, i, a, j, b)] - H.eri[eidx(K, j, a, i, b)];
    if constexpr (!FULL) {
      e.H = fabs(val);
      return e;
    }
    uint64_t ml = lo, mh = hi;
    const int g = apply_double(ml, mh, 2 * i + sg, 2 * j + sg, 2 * a + sg, 2 * b + sg);
    e.H = g ? -val : val;
    e.mlo = ml; e.mhi = mh;
    return e;
  }
  // opposite-spin double (i alpha, j beta) -> (a alpha, b beta): with the spin
  // orbitals sorted, <AB||IJ> = +(ai|bj) when the alpha hole and the alpha
  // particle come first together, -(ai|bj) otherwise
  const uint32_t t = r - H.off_dab;
  const uint32_t sa = mdiv(t, H.mg_nsb);
  const uint32_t sb = t - sa * H.nsb;
  const uint32_t ii = mdiv(sa, H.mg_va);
  const uint32_t aa = sa - ii * uint32_t(H.va);
  const uint32_t jj = mdiv(sb, H.mg_vb);
  const uint32_t bb = sb - jj * uint32_t(H.vb);
  const int i = L.oa[ii], a = L.va[aa], j = L.ob[jj], b = L.vb[bb];
  double val = H.eri[eidx(K, i, a, j, b)];
  if constexpr (!FULL) {
    e.H = fabs(val);
    return e;
  }
  if ((i <= j) != (a <= b)) val = -val;
  const int Ia = 2 * i, Jb = 2 * j + 1, Aa = 2 * a, Bb = 2 * b + 1;
  uint64_t ml = lo, mh = hi;
  const int g = apply_double(ml, mh, min(Ia, Jb), max(Ia, Jb), min(Aa, Bb), max(Aa, Bb));
  e.H = g ? -val : val;
  e.mlo = ml; e.mhi = mh;
  return e;
}

__device__ inline uint64_t wave_sum_u64(uint64_t x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

__device__ inline uint64_t wave_incl_scan_u64(uint64_t x) {
  const int l = lane_id();
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = __shfl_up(x, o);
    if (l >= o) x += y;
  }
  return x;
}

__device__ inline uint64_t proposal_weight(double absH, int qshift) {
  return uint64_t(ceil(ldexp(absH, qshift)));
}

// floor(U * Q / 2^128) with U = (u3 u2 u1 u0) in 32-bit words, Q < 2^60
__device__ inline uint64_t scaled_draw(const uint32_t U[4], uint64_t Q) {
  const uint64_t ulo = uint64_t(U[0]) | (uint64_t(U[1]) << 32);
  const uint64_t uhi = uint64_t(U[2]) | (uint64_t(U[3]) << 32);
  const uint64_t p_lo_hi = __umul64hi(ulo, Q);          // floor(ulo * Q / 2^64)
  const uint64_t a_lo = uhi * Q, a_hi = __umul64hi(uhi, Q);
  const uint64_t s = a_lo + p_lo_hi;
  return a_hi + (s < a_lo ? 1ull : 0ull);
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

__global__ void k_validate(const uint64_t* samples, int64_t N, int K, int na, int nb, int* bad) {
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const uint64_t lo = samples[2 * n], hi = samples[2 * n + 1];
  int a = 0, b = 0;
  for (int p = 0; p < K; ++p) {
    a += bit_at(lo, hi, 2 * p) ? 1 : 0;
    b += bit_at(lo, hi, 2 * p + 1) ? 1 : 0;
  }
  const int K2 = 2 * K;
  const uint64_t sl = K2 >= 64 ? 0ull : (lo >> K2);
  const uint64_t sh = K2 >= 128 ? 0ull : (K2 >= 64 ? (hi >> (K2 - 64)) : hi);
  if (a != na || b != nb || sl || sh) *bad = 1;
}

// Pass 1 (screening): per chunk of 64 ranks of a sample the ballot of the
// deterministic ranks and the sum of the remainder's proposal weights, then per
// segment the running sums.  |H_nm| alone decides both, so no sign and no ONV
// is formed.  Doubles go by orbital pair: a workgroup stages the K x K integral
// slab of one pair in LDS and serves every sample of a batch in which that pair
// appears (hole and particle of the alpha spin for opposite-spin doubles, the
// two holes for equal-spin ones), so a slab is read once per batch instead of
// once per sample.  Singles go by sample.  A scan per segment then turns the
// chunk sums into running sums.

// (n_alpha, n_beta) electrons and no bit beyond 2K: the samples whose elements exist
__device__ inline bool onv_ok(const HamDev& H, uint64_t lo, uint64_t hi) {
  const uint64_t EVEN = 0x5555555555555555ull;
  const int K2 = 2 * H.K;
  const uint64_t slo = K2 >= 64 ? 0ull : (lo >> K2);
  const uint64_t shi = K2 >= 128 ? 0ull : (K2 >= 64 ? (hi >> (K2 - 64)) : hi);
  return __popcll(lo & EVEN) + __popcll(hi & EVEN) == H.na &&
         __popcll(lo & ~EVEN) + __popcll(hi & ~EVEN) == H.nb && slo == 0 && shi == 0;
}

// the n lowest bits of a word (all for n >= 64, none for n <= 0)
__device__ inline uint64_t lowest(int n) { return n <= 0 ? 0ull : (n >= 64 ? ~0ull : ((1ull << n) - 1ull)); }

// occupied spin orbitals 2q + sigma with q < p
__device__ inline int occ_below_spin(uint64_t lo, uint64_t hi, int p, int sigma) {
  const uint64_t sp = sigma ? 0xAAAAAAAAAAAAAAAAull : 0x5555555555555555ull;
  return __popcll(lo & sp & lowest(2 * p)) + __popcll(hi & sp & lowest(2 * p - 64));
}

// value of lane l (wave-uniform) of a 64-bit register
__device__ inline uint64_t lane_u64(uint64_t x, int l) {
  const uint32_t a = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(x)), l));
  const uint32_t b = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(x >> 32)), l));
  return (uint64_t(b) << 32) | a;
}

__device__ inline void screen(double hv, double eps, int qshift, bool valid, bool& det, uint64_t& q) {
  const double ah = fabs(hv);
  det = valid && hv != 0.0 && ah >= eps;
  q = (valid && hv != 0.0 && !det) ? proposal_weight(ah, qshift) : 0ull;
}

// the ranks [rb, re) of one sample (chunk row at masks/qsum + row); hval(e)
// gives H at rank rb + e for the lanes inside the block.  Lane l takes rank
// 64 c + l of chunk c; a chunk wholly inside the block is stored, a border
// chunk is added atomically.
template <class F>
__device__ inline void scr_block(uint64_t* masks, uint64_t* qsum, int64_t row, uint32_t rb, uint32_t re, double eps,
                                 int qshift, F&& hval) {
  const uint32_t lane = uint32_t(lane_id());
  for (uint32_t c = rb >> 6; c * 64u < re; ++c) {
    const uint32_t r = c * 64u + lane;
    const bool valid = r >= rb && r < re;
    const double hv = valid ? hval(r - rb) : 0.0;
    bool det;
    uint64_t q;
    screen(hv, eps, qshift, valid, det, q);
    const uint64_t bal = __ballot(det);
    const uint64_t qs = wave_sum_u64(q);
    if (lane == 0) {
      uint64_t* m = masks + row + c;
      uint64_t* s = qsum + row + c;
      if (c * 64u >= rb && c * 64u + 64u <= re) {
        *m = bal;
        *s = qs;
      } else {
        if (bal) atomicOr((unsigned long long*)m, (unsigned long long)bal);
        if (qs) atomicAdd((unsigned long long*)s, (unsigned long long)qs);
      }
    }
  }
}

__global__ void k_scr_zero(uint64_t* a, uint64_t* b, int64_t n) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x) {
    a[t] = 0ull;
    b[t] = 0ull;
  }
}

// singles: one wavefront per sample over the ranks below off_daa
__global__ __launch_bounds__(256) void k_scr_singles(HamDev H, EnumGeom G, const uint64_t* samples, int64_t N,
                                                     double eps, int qshift, uint64_t* masks, uint64_t* qsum) {
  __shared__ Lists lists[4];
  const int wv = threadIdx.x >> 6;
  const int64_t n = int64_t(blockIdx.x) * 4 + wv;
  if (n >= N) return;
  const uint64_t lo = samples[2 * n], hi = samples[2 * n + 1];
  Lists& L = lists[wv];
  if (!decode_lists(H, lo, hi, L)) return;
  scr_block(masks, qsum, n * G.nchunks, 0u, H.off_daa, eps, qshift,
            [&](uint32_t r) { return element<false>(H, L, lo, hi, r).H; });
}

// Pair kernels.  What screening makes of a double excitation's |H_nm| depends
// on the four orbitals only, so a workgroup codes its slab once when it stages
// it: -1 for a deterministic element, else the proposal weight (0 for a
// vanishing one), an integer below 2^41 that FP64 holds exactly, as it holds
// every sum of 64 of them.  The ranks of one (sample, pair) form a contiguous
// block; a wavefront turns the blocks of its 64 samples into a list of chunk
// tasks and gives each lane one chunk, which the lane walks rank by rank with
// incremental indices, collecting its own deterministic bits and weight sum: no
// cross-lane reduction per chunk.  A chunk wholly inside its block is stored;
// a border chunk, shared with the neighbouring pair's block, is added with
// 64-bit atomics (exact in any order).

constexpr int kScrWaves = 4;                // wavefronts per workgroup of the pair kernels
constexpr int kScrBatch = 64 * kScrWaves;   // samples per workgroup (64 per wavefront)

__device__ inline double scr_code(double hv, double eps, int qshift) {
  if (hv == 0.0) return 0.0;
  const double ah = fabs(hv);
  return ah >= eps ? -1.0 : ceil(ldexp(ah, qshift));
}

// the largest s with first[s] <= t (first ascending over 64 slots, first[0] = 0)
__device__ inline int scr_slot(const int* first, int t) {
  int s = 0;
  for (int step = 32; step > 0; step >>= 1) s += first[s + step] <= t ? step : 0;
  return s;
}

// one lane's chunk after its walk over the ranks k0 <= k < k1 of it: bits
// holds the deterministic flags shifted in from the top (rank k1 - 1 at bit
// 63), qacc the sum of the codes, i.e. the weight sum minus the number of
// deterministic ranks (integers below 2^47, exact in FP64).  A chunk wholly
// inside its block is stored, a border chunk added.
__device__ inline void scr_finish(uint64_t* masks, uint64_t* qsum, int64_t at, int k0, int k1, uint64_t bits,
                                  double qacc) {
  bits = k1 == 64 ? bits : (bits >> (64 - k1));
  const uint64_t q = uint64_t(qacc + double(__popcll(bits)));
  if (k0 == 0 && k1 == 64) {
    masks[at] = bits;
    qsum[at] = q;
  } else {
    if (bits) atomicOr((unsigned long long*)(masks + at), (unsigned long long)bits);
    if (q) atomicAdd((unsigned long long*)(qsum + at), (unsigned long long)q);
  }
}

// per-wavefront LDS of the pair kernels: orbital lists of its 64 samples
// (stride bytes each, a multiple of 4; nlist lists per sample), then per
// sample its first task, its block starts and its number of spin-0 tasks
__host__ __device__ inline size_t scr_wave_bytes(int stride, int nlist) {
  return size_t(64) * stride * nlist + 4 * 64 * sizeof(int);
}

// opposite-spin doubles (i alpha -> a alpha, j beta -> b beta), workgroup per
// (i, a), i != a, and batch of samples: slab (ia|jb) over (j, b), contiguous in
// HBM.  A sample's list holds its beta orbitals, occupied then virtual.
__global__ __launch_bounds__(64 * kScrWaves) void k_scr_os(HamDev H, EnumGeom G, const uint64_t* samples, int64_t N,
                                                           double eps, int qshift, int stride, uint64_t* masks,
                                                           uint64_t* qsum) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int K = H.K;
  const int i = int(blockIdx.x) / (K - 1), t = int(blockIdx.x) % (K - 1);
  const int a = t + (t >= i ? 1 : 0);
  double* code = reinterpret_cast<double*>(smem);
  const int wv = threadIdx.x >> 6, lane = lane_id();
  uint8_t* orb = smem + size_t(K) * K * 8 + wv * scr_wave_bytes(stride, 1);
  int* first = reinterpret_cast<int*>(orb + 64 * stride);
  uint32_t* rbs = reinterpret_cast<uint32_t*>(first + 64);
  const double* src = H.eri + (size_t(i) * K + a) * K * K;
  for (int u = threadIdx.x; u < K * K; u += blockDim.x) code[u] = scr_code(src[u], eps, qshift);
  const int64_t nbase = int64_t(blockIdx.y) * kScrBatch + wv * 64;
  const int64_t n = nbase + lane;
  uint64_t lo = 0, hi = 0;
  bool ok = false;
  if (n < N) {
    lo = samples[2 * n];
    hi = samples[2 * n + 1];
    ok = bit_at(lo, hi, 2 * i) && !bit_at(lo, hi, 2 * a) && onv_ok(H, lo, hi);
  }
  const uint32_t nsb = H.nsb;
  uint32_t rb = 0, nck = 0;
  if (ok) {
    const uint32_t ii = uint32_t(occ_below_spin(lo, hi, i, 0));
    const uint32_t aa = uint32_t(a - occ_below_spin(lo, hi, a, 0));
    rb = H.off_dab + (ii * uint32_t(H.va) + aa) * nsb;
    nck = ((rb + nsb - 1u) >> 6) - (rb >> 6) + 1u;
  }
  for (uint64_t todo = __ballot(ok); todo; todo &= todo - 1) {
    const int l = __ffsll((unsigned long long)todo) - 1;
    const uint64_t slo = lane_u64(lo, l), shi = lane_u64(hi, l);
    const bool in = lane < K;
    const bool x = in && bit_at(slo, shi, 2 * lane + 1);
    const int r = __popcll(__ballot(x) & __lanemask_lt());
    if (in) orb[l * stride + (x ? r : H.nb + (lane - r))] = uint8_t(lane);
  }
  const uint32_t incl = uint32_t(wave_incl_scan_u64(nck));
  first[lane] = int(incl - nck);
  rbs[lane] = rb;
  const int T = int(lane_u64(incl, 63));
  __syncthreads();
  const int nb = H.nb, vb = H.vb;
  for (int t0 = 0; t0 < T; t0 += 64) {
    const int tk = t0 + lane;
    if (tk >= T) break;
    const int s = scr_slot(first, tk);
    const uint32_t b0 = rbs[s], b1 = b0 + nsb;
    const uint32_t c = (b0 >> 6) + uint32_t(tk - first[s]);
    const uint32_t cb = c * 64u;
    const int k0 = int(max(b0, cb) - cb), k1 = int(min(b1, cb + 64u) - cb);
    const uint32_t e = cb + uint32_t(k0) - b0;
    const uint8_t* ol = orb + s * stride;
    int jj = int(mdiv(e, H.mg_vb));
    int vx = nb + int(e) - jj * vb;                 // list index of the beta particle
    uint32_t rowoff = __umul24(ol[jj], uint32_t(K));
    uint64_t bits = 0;
    double qacc = 0.0;
    for (int k = k0; k < k1; ++k) {
      const double cv = code[rowoff + ol[vx]];
      bits = (bits >> 1) | (cv < 0.0 ? 0x8000000000000000ull : 0ull);
      qacc += cv;
      const bool wrap = ++vx == K;
      jj += wrap ? 1 : 0;
      vx = wrap ? nb : vx;
      rowoff = __umul24(ol[jj], uint32_t(K));
    }
    scr_finish(masks, qsum, (nbase + s) * G.nchunks + c, k0, k1, bits, qacc);
  }
}

// equal-spin doubles (i < j -> a < b, both spins), workgroup per hole pair
// (i, j) and batch of samples: slab (ia|jb) - (ja|ib) over (a, b), where
// (ja|ib) = (ib|ja) is the transposed entry as the stored integrals are exactly
// 8-fold symmetric.  A sample's lists hold its virtual orbitals of each spin.
__global__ __launch_bounds__(64 * kScrWaves) void k_scr_ss(HamDev H, EnumGeom G, const uint64_t* samples, int64_t N,
                                                           double eps, int qshift, int stride, uint64_t* masks,
                                                           uint64_t* qsum) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int K = H.K;
  int i, j;
  unpair(blockIdx.x, K, i, j);
  double* code = reinterpret_cast<double*>(smem);
  const int wv = threadIdx.x >> 6, lane = lane_id();
  uint8_t* vl = smem + size_t(K) * K * 8 + wv * scr_wave_bytes(stride, 2);
  int* first = reinterpret_cast<int*>(vl + 2 * 64 * stride);
  uint32_t* rbs = reinterpret_cast<uint32_t*>(first + 64);   // [2][64]
  int* nck0s = reinterpret_cast<int*>(rbs + 128);
  // stage (ia|jb) over (a, b), then code the upper triangle a < b (the only
  // entries read) in place: entry (a, b) and its transpose belong to one thread
  for (int u = threadIdx.x; u < K * K; u += blockDim.x) {
    const int a = u / K, b = u % K;
    code[u] = H.eri[((size_t(i) * K + a) * K + j) * K + b];
  }
  __syncthreads();
  for (int u = threadIdx.x; u < K * K; u += blockDim.x) {
    const int a = u / K, b = u % K;
    if (a < b) code[u] = scr_code(code[u] - code[b * K + a], eps, qshift);
  }
  const int64_t nbase = int64_t(blockIdx.y) * kScrBatch + wv * 64;
  const int64_t n = nbase + lane;
  uint64_t lo = 0, hi = 0;
  bool okv = false;
  if (n < N) {
    lo = samples[2 * n];
    hi = samples[2 * n + 1];
    okv = onv_ok(H, lo, hi);
  }
  // per spin: the block [rb, rb + npv) when both holes are occupied
  uint32_t rbv[2] = {0u, 0u}, nck[2] = {0u, 0u};
  bool ok[2];
  for (int sg = 0; sg < 2; ++sg) {
    ok[sg] = okv && bit_at(lo, hi, 2 * i + sg) && bit_at(lo, hi, 2 * j + sg);
    const uint32_t npv = sg ? H.npb_v : H.npa_v;
    if (ok[sg] && npv > 0u) {
      const int ne = sg ? H.nb : H.na;
      const int ii = occ_below_spin(lo, hi, i, sg), jj = occ_below_spin(lo, hi, j, sg);
      rbv[sg] = (sg ? H.off_dbb : H.off_daa) + uint32_t(pair_start(ii, ne) + (jj - ii - 1)) * npv;
      nck[sg] = ((rbv[sg] + npv - 1u) >> 6) - (rbv[sg] >> 6) + 1u;
    }
    for (uint64_t todo = __ballot(nck[sg] > 0u); todo; todo &= todo - 1) {
      const int l = __ffsll((unsigned long long)todo) - 1;
      const uint64_t slo = lane_u64(lo, l), shi = lane_u64(hi, l);
      const bool in = lane < K;
      const bool x = in && bit_at(slo, shi, 2 * lane + sg);
      const int r = __popcll(__ballot(x) & __lanemask_lt());
      if (in && !x) vl[(sg * 64 + l) * stride + (lane - r)] = uint8_t(lane);
    }
  }
  const uint32_t tot = nck[0] + nck[1];
  const uint32_t incl = uint32_t(wave_incl_scan_u64(tot));
  first[lane] = int(incl - tot);
  rbs[lane] = rbv[0];
  rbs[64 + lane] = rbv[1];
  nck0s[lane] = int(nck[0]);
  const int T = int(lane_u64(incl, 63));
  __syncthreads();
  for (int t0 = 0; t0 < T; t0 += 64) {
    const int tk = t0 + lane;
    if (tk >= T) break;
    const int s = scr_slot(first, tk);
    int u = tk - first[s];
    const int n0 = nck0s[s];
    const int sg = u < n0 ? 0 : 1;
    u -= sg ? n0 : 0;
    const uint32_t npv = sg ? H.npb_v : H.npa_v;
    const uint32_t b0 = rbs[sg * 64 + s];
    const uint32_t b1 = b0 + npv;
    const uint32_t c = (b0 >> 6) + uint32_t(u);
    const uint32_t cb = c * 64u;
    const int k0 = int(max(b0, cb) - cb), k1 = int(min(b1, cb + 64u) - cb);
    const uint32_t e = cb + uint32_t(k0) - b0;
    const int nv = sg ? H.vb : H.va;
    const uint8_t* ls = vl + (sg * 64 + s) * stride;
    int aa, bb;
    unpair(e, nv, aa, bb);
    uint32_t rowoff = __umul24(ls[aa], uint32_t(K));
    uint64_t bits = 0;
    double qacc = 0.0;
    for (int k = k0; k < k1; ++k) {
      const double cv = code[rowoff + ls[bb]];
      bits = (bits >> 1) | (cv < 0.0 ? 0x8000000000000000ull : 0ull);
      qacc += cv;
      const bool wrap = ++bb == nv;
      aa += wrap ? 1 : 0;
      bb = wrap ? aa + 1 : bb;
      rowoff = __umul24(ls[aa], uint32_t(K));
    }
    scr_finish(masks, qsum, (nbase + s) * G.nchunks + c, k0, k1, bits, qacc);
  }
}

// running sums: one wavefront per (sample, segment); qpref holds the chunk
// sums on entry and their inclusive prefix within the segment on exit
__global__ __launch_bounds__(256) void k_scr_scan(EnumGeom G, int64_t N, const uint64_t* masks, uint64_t* qpref,
                                                  uint64_t* segq, uint32_t* segd) {
  const int wv = threadIdx.x >> 6, lane = lane_id();
  const int64_t unit = int64_t(blockIdx.x) * 4 + wv;
  if (unit >= N * G.S) return;
  const int64_t n = unit / G.S;
  const int s = int(unit % G.S);
  const int c0 = s * G.cps, c1 = min(c0 + G.cps, G.nchunks);
  const int64_t row = n * G.nchunks;
  uint64_t carry = 0;
  uint32_t d = 0;
  for (int c = c0; c < c1; c += 64) {
    const int cc = c + lane;
    const uint64_t qv = cc < c1 ? qpref[row + cc] : 0ull;
    const uint64_t mv = cc < c1 ? masks[row + cc] : 0ull;
    const uint64_t incl = wave_incl_scan_u64(qv);
    if (cc < c1) qpref[row + cc] = carry + incl;
    carry += __shfl(incl, 63);
    d += uint32_t(wave_sum_u64(uint64_t(__popcll(mv))));
  }
  if (lane == 0) {
    segq[n * G.S + s] = carry;
    segd[n * G.S + s] = d;
  }
}

// Per sample: segment totals -> exclusive segment offsets (in place), Q_n, |D_n|.
__global__ void k_sample_scan(EnumGeom G, int64_t N, uint64_t* segq, uint32_t* segd, uint64_t* Qn,
                              int64_t* Dn) {
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= N) return;
  uint64_t q = 0;
  int64_t d = 0;
  for (int s = 0; s < G.S; ++s) {
    const uint64_t tq = segq[n * G.S + s];
    const uint32_t td = segd[n * G.S + s];
    segq[n * G.S + s] = q;
    segd[n * G.S + s] = uint32_t(d);
    q += tq;
    d += td;
  }
  Qn[n] = q;
  Dn[n] = d;
}

constexpr int kMaxDraws = 1024;

// Draws of one sample per workgroup: Philox -> r in [0, Q) -> segment ->
// chunk (binary search over the inclusive prefixes) -> lane (wavefront scan of
// the chunk's weights); then sort the drawn ranks and merge duplicates.
__global__ __launch_bounds__(256) void k_draw(HamDev H, EnumGeom G, const uint64_t* samples, int64_t N,
                                              double eps, int qshift, int n_eps, DrawKeys keys,
                                              const uint64_t* qpref, const uint64_t* segq_off,
                                              const uint64_t* Qn, int32_t* urank, double* ucoef,
                                              uint64_t* um, int64_t* Un) {
  __shared__ Lists L;
  __shared__ int32_t chunk_of[kMaxDraws];
  __shared__ uint64_t rin_of[kMaxDraws];
  __shared__ int32_t rank_of[kMaxDraws];
  __shared__ int32_t idx_of[kMaxDraws];
  __shared__ double h_of[kMaxDraws];
  __shared__ uint64_t q_of[kMaxDraws];
  __shared__ uint64_t mlo_of[kMaxDraws], mhi_of[kMaxDraws];
  const int64_t n = blockIdx.x;
  const int tid = threadIdx.x, wv = tid >> 6, lane = lane_id();
  const uint64_t Q = Qn[n];
  if (Q == 0 || n_eps == 0) {
    if (tid == 0) Un[n] = 0;
    return;
  }
  const uint64_t lo = samples[2 * n], hi = samples[2 * n + 1];
  if (wv == 0) decode_lists(H, lo, hi, L);
  __syncthreads();
  const uint64_t* qp = qpref + n * G.nchunks;
  for (int k = tid; k < n_eps; k += blockDim.x) {
    uint32_t U[4];
    philox4x32_10(keys.sample_base + uint32_t(n), uint32_t(k), keys.ctr2, keys.ctr3, keys.key0, keys.key1, U);
    const uint64_t r = scaled_draw(U, Q);
    int s = 0;
    while (s + 1 < G.S && segq_off[n * G.S + s + 1] <= r) ++s;
    const uint64_t rr = r - segq_off[n * G.S + s];
    const int c0 = s * G.cps, c1 = min(c0 + G.cps, G.nchunks);
    int lo_c = c0, hi_c = c1 - 1;          // first chunk with inclusive prefix > rr
    while (lo_c < hi_c) {
      const int mid = (lo_c + hi_c) >> 1;
      if (qp[mid] > rr) hi_c = mid; else lo_c = mid + 1;
    }
    chunk_of[k] = lo_c;
    rin_of[k] = rr - (lo_c > c0 ? qp[lo_c - 1] : 0ull);
    rank_of[k] = 0;      // overwritten below; keeps every entry defined
    h_of[k] = 0.0;
    q_of[k] = 1;
    mlo_of[k] = lo;
    mhi_of[k] = hi;
  }
  __syncthreads();
  for (int k = wv; k < n_eps; k += 4) {
    const int c = chunk_of[k];
    const uint32_t r = uint32_t(c) * 64u + uint32_t(lane);
    Elem e{0.0, 0, 0};
    if (r < H.n_conn) e = element(H, L, lo, hi, r);
    const double ah = fabs(e.H);
    const bool det = e.H != 0.0 && ah >= eps;
    const uint64_t q = (e.H != 0.0 && !det) ? proposal_weight(ah, qshift) : 0ull;
    const uint64_t incl = wave_incl_scan_u64(q);
    const uint64_t hit = __ballot(incl > rin_of[k] && q > 0);
    const int pick = __ffsll((unsigned long long)hit) - 1;   // lowest lane: first prefix exceeding r
    if (lane == pick) {
      rank_of[k] = int32_t(r);
      h_of[k] = e.H;
      q_of[k] = q;
      mlo_of[k] = e.mlo;
      mhi_of[k] = e.mhi;
    }
  }
  __syncthreads();
  // sort (rank, draw index) by rank: bitonic sort over the next power of two
  int P2 = 1;
  while (P2 < n_eps) P2 <<= 1;
  for (int k = tid; k < P2; k += blockDim.x) {
    idx_of[k] = k;
    if (k >= n_eps) rank_of[k] = 0x7fffffff;
  }
  __syncthreads();
  for (int size = 2; size <= P2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int k = tid; k < P2; k += blockDim.x) {
        const int o = k ^ stride;
        if (o > k) {
          const bool up = (k & size) == 0;
          const int32_t a = rank_of[k], b = rank_of[o];
          const int32_t ia = idx_of[k], ib = idx_of[o];
          const bool swap = up ? (a > b || (a == b && ia > ib)) : (a < b || (a == b && ia < ib));
          if (swap) {
            rank_of[k] = b; rank_of[o] = a;
            idx_of[k] = ib; idx_of[o] = ia;
          }
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    int64_t u = 0;
    const double Qd = double(Q), nd = double(n_eps);
    int k = 0;
    while (k < n_eps) {
      int k2 = k;
      while (k2 < n_eps && rank_of[k2] == rank_of[k]) ++k2;
      const int d = idx_of[k];
      const double w = h_of[d] * (Qd / (double(q_of[d]) * nd));
      urank[n * n_eps + u] = rank_of[k];
      ucoef[n * n_eps + u] = double(k2 - k) * w;
      um[2 * (n * n_eps + u)] = mlo_of[d];
      um[2 * (n * n_eps + u) + 1] = mhi_of[d];
      ++u;
      k = k2;
    }
    Un[n] = u;
  }
}

// rowptr[n] = sum_{n' < n} (1 + |D_n'| + U_n'), single workgroup of 1024 threads
__global__ __launch_bounds__(1024) void k_row_counts(int64_t N, const int64_t* Dn, const int64_t* Un,
                                                     int64_t* rowptr) {
  __shared__ int64_t part[1024];
  __shared__ int64_t carry;
  const int tid = threadIdx.x;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < N; base += 1024) {
    const int64_t n = base + tid;
    const int64_t v = n < N ? 1 + Dn[n] + Un[n] : 0;
    part[tid] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int64_t y = tid >= o ? part[tid - o] : 0;
      __syncthreads();
      part[tid] += y;
      __syncthreads();
    }
    if (n < N) rowptr[n] = carry + part[tid] - v;
    __syncthreads();
    if (tid == 1023) carry += part[1023];
    __syncthreads();
  }
  if (tid == 0) rowptr[N] = carry;
}

// Pass 2: write the rows.  Unit (n, s) writes the deterministic rows of its
// segment in rank order; segment 0 also writes the sample's own row and its
// unique drawn rows.
// Rows of samples [n0, n1) are written at (global row index - row_base).
__global__ __launch_bounds__(256) void k_fill(HamDev H, EnumGeom G, const uint64_t* samples, int64_t n0,
                                              int64_t n1, const uint64_t* masks, const uint32_t* segd_off,
                                              const int64_t* rowptr, int64_t row_base, const int64_t* Dn,
                                              const int64_t* Un, const int32_t* urank,
                                              const double* ucoef, const uint64_t* um, int n_eps,
                                              Rows rows) {
  __shared__ Lists lists[4];
  const int wv = threadIdx.x >> 6, lane = lane_id();
  const int64_t unit = int64_t(blockIdx.x) * 4 + wv;
  if (unit >= (n1 - n0) * G.S) return;
  const int64_t n = n0 + unit / G.S;
  const int s = int(unit % G.S);
  const uint64_t lo = samples[2 * n], hi = samples[2 * n + 1];
  Lists& L = lists[wv];
  decode_lists(H, lo, hi, L);
  const int64_t r0 = rowptr[n] - row_base;
  int64_t pos = r0 + 1 + segd_off[n * G.S + s];
  const int c0 = s * G.cps, c1 = min(c0 + G.cps, G.nchunks);
  // the deterministic ranks of 64 chunks at a time, compacted: lane l takes the
  // l-th set bit of the round (rank order), so every lane evaluates an element
  for (int cb = c0; cb < c1; cb += 64) {
    const int cl = cb + lane;
    const uint64_t mk = cl < c1 ? masks[n * G.nchunks + cl] : 0ull;
    const int cnt = __popcll(mk);
    int incl = cnt;   // inclusive scan of the set-bit counts over the lanes
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int v = __shfl_up(incl, d);
      if (lane >= d) incl += v;
    }
    const int excl = incl - cnt;
    const int total = __shfl(incl, 63);
    for (int j0 = 0; j0 < total; j0 += 64) {
      const int j = j0 + lane;
      // the chunk holding set bit j: the last lane c with excl_c <= j
      int c = 0;
#pragma unroll
      for (int step = 32; step > 0; step >>= 1)
        if (__shfl(excl, c + step) <= j) c += step;
      // the position of its (j - excl_c)-th set bit, by halving
      const uint64_t m = __shfl(mk, c);
      int kk = j - __shfl(excl, c), bit = 0;
#pragma unroll
      for (int w = 32; w > 0; w >>= 1) {
        const int cw = __popcll((m >> bit) & ((1ull << w) - 1ull));
        if (kk >= cw) {
          bit += w;
          kk -= cw;
        }
      }
      if (j < total) {
        const uint32_t r = uint32_t(cb + c) * 64u + uint32_t(bit);
        const Elem e = element(H, L, lo, hi, r);
        const int64_t at = pos + j;
        rows.m[2 * at] = e.mlo;
        rows.m[2 * at + 1] = e.mhi;
        rows.coef[at] = e.H;
        rows.owner[at] = int32_t(n);
        if (rows.rank) rows.rank[at] = int64_t(r);
        if (rows.t0) row_sites(e.mlo, e.mhi, lo, hi, H.K, rows.t0 + at, rows.sec ? rows.sec + at : nullptr);
      }
    }
    pos += total;
  }
  if (s == 0) {
    if (lane == 0) {
      rows.m[2 * r0] = lo;
      rows.m[2 * r0 + 1] = hi;
      rows.coef[r0] = 0.0;
      rows.owner[r0] = int32_t(n);
      if (rows.rank) rows.rank[r0] = -1;
      if (rows.t0) rows.t0[r0] = uint8_t(H.K);
      if (rows.sec) rows.sec[r0] = uint32_t(H.K) | (uint32_t(H.K) << 16);
    }
    const int64_t u = Un[n];
    const int64_t d0 = r0 + 1 + Dn[n];
    for (int64_t t = lane; t < u; t += 64) {
      const int64_t at = d0 + t;
      rows.m[2 * at] = um[2 * (n * n_eps + t)];
      rows.m[2 * at + 1] = um[2 * (n * n_eps + t) + 1];
      rows.coef[at] = ucoef[n * n_eps + t];
      rows.owner[at] = int32_t(n);
      if (rows.rank) rows.rank[at] = urank[n * n_eps + t];
      if (rows.t0)
        row_sites(um[2 * (n * n_eps + t)], um[2 * (n * n_eps + t) + 1], lo, hi, H.K, rows.t0 + at,
                  rows.sec ? rows.sec + at : nullptr);
    }
  }
}

// H_nn = e_core + sum_P h_PP + 1/2 sum_{P,Q occ} <PQ||PQ>, one thread per
// sample, over the occupied spin orbitals in ascending order (the order of the
// plain definition); <PQ||PQ> = (pp|qq) - delta_{sigma_P sigma_Q} (pq|qp) from
// the K x K tables of those entries
__device__ inline int next_set(uint64_t& lo, uint64_t& hi) {
  // by selects (a branch per word would put (lo, hi) in scratch)
  const bool l = lo != 0;
  const uint64_t w = l ? lo : hi;
  const int P = (l ? 0 : 64) + __ffsll((unsigned long long)w) - 1;
  const uint64_t nw = w & (w - 1);
  lo = l ? nw : lo;
  hi = l ? hi : nw;
  return P;
}

__global__ void k_diag(HamDev H, const uint64_t* samples, int64_t N, double* hdiag) {
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const uint64_t lo = samples[2 * n], hi = samples[2 * n + 1];
  const int K = H.K;
  const double* J = H.jk;
  const double* X = H.jk + size_t(K) * K;
  double d1 = 0.0;
  for (uint64_t a = lo, b = hi; a | b;) {
    const int p = next_set(a, b) >> 1;
    d1 += H.h[p * K + p];
  }
  double d2 = 0.0;
  for (uint64_t a = lo, b = hi; a | b;) {
    const int P = next_set(a, b), p = P >> 1;
    for (uint64_t c = lo, d = hi; c | d;) {
      const int Q = next_set(c, d), q = Q >> 1;
      const double g1 = J[p * K + q];
      const double g2 = ((P & 1) == (Q & 1)) ? X[p * K + q] : 0.0;
      d2 += (g1 - g2);
    }
  }
  hdiag[n] = H.ecore + d1 + 0.5 * d2;
}

// every connected determinant of every sample (Hamiltonian-engine entry point)
__global__ __launch_bounds__(256) void k_connected(HamDev H, const uint64_t* samples, int64_t N,
                                                   int nchunks, uint64_t* m_out, double* h_out) {
  __shared__ Lists lists[4];
  const int wv = threadIdx.x >> 6, lane = lane_id();
  const int64_t unit = int64_t(blockIdx.x) * 4 + wv;
  if (unit >= N * nchunks) return;
  const int64_t n = unit / nchunks;
  const int c = int(unit % nchunks);
  const uint64_t lo = samples[2 * n], hi = samples[2 * n + 1];
  Lists& L = lists[wv];
  const bool ok = decode_lists(H, lo, hi, L);
  const uint32_t r = uint32_t(c) * 64u + uint32_t(lane);
  if (r >= H.n_conn) return;
  Elem e{0.0, 0, 0};
  if (ok) e = element(H, L, lo, hi, r);
  const int64_t at = n * int64_t(H.n_conn) + r;
  if (m_out) {
    m_out[2 * at] = e.mlo;
    m_out[2 * at + 1] = e.mhi;
  }
  if (h_out) h_out[at] = e.H;
}

inline unsigned grid_for(int64_t units, int per_block) {
  return unsigned((units + per_block - 1) / per_block);
}

}  // namespace

hipError_t launch_validate(const uint64_t* samples, int64_t N, int K, int na, int nb, int* bad,
                           hipStream_t st) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate, dim3(grid_for(N, 256)), dim3(256), 0, st, samples, N, K, na, nb, bad);
  return hipGetLastError();
}

hipError_t launch_enum_count(const HamDev& H, const EnumGeom& G, const uint64_t* samples, int64_t N,
                             double eps, int qshift, uint64_t* masks, uint64_t* qpref, uint64_t* segq,
                             uint32_t* segd, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  if (H.K < 1 || H.K > 64) return hipErrorInvalidValue;
  const int64_t nc = N * G.nchunks;
  hipLaunchKernelGGL(k_scr_zero, dim3(unsigned(std::min<int64_t>((nc + 255) / 256, 16384))), dim3(256), 0, st,
                     masks, qpref, nc);
  if (H.off_daa > 0)
    hipLaunchKernelGGL(k_scr_singles, dim3(grid_for(N, 4)), dim3(256), 0, st, H, G, samples, N, eps, qshift,
                       masks, qpref);
  // pair kernels: grid x = orbital pairs (K(K-1)/2 hole pairs i < j, K(K-1)
  // hole-particle pairs i != a), y = batches of kScrBatch samples (launched in
  // slices of at most 65535 batches); LDS: the coded slab and per wavefront the
  // orbital lists of its samples
  const int st_os = (H.K + 3) & ~3, st_ss = (std::max(H.va, H.vb) + 3) & ~3;
  const size_t slab = size_t(H.K) * H.K * 8;
  const size_t lds_os = slab + kScrWaves * scr_wave_bytes(st_os, 1);
  const size_t lds_ss = slab + kScrWaves * scr_wave_bytes(st_ss, 2);
  const int64_t nbatch = (N + kScrBatch - 1) / kScrBatch;
  for (int64_t b0 = 0; b0 < nbatch; b0 += 65535) {
    const int64_t nb = std::min<int64_t>(nbatch - b0, 65535);
    const uint64_t* sm = samples + 2 * b0 * kScrBatch;
    const int64_t Nb = std::min<int64_t>(N - b0 * kScrBatch, nb * kScrBatch);
    uint64_t* mk = masks + b0 * kScrBatch * G.nchunks;
    uint64_t* qs = qpref + b0 * kScrBatch * G.nchunks;
    if (H.off_dab > H.off_daa)
      hipLaunchKernelGGL(k_scr_ss, dim3(unsigned(H.K * (H.K - 1) / 2), unsigned(nb)), dim3(64 * kScrWaves), lds_ss, st,
                         H, G, sm, Nb, eps, qshift, st_ss, mk, qs);
    if (H.n_conn > H.off_dab)
      hipLaunchKernelGGL(k_scr_os, dim3(unsigned(H.K * (H.K - 1)), unsigned(nb)), dim3(64 * kScrWaves), lds_os, st,
                         H, G, sm, Nb, eps, qshift, st_os, mk, qs);
  }
  hipLaunchKernelGGL(k_scr_scan, dim3(grid_for(N * G.S, 4)), dim3(256), 0, st, G, N, masks, qpref, segq, segd);
  return hipGetLastError();
}

hipError_t launch_sample_scan(const EnumGeom& G, int64_t N, uint64_t* segq, uint32_t* segd,
                              uint64_t* Qn, int64_t* Dn, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sample_scan, dim3(grid_for(N, 256)), dim3(256), 0, st, G, N, segq, segd, Qn, Dn);
  return hipGetLastError();
}

hipError_t launch_draw(const HamDev& H, const EnumGeom& G, const uint64_t* samples, int64_t N,
                       double eps, int qshift, int n_eps, DrawKeys keys, const uint64_t* qpref,
                       const uint64_t* segq_off, const uint64_t* Qn, int32_t* urank, double* ucoef,
                       uint64_t* um, int64_t* Un, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  if (n_eps > kMaxDraws) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_draw, dim3(unsigned(N)), dim3(256), 0, st, H, G, samples, N, eps, qshift, n_eps,
                     keys, qpref, segq_off, Qn, urank, ucoef, um, Un);
  return hipGetLastError();
}

hipError_t launch_row_counts(int64_t N, const int64_t* Dn, const int64_t* Un, int64_t* rowptr,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_row_counts, dim3(1), dim3(1024), 0, st, N, Dn, Un, rowptr);
  return hipGetLastError();
}

hipError_t launch_fill(const HamDev& H, const EnumGeom& G, const uint64_t* samples, int64_t n0, int64_t n1,
                       const uint64_t* masks, const uint32_t* segd_off, const int64_t* rowptr,
                       int64_t row_base, const int64_t* Dn, const int64_t* Un, const int32_t* urank,
                       const double* ucoef, const uint64_t* um, int n_eps, Rows rows, hipStream_t st) {
  if (n1 <= n0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(grid_for((n1 - n0) * G.S, 4)), dim3(256), 0, st, H, G, samples, n0, n1,
                     masks, segd_off, rowptr, row_base, Dn, Un, urank, ucoef, um, n_eps, rows);
  return hipGetLastError();
}

hipError_t launch_diag(const HamDev& H, const uint64_t* samples, int64_t N, double* hdiag,
                       hipStream_t st) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag, dim3(grid_for(N, 64)), dim3(64), 0, st, H, samples, N, hdiag);
  return hipGetLastError();
}

hipError_t launch_connected(const HamDev& H, const uint64_t* samples, int64_t N, uint64_t* m_out,
                            double* h_out, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  const int nchunks = int((H.n_conn + 63) / 64);
  hipLaunchKernelGGL(k_connected, dim3(grid_for(N * nchunks, 4)), dim3(256), 0, st, H, samples, N,
                     nchunks, m_out, h_out);
  return hipGetLastError();
}

}  // namespace nqs
