// BDG-RNN / MPS-RNN forward in FP64 and FP32 on gfx950 (arXiv:2507.19276,
// Sec. 2.1 Eqs. (9)-(10), Sec. 2.2 Eq. (12) without the tensor term): per
// site i the candidates h_i^s = sum_{j in N(i)} M_ij^s h_j + v_i^s for the
// four local states, the conditional P^s = h^T eta h normalised over the
// states allowed by the particle-number / S_z mask (Sec. 3, Eqs. (23)-(24)),
// the phase sign of w^T h + c, and the carried state h_i^{s_i}.  With complex
// parameters (CPLX) the kernel runs on the realified 2chi-unit state (block
// matrices [[Re M, -Im M], [Im M, Re M]]) and multiplies the per-site phase
// factors z_i = w_i^T h_i + c_i, Re z from w' = [Re w; -Im w] and Im z from
// w2 = [Im w; Re w].
//
// Bond contractions run on MFMA in the transposed form
//   H_i^T [4chi x rows] = W_i^T [4chi x d_i chi] . X_i^T [d_i chi x rows]
// so that rows are the N dimension of 16x16 MFMA tiles and every lane holds 4
// consecutive hidden units of one row and candidate in the MFMA output layout.
// Carried hidden states live in a lane-private LDS ring of
// W = (max parent offset + 1) slots.
#include "device.h"
#include "philox.h"

namespace nqs {
namespace {

// Forward amplitude kernel.  One wavefront owns NTL tiles of 16 rows.
//
// Operands.  The A stream holds, for every forward edge e (the parents of each
// site in order; a parentless site has one zero edge), KS = CH/4 k-steps of NT
// values per lane.  k-step q = 4 tt + v pairs lane group g with parent unit
// 16 tt + 4 g + v, which is exactly the unit that lane (j, g) produced for
// row j in register v of output tile tt of the parent site.  The B operand of
// every MFMA is therefore the lane's own carried state, kept in a lane-private
// LDS ring: no cross-lane exchange and no barrier between sites.
//
// The accumulators start from the bias v_i^s, so after the contractions
// acc[t][s*TPC + tt] holds the candidates h_i^s for units 16 tt + 4 g + 0..3.
// The A operands are fetched PQ k-steps ahead of their MFMAs (see
// prefetch_ksteps), across edge and site boundaries, so their latency hides
// behind the contractions and the epilogue.
//
// FOLD: the operands carry sigma = sqrt(eta) (A' = sigma_i M / sigma_j,
// v' = sigma v, w' = w / sigma, all eta > 0), so the ring holds sigma h and
// P^s = sum_u x'^2 needs no eta.  STORE and SEED: see PsiStates (the
// samples' pass that stores states, and the resumed row pass).  CPLX: phs
// receives arg prod_i z_i per row; the stored and resumed prefix states carry
// the product of the phase factors so far (pz, npz).
// A operands in flight: PQ k-steps of the A stream, the largest divisor of
// the KS k-steps of an edge whose NT values per lane fit 128 registers (64 in
// the tensor-term, complex and sampling forms, whose own registers would
// spill otherwise).  The stream is read as a rolling window: k-step q takes
// its values from slot q % PQ, which then receives k-step q + PQ (of this
// edge, or of the next edge past the last k-step), so every load is issued PQ
// k-steps before its MFMAs and no register copies are needed between edges.
// At one wavefront per SIMD nothing else hides a load that is waited for.
template <typename T> constexpr int prefetch_ksteps(int CH, bool lean) {
  const int ks = CH / 4, per = (CH / 4) * int(sizeof(T) / 4), budget = lean ? 64 : 128;
  int pq = 1;
  for (int d = 1; d <= ks; ++d)
    if (ks % d == 0 && d * per <= budget) pq = d;
  return pq;
}

template <typename T, int CH, int NTL, bool FOLD, int STORE, bool SEED, bool SAMPLE, bool CPLX, bool TN, bool D1>
__global__ __launch_bounds__(256) void k_psi_mt(PsiParams<T> P, const uint64_t* __restrict__ m, int64_t R,
                                                double* __restrict__ lphi, int8_t* __restrict__ sphi, int wpb,
                                                PsiStates<T> X, SampleArgs SA, double* __restrict__ phs) {
  // every floating-point operation below is written out (explicit fma where
  // one is meant), so that all instances of this kernel round alike: a row
  // resumed from its sample's stored state ends bit-identical to a row
  // computed from site 0
#pragma clang fp contract(off)
  static_assert(!CPLX || !SAMPLE, "sampling needs no phase");
  extern __shared__ __align__(16) unsigned char smem[];
  typedef typename V4<T>::type V;
  constexpr int TPC = CH / 16, NT = 4 * TPC, KS = CH / 4, RW = 16 * NTL;
  constexpr int PQ = prefetch_ksteps<T>(CH, TN || CPLX || SAMPLE);
  static_assert(KS % PQ == 0, "the A window slots repeat every PQ k-steps");
  constexpr int ES = KS * NT * 64;              // A values per edge
  constexpr int SLOT = NTL * TPC * 64;          // V entries per ring slot
  // the wavefront index is uniform: keep it (and all that derives from it:
  // rows, start site, edge and slot counters) in scalar registers
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int j = lane & 15, g = lane >> 4;
  const int own = NTL == 4 ? g : (NTL == 2 ? (g >> 1) : 0);
  const int64_t base = (int64_t(blockIdx.x) * wpb + wv) * RW;
  if (base >= R) return;   // surplus wavefront of the last block (no block barrier below)
  // ring: W slots of carried states (site i writes slot wsl[i]; a zero edge,
  // slot index W, reads no slot); entry ((slot * NTL + t) * TPC + tt) * 64 +
  // lane belongs to this lane only
  V* ring = reinterpret_cast<V*>(smem) + size_t(wv) * P.W * SLOT + lane;
  // edge tables and c are uniform and read-only: scalar loads
  const CInt* fptr = (const CInt*)(P.pptr);
  const CInt* slots = (const CInt*)(P.slot);
  const CInt* wsl = (const CInt*)(P.wsl);
  const CT<T>* cc = (const CT<T>*)(P.c);
  const CT<T>* cc2 = (const CT<T>*)(P.c2);
  const CInt* tsite = (const CInt*)(P.tsite);
  // SEED: positions base.. map to rows X.perm[pos], sorted by their first
  // changed site, and the wavefront starts at the site of its first row
  const int i0 = SEED ? int(((const __attribute__((address_space(4))) uint8_t*)X.t0)[base]) : 0;
  uint64_t lo[NTL], hi[NTL];
  int64_t rowt[NTL];
  uint64_t olo = 0, ohi = 0;
#pragma unroll
  for (int t = 0; t < NTL; ++t) {
    const int64_t r = base + 16 * t + j;
    const int64_t rr = r < R ? r : R - 1;
    rowt[t] = SEED ? int64_t(X.perm[rr]) : rr;
    lo[t] = SAMPLE ? 0ull : m[2 * rowt[t]];
    hi[t] = SAMPLE ? 0ull : m[2 * rowt[t] + 1];
    if (t == own) { olo = lo[t]; ohi = hi[t]; }
  }
  const bool olive = base + 16 * own + j < R;
  int64_t orow = rowt[0];
#pragma unroll
  for (int t = 1; t < NTL; ++t)
    if (t == own) orow = rowt[t];
  T prod = T(1);
  T zr = T(1), zi = T(0);   // CPLX: product of the phase factors, rescaled by powers of two
  int pexp = 0, sgn = 1, ca = 0, cb = 0, e = 0;
  bool bad = false;
  if (SEED && i0 > 0) {
    // carried states of the parents of sites >= i0 and the log-product state
    // before site i0, taken from the row's sample (rows agree with their
    // sample on every site below their first changed site >= i0)
    // With a node level (X.unode), a row's node covers the sites from its
    // changed site nc1 on: the node agrees with the row below the row's
    // resume site, the sample below nc1.
    // The node's carried state after site s is in slot nco + popcount(nmk &
    // bits below s); one record per node.
    int nd[NTL], nb[NTL];
    int64_t no[NTL], nco[NTL];
    uint64_t nmk[NTL];
#pragma unroll
    for (int t = 0; t < NTL; ++t) {
      nd[t] = X.unode ? X.unode[rowt[t]] : -1;
      NodeRec q{0, 0, 0ull, P.K + 1, 0};
      if (nd[t] >= 0) q = X.nrec[nd[t]];
      nb[t] = q.c1;
      no[t] = q.off;
      nco[t] = q.coff;
      nmk[t] = q.need;
    }
    // the states live at i0 (read by a site >= i0; distinct slots)
    for (uint64_t lv = ((const __attribute__((address_space(4))) uint64_t*)P.live)[i0]; lv; lv &= lv - 1) {
      const int s = __builtin_ctzll(lv);
      V* wr = ring + size_t(wsl[s]) * SLOT;
#pragma unroll
      for (int t = 0; t < NTL; ++t) {
        const T* src = s >= nb[t] ? X.nhs + size_t(nco[t] + __popcll(nmk[t] & low_bits(s))) * CH + 4 * g
                                  : X.hs + (size_t(s) * X.ns + X.owner[rowt[t]]) * CH + 4 * g;
#pragma unroll
        for (int tt = 0; tt < TPC; ++tt) wr[(t * TPC + tt) * 64] = *reinterpret_cast<const V*>(src + 16 * tt);
      }
    }
    int ond = nd[0], onb = nb[0];
    int64_t ono = no[0];
#pragma unroll
    for (int t = 1; t < NTL; ++t)
      if (t == own) { ond = nd[t]; onb = nb[t]; ono = no[t]; }
    if (i0 >= onb) {
      const size_t so = size_t(ono + (i0 - onb));
      const LogProd<T> lp = X.nlp[so];
      prod = lp.m;
      pexp = lp.e;
      sgn = lp.s;
      if (CPLX) {
        zr = X.npz[2 * so];
        zi = X.npz[2 * so + 1];
      }
    } else {
      const size_t so = size_t(i0) * X.ns + X.owner[orow];
      prod = X.pm[so];
      pexp = X.pe[so];
      sgn = X.pg[so];
      if (CPLX) {
        zr = X.pz[2 * so];
        zi = X.pz[2 * so + 1];
      }
    }
    (void)ond;
    const uint64_t below = low_bits(2 * i0), belowh = low_bits(2 * i0 - 64);
    ca = __popcll(olo & below & 0x5555555555555555ull) + __popcll(ohi & belowh & 0x5555555555555555ull);
    cb = __popcll(olo & below & 0xAAAAAAAAAAAAAAAAull) + __popcll(ohi & belowh & 0xAAAAAAAAAAAAAAAAull);
    e = fptr[i0];
  }
  const T* __restrict__ Ab = P.A + lane;
  T an[PQ][NT];
#pragma unroll
  for (int q = 0; q < PQ; ++q)
#pragma unroll
    for (int ot = 0; ot < NT; ++ot) an[q][ot] = Ab[size_t(e) * ES + (q * NT + ot) * 64];
  // bias v of the next site, fetched one site ahead where it fits in 64
  // registers (otherwise at the start of the site): the accumulators start
  // from it
  constexpr bool BPF = NT * 4 * int(sizeof(T) / 4) <= 64;
  V vn[NT];
  auto fetch_bias = [&](int i) {
#pragma unroll
    for (int ot = 0; ot < NT; ++ot)
      vn[ot] = *reinterpret_cast<const V*>(P.v + (size_t(i) * 4 + ot / TPC) * CH + 16 * (ot % TPC) + 4 * g);
  };
  if (BPF) fetch_bias(i0 < P.K ? i0 : 0);
  // STORE 1: the log-product state before each site and the carried state
  // after it, for rows r < X.ns; STORE 2 (node units): compact, for the sites
  // nc1 .. ne1 of each unit
  int sc1 = 0, se1 = -1;
  int64_t soff = 0;
  if (STORE == 2) {
    const NodeRec q = X.nrec[orow];
    sc1 = q.c1;
    se1 = q.e1;
    soff = q.off;
  }
  // STORE 2: each unit's carried states go to the sites its record marks
  // (the sites some row reads; every site from nc1 on for the tensor-term
  // kernels)
  int tc1[NTL], te1[NTL];
  int64_t toff[NTL];
  uint64_t tneed[NTL];
#pragma unroll
  for (int t = 0; t < NTL; ++t) {
    NodeRec q{0, 0, 0ull, 0, -1};
    if (STORE == 2) q = X.nrec[rowt[t]];
    tc1[t] = q.c1;
    te1[t] = q.e1;
    toff[t] = q.coff;
    tneed[t] = q.need;
  }
  auto store_pre = [&](int i) {
    const bool writer = NTL == 4 || (NTL == 2 ? (g & 1) == 0 : g == 0);
    if (STORE == 1 && X.pm && writer && olive && orow < X.ns) {
      const size_t so = size_t(i) * X.ns + orow;
      X.pm[so] = prod;
      X.pe[so] = pexp;
      X.pg[so] = int8_t(sgn);
      if (CPLX) {
        X.pz[2 * so] = zr;
        X.pz[2 * so + 1] = zi;
      }
    }
    if (STORE == 2 && writer && olive && i >= sc1 && i <= se1) {
      const size_t so = size_t(soff + (i - sc1));
      X.nlp[so] = LogProd<T>{prod, pexp, sgn};
      if (CPLX) {
        X.npz[2 * so] = zr;
        X.npz[2 * so + 1] = zi;
      }
    }
  };
  // a node wavefront stops after the largest resume site of its nodes' rows
  int iend = P.K;
  if constexpr (STORE == 2) {
    int em = 0;
#pragma unroll
    for (int t = 0; t < NTL; ++t) em = te1[t] > em ? te1[t] : em;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const int x = __shfl_xor(em, o);
      em = x > em ? x : em;
    }
    iend = __builtin_amdgcn_readfirstlane(em < P.K ? em : P.K);
  }
  for (int i = i0; i < iend; ++i) {
    store_pre(i);
    const int wslot = wsl[i];
    V acc[NTL][NT], wv4[TPC], ev4[TPC], w2v4[TPC];
    // w and eta of this site are needed only after the contractions
#pragma unroll
    for (int tt = 0; tt < TPC; ++tt) {
      wv4[tt] = *reinterpret_cast<const V*>(P.w + size_t(i) * CH + 16 * tt + 4 * g);
      if (!FOLD) ev4[tt] = *reinterpret_cast<const V*>(P.eta + size_t(i) * CH + 16 * tt + 4 * g);
      if (CPLX) w2v4[tt] = *reinterpret_cast<const V*>(P.w2 + size_t(i) * CH + 16 * tt + 4 * g);
    }
    const int e0s = fptr[i], e1 = fptr[i + 1];
    // TN: the site's tensor term (chi' = tQ, 0 for none) and its operand streams
    int tQ = 0, toP = 0, toC = 0, toK = 0;
    if constexpr (TN) {
      tQ = tsite[4 * i];
      toP = tsite[4 * i + 1];
      toC = tsite[4 * i + 2];
      toK = tsite[4 * i + 3];
    }
    V pr0[NTL], pr1[NTL], pr2[NTL];   // TN: projections p_j = K_j^T h_j of the parents
#pragma unroll
    for (int t = 0; t < NTL; ++t) pr2[t] = V{0, 0, 0, 0};
    // one edge: a chi-wide slice of the contraction over the parents (TN: and
    // the projection of the parent's state into pt)
    // (first: the edge's first MFMAs start from the bias registers instead of
    // copies of them in the accumulators)
    auto edge = [&](V (&pt)[NTL], auto first) {
      // the edge index is wave-uniform: in a scalar register its slot comes
      // from a scalar load, so reading it does not wait for the vector loads
      // in flight (the A operands prefetched for this edge and the next)
      const int eu = __builtin_amdgcn_readfirstlane(e);
      const T* Ae = Ab + size_t(eu) * ES;
      V b[NTL][TPC];
      const int sl = slots[eu];
      const bool zero = sl >= P.W;   // a parentless site's zero edge: zero operand
      const V* rp = ring + size_t(zero ? 0 : sl) * SLOT;
#pragma unroll
      for (int t = 0; t < NTL; ++t)
#pragma unroll
        for (int tt = 0; tt < TPC; ++tt) b[t][tt] = zero ? V{0, 0, 0, 0} : rp[(t * TPC + tt) * 64];
      // rolling A window: slot q % PQ, once its MFMAs are issued, receives
      // k-step q + PQ of the stream (past this edge's last k-step: the next
      // edge's; the stream carries one zero edge past the last one)
#pragma unroll
      for (int q = 0; q < KS; ++q)
#pragma unroll
        for (int ot = 0; ot < NT; ++ot) {
          const T a = an[q % PQ][ot];
#pragma unroll
          for (int t = 0; t < NTL; ++t)
            acc[t][ot] = mfma(a, b[t][q / 4][q % 4], decltype(first)::value && q == 0 ? vn[ot] : acc[t][ot]);
          an[q % PQ][ot] = Ae[((q + PQ) * NT + ot) * 64];
        }
      if constexpr (TN) {
        if (tQ > 0) {
          // projection of this parent's state: one 16-row output tile whose
          // lane group g holds p[2g + v] in registers v = 0, 1
          const T* Ap = P.TA + toP + size_t(e - e0s) * KS * 64 + lane;
#pragma unroll
          for (int t = 0; t < NTL; ++t) pt[t] = V{0, 0, 0, 0};
#pragma unroll
          for (int q = 0; q < KS; ++q) {
            const T a = Ap[q * 64];
#pragma unroll
            for (int t = 0; t < NTL; ++t) pt[t] = mfma(a, b[t][q / 4][q % 4], pt[t]);
          }
        }
      }
    };
    if (!BPF) fetch_bias(i);
    // the contractions run at raised wave priority: an MFMA then issues as soon
    // as the matrix core frees up, and the other wavefronts' epilogues fill
    // the VALU slots in between
    __builtin_amdgcn_s_setprio(PRIO);
    if constexpr (D1) {
      edge(pr0, std::true_type{});
      ++e;
      if (BPF) fetch_bias(i + 1 < P.K ? i + 1 : i);
    } else {
      if (TN && tQ > 0) {
        // a tensor site has 2 or 3 parents: each edge's projection into its own registers
#pragma unroll
        for (int ot = 0; ot < NT; ++ot)
#pragma unroll
          for (int t = 0; t < NTL; ++t) acc[t][ot] = vn[ot];
        if (BPF) fetch_bias(i + 1 < P.K ? i + 1 : i);
        edge(pr0, std::false_type{});
        ++e;
        edge(pr1, std::false_type{});
        if (++e < e1) {
          edge(pr2, std::false_type{});
          ++e;
        }
      } else {
        // the first edge's MFMAs start from the bias registers (no copies of
        // them in the accumulators), the later edges accumulate
        edge(pr0, std::true_type{});
        ++e;
        if (BPF) fetch_bias(i + 1 < P.K ? i + 1 : i);
        for (; e < e1; ++e) edge(pr0, std::false_type{});
      }
    }
    if constexpr (TN) {
      if (tQ > 0) {
        // core contraction q^s[i'] = sum_a U^s[i'][a] prod_j p_j[a_j] as two
        // 16-row MFMA tiles over (s, i') (8 rows per state), the k-steps over
        // (a_1 .. a_(d-1), v) with a_d = 2g + v from the lane's own projection
        // registers and the other factors broadcast from the row's four lanes;
        // then t^s = K0 q^s into the candidates, k-steps over the lane's own q
        // registers
        const int d = e1 - e0s;
        const T* Ac = P.TA + toC + lane;
        const T* Ak = P.TA + toK + lane;
#pragma unroll
        for (int t = 0; t < NTL; ++t) {
          const V plast = d == 3 ? pr2[t] : pr1[t];
          V q0 = V{0, 0, 0, 0}, q1 = V{0, 0, 0, 0};
          int kk = 0;
#pragma unroll
          for (int a1 = 0; a1 < 8; ++a1) {
            if (a1 >= tQ) break;
            // p_1[a1] from the lane of the row that holds it (a = 2 g + v)
            const T b0 = __shfl(pr0[t][a1 & 1], j + 16 * (a1 >> 1));
#pragma unroll
            for (int a2 = 0; a2 < 8; ++a2) {
              if (a2 >= (d == 3 ? tQ : 1)) break;
              const T f = d == 3 ? b0 * __shfl(pr1[t][a2 & 1], j + 16 * (a2 >> 1)) : b0;
#pragma unroll
              for (int v = 0; v < 2; ++v) {
                const T bv = f * plast[v];
                q0 = mfma(Ac[(size_t(kk) * 2 + 0) * 64], bv, q0);
                q1 = mfma(Ac[(size_t(kk) * 2 + 1) * 64], bv, q1);
                ++kk;
              }
            }
          }
#pragma unroll
          for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int tt = 0; tt < TPC; ++tt)
#pragma unroll
              for (int v = 0; v < 4; ++v)
                acc[t][s * TPC + tt] =
                    mfma(Ak[((s * TPC + tt) * 4 + v) * 64], s < 2 ? q0[v] : q1[v], acc[t][s * TPC + tt]);
        }
      }
    }
    __builtin_amdgcn_s_setprio(0);
    if constexpr (SAMPLE) {
      // sampling: the row's local state is drawn from its masked conditionals
      // before the carried state is selected
      T pp[4][NTL], dp[NTL];
#pragma unroll
      for (int t = 0; t < NTL; ++t) {
        dp[t] = T(0);
#pragma unroll
        for (int s = 0; s < 4; ++s) pp[s][t] = T(0);
      }
#pragma unroll
      for (int tt = 0; tt < TPC; ++tt)
#pragma unroll
        for (int t = 0; t < NTL; ++t)
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const V x = acc[t][s * TPC + tt];
            const V ex = FOLD ? x : ev4[tt] * x;
            T q = pp[s][t];
            q = tfma(ex.x, x.x, q);
            q = tfma(ex.y, x.y, q);
            q = tfma(ex.z, x.z, q);
            q = tfma(ex.w, x.w, q);
            pp[s][t] = q;
          }
      T ps[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) ps[s] = ReduceOwn<T, NTL>::run(pp[s]);
      const int rest = P.K - 1 - i;
      T pr[4], Z = T(0);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        pr[s] = allowed(ca, cb, s, rest, P.na, P.nb) ? ps[s] : T(0);
        Z += pr[s];
      }
      // the particle's uniform for this site (53-bit fraction of Philox words 0, 1)
      const uint64_t pid = uint64_t(SA.p0 + base + 16 * own + j);
      uint32_t U[4];
      philox4x32_10(uint32_t(pid), uint32_t(pid >> 32), uint32_t(i), kSampleTag, SA.k0, SA.k1, U);
      const double u = double(((uint64_t(U[1]) << 32) | U[0]) >> 11) * 0x1p-53;
      const T target = T(u) * Z;
      T run = T(0);
      int pick = -1, last = -1;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if (pr[s] > T(0)) {
          last = s;
          run += pr[s];
          if (pick < 0 && run > target) pick = s;
        }
      }
      if (pick < 0) pick = last;
      if (pick < 0) {                     // no state has weight: the row is dead
        bad = true;
        pick = 0;
      }
      // the draw of row j of tile t sits in the lane group that owns tile t
      int ch[NTL];
#pragma unroll
      for (int t = 0; t < NTL; ++t)
        ch[t] = NTL == 4 ? __shfl(pick, j + 16 * t) : (NTL == 2 ? __shfl(pick, j + 32 * t) : pick);
      V* wr = ring + size_t(wslot) * SLOT;
#pragma unroll
      for (int tt = 0; tt < TPC; ++tt) {
        const V ww = wv4[tt];
#pragma unroll
        for (int t = 0; t < NTL; ++t) {
          // named copies: a select between two elements of acc would otherwise
          // become an indexed read and move acc to scratch
          const V x0 = acc[t][0 * TPC + tt], x1 = acc[t][1 * TPC + tt];
          const V x2 = acc[t][2 * TPC + tt], x3 = acc[t][3 * TPC + tt];
          const V sel01 = (ch[t] & 1) ? x1 : x0;
          const V sel23 = (ch[t] & 1) ? x3 : x2;
          const V sel = (ch[t] & 2) ? sel23 : sel01;
          T d = dp[t];
          d = tfma(ww.x, sel.x, d);
          d = tfma(ww.y, sel.y, d);
          d = tfma(ww.z, sel.z, d);
          d = tfma(ww.w, sel.w, d);
          dp[t] = d;
          wr[(t * TPC + tt) * 64] = sel;
        }
      }
      const T dot = ReduceOwn<T, NTL>::run(dp) + T(cc[i]);
      // the drawn state's weight by selects (an indexed read would put pr in scratch)
      const T w01 = (pick & 1) ? pr[1] : pr[0];
      const T w23 = (pick & 1) ? pr[3] : pr[2];
      int ex;
      prod = tfrexp(prod * (((pick & 2) ? w23 : w01) / Z), &ex);
      pexp += ex;
      if (dot < T(0)) sgn = -sgn;
      ca += pick & 1;
      cb += pick >> 1;
      const int P2 = 2 * i;
      if (P2 < 64) olo |= uint64_t(pick) << P2; else ohi |= uint64_t(pick) << (P2 - 64);
      continue;
    }
    // epilogue in the MFMA output layout: lane (j, g) holds units 16tt+4g..+3
    int si[NTL];
#pragma unroll
    for (int t = 0; t < NTL; ++t) si[t] = site_state(lo[t], hi[t], i);
    // FP64: the drawn candidate as a one-hot blend (4 FP64 operations per
    // double instead of 6 32-bit selects); the selected value plus signed
    // zeros is that value
    T oh[NTL][4];
#pragma unroll
    for (int t = 0; t < NTL; ++t)
#pragma unroll
      for (int s = 0; s < 4; ++s) oh[t][s] = si[t] == s ? T(1) : T(0);
    T pp[4][NTL], dp[NTL], dq[NTL];
#pragma unroll
    for (int t = 0; t < NTL; ++t) {
      dp[t] = T(0);
      dq[t] = T(0);
#pragma unroll
      for (int s = 0; s < 4; ++s) pp[s][t] = T(0);
    }
    V* wr = ring + size_t(wslot) * SLOT;
#pragma unroll
    for (int tt = 0; tt < TPC; ++tt) {
      const V ww = wv4[tt];
#pragma unroll
      for (int t = 0; t < NTL; ++t) {
        V x[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          x[s] = acc[t][s * TPC + tt];
          const V ex = FOLD ? x[s] : ev4[tt] * x[s];
          T q = pp[s][t];
          q = tfma(ex.x, x[s].x, q);
          q = tfma(ex.y, x[s].y, q);
          q = tfma(ex.z, x[s].z, q);
          q = tfma(ex.w, x[s].w, q);
          pp[s][t] = q;
        }
        V sel;
        if constexpr (sizeof(T) == 8 && !SAMPLE) {
          sel = x[0] * oh[t][0];
#pragma unroll
          for (int s = 1; s < 4; ++s) {
            sel.x = tfma(x[s].x, oh[t][s], sel.x);
            sel.y = tfma(x[s].y, oh[t][s], sel.y);
            sel.z = tfma(x[s].z, oh[t][s], sel.z);
            sel.w = tfma(x[s].w, oh[t][s], sel.w);
          }
        } else {
          const V sel01 = (si[t] & 1) ? x[1] : x[0];
          const V sel23 = (si[t] & 1) ? x[3] : x[2];
          sel = (si[t] & 2) ? sel23 : sel01;
        }
        T d = dp[t];
        d = tfma(ww.x, sel.x, d);
        d = tfma(ww.y, sel.y, d);
        d = tfma(ww.z, sel.z, d);
        d = tfma(ww.w, sel.w, d);
        dp[t] = d;
        if (CPLX) {
          const V w2 = w2v4[tt];
          T d2 = dq[t];
          d2 = tfma(w2.x, sel.x, d2);
          d2 = tfma(w2.y, sel.y, d2);
          d2 = tfma(w2.z, sel.z, d2);
          d2 = tfma(w2.w, sel.w, d2);
          dq[t] = d2;
        }
        wr[(t * TPC + tt) * 64] = sel;
        if (STORE == 1) {
          // positions past R (up to the stride X.ns) get the last row's state:
          // the adjoint reads padded rows
          const int64_t r = base + 16 * t + j;
          if (r < X.ns) *reinterpret_cast<V*>(X.hs + (size_t(i) * X.ns + r) * CH + 16 * tt + 4 * g) = sel;
        }
        if (STORE == 2 && base + 16 * t + j < R && i < te1[t] && ((tneed[t] >> i) & 1ull))
          *reinterpret_cast<V*>(X.nhs + size_t(toff[t] + __popcll(tneed[t] & low_bits(i))) * CH + 16 * tt + 4 * g) =
              sel;
      }
    }
    T ps[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) ps[s] = ReduceOwn<T, NTL>::run(pp[s]);
    const T dot = ReduceOwn<T, NTL>::run(dp) + T(cc[i]);
    if (CPLX) {
      // z <- z (Re z_i + i Im z_i), then an exact power-of-two rescale; a zero
      // factor has no argument and is left out (arg 0 = 0)
      const T di = ReduceOwn<T, NTL>::run(dq) + T(cc2[i]);
      if (dot != T(0) || di != T(0)) {
        const T nr = zr * dot - zi * di;
        const T ni = zr * di + zi * dot;
        const T an = fabs(nr) > fabs(ni) ? fabs(nr) : fabs(ni);
        int ez;
        (void)tfrexp(an, &ez);
        zr = ldexp(nr, -ez);
        zi = ldexp(ni, -ez);
      }
    }
    // per-row work, once per row: lane group g owns tile own(g)
    const int osi = site_state(olo, ohi, i);
    const int rest = P.K - 1 - i;
    T Z = T(0);
#pragma unroll
    for (int s = 0; s < 4; ++s)
      if (allowed(ca, cb, s, rest, P.na, P.nb)) Z += ps[s];
    if (!allowed(ca, cb, osi, rest, P.na, P.nb)) bad = true;
    const T p01 = (osi & 1) ? ps[1] : ps[0];
    const T p23 = (osi & 1) ? ps[3] : ps[2];
    const T psi_ = (osi & 2) ? p23 : p01;
    int ex;
    prod = tfrexp(prod * (psi_ / Z), &ex);
    pexp += ex;
    if (!CPLX && dot < T(0)) sgn = -sgn;
    ca += osi & 1;
    cb += osi >> 1;
  }
  store_pre(iend);
  const bool writer = NTL == 4 || (NTL == 2 ? (g & 1) == 0 : g == 0);
  if (writer && olive) {
    lphi[orow] = bad ? -INFINITY : 0.5 * (log(double(prod)) + double(pexp) * 0.69314718055994530942);
    sphi[orow] = int8_t(bad ? 0 : sgn);
    if (CPLX) phs[orow] = bad ? 0.0 : atan2(double(zi), double(zr));
    if (SAMPLE) {
      SA.out[2 * orow] = olo;
      SA.out[2 * orow + 1] = ohi;
    }
  }
}

#ifndef NQS_NTL_F32_16
#define NQS_NTL_F32_16 4
#endif
template <typename T> constexpr int ntiles(int CH) {
  return sizeof(T) == 4 ? (CH <= 16 ? NQS_NTL_F32_16 : (CH <= 32 ? 4 : 1)) : (CH <= 32 ? 2 : 1);
}

template <typename T, int CH, bool FOLD, int STORE, bool SEED, bool SAMPLE = false, bool CPLX = false,
          bool TN = false, bool D1 = false>
hipError_t run_psi_mt(const PsiParams<T>& P, const uint64_t* m, int64_t R, double* lphi, int8_t* sphi,
                      hipStream_t st, const PsiStates<T>& X, const SampleArgs& SA = SampleArgs(),
                      double* phs = nullptr) {
  if (R <= 0) return hipSuccess;
  // the sampling epilogue and the tensor term need more registers: at chip 32
  // two tiles in FP32 (four spill) and one for the FP64 tensor term
  constexpr int NTL = TN && sizeof(T) == 8 && CH == 32 ? 1
                      : ((SAMPLE || TN) && sizeof(T) == 4 && CH == 32 ? 2 : ntiles<T>(CH));
  const size_t per_wave = size_t(P.W) * 16 * NTL * CH * sizeof(T);
  int wpb = 4;
  while (wpb > 1 && per_wave * wpb > 64 * 1024) wpb >>= 1;
  if (per_wave * wpb > 160 * 1024) return hipErrorInvalidValue;
  const int64_t tiles = (R + 16 * NTL - 1) / (16 * NTL);
  const int64_t blocks = (tiles + wpb - 1) / wpb;
  static_assert(!(D1 && TN), "a tensor site has two or three edges");
  static_assert(NTL <= 4, "the node-need marks assume at most 64 rows per wavefront");
  hipLaunchKernelGGL((k_psi_mt<T, CH, NTL, FOLD, STORE, SEED, SAMPLE, CPLX, TN, D1>), dim3(unsigned(blocks)),
                     dim3(64 * wpb), per_wave * wpb, st, P, m, R, lphi, sphi, wpb, X, SA, phs);
  return hipGetLastError();
}

// the eloc modes without the tensor term; D1: every site has one edge
template <typename T, int CH, bool D1>
hipError_t run_psi_modes(const PsiParams<T>& P, const uint64_t* m, int64_t R, double* lphi, int8_t* sphi,
                         hipStream_t st, const PsiStates<T>& X, int mode, double* phs) {
  if (phs) {
    // complex parameters: the phase of each row
    if (!P.w2 || !P.c2) return hipErrorInvalidValue;
    const SampleArgs no;
    switch (mode) {
      case PSI_PLAIN:
        if (P.folded) return run_psi_mt<T, CH, true, 0, false, false, true, false, D1>(P, m, R, lphi, sphi, st, X, no, phs);
        return run_psi_mt<T, CH, false, 0, false, false, true, false, D1>(P, m, R, lphi, sphi, st, X, no, phs);
      case PSI_STORE:
        if (!X.pz && X.pm) return hipErrorInvalidValue;
        if (P.folded) return run_psi_mt<T, CH, true, 1, false, false, true, false, D1>(P, m, R, lphi, sphi, st, X, no, phs);
        return run_psi_mt<T, CH, false, 1, false, false, true, false, D1>(P, m, R, lphi, sphi, st, X, no, phs);
      case PSI_SEED:
        if (!X.pz || (X.unode && !X.npz)) return hipErrorInvalidValue;
        if (P.folded) return run_psi_mt<T, CH, true, 0, true, false, true, false, D1>(P, m, R, lphi, sphi, st, X, no, phs);
        return run_psi_mt<T, CH, false, 0, true, false, true, false, D1>(P, m, R, lphi, sphi, st, X, no, phs);
      case PSI_NODE:
        if (!X.pz || !X.npz) return hipErrorInvalidValue;
        if (P.folded) return run_psi_mt<T, CH, true, 2, true, false, true, false, D1>(P, m, R, lphi, sphi, st, X, no, phs);
        return run_psi_mt<T, CH, false, 2, true, false, true, false, D1>(P, m, R, lphi, sphi, st, X, no, phs);
      default:
        return hipErrorInvalidValue;
    }
  }
  switch (mode) {
    case PSI_PLAIN:
      if (P.folded) return run_psi_mt<T, CH, true, 0, false, false, false, false, D1>(P, m, R, lphi, sphi, st, X);
      return run_psi_mt<T, CH, false, 0, false, false, false, false, D1>(P, m, R, lphi, sphi, st, X);
    case PSI_STORE:
      if (P.folded) return run_psi_mt<T, CH, true, 1, false, false, false, false, D1>(P, m, R, lphi, sphi, st, X);
      return run_psi_mt<T, CH, false, 1, false, false, false, false, D1>(P, m, R, lphi, sphi, st, X);
    case PSI_SEED:
      if (P.folded) return run_psi_mt<T, CH, true, 0, true, false, false, false, D1>(P, m, R, lphi, sphi, st, X);
      return run_psi_mt<T, CH, false, 0, true, false, false, false, D1>(P, m, R, lphi, sphi, st, X);
    case PSI_NODE:
      if (P.folded) return run_psi_mt<T, CH, true, 2, true, false, false, false, D1>(P, m, R, lphi, sphi, st, X);
      return run_psi_mt<T, CH, false, 2, true, false, false, false, D1>(P, m, R, lphi, sphi, st, X);
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T, int CH>
hipError_t run_psi_ch(const PsiParams<T>& P, const uint64_t* m, int64_t R, double* lphi, int8_t* sphi,
                      hipStream_t st, const PsiStates<T>& X, int mode, double* phs) {
  if (P.TA) {
    // tensor term on MFMA (chip <= 32, chi' <= 8)
    if constexpr (CH <= 32) {
      if (phs) return hipErrorInvalidValue;
      const SampleArgs no;
      switch (mode) {
        case PSI_PLAIN:
          if (P.folded) return run_psi_mt<T, CH, true, 0, false, false, false, true>(P, m, R, lphi, sphi, st, X, no);
          return run_psi_mt<T, CH, false, 0, false, false, false, true>(P, m, R, lphi, sphi, st, X, no);
        case PSI_STORE:
          if (P.folded) return run_psi_mt<T, CH, true, 1, false, false, false, true>(P, m, R, lphi, sphi, st, X, no);
          return run_psi_mt<T, CH, false, 1, false, false, false, true>(P, m, R, lphi, sphi, st, X, no);
        case PSI_SEED:
          if (P.folded) return run_psi_mt<T, CH, true, 0, true, false, false, true>(P, m, R, lphi, sphi, st, X, no);
          return run_psi_mt<T, CH, false, 0, true, false, false, true>(P, m, R, lphi, sphi, st, X, no);
        case PSI_NODE:
          if (P.folded) return run_psi_mt<T, CH, true, 2, true, false, false, true>(P, m, R, lphi, sphi, st, X, no);
          return run_psi_mt<T, CH, false, 2, true, false, false, true>(P, m, R, lphi, sphi, st, X, no);
        default:
          return hipErrorInvalidValue;
      }
    }
    return hipErrorInvalidValue;
  }
  if constexpr (CH <= 32) {
    if (P.d1) return run_psi_modes<T, CH, true>(P, m, R, lphi, sphi, st, X, mode, phs);
  }
  return run_psi_modes<T, CH, false>(P, m, R, lphi, sphi, st, X, mode, phs);
}

template <typename T, int CH>
hipError_t run_sample_ch(const PsiParams<T>& P, int64_t R, double* lphi, int8_t* sphi, hipStream_t st,
                         const SampleArgs& SA) {
  if (P.TA) {
    if constexpr (CH <= 32) {
      if (P.folded)
        return run_psi_mt<T, CH, true, 0, false, true, false, true>(P, nullptr, R, lphi, sphi, st, PsiStates<T>(), SA);
      return run_psi_mt<T, CH, false, 0, false, true, false, true>(P, nullptr, R, lphi, sphi, st, PsiStates<T>(), SA);
    }
    return hipErrorInvalidValue;
  }
  if constexpr (CH <= 32) {
    if (P.d1) {
      if (P.folded)
        return run_psi_mt<T, CH, true, 0, false, true, false, false, true>(P, nullptr, R, lphi, sphi, st, PsiStates<T>(),
                                                                          SA);
      return run_psi_mt<T, CH, false, 0, false, true, false, false, true>(P, nullptr, R, lphi, sphi, st, PsiStates<T>(),
                                                                         SA);
    }
  }
  if (P.folded) return run_psi_mt<T, CH, true, 0, false, true>(P, nullptr, R, lphi, sphi, st, PsiStates<T>(), SA);
  return run_psi_mt<T, CH, false, 0, false, true>(P, nullptr, R, lphi, sphi, st, PsiStates<T>(), SA);
}

template <typename T>
hipError_t dispatch_sample(const PsiParams<T>& P, int64_t R, double* lphi, int8_t* sphi, hipStream_t st,
                           const SampleArgs& SA) {
  switch (P.chip) {
    case 16: return run_sample_ch<T, 16>(P, R, lphi, sphi, st, SA);
    case 32: return run_sample_ch<T, 32>(P, R, lphi, sphi, st, SA);
    case 48: return run_sample_ch<T, 48>(P, R, lphi, sphi, st, SA);
    case 64: return run_sample_ch<T, 64>(P, R, lphi, sphi, st, SA);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t dispatch_psi(const PsiParams<T>& P, const uint64_t* m, int64_t R, double* lphi,
                        int8_t* sphi, hipStream_t st, const PsiStates<T>& X, int mode, double* phs) {
  switch (P.chip) {
    case 16: return run_psi_ch<T, 16>(P, m, R, lphi, sphi, st, X, mode, phs);
    case 32: return run_psi_ch<T, 32>(P, m, R, lphi, sphi, st, X, mode, phs);
    case 48: return run_psi_ch<T, 48>(P, m, R, lphi, sphi, st, X, mode, phs);
    case 64: return run_psi_ch<T, 64>(P, m, R, lphi, sphi, st, X, mode, phs);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_psi_f64(const PsiParams<double>& P, const uint64_t* m, int64_t R, double* lphi,
                          int8_t* sphi, hipStream_t st, const PsiStates<double>& X, int mode, double* phs) {
  return dispatch_psi<double>(P, m, R, lphi, sphi, st, X, mode, phs);
}

hipError_t launch_psi_f32(const PsiParams<float>& P, const uint64_t* m, int64_t R, double* lphi,
                          int8_t* sphi, hipStream_t st, const PsiStates<float>& X, int mode, double* phs) {
  return dispatch_psi<float>(P, m, R, lphi, sphi, st, X, mode, phs);
}

hipError_t launch_sample_f64(const PsiParams<double>& P, int64_t R, double* lphi, int8_t* sphi, hipStream_t st,
                             const SampleArgs& SA) {
  return dispatch_sample<double>(P, R, lphi, sphi, st, SA);
}

hipError_t launch_sample_f32(const PsiParams<float>& P, int64_t R, double* lphi, int8_t* sphi, hipStream_t st,
                             const SampleArgs& SA) {
  return dispatch_sample<float>(P, R, lphi, sphi, st, SA);
}

}  // namespace nqs
