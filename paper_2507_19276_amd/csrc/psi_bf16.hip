// BDG-RNN / MPS-RNN forward with BF16 bond contractions on gfx950
// (arXiv:2507.19276, Sec. 2.1 Eqs. (9)-(10), Sec. 2.2 Eq. (12) without the
// tensor term; the reduced-precision form of the amplitude evaluation): BF16
// operands on MFMA with FP32 accumulation, FP32 epilogue, scaled carried
// states.
//
// Same organisation as the FP64/FP32 kernel (psi.hip): a wavefront owns NTL
// tiles of 16 rows, rows are the N dimension of the MFMA, and the A operand is
// k-permuted so that the B operand of every MFMA is the lane's own carried
// state (lane (j, g) holds units 16 tt + 4 g + 0..3 of row j).  A k-step of the
// 16x16x32 BF16 MFMA takes two of a lane's quads (tt = 2q, 2q+1: element e is
// unit 16 (2q + e/4) + 4 g + e%4); when chip/16 is odd the last quad goes
// through one 16x16x16 step (element e is unit 16 tt + 4 g + e).
//
// Scaled states.  The ring keeps each carried state as BF16 h / 2^E, with one
// exponent E per ring slot shared by the wavefront.  A site with parents of
// exponents E_p works at E_ref = max E_p: parents with E_p < E_ref are scaled
// by 2^(E_p - E_ref), the accumulators start from v / 2^E_ref and the sign
// test uses c / 2^E_ref.  The conditionals P^s / sum P and the sign of
// w^T h + c do not depend on a common power-of-two scale, and every operation
// here (BF16 rounding, MFMA products and sums, FP32 arithmetic) commutes with
// it exactly barring underflow, so the result does not depend on the
// exponents chosen.  A new state keeps E_ref unless the largest normaliser Z
// of the wavefront leaves [2^-40, 2^40]; then it is renormalised by 2^(e/2)
// with e the exponent of that Z, which keeps every operand far from the ends
// of the FP32/BF16 range whatever the magnitudes of v and M.
//
// Split form (SPLIT): every operand is carried as two BF16 parts, x = hi + lo
// with hi = bf16(x) and lo = bf16(x - hi), the A stream as well (built on the
// host) and the carried states (hi and lo quads in the ring); each k-step
// runs three MFMAs, hi.hi + hi.lo + lo.hi, all on the BF16 matrix cores with
// FP32 accumulation.  The dropped lo.lo product and the representation error
// are below 2^-16 of each product, so the states carry relative errors near
// 2^-15 instead of 2^-8.  Power-of-two scaling applies to both parts alike.
#include "device.h"
#include <type_traits>

namespace nqs {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef unsigned u2 __attribute__((ext_vector_type(2)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

__device__ inline f4 mfma_k32(u4 a, u4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0,
                                                 0);
}
__device__ inline f4 mfma_k16(u2 a, u2 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, a), __builtin_bit_cast(s4, b), c, 0, 0,
                                                   0);
}

// four FP32 values to a BF16 quad (round to nearest even)
__device__ inline u2 pack_bf16(f4 x) {
  const bf2 lo = {(__bf16)x.x, (__bf16)x.y};
  const bf2 hi = {(__bf16)x.z, (__bf16)x.w};
  return u2{__builtin_bit_cast(unsigned, lo), __builtin_bit_cast(unsigned, hi)};
}
__device__ inline f4 unpack_bf16(u2 q) {
  return f4{__uint_as_float(q.x << 16), __uint_as_float(q.x & 0xFFFF0000u), __uint_as_float(q.y << 16),
            __uint_as_float(q.y & 0xFFFF0000u)};
}
// a BF16 quad times 2^k, k <= 0 (exact barring underflow)
__device__ inline u2 scale_bf16(u2 q, int k) {
  f4 x = unpack_bf16(q);
  x.x = ldexpf(x.x, k);
  x.y = ldexpf(x.y, k);
  x.z = ldexpf(x.z, k);
  x.w = ldexpf(x.w, k);
  return pack_bf16(x);
}

// maximum over the wavefront (all lanes receive it)
__device__ inline float wave_max(float x) {
  float a, b;
  pl32(x, x, a, b);
  x = fmaxf(a, b);
  pl16(x, x, a, b);
  x = fmaxf(a, b);
  // within each row of 16 lanes: rotations by 1, 2, 4, 8 (DPP row_ror)
  x = fmaxf(x, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x121, 0xF, 0xF, false)));
  x = fmaxf(x, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x122, 0xF, 0xF, false)));
  x = fmaxf(x, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x124, 0xF, 0xF, false)));
  x = fmaxf(x, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x128, 0xF, 0xF, false)));
  return x;
}
__device__ inline int wave_max(int x) {
  float a, b;
  pl32(__int_as_float(x), __int_as_float(x), a, b);
  x = max(__float_as_int(a), __float_as_int(b));
  pl16(__int_as_float(x), __int_as_float(x), a, b);
  x = max(__float_as_int(a), __float_as_int(b));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x121, 0xF, 0xF, false));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x122, 0xF, 0xF, false));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x124, 0xF, 0xF, false));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false));
  return x;
}

template <int CH> constexpr int ntiles_b16() { return CH <= 16 ? 4 : (CH <= 32 ? 2 : 1); }

template <int CH, int NTL, bool FOLD, bool STORE, bool SEED, bool D1, bool SPLIT>
__global__ __launch_bounds__(256) void k_psi_b16(B16Params P, const uint64_t* __restrict__ m, int64_t R,
                                                 double* __restrict__ lphi, int8_t* __restrict__ sphi, int wpb,
                                                 B16States X) {
  // explicit floating-point operations only (see psi.hip): resumed rows end
  // bit-identical to rows evaluated from site 0
#pragma clang fp contract(off)
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int TPC = CH / 16, NT = 4 * TPC, NP = TPC / 2, ODD = TPC & 1, RW = 16 * NTL;
  constexpr int SLOT = NTL * TPC * 64;                          // quads per ring slot and part
  constexpr int PARTS = SPLIT ? 2 : 1;                          // hi (and lo) quads per slot
  constexpr int64_t EQ = int64_t(NP) * NT * 64 * 2 + ODD * NT * 64;       // A stream: u2 units per edge
  // A operands: with pair steps only and where it costs no occupancy (32
  // registers), a rolling window of one k-step (each k-step's slot, once its
  // MFMAs are issued, receives the next k-step of the stream, the next edge's
  // first past the last); otherwise the next edge's first k-step is fetched
  // ahead where it fits
  constexpr bool ROLL = !ODD && NT * 4 * PARTS <= 32;
  constexpr bool APF = !ROLL && NT * (NP ? 4 : 2) * PARTS <= 32;
  // the bias is fetched at the start of its site, not a site ahead: the 32
  // registers a prefetch holds cost a wavefront per SIMD at chip 16 and 32
  // (measured at chip 32: 124 -> 109 ms per launch on the K = 50 batch with
  // three wavefronts per SIMD instead of two)
  constexpr bool BPF = false;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int j = lane & 15, g = lane >> 4;
  const int own = NTL == 4 ? g : (NTL == 2 ? (g >> 1) : 0);
  const int64_t base = (int64_t(blockIdx.x) * wpb + wv) * RW;
  if (base >= R) return;   // surplus wavefront of the last block (no block barrier below)
  // per wavefront: W slots of quads (each slot: the hi part, then with SPLIT
  // the lo part), then W exponents, all lane-private (every lane keeps its
  // own copy of the wavefront-uniform exponents); site i writes slot wsl[i],
  // a zero edge (slot index W) reads no slot
  const size_t wbytes = size_t(P.W) * (SLOT * 8 * PARTS + 64 * 4);
  u2* ring = reinterpret_cast<u2*>(smem + size_t(wv) * wbytes) + lane;
  int* Ering = reinterpret_cast<int*>(smem + size_t(wv) * wbytes + size_t(P.W) * SLOT * 8 * PARTS) + lane;
  const CInt* fptr = (const CInt*)(P.pptr);
  const CInt* slots = (const CInt*)(P.slot);
  const CInt* wsl = (const CInt*)(P.wsl);
  const CT<float>* cc = (const CT<float>*)(P.c);
  const int i0 = SEED ? int(((const __attribute__((address_space(4))) uint8_t*)X.t0)[base]) : 0;
  uint64_t lo[NTL], hi[NTL];
  int64_t rowt[NTL];
  uint64_t olo = 0, ohi = 0;
#pragma unroll
  for (int t = 0; t < NTL; ++t) {
    const int64_t r = base + 16 * t + j;
    const int64_t rr = r < R ? r : R - 1;
    rowt[t] = SEED ? int64_t(X.perm[rr]) : rr;
    lo[t] = m[2 * rowt[t]];
    hi[t] = m[2 * rowt[t] + 1];
    if (t == own) { olo = lo[t]; ohi = hi[t]; }
  }
  const bool olive = base + 16 * own + j < R;
  int64_t orow = rowt[0];
#pragma unroll
  for (int t = 1; t < NTL; ++t)
    if (t == own) orow = rowt[t];
  float prod = 1.0f;
  int pexp = 0, sgn = 1, ca = 0, cb = 0, e = 0;
  bool bad = false;
  if (SEED && i0 > 0) {
    // carried states of the parents of sites >= i0 from the rows' samples,
    // brought to one exponent per slot (the wavefront's largest)
    // the states live at i0 (read by a site >= i0; distinct slots)
    for (uint64_t lv = ((const __attribute__((address_space(4))) uint64_t*)P.live)[i0]; lv; lv &= lv - 1) {
      const int s = __builtin_ctzll(lv);
      int es[NTL], emax = -(1 << 30);
#pragma unroll
      for (int t = 0; t < NTL; ++t) {
        es[t] = X.he[size_t(s) * X.ns + X.owner[rowt[t]]];
        emax = max(emax, es[t]);
      }
      const int ew = __builtin_amdgcn_readfirstlane(wave_max(emax));
      u2* wr = ring + size_t(wsl[s]) * SLOT * PARTS;
#pragma unroll
      for (int t = 0; t < NTL; ++t) {
        const size_t so = (size_t(s) * X.ns + X.owner[rowt[t]]) * CH + 4 * g;
        const u2* src = reinterpret_cast<const u2*>(X.hs + so);
#pragma unroll
        for (int tt = 0; tt < TPC; ++tt) {
          u2 q = src[4 * tt];
          if (es[t] != ew) q = scale_bf16(q, es[t] - ew);
          wr[(t * TPC + tt) * 64] = q;
          if constexpr (SPLIT) {
            u2 ql = reinterpret_cast<const u2*>(X.hs_lo + so)[4 * tt];
            if (es[t] != ew) ql = scale_bf16(ql, es[t] - ew);
            wr[SLOT + (t * TPC + tt) * 64] = ql;
          }
        }
      }
      Ering[wsl[s] * 64] = ew;
    }
    const size_t so = size_t(i0) * X.ns + X.owner[orow];
    prod = X.pm[so];
    pexp = X.pe[so];
    sgn = X.pg[so];
    const uint64_t below = low_bits(2 * i0), belowh = low_bits(2 * i0 - 64);
    ca = __popcll(olo & below & 0x5555555555555555ull) + __popcll(ohi & belowh & 0x5555555555555555ull);
    cb = __popcll(olo & below & 0xAAAAAAAAAAAAAAAAull) + __popcll(ohi & belowh & 0xAAAAAAAAAAAAAAAAull);
    e = fptr[i0];
  }
  // A stream in u2 units: per edge NP pair steps of [ot][lane] u4, then (ODD)
  // one step of [ot][lane] u2
  const u2* __restrict__ Ab = reinterpret_cast<const u2*>(P.A);
  const u2* __restrict__ Abl = reinterpret_cast<const u2*>(P.Alo);   // SPLIT: lo parts, same layout
  typedef typename std::conditional<(NP > 0), u4, u2>::type FA;   // first k-step operand type
  constexpr int NA = APF || ROLL ? NT : 1;
  FA an[NA], anl[NA];   // anl: lo parts (SPLIT only)
  auto first_step = [&](const u2* base, int64_t edge, FA (&dst)[NA]) {
#pragma unroll
    for (int ot = 0; ot < NA; ++ot) {
      if constexpr (NP > 0)
        dst[ot] = reinterpret_cast<const u4*>(base + edge * EQ)[ot * 64 + lane];
      else
        dst[ot] = (base + edge * EQ)[ot * 64 + lane];
    }
  };
  if (APF || ROLL) first_step(Ab, e, an);
  if ((APF || ROLL) && SPLIT) first_step(Abl, e, anl);
  f4 vn[NT];
  auto fetch_bias = [&](int i) {
#pragma unroll
    for (int ot = 0; ot < NT; ++ot)
      vn[ot] = *reinterpret_cast<const f4*>(P.v + (size_t(i) * 4 + ot / TPC) * CH + 16 * (ot % TPC) + 4 * g);
  };
  if (BPF) fetch_bias(i0 < P.K ? i0 : 0);
  auto store_pre = [&](int i) {
    const bool writer = NTL == 4 || (NTL == 2 ? (g & 1) == 0 : g == 0);
    if (STORE && writer && olive && orow < X.ns) {
      const size_t so = size_t(i) * X.ns + orow;
      X.pm[so] = prod;
      X.pe[so] = pexp;
      X.pg[so] = int8_t(sgn);
    }
  };
  for (int i = i0; i < P.K; ++i) {
    store_pre(i);
    const int wslot = wsl[i];
    f4 acc[NTL][NT], wv4[TPC], ev4[TPC];
#pragma unroll
    for (int tt = 0; tt < TPC; ++tt) {
      wv4[tt] = *reinterpret_cast<const f4*>(P.w + size_t(i) * CH + 16 * tt + 4 * g);
      if (!FOLD) ev4[tt] = *reinterpret_cast<const f4*>(P.eta + size_t(i) * CH + 16 * tt + 4 * g);
    }
    const int e1 = fptr[i + 1];
    // the parents' common exponent (a zero edge counts as exponent 0)
    int eref = -(1 << 30);
    for (int ee = e; ee < e1; ++ee)
      eref = max(eref, slots[ee] >= P.W ? 0 : __builtin_amdgcn_readfirstlane(Ering[slots[ee] * 64]));
    // (first: the edge's first MFMAs start from the scaled bias registers
    // instead of copies of them in the accumulators)
    auto edge = [&](auto first) {
      const u2* Ae = Ab + int64_t(e) * EQ;
      const u2* Ael = Abl + int64_t(e) * EQ;
      const int sl = slots[e];
      const bool zero = sl >= P.W;   // a parentless site's zero edge: zero operand
      const int ep = zero ? 0 : __builtin_amdgcn_readfirstlane(Ering[sl * 64]);
      u2 b[NTL][TPC], bl[NTL][SPLIT ? TPC : 1];
      const u2* rp = ring + size_t(zero ? 0 : sl) * SLOT * PARTS;
#pragma unroll
      for (int t = 0; t < NTL; ++t)
#pragma unroll
        for (int tt = 0; tt < TPC; ++tt) {
          b[t][tt] = zero ? u2{0u, 0u} : rp[(t * TPC + tt) * 64];
          if constexpr (SPLIT) bl[t][tt] = zero ? u2{0u, 0u} : rp[SLOT + (t * TPC + tt) * 64];
        }
      if (ep != eref) {
#pragma unroll
        for (int t = 0; t < NTL; ++t)
#pragma unroll
          for (int tt = 0; tt < TPC; ++tt) {
            b[t][tt] = scale_bf16(b[t][tt], ep - eref);
            if constexpr (SPLIT) bl[t][tt] = scale_bf16(bl[t][tt], ep - eref);
          }
      }
      FA nx[APF ? NT : 1], nxl[APF ? NT : 1];
      // (the stream carries one zero edge past the last)
      if constexpr (APF) {
        first_step(Ab, int64_t(e) + 1, nx);
        if constexpr (SPLIT) first_step(Abl, int64_t(e) + 1, nxl);
      }
#pragma unroll
      for (int q = 0; q < NP; ++q)
#pragma unroll
        for (int ot = 0; ot < NT; ++ot) {
          u4 a, al;
          if constexpr (ROLL)
            a = an[ot];
          else if constexpr (NP > 0 && APF)
            a = q == 0 ? an[ot] : reinterpret_cast<const u4*>(Ae)[(q * NT + ot) * 64 + lane];
          else
            a = reinterpret_cast<const u4*>(Ae)[(q * NT + ot) * 64 + lane];
          if constexpr (SPLIT) {
            if constexpr (ROLL)
              al = anl[ot];
            else if constexpr (NP > 0 && APF)
              al = q == 0 ? anl[ot] : reinterpret_cast<const u4*>(Ael)[(q * NT + ot) * 64 + lane];
            else
              al = reinterpret_cast<const u4*>(Ael)[(q * NT + ot) * 64 + lane];
          }
#pragma unroll
          for (int t = 0; t < NTL; ++t) {
            const u4 bq = {b[t][2 * q].x, b[t][2 * q].y, b[t][2 * q + 1].x, b[t][2 * q + 1].y};
            acc[t][ot] = mfma_k32(a, bq, decltype(first)::value && q == 0 ? vn[ot] : acc[t][ot]);
            if constexpr (SPLIT) {
              const u4 bql = {bl[t][2 * q].x, bl[t][2 * q].y, bl[t][2 * q + 1].x, bl[t][2 * q + 1].y};
              acc[t][ot] = mfma_k32(a, bql, acc[t][ot]);
              acc[t][ot] = mfma_k32(al, bq, acc[t][ot]);
            }
          }
          if constexpr (ROLL) {
            an[ot] = reinterpret_cast<const u4*>(Ae)[((q + 1) * NT + ot) * 64 + lane];
            if constexpr (SPLIT) anl[ot] = reinterpret_cast<const u4*>(Ael)[((q + 1) * NT + ot) * 64 + lane];
          }
        }
      if constexpr (ODD) {
#pragma unroll
        for (int ot = 0; ot < NT; ++ot) {
          u2 a, al;
          if constexpr (NP == 0 && APF)
            a = an[ot];
          else
            a = (Ae + int64_t(NP) * NT * 64 * 2)[ot * 64 + lane];
          if constexpr (SPLIT) {
            if constexpr (NP == 0 && APF)
              al = anl[ot];
            else
              al = (Ael + int64_t(NP) * NT * 64 * 2)[ot * 64 + lane];
          }
#pragma unroll
          for (int t = 0; t < NTL; ++t) {
            acc[t][ot] = mfma_k16(a, b[t][TPC - 1], decltype(first)::value && NP == 0 ? vn[ot] : acc[t][ot]);
            if constexpr (SPLIT) {
              acc[t][ot] = mfma_k16(a, bl[t][TPC - 1], acc[t][ot]);
              acc[t][ot] = mfma_k16(al, b[t][TPC - 1], acc[t][ot]);
            }
          }
        }
      }
      if constexpr (APF) {
#pragma unroll
        for (int ot = 0; ot < NT; ++ot) {
          an[ot] = nx[ot];
          if constexpr (SPLIT) anl[ot] = nxl[ot];
        }
      }
    };
    if (!BPF) fetch_bias(i);
    const float sc = ldexpf(1.0f, -eref);
    __builtin_amdgcn_s_setprio(PRIO);
    if constexpr (D1 || ROLL) {
      // the bias at the parents' exponent, in place (exact: sc is a power of
      // two); the first edge's MFMAs start from it, the later edges accumulate
      // (D1: every site has exactly one edge)
      if (eref != 0) {
#pragma unroll
        for (int ot = 0; ot < NT; ++ot) vn[ot] = vn[ot] * sc;
      }
      edge(std::true_type{});
      ++e;
      if (BPF) fetch_bias(i + 1 < P.K ? i + 1 : i);
      if constexpr (!D1)
        for (; e < e1; ++e) edge(std::false_type{});
    } else {
      // (the bias registers stay free for the next site's: fewer registers
      // live through the first edge where no rolling window holds them)
      if (eref == 0) {
#pragma unroll
        for (int ot = 0; ot < NT; ++ot)
#pragma unroll
          for (int t = 0; t < NTL; ++t) acc[t][ot] = vn[ot];
      } else {
#pragma unroll
        for (int ot = 0; ot < NT; ++ot) {
          const f4 vsc = vn[ot] * sc;
#pragma unroll
          for (int t = 0; t < NTL; ++t) acc[t][ot] = vsc;
        }
      }
      if (BPF) fetch_bias(i + 1 < P.K ? i + 1 : i);
      do edge(std::false_type{}); while (++e < e1);
    }
    __builtin_amdgcn_s_setprio(0);
    // epilogue (FP32): P^s, selection, w.h; the new states are written after
    // the renormalisation decision
    int si[NTL];
#pragma unroll
    for (int t = 0; t < NTL; ++t) si[t] = site_state(lo[t], hi[t], i);
    float pp[4][NTL], dp[NTL];
    f4 selv[NTL][TPC];
#pragma unroll
    for (int t = 0; t < NTL; ++t) {
      dp[t] = 0.0f;
#pragma unroll
      for (int s = 0; s < 4; ++s) pp[s][t] = 0.0f;
    }
#pragma unroll
    for (int tt = 0; tt < TPC; ++tt) {
      const f4 ww = wv4[tt];
#pragma unroll
      for (int t = 0; t < NTL; ++t) {
        f4 x[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          x[s] = acc[t][s * TPC + tt];
          const f4 ex = FOLD ? x[s] : ev4[tt] * x[s];
          float q = pp[s][t];
          q = tfma(ex.x, x[s].x, q);
          q = tfma(ex.y, x[s].y, q);
          q = tfma(ex.z, x[s].z, q);
          q = tfma(ex.w, x[s].w, q);
          pp[s][t] = q;
        }
        const f4 sel01 = (si[t] & 1) ? x[1] : x[0];
        const f4 sel23 = (si[t] & 1) ? x[3] : x[2];
        const f4 sel = (si[t] & 2) ? sel23 : sel01;
        float d = dp[t];
        d = tfma(ww.x, sel.x, d);
        d = tfma(ww.y, sel.y, d);
        d = tfma(ww.z, sel.z, d);
        d = tfma(ww.w, sel.w, d);
        dp[t] = d;
        selv[t][tt] = sel;
      }
    }
    float ps[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) ps[s] = ReduceOwn<float, NTL>::run(pp[s]);
    const float dot = ReduceOwn<float, NTL>::run(dp) + float(cc[i]) * sc;
    const int osi = site_state(olo, ohi, i);
    const int rest = P.K - 1 - i;
    float Z = 0.0f;
#pragma unroll
    for (int s = 0; s < 4; ++s)
      if (allowed(ca, cb, s, rest, P.na, P.nb)) Z += ps[s];
    if (!allowed(ca, cb, osi, rest, P.na, P.nb)) bad = true;
    const float p01 = (osi & 1) ? ps[1] : ps[0];
    const float p23 = (osi & 1) ? ps[3] : ps[2];
    const float psi_ = (osi & 2) ? p23 : p01;
    int ex;
    prod = tfrexp(prod * (psi_ / Z), &ex);
    pexp += ex;
    if (dot < 0.0f) sgn = -sgn;
    ca += osi & 1;
    cb += osi >> 1;
    // renormalise the new states when the wavefront's largest Z leaves
    // [2^-40, 2^40] (Z = sum_s |x_s|^2 bounds every unit of the state by sqrt(Z))
    const float zmax = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wave_max(Z))));
    int ez = 0;
    if (zmax > 0.0f && zmax < INFINITY) (void)frexpf(zmax, &ez);
    const int kz = (ez > 40 || ez < -40) ? (ez >> 1) : 0;
    const int enew = eref + kz;
    u2* wr = ring + size_t(wslot) * SLOT * PARTS;
#pragma unroll
    for (int t = 0; t < NTL; ++t)
#pragma unroll
      for (int tt = 0; tt < TPC; ++tt) {
        f4 v = selv[t][tt];
        if (kz != 0) v = v * ldexpf(1.0f, -kz);
        const u2 q = pack_bf16(v);
        wr[(t * TPC + tt) * 64] = q;
        u2 ql = u2{0u, 0u};
        if constexpr (SPLIT) {
          ql = pack_bf16(v - unpack_bf16(q));   // v - hi is exact in FP32
          wr[SLOT + (t * TPC + tt) * 64] = ql;
        }
        if (STORE) {
          const int64_t r = base + 16 * t + j;
          const size_t so = (size_t(i) * X.ns + r) * CH + 16 * tt + 4 * g;
          if (r < X.ns) {
            *reinterpret_cast<u2*>(X.hs + so) = q;
            if constexpr (SPLIT) *reinterpret_cast<u2*>(X.hs_lo + so) = ql;
          }
        }
      }
    Ering[wslot * 64] = enew;
    if (STORE) {
#pragma unroll
      for (int t = 0; t < NTL; ++t) {
        const int64_t r = base + 16 * t + j;
        if (g == 0 && r < X.ns) X.he[size_t(i) * X.ns + r] = enew;
      }
    }
  }
  store_pre(P.K);
  const bool writer = NTL == 4 || (NTL == 2 ? (g & 1) == 0 : g == 0);
  if (writer && olive) {
    lphi[orow] = bad ? -INFINITY : 0.5 * (log(double(prod)) + double(pexp) * 0.69314718055994530942);
    sphi[orow] = int8_t(bad ? 0 : sgn);
  }
}

template <int CH, bool FOLD, bool STORE, bool SEED, bool D1, bool SPLIT>
hipError_t run_b16(const B16Params& P, const uint64_t* m, int64_t R, double* lphi, int8_t* sphi, hipStream_t st,
                   const B16States& X) {
  if (R <= 0) return hipSuccess;
  if (SPLIT && (!P.Alo || (STORE && !X.hs_lo) || (SEED && !X.hs_lo))) return hipErrorInvalidValue;
  constexpr int NTL = ntiles_b16<CH>();
  constexpr int TPC = CH / 16;
  const size_t per_wave = size_t(P.W) * (NTL * TPC * 64 * 8 * (SPLIT ? 2 : 1) + 64 * 4);
  int wpb = 4;
  while (wpb > 1 && per_wave * wpb > 64 * 1024) wpb >>= 1;
  if (per_wave * wpb > 160 * 1024) return hipErrorInvalidValue;
  const int64_t tiles = (R + 16 * NTL - 1) / (16 * NTL);
  const int64_t blocks = (tiles + wpb - 1) / wpb;
  hipLaunchKernelGGL((k_psi_b16<CH, NTL, FOLD, STORE, SEED, D1, SPLIT>), dim3(unsigned(blocks)), dim3(64 * wpb),
                     per_wave * wpb, st, P, m, R, lphi, sphi, wpb, X);
  return hipGetLastError();
}

// D1: every site has one edge
template <int CH, bool D1, bool SPLIT>
hipError_t run_b16_modes(const B16Params& P, const uint64_t* m, int64_t R, double* lphi, int8_t* sphi,
                         hipStream_t st, const B16States& X, int mode) {
  switch (mode) {
    case PSI_PLAIN:
      if (P.folded) return run_b16<CH, true, false, false, D1, SPLIT>(P, m, R, lphi, sphi, st, X);
      return run_b16<CH, false, false, false, D1, SPLIT>(P, m, R, lphi, sphi, st, X);
    case PSI_STORE:
      if (P.folded) return run_b16<CH, true, true, false, D1, SPLIT>(P, m, R, lphi, sphi, st, X);
      return run_b16<CH, false, true, false, D1, SPLIT>(P, m, R, lphi, sphi, st, X);
    case PSI_SEED:
      if (P.folded) return run_b16<CH, true, false, true, D1, SPLIT>(P, m, R, lphi, sphi, st, X);
      return run_b16<CH, false, false, true, D1, SPLIT>(P, m, R, lphi, sphi, st, X);
    default:
      return hipErrorInvalidValue;
  }
}

template <int CH, bool SPLIT>
hipError_t run_b16_ch(const B16Params& P, const uint64_t* m, int64_t R, double* lphi, int8_t* sphi,
                      hipStream_t st, const B16States& X, int mode) {
  if constexpr (CH <= 32) {
    if (P.d1) return run_b16_modes<CH, true, SPLIT>(P, m, R, lphi, sphi, st, X, mode);
  }
  return run_b16_modes<CH, false, SPLIT>(P, m, R, lphi, sphi, st, X, mode);
}

}  // namespace

hipError_t launch_psi_bf16(const B16Params& P, const uint64_t* m, int64_t R, double* lphi, int8_t* sphi,
                           hipStream_t st, const B16States& X, int mode, bool split) {
  if (split) {
    switch (P.chip) {
      case 16: return run_b16_ch<16, true>(P, m, R, lphi, sphi, st, X, mode);
      case 32: return run_b16_ch<32, true>(P, m, R, lphi, sphi, st, X, mode);
      case 48: return run_b16_ch<48, true>(P, m, R, lphi, sphi, st, X, mode);
      case 64: return run_b16_ch<64, true>(P, m, R, lphi, sphi, st, X, mode);
      default: return hipErrorInvalidValue;
    }
  }
  switch (P.chip) {
    case 16: return run_b16_ch<16, false>(P, m, R, lphi, sphi, st, X, mode);
    case 32: return run_b16_ch<32, false>(P, m, R, lphi, sphi, st, X, mode);
    case 48: return run_b16_ch<48, false>(P, m, R, lphi, sphi, st, X, mode);
    case 64: return run_b16_ch<64, false>(P, m, R, lphi, sphi, st, X, mode);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace nqs
