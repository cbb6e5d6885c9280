// BDG-TensorRNN forward (Sec. 2.2, Eqs. (12)-(13)) on gfx950: log|Phi| and
// sign Phi of rows, or exact autoregressive draws from Phi^2 (Sec. 2.1, masks
// of Sec. 3).  At a site with d >= 2 parents the candidates gain the tensor
// term in Tucker form,
//   t^s = K0 q^s,  q^s[i'] = sum_a U^s[i'][a_1..a_d] prod_j p_j[a_j],
//   p_j = K_j^T h_(parent j),
// with chi' = ceil(chi^(2/(d+1))) <= 16 and d <= 3.
//
// One thread per row.  Every parameter is the same for all rows, so the
// kernel reads the weights through the constant address space (scalar loads,
// used directly as SGPR operands of the FMAs) and keeps only row data in
// vector registers: a chunk of 16 candidate units, and in LDS the row's carried
// states of the last W sites ([slot][unit][thread], thread fastest, rw =
// ceil4(chi) units: the parameter blocks are zero beyond chi, so the padded
// units of a chunk are never stored or read) plus the projections p and the
// core contraction q.  Each candidate chunk is
// accumulated over (parent, unit) pairs with one LDS read per 16 FMAs.  The
// parameter layout is the library's (see runtime.cpp): per edge M^T as
// [s][k][u], per site v, eta, w, c, and per tensor site K0^T [i'][u], K_j as
// [j][v][a padded to QP] and U^s as [s][i'][a_1..a_(d-1)][a_d padded to QP],
// QP = 8 when every chi' <= 8, else 16, all padded to chip = ceil16(chi)
// units.  The projections and the core contraction are unrolled over QP
// (zero-padded) entries, so every weight row is one scalar QP-dword load
// feeding QP FMAs.
#include "device.h"
#include "philox.h"

namespace nqs {
namespace {

constexpr int kTnThreads = 64;

template <typename T, int QP, bool SAMPLE>
__global__ __launch_bounds__(kTnThreads) void k_psi_tn(TnParams<T> P, const uint64_t* __restrict__ m, int64_t R,
                                                       double* __restrict__ lphi, int8_t* __restrict__ sphi,
                                                       SampleArgs SA) {
#pragma clang fp contract(off)
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  constexpr int NT = kTnThreads;
  const int CP = P.chip, RW = P.rw;
  T* ring = reinterpret_cast<T*>(smem);                          // [W][rw][NT]
  T* pl = ring + size_t(P.W) * RW * NT;                          // [QP][NT]: first projection (d = 3)
  auto RG = [&](int slot, int k) -> T& { return ring[(size_t(slot) * RW + k) * NT + tid]; };
  auto PL = [&](int a) -> T& { return pl[a * NT + tid]; };
  const int64_t r = int64_t(blockIdx.x) * NT + tid;
  const bool live = r < R;
  const int64_t rr = live ? r : R - 1;
  const uint64_t lo = SAMPLE ? 0ull : m[2 * rr], hi = SAMPLE ? 0ull : m[2 * rr + 1];
  uint64_t olo = 0, ohi = 0;
  const CT<T>* W = (const CT<T>*)P.prm;
  const CInt* pptr = (const CInt*)P.pptr;
  const CInt* edge = (const CInt*)P.edge;
  const CInt* site = (const CInt*)P.site;
  T prod = T(1);
  int pexp = 0, sgn = 1, ca = 0, cb = 0;
  bool bad = false;
  // projections p_0..p_(d-1) (QP entries each, zero beyond chi') and the
  // core contraction q^s (QP entries, zero beyond chi')
  T p0[QP], p1[QP], p2[QP], q[QP];
  auto core = [&](int s, int Q, int d, int offU) {
#pragma unroll
    for (int ip = 0; ip < QP; ++ip) {
      q[ip] = T(0);
      if (ip >= Q) continue;
      T acc = T(0);
      if (d == 2) {
        const int base = offU + (s * Q + ip) * Q * QP;
#pragma unroll
        for (int a1 = 0; a1 < QP; ++a1) {
          if (a1 >= Q) continue;
          T in = T(0);
#pragma unroll
          for (int a2 = 0; a2 < QP; ++a2) in = tfma(T(W[base + a1 * QP + a2]), p1[a2], in);
          acc = tfma(p0[a1], in, acc);
        }
      } else {
        const int base = offU + (s * Q + ip) * Q * Q * QP;
        for (int a1 = 0; a1 < Q; ++a1) {
          T in = T(0);
#pragma unroll
          for (int a2 = 0; a2 < QP; ++a2) {
            if (a2 >= Q) continue;
            T in3 = T(0);
#pragma unroll
            for (int a3 = 0; a3 < QP; ++a3) in3 = tfma(T(W[base + (a1 * Q + a2) * QP + a3]), p2[a3], in3);
            in = tfma(p1[a2], in3, in);
          }
          acc = tfma(PL(a1), in, acc);
        }
      }
      q[ip] = acc;
    }
  };
  for (int i = 0; i < P.K; ++i) {
    const int e0 = pptr[i], e1 = pptr[i + 1], d = e1 - e0;
    const int offV = site[8 * i], offEta = site[8 * i + 1], offW = site[8 * i + 2], offC = site[8 * i + 3];
    const int Q = site[8 * i + 4], offK0 = site[8 * i + 5], offKj = site[8 * i + 6], offU = site[8 * i + 7];
    const int wslot = i % P.W;
    // projections of the parents' states on their factor matrices
    if (Q) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        if (j >= d) continue;
        const int ps = edge[2 * (e0 + j) + 1];
        T pa[QP];
#pragma unroll
        for (int a = 0; a < QP; ++a) pa[a] = T(0);
#pragma unroll 4
        for (int v = 0; v < RW; ++v) {
          const T hv = RG(ps, v);
#pragma unroll
          for (int a = 0; a < QP; ++a) pa[a] = tfma(T(W[offKj + (j * CP + v) * QP + a]), hv, pa[a]);
        }
#pragma unroll
        for (int a = 0; a < QP; ++a) {
          if (j == 0) p0[a] = pa[a];
          if (j == 1) p1[a] = pa[a];
          if (j == 2) p2[a] = pa[a];
        }
      }
      if (d == 3) {
#pragma unroll
        for (int a = 0; a < QP; ++a) PL(a) = p0[a];
      }
    }
    const int si = SAMPLE ? 0 : site_state(lo, hi, i);
    T Ps[4];
    T dot = T(W[offC]);
    // candidate s in chunks of 16 units; P^s accumulated; with STORE_S the
    // chunk of the row's own state is written to the ring and w.h accumulated
    auto candidate = [&](int s, bool uniform_s, bool store) {
      T Pacc = T(0);
      if (Q) core(s, Q, d, offU);
      for (int uc = 0; uc < CP; uc += 16) {
        T acc[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) acc[u] = T(W[offV + s * CP + uc + u]);
        for (int e = e0; e < e1; ++e) {
          const int offM = edge[2 * e], ps = edge[2 * e + 1];
#pragma unroll 4
          for (int k = 0; k < RW; ++k) {
            const T hk = RG(ps, k);
#pragma unroll
            for (int u = 0; u < 16; ++u) acc[u] = tfma(T(W[offM + (s * CP + k) * CP + uc + u]), hk, acc[u]);
          }
        }
        if (Q) {
#pragma unroll
          for (int ip = 0; ip < QP; ++ip) {
            if (ip >= Q) continue;
#pragma unroll
            for (int u = 0; u < 16; ++u) acc[u] = tfma(T(W[offK0 + ip * CP + uc + u]), q[ip], acc[u]);
          }
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const T ex = T(W[offEta + uc + u]) * acc[u];
          Pacc = tfma(ex, acc[u], Pacc);
        }
        if (store) {
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            if (uc + u < RW && (uniform_s ? (s == si) : true)) {
              RG(wslot, uc + u) = acc[u];
              dot = tfma(T(W[offW + uc + u]), acc[u], dot);
            }
          }
        }
      }
      return Pacc;
    };
    for (int s = 0; s < 4; ++s) Ps[s] = candidate(s, true, !SAMPLE);
    const int rest = P.K - 1 - i;
    T Z = T(0);
#pragma unroll
    for (int s = 0; s < 4; ++s)
      if (allowed(ca, cb, s, rest, P.na, P.nb)) Z += Ps[s];
    int pick = si;
    if (SAMPLE) {
      const uint64_t pid = uint64_t(SA.p0 + rr);
      uint32_t U4[4];
      philox4x32_10(uint32_t(pid), uint32_t(pid >> 32), uint32_t(i), kSampleTag, SA.k0, SA.k1, U4);
      const double uu = double(((uint64_t(U4[1]) << 32) | U4[0]) >> 11) * 0x1p-53;
      const T target = T(uu) * Z;
      T run = T(0);
      int last = -1;
      pick = -1;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const T pr = allowed(ca, cb, s, rest, P.na, P.nb) ? Ps[s] : T(0);
        if (pr > T(0)) {
          last = s;
          run += pr;
          if (pick < 0 && run > target) pick = s;
        }
      }
      if (pick < 0) pick = last;
      if (pick < 0) {
        bad = true;
        pick = 0;
      }
      candidate(pick, false, true);     // the drawn state's candidate into the ring
      const int P2 = 2 * i;
      if (P2 < 64) olo |= uint64_t(pick) << P2; else ohi |= uint64_t(pick) << (P2 - 64);
    } else if (!allowed(ca, cb, si, rest, P.na, P.nb)) {
      bad = true;
    }
    const T p01 = (pick & 1) ? Ps[1] : Ps[0];
    const T p23 = (pick & 1) ? Ps[3] : Ps[2];
    const T pp = (pick & 2) ? p23 : p01;
    int ex;
    prod = tfrexp(prod * (pp / Z), &ex);
    pexp += ex;
    if (dot < T(0)) sgn = -sgn;
    ca += pick & 1;
    cb += pick >> 1;
  }
  if (live) {
    lphi[r] = bad ? -INFINITY : 0.5 * (log(double(prod)) + double(pexp) * 0.69314718055994530942);
    sphi[r] = int8_t(bad ? 0 : sgn);
    if (SAMPLE) {
      SA.out[2 * r] = olo;
      SA.out[2 * r + 1] = ohi;
    }
  }
}

template <typename T, bool SAMPLE>
hipError_t run_tn(const TnParams<T>& P, const uint64_t* m, int64_t R, double* lphi, int8_t* sphi, hipStream_t st,
                  const SampleArgs& SA) {
  if (R <= 0) return hipSuccess;
  const size_t lds = (size_t(P.W) * P.rw + 16) * kTnThreads * sizeof(T);
  if (lds > 64 * 1024 || P.rw > P.chip || P.rw < P.chi) return hipErrorInvalidValue;
  const dim3 grid(unsigned((R + kTnThreads - 1) / kTnThreads));
  if (P.qp == 8)
    hipLaunchKernelGGL((k_psi_tn<T, 8, SAMPLE>), grid, dim3(kTnThreads), lds, st, P, m, R, lphi, sphi, SA);
  else if (P.qp == 16)
    hipLaunchKernelGGL((k_psi_tn<T, 16, SAMPLE>), grid, dim3(kTnThreads), lds, st, P, m, R, lphi, sphi, SA);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

size_t tn_lds_bytes(int W, int rw, int precision) {
  return (size_t(W) * rw + 16) * kTnThreads * (precision == 0 ? 8 : 4);
}

hipError_t launch_psi_tn_f64(const TnParams<double>& P, const uint64_t* m, int64_t R, double* lphi, int8_t* sphi,
                             hipStream_t st) {
  return run_tn<double, false>(P, m, R, lphi, sphi, st, SampleArgs());
}
hipError_t launch_psi_tn_f32(const TnParams<float>& P, const uint64_t* m, int64_t R, double* lphi, int8_t* sphi,
                             hipStream_t st) {
  return run_tn<float, false>(P, m, R, lphi, sphi, st, SampleArgs());
}
hipError_t launch_sample_tn_f64(const TnParams<double>& P, int64_t R, double* lphi, int8_t* sphi, hipStream_t st,
                                const SampleArgs& SA) {
  return run_tn<double, true>(P, nullptr, R, lphi, sphi, st, SA);
}
hipError_t launch_sample_tn_f32(const TnParams<float>& P, int64_t R, double* lphi, int8_t* sphi, hipStream_t st,
                                const SampleArgs& SA) {
  return run_tn<float, true>(P, nullptr, R, lphi, sphi, st, SA);
}

}  // namespace nqs
