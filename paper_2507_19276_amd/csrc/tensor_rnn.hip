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

// hs (nullable, not with SAMPLE): the carried state h_i^{s_i} of every row r <
// ns and site i as hs[(i ns + r) chip + u], u < rw (the adjoint's layout; rows
// past R repeat the last row, units from rw on are left as they are)
template <typename T, int QP, bool SAMPLE>
__global__ __launch_bounds__(kTnThreads) void k_psi_tn(TnParams<T> P, const uint64_t* __restrict__ m, int64_t R,
                                                       double* __restrict__ lphi, int8_t* __restrict__ sphi,
                                                       SampleArgs SA, T* __restrict__ hs, int64_t ns) {
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
    if (!SAMPLE && hs && r < ns)
      for (int u = 0; u < RW; ++u) hs[(size_t(i) * ns + r) * CP + u] = RG(wslot, u);
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
                  const SampleArgs& SA, T* hs = nullptr, int64_t ns = 0) {
  if (R <= 0) return hipSuccess;
  const size_t lds = (size_t(P.W) * P.rw + 16) * kTnThreads * sizeof(T);
  if (lds > 64 * 1024 || P.rw > P.chip || P.rw < P.chi) return hipErrorInvalidValue;
  // the store covers rows up to ns, which the grid must reach
  const int64_t span = hs ? (ns > R ? ns : R) : R;
  const dim3 grid(unsigned((span + kTnThreads - 1) / kTnThreads));
  if (P.qp == 8)
    hipLaunchKernelGGL((k_psi_tn<T, 8, SAMPLE>), grid, dim3(kTnThreads), lds, st, P, m, R, lphi, sphi, SA, hs, ns);
  else if (P.qp == 16)
    hipLaunchKernelGGL((k_psi_tn<T, 16, SAMPLE>), grid, dim3(kTnThreads), lds, st, P, m, R, lphi, sphi, SA, hs, ns);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---- adjoint of the tensor term ------------------------------------------
// For a site i with a tensor term and the rows r < Rpad of the adjoint's sweep
// (carried states Hbuf[(site Rpad + r) chip + u] from the forward's store):
//   pre:  p_j = K_j^T h_(parent j), q^s = U^s (p_1 x .. x p_d), t^s = K0 q^s;
//         t is added to the candidates the sweep's site kernel recomputes;
//   post: dq^s = K0^T dcand^s, dp_j[b] = sum over s, i', a with a_j = b of
//         dq^s[i'] U^s[i'][a] prod_{l != j} p_l[a_l], dcarry_(parent j) += K_j dp_j;
//   cols: dK0 = sum_rows sum_s dcand^s q^s^T, dK_j = sum_rows h_j dp_j^T,
//         dU^s[i'][a] = sum_rows dq^s[i'] prod_j p_j[a_j], per split of rows.
// One thread per row (pre, post) or per (split, gradient entry) (cols); the
// weights come from the forward's kernel layout.  Row scratch p, q, dp, dq is
// [row][3 or 4][kTq].
constexpr int kTq = 16;

template <typename T>
struct TnSite {
  int e0, d, Q, offK0, offKj, offU;
};

template <typename T>
__device__ inline TnSite<T> tn_site(const TnParams<T>& P, int i) {
  TnSite<T> S;
  S.e0 = P.pptr[i];
  S.d = P.pptr[i + 1] - S.e0;
  S.Q = P.site[8 * i + 4];
  S.offK0 = P.site[8 * i + 5];
  S.offKj = P.site[8 * i + 6];
  S.offU = P.site[8 * i + 7];
  return S;
}

// U^s[i'][a_1..a_d] in the kernel layout (last index padded to qp)
template <typename T>
__device__ inline T tn_core(const TnParams<T>& P, const TnSite<T>& S, int s, int ip, int a1, int a2, int a3) {
  if (S.d == 2) return P.prm[S.offU + (size_t(s * S.Q + ip) * S.Q + a1) * P.qp + a2];
  return P.prm[S.offU + (size_t(s * S.Q + ip) * S.Q * S.Q + a1 * S.Q + a2) * P.qp + a3];
}

template <typename T>
__global__ void k_tn_bwd_pre(TnParams<T> P, const int* pidx, int i, int64_t Rpad, const T* Hbuf, T* TT, T* PJ,
                             T* QS) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= Rpad) return;
  const TnSite<T> S = tn_site(P, i);
  const int CP = P.chip, chi = P.chi, Q = S.Q;
  T p[3][kTq], q[4][kTq];
  for (int j = 0; j < S.d; ++j) {
    const T* h = Hbuf + (size_t(pidx[S.e0 + j]) * Rpad + r) * CP;
    for (int a = 0; a < Q; ++a) {
      T acc = T(0);
      for (int v = 0; v < chi; ++v) acc += P.prm[S.offKj + (j * CP + v) * P.qp + a] * h[v];
      p[j][a] = acc;
      PJ[(size_t(r) * 3 + j) * kTq + a] = acc;
    }
  }
  const int Q3 = S.d == 3 ? Q : 1;
  for (int s = 0; s < 4; ++s)
    for (int ip = 0; ip < Q; ++ip) {
      T acc = T(0);
      for (int a1 = 0; a1 < Q; ++a1)
        for (int a2 = 0; a2 < Q; ++a2)
          for (int a3 = 0; a3 < Q3; ++a3) {
            T f = p[0][a1] * p[1][a2];
            if (S.d == 3) f *= p[2][a3];
            acc += tn_core(P, S, s, ip, a1, a2, a3) * f;
          }
      q[s][ip] = acc;
      QS[(size_t(r) * 4 + s) * kTq + ip] = acc;
    }
  for (int s = 0; s < 4; ++s)
    for (int u = 0; u < CP; ++u) {
      T t = T(0);
      if (u < chi)
        for (int ip = 0; ip < Q; ++ip) t += P.prm[S.offK0 + ip * CP + u] * q[s][ip];
      TT[(size_t(r) * 4 + s) * CP + u] = t;
    }
}

template <typename T>
__global__ void k_tn_bwd_post(TnParams<T> P, const int* pidx, int i, int64_t Rpad, const T* Dc, const T* PJ, T* DQ,
                              T* DP, T* dcarry) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= Rpad) return;
  const TnSite<T> S = tn_site(P, i);
  const int CP = P.chip, chi = P.chi, Q = S.Q;
  T p[3][kTq], dq[4][kTq], dp[3][kTq];
  for (int j = 0; j < S.d; ++j)
    for (int a = 0; a < Q; ++a) {
      p[j][a] = PJ[(size_t(r) * 3 + j) * kTq + a];
      dp[j][a] = T(0);
    }
  for (int s = 0; s < 4; ++s)
    for (int ip = 0; ip < Q; ++ip) {
      T acc = T(0);
      for (int u = 0; u < chi; ++u) acc += P.prm[S.offK0 + ip * CP + u] * Dc[(size_t(r) * 4 + s) * CP + u];
      dq[s][ip] = acc;
      DQ[(size_t(r) * 4 + s) * kTq + ip] = acc;
    }
  const int Q3 = S.d == 3 ? Q : 1;
  for (int s = 0; s < 4; ++s)
    for (int ip = 0; ip < Q; ++ip) {
      const T g = dq[s][ip];
      if (g == T(0)) continue;
      for (int a1 = 0; a1 < Q; ++a1)
        for (int a2 = 0; a2 < Q; ++a2)
          for (int a3 = 0; a3 < Q3; ++a3) {
            const T u = tn_core(P, S, s, ip, a1, a2, a3) * g;
            if (S.d == 2) {
              dp[0][a1] += u * p[1][a2];
              dp[1][a2] += u * p[0][a1];
            } else {
              dp[0][a1] += u * p[1][a2] * p[2][a3];
              dp[1][a2] += u * p[0][a1] * p[2][a3];
              dp[2][a3] += u * p[0][a1] * p[1][a2];
            }
          }
    }
  for (int j = 0; j < S.d; ++j) {
    for (int b = 0; b < Q; ++b) DP[(size_t(r) * 3 + j) * kTq + b] = dp[j][b];
    T* dc = dcarry + (size_t(pidx[S.e0 + j]) * Rpad + r) * CP;
    for (int v = 0; v < chi; ++v) {
      T acc = T(0);
      for (int b = 0; b < Q; ++b) acc += P.prm[S.offKj + (j * CP + v) * P.qp + b] * dp[j][b];
      dc[v] += acc;
    }
  }
}

template <typename T>
__global__ void k_tn_bwd_cols(TnParams<T> P, const int* pidx, int i, int64_t Rpad, int rows_per_split, int nsplit,
                              const T* Hbuf, const T* Dc, const T* PJ, const T* QS, const T* DQ, const T* DP,
                              int64_t offTK, int64_t offTU, double* gpart, int64_t n_params) {
  const TnSite<T> S = tn_site(P, i);
  const int CP = P.chip, chi = P.chi, Q = S.Q, d = S.d;
  int nQd = 1;
  for (int k = 0; k < d; ++k) nQd *= Q;
  const int nK = chi * Q, ncol = (d + 1) * nK + 4 * Q * nQd;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(ncol) * nsplit) return;
  const int split = int(t / ncol), col = int(t % ncol);
  const int64_t r0 = int64_t(split) * rows_per_split;
  const int64_t r1 = r0 + rows_per_split < Rpad ? r0 + rows_per_split : Rpad;
  double acc = 0.0;
  int64_t out;
  if (col < nK) {                       // dK0[u][i']
    const int u = col / Q, ip = col % Q;
    for (int64_t r = r0; r < r1; ++r)
      for (int s = 0; s < 4; ++s)
        acc += double(Dc[(size_t(r) * 4 + s) * CP + u]) * double(QS[(size_t(r) * 4 + s) * kTq + ip]);
    out = offTK + col;
  } else if (col < (d + 1) * nK) {      // dK_j[v][b]
    const int c = col - nK, j = c / nK, v = (c / Q) % chi, b = c % Q;
    const T* h = Hbuf + size_t(pidx[S.e0 + j]) * Rpad * CP + v;
    for (int64_t r = r0; r < r1; ++r) acc += double(h[size_t(r) * CP]) * double(DP[(size_t(r) * 3 + j) * kTq + b]);
    out = offTK + (j + 1) * nK + v * Q + b;
  } else {                              // dU^s[i'][a_1..a_d], a_d fastest
    const int c = col - (d + 1) * nK, s = c / (Q * nQd), ip = (c / nQd) % Q, f = c % nQd;
    int a[3] = {0, 0, 0}, rem = f;
    for (int j = d - 1; j >= 0; --j) {
      a[j] = rem % Q;
      rem /= Q;
    }
    for (int64_t r = r0; r < r1; ++r) {
      T prod = DQ[(size_t(r) * 4 + s) * kTq + ip];
      for (int j = 0; j < d; ++j) prod *= PJ[(size_t(r) * 3 + j) * kTq + a[j]];
      acc += double(prod);
    }
    out = offTU + (int64_t(s) * Q + ip) * nQd + f;
  }
  gpart[size_t(split) * n_params + out] = acc;
}

template <typename T>
hipError_t tn_bwd_site(const TnAdj<T>& A, const int* pidx, int i, int stage, int64_t Rpad, const T* Hbuf,
                       const T* Dc, T* dcarry, int rows_per_split, int nsplit, double* gpart, int64_t n_params,
                       hipStream_t st) {
  const unsigned rb = unsigned((Rpad + 63) / 64);
  if (stage == 0) {
    hipLaunchKernelGGL(k_tn_bwd_pre<T>, dim3(rb), dim3(64), 0, st, A.P, pidx, i, Rpad, Hbuf, A.TT, A.PJ, A.QS);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_tn_bwd_post<T>, dim3(rb), dim3(64), 0, st, A.P, pidx, i, Rpad, Dc, A.PJ, A.DQ, A.DP, dcarry);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int Q = A.tq_host[i], d = A.d_host[i];
  int64_t nQd = 1;
  for (int k = 0; k < d; ++k) nQd *= Q;
  const int64_t ncol = int64_t(d + 1) * A.P.chi * Q + 4 * Q * nQd;
  hipLaunchKernelGGL(k_tn_bwd_cols<T>, dim3(unsigned((ncol * nsplit + 255) / 256)), dim3(256), 0, st, A.P, pidx, i,
                     Rpad, rows_per_split, nsplit, Hbuf, Dc, A.PJ, A.QS, A.DQ, A.DP, A.offTK_host[i],
                     A.offTU_host[i], gpart, n_params);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_tn_bwd_site(const TnAdj<double>& A, const int* pidx, int i, int stage, int64_t Rpad,
                              const double* Hbuf, const double* Dc, double* dcarry, int rows_per_split, int nsplit,
                              double* gpart, int64_t n_params, hipStream_t st) {
  return tn_bwd_site<double>(A, pidx, i, stage, Rpad, Hbuf, Dc, dcarry, rows_per_split, nsplit, gpart, n_params, st);
}
hipError_t launch_tn_bwd_site(const TnAdj<float>& A, const int* pidx, int i, int stage, int64_t Rpad,
                              const float* Hbuf, const float* Dc, float* dcarry, int rows_per_split, int nsplit,
                              double* gpart, int64_t n_params, hipStream_t st) {
  return tn_bwd_site<float>(A, pidx, i, stage, Rpad, Hbuf, Dc, dcarry, rows_per_split, nsplit, gpart, n_params, st);
}

size_t tn_lds_bytes(int W, int rw, int precision) {
  return (size_t(W) * rw + 16) * kTnThreads * (precision == 0 ? 8 : 4);
}

hipError_t launch_psi_tn_f64(const TnParams<double>& P, const uint64_t* m, int64_t R, double* lphi, int8_t* sphi,
                             hipStream_t st, double* hs, int64_t ns) {
  return run_tn<double, false>(P, m, R, lphi, sphi, st, SampleArgs(), hs, ns);
}
hipError_t launch_psi_tn_f32(const TnParams<float>& P, const uint64_t* m, int64_t R, double* lphi, int8_t* sphi,
                             hipStream_t st, float* hs, int64_t ns) {
  return run_tn<float, false>(P, m, R, lphi, sphi, st, SampleArgs(), hs, ns);
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
