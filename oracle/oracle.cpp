// FP64 CPU oracle for the semi-stochastic local energy of arXiv:2507.19276.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
// call this file; it exists so that tests, the smoke check and the CPU
// baseline of the benchmark can compare the HIP library against plain,
// slow, obviously correct definitions.  It shares no code, header, table or
// helper with the HIP library.
//
// Build: g++ -O3 -march=x86-64-v3 -fopenmp -ffp-contract=off -shared -fPIC (see build.py;
// the CPU-baseline timing uses -march=native for the host it runs on).
// -ffp-contract=off is essential: Hamiltonian elements are compared bit for
// bit with the GPU, so no multiply-add may be fused behind our back.
//
// What each part follows in the paper:
//   * Hamiltonian, Sec. 2.1 Eq. (2): H = sum h_pq a+_p a_q
//       + 1/4 sum <pq||rs> a+_p a+_q a_s a_r over spin orbitals.
//   * ONV ordering, Sec. 3: x_{2p} = n_{p alpha}, x_{2p+1} = n_{p beta}.
//   * Local energy, Sec. 2.1 Eq. (6); deterministic part Eq. (20), stochastic
//     part Eq. (21), their sum Eq. (22) (Sec. 2.4).
//   * MPS-RNN / BDG-RNN amplitude, Sec. 2.1 Eqs. (9)-(10), Sec. 2.2 Eq. (12)
//     (the BDG-TensorRNN adds the tensor term of Eq. (12) in the Tucker form
//     of Eq. (13) at every site with two or more parents); conditional
//     P_t = h^T eta h; phase from w^T h + c (Sec. 2.1).
//   * Particle-number / S_z masking of the conditionals, Sec. 3 Eqs. (23)-(24).
//   * Correlator factorisation Psi = f Phi with cos-RBM f, Sec. 2.3
//     Eqs. (14)-(15), or the Ising-RBM f of Eq. (16) (the cos-RBM argument plus
//     half the quadratic form of a full N_v x N_v matrix per hidden unit, over
//     all ordered pairs, the diagonal included); reweighted local energy
//     Eq. (18).
//   * Gradient of ln|Psi| used by Eqs. (7) and (19).
//
// Readings of points the paper leaves open (each one listed in the design
// notes of the repository):
//   - spatial chemist integrals (pq|rs) give <PQ|RS> = (pr|qs) for matching
//     spins, zero otherwise;
//   - |n> = prod_{P ascending} (a+_P)^{x_P} |vac>, lowest index leftmost; signs
//     are obtained by applying the operators one at a time to a bit array;
//   - local state of spatial site t is s = n_alpha + 2 n_beta;
//   - one matrix M_ij^{s_i} per (site, parent) edge, indexed by the child's
//     local state; a site without parents has h = v;
//   - the conditional is normalised over the local states that keep the
//     electron counts reachable (exact feasibility mask);
//   - real parameters: phase = sign(w^T h + c) with sign(0) = +1; complex
//     parameters (M, v, w, c complex, eta real and non-negative; Sec. 2.1):
//     P_t = h^dagger eta h, phase of site t = arg(w^T h + c) (no conjugation
//     of w, arg 0 = 0), total phase their sum, reported in [-pi, pi]; the
//     correlator stays real and its sign adds 0 or pi;
//   - the deterministic set is |H_nm| >= eps with H_nm != 0, m != n; the
//     remainder 0 < |H_nm| < eps is sampled with replacement with integer
//     weights q = ceil(|H| 2^(40-e)), eps = f 2^e, f in [0.5,1);
//   - draws use Philox4x32-10 (Salmon et al., SC'11) with key (seed lo, hi) and
//     counter (sample index, draw index, stream lo, stream hi); the 128-bit
//     output U (word 0 least significant) picks r = floor(U Q / 2^128).
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>
#include <map>
#include <algorithm>
#include <omp.h>

namespace {

typedef unsigned __int128 u128;

// --------------------------------------------------------------------------
// integrals over spin orbitals (P = 2p + sigma)
// --------------------------------------------------------------------------
struct Ham {
  int K;
  const double* h;    // K*K
  const double* eri;  // K^4, chemist (pq|rs)
  double ecore;
};

inline int spatial(int P) { return P >> 1; }
inline int spin(int P) { return P & 1; }

double h_so(const Ham& H, int P, int Q) {
  if (spin(P) != spin(Q)) return 0.0;
  return H.h[spatial(P) * H.K + spatial(Q)];
}

// physicist <PQ|RS> = (PR|QS) = (pr|qs) delta(sP,sR) delta(sQ,sS)
double g_so(const Ham& H, int P, int Q, int R, int S) {
  if (spin(P) != spin(R) || spin(Q) != spin(S)) return 0.0;
  const size_t K = H.K;
  const size_t p = spatial(P), q = spatial(Q), r = spatial(R), s = spatial(S);
  return H.eri[((p * K + r) * K + q) * K + s];
}

// antisymmetrised <PQ||RS> = <PQ|RS> - <PQ|SR>
double anti(const Ham& H, int P, int Q, int R, int S) {
  return g_so(H, P, Q, R, S) - g_so(H, P, Q, S, R);
}

// --------------------------------------------------------------------------
// occupation-number vectors as plain bit arrays
// --------------------------------------------------------------------------
struct Det {
  int n;            // number of spin orbitals (2K)
  uint8_t x[128];
};

Det det_from_words(int K, const uint64_t* w) {
  Det d;
  d.n = 2 * K;
  for (int P = 0; P < 128; ++P) d.x[P] = 0;
  for (int P = 0; P < 2 * K; ++P) d.x[P] = (w[P >> 6] >> (P & 63)) & 1u;
  return d;
}

void det_to_words(const Det& d, uint64_t* w) {
  w[0] = w[1] = 0;
  for (int P = 0; P < d.n; ++P)
    if (d.x[P]) w[P >> 6] |= uint64_t(1) << (P & 63);
}

// a_P |d>: 0 if empty, else (-1)^(number of occupied Q < P); updates d.
int annihilate(Det& d, int P) {
  if (!d.x[P]) return 0;
  int c = 0;
  for (int Q = 0; Q < P; ++Q) c += d.x[Q];
  d.x[P] = 0;
  return (c & 1) ? -1 : 1;
}

// a+_P |d>: 0 if occupied, else (-1)^(number of occupied Q < P); updates d.
int create(Det& d, int P) {
  if (d.x[P]) return 0;
  int c = 0;
  for (int Q = 0; Q < P; ++Q) c += d.x[Q];
  d.x[P] = 1;
  return (c & 1) ? -1 : 1;
}

bool count_ok(const Det& d, int K, int na, int nb) {
  int a = 0, b = 0;
  for (int p = 0; p < K; ++p) { a += d.x[2 * p]; b += d.x[2 * p + 1]; }
  for (int P = 2 * K; P < 128; ++P) if (d.x[P]) return false;
  return a == na && b == nb;
}

// --------------------------------------------------------------------------
// Slater-Condon rules
// --------------------------------------------------------------------------

// <n|H|n> = e_core + sum_P h_PP + 1/2 sum_{P,Q occ} <PQ||PQ>
double diag_element(const Ham& H, const Det& n) {
  double d1 = 0.0;
  for (int P = 0; P < n.n; ++P)
    if (n.x[P]) d1 += h_so(H, P, P);
  double d2 = 0.0;
  for (int P = 0; P < n.n; ++P) {
    if (!n.x[P]) continue;
    for (int Q = 0; Q < n.n; ++Q)
      if (n.x[Q]) d2 += anti(H, P, Q, P, Q);
  }
  return H.ecore + d1 + 0.5 * d2;
}

struct Conn {
  uint64_t m[2];
  double H;
};

// single I -> A: |m> = g a+_A a_I |n>, H_mn = g (h_AI + sum_{J occ in n} <AJ||IJ>)
Conn single_exc(const Ham& H, const Det& n, int I, int A) {
  Det d = n;
  int g = annihilate(d, I);
  g *= create(d, A);
  double acc = h_so(H, A, I);
  for (int J = 0; J < n.n; ++J)
    if (n.x[J]) acc += anti(H, A, J, I, J);
  Conn c;
  det_to_words(d, c.m);
  c.H = g * acc;
  return c;
}

// double (I<J) -> (A<B): |m> = g a+_A a+_B a_J a_I |n>, H_mn = g <AB||IJ>
Conn double_exc(const Ham& H, const Det& n, int I, int J, int A, int B) {
  if (I > J) std::swap(I, J);
  if (A > B) std::swap(A, B);
  Det d = n;
  int g = annihilate(d, I);
  g *= annihilate(d, J);
  g *= create(d, B);
  g *= create(d, A);
  Conn c;
  det_to_words(d, c.m);
  c.H = g * anti(H, A, B, I, J);
  return c;
}

// All S_z-conserving singles and doubles of n in the canonical order:
//   alpha singles, beta singles, alpha-alpha doubles, beta-beta doubles,
//   alpha-beta doubles; inside each block the nested loops below (holes
//   outer, particles inner, ascending spatial indices, pairs i<j in
//   lexicographic order).
void connected(const Ham& H, const Det& n, std::vector<Conn>& out) {
  const int K = H.K;
  std::vector<int> oa, va, ob, vb;
  for (int p = 0; p < K; ++p) {
    (n.x[2 * p] ? oa : va).push_back(p);
    (n.x[2 * p + 1] ? ob : vb).push_back(p);
  }
  out.clear();
  for (int i : oa) for (int a : va) out.push_back(single_exc(H, n, 2 * i, 2 * a));
  for (int i : ob) for (int a : vb) out.push_back(single_exc(H, n, 2 * i + 1, 2 * a + 1));
  for (int s = 0; s < 2; ++s) {
    const std::vector<int>& o = s ? ob : oa;
    const std::vector<int>& v = s ? vb : va;
    for (size_t i = 0; i < o.size(); ++i)
      for (size_t j = i + 1; j < o.size(); ++j)
        for (size_t a = 0; a < v.size(); ++a)
          for (size_t b = a + 1; b < v.size(); ++b)
            out.push_back(double_exc(H, n, 2 * o[i] + s, 2 * o[j] + s, 2 * v[a] + s, 2 * v[b] + s));
  }
  for (int i : oa)
    for (int a : va)
      for (int j : ob)
        for (int b : vb)
          out.push_back(double_exc(H, n, 2 * i, 2 * j + 1, 2 * a, 2 * b + 1));
}

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): 10 rounds of the 4x32 Philox S-box, key bumped by
// the Weyl constants between rounds.
// --------------------------------------------------------------------------
void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k[2] = {key_in[0], key_in[1]};
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k[0] += W0; k[1] += W1; }
    const uint64_t p0 = uint64_t(M0) * c[0];
    const uint64_t p1 = uint64_t(M1) * c[2];
    const uint32_t hi0 = uint32_t(p0 >> 32), lo0 = uint32_t(p0);
    const uint32_t hi1 = uint32_t(p1 >> 32), lo1 = uint32_t(p1);
    uint32_t n[4];
    n[0] = hi1 ^ c[1] ^ k[0];
    n[1] = lo1;
    n[2] = hi0 ^ c[3] ^ k[1];
    n[3] = lo0;
    std::memcpy(c, n, sizeof c);
  }
  std::memcpy(out, c, sizeof c);
}

// --------------------------------------------------------------------------
// BDG-RNN / MPS-RNN amplitude and cos-RBM correlator (direct definition)
// --------------------------------------------------------------------------
struct Ansatz {
  int K, chi, na, nb, nh;
  bool ising, tensor;
  std::vector<int> chiq;                    // Tucker rank chi' of each site (0: no tensor term)
  std::vector<size_t> offTK, offTU;         // per site: factor matrices [d+1][chi][chi'], cores [4][chi'^(d+1)]
  const int* pptr;
  const int* pidx;
  const double* prm;
  std::vector<size_t> offM;                 // per edge: [4][chi][chi]
  std::vector<size_t> offV, offEta, offW, offC;
  size_t offB = 0, offWc = 0, offW2 = 0, total = 0;
};

// smallest integer c >= 1 with c^(d+1) >= chi^2, i.e. ceil(chi^(2/(d+1))) (Sec. 2.2)
int tucker_rank(int chi, int d) {
  int c = 1;
  for (;; ++c) {
    double p = 1.0;
    for (int k = 0; k <= d; ++k) p *= c;
    if (p >= double(chi) * chi) return c;
  }
}

size_t ipow(size_t b, int e) {
  size_t r = 1;
  for (int k = 0; k < e; ++k) r *= b;
  return r;
}

// variant: bit 0 = Ising-RBM correlator (with nh > 0), bit 1 = BDG-TensorRNN
Ansatz make_ansatz(int K, int chi, int na, int nb, const int* pptr, const int* pidx,
                   int nh, int variant, const double* prm) {
  Ansatz A;
  A.K = K; A.chi = chi; A.na = na; A.nb = nb; A.nh = nh;
  A.ising = nh > 0 && (variant & 1) != 0;
  A.tensor = (variant & 2) != 0;
  A.pptr = pptr; A.pidx = pidx; A.prm = prm;
  size_t o = 0;
  A.offM.resize(pptr[K]);
  A.offV.resize(K); A.offEta.resize(K); A.offW.resize(K); A.offC.resize(K);
  for (int i = 0; i < K; ++i) {
    for (int e = pptr[i]; e < pptr[i + 1]; ++e) { A.offM[e] = o; o += size_t(4) * chi * chi; }
    A.offV[i] = o; o += size_t(4) * chi;
    A.offEta[i] = o; o += chi;
    A.offW[i] = o; o += chi;
    A.offC[i] = o; o += 1;
  }
  A.offB = o; o += nh;
  A.offWc = o; o += size_t(nh) * 2 * K;
  A.offW2 = o;
  if (A.ising) o += size_t(nh) * 4 * K * K;   // [nh][2K][2K]
  // tensor block (after everything else): per site with d >= 2 parents the
  // factor matrices K^(0) (output mode) and K^(1..d) (one per parent, in
  // ascending parent order), each chi x chi' row-major, shared by the local
  // states; then the cores U^s, s = 0..3, each chi'^(d+1) with index order
  // [i'][a_1]...[a_d] row-major
  A.chiq.assign(K, 0);
  A.offTK.assign(K, 0);
  A.offTU.assign(K, 0);
  for (int i = 0; i < K && A.tensor; ++i) {
    const int d = pptr[i + 1] - pptr[i];
    if (d < 2) continue;
    const int q = tucker_rank(chi, d);
    A.chiq[i] = q;
    A.offTK[i] = o; o += size_t(d + 1) * chi * q;
    A.offTU[i] = o; o += 4 * ipow(q, d + 1);
  }
  A.total = o;
  return A;
}

// feasibility of local state s at site i given counts over sites < i
bool allowed(const Ansatz& A, int i, int a_prev, int b_prev, int s) {
  const int a = a_prev + (s & 1), b = b_prev + (s >> 1);
  const int rest = A.K - 1 - i;
  return a <= A.na && a + rest >= A.na && b <= A.nb && b + rest >= A.nb;
}

struct Trace {  // per-site forward quantities kept for the reverse sweep
  std::vector<double> cand;  // [K][4][chi]
  std::vector<double> p;     // [K][4]
  std::vector<double> Z;     // [K]
  std::vector<uint8_t> ok;   // [K][4]
  std::vector<int> s;        // [K]
};

// Tucker form of the tensor term at site i (Eq. (13)): the parents' states
// projected on their factor matrices, p_j = K^(j)^T h_(parent j) [d][chi'],
// then q^s[i'] = sum_a U^s[i'][a_1..a_d] prod_j p_j[a_j] and
// t^s = K^(0) q^s.  Returns q [4][chi'] and p [d][chi'].
void tensor_forward(const Ansatz& A, int i, const std::vector<double>& carried, std::vector<double>& p,
                    std::vector<double>& q) {
  const int chi = A.chi, qd = A.chiq[i], d = A.pptr[i + 1] - A.pptr[i];
  p.assign(size_t(d) * qd, 0.0);
  for (int j = 0; j < d; ++j) {
    const double* Kj = A.prm + A.offTK[i] + size_t(j + 1) * chi * qd;
    const double* hj = carried.data() + size_t(A.pidx[A.pptr[i] + j]) * chi;
    for (int a = 0; a < qd; ++a) {
      double acc = 0.0;
      for (int v = 0; v < chi; ++v) acc += Kj[size_t(v) * qd + a] * hj[v];
      p[size_t(j) * qd + a] = acc;
    }
  }
  const size_t na = ipow(qd, d);   // multi-indices a = (a_1..a_d), a_d fastest
  q.assign(size_t(4) * qd, 0.0);
  std::vector<int> a(d);
  for (int s = 0; s < 4; ++s)
    for (int ip = 0; ip < qd; ++ip) {
      const double* U = A.prm + A.offTU[i] + (size_t(s) * qd + ip) * na;
      double acc = 0.0;
      for (size_t f = 0; f < na; ++f) {
        size_t r = f;
        double prod = 1.0;
        for (int j = d - 1; j >= 0; --j) {
          a[j] = int(r % qd);
          r /= qd;
        }
        for (int j = 0; j < d; ++j) prod *= p[size_t(j) * qd + a[j]];
        acc += U[f] * prod;
      }
      q[size_t(s) * qd + ip] = acc;
    }
}

// candidates h_i^s = sum_{j in N(i)} M_ij^s h_j [+ K^(0) q^s] + v_i^s for s = 0..3
void site_candidates(const Ansatz& A, int i, const std::vector<double>& carried, double* cand) {
  const int chi = A.chi;
  std::vector<double> p, q;
  const int qd = A.chiq[i];
  if (qd) tensor_forward(A, i, carried, p, q);
  for (int s = 0; s < 4; ++s) {
    for (int u = 0; u < chi; ++u) {
      double acc = 0.0;
      for (int e = A.pptr[i]; e < A.pptr[i + 1]; ++e) {
        const int j = A.pidx[e];
        const double* M = A.prm + A.offM[e] + size_t(s) * chi * chi + size_t(u) * chi;
        const double* hj = carried.data() + size_t(j) * chi;
        for (int k = 0; k < chi; ++k) acc += M[k] * hj[k];
      }
      if (qd) {
        const double* K0 = A.prm + A.offTK[i] + size_t(u) * qd;
        double t = 0.0;
        for (int ip = 0; ip < qd; ++ip) t += K0[ip] * q[size_t(s) * qd + ip];
        acc += t;
      }
      cand[s * chi + u] = acc + A.prm[A.offV[i] + s * chi + u];
    }
  }
}

// log|Phi(n)| and sign Phi(n); returns false for an ONV outside the sector.
// margin (nullable): the smallest relative size of the sign argument over
// the sites, |w_i . h_i + c_i| / (||w_i|| ||h_i|| + |c_i|); a perturbation of
// the states of relative norm rho can flip the sign only where it is < rho.
bool phi_eval(const Ansatz& A, const Det& n, double* logabs, int* sgn, Trace* tr, double* margin = nullptr) {
  const int K = A.K, chi = A.chi;
  std::vector<double> carried(size_t(K) * chi, 0.0);
  std::vector<double> cand(4 * chi);
  if (tr) {
    tr->cand.assign(size_t(K) * 4 * chi, 0.0);
    tr->p.assign(size_t(K) * 4, 0.0);
    tr->Z.assign(K, 0.0);
    tr->ok.assign(size_t(K) * 4, 0);
    tr->s.assign(K, 0);
  }
  double la = 0.0;
  int sg = 1;
  int a_prev = 0, b_prev = 0;
  for (int i = 0; i < K; ++i) {
    const int si = n.x[2 * i] + 2 * n.x[2 * i + 1];
    site_candidates(A, i, carried, cand.data());
    double p[4], Z = 0.0;
    bool ok[4];
    for (int s = 0; s < 4; ++s) {
      double acc = 0.0;
      for (int u = 0; u < chi; ++u) acc += A.prm[A.offEta[i] + u] * cand[s * chi + u] * cand[s * chi + u];
      p[s] = acc;
      ok[s] = allowed(A, i, a_prev, b_prev, s);
      if (ok[s]) Z += p[s];
    }
    if (!ok[si]) { *logabs = -std::numeric_limits<double>::infinity(); *sgn = 0; return false; }
    la += 0.5 * (std::log(p[si]) - std::log(Z));
    double t = A.prm[A.offC[i]];
    for (int u = 0; u < chi; ++u) t += A.prm[A.offW[i] + u] * cand[si * chi + u];
    if (t < 0) sg = -sg;
    if (margin) {
      double ww = 0.0, hh = 0.0;
      for (int u = 0; u < chi; ++u) {
        ww += A.prm[A.offW[i] + u] * A.prm[A.offW[i] + u];
        hh += cand[si * chi + u] * cand[si * chi + u];
      }
      const double mu = std::fabs(t) / (std::sqrt(ww) * std::sqrt(hh) + std::fabs(A.prm[A.offC[i]]));
      if (i == 0 || mu < *margin) *margin = mu;
    }
    for (int u = 0; u < chi; ++u) carried[size_t(i) * chi + u] = cand[si * chi + u];
    if (tr) {
      std::copy(cand.begin(), cand.end(), tr->cand.begin() + size_t(i) * 4 * chi);
      for (int s = 0; s < 4; ++s) { tr->p[i * 4 + s] = p[s]; tr->ok[i * 4 + s] = ok[s]; }
      tr->Z[i] = Z;
      tr->s[i] = si;
    }
    a_prev += si & 1;
    b_prev += si >> 1;
  }
  *logabs = la;
  *sgn = sg;
  return true;
}

// cos-RBM: theta_k = b_k + sum_P W_kP x_P; Ising-RBM adds
// (1/2) sum_{P,Q} W2_kPQ x_P x_Q; f = prod_k cos(theta_k)
double corr_theta(const Ansatz& A, const Det& n, int k) {
  const int nv = 2 * A.K;
  double th = A.prm[A.offB + k];
  for (int P = 0; P < nv; ++P)
    if (n.x[P]) th += A.prm[A.offWc + size_t(k) * nv + P];
  if (A.ising) {
    // x_P x_Q is nonzero only for occupied P and Q
    double q = 0.0;
    for (int P = 0; P < nv; ++P) {
      if (!n.x[P]) continue;
      for (int Q = 0; Q < nv; ++Q)
        if (n.x[Q]) q += A.prm[A.offW2 + (size_t(k) * nv + P) * nv + Q];
    }
    th += 0.5 * q;
  }
  return th;
}

// margin (nullable): min_k |cos theta_k| / (1 + |theta_k|), the distance of
// the correlator from a sign change relative to the size of its argument;
// sens (nullable): sum_k (1 + |theta_k|) / |cos theta_k|, so that relative
// errors of size u (1 + |theta_k|) in each cos theta_k move log|f| by at most
// u sens to first order
void corr_eval(const Ansatz& A, const Det& n, double* logabs, int* sgn, double* margin = nullptr,
               double* sens = nullptr) {
  double la = 0.0;
  int sg = 1;
  for (int k = 0; k < A.nh; ++k) {
    const double th = corr_theta(A, n, k);
    const double c = std::cos(th);
    la += std::log(std::fabs(c));
    if (c < 0) sg = -sg;
    if (margin) {
      const double mu = std::fabs(c) / (1.0 + std::fabs(th));
      if (k == 0 || mu < *margin) *margin = mu;
    }
    if (sens) *sens = (k == 0 ? 0.0 : *sens) + (1.0 + std::fabs(th)) / std::fabs(c);
  }
  *logabs = la;
  *sgn = sg;
}

struct Amp {
  double lphi, lf;
  int sphi, sf;
  double phase;   // phase of Phi (complex parameters); 0 for real parameters
  bool valid;
  double mphi = HUGE_VAL, mf = HUGE_VAL;   // sign margins of Phi and of f (real parameters)
  double sens = 0.0;                        // log sensitivity of f (corr_eval)
};

Amp amp_eval(const Ansatz& A, const Det& n) {
  Amp r;
  r.phase = 0.0;
  r.valid = phi_eval(A, n, &r.lphi, &r.sphi, nullptr, &r.mphi);
  r.lf = 0.0; r.sf = 1;
  if (A.nh) corr_eval(A, n, &r.lf, &r.sf, &r.mf, &r.sens);
  return r;
}

// --------------------------------------------------------------------------
// reverse sweep: g * d ln|Psi(n)| / d theta accumulated into grad
// --------------------------------------------------------------------------

// reverse of the tensor term at site i, given dc = d/d h_i^s [4][chi]:
// dK0 = sum_s dc^s q^s^T, dq^s = K0^T dc^s, dU^s[i'][a] = dq^s[i'] prod_j p_j[a_j],
// dp_j[b] = sum_{s,i',a: a_j = b} dq^s[i'] U^s[i'][a] prod_{l != j} p_l[a_l],
// dK^(j) = h_j dp_j^T, d h_j += K^(j) dp_j
void tensor_reverse(const Ansatz& A, int i, const std::vector<double>& carried, const double* dc, double* grad,
                    std::vector<double>& dcarry) {
  const int chi = A.chi, qd = A.chiq[i], d = A.pptr[i + 1] - A.pptr[i];
  std::vector<double> p, q;
  tensor_forward(A, i, carried, p, q);
  const double* K0 = A.prm + A.offTK[i];
  double* dK0 = grad + A.offTK[i];
  std::vector<double> dq(size_t(4) * qd, 0.0);
  for (int s = 0; s < 4; ++s)
    for (int u = 0; u < chi; ++u)
      for (int ip = 0; ip < qd; ++ip) {
        dK0[size_t(u) * qd + ip] += dc[s * chi + u] * q[size_t(s) * qd + ip];
        dq[size_t(s) * qd + ip] += K0[size_t(u) * qd + ip] * dc[s * chi + u];
      }
  const size_t na = ipow(qd, d);
  std::vector<double> dp(size_t(d) * qd, 0.0);
  std::vector<int> a(d);
  for (int s = 0; s < 4; ++s)
    for (int ip = 0; ip < qd; ++ip) {
      const double* U = A.prm + A.offTU[i] + (size_t(s) * qd + ip) * na;
      double* dU = grad + A.offTU[i] + (size_t(s) * qd + ip) * na;
      const double g = dq[size_t(s) * qd + ip];
      for (size_t f = 0; f < na; ++f) {
        size_t r = f;
        for (int j = d - 1; j >= 0; --j) {
          a[j] = int(r % qd);
          r /= qd;
        }
        double prod = 1.0;
        for (int j = 0; j < d; ++j) prod *= p[size_t(j) * qd + a[j]];
        dU[f] += g * prod;
        for (int j = 0; j < d; ++j) {
          double other = 1.0;
          for (int l = 0; l < d; ++l)
            if (l != j) other *= p[size_t(l) * qd + a[l]];
          dp[size_t(j) * qd + a[j]] += g * U[f] * other;
        }
      }
    }
  for (int j = 0; j < d; ++j) {
    const int par = A.pidx[A.pptr[i] + j];
    const double* Kj = A.prm + A.offTK[i] + size_t(j + 1) * chi * qd;
    double* dKj = grad + A.offTK[i] + size_t(j + 1) * chi * qd;
    const double* hj = carried.data() + size_t(par) * chi;
    for (int v = 0; v < chi; ++v)
      for (int b = 0; b < qd; ++b) {
        dKj[size_t(v) * qd + b] += hj[v] * dp[size_t(j) * qd + b];
        dcarry[size_t(par) * chi + v] += Kj[size_t(v) * qd + b] * dp[size_t(j) * qd + b];
      }
  }
}
void grad_accumulate(const Ansatz& A, const Det& n, double g, double* grad) {
  const int K = A.K, chi = A.chi;
  Trace tr;
  double la;
  int sg;
  if (!phi_eval(A, n, &la, &sg, &tr)) return;
  std::vector<double> carried(size_t(K) * chi);
  for (int i = 0; i < K; ++i)
    for (int u = 0; u < chi; ++u)
      carried[size_t(i) * chi + u] = tr.cand[(size_t(i) * 4 + tr.s[i]) * chi + u];
  std::vector<double> dcarry(size_t(K) * chi, 0.0);
  std::vector<double> dcand(4 * chi);
  for (int i = K - 1; i >= 0; --i) {
    const int si = tr.s[i];
    const double psi_ = tr.p[i * 4 + si], Z = tr.Z[i];
    const double* eta = A.prm + A.offEta[i];
    const double* cand = tr.cand.data() + size_t(i) * 4 * chi;
    for (int s = 0; s < 4; ++s)
      for (int u = 0; u < chi; ++u) {
        double d = 0.0;
        if (tr.ok[i * 4 + s]) {
          if (s == si) d += g * eta[u] * cand[s * chi + u] / psi_;
          d -= g * eta[u] * cand[s * chi + u] / Z;
        }
        if (s == si) d += dcarry[size_t(i) * chi + u];
        dcand[s * chi + u] = d;
      }
    for (int u = 0; u < chi; ++u) {
      double d = 0.5 * cand[si * chi + u] * cand[si * chi + u] / psi_;
      for (int s = 0; s < 4; ++s)
        if (tr.ok[i * 4 + s]) d -= 0.5 * cand[s * chi + u] * cand[s * chi + u] / Z;
      grad[A.offEta[i] + u] += g * d;
    }
    for (int s = 0; s < 4; ++s)
      for (int u = 0; u < chi; ++u) grad[A.offV[i] + s * chi + u] += dcand[s * chi + u];
    for (int e = A.pptr[i]; e < A.pptr[i + 1]; ++e) {
      const int j = A.pidx[e];
      const double* hj = carried.data() + size_t(j) * chi;
      for (int s = 0; s < 4; ++s) {
        const double* M = A.prm + A.offM[e] + size_t(s) * chi * chi;
        double* dM = grad + A.offM[e] + size_t(s) * chi * chi;
        for (int u = 0; u < chi; ++u) {
          const double du = dcand[s * chi + u];
          for (int k = 0; k < chi; ++k) {
            dM[u * chi + k] += du * hj[k];
            dcarry[size_t(j) * chi + k] += M[u * chi + k] * du;
          }
        }
      }
    }
    if (A.chiq[i]) tensor_reverse(A, i, carried, dcand.data(), grad, dcarry);
  }
  if (A.nh) {
    const int nv = 2 * K;
    for (int k = 0; k < A.nh; ++k) {
      const double dth = -g * std::tan(corr_theta(A, n, k));
      grad[A.offB + k] += dth;
      for (int P = 0; P < nv; ++P)
        if (n.x[P]) grad[A.offWc + size_t(k) * nv + P] += dth;
      if (A.ising)
        for (int P = 0; P < nv; ++P) {
          if (!n.x[P]) continue;
          for (int Q = 0; Q < nv; ++Q)
            if (n.x[Q]) grad[A.offW2 + (size_t(k) * nv + P) * nv + Q] += 0.5 * dth;
        }
    }
  }
}

// --------------------------------------------------------------------------
// complex parameters (Sec. 2.1: the MPS-RNN over C^chi).  M, v, w, c are
// complex and stored as (re, im) pairs; eta stays real.  Per site
// h^s = sum_j M_ij^s h_j + v^s, P^s = sum_u eta_u |h^s_u|^2 (normalised over
// the allowed states as in the real case), phase_i = arg(w_i^T h_i^{s_i} + c_i).
// Packed layout per site: M (per parent, [4][chi][chi] pairs), v ([4][chi]
// pairs), eta (chi reals), w (chi pairs), c (one pair); then the real
// correlator block as in the real layout.
// --------------------------------------------------------------------------
typedef std::complex<double> cplx;

struct CxAnsatz {
  int K, chi, na, nb;
  const int* pptr;
  const int* pidx;
  const double* prm;
  std::vector<size_t> offM, offV, offEta, offW, offC;   // offsets in doubles
  Ansatz corr;                                          // the correlator part (real)
  size_t total = 0;
  cplx at(size_t off) const { return cplx(prm[off], prm[off + 1]); }
};

CxAnsatz make_cx_ansatz(int K, int chi, int na, int nb, const int* pptr, const int* pidx, int nh, bool ising,
                        const double* prm) {
  CxAnsatz A;
  A.K = K; A.chi = chi; A.na = na; A.nb = nb;
  A.pptr = pptr; A.pidx = pidx; A.prm = prm;
  size_t o = 0;
  A.offM.resize(pptr[K]);
  A.offV.resize(K); A.offEta.resize(K); A.offW.resize(K); A.offC.resize(K);
  for (int i = 0; i < K; ++i) {
    for (int e = pptr[i]; e < pptr[i + 1]; ++e) { A.offM[e] = o; o += size_t(8) * chi * chi; }
    A.offV[i] = o; o += size_t(8) * chi;
    A.offEta[i] = o; o += chi;
    A.offW[i] = o; o += size_t(2) * chi;
    A.offC[i] = o; o += 2;
  }
  Ansatz& C = A.corr;
  C.K = K; C.chi = chi; C.na = na; C.nb = nb; C.nh = nh;
  C.ising = nh > 0 && ising;
  C.tensor = false;
  C.pptr = pptr; C.pidx = pidx; C.prm = prm;
  C.offB = o; o += nh;
  C.offWc = o; o += size_t(nh) * 2 * K;
  C.offW2 = o;
  if (C.ising) o += size_t(nh) * 4 * K * K;
  A.total = o;
  C.total = o;
  return A;
}

bool cx_allowed(const CxAnsatz& A, int i, int a_prev, int b_prev, int s) {
  const int a = a_prev + (s & 1), b = b_prev + (s >> 1);
  const int rest = A.K - 1 - i;
  return a <= A.na && a + rest >= A.na && b <= A.nb && b + rest >= A.nb;
}

// h_i^s[u] = sum_{j in N(i)} sum_k M_ij^s[u][k] h_j[k] + v_i^s[u]
void cx_site_candidates(const CxAnsatz& A, int i, const std::vector<cplx>& carried, cplx* cand) {
  const int chi = A.chi;
  for (int s = 0; s < 4; ++s)
    for (int u = 0; u < chi; ++u) {
      cplx acc = 0.0;
      for (int e = A.pptr[i]; e < A.pptr[i + 1]; ++e) {
        const int j = A.pidx[e];
        for (int k = 0; k < chi; ++k)
          acc += A.at(A.offM[e] + 2 * ((size_t(s) * chi + u) * chi + k)) * carried[size_t(j) * chi + k];
      }
      cand[s * chi + u] = acc + A.at(A.offV[i] + 2 * (size_t(s) * chi + u));
    }
}

struct CxTrace {
  std::vector<cplx> cand;    // [K][4][chi]
  std::vector<double> p;     // [K][4]
  std::vector<double> Z;     // [K]
  std::vector<uint8_t> ok;   // [K][4]
  std::vector<int> s;        // [K]
  std::vector<cplx> z;       // [K]: w^T h + c
};

// log|Phi(n)| and the phase sum_i arg(w_i^T h_i + c_i) (not wrapped)
bool cx_phi_eval(const CxAnsatz& A, const Det& n, double* logabs, double* phase, CxTrace* tr) {
  const int K = A.K, chi = A.chi;
  std::vector<cplx> carried(size_t(K) * chi, 0.0), cand(4 * chi);
  if (tr) {
    tr->cand.assign(size_t(K) * 4 * chi, 0.0);
    tr->p.assign(size_t(K) * 4, 0.0);
    tr->Z.assign(K, 0.0);
    tr->ok.assign(size_t(K) * 4, 0);
    tr->s.assign(K, 0);
    tr->z.assign(K, 0.0);
  }
  double la = 0.0, ph = 0.0;
  int a_prev = 0, b_prev = 0;
  for (int i = 0; i < K; ++i) {
    const int si = n.x[2 * i] + 2 * n.x[2 * i + 1];
    cx_site_candidates(A, i, carried, cand.data());
    double p[4], Z = 0.0;
    bool ok[4];
    for (int s = 0; s < 4; ++s) {
      double acc = 0.0;
      for (int u = 0; u < chi; ++u) acc += A.prm[A.offEta[i] + u] * std::norm(cand[s * chi + u]);
      p[s] = acc;
      ok[s] = cx_allowed(A, i, a_prev, b_prev, s);
      if (ok[s]) Z += p[s];
    }
    if (!ok[si]) { *logabs = -std::numeric_limits<double>::infinity(); *phase = 0.0; return false; }
    la += 0.5 * (std::log(p[si]) - std::log(Z));
    cplx z = A.at(A.offC[i]);
    for (int u = 0; u < chi; ++u) z += A.at(A.offW[i] + 2 * u) * cand[si * chi + u];
    ph += std::arg(z);
    for (int u = 0; u < chi; ++u) carried[size_t(i) * chi + u] = cand[si * chi + u];
    if (tr) {
      std::copy(cand.begin(), cand.end(), tr->cand.begin() + size_t(i) * 4 * chi);
      for (int s = 0; s < 4; ++s) { tr->p[i * 4 + s] = p[s]; tr->ok[i * 4 + s] = ok[s]; }
      tr->Z[i] = Z;
      tr->s[i] = si;
      tr->z[i] = z;
    }
    a_prev += si & 1;
    b_prev += si >> 1;
  }
  *logabs = la;
  *phase = ph;
  return true;
}

double wrap_phase(double x) { return std::remainder(x, 2.0 * M_PI); }

Amp cx_amp_eval(const CxAnsatz& A, const Det& n) {
  Amp r;
  r.sphi = 1;
  r.valid = cx_phi_eval(A, n, &r.lphi, &r.phase, nullptr);
  r.lf = 0.0; r.sf = 1;
  if (A.corr.nh) corr_eval(A.corr, n, &r.lf, &r.sf);
  return r;
}

// Reverse sweep of ga ln|Psi(n)| + gp phase(n) over the packed parameters.
// A real function L of a complex quantity y has the gradient pair
// G_y = dL/dRe y + i dL/dIm y; through y = a x (a fixed) it pulls back as
// G_x = conj(a) G_y and G_a = conj(x) G_y.  From ln P: G_h = ga eta h
// ([s = s_i]/P^{s_i} - [s allowed]/Z); from arg z: G_z = gp i z / |z|^2.
void cx_grad_accumulate(const CxAnsatz& A, const Det& n, double ga, double gp, double* grad) {
  const int K = A.K, chi = A.chi;
  CxTrace tr;
  double la, ph;
  if (!cx_phi_eval(A, n, &la, &ph, &tr)) return;
  auto add = [&](size_t off, cplx g) { grad[off] += g.real(); grad[off + 1] += g.imag(); };
  std::vector<cplx> carried(size_t(K) * chi);
  for (int i = 0; i < K; ++i)
    for (int u = 0; u < chi; ++u) carried[size_t(i) * chi + u] = tr.cand[(size_t(i) * 4 + tr.s[i]) * chi + u];
  std::vector<cplx> dcarry(size_t(K) * chi, 0.0), dcand(4 * chi);
  for (int i = K - 1; i >= 0; --i) {
    const int si = tr.s[i];
    const double psi_ = tr.p[i * 4 + si], Z = tr.Z[i];
    const double* eta = A.prm + A.offEta[i];
    const cplx* cand = tr.cand.data() + size_t(i) * 4 * chi;
    for (int s = 0; s < 4; ++s)
      for (int u = 0; u < chi; ++u) {
        cplx d = 0.0;
        if (tr.ok[i * 4 + s]) {
          if (s == si) d += ga * eta[u] * cand[s * chi + u] / psi_;
          d -= ga * eta[u] * cand[s * chi + u] / Z;
        }
        if (s == si) d += dcarry[size_t(i) * chi + u];
        dcand[s * chi + u] = d;
      }
    const cplx z = tr.z[i];
    const double z2 = std::norm(z);
    if (z2 > 0.0) {
      const cplx Gz = gp * cplx(-z.imag(), z.real()) / z2;
      add(A.offC[i], Gz);
      for (int u = 0; u < chi; ++u) {
        add(A.offW[i] + 2 * u, std::conj(cand[si * chi + u]) * Gz);
        dcand[si * chi + u] += std::conj(A.at(A.offW[i] + 2 * u)) * Gz;
      }
    }
    for (int u = 0; u < chi; ++u) {
      double d = 0.5 * std::norm(cand[si * chi + u]) / psi_;
      for (int s = 0; s < 4; ++s)
        if (tr.ok[i * 4 + s]) d -= 0.5 * std::norm(cand[s * chi + u]) / Z;
      grad[A.offEta[i] + u] += ga * d;
    }
    for (int s = 0; s < 4; ++s)
      for (int u = 0; u < chi; ++u) add(A.offV[i] + 2 * (size_t(s) * chi + u), dcand[s * chi + u]);
    for (int e = A.pptr[i]; e < A.pptr[i + 1]; ++e) {
      const int j = A.pidx[e];
      for (int s = 0; s < 4; ++s)
        for (int u = 0; u < chi; ++u) {
          const cplx du = dcand[s * chi + u];
          for (int k = 0; k < chi; ++k) {
            const size_t off = A.offM[e] + 2 * ((size_t(s) * chi + u) * chi + k);
            add(off, du * std::conj(carried[size_t(j) * chi + k]));
            dcarry[size_t(j) * chi + k] += std::conj(A.at(off)) * du;
          }
        }
    }
  }
  const Ansatz& C = A.corr;
  if (C.nh) {
    const int nv = 2 * K;
    for (int k = 0; k < C.nh; ++k) {
      const double dth = -ga * std::tan(corr_theta(C, n, k));
      grad[C.offB + k] += dth;
      for (int P = 0; P < nv; ++P)
        if (n.x[P]) grad[C.offWc + size_t(k) * nv + P] += dth;
      if (C.ising)
        for (int P = 0; P < nv; ++P) {
          if (!n.x[P]) continue;
          for (int Q = 0; Q < nv; ++Q)
            if (n.x[Q]) grad[C.offW2 + (size_t(k) * nv + P) * nv + Q] += 0.5 * dth;
        }
    }
  }
}

// exact autoregressive draws from Phi^2 with complex parameters (the same
// selection rule as the real sampler; P^s from |h^s|^2)
int cx_sample(int K, int chi, int na, int nb, const int* pptr, const int* pidx, const double* prm,
              const double* u, int64_t N, uint64_t* out) {
  CxAnsatz A = make_cx_ansatz(K, chi, na, nb, pptr, pidx, 0, false, prm);
  for (int64_t t = 0; t < N; ++t) {
    Det d;
    d.n = 2 * K;
    std::memset(d.x, 0, sizeof d.x);
    std::vector<cplx> carried(size_t(K) * chi, 0.0), cand(4 * chi);
    int a_prev = 0, b_prev = 0;
    for (int i = 0; i < K; ++i) {
      cx_site_candidates(A, i, carried, cand.data());
      double p[4], Z = 0.0;
      for (int s = 0; s < 4; ++s) {
        double acc = 0.0;
        for (int uu = 0; uu < chi; ++uu) acc += prm[A.offEta[i] + uu] * std::norm(cand[s * chi + uu]);
        p[s] = cx_allowed(A, i, a_prev, b_prev, s) ? acc : 0.0;
        Z += p[s];
      }
      const double target = u[t * K + i] * Z;
      double run = 0.0;
      int pick = -1, last = -1;
      for (int s = 0; s < 4; ++s) {
        if (p[s] <= 0.0) continue;
        last = s;
        run += p[s];
        if (run > target) { pick = s; break; }
      }
      if (pick < 0) pick = last;
      d.x[2 * i] = pick & 1;
      d.x[2 * i + 1] = pick >> 1;
      for (int uu = 0; uu < chi; ++uu) carried[size_t(i) * chi + uu] = cand[pick * chi + uu];
      a_prev += pick & 1;
      b_prev += pick >> 1;
    }
    det_to_words(d, out + 2 * t);
  }
  return 0;
}

// --------------------------------------------------------------------------
// semi-stochastic local energy for one sample
// --------------------------------------------------------------------------
struct ElocOut {
  double eloc, etnum, logabs, fsq;
  double sabs;                       // |H_nn| + sum over the summed terms of |coefficient| |Psi(m)/Psi(n)|
  double ebound[4];                  // per bound column: sum of |term| x term_weight over the terms
  double mphi, mf;                   // sign margins of Phi(n) and f(n)
  double eloc_im, etnum_im, phase;   // complex parameters: imaginary parts, phase of Psi(n)
  int sign;
  int64_t n_det, n_rem, n_uniq;
  uint64_t Q;
};

// integer proposal weight of a remainder element (|H| < eps, H != 0)
uint64_t proposal_weight(double absH, double eps) {
  int e;
  std::frexp(eps, &e);                      // eps = f 2^e, f in [0.5, 1)
  return uint64_t(std::ceil(std::ldexp(absH, 40 - e)));
}

// floor(U * Q / 2^128) for a 128-bit U given as four 32-bit words (LS first)
uint64_t scaled_draw(const uint32_t U[4], uint64_t Q) {
  const uint64_t ulo = uint64_t(U[0]) | (uint64_t(U[1]) << 32);
  const uint64_t uhi = uint64_t(U[2]) | (uint64_t(U[3]) << 32);
  const u128 t = u128(uhi) * Q + ((u128(ulo) * Q) >> 64);
  return uint64_t(t >> 64);
}

// Error model of the reduced-precision paths (one column per precision):
// the bond contractions carry relative state errors up to kappa and move
// log|Phi| of any row by at most L; the correlator's cos theta is evaluated
// with relative error u_f (1 + |theta|), which moves log|f| by at most
// u_f sens and can flip its sign only where its margin is below
// kappa_f = 8 u_f.
struct BoundCol {
  double L, kappa;
};

// How far a term x of E_loc(n) may move under that model, as a multiple of
// |x|: its ratio is within e^{+-delta}, delta = 2 L + u_f (sens(m) + sens(n))
// (both amplitudes' log errors), giving e^delta - 1; where a sign can flip (a
// Phi margin of the row or of the sample below kappa, or the row's correlator
// margin below kappa_f) the term may also change sign, adding 2, and a
// correlator margin below kappa_f may grow |f(m)| by up to 1 + kappa_f /
// margin, adding 2 kappa_f / margin.
double term_weight(const Amp& an, const Amp& am, const BoundCol& b, double u_f) {
  const double kf = 8.0 * u_f;
  const double delta = 2.0 * b.L + u_f * (am.sens + an.sens);
  double w = std::expm1(delta);
  if (am.mphi < b.kappa || an.mphi < b.kappa || am.mf < kf) w += 2.0;
  if (am.mf < kf) w += 2.0 * kf / am.mf;
  return w;
}

template <class AmpFn>
ElocOut eloc_one(const Ham& H, const Det& n, int64_t sample_idx, double eps, int n_eps,
                 uint64_t seed, uint64_t stream, AmpFn amp,
                 std::vector<int64_t>* det_ranks, std::vector<int64_t>* draw_ranks,
                 const BoundCol* cols = nullptr, int n_cols = 0, double u_f = 0.0) {
  ElocOut o{};
  std::vector<Conn> conns;
  connected(H, n, conns);
  const double Hnn = diag_element(H, n);
  const Amp an = amp(n);
  o.mphi = an.mphi;
  o.mf = an.mf;
  o.logabs = an.lphi + an.lf;
  o.sign = an.sphi * an.sf;
  o.fsq = std::exp(2.0 * an.lf);
  o.phase = wrap_phase(an.phase + (o.sign < 0 ? M_PI : 0.0));
  // Psi(m)/Psi(n) = s e^{ln|Psi(m)| - ln|Psi(n)|} e^{i (phase_m - phase_n)} with the
  // real signs s of Phi and f; for real parameters the phase factor is exactly 1
  double ed = 0.0, ed_t = 0.0;     // E^d and its reweighted numerator part
  double ed_i = 0.0, ed_ti = 0.0;  // their imaginary parts
  std::vector<int64_t> rem;       // ranks of the remainder, in canonical order
  std::vector<uint64_t> q;
  for (size_t r = 0; r < conns.size(); ++r) {
    const double h = conns[r].H;
    if (h == 0.0) continue;
    if (std::fabs(h) >= eps) {
      Det m = det_from_words(H.K, conns[r].m);
      const Amp am = amp(m);
      const int s = an.sphi * an.sf * am.sphi * am.sf;
      const double x = h * s * std::exp(am.lphi + am.lf - an.lphi - an.lf);
      const double xt = h * s * std::exp(an.lf + am.lf + am.lphi - an.lphi);
      const double cr = std::cos(am.phase - an.phase), ci = std::sin(am.phase - an.phase);
      ed += x * cr;
      ed_t += xt * cr;
      ed_i += x * ci;
      ed_ti += xt * ci;
      o.sabs += std::fabs(x);
      for (int q = 0; q < n_cols; ++q) o.ebound[q] += std::fabs(x) * term_weight(an, am, cols[q], u_f);
      ++o.n_det;
      if (det_ranks) det_ranks->push_back(int64_t(r));
    } else {
      rem.push_back(int64_t(r));
      q.push_back(proposal_weight(std::fabs(h), eps));
    }
  }
  o.n_rem = int64_t(rem.size());
  uint64_t Q = 0;
  for (uint64_t x : q) Q += x;
  o.Q = Q;
  double es = 0.0, es_t = 0.0, es_i = 0.0, es_ti = 0.0;
  if (n_eps > 0 && Q > 0) {
    std::vector<int64_t> picked;
    for (int k = 0; k < n_eps; ++k) {
      const uint32_t ctr[4] = {uint32_t(uint64_t(sample_idx)), uint32_t(k), uint32_t(stream),
                               uint32_t(stream >> 32)};
      const uint32_t key[2] = {uint32_t(seed), uint32_t(seed >> 32)};
      uint32_t U[4];
      philox4x32_10(ctr, key, U);
      const uint64_t r = scaled_draw(U, Q);
      uint64_t run = 0;
      size_t t = 0;
      for (; t < q.size(); ++t) {
        run += q[t];
        if (run > r) break;
      }
      const int64_t rank = rem[t];
      picked.push_back(rank);
      if (draw_ranks) draw_ranks->push_back(rank);
      const double h = conns[rank].H;
      const double w = h * (double(Q) / (double(q[t]) * double(n_eps)));
      Det m = det_from_words(H.K, conns[rank].m);
      const Amp am = amp(m);
      const int s = an.sphi * an.sf * am.sphi * am.sf;
      const double x = w * s * std::exp(am.lphi + am.lf - an.lphi - an.lf);
      const double xt = w * s * std::exp(an.lf + am.lf + am.lphi - an.lphi);
      const double cr = std::cos(am.phase - an.phase), ci = std::sin(am.phase - an.phase);
      es += x * cr;
      es_t += xt * cr;
      es_i += x * ci;
      es_ti += xt * ci;
      o.sabs += std::fabs(x);
      for (int q = 0; q < n_cols; ++q) o.ebound[q] += std::fabs(x) * term_weight(an, am, cols[q], u_f);
    }
    std::sort(picked.begin(), picked.end());
    o.n_uniq = int64_t(std::unique(picked.begin(), picked.end()) - picked.begin());
  }
  o.eloc = Hnn + ed + es;
  o.sabs += std::fabs(Hnn);
  o.etnum = o.fsq * Hnn + ed_t + es_t;
  o.eloc_im = ed_i + es_i;
  o.etnum_im = ed_ti + es_ti;
  if (!an.valid || !std::isfinite(o.logabs)) { o.eloc = o.etnum = o.eloc_im = o.etnum_im = std::nan(""); }
  return o;
}

int nthreads_or_default(int nt) { return nt > 0 ? nt : omp_get_max_threads(); }

}  // namespace

// ==========================================================================
// C entry points for the Python test wrapper
// ==========================================================================
extern "C" {

int or_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  philox4x32_10(ctr, key, out);
  return 0;
}

uint64_t or_proposal_weight(double absH, double eps) { return proposal_weight(absH, eps); }

uint64_t or_scaled_draw(const uint32_t* U, uint64_t Q) { return scaled_draw(U, Q); }

// diagonal elements for N samples; returns -1 for a sample outside the sector
int or_hdiag(int K, int na, int nb, const double* h, const double* eri, double ecore,
             const uint64_t* samples, int64_t N, double* out) {
  Ham H{K, h, eri, ecore};
  for (int64_t i = 0; i < N; ++i) {
    Det d = det_from_words(K, samples + 2 * i);
    if (!count_ok(d, K, na, nb)) return -1;
    out[i] = diag_element(H, d);
  }
  return 0;
}

// connected determinants of one sample in canonical order; returns their
// number (written only up to cap) or -1 for an invalid sample
int64_t or_connected(int K, int na, int nb, const double* h, const double* eri, double ecore,
                     const uint64_t* sample, uint64_t* m_out, double* h_out, int64_t cap) {
  Ham H{K, h, eri, ecore};
  Det d = det_from_words(K, sample);
  if (!count_ok(d, K, na, nb)) return -1;
  std::vector<Conn> c;
  connected(H, d, c);
  for (int64_t r = 0; r < int64_t(c.size()) && r < cap; ++r) {
    m_out[2 * r] = c[r].m[0];
    m_out[2 * r + 1] = c[r].m[1];
    h_out[r] = c[r].H;
  }
  return int64_t(c.size());
}

int or_tucker_rank(int chi, int d) { return tucker_rank(chi, d); }

// variant bits: 1 Ising-RBM correlator, 2 BDG-TensorRNN, 4 complex parameters
// (not combined with 2)
int64_t or_n_params(int K, int chi, const int* pptr, int nh, int variant) {
  if (variant & 4) {
    if (variant & 2) return -1;
    return int64_t(make_cx_ansatz(K, chi, 0, 0, pptr, nullptr, nh, variant & 1, nullptr).total);
  }
  Ansatz A = make_ansatz(K, chi, 0, 0, pptr, nullptr, nh, variant, nullptr);
  return int64_t(A.total);
}

// complex parameters: log|Phi|, phase of Phi in [-pi, pi], log|f|, sign f
int or_amplitudes_cx(int K, int chi, int na, int nb, const int* pptr, const int* pidx, int nh, int variant,
                     const double* prm, const uint64_t* samples, int64_t N, double* lphi, double* phase,
                     double* lf, int* sf, int nthreads) {
  CxAnsatz A = make_cx_ansatz(K, chi, na, nb, pptr, pidx, nh, variant & 1, prm);
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads_or_default(nthreads))
  for (int64_t i = 0; i < N; ++i) {
    Det d = det_from_words(K, samples + 2 * i);
    Amp a = cx_amp_eval(A, d);
    lphi[i] = a.lphi; phase[i] = wrap_phase(a.phase); lf[i] = a.lf; sf[i] = a.sf;
  }
  return 0;
}

// complex parameters: sum_n (ga_n d ln|Psi(n)| + gp_n d phase(n)) / d theta
// over the packed parameters (re and im of a complex parameter are two reals)
int or_grad_cx(int K, int chi, int na, int nb, const int* pptr, const int* pidx, int nh, int variant,
               const double* prm, const uint64_t* samples, int64_t N, const double* ga, const double* gp,
               double* grad, int nthreads) {
  CxAnsatz A = make_cx_ansatz(K, chi, na, nb, pptr, pidx, nh, variant & 1, prm);
  const int nt = nthreads_or_default(nthreads);
  std::vector<std::vector<double>> part(nt, std::vector<double>(A.total, 0.0));
#pragma omp parallel for schedule(static) num_threads(nt)
  for (int64_t i = 0; i < N; ++i) {
    Det d = det_from_words(K, samples + 2 * i);
    cx_grad_accumulate(A, d, ga[i], gp ? gp[i] : 0.0, part[omp_get_thread_num()].data());
  }
  for (int t = 0; t < nt; ++t)
    for (size_t k = 0; k < A.total; ++k) grad[k] += part[t][k];
  return 0;
}

// log|Phi|, sign Phi, log|f|, sign f for N samples
int or_amplitudes(int K, int chi, int na, int nb, const int* pptr, const int* pidx, int nh, int variant,
                  const double* prm, const uint64_t* samples, int64_t N, double* lphi,
                  int* sphi, double* lf, int* sf, double* mphi, double* mf, double* fsens, int nthreads) {
  Ansatz A = make_ansatz(K, chi, na, nb, pptr, pidx, nh, variant, prm);
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads_or_default(nthreads))
  for (int64_t i = 0; i < N; ++i) {
    Det d = det_from_words(K, samples + 2 * i);
    Amp a = amp_eval(A, d);
    lphi[i] = a.lphi; sphi[i] = a.sphi; lf[i] = a.lf; sf[i] = a.sf;
    if (mphi) mphi[i] = a.mphi;
    if (mf) mf[i] = a.mf;
    if (fsens) fsens[i] = a.sens;
  }
  return 0;
}

// the uniform of draw t at site i for the counter-keyed sampler: the 53-bit
// fraction of words 0, 1 of Philox4x32-10 at counter (t lo, t hi, i, 0x53414D50)
// under key (seed lo, seed hi)
double sampler_uniform(uint64_t seed, uint64_t t, int i) {
  const uint32_t ctr[4] = {uint32_t(t), uint32_t(t >> 32), uint32_t(i), 0x53414D50u};
  const uint32_t key[2] = {uint32_t(seed), uint32_t(seed >> 32)};
  uint32_t w[4];
  philox4x32_10(ctr, key, w);
  const uint64_t bits = ((uint64_t(w[1]) << 32) | w[0]) >> 11;
  return double(bits) / 9007199254740992.0;   // 2^53
}

// exact autoregressive draws from Phi^2 using the caller's uniforms u[N][K]
int or_sample(int K, int chi, int na, int nb, const int* pptr, const int* pidx, int variant,
              const double* prm, const double* u, int64_t N, uint64_t* out) {
  if (variant & 4) return cx_sample(K, chi, na, nb, pptr, pidx, prm, u, N, out);
  Ansatz A = make_ansatz(K, chi, na, nb, pptr, pidx, 0, variant & 2, prm);
  for (int64_t t = 0; t < N; ++t) {
    Det d;
    d.n = 2 * K;
    std::memset(d.x, 0, sizeof d.x);
    std::vector<double> carried(size_t(K) * chi, 0.0), cand(4 * chi);
    int a_prev = 0, b_prev = 0;
    for (int i = 0; i < K; ++i) {
      site_candidates(A, i, carried, cand.data());
      double p[4], Z = 0.0;
      for (int s = 0; s < 4; ++s) {
        double acc = 0.0;
        for (int uu = 0; uu < chi; ++uu) acc += A.prm[A.offEta[i] + uu] * cand[s * chi + uu] * cand[s * chi + uu];
        p[s] = allowed(A, i, a_prev, b_prev, s) ? acc : 0.0;
        Z += p[s];
      }
      const double target = u[t * K + i] * Z;
      double run = 0.0;
      int pick = -1, last = -1;
      for (int s = 0; s < 4; ++s) {
        if (p[s] <= 0.0) continue;
        last = s;
        run += p[s];
        if (run > target) { pick = s; break; }
      }
      if (pick < 0) pick = last;
      d.x[2 * i] = pick & 1;
      d.x[2 * i + 1] = pick >> 1;
      for (int uu = 0; uu < chi; ++uu) carried[size_t(i) * chi + uu] = cand[pick * chi + uu];
      a_prev += pick & 1;
      b_prev += pick >> 1;
    }
    det_to_words(d, out + 2 * t);
  }
  return 0;
}

// draws t = t0 .. t0+N-1 of the counter-keyed sampler (uniforms from
// sampler_uniform), then merged: unique ONVs in ascending (hi, lo) order with
// their counts; returns the number of unique ONVs (at most cap are written)
int64_t or_sample_unique(int K, int chi, int na, int nb, const int* pptr, const int* pidx, int variant,
                         const double* prm, uint64_t seed, int64_t t0, int64_t N, int64_t cap, uint64_t* out,
                         int64_t* counts) {
  std::vector<double> u(size_t(N) * K);
  for (int64_t t = 0; t < N; ++t)
    for (int i = 0; i < K; ++i) u[size_t(t) * K + i] = sampler_uniform(seed, uint64_t(t0 + t), i);
  std::vector<uint64_t> d(size_t(N) * 2);
  or_sample(K, chi, na, nb, pptr, pidx, variant, prm, u.data(), N, d.data());
  std::map<std::pair<uint64_t, uint64_t>, int64_t> merged;   // ordered by (hi, lo)
  for (int64_t t = 0; t < N; ++t) ++merged[{d[2 * t + 1], d[2 * t]}];
  int64_t k = 0;
  for (const auto& kv : merged) {
    if (k < cap) {
      out[2 * k] = kv.first.second;
      out[2 * k + 1] = kv.first.first;
      counts[k] = kv.second;
    }
    ++k;
  }
  return k;
}

// sum_n g_n d ln|Psi(n)| / d theta, accumulated into grad (length n_params)
int or_grad(int K, int chi, int na, int nb, const int* pptr, const int* pidx, int nh, int variant,
            const double* prm, const uint64_t* samples, int64_t N, const double* g,
            double* grad, int nthreads) {
  Ansatz A = make_ansatz(K, chi, na, nb, pptr, pidx, nh, variant, prm);
  const int nt = nthreads_or_default(nthreads);
  std::vector<std::vector<double>> part(nt, std::vector<double>(A.total, 0.0));
#pragma omp parallel for schedule(static) num_threads(nt)
  for (int64_t i = 0; i < N; ++i) {
    Det d = det_from_words(K, samples + 2 * i);
    grad_accumulate(A, d, g[i], part[omp_get_thread_num()].data());
  }
  for (int t = 0; t < nt; ++t)
    for (size_t k = 0; k < A.total; ++k) grad[k] += part[t][k];
  return 0;
}

// semi-stochastic local energies with the BDG-RNN x cos-RBM amplitude; the
// draw counter of sample i is sample_base + i.  Optional per-sample counters
// n_det / n_rem / n_uniq (nullable).
int or_eloc(int K, int na, int nb, const double* h, const double* eri, double ecore,
            int chi, const int* pptr, const int* pidx, int nh, int variant, const double* prm,
            const uint64_t* samples, int64_t N, double eps, int n_eps, uint64_t seed,
            uint64_t stream, int64_t sample_base, double* eloc, double* etnum, double* logabs,
            int8_t* sign, double* fsq, int64_t* n_det, int64_t* n_rem, int64_t* n_uniq,
            double* sabs, const double* bound_L, const double* bound_kappa, int n_cols, double u_f,
            double* ebound, double* mphi, double* mf, int nthreads) {
  if (n_cols < 0 || n_cols > 4) return -2;
  BoundCol cols[4];
  for (int q = 0; q < n_cols; ++q) cols[q] = BoundCol{bound_L[q], bound_kappa[q]};
  Ham H{K, h, eri, ecore};
  Ansatz A = make_ansatz(K, chi, na, nb, pptr, pidx, nh, variant, prm);
  for (int64_t i = 0; i < N; ++i) {
    Det d = det_from_words(K, samples + 2 * i);
    if (!count_ok(d, K, na, nb)) return -1;
  }
  auto amp = [&](const Det& d) { return amp_eval(A, d); };
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads_or_default(nthreads))
  for (int64_t i = 0; i < N; ++i) {
    Det d = det_from_words(K, samples + 2 * i);
    ElocOut o = eloc_one(H, d, sample_base + i, eps, n_eps, seed, stream, amp, nullptr, nullptr, cols, n_cols, u_f);
    eloc[i] = o.eloc; etnum[i] = o.etnum; logabs[i] = o.logabs; sign[i] = int8_t(o.sign);
    fsq[i] = o.fsq;
    if (n_det) n_det[i] = o.n_det;
    if (n_rem) n_rem[i] = o.n_rem;
    if (n_uniq) n_uniq[i] = o.n_uniq;
    if (sabs) sabs[i] = o.sabs;
    for (int q = 0; q < n_cols && ebound; ++q) ebound[i * n_cols + q] = o.ebound[q];
    if (mphi) mphi[i] = o.mphi;
    if (mf) mf[i] = o.mf;
  }
  return 0;
}

// complex parameters: E_loc and Etilde_num as (re, im), log|Psi|, the phase
// of Psi in [-pi, pi] (the correlator's sign included), |f|^2
int or_eloc_cx(int K, int na, int nb, const double* h, const double* eri, double ecore,
               int chi, const int* pptr, const int* pidx, int nh, int variant, const double* prm,
               const uint64_t* samples, int64_t N, double eps, int n_eps, uint64_t seed,
               uint64_t stream, int64_t sample_base, double* eloc, double* eloc_im, double* etnum,
               double* etnum_im, double* logabs, double* phase, double* fsq, int64_t* n_det,
               int64_t* n_rem, int64_t* n_uniq, double* sabs, int nthreads) {
  Ham H{K, h, eri, ecore};
  CxAnsatz A = make_cx_ansatz(K, chi, na, nb, pptr, pidx, nh, variant & 1, prm);
  for (int64_t i = 0; i < N; ++i) {
    Det d = det_from_words(K, samples + 2 * i);
    if (!count_ok(d, K, na, nb)) return -1;
  }
  auto amp = [&](const Det& d) { return cx_amp_eval(A, d); };
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads_or_default(nthreads))
  for (int64_t i = 0; i < N; ++i) {
    Det d = det_from_words(K, samples + 2 * i);
    ElocOut o = eloc_one(H, d, sample_base + i, eps, n_eps, seed, stream, amp, nullptr, nullptr);
    eloc[i] = o.eloc; eloc_im[i] = o.eloc_im; etnum[i] = o.etnum; etnum_im[i] = o.etnum_im;
    logabs[i] = o.logabs; phase[i] = o.phase; fsq[i] = o.fsq;
    if (n_det) n_det[i] = o.n_det;
    if (n_rem) n_rem[i] = o.n_rem;
    if (n_uniq) n_uniq[i] = o.n_uniq;
    if (sabs) sabs[i] = o.sabs;
  }
  return 0;
}

// one sample in detail: deterministic ranks, drawn ranks (in draw order), Q
int or_eloc_detail(int K, int na, int nb, const double* h, const double* eri, double ecore,
                   int chi, const int* pptr, const int* pidx, int nh, int variant, const double* prm,
                   const uint64_t* sample, int64_t sample_idx, double eps, int n_eps,
                   uint64_t seed, uint64_t stream, int64_t* det_ranks, int64_t det_cap,
                   int64_t* n_det_out, int64_t* draw_ranks, uint64_t* Q_out, double* eloc_out) {
  Ham H{K, h, eri, ecore};
  Ansatz A = make_ansatz(K, chi, na, nb, pptr, pidx, nh, variant, prm);
  Det d = det_from_words(K, sample);
  if (!count_ok(d, K, na, nb)) return -1;
  auto amp = [&](const Det& x) { return amp_eval(A, x); };
  std::vector<int64_t> dr, wr;
  ElocOut o = eloc_one(H, d, sample_idx, eps, n_eps, seed, stream, amp, &dr, &wr);
  *n_det_out = int64_t(dr.size());
  for (size_t t = 0; t < dr.size() && int64_t(t) < det_cap; ++t) det_ranks[t] = dr[t];
  for (size_t t = 0; t < wr.size(); ++t) draw_ranks[t] = wr[t];
  *Q_out = o.Q;
  *eloc_out = o.eloc;
  return 0;
}

// The cotangent of the VMC gradient for real parameters (Sec. 2.3, Eq. (19)):
// with weights c_n over the samples, B = sum c |f|^2 / sum c and
// E = sum c Etilde_num / sum c |f|^2, the gradient is
// 2 <d ln|Psi| (Etilde_loc - |f~|^2 E)> = sum_n cot_n d ln|Psi(n)|,
// cot_n = 2 c_n (Etilde_num(n) - |f_n|^2 E) / sum c |f|^2.
int or_reweighted_cotangent(int64_t N, const double* counts, const double* etnum, const double* fsq,
                            double* cot, double* E_out) {
  double sc_f2 = 0.0, sc_et = 0.0;
  for (int64_t n = 0; n < N; ++n) {
    sc_f2 += counts[n] * fsq[n];
    sc_et += counts[n] * etnum[n];
  }
  const double E = sc_et / sc_f2;
  for (int64_t n = 0; n < N; ++n) cot[n] = 2.0 * counts[n] * (etnum[n] - fsq[n] * E) / sc_f2;
  *E_out = E;
  return 0;
}

// Complex parameters: the gradient of E = <H> over the real and imaginary
// parts of the parameters is 2 Re <(E_loc - E)^* d ln Psi> with d ln Psi =
// d ln|Psi| + i d phase, i.e. 2 <Re(E_loc - E) d ln|Psi| + Im E_loc d phase>;
// reweighted as in Eq. (19): cot_abs_n = 2 c_n (Re Etilde_num(n) - |f_n|^2 E)
// / sum c |f|^2 and cot_phase_n = 2 c_n Im Etilde_num(n) / sum c |f|^2, with
// E = sum c Re Etilde_num / sum c |f|^2.
int or_reweighted_cotangent_cx(int64_t N, const double* counts, const double* etnum, const double* etnum_im,
                               const double* fsq, double* cot_abs, double* cot_phase, double* E_out) {
  double sc_f2 = 0.0, sc_et = 0.0;
  for (int64_t n = 0; n < N; ++n) {
    sc_f2 += counts[n] * fsq[n];
    sc_et += counts[n] * etnum[n];
  }
  const double E = sc_et / sc_f2;
  for (int64_t n = 0; n < N; ++n) {
    cot_abs[n] = 2.0 * counts[n] * (etnum[n] - fsq[n] * E) / sc_f2;
    cot_phase[n] = 2.0 * counts[n] * etnum_im[n] / sc_f2;
  }
  *E_out = E;
  return 0;
}

// One AdamW step (Loshchilov and Hutter, decoupled weight decay; the
// formulation of PyTorch's AdamW): p <- p (1 - lr wd); m <- b1 m + (1 - b1) g;
// v <- b2 v + (1 - b2) g^2; p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
int or_adamw(int64_t n, double* p, const double* g, double* m, double* v, int64_t t, double lr, double b1,
             double b2, double eps, double wd) {
  const double c1 = 1.0 - std::pow(b1, double(t)), c2 = 1.0 - std::pow(b2, double(t));
  for (int64_t k = 0; k < n; ++k) {
    p[k] *= 1.0 - lr * wd;
    m[k] = b1 * m[k] + (1.0 - b1) * g[k];
    v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
    const double mh = m[k] / c1, vh = v[k] / c2;
    p[k] -= lr * mh / (std::sqrt(vh) + eps);
  }
  return 0;
}

// Projection of the packed parameters onto the constraint eta >= 0 of the
// conditional P = h^T eta h (Sec. 2.1): every negative eta entry becomes 0
// (NaN stays NaN, so a diverged step is still refused when bound).  Applied
// after each AdamW update of a VMC step: projected gradient descent.
int or_project_eta(int K, int chi, const int* pptr, int nh, int variant, double* p) {
  const bool cx = (variant & 4) != 0;
  std::vector<size_t> off;
  if (cx) off = make_cx_ansatz(K, chi, 0, 0, pptr, nullptr, nh, (variant & 1) != 0, nullptr).offEta;
  else off = make_ansatz(K, chi, 0, 0, pptr, nullptr, nh, variant, nullptr).offEta;
  for (int i = 0; i < K; ++i)
    for (int u = 0; u < chi; ++u)
      if (p[off[i] + u] < 0.0) p[off[i] + u] = 0.0;
  return 0;
}

// local energies with the amplitude given as a table over sorted ONV keys
// (keys as [T][2] words, ascending as 128-bit integers); an ONV missing from
// the table has amplitude 0.
int or_eloc_table(int K, int na, int nb, const double* h, const double* eri, double ecore,
                  const uint64_t* keys, const double* vals, int64_t T,
                  const uint64_t* samples, int64_t N, double eps, int n_eps, uint64_t seed,
                  uint64_t stream, double* eloc, int nthreads) {
  Ham H{K, h, eri, ecore};
  auto lookup = [&](const Det& d) {
    uint64_t w[2];
    det_to_words(d, w);
    const u128 key = (u128(w[1]) << 64) | w[0];
    int64_t lo = 0, hi = T;
    while (lo < hi) {
      const int64_t mid = (lo + hi) / 2;
      const u128 km = (u128(keys[2 * mid + 1]) << 64) | keys[2 * mid];
      if (km < key) lo = mid + 1; else hi = mid;
    }
    Amp a;
    a.lf = 0.0; a.sf = 1; a.phase = 0.0; a.valid = true;
    const u128 kf = lo < T ? ((u128(keys[2 * lo + 1]) << 64) | keys[2 * lo]) : 0;
    const double v = (lo < T && kf == key) ? vals[lo] : 0.0;
    a.lphi = std::log(std::fabs(v));
    a.sphi = v < 0 ? -1 : 1;
    return a;
  };
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads_or_default(nthreads))
  for (int64_t i = 0; i < N; ++i) {
    Det d = det_from_words(K, samples + 2 * i);
    ElocOut o = eloc_one(H, d, i, eps, n_eps, seed, stream, lookup, nullptr, nullptr);
    eloc[i] = o.eloc;
  }
  return 0;
}

}  // extern "C"
