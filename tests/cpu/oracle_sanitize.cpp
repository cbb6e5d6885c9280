// Host-only driver for sanitizer builds of the FP64 oracle (test
// infrastructure): links oracle/oracle.cpp and calls every C entry point on
// a small seeded instance (K = 6, 3 alpha + 3 beta, chain and NN+NNN
// graphs, cos-RBM / Ising-RBM correlators, the tensor term, complex
// parameters), so that AddressSanitizer and UndefinedBehaviorSanitizer see
// the oracle's indexing and arithmetic on real inputs.  Prints "ok".
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

extern "C" {
int or_hdiag(int K, int na, int nb, const double* h, const double* eri, double ecore, const uint64_t* samples,
             int64_t N, double* out);
int64_t or_connected(int K, int na, int nb, const double* h, const double* eri, double ecore,
                     const uint64_t* sample, uint64_t* m_out, double* h_out, int64_t cap);
int64_t or_n_params(int K, int chi, const int* pptr, int nh, int variant);
int or_amplitudes(int K, int chi, int na, int nb, const int* pptr, const int* pidx, int nh, int variant,
                  const double* prm, const uint64_t* samples, int64_t N, double* lphi, int* sphi, double* lf,
                  int* sf, double* mphi, double* mf, double* fsens, int nthreads);
int or_amplitudes_cx(int K, int chi, int na, int nb, const int* pptr, const int* pidx, int nh, int variant,
                     const double* prm, const uint64_t* samples, int64_t N, double* lphi, double* phase,
                     double* lf, int* sf, int nthreads);
int or_grad(int K, int chi, int na, int nb, const int* pptr, const int* pidx, int nh, int variant,
            const double* prm, const uint64_t* samples, int64_t N, const double* g, double* grad, int nthreads);
int or_grad_cx(int K, int chi, int na, int nb, const int* pptr, const int* pidx, int nh, int variant,
               const double* prm, const uint64_t* samples, int64_t N, const double* ga, const double* gp,
               double* grad, int nthreads);
int64_t or_sample_unique(int K, int chi, int na, int nb, const int* pptr, const int* pidx, int variant,
                         const double* prm, uint64_t seed, int64_t t0, int64_t N, int64_t cap, uint64_t* out,
                         int64_t* counts);
int or_eloc(int K, int na, int nb, const double* h, const double* eri, double ecore, int chi, const int* pptr,
            const int* pidx, int nh, int variant, const double* prm, const uint64_t* samples, int64_t N,
            double eps, int n_eps, uint64_t seed, uint64_t stream, int64_t sample_base, double* eloc,
            double* etnum, double* logabs, int8_t* sign, double* fsq, int64_t* n_det, int64_t* n_rem,
            int64_t* n_uniq, double* sabs, const double* bound_L, const double* bound_kappa, int n_cols,
            double u_f, double* ebound, double* mphi, double* mf, int nthreads);
int or_eloc_cx(int K, int na, int nb, const double* h, const double* eri, double ecore, int chi, const int* pptr,
               const int* pidx, int nh, int variant, const double* prm, const uint64_t* samples, int64_t N,
               double eps, int n_eps, uint64_t seed, uint64_t stream, int64_t sample_base, double* eloc,
               double* eloc_im, double* etnum, double* etnum_im, double* logabs, double* phase, double* fsq,
               int64_t* n_det, int64_t* n_rem, int64_t* n_uniq, double* sabs, int nthreads);
int or_eloc_detail(int K, int na, int nb, const double* h, const double* eri, double ecore, int chi,
                   const int* pptr, const int* pidx, int nh, int variant, const double* prm,
                   const uint64_t* sample, int64_t sample_idx, double eps, int n_eps, uint64_t seed,
                   uint64_t stream, int64_t* det_ranks, int64_t det_cap, int64_t* n_det_out, int64_t* draw_ranks,
                   uint64_t* Q_out, double* eloc_out);
int or_eloc_table(int K, int na, int nb, const double* h, const double* eri, double ecore, const uint64_t* keys,
                  const double* vals, int64_t T, const uint64_t* samples, int64_t N, double eps, int n_eps,
                  uint64_t seed, uint64_t stream, double* eloc, int nthreads);
int or_reweighted_cotangent(int64_t N, const double* counts, const double* etnum, const double* fsq, double* cot,
                            double* E_out);
int or_adamw(int64_t n, double* p, const double* g, double* m, double* v, int64_t t, double lr, double b1,
             double b2, double eps, double wd);
int or_project_eta(int K, int chi, const int* pptr, int nh, int variant, double* p);
}

namespace {

uint64_t g_state = 0x9E3779B97F4A7C15ull;
double uniform() {   // splitmix64 -> [0, 1)
  uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return double(z >> 11) * (1.0 / 9007199254740992.0);
}
double gauss() { return std::sqrt(-2.0 * std::log(1.0 - uniform())) * std::cos(6.283185307179586 * uniform()); }

int fails = 0;
void check(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAILED %s\n", what);
    ++fails;
  }
}

}  // namespace

int main() {
  const int K = 6, na = 3, nb = 3, chi = 4, nh = 6;
  // symmetric h and 8-fold symmetric (pq|rs)
  std::vector<double> h(K * K), eri(size_t(K) * K * K * K);
  for (int p = 0; p < K; ++p)
    for (int q = 0; q <= p; ++q) h[p * K + q] = h[q * K + p] = 0.3 * gauss();
  auto E = [&](int p, int q, int r, int s) -> double& { return eri[((size_t(p) * K + q) * K + r) * K + s]; };
  for (int p = 0; p < K; ++p)
    for (int q = 0; q < K; ++q)
      for (int r = 0; r < K; ++r)
        for (int s = 0; s < K; ++s) {
          if (p < q || r < s || p * K + q < r * K + s) continue;
          const double v = 0.1 * gauss();
          for (auto t : {std::array<int, 4>{p, q, r, s}, {q, p, r, s}, {p, q, s, r}, {q, p, s, r},
                         {r, s, p, q}, {s, r, p, q}, {r, s, q, p}, {s, r, q, p}})
            E(t[0], t[1], t[2], t[3]) = v;
        }
  // every ONV of the sector (interleaved bits P = 2p + sigma), ascending
  std::vector<uint64_t> all;
  for (uint64_t x = 0; x < (uint64_t(1) << (2 * K)); ++x) {
    int a = 0, b = 0;
    for (int p = 0; p < K; ++p) {
      a += (x >> (2 * p)) & 1;
      b += (x >> (2 * p + 1)) & 1;
    }
    if (a == na && b == nb) { all.push_back(x); all.push_back(0); }
  }
  const int64_t T = int64_t(all.size() / 2);
  check(T == 400, "sector size");
  const int64_t N = 24;
  std::vector<uint64_t> smp(all.begin(), all.begin() + 2 * N);
  // chain and NN+NNN graphs
  std::vector<int> ptr_c{0}, idx_c, ptr_n{0}, idx_n;
  for (int i = 0; i < K; ++i) {
    if (i >= 1) idx_c.push_back(i - 1);
    ptr_c.push_back(int(idx_c.size()));
    if (i >= 2) idx_n.push_back(i - 2);
    if (i >= 1) idx_n.push_back(i - 1);
    ptr_n.push_back(int(idx_n.size()));
  }
  std::vector<double> hd(N);
  check(or_hdiag(K, na, nb, h.data(), eri.data(), 0.0, smp.data(), N, hd.data()) == 0, "hdiag");
  std::vector<uint64_t> mo(2 * 200);
  std::vector<double> ho(200);
  check(or_connected(K, na, nb, h.data(), eri.data(), 0.0, smp.data(), mo.data(), ho.data(), 200) == 117,
        "connected count");
  // real ansatze: plain cos-RBM (0), Ising-RBM (1) on the chain; tensor term (2) on NN+NNN
  for (int variant : {0, 1, 2}) {
    const bool tensor = variant == 2;
    const int* pp = tensor ? ptr_n.data() : ptr_c.data();
    const int* pi = tensor ? idx_n.data() : idx_c.data();
    const int nhv = tensor ? 0 : nh;
    const int64_t np = or_n_params(K, chi, pp, nhv, variant);
    check(np > 0, "n_params");
    std::vector<double> prm(np);
    for (auto& x : prm) x = 0.3 * gauss();
    // eta entries positive: every site's eta block follows its M blocks and v (4 chi)
    int64_t o = 0;
    for (int i = 0; i < K; ++i) {
      o += int64_t(pp[i + 1] - pp[i]) * 4 * chi * chi + 4 * chi;
      for (int u = 0; u < chi; ++u) prm[o + u] = 0.5 + uniform();
      o += 2 * chi + 1;
    }
    std::vector<double> lphi(N), lf(N), mphi(N), mf(N), fs(N);
    std::vector<int> sphi(N), sf(N);
    check(or_amplitudes(K, chi, na, nb, pp, pi, nhv, variant, prm.data(), smp.data(), N, lphi.data(), sphi.data(),
                        lf.data(), sf.data(), mphi.data(), mf.data(), fs.data(), 2) == 0, "amplitudes");
    std::vector<double> el(N), et(N), la(N), f2(N), sa(N), eb(2 * N), m1(N), m2(N);
    std::vector<int8_t> sg(N);
    std::vector<int64_t> nd(N), nr(N), nu(N);
    const double bl[2] = {1e-6, 1e-2}, bk[2] = {1e-7, 1e-2};
    check(or_eloc(K, na, nb, h.data(), eri.data(), 0.0, chi, pp, pi, nhv, variant, prm.data(), smp.data(), N, 0.05,
                  20, 7, 1, 0, el.data(), et.data(), la.data(), sg.data(), f2.data(), nd.data(), nr.data(), nu.data(),
                  sa.data(), bl, bk, 2, 4e-7, eb.data(), m1.data(), m2.data(), 2) == 0, "eloc");
    for (int64_t n = 0; n < N; ++n) check(std::isfinite(el[n]) && std::fabs(el[n]) <= sa[n] * (1 + 1e-12), "eloc finite");
    std::vector<double> g(N, 1.0), grad(np, 0.0);
    check(or_grad(K, chi, na, nb, pp, pi, nhv, variant, prm.data(), smp.data(), N, g.data(), grad.data(), 2) == 0,
          "grad");
    std::vector<uint64_t> us(2 * 300);
    std::vector<int64_t> uc(300);
    check(or_sample_unique(K, chi, na, nb, pp, pi, variant & 2, prm.data(), 11, 0, 300, 300, us.data(),
                           uc.data()) > 0, "sample_unique");
    std::vector<int64_t> dr(200), drw(20);
    int64_t ndet = 0;
    uint64_t Q = 0;
    double e1 = 0;
    check(or_eloc_detail(K, na, nb, h.data(), eri.data(), 0.0, chi, pp, pi, nhv, variant, prm.data(), smp.data(), 0,
                         0.05, 20, 7, 1, dr.data(), 200, &ndet, drw.data(), &Q, &e1) == 0, "eloc_detail");
    std::vector<double> mm(np, 0.0), vv(np, 0.0), cot(N);
    double Ew = 0;
    std::vector<double> cnt(N, 1.0);
    check(or_reweighted_cotangent(N, cnt.data(), et.data(), f2.data(), cot.data(), &Ew) == 0, "cotangent");
    check(or_adamw(np, prm.data(), grad.data(), mm.data(), vv.data(), 1, 1e-2, 0.9, 0.999, 1e-8, 1e-3) == 0, "adamw");
    check(or_project_eta(K, chi, pp, nhv, variant, prm.data()) == 0, "project_eta");
  }
  // complex parameters (variant 4) with a cos-RBM correlator
  {
    const int64_t np = or_n_params(K, chi, ptr_c.data(), nh, 4);
    std::vector<double> prm(np);
    for (auto& x : prm) x = 0.3 * gauss();
    int64_t o = 0;
    for (int i = 0; i < K; ++i) {
      o += int64_t(ptr_c[i + 1] - ptr_c[i]) * 8 * chi * chi + 8 * chi;
      for (int u = 0; u < chi; ++u) prm[o + u] = 0.5 + uniform();
      o += chi + 2 * chi + 2;
    }
    std::vector<double> lphi(N), ph(N), lf(N);
    std::vector<int> sf(N);
    check(or_amplitudes_cx(K, chi, na, nb, ptr_c.data(), idx_c.data(), nh, 4, prm.data(), smp.data(), N,
                           lphi.data(), ph.data(), lf.data(), sf.data(), 2) == 0, "amplitudes_cx");
    std::vector<double> er(N), ei(N), tr(N), ti(N), la(N), phase(N), f2(N), sa(N);
    std::vector<int64_t> nd(N), nr(N), nu(N);
    check(or_eloc_cx(K, na, nb, h.data(), eri.data(), 0.0, chi, ptr_c.data(), idx_c.data(), nh, 4, prm.data(),
                     smp.data(), N, 0.05, 20, 7, 1, 0, er.data(), ei.data(), tr.data(), ti.data(), la.data(),
                     phase.data(), f2.data(), nd.data(), nr.data(), nu.data(), sa.data(), 2) == 0, "eloc_cx");
    std::vector<double> ga(N, 1.0), gp(N, 0.5), grad(np, 0.0);
    check(or_grad_cx(K, chi, na, nb, ptr_c.data(), idx_c.data(), nh, 4, prm.data(), smp.data(), N, ga.data(),
                     gp.data(), grad.data(), 2) == 0, "grad_cx");
  }
  // a table amplitude over the whole sector
  {
    std::vector<double> vals(T);
    for (auto& x : vals) x = gauss();
    std::vector<double> el(N);
    check(or_eloc_table(K, na, nb, h.data(), eri.data(), 0.0, all.data(), vals.data(), T, smp.data(), N, 0.05, 20,
                        7, 1, el.data(), 2) == 0, "eloc_table");
  }
  std::printf(fails ? "failed %d\n" : "ok\n", fails);
  return fails ? 1 : 0;
}
