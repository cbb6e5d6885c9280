"""Pins of the oracle quantities behind the reduced-precision error bounds:
the absolute sum S_n of the local-energy terms (Sec. 2.1 Eq. (6), Sec. 2.4
Eqs. (20)-(22)), the sign margins of Phi (the phase of real parameters,
sign(w^T h + c), Sec. 2.1) and of the cos-RBM factor (Sec. 2.3 Eq. (15)), and
the flip allowance A_n(kappa) built from them.  Each is checked against its
definition evaluated through other oracle functions, or a closed form."""
import numpy as np
import pytest

import oracle
from paper_2507_19276_amd import workloads as W


def site_offsets(K, chi, parent_ptr):
    """(v, eta, w, c) offsets of each site in the packed real layout."""
    o, out = 0, []
    for i in range(K):
        o += (int(parent_ptr[i + 1]) - int(parent_ptr[i])) * 4 * chi * chi
        out.append((o, o + 4 * chi, o + 5 * chi, o + 6 * chi))
        o += 6 * chi + 1
    return out


def _terms(w, samples, params=None, nh=None):
    """|H_nn| and the exact (eps = 0) terms H_nm Psi(m)/Psi(n) of each sample,
    from the connected list and the amplitudes of every determinant."""
    params = w.params if params is None else params
    nh = w.n_hidden if nh is None else nh
    out = []
    for s in samples:
        rm, rh = oracle.connected(w.K, w.n_alpha, w.n_beta, w.h, w.eri, s)
        keep = rh != 0.0
        rm, rh = rm[keep], rh[keep]
        amp = oracle.amplitudes(w.K, w.chi, w.n_alpha, w.n_beta, w.parent_ptr, w.parent_idx, nh, params,
                                np.vstack([s[None], rm]))
        r = amp["sign"][1:] * amp["sign"][0] * np.exp(amp["logabs"][1:] - amp["logabs"][0])
        hd = oracle.hdiag(w.K, w.n_alpha, w.n_beta, w.h, w.eri, s[None])[0]
        out.append((hd, rh * r, amp))
    return out


@pytest.mark.parametrize("nh", [0, 6])
def test_sabs_is_the_absolute_sum_of_the_terms(nh):
    w = W.make_workload("c1")
    smp = w.samples[:24]
    prm = W.ansatz_params(w.K, w.chi, w.parent_ptr, w.parent_idx, nh, 17)
    ref = oracle.eloc(w.K, w.n_alpha, w.n_beta, w.h, w.eri, w.chi, w.parent_ptr, w.parent_idx, nh, prm, smp)
    for k, (hd, t, _) in enumerate(_terms(w, smp, params=prm, nh=nh)):
        S = abs(hd) + np.abs(t).sum()
        assert abs(ref["sabs"][k] - S) <= 1e-12 * S
        assert abs(ref["eloc"][k]) <= ref["sabs"][k] * (1 + 1e-14)      # triangle inequality


def test_sabs_counts_every_draw():
    """With draws: S_n = |H_nn| + sum_D |H r| + sum over the N_eps draws of
    |H Q / (N_eps q) r| (each draw counted, duplicates included)."""
    w = W.make_workload("c1")
    eps, n_eps, seed = 0.05, 37, 9
    for k in range(6):
        s = w.samples[k]
        ref = oracle.eloc(w.K, w.n_alpha, w.n_beta, w.h, w.eri, w.chi, w.parent_ptr, w.parent_idx, 0, w.params,
                          s[None], eps=eps, n_eps=n_eps, seed=seed, sample_base=k)
        d = oracle.eloc_detail(w.K, w.n_alpha, w.n_beta, w.h, w.eri, w.chi, w.parent_ptr, w.parent_idx, 0,
                               w.params, s, k, eps, n_eps, seed=seed)
        rm, rh = oracle.connected(w.K, w.n_alpha, w.n_beta, w.h, w.eri, s)
        amp = oracle.amplitudes(w.K, w.chi, w.n_alpha, w.n_beta, w.parent_ptr, w.parent_idx, 0, w.params,
                                np.vstack([s[None], rm]))
        ratio = np.exp(amp["logabs"][1:] - amp["logabs"][0])
        hd = oracle.hdiag(w.K, w.n_alpha, w.n_beta, w.h, w.eri, s[None])[0]
        S = abs(hd) + np.abs(rh[d["det_ranks"]] * ratio[d["det_ranks"]]).sum()
        for rk in d["draw_ranks"]:
            q = oracle.proposal_weight(abs(rh[rk]), eps)
            S += abs(rh[rk] * d["Q"] / (q * n_eps)) * ratio[rk]
        assert abs(ref["sabs"][0] - S) <= 1e-12 * S


def test_phi_margin_closed_forms():
    w = W.make_workload("c1")
    offs = site_offsets(w.K, w.chi, w.parent_ptr)
    smp = W.all_onvs(w.K, w.n_alpha, w.n_beta)
    p = w.params.copy()
    for (_, _, ow, oc) in offs:           # w = 0, c = 1 at every site: |c| / |c|
        p[ow:ow + w.chi] = 0.0
        p[oc] = 1.0
    a = oracle.amplitudes(w.K, w.chi, w.n_alpha, w.n_beta, w.parent_ptr, w.parent_idx, 0, p, smp)
    np.testing.assert_array_equal(a["margin_phi"], 1.0)
    assert np.isinf(a["margin_f"]).all()
    # site 0 (no parents, h = v^{s_0}) with w = e_0 and c = 0: |v^{s_0}_0| / ||v^{s_0}||
    ov, _, ow, oc = offs[0]
    p[ow] = 1.0
    p[oc] = 0.0
    a = oracle.amplitudes(w.K, w.chi, w.n_alpha, w.n_beta, w.parent_ptr, w.parent_idx, 0, p, smp)
    v = p[ov:ov + 4 * w.chi].reshape(4, w.chi)
    s0 = (smp[:, 0] & 1).astype(int) + 2 * ((smp[:, 0] >> 1) & 1).astype(int)
    want = np.minimum(1.0, np.abs(v[s0, 0]) / np.linalg.norm(v[s0], axis=1))
    np.testing.assert_allclose(a["margin_phi"], want, rtol=1e-14)


def test_correlator_margin_closed_form():
    """W = 0 gives theta_k = b_k for every ONV: margin_f = min_k |cos b_k| / (1 + |b_k|)."""
    w = W.make_workload("c1")
    nh = 6
    pr = np.concatenate([w.params, np.zeros(nh + nh * 2 * w.K)])
    b = np.array([0.3, -1.2, 1.5, 2.9, -0.7, 1.55])
    pr[w.params.size:w.params.size + nh] = b
    a = oracle.amplitudes(w.K, w.chi, w.n_alpha, w.n_beta, w.parent_ptr, w.parent_idx, nh, pr, w.samples[:8])
    want = np.min(np.abs(np.cos(b)) / (1 + np.abs(b)))
    np.testing.assert_allclose(a["margin_f"], want, rtol=1e-14)


def test_bound_weights_without_correlator():
    """Without a correlator: L > 0 and kappa below every margin give
    expm1(2L) (S_n - |H_nn|); L = 0 and a kappa between margins give 2 x the
    |term| mass of the rows whose margin, or whose sample's, is below kappa;
    kappa >= 1 (margins never exceed 1) counts every term."""
    w = W.make_workload("c1")
    smp = w.samples[:16]
    terms = _terms(w, smp)
    mus = np.concatenate([t[2]["margin_phi"] for t in terms])
    cols = ((1e-3, 0.5 * mus.min()), (0.0, float(np.median(mus))), (0.0, 1.0))
    ref = oracle.eloc(w.K, w.n_alpha, w.n_beta, w.h, w.eri, w.chi, w.parent_ptr, w.parent_idx, 0, w.params, smp,
                      bounds=cols, u_f=0.0)
    for k, (hd, t, amp) in enumerate(terms):
        S = ref["sabs"][k] - abs(hd)
        assert abs(ref["ebound"][k, 0] - np.expm1(2e-3) * S) <= 1e-12 * S
        mrow, msmp = amp["margin_phi"][1:], amp["margin_phi"][0]
        flip = (mrow < cols[1][1]) | (msmp < cols[1][1])
        want = 2.0 * np.abs(t[flip]).sum()
        assert abs(ref["ebound"][k, 1] - want) <= 1e-12 * max(want, 1.0), k
        assert abs(ref["ebound"][k, 2] - 2 * S) <= 1e-12 * S


def test_correlator_sensitivity_and_its_bound_weight():
    """corr_sens = sum_k (1 + |theta_k|) / |cos theta_k| (closed form at W = 0);
    with L = 0, kappa = 0 and u_f > 0 (no margin below 8 u_f here) each term
    gets the weight expm1(u_f (corr_sens(m) + corr_sens(n)))."""
    w = W.make_workload("c1")
    nh = 6
    pr = np.concatenate([w.params, np.zeros(nh + nh * 2 * w.K)])
    b = np.array([0.3, -1.2, 1.5, 2.9, -0.7, 1.1])
    pr[w.params.size:w.params.size + nh] = b
    a = oracle.amplitudes(w.K, w.chi, w.n_alpha, w.n_beta, w.parent_ptr, w.parent_idx, nh, pr, w.samples[:4])
    np.testing.assert_allclose(a["corr_sens"], np.sum((1 + np.abs(b)) / np.abs(np.cos(b))), rtol=1e-14)
    prm = W.ansatz_params(w.K, w.chi, w.parent_ptr, w.parent_idx, nh, 23)
    smp = w.samples[:10]
    uf = 1e-4
    ref = oracle.eloc(w.K, w.n_alpha, w.n_beta, w.h, w.eri, w.chi, w.parent_ptr, w.parent_idx, nh, prm, smp,
                      bounds=((0.0, 0.0),), u_f=uf)
    for k, s in enumerate(smp):
        rm, rh = oracle.connected(w.K, w.n_alpha, w.n_beta, w.h, w.eri, s)
        keep = rh != 0.0
        rm, rh = rm[keep], rh[keep]
        amp = oracle.amplitudes(w.K, w.chi, w.n_alpha, w.n_beta, w.parent_ptr, w.parent_idx, nh, prm,
                                np.vstack([s[None], rm]))
        assert np.all(amp["margin_f"] >= 8 * uf)
        x = np.abs(rh) * np.exp(amp["logabs"][1:] - amp["logabs"][0])
        want = (x * np.expm1(uf * (amp["corr_sens"][1:] + amp["corr_sens"][0]))).sum()
        assert abs(ref["ebound"][k, 0] - want) <= 1e-12 * want


def test_bound_covers_an_actual_flip():
    """Make the sign of Phi at site 0 (parentless, h = v^{s_0}) the sign of
    v^{s_0}[0] (w_0 = e_0, c_0 = 0) and set that component to +delta or
    -delta for the local state s = 1: rows whose site 0 is in state 1, of
    samples whose site 0 is not, change sign and nothing else changes beyond
    O(delta).  Their row margin is delta / ||v^1||, so the bound at a kappa
    above it covers the change; at a kappa below every margin it is 0
    although E_loc moved: the flip term of the bound is needed."""
    w = W.make_workload("c1")
    chi = w.chi
    ov, _, ow, oc = site_offsets(w.K, chi, w.parent_ptr)[0]
    p = w.params.copy()
    p[ow:ow + chi] = 0.0
    p[ow] = 1.0
    p[oc] = 0.0
    delta = 1e-9
    p[ov + chi] = delta
    q = p.copy()
    q[ov + chi] = -delta
    mu = delta / np.linalg.norm(p[ov + chi:ov + 2 * chi])
    allv = W.all_onvs(w.K, w.n_alpha, w.n_beta)
    s0 = (allv[:, 0] & 1).astype(int) + 2 * ((allv[:, 0] >> 1) & 1).astype(int)
    smp = allv[s0 != 1][:40]
    a = oracle.eloc(w.K, w.n_alpha, w.n_beta, w.h, w.eri, chi, w.parent_ptr, w.parent_idx, 0, p, smp,
                    bounds=((0.0, 1e-3 * mu), (1e-7, 4 * mu)))
    b = oracle.eloc(w.K, w.n_alpha, w.n_beta, w.h, w.eri, chi, w.parent_ptr, w.parent_idx, 0, q, smp)
    dE = np.abs(a["eloc"] - b["eloc"])
    assert dE.max() > 1e-2
    assert np.all(dE <= a["ebound"][:, 1])
    assert np.all(a["ebound"][:, 0] == 0.0)
