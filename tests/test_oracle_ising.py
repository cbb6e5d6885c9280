"""Pins of the oracle's Ising-RBM correlator (Sec. 2.3, Eq. (16)): theta_k is
the cos-RBM argument plus one half of the quadratic form of W2_k over the
occupations, f = prod_k cos(theta_k).  Each pin reduces it to something fixed
independently: the cos-RBM (itself pinned by closed forms), a quadratic form's
invariances, a closed form, finite differences and the dense FCI definition
of the local energy."""
import numpy as np
import pytest

import oracle
from bruteforce import dense_hamiltonian, int_to_words
from paper_2507_19276_amd import workloads as W


def _setup(nh=4, K=6, na=3, nb=3, chi=3, graph="nnn", seed=21):
    h, eri = W.chain_integrals(K, seed)
    pp, pi = {"chain": W.graph_chain, "nnn": W.graph_nn_nnn}[graph](K)
    prm = W.ansatz_params(K, chi, pp, pi, nh, seed + 1, corr_scale=0.3, ising=True)
    onvs = W.all_onvs(K, na, nb)
    nv = 2 * K
    base = prm.size - nh * (nv + 1) - nh * nv * nv
    return dict(K=K, na=na, nb=nb, chi=chi, pp=pp, pi=pi, nh=nh, prm=prm, onvs=onvs, nv=nv, base=base,
                h=h, eri=eri)


def _amps(s, prm, ising=True, nh=None, samples=None):
    return oracle.amplitudes(s["K"], s["chi"], s["na"], s["nb"], s["pp"], s["pi"], s["nh"] if nh is None else nh,
                             prm, s["onvs"] if samples is None else samples, ising=ising)


def _split(s, prm):
    nh, nv, b0 = s["nh"], s["nv"], s["base"]
    bias = prm[b0:b0 + nh]
    W1 = prm[b0 + nh:b0 + nh + nh * nv].reshape(nh, nv)
    W2 = prm[b0 + nh + nh * nv:].reshape(nh, nv, nv)
    return bias, W1, W2


def _cos_prm(s, prm):
    """The same parameters without the quadratic block (cos-RBM layout)."""
    return prm[:s["base"] + s["nh"] * (s["nv"] + 1)].copy()


def test_zero_quadratic_is_the_cos_rbm():
    s = _setup()
    prm = s["prm"].copy()
    _, _, W2 = _split(s, prm)
    W2[:] = 0.0
    a = _amps(s, prm)
    c = _amps(s, _cos_prm(s, prm), ising=False)
    assert np.array_equal(a["lf"], c["lf"]) and np.array_equal(a["sf"], c["sf"])
    assert np.array_equal(a["lphi"], c["lphi"])


def test_antisymmetric_quadratic_has_no_effect():
    """x^T A x = 0 for antisymmetric A: a sum over ordered pairs (both P, Q and
    Q, P) is required."""
    s = _setup()
    prm = s["prm"].copy()
    _, _, W2 = _split(s, prm)
    rng = np.random.default_rng(5)
    A = rng.standard_normal(W2.shape)
    W2[:] = A - A.transpose(0, 2, 1)
    a = _amps(s, prm)
    W2[:] = 0.0
    z = _amps(s, prm)
    np.testing.assert_allclose(a["lf"], z["lf"], rtol=0, atol=1e-12)
    assert np.array_equal(a["sf"], z["sf"])


def test_diagonal_quadratic_is_half_a_linear_term():
    """x_P^2 = x_P: a diagonal W2 acts as W1 + diag(W2) / 2 (pins the factor
    one half and the inclusion of P = Q)."""
    s = _setup()
    prm = s["prm"].copy()
    _, W1, W2 = _split(s, prm)
    rng = np.random.default_rng(6)
    d = rng.standard_normal((s["nh"], s["nv"]))
    W2[:] = 0.0
    for k in range(s["nh"]):
        W2[k][np.diag_indices(s["nv"])] = d[k]
    a = _amps(s, prm)
    cp = _cos_prm(s, prm)
    cp[s["base"] + s["nh"]:] = (W1 + d / 2).reshape(-1)
    c = _amps(s, cp, ising=False)
    np.testing.assert_allclose(a["lf"], c["lf"], rtol=0, atol=1e-12)
    assert np.array_equal(a["sf"], c["sf"])


def test_single_symmetric_pair_closed_form():
    """One hidden unit, b = W1 = 0, W2[P, Q] = W2[Q, P] = a (P != Q):
    theta = a x_P x_Q, so f = cos(a) exactly where both are occupied, else 1."""
    s = _setup(nh=1)
    prm = s["prm"].copy()
    bias, W1, W2 = _split(s, prm)
    bias[:] = 0.0
    W1[:] = 0.0
    W2[:] = 0.0
    P, Q, a = 2, 9, 2.3
    W2[0, P, Q] = W2[0, Q, P] = a
    out = _amps(s, prm)
    xP = np.array([(int(x[0]) >> P) & 1 for x in s["onvs"]])
    xQ = np.array([(int(x[0]) >> Q) & 1 for x in s["onvs"]])
    both = (xP & xQ).astype(bool)
    assert both.any() and (~both).any()
    np.testing.assert_allclose(out["lf"][both], np.log(abs(np.cos(a))), rtol=0, atol=1e-15)
    assert np.all(out["lf"][~both] == 0.0)
    assert np.all(out["sf"][both] == -1) and np.all(out["sf"][~both] == 1)   # cos(2.3) < 0


def test_grad_matches_finite_differences():
    s = _setup(nh=3)
    rng = np.random.default_rng(7)
    samples = s["onvs"][rng.choice(len(s["onvs"]), 10, replace=False)]
    g = rng.standard_normal(len(samples))
    gr = oracle.grad(s["K"], s["chi"], s["na"], s["nb"], s["pp"], s["pi"], s["nh"], s["prm"], samples, g,
                     ising=True)
    b0 = s["base"]
    # correlator block (b, W1, W2) and a few ansatz entries
    idx = np.concatenate([rng.choice(np.arange(b0, s["prm"].size), 60, replace=False),
                          rng.choice(b0, 10, replace=False)])
    hstep = 1e-6
    fd = []
    for k in idx:
        p1, p2 = s["prm"].copy(), s["prm"].copy()
        p1[k] += hstep
        p2[k] -= hstep
        fd.append((_amps(s, p1, samples=samples)["logabs"] - _amps(s, p2, samples=samples)["logabs"]) @ g
                  / (2 * hstep))
    np.testing.assert_allclose(gr[idx], np.array(fd), rtol=1e-6, atol=1e-8)


def test_exact_eloc_matches_dense_definition():
    """eps = 0 with the Ising-RBM correlator: E_loc(n) = (H Psi)(n) / Psi(n)
    over the whole sector, Psi = f Phi from the oracle's amplitudes."""
    s = _setup(nh=5, graph="chain")
    basis, H = dense_hamiltonian(s["h"], s["eri"], s["na"], s["nb"])
    keys = np.array([int_to_words(int(b)) for b in basis], dtype=np.uint64)
    a = _amps(s, s["prm"], samples=keys)
    psi = a["sign"] * np.exp(a["logabs"])
    out = oracle.eloc(s["K"], s["na"], s["nb"], s["h"], s["eri"], s["chi"], s["pp"], s["pi"], s["nh"], s["prm"],
                      keys, ising=True)
    np.testing.assert_allclose(out["eloc"], (H @ psi) / psi, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(out["fsq"], np.exp(2 * a["lf"]), rtol=1e-13)
