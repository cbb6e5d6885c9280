"""Pins of the oracle's VMC step pieces: the reweighted gradient of Sec. 2.3
Eq. (19) against finite differences of the exact energy over a whole sector,
and AdamW against torch.optim.AdamW."""
import numpy as np
import pytest
import torch

import oracle
from bruteforce import dense_hamiltonian, int_to_words
from paper_2507_19276_amd import workloads as W


def test_adamw_matches_torch():
    rng = np.random.default_rng(3)
    n = 37
    p0 = rng.standard_normal(n)
    lr, b1, b2, eps, wd = 3e-2, 0.9, 0.999, 1e-8, 0.05
    pt = torch.nn.Parameter(torch.tensor(p0, dtype=torch.float64))
    opt = torch.optim.AdamW([pt], lr=lr, betas=(b1, b2), eps=eps, weight_decay=wd)
    p, m, v = p0.copy(), np.zeros(n), np.zeros(n)
    for t in range(1, 8):
        g = rng.standard_normal(n) * (10.0 ** rng.integers(-3, 2))
        pt.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = oracle.adamw(p, g, m, v, t, lr, b1, b2, eps, wd)
        np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("nh,ising", [(0, False), (4, False), (3, True)])
def test_reweighted_gradient_is_the_exact_gradient(nh, ising):
    """With the sample weights equal to Phi^2 over the whole sector and eps = 0,
    the estimator of Eq. (19) is the exact gradient of <Psi|H|Psi>/<Psi|Psi>."""
    K, na, nb, chi = 6, 3, 3, 3
    h, eri = W.chain_integrals(K, 41)
    pp, pi = W.graph_nn_nnn(K)
    prm = W.ansatz_params(K, chi, pp, pi, nh, 42, corr_scale=0.3, ising=ising)
    basis, H = dense_hamiltonian(h, eri, na, nb)
    keys = np.array([int_to_words(int(b)) for b in basis], dtype=np.uint64)

    def energy(p):
        a = oracle.amplitudes(K, chi, na, nb, pp, pi, nh, p, keys, ising=ising)
        psi = a["sign"] * np.exp(a["logabs"])
        return psi @ H @ psi / (psi @ psi)

    a = oracle.amplitudes(K, chi, na, nb, pp, pi, nh, prm, keys, ising=ising)
    phi2 = np.exp(2 * a["lphi"])
    out = oracle.eloc(K, na, nb, h, eri, chi, pp, pi, nh, prm, keys, ising=ising)
    cot, E = oracle.reweighted_cotangent(phi2, out["etnum"], out["fsq"])
    assert abs(E - energy(prm)) < 1e-11
    g = oracle.grad(K, chi, na, nb, pp, pi, nh, prm, keys, cot, ising=ising)
    rng = np.random.default_rng(5)
    idx = rng.choice(prm.size, 40, replace=False)
    hs = 1e-6
    for k in idx:
        p1, p2 = prm.copy(), prm.copy()
        p1[k] += hs
        p2[k] -= hs
        fd = (energy(p1) - energy(p2)) / (2 * hs)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(fd), 1e-3), (k, fd, g[k])


def test_cotangent_without_correlator_is_plain_vmc():
    """f = 1: cot_n = 2 c_n (E_loc(n) - <E>) / sum c (Eq. (7))."""
    rng = np.random.default_rng(8)
    c = rng.integers(1, 5, 20).astype(float)
    el = rng.standard_normal(20)
    cot, E = oracle.reweighted_cotangent(c, el, np.ones(20))
    Eb = (c * el).sum() / c.sum()
    assert abs(E - Eb) < 1e-15
    np.testing.assert_allclose(cot, 2 * c * (el - Eb) / c.sum(), rtol=1e-14, atol=1e-16)
