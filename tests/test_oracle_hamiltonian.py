"""Pins of the oracle's Hamiltonian machinery (Sec. 2.1 Eq. (2), Slater-Condon
rules of Sec. 2.4) against operator algebra that uses no Slater-Condon rule."""
import math

import numpy as np
import pytest

import oracle
from bruteforce import apply_hamiltonian, dense_hamiltonian, int_to_words, words_to_int
from paper_2507_19276_amd import workloads as W


def n_conn_closed_form(K, na, nb):
    singles = na * (K - na) + nb * (K - nb)
    same = math.comb(na, 2) * math.comb(K - na, 2) + math.comb(nb, 2) * math.comb(K - nb, 2)
    opp = na * (K - na) * nb * (K - nb)
    return singles + same + opp


@pytest.fixture(scope="module")
def c1():
    return W.make_workload("c1")


def test_philox_known_answers():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    n = 0
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        out = oracle.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]
        n += 1
    assert n == 3


def test_integral_symmetries():
    for name in ("c1", "c2", "c4a", "c4b"):
        w = W.make_workload(name, n_samples=4)
        e = w.eri
        assert np.array_equal(w.h, w.h.T)
        for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (1, 0, 3, 2), (3, 2, 1, 0)]:
            assert np.array_equal(e, e.transpose(perm)), (name, perm)


def test_dense_fci_matches_slater_condon(c1):
    """Every oracle row (diagonal + connected) equals the Jordan-Wigner matrix."""
    w = c1
    basis, H = dense_hamiltonian(w.h, w.eri, w.n_alpha, w.n_beta, e_core=0.37)
    assert len(basis) == 400
    pos = {int(b): k for k, b in enumerate(basis)}
    samples = np.array([int_to_words(int(b)) for b in basis], dtype=np.uint64)
    diag = oracle.hdiag(w.K, w.n_alpha, w.n_beta, w.h, w.eri, samples, e_core=0.37)
    np.testing.assert_allclose(diag, np.diag(H), rtol=0, atol=1e-12)
    for k, b in enumerate(basis):
        m, hv = oracle.connected(w.K, w.n_alpha, w.n_beta, w.h, w.eri, samples[k])
        assert len(m) == n_conn_closed_form(6, 3, 3) == 117
        row = np.zeros(len(basis))
        for mm, v in zip(m, hv):
            j = pos[words_to_int(mm)]
            assert row[j] == 0.0, "each connected determinant appears once"
            row[j] = v
        off = H[:, k].copy()
        off[k] = 0.0
        np.testing.assert_allclose(row, off, rtol=0, atol=1e-12)


@pytest.mark.parametrize("name,nsamp", [("c2", 2), ("c4a", 2), ("c4b", 2)])
def test_term_by_term_rows(name, nsamp):
    """Rows for K = 18-20 against H applied term by term to the determinant."""
    w = W.make_workload(name, n_samples=nsamp)
    for s in w.samples:
        n = words_to_int(s)
        ref = apply_hamiltonian(w.h, w.eri, n)
        m, hv = oracle.connected(w.K, w.n_alpha, w.n_beta, w.h, w.eri, s)
        got = {words_to_int(mm): v for mm, v in zip(m, hv) if v != 0.0}
        assert len(m) == n_conn_closed_form(w.K, w.n_alpha, w.n_beta)
        d = oracle.hdiag(w.K, w.n_alpha, w.n_beta, w.h, w.eri, s[None])[0]
        assert abs(ref.pop(n) - d) < 1e-11
        assert set(got) == set(ref)
        for key in got:
            assert abs(got[key] - ref[key]) < 1e-12


@pytest.mark.slow
def test_term_by_term_two_words():
    """K = 36 (spin orbitals beyond bit 63 live in the second word)."""
    h, eri = W.chain_integrals(36, 99)
    s = W.random_onvs(36, 18, 18, 1, 7)[0]
    n = words_to_int(s)
    ref = apply_hamiltonian(h, eri, n)
    m, hv = oracle.connected(36, 18, 18, h, eri, s)
    got = {words_to_int(mm): v for mm, v in zip(m, hv) if v != 0.0}
    ref.pop(n)
    assert set(got) == set(ref)
    assert max(abs(got[k] - ref[k]) for k in got) < 1e-12


def test_hermiticity():
    w = W.make_workload("c2", n_samples=3)
    for s in w.samples:
        m, hv = oracle.connected(w.K, w.n_alpha, w.n_beta, w.h, w.eri, s)
        n = words_to_int(s)
        for idx in (0, 5, 150, 300, 4000, 9000, len(m) - 1):
            mm, hnm = m[idx], hv[idx]
            m2, h2 = oracle.connected(w.K, w.n_alpha, w.n_beta, w.h, w.eri, mm)
            back = {words_to_int(x): v for x, v in zip(m2, h2)}
            assert back[n] == hnm


def test_connected_counts_closed_form():
    for K, na, nb, expect in [(6, 3, 3, 117), (20, 10, 10, 14250), (20, 15, 15, 7875),
                              (18, 9, 9, 9315), (12, 6, 6, 1818)]:
        assert n_conn_closed_form(K, na, nb) == expect
        h, eri = W.chain_integrals(K, 5)
        s = W.random_onvs(K, na, nb, 1, 3)[0]
        m, _ = oracle.connected(K, na, nb, h, eri, s)
        assert len(m) == expect
        assert len({words_to_int(x) for x in m}) == expect


def test_invalid_sample_rejected(c1):
    bad = np.array([[0b111, 0]], dtype=np.uint64)   # 2 alpha + 1 beta electrons
    with pytest.raises(ValueError):
        oracle.hdiag(6, 3, 3, c1.h, c1.eri, bad)
