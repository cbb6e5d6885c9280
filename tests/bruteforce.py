"""Brute-force references that pin the oracle without sharing its method.

* dense_hamiltonian: the second-quantised Hamiltonian of Sec. 2.1 Eq. (2)
  built as a sparse matrix over the full Fock space from Jordan-Wigner
  annihilators, then restricted to one (n_alpha, n_beta) sector.  No
  Slater-Condon rule is used: every term h_PQ a+_P a_Q and
  1/4 <PQ||RS> a+_P a+_Q a_S a_R is a matrix product.
* apply_hamiltonian: the same Hamiltonian applied term by term to a single
  determinant (Python integers as bit strings), for orbital counts where the
  Fock space is too large to build.

Sign convention: basis state n (an integer, bit P = x_P) is
prod_{P ascending} (a+_P)^{x_P} |vac>, so a_P |n> = (-1)^{#occupied Q<P} |n - P>.
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np
import scipy.sparse as sp


def spin_orbital_integrals(h: np.ndarray, eri: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """h_PQ = h_pq [sP=sQ]; anti[P,Q,R,S] = <PQ|RS> - <PQ|SR>, <PQ|RS> = (pr|qs) [sP=sR][sQ=sS]."""
    K = h.shape[0]
    n = 2 * K
    sp_ = np.arange(n) // 2
    sg = np.arange(n) % 2
    hso = h[sp_[:, None], sp_[None, :]] * (sg[:, None] == sg[None, :])
    P, Q, R, S = np.meshgrid(*([np.arange(n)] * 4), indexing="ij")
    g = eri[sp_[P], sp_[R], sp_[Q], sp_[S]] * (sg[P] == sg[R]) * (sg[Q] == sg[S])
    gx = eri[sp_[P], sp_[S], sp_[Q], sp_[R]] * (sg[P] == sg[S]) * (sg[Q] == sg[R])
    return hso, g - gx


def jw_annihilators(n_so: int):
    dim = 1 << n_so
    idx = np.arange(dim, dtype=np.int64)
    ops = []
    for P in range(n_so):
        src = idx[((idx >> P) & 1) == 1]
        dst = src ^ (1 << P)
        below = np.bitwise_count((src & ((1 << P) - 1)).astype(np.uint64)).astype(np.int64)
        sign = np.where(below % 2 == 1, -1.0, 1.0)
        ops.append(sp.csr_matrix((sign, (dst, src)), shape=(dim, dim)))
    return ops


def dense_hamiltonian(h: np.ndarray, eri: np.ndarray, na: int, nb: int, e_core: float = 0.0):
    """(sector basis as ints ascending, dense H over the sector)."""
    K = h.shape[0]
    n = 2 * K
    assert n <= 16, "full Fock space only for tiny systems"
    hso, anti = spin_orbital_integrals(h, eri)
    a = jw_annihilators(n)
    ad = [x.T.tocsr() for x in a]
    dim = 1 << n
    H = sp.csr_matrix((dim, dim))
    for P in range(n):
        for Q in range(n):
            if hso[P, Q] != 0.0:
                H = H + hso[P, Q] * (ad[P] @ a[Q])
    pair_c = {(P, Q): (ad[P] @ ad[Q]).tocsr() for P in range(n) for Q in range(n) if P != Q}
    for P in range(n):
        for Q in range(n):
            if P == Q:
                continue
            acc = sp.csr_matrix((dim, dim))
            for R in range(n):
                for S in range(n):
                    if R == S or anti[P, Q, R, S] == 0.0:
                        continue
                    # a_S a_R = (a+_R a+_S)^T
                    acc = acc + anti[P, Q, R, S] * pair_c[(R, S)].T
            H = H + 0.25 * (pair_c[(P, Q)] @ acc)
    idx = np.arange(dim)
    ca = np.zeros(dim, dtype=np.int64)
    cb = np.zeros(dim, dtype=np.int64)
    for p in range(K):
        ca += (idx >> (2 * p)) & 1
        cb += (idx >> (2 * p + 1)) & 1
    basis = idx[(ca == na) & (cb == nb)]
    Hs = H[basis][:, basis].toarray() + e_core * np.eye(len(basis))
    return basis, Hs


def _annih(n: int, P: int):
    if not (n >> P) & 1:
        return 0, 0
    s = -1 if bin(n & ((1 << P) - 1)).count("1") % 2 else 1
    return s, n ^ (1 << P)


def _creat(n: int, P: int):
    if (n >> P) & 1:
        return 0, 0
    s = -1 if bin(n & ((1 << P) - 1)).count("1") % 2 else 1
    return s, n | (1 << P)


def apply_hamiltonian(h: np.ndarray, eri: np.ndarray, n: int, e_core: float = 0.0) -> Dict[int, float]:
    """H|n> term by term: {m: <m|H|n>} over all m reached (zeros kept out)."""
    K = h.shape[0]
    nso = 2 * K
    out: Dict[int, float] = {}

    def add(m, v):
        out[m] = out.get(m, 0.0) + v

    add(n, e_core)
    occ = [P for P in range(nso) if (n >> P) & 1]
    for P in range(nso):
        for Q in occ:
            if P % 2 != Q % 2:
                continue
            hv = float(h[P // 2, Q // 2])
            s1, m1 = _annih(n, Q)
            s2, m2 = _creat(m1, P)
            if s2:
                add(m2, hv * s1 * s2)
    # two-body: only R, S occupied contribute; P, Q must be empty afterwards
    for R in occ:
        for S in occ:
            if R == S:
                continue
            s1, m1 = _annih(n, R)
            s2, m2 = _annih(m1, S)
            empty = [P for P in range(nso) if not (m2 >> P) & 1]
            for Q in empty:
                s3, m3 = _creat(m2, Q)
                for P in empty:
                    if P == Q:
                        continue
                    s4, m4 = _creat(m3, P)
                    # <PQ||RS> = <PQ|RS> - <PQ|SR>
                    g1 = eri[P // 2, R // 2, Q // 2, S // 2] if (P % 2 == R % 2 and Q % 2 == S % 2) else 0.0
                    g2 = eri[P // 2, S // 2, Q // 2, R // 2] if (P % 2 == S % 2 and Q % 2 == R % 2) else 0.0
                    v = g1 - g2
                    if v != 0.0:
                        add(m4, 0.25 * v * s1 * s2 * s3 * s4)
    return {m: v for m, v in out.items() if v != 0.0}


def words_to_int(w) -> int:
    return int(w[0]) | (int(w[1]) << 64)


def int_to_words(x: int):
    return (x & 0xFFFFFFFFFFFFFFFF, x >> 64)
