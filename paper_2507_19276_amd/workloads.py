"""Seeded synthetic inputs for the semi-stochastic local-energy path.

This module only *makes inputs*: integrals, graphs, packed ansatz parameters,
occupation-number vectors and uniform random numbers.  It holds none of the
method's arithmetic (no Hamiltonian elements, no amplitudes, no local
energies), so that the FP64 oracle and the HIP library can both be fed from it
without sharing any computation.

The paper's own workloads (H-chains from PySCF, the Fe2S2 CAS(30e,20o) FCIDUMP,
the 3x3x2 H18 cluster, all in Sec. 4) need integrals and optimised parameters
that are not available; the generators below reproduce their *shapes*:

* chain-like integrals: magnitudes decay exponentially with the index spread,
  decay length 2 (H-chain in orthonormalised atomic orbitals, Sec. 4.1);
* dense integrals: h and (pq|rs) ~ N(0, 0.1) with no decay (Fe2S2-like active
  space, Sec. 4.2);
* lattice integrals: decay with the lattice distance of a 3x3x2 cluster
  (H18, Sec. 4.3).

Conventions (shared by every consumer):

* spatial orbitals p = 0..K-1; spin orbital P = 2p + sigma (sigma 0 = alpha,
  1 = beta), i.e. the interleaved order of Sec. 3 (the x_0 x_1 ... listing);
* an ONV is two little-endian uint64 words: bit P of the 128-bit integer is
  x_P (so K <= 64);
* chemist integrals eri[p, q, r, s] = (pq|rs), real, 8-fold symmetric;
* the BDG graph is given by parent lists N(i) (parents have lower index),
  stored as CSR (parent_ptr[K+1], parent_idx[...]) with ascending parents;
* packed parameter layout, per site i ascending: for each parent j in N(i)
  ascending, for local state s = 0..3, the chi x chi matrix M_ij^s row-major
  (h_out[u] = sum_k M[u, k] h_in[k]); then v_i^s (4 x chi), eta_i (chi),
  w_i (chi), c_i (1).  After all sites the cos-RBM correlator: b (N_h) then
  W (N_h x 2K, row-major, column P = spin orbital P); with the Ising-RBM
  correlator, then W2 (N_h x 2K x 2K, row-major: W2[k, P, Q]).  With the
  BDG-TensorRNN term, last, per site i ascending with d_i >= 2 parents: the
  factor matrices K^(0) (output mode) and K^(1..d) (one per parent, ascending),
  each chi x chi' row-major, then the cores U^s (s = 0..3), each chi'^(d+1)
  with index order [i', a_1, ..., a_d]; chi' = ceil(chi^(2/(d+1))).
  With complex parameters the same order, M, v, w and c complex and stored
  as (re, im) pairs (M: 4 x chi x chi pairs, v: 4 x chi pairs, w: chi pairs,
  c: one pair), eta real; the correlator block stays real.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

SEED_BASE = 20250725


# ---------------------------------------------------------------------------
# graphs (parent lists, edges oriented from lower to higher site index)
# ---------------------------------------------------------------------------

def _csr_from_parents(parents: Sequence[Sequence[int]]) -> Tuple[np.ndarray, np.ndarray]:
    ptr = [0]
    idx: List[int] = []
    for i, ps in enumerate(parents):
        ps = sorted(set(int(p) for p in ps))
        assert all(0 <= p < i for p in ps), "parents must precede the site"
        idx.extend(ps)
        ptr.append(len(idx))
    return np.asarray(ptr, dtype=np.int32), np.asarray(idx, dtype=np.int32)


def graph_chain(K: int) -> Tuple[np.ndarray, np.ndarray]:
    """1D MPS-RNN: site i has the single parent i-1 (BDG(1) on a chain)."""
    return _csr_from_parents([[i - 1] if i > 0 else [] for i in range(K)])


def graph_nn_nnn(K: int) -> Tuple[np.ndarray, np.ndarray]:
    """Nearest + next-nearest neighbour chain: parents {i-1, i-2}."""
    return _csr_from_parents([[j for j in (i - 1, i - 2) if j >= 0] for i in range(K)])


def lattice_coords(dims: Tuple[int, int, int]) -> np.ndarray:
    """Site (x*ny + y)*nz + z of an nx x ny x nz lattice -> (x, y, z)."""
    nx, ny, nz = dims
    out = np.zeros((nx * ny * nz, 3), dtype=np.int64)
    for x in range(nx):
        for y in range(ny):
            for z in range(nz):
                out[(x * ny + y) * nz + z] = (x, y, z)
    return out


def graph_lattice(dims: Tuple[int, int, int]) -> Tuple[np.ndarray, np.ndarray]:
    """Nearest-neighbour lattice edges oriented low -> high site index."""
    xyz = lattice_coords(dims)
    K = len(xyz)
    parents: List[List[int]] = [[] for _ in range(K)]
    for i in range(K):
        for j in range(i):
            if np.abs(xyz[i] - xyz[j]).sum() == 1:
                parents[i].append(j)
    return _csr_from_parents(parents)


def max_parent_offset(parent_ptr: np.ndarray, parent_idx: np.ndarray) -> int:
    K = len(parent_ptr) - 1
    off = 0
    for i in range(K):
        for e in range(parent_ptr[i], parent_ptr[i + 1]):
            off = max(off, i - int(parent_idx[e]))
    return off


# ---------------------------------------------------------------------------
# integrals
# ---------------------------------------------------------------------------

def _canonical_index(K: int) -> np.ndarray:
    """For every (p,q,r,s) the flat index of its 8-fold canonical representative."""
    p, q, r, s = np.meshgrid(*([np.arange(K)] * 4), indexing="ij")
    a, b = np.maximum(p, q), np.minimum(p, q)
    c, d = np.maximum(r, s), np.minimum(r, s)
    ab = a * (a + 1) // 2 + b
    cd = c * (c + 1) // 2 + d
    swap = ab < cd
    A = np.where(swap, c, a)
    B = np.where(swap, d, b)
    C = np.where(swap, a, c)
    D = np.where(swap, b, d)
    return ((A * K + B) * K + C) * K + D


def _symmetrize8(raw: np.ndarray) -> np.ndarray:
    K = raw.shape[0]
    flat = raw.reshape(-1)
    return flat[_canonical_index(K)].reshape(K, K, K, K).copy()


def chain_integrals(K: int, seed: int, ell: float = 2.0) -> Tuple[np.ndarray, np.ndarray]:
    """1D-chain-like integrals: h_pq ~ N(0, sigma = exp(-|p-q|/ell)) and
    (pq|rs) = z * exp(-spread/ell), z ~ N(0,1), spread = max - min of {p,q,r,s};
    both exactly symmetric (h) / 8-fold symmetric (eri)."""
    rng = np.random.default_rng(seed)
    idx = np.arange(K)
    dist = np.abs(idx[:, None] - idx[None, :])
    h = rng.standard_normal((K, K)) * np.exp(-dist / ell)
    h = np.triu(h) + np.triu(h, 1).T
    z = rng.standard_normal((K, K, K, K))
    p, q, r, s = np.meshgrid(idx, idx, idx, idx, indexing="ij")
    mx = np.maximum(np.maximum(p, q), np.maximum(r, s))
    mn = np.minimum(np.minimum(p, q), np.minimum(r, s))
    eri = _symmetrize8(z * np.exp(-(mx - mn) / ell))
    return np.ascontiguousarray(h), np.ascontiguousarray(eri)


def dense_integrals(K: int, seed: int, sigma: float = 0.1) -> Tuple[np.ndarray, np.ndarray]:
    """Dense, non-decaying integrals: h_pq, (pq|rs) ~ N(0, sigma) (sigma = std)."""
    rng = np.random.default_rng(seed)
    h = rng.standard_normal((K, K)) * sigma
    h = np.triu(h) + np.triu(h, 1).T
    eri = _symmetrize8(rng.standard_normal((K, K, K, K)) * sigma)
    return np.ascontiguousarray(h), np.ascontiguousarray(eri)


def lattice_integrals(dims: Tuple[int, int, int], seed: int, ell: float = 2.0) -> Tuple[np.ndarray, np.ndarray]:
    """Integrals whose magnitude decays with Manhattan lattice distance:
    h_pq ~ N(0, exp(-d(p,q)/ell)); (pq|rs) = z exp(-D/ell) with D the largest
    pairwise distance among {p,q,r,s}."""
    rng = np.random.default_rng(seed)
    xyz = lattice_coords(dims)
    K = len(xyz)
    d = np.abs(xyz[:, None, :] - xyz[None, :, :]).sum(-1)
    h = rng.standard_normal((K, K)) * np.exp(-d / ell)
    h = np.triu(h) + np.triu(h, 1).T
    z = rng.standard_normal((K, K, K, K))
    idx = np.arange(K)
    p, q, r, s = np.meshgrid(idx, idx, idx, idx, indexing="ij")
    D = np.maximum.reduce([d[p, q], d[p, r], d[p, s], d[q, r], d[q, s], d[r, s]])
    eri = _symmetrize8(z * np.exp(-D / ell))
    return np.ascontiguousarray(h), np.ascontiguousarray(eri)


# ---------------------------------------------------------------------------
# ansatz parameters
# ---------------------------------------------------------------------------

def tucker_rank(chi: int, d: int) -> int:
    """Shape of the tensor block: the smallest c with c^(d+1) >= chi^2."""
    c = 1
    while c ** (d + 1) < chi * chi:
        c += 1
    return c


def tensor_block_sizes(K: int, chi: int, parent_ptr: np.ndarray) -> List[Tuple[int, int, int]]:
    """(site, d, chi') of every site carrying a tensor term (d >= 2)."""
    out = []
    for i in range(K):
        d = int(parent_ptr[i + 1] - parent_ptr[i])
        if d >= 2:
            out.append((i, d, tucker_rank(chi, d)))
    return out


def n_params(K: int, chi: int, parent_ptr: np.ndarray, n_hidden: int, ising: bool = False,
             tensor: bool = False, cplx: bool = False) -> int:
    sum_d = int(parent_ptr[-1])
    corr = n_hidden * (2 * K + 1) + (n_hidden * 4 * K * K if ising else 0)
    if cplx:
        # M, v, w, c complex (two reals each), eta real
        assert not tensor
        return sum_d * 8 * chi * chi + K * (8 * chi + chi + 2 * chi + 2) + (corr if n_hidden else 0)
    tens = sum((d + 1) * chi * q + 4 * q ** (d + 1) for _, d, q in tensor_block_sizes(K, chi, parent_ptr)) \
        if tensor else 0
    return sum_d * 4 * chi * chi + K * (4 * chi + chi + chi + 1) + (corr if n_hidden else 0) + tens


def ansatz_params(K: int, chi: int, parent_ptr: np.ndarray, parent_idx: np.ndarray,
                  n_hidden: int, seed: int, corr_scale: float = 0.1, ising: bool = False,
                  tensor: bool = False, tensor_scale: float = 0.1, cplx: bool = False) -> np.ndarray:
    """Random-init parameters in the packed layout (module docstring):
    M ~ N(0, var 1/(chi*max(d_i,1))), v ~ N(0,1), eta ~ U[0.5,1.5], w, c ~ N(0,1),
    correlator b, W ~ N(0, corr_scale^2), Ising W2 ~ N(0, corr_scale^2 / K) (its
    ~K^2 occupied pairs then spread theta about as much as W's ~K terms);
    tensor factors K ~ N(0, 1/chi), cores U ~ N(0, tensor_scale^2 / chi'^d) (the term is quadratic
    in the hidden states at two parents, so random states can grow without
    bound along a K = 20 chain: at tensor_scale = 0.3 some reach |h| ~ 1e79,
    beyond FP32; at 0.1 the largest |h| is ~25 and the term still shifts
    log|Phi| by ~0.15).  With cplx: M, v, w, c complex, stored as (re, im)
    pairs, each part with half the variance of the real case (so that |M|^2,
    |v|^2 have the real case's mean); eta as in the real case."""
    rng = np.random.default_rng(seed)
    out: List[np.ndarray] = []
    if cplx:
        assert not tensor
        h = math.sqrt(0.5)
        for i in range(K):
            d = int(parent_ptr[i + 1] - parent_ptr[i])
            std = 1.0 / math.sqrt(chi * max(d, 1))
            for _ in range(d):
                out.append(rng.standard_normal(8 * chi * chi) * (std * h))   # M (re, im)
            out.append(rng.standard_normal(8 * chi) * h)      # v
            out.append(rng.uniform(0.5, 1.5, chi))            # eta
            out.append(rng.standard_normal(2 * chi) * h)      # w
            out.append(rng.standard_normal(2) * h)            # c
        if n_hidden:
            out.append(rng.standard_normal(n_hidden) * corr_scale)
            out.append(rng.standard_normal(n_hidden * 2 * K) * corr_scale)
            if ising:
                out.append(rng.standard_normal(n_hidden * 4 * K * K) * (corr_scale / math.sqrt(K)))
        p = np.concatenate(out).astype(np.float64)
        assert p.size == n_params(K, chi, parent_ptr, n_hidden, ising, False, True)
        return p
    for i in range(K):
        d = int(parent_ptr[i + 1] - parent_ptr[i])
        std = 1.0 / math.sqrt(chi * max(d, 1))
        for _ in range(d):
            out.append(rng.standard_normal(4 * chi * chi) * std)
        out.append(rng.standard_normal(4 * chi))          # v
        out.append(rng.uniform(0.5, 1.5, chi))            # eta
        out.append(rng.standard_normal(chi))              # w
        out.append(rng.standard_normal(1))                # c
    if n_hidden:
        out.append(rng.standard_normal(n_hidden) * corr_scale)            # b
        out.append(rng.standard_normal(n_hidden * 2 * K) * corr_scale)    # W
        if ising:
            out.append(rng.standard_normal(n_hidden * 4 * K * K) * (corr_scale / math.sqrt(K)))   # W2
    if tensor:
        for _, d, q in tensor_block_sizes(K, chi, parent_ptr):
            out.append(rng.standard_normal((d + 1) * chi * q) / math.sqrt(chi))                 # K^(0..d)
            out.append(rng.standard_normal(4 * q ** (d + 1)) * (tensor_scale / math.sqrt(q ** d)))   # U^s
    p = np.concatenate(out).astype(np.float64)
    assert p.size == n_params(K, chi, parent_ptr, n_hidden, ising, tensor)
    return p


# ---------------------------------------------------------------------------
# occupation-number vectors
# ---------------------------------------------------------------------------

def onv_from_occ(K: int, occ_a: Sequence[int], occ_b: Sequence[int]) -> Tuple[int, int]:
    v = 0
    for p in occ_a:
        v |= 1 << (2 * p)
    for p in occ_b:
        v |= 1 << (2 * p + 1)
    return v & 0xFFFFFFFFFFFFFFFF, v >> 64


def onv_to_int(words) -> int:
    return int(words[0]) | (int(words[1]) << 64)


def random_onvs(K: int, n_alpha: int, n_beta: int, N: int, seed: int,
                unique: bool = True) -> np.ndarray:
    """N valid ONVs (exactly n_alpha alpha and n_beta beta electrons), drawn
    uniformly; with unique=True all rows are distinct.  Returns uint64 [N, 2]."""
    rng = np.random.default_rng(seed)
    seen = set()
    rows: List[Tuple[int, int]] = []
    total = math.comb(K, n_alpha) * math.comb(K, n_beta)
    if unique and N > total:
        raise ValueError(f"only {total} distinct ONVs exist")
    while len(rows) < N:
        m = N - len(rows)
        ka = np.argsort(rng.random((m, K)), axis=1)[:, :n_alpha]
        kb = np.argsort(rng.random((m, K)), axis=1)[:, :n_beta]
        for a, b in zip(ka, kb):
            w = onv_from_occ(K, a.tolist(), b.tolist())
            if unique:
                if w in seen:
                    continue
                seen.add(w)
            rows.append(w)
            if len(rows) == N:
                break
    return np.asarray(rows, dtype=np.uint64).reshape(N, 2)


def all_onvs(K: int, n_alpha: int, n_beta: int) -> np.ndarray:
    """Every ONV of the (n_alpha, n_beta) sector, in increasing integer order."""
    from itertools import combinations
    out = []
    for a in combinations(range(K), n_alpha):
        for b in combinations(range(K), n_beta):
            out.append(onv_from_occ(K, a, b))
    arr = np.asarray(out, dtype=np.uint64).reshape(-1, 2)
    key = [onv_to_int(r) for r in arr]
    return arr[np.argsort(np.asarray(key, dtype=object))]


def uniforms(shape, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).random(shape)


# seed of the exact draws from Phi^2 that make a workload's sample batch
# (the workload's seed plus this offset)
PHI2_SEED_OFFSET = 11


def draw_until_unique(draw, n_unique: int, max_draws: int = 1 << 22):
    """Sample batch of n_unique distinct ONVs from a counter-keyed sampler.

    draw(n) must return (unique ONVs, counts) of the draws 0 .. n-1; a
    counter-keyed sampler (each draw a function of its index) only appends
    draws when n grows.  Starting from n = n_unique, each round adds the
    number of ONVs still missing, so no round can overshoot: the loop stops at
    the smallest n whose draws hold n_unique distinct ONVs (or at max_draws).
    Returns (ONVs, counts, n) as draw returned them; fewer than n_unique ONVs
    only if max_draws was reached.  This is bookkeeping around a sampler that
    is passed in; no draw is made here."""
    n = int(n_unique)
    while True:
        u, c = draw(n)
        if len(u) >= n_unique or n >= max_draws:
            return u, c, n
        n = min(n + n_unique - len(u), int(max_draws))


def top_up(samples: np.ndarray, counts: np.ndarray, K: int, n_alpha: int, n_beta: int, N: int,
           seed: int):
    """Fill a batch of distinct ONVs up to N with uniform random valid ONVs not
    already in it (count 1 each): used only when the draws held fewer than N
    distinct ONVs.  Returns (samples, counts, number added)."""
    have = {onv_to_int(r) for r in samples}
    extra = []
    if len(samples) < N:
        pool = random_onvs(K, n_alpha, n_beta, min(4 * N, math.comb(K, n_alpha) * math.comb(K, n_beta)), seed)
        for r in pool:
            if onv_to_int(r) not in have:
                have.add(onv_to_int(r))
                extra.append(r)
                if len(samples) + len(extra) == N:
                    break
    if not extra:
        return samples, counts, 0
    return (np.vstack([samples, np.asarray(extra, dtype=np.uint64)]),
            np.concatenate([counts, np.ones(len(extra), dtype=counts.dtype)]), len(extra))


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    K: int
    n_alpha: int
    n_beta: int
    h: np.ndarray
    eri: np.ndarray
    e_core: float
    chi: int
    parent_ptr: np.ndarray
    parent_idx: np.ndarray
    n_hidden: int
    params: np.ndarray
    samples: np.ndarray
    eps: float
    n_eps: int
    seed: int
    precision: str
    ising: bool = False
    tensor: bool = False
    cplx: bool = False

    @property
    def n_samples(self) -> int:
        return int(self.samples.shape[0])


def _graph(kind: str, K: int):
    if kind == "chain":
        return graph_chain(K)
    if kind == "nnn":
        return graph_nn_nnn(K)
    if kind == "lattice332":
        return graph_lattice((3, 3, 2))
    if kind == "lattice222":
        return graph_lattice((2, 2, 2))
    raise ValueError(kind)


def make_workload(name: str, n_samples: Optional[int] = None, seed_offset: int = 0) -> Workload:
    """The synthetic stand-ins for the paper's systems (module docstring).

    c1  K=6,  3a+3b, chain integrals, MPS-RNN chain chi=4, 256 samples, eps=0
    c2  K=20, 10a+10b, chain integrals, chain graph chi=16, 4096 unique samples,
        eps=1e-3, N_eps=64
    c3  K=50, 25a+25b, chain integrals, NN+NNN graph chi=32, cos-RBM N_h=100,
        16384 unique samples, eps=1e-2, N_eps=100
    c4a K=20, 15a+15b, dense N(0,0.1) integrals, NN+NNN chi=64, 8192 samples,
        eps=1e-2, N_eps=1000
    c4b K=18 on 3x3x2, 9a+9b, lattice integrals, lattice graph chi=64,
        8192 samples, eps=1e-2, N_eps=100
    c1i c1 with an Ising-RBM correlator, N_h = 2 N_v = 24
    c1t K=6, 3a+3b, NN+NNN graph, BDG-TensorRNN chi=4 (chi' = 3), 256 samples
    c8t K=8 on a 2x2x2 lattice (in-degrees up to 3), 4a+4b, BDG-TensorRNN chi=4
        (chi' = 3 at two parents, 2 at three), 256 samples
    c2t K=20, 10a+10b, chain integrals, NN+NNN graph, BDG(2)-TensorRNN chi=16
        (chi' = 7), 4096 unique samples, eps=1e-3, N_eps=64
    c2i c2 with an Ising-RBM correlator, N_h = 2 N_v = 80 (alpha = 2, as in
        Sec. 4), 4096 unique samples
    c1c c1 with complex parameters and a cos-RBM correlator, N_h = 12
    c2c c2 with complex parameters (chi = 16 complex units), 4096 unique samples
    """
    base = SEED_BASE + 1000 * seed_offset
    spec = {
        "c1": dict(K=6, ne=(3, 3), integ="chain", graph="chain", chi=4, nh=0, N=256, uniq=False,
                   eps=0.0, neps=0, prec="f64", s=1),
        "c2": dict(K=20, ne=(10, 10), integ="chain", graph="chain", chi=16, nh=0, N=4096, uniq=True,
                   eps=1e-3, neps=64, prec="f32", s=2),
        "c3": dict(K=50, ne=(25, 25), integ="chain", graph="nnn", chi=32, nh=100, N=16384, uniq=True,
                   eps=1e-2, neps=100, prec="bf16", s=3),
        "c4a": dict(K=20, ne=(15, 15), integ="dense", graph="nnn", chi=64, nh=0, N=8192, uniq=True,
                    eps=1e-2, neps=1000, prec="f32", s=4),
        "c4b": dict(K=18, ne=(9, 9), integ="lattice", graph="lattice332", chi=64, nh=0, N=8192,
                    uniq=True, eps=1e-2, neps=100, prec="f32", s=5),
        "c1i": dict(K=6, ne=(3, 3), integ="chain", graph="chain", chi=4, nh=24, N=256, uniq=False,
                    eps=0.0, neps=0, prec="f64", s=6, ising=True),
        "c2i": dict(K=20, ne=(10, 10), integ="chain", graph="chain", chi=16, nh=80, N=4096, uniq=True,
                    eps=1e-3, neps=64, prec="f32", s=7, ising=True),
        "c1t": dict(K=6, ne=(3, 3), integ="chain", graph="nnn", chi=4, nh=0, N=256, uniq=False,
                    eps=0.0, neps=0, prec="f64", s=8, tensor=True),
        "c8t": dict(K=8, ne=(4, 4), integ="lattice222", graph="lattice222", chi=4, nh=0, N=256, uniq=False,
                    eps=0.0, neps=0, prec="f64", s=9, tensor=True),
        "c2t": dict(K=20, ne=(10, 10), integ="chain", graph="nnn", chi=16, nh=0, N=4096, uniq=True,
                    eps=1e-3, neps=64, prec="f32", s=10, tensor=True),
        "c1c": dict(K=6, ne=(3, 3), integ="chain", graph="chain", chi=4, nh=12, N=256, uniq=False,
                    eps=0.0, neps=0, prec="f64", s=11, cplx=True),
        "c2c": dict(K=20, ne=(10, 10), integ="chain", graph="chain", chi=16, nh=0, N=4096, uniq=True,
                    eps=1e-3, neps=64, prec="f32", s=12, cplx=True),
    }[name]
    ising = spec.get("ising", False)
    tensor = spec.get("tensor", False)
    cplx = spec.get("cplx", False)
    K = spec["K"]
    seed = base + 100 * spec["s"]
    if spec["integ"] == "chain":
        h, eri = chain_integrals(K, seed + 1)
    elif spec["integ"] == "dense":
        h, eri = dense_integrals(K, seed + 1)
    elif spec["integ"] == "lattice222":
        h, eri = lattice_integrals((2, 2, 2), seed + 1)
    else:
        h, eri = lattice_integrals((3, 3, 2), seed + 1)
    pp, pi = _graph(spec["graph"], K)
    params = ansatz_params(K, spec["chi"], pp, pi, spec["nh"], seed + 2, ising=ising, tensor=tensor, cplx=cplx)
    N = spec["N"] if n_samples is None else n_samples
    na, nb = spec["ne"]
    samples = random_onvs(K, na, nb, N, seed + 3, unique=spec["uniq"])
    return Workload(name=name, K=K, n_alpha=na, n_beta=nb, h=h, eri=eri, e_core=0.0,
                    chi=spec["chi"], parent_ptr=pp, parent_idx=pi, n_hidden=spec["nh"],
                    params=params, samples=samples, eps=spec["eps"], n_eps=spec["neps"],
                    seed=seed + 4, precision=spec["prec"], ising=ising, tensor=tensor, cplx=cplx)


def serving_instances(seed_offset: int = 0) -> List[Dict]:
    """The 12 serving instances: norb in {12,20,36,50} x chi in {16,32,64},
    half filling, chain-like integrals, NN+NNN graph, no correlator."""
    out = []
    base = SEED_BASE + 1000 * seed_offset + 7000
    for K in (12, 20, 36, 50):
        h, eri = chain_integrals(K, base + K)
        pp, pi = graph_nn_nnn(K)
        for chi in (16, 32, 64):
            out.append(dict(K=K, n_alpha=K // 2, n_beta=K // 2, h=h, eri=eri, chi=chi,
                            parent_ptr=pp, parent_idx=pi,
                            params=ansatz_params(K, chi, pp, pi, 0, base + 10 * K + chi)))
    return out


def serving_requests(n_requests: int, rate_hz: float, n_instances: int, seed: int,
                     n_min: int = 256, n_max: int = 16384):
    """Poisson arrivals (exponential gaps at rate_hz), an instance drawn
    uniformly, batch size floor(exp U[ln n_min, ln n_max])."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    t = np.cumsum(gaps) - gaps[0]
    inst = rng.integers(0, n_instances, n_requests)
    ns = np.floor(np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_requests))).astype(np.int64)
    return [dict(t=float(t[k]), instance=int(inst[k]), n=int(ns[k]), seed=int(seed * 1000 + k))
            for k in range(n_requests)]
