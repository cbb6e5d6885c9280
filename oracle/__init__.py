"""FP64 CPU oracle for the semi-stochastic local energy (arXiv:2507.19276).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py, never by the product library.  It shares no
code with the HIP path.  The arithmetic lives in oracle.cpp (plain loops,
FP64, no fused multiply-add); this module only marshals numpy arrays.

Every function returns plain numpy arrays.  Parameters, graphs and samples
use the conventions documented in paper_2507_19276_amd.workloads (the
input generators, which hold none of the method's arithmetic).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = C.c_double
_i = C.c_int
_i64 = C.c_int64
_u64 = C.c_uint64
_p = C.c_void_p


def use_library(path: str) -> None:
    """Load the oracle from another build of oracle.cpp (for instance one
    compiled for the host CPU by build.build(native=True)); call before any
    other function of this module."""
    global _LIB_PATH, _lib
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    _LIB_PATH = path


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    lib.or_philox4x32_10.argtypes = [_p, _p, _p]
    lib.or_proposal_weight.argtypes = [_d, _d]
    lib.or_proposal_weight.restype = _u64
    lib.or_scaled_draw.argtypes = [_p, _u64]
    lib.or_scaled_draw.restype = _u64
    lib.or_hdiag.argtypes = [_i, _i, _i, _p, _p, _d, _p, _i64, _p]
    lib.or_connected.argtypes = [_i, _i, _i, _p, _p, _d, _p, _p, _p, _i64]
    lib.or_connected.restype = _i64
    lib.or_n_params.argtypes = [_i, _i, _p, _i, _i]
    lib.or_n_params.restype = _i64
    lib.or_amplitudes.argtypes = [_i, _i, _i, _i, _p, _p, _i, _i, _p, _p, _i64, _p, _p, _p, _p, _p, _p, _p, _i]
    lib.or_sample.argtypes = [_i, _i, _i, _i, _p, _p, _i, _p, _p, _i64, _p]
    lib.or_sample_unique.argtypes = [_i, _i, _i, _i, _p, _p, _i, _p, _u64, _i64, _i64, _i64, _p, _p]
    lib.or_sample_unique.restype = _i64
    lib.or_grad.argtypes = [_i, _i, _i, _i, _p, _p, _i, _i, _p, _p, _i64, _p, _p, _i]
    lib.or_eloc.argtypes = [_i, _i, _i, _p, _p, _d, _i, _p, _p, _i, _i, _p, _p, _i64, _d, _i, _u64,
                            _u64, _i64, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _i, _d, _p, _p, _p, _i]
    lib.or_eloc_detail.argtypes = [_i, _i, _i, _p, _p, _d, _i, _p, _p, _i, _i, _p, _p, _i64, _d, _i,
                                   _u64, _u64, _p, _i64, _p, _p, _p, _p]
    lib.or_eloc_table.argtypes = [_i, _i, _i, _p, _p, _d, _p, _p, _i64, _p, _i64, _d, _i, _u64,
                                  _u64, _p, _i]
    lib.or_tucker_rank.argtypes = [_i, _i]
    lib.or_project_eta.argtypes = [_i, _i, _p, _i, _i, _p]
    lib.or_reweighted_cotangent.argtypes = [_i64, _p, _p, _p, _p, _p]
    lib.or_adamw.argtypes = [_i64, _p, _p, _p, _p, _i64, _d, _d, _d, _d, _d]
    lib.or_amplitudes_cx.argtypes = [_i, _i, _i, _i, _p, _p, _i, _i, _p, _p, _i64, _p, _p, _p, _p, _i]
    lib.or_grad_cx.argtypes = [_i, _i, _i, _i, _p, _p, _i, _i, _p, _p, _i64, _p, _p, _p, _i]
    lib.or_eloc_cx.argtypes = [_i, _i, _i, _p, _p, _d, _i, _p, _p, _i, _i, _p, _p, _i64, _d, _i, _u64,
                               _u64, _i64, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _i]
    lib.or_reweighted_cotangent_cx.argtypes = [_i64, _p, _p, _p, _p, _p, _p, _p]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u64a(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 of a 4-word counter under a 2-word key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().or_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def proposal_weight(absH: float, eps: float) -> int:
    return int(_load().or_proposal_weight(float(absH), float(eps)))


def scaled_draw(U_words, Q: int) -> int:
    u = np.ascontiguousarray(U_words, dtype=np.uint32)
    return int(_load().or_scaled_draw(_ptr(u), int(Q)))


def hdiag(K, na, nb, h, eri, samples, e_core=0.0) -> np.ndarray:
    s = _u64a(samples).reshape(-1, 2)
    out = np.zeros(len(s))
    h, eri = _f64(h), _f64(eri)
    rc = _load().or_hdiag(K, na, nb, _ptr(h), _ptr(eri), e_core, _ptr(s), len(s), _ptr(out))
    if rc != 0:
        raise ValueError("sample outside the (n_alpha, n_beta) sector")
    return out


def connected(K, na, nb, h, eri, sample, e_core=0.0):
    """(m[Nconn,2] uint64, H[Nconn]) in canonical rank order for one sample."""
    s = _u64a(sample).reshape(2)
    h, eri = _f64(h), _f64(eri)
    lib = _load()
    n = lib.or_connected(K, na, nb, _ptr(h), _ptr(eri), e_core, _ptr(s), None, None, 0)
    if n < 0:
        raise ValueError("sample outside the (n_alpha, n_beta) sector")
    m = np.zeros((n, 2), dtype=np.uint64)
    H = np.zeros(n)
    lib.or_connected(K, na, nb, _ptr(h), _ptr(eri), e_core, _ptr(s), _ptr(m), _ptr(H), n)
    return m, H


def _variant(ising, tensor, cplx=False):
    if tensor and cplx:
        raise ValueError("complex parameters are not combined with the tensor-RNN term")
    return int(bool(ising)) | (int(bool(tensor)) << 1) | (int(bool(cplx)) << 2)


def wrap_phase(x):
    """Angles reduced to [-pi, pi]."""
    return np.remainder(np.asarray(x) + np.pi, 2 * np.pi) - np.pi


def tucker_rank(chi: int, d: int) -> int:
    """chi' = ceil(chi^(2/(d+1))) of a site with d parents (Sec. 2.2)."""
    return int(_load().or_tucker_rank(chi, d))


def n_params(K, chi, parent_ptr, n_hidden, ising: bool = False, tensor: bool = False, cplx: bool = False) -> int:
    pp = _i32(parent_ptr)
    return int(_load().or_n_params(K, chi, _ptr(pp), n_hidden, _variant(ising, tensor, cplx)))


def amplitudes(K, chi, na, nb, parent_ptr, parent_idx, n_hidden, params, samples,
               nthreads: int = 0, ising: bool = False, tensor: bool = False,
               cplx: bool = False) -> Dict[str, np.ndarray]:
    """log|Phi|, sign Phi, log|f|, sign f for every sample (f: cos-RBM, or
    Ising-RBM when ising; Phi with the BDG-TensorRNN term when tensor).  With
    complex parameters (cplx): phase_phi (the phase of Phi) in place of sign
    Phi, and phase = the phase of Psi (sign f included), both in [-pi, pi].
    Real parameters also give the sign margins: margin_phi = min over sites of
    |w.h + c| / (||w|| ||h|| + |c|) and margin_f = min over hidden units of
    |cos theta| / (1 + |theta|) (inf without a correlator), and
    corr_sens = sum over hidden units of (1 + |theta|) / |cos theta| (0
    without a correlator)."""
    pp, pi, prm = _i32(parent_ptr), _i32(parent_idx), _f64(params)
    s = _u64a(samples).reshape(-1, 2)
    N = len(s)
    lphi, lf = np.zeros(N), np.zeros(N)
    sphi, sf = np.zeros(N, dtype=np.int32), np.zeros(N, dtype=np.int32)
    if cplx:
        ph = np.zeros(N)
        _load().or_amplitudes_cx(K, chi, na, nb, _ptr(pp), _ptr(pi), n_hidden, _variant(ising, False, True),
                                 _ptr(prm), _ptr(s), N, _ptr(lphi), _ptr(ph), _ptr(lf), _ptr(sf), nthreads)
        return dict(lphi=lphi, phase_phi=ph, lf=lf, sf=sf, logabs=lphi + lf,
                    phase=wrap_phase(ph + np.where(sf < 0, np.pi, 0.0)))
    mphi, mf, fs = np.zeros(N), np.zeros(N), np.zeros(N)
    _load().or_amplitudes(K, chi, na, nb, _ptr(pp), _ptr(pi), n_hidden, _variant(ising, tensor), _ptr(prm), _ptr(s), N,
                          _ptr(lphi), _ptr(sphi), _ptr(lf), _ptr(sf), _ptr(mphi), _ptr(mf), _ptr(fs), nthreads)
    return dict(lphi=lphi, sphi=sphi, lf=lf, sf=sf, logabs=lphi + lf, sign=sphi * sf, margin_phi=mphi,
                margin_f=mf, corr_sens=fs)


def sample(K, chi, na, nb, parent_ptr, parent_idx, params, u, tensor: bool = False,
           cplx: bool = False) -> np.ndarray:
    """Exact autoregressive draws from Phi^2; u is uniform [N, K]."""
    pp, pi, prm = _i32(parent_ptr), _i32(parent_idx), _f64(params)
    uu = _f64(u)
    N = uu.shape[0]
    out = np.zeros((N, 2), dtype=np.uint64)
    _load().or_sample(K, chi, na, nb, _ptr(pp), _ptr(pi), _variant(False, tensor, cplx), _ptr(prm), _ptr(uu), N,
                      _ptr(out))
    return out


def sample_unique(K, chi, na, nb, parent_ptr, parent_idx, params, seed: int, n_draws: int, draw_base: int = 0,
                  tensor: bool = False, cplx: bool = False):
    """Draws draw_base .. draw_base+n_draws-1 of the counter-keyed sampler (the
    uniform of draw t at site i comes from Philox4x32-10 at counter
    (t lo, t hi, i, 0x53414D50), key (seed lo, seed hi)), merged into unique
    ONVs in ascending (hi, lo) order with counts."""
    pp, pi, prm = _i32(parent_ptr), _i32(parent_idx), _f64(params)
    cap = max(int(n_draws), 1)
    out = np.zeros((cap, 2), dtype=np.uint64)
    cnt = np.zeros(cap, dtype=np.int64)
    n = _load().or_sample_unique(K, chi, na, nb, _ptr(pp), _ptr(pi), _variant(False, tensor, cplx), _ptr(prm),
                                 int(seed) & 0xFFFFFFFFFFFFFFFF,
                                 int(draw_base), int(n_draws), cap, _ptr(out), _ptr(cnt))
    return out[:n], cnt[:n]


def grad(K, chi, na, nb, parent_ptr, parent_idx, n_hidden, params, samples, g,
         nthreads: int = 0, ising: bool = False, tensor: bool = False, cplx: bool = False,
         g_phase=None) -> np.ndarray:
    """sum_n g_n d ln|Psi(n)| / d theta over the packed parameter vector; with
    complex parameters also + g_phase_n d phase(n) / d theta (the real and
    imaginary part of a complex parameter are two entries)."""
    pp, pi, prm = _i32(parent_ptr), _i32(parent_idx), _f64(params)
    s = _u64a(samples).reshape(-1, 2)
    gg = _f64(g)
    out = np.zeros(prm.size)
    if cplx:
        gp = np.zeros(len(s)) if g_phase is None else _f64(g_phase)
        _load().or_grad_cx(K, chi, na, nb, _ptr(pp), _ptr(pi), n_hidden, _variant(ising, False, True), _ptr(prm),
                           _ptr(s), len(s), _ptr(gg), _ptr(gp), _ptr(out), nthreads)
        return out
    _load().or_grad(K, chi, na, nb, _ptr(pp), _ptr(pi), n_hidden, _variant(ising, tensor), _ptr(prm), _ptr(s), len(s),
                    _ptr(gg), _ptr(out), nthreads)
    return out


def eloc(K, na, nb, h, eri, chi, parent_ptr, parent_idx, n_hidden, params, samples,
         eps=0.0, n_eps=0, seed=0, stream=0, e_core=0.0, nthreads: int = 0,
         sample_base: int = 0, ising: bool = False, tensor: bool = False,
         cplx: bool = False, bounds=(), u_f: float = 0.0) -> Dict[str, np.ndarray]:
    """Semi-stochastic local energies and the reweighted numerators; the draws
    of sample i use Philox counter word 0 = sample_base + i.  With complex
    parameters eloc and etnum are complex128 and phase (of Psi) replaces sign.
    sabs[i] = |H_nn| + sum over the summed terms of |coefficient| |Psi(m)/Psi(n)|
    (each draw counted once per draw): the scale of the cancellation in the
    sum, which bounds how far a relative error of the amplitude ratios can
    move E_loc.  Real parameters: margin_phi / margin_f are the sign margins of
    the sample (see amplitudes).  bounds = up to four (L, kappa) pairs and u_f
    give ebound[i, q] = sum over the terms of |term| times
    expm1(2 L + u_f (corr_sens(m) + corr_sens(n))), plus 2 where a sign may
    flip (a Phi margin of the row or the sample below kappa, or the row's
    correlator margin below 8 u_f), plus 2 (8 u_f) / margin_f where that
    margin is below 8 u_f: how far E_loc can move when every log|Phi| is off
    by at most L, states carry relative errors up to kappa and each cos theta
    relative errors up to u_f (1 + |theta|)."""
    h, eri = _f64(h), _f64(eri)
    pp, pi, prm = _i32(parent_ptr), _i32(parent_idx), _f64(params)
    s = _u64a(samples).reshape(-1, 2)
    N = len(s)
    if cplx:
        o = {k: np.zeros(N) for k in ("er", "ei", "tr", "ti", "logabs", "phase", "fsq", "sabs")}
        cnt = {k: np.zeros(N, dtype=np.int64) for k in ("n_det", "n_rem", "n_uniq")}
        rc = _load().or_eloc_cx(K, na, nb, _ptr(h), _ptr(eri), e_core, chi, _ptr(pp), _ptr(pi), n_hidden,
                                _variant(ising, False, True), _ptr(prm), _ptr(s), N, eps, n_eps, seed, stream,
                                sample_base, _ptr(o["er"]), _ptr(o["ei"]), _ptr(o["tr"]), _ptr(o["ti"]),
                                _ptr(o["logabs"]), _ptr(o["phase"]), _ptr(o["fsq"]), _ptr(cnt["n_det"]),
                                _ptr(cnt["n_rem"]), _ptr(cnt["n_uniq"]), _ptr(o["sabs"]), nthreads)
        if rc != 0:
            raise ValueError("sample outside the (n_alpha, n_beta) sector")
        out = dict(eloc=o["er"] + 1j * o["ei"], etnum=o["tr"] + 1j * o["ti"], logabs=o["logabs"],
                   phase=o["phase"], fsq=o["fsq"], sabs=o["sabs"])
        out.update(cnt)
        return out
    bl = np.ascontiguousarray(np.asarray([b[0] for b in bounds], dtype=np.float64).reshape(-1))
    bk = np.ascontiguousarray(np.asarray([b[1] for b in bounds], dtype=np.float64).reshape(-1))
    if bl.size > 4:
        raise ValueError("at most four bound columns")
    out = {k: np.zeros(N) for k in ("eloc", "etnum", "logabs", "fsq", "sabs", "margin_phi", "margin_f")}
    out["ebound"] = np.zeros((N, bl.size))
    sign = np.zeros(N, dtype=np.int8)
    cnt = {k: np.zeros(N, dtype=np.int64) for k in ("n_det", "n_rem", "n_uniq")}
    rc = _load().or_eloc(K, na, nb, _ptr(h), _ptr(eri), e_core, chi, _ptr(pp), _ptr(pi), n_hidden,
                         _variant(ising, tensor), _ptr(prm), _ptr(s), N, eps, n_eps, seed, stream, sample_base, _ptr(out["eloc"]),
                         _ptr(out["etnum"]), _ptr(out["logabs"]), _ptr(sign), _ptr(out["fsq"]),
                         _ptr(cnt["n_det"]), _ptr(cnt["n_rem"]), _ptr(cnt["n_uniq"]), _ptr(out["sabs"]),
                         _ptr(bl), _ptr(bk), int(bl.size), float(u_f), _ptr(out["ebound"]), _ptr(out["margin_phi"]),
                         _ptr(out["margin_f"]), nthreads)
    if rc != 0:
        raise ValueError("sample outside the (n_alpha, n_beta) sector")
    out["sign"] = sign
    out.update(cnt)
    return out


def eloc_detail(K, na, nb, h, eri, chi, parent_ptr, parent_idx, n_hidden, params, sample,
                sample_idx, eps, n_eps, seed=0, stream=0, e_core=0.0, ising: bool = False,
                tensor: bool = False):
    """One sample: deterministic ranks, drawn ranks in draw order, Q, E_loc."""
    h, eri = _f64(h), _f64(eri)
    pp, pi, prm = _i32(parent_ptr), _i32(parent_idx), _f64(params)
    s = _u64a(sample).reshape(2)
    cap = 4_000_000
    det = np.zeros(cap, dtype=np.int64)
    nd = np.zeros(1, dtype=np.int64)
    draws = np.zeros(max(n_eps, 1), dtype=np.int64)
    Q = np.zeros(1, dtype=np.uint64)
    e = np.zeros(1)
    rc = _load().or_eloc_detail(K, na, nb, _ptr(h), _ptr(eri), e_core, chi, _ptr(pp), _ptr(pi),
                                n_hidden, _variant(ising, tensor), _ptr(prm), _ptr(s), sample_idx, eps, n_eps, seed, stream,
                                _ptr(det), cap, _ptr(nd), _ptr(draws), _ptr(Q), _ptr(e))
    if rc != 0:
        raise ValueError("sample outside the (n_alpha, n_beta) sector")
    n = int(nd[0])
    ndraw = n_eps if int(Q[0]) > 0 else 0
    return dict(det_ranks=det[:n].copy(), draw_ranks=draws[:ndraw].copy(), Q=int(Q[0]),
                eloc=float(e[0]))


def eloc_table(K, na, nb, h, eri, keys, vals, samples, eps=0.0, n_eps=0, seed=0, stream=0,
               e_core=0.0, nthreads: int = 0) -> np.ndarray:
    """Local energies with the amplitude given as a lookup table over ONVs
    (keys uint64 [T,2] sorted ascending as 128-bit integers)."""
    h, eri = _f64(h), _f64(eri)
    k, v = _u64a(keys).reshape(-1, 2), _f64(vals)
    s = _u64a(samples).reshape(-1, 2)
    out = np.zeros(len(s))
    _load().or_eloc_table(K, na, nb, _ptr(h), _ptr(eri), e_core, _ptr(k), _ptr(v), len(k),
                          _ptr(s), len(s), eps, n_eps, seed, stream, _ptr(out), nthreads)
    return out


def reweighted_cotangent(counts, etnum, fsq):
    """(cot, E): the VJP cotangent of the reweighted VMC gradient for real
    parameters (Sec. 2.3, Eq. (19)) and the reweighted energy."""
    c, et, f2 = _f64(counts), _f64(etnum), _f64(fsq)
    cot = np.zeros(len(c))
    E = np.zeros(1)
    _load().or_reweighted_cotangent(len(c), _ptr(c), _ptr(et), _ptr(f2), _ptr(cot), _ptr(E))
    return cot, float(E[0])


def reweighted_cotangent_cx(counts, etnum, fsq):
    """(cot_abs, cot_phase, E) for complex parameters: the cotangents of
    ln|Psi| and of the phase in 2 Re <(E_loc - E)^* d ln Psi>, reweighted as in
    Eq. (19); etnum complex."""
    c, f2 = _f64(counts), _f64(fsq)
    et = np.asarray(etnum)
    tr, ti = _f64(et.real), _f64(et.imag)
    ca, cp = np.zeros(len(c)), np.zeros(len(c))
    E = np.zeros(1)
    _load().or_reweighted_cotangent_cx(len(c), _ptr(c), _ptr(tr), _ptr(ti), _ptr(f2), _ptr(ca), _ptr(cp), _ptr(E))
    return ca, cp, float(E[0])


def adamw(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    """One AdamW step on copies: returns (params, m, v)."""
    p, g = _f64(params).copy(), _f64(grad)
    mm, vv = _f64(m).copy(), _f64(v).copy()
    _load().or_adamw(p.size, _ptr(p), _ptr(g), _ptr(mm), _ptr(vv), int(step), lr, beta1, beta2, eps, weight_decay)
    return p, mm, vv


def project_eta(K, chi, parent_ptr, n_hidden, params, ising=False, tensor=False, cplx=False):
    """A copy of the packed parameters with every negative eta entry set to 0
    (the constraint eta >= 0 of Sec. 2.1)."""
    pp, p = _i32(parent_ptr), _f64(params).copy()
    _load().or_project_eta(K, chi, _ptr(pp), n_hidden, _variant(ising, tensor, cplx), _ptr(p))
    return p


def vmc_step(K, na, nb, h, eri, chi, parent_ptr, parent_idx, n_hidden, params, m, v, step, n_draws,
             sample_seed, draw_base=0, eps=0.0, n_eps=0, eloc_seed=0, stream=0, lr=1e-3, beta1=0.9,
             beta2=0.999, adam_eps=1e-8, weight_decay=0.0, e_core=0.0, ising=False, tensor=False, cplx=False):
    """One VMC step in the paper's order: exact draws from Phi^2 merged into
    unique samples with counts, semi-stochastic local energies, the reweighted
    gradient of Eq. (19) (through the cotangent above and the gradient of
    ln|Psi|, and of the phase with complex parameters), and one AdamW update
    (complex parameters as pairs of reals) followed by the projection of eta
    onto eta >= 0."""
    uniq, cnt = sample_unique(K, chi, na, nb, parent_ptr, parent_idx, params, sample_seed, n_draws, draw_base,
                              tensor=tensor, cplx=cplx)
    out = eloc(K, na, nb, h, eri, chi, parent_ptr, parent_idx, n_hidden, params, uniq, eps=eps, n_eps=n_eps,
               seed=eloc_seed, stream=stream, e_core=e_core, ising=ising, tensor=tensor, cplx=cplx)
    if cplx:
        cot, cotp, E = reweighted_cotangent_cx(cnt.astype(np.float64), out["etnum"], out["fsq"])
        g = grad(K, chi, na, nb, parent_ptr, parent_idx, n_hidden, params, uniq, cot, ising=ising, cplx=True,
                 g_phase=cotp)
        p, mm, vv = adamw(params, g, m, v, step, lr, beta1, beta2, adam_eps, weight_decay)
        p = project_eta(K, chi, parent_ptr, n_hidden, p, ising=ising, cplx=True)
        return dict(params=p, m=mm, v=vv, grad=g, E=E, samples=uniq, counts=cnt, eloc=out)
    cot, E = reweighted_cotangent(cnt.astype(np.float64), out["etnum"], out["fsq"])
    g = grad(K, chi, na, nb, parent_ptr, parent_idx, n_hidden, params, uniq, cot, ising=ising, tensor=tensor)
    p, mm, vv = adamw(params, g, m, v, step, lr, beta1, beta2, adam_eps, weight_decay)
    p = project_eta(K, chi, parent_ptr, n_hidden, p, ising=ising, tensor=tensor)
    return dict(params=p, m=mm, v=vv, grad=g, E=E, samples=uniq, counts=cnt, eloc=out)
