"""Python binding of libnqs (include/nqs.h): argument marshalling only.

Every step of the local-energy path runs in the HIP library; this module
passes device pointers of torch tensors and the current HIP stream.  It never
computes a result itself and raises if the library is not built.

Samples are int64 tensors of shape [N, 2] on the GPU holding the two uint64
words of each ONV (bit P = occupation of spin orbital P = 2p + sigma).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnqs.so")

NQS_OK, NQS_EINVAL, NQS_ENOMEM, NQS_EDEVICE, NQS_EUNSUPPORTED, NQS_EBUSY = range(6)
PRECISIONS = {"f64": 0, "f32": 1, "bf16": 2, "bf16x3": 3}


class NqsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nqs error {code}: {msg}")
        self.code = code


class ElocOpts(C.Structure):
    _fields_ = [("eps", C.c_double), ("n_eps", C.c_int32), ("precision", C.c_int32),
                ("seed", C.c_uint64), ("stream_id", C.c_uint64), ("sample_base", C.c_int32),
                ("max_rows_per_pass", C.c_int32), ("flags", C.c_int32)]


ELOC_FULL_RECOMPUTE = 1
ANSATZ_TENSOR = 0x10
ANSATZ_COMPLEX = 0x20


class ElocStats(C.Structure):
    _fields_ = [("n_samples", C.c_int64), ("n_conn", C.c_int64), ("n_rows", C.c_int64),
                ("n_det_rows", C.c_int64), ("n_draw_rows", C.c_int64), ("n_zero_amp", C.c_int64),
                ("sum_c", C.c_double), ("B", C.c_double), ("E", C.c_double), ("var", C.c_double),
                ("ms_enumerate", C.c_double), ("ms_draw", C.c_double), ("ms_rows", C.c_double),
                ("ms_amplitude", C.c_double), ("ms_reduce", C.c_double), ("n_passes", C.c_int64),
                ("n_site_rows", C.c_int64), ("ms_psi", C.c_double), ("psi_flops", C.c_double),
                ("E_im", C.c_double)]

    def to_dict(self) -> Dict[str, float]:
        return {k: getattr(self, k) for k, _ in self._fields_}


class VmcOpts(C.Structure):
    _fields_ = [("n_draws", C.c_int64), ("sample_seed", C.c_uint64), ("draw_base", C.c_int64),
                ("max_draws_per_pass", C.c_int64), ("eloc", ElocOpts), ("lr", C.c_double),
                ("beta1", C.c_double), ("beta2", C.c_double), ("adam_eps", C.c_double),
                ("weight_decay", C.c_double), ("step", C.c_int64)]


class VmcStats(C.Structure):
    _fields_ = [("n_unique", C.c_int64), ("E", C.c_double), ("var", C.c_double), ("B", C.c_double),
                ("grad_norm", C.c_double), ("ms_sample", C.c_double), ("ms_eloc", C.c_double),
                ("ms_grad", C.c_double), ("ms_update", C.c_double)]

    def to_dict(self) -> Dict[str, float]:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_p = C.c_void_p


def lib():
    """The loaded library; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2507_19276_amd/build.py "
                           "(there is no fallback path)")
    L = C.CDLL(LIB_PATH)
    L.nqs_last_error.restype = C.c_char_p
    L.nqs_version.restype = C.c_char_p
    L.nqs_ctx_create.argtypes = [C.c_int, C.POINTER(_p)]
    L.nqs_ctx_destroy.argtypes = [_p]
    L.nqs_ctx_fail_alloc_at.argtypes = [_p, C.c_int64]
    L.nqs_ctx_set_node_capacity.argtypes = [_p, C.c_double]
    L.nqs_ctx_pool_bytes.argtypes = [_p, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
    L.nqs_ctx_pool_peak.argtypes = [_p, C.POINTER(C.c_size_t), C.c_int]
    L.nqs_ctx_set_pool_limit.argtypes = [_p, C.c_size_t]
    L.nqs_instance_create.argtypes = [_p, C.c_int, C.c_int, C.c_int, _p, _p, C.c_double, C.POINTER(_p)]
    L.nqs_instance_destroy.argtypes = [_p]
    L.nqs_instance_n_conn.argtypes = [_p]
    L.nqs_instance_n_conn.restype = C.c_int64
    L.nqs_connected.argtypes = [_p, _p, _p, C.c_int64, _p, _p, _p, _p]
    L.nqs_ansatz_create.argtypes = [_p, C.c_int, C.c_int, C.c_int, C.c_int, _p, _p, C.c_int, C.c_int32,
                                    C.POINTER(_p)]
    L.nqs_ansatz_destroy.argtypes = [_p]
    L.nqs_ansatz_n_params.argtypes = [_p]
    L.nqs_ansatz_n_params.restype = C.c_int64
    L.nqs_ansatz_bind_params.argtypes = [_p, _p, _p]
    L.nqs_logpsi.argtypes = [_p, _p, _p, C.c_int64, C.c_int32, _p, _p, _p]
    L.nqs_logpsi_vjp.argtypes = [_p, _p, _p, C.c_int64, _p, C.c_int32, _p, _p]
    L.nqs_logpsi_phase.argtypes = [_p, _p, _p, C.c_int64, C.c_int32, _p, _p, _p]
    L.nqs_logpsi_vjp_phase.argtypes = [_p, _p, _p, C.c_int64, _p, _p, C.c_int32, _p, _p]
    L.nqs_eloc_complex.argtypes = [_p, _p, _p, _p, _p, C.c_int64, C.POINTER(ElocOpts), _p, _p, _p, _p, _p, _p, _p,
                                   C.POINTER(ElocStats), _p]
    L.nqs_eloc.argtypes = [_p, _p, _p, _p, _p, C.c_int64, C.POINTER(ElocOpts), _p, _p, _p, _p, _p,
                           C.POINTER(ElocStats), _p]
    L.nqs_eloc_noalloc.argtypes = [_p, _p, _p, _p, _p, C.c_int64, C.POINTER(ElocOpts), _p, _p, _p, _p, _p, _p]
    L.nqs_rows.argtypes = [_p, _p, _p, C.c_int64, C.POINTER(ElocOpts), C.c_int64, _p, _p, _p, _p, _p, _p,
                           C.POINTER(C.c_int64), _p]
    L.nqs_sample.argtypes = [_p, _p, C.c_int64, C.c_uint64, C.c_int64, C.c_int32, C.c_int64, C.c_int64, _p, _p,
                             _p, _p, C.POINTER(C.c_int64), _p]
    L.nqs_vmc_step.argtypes = [_p, _p, _p, C.POINTER(VmcOpts), _p, _p, _p, _p, C.POINTER(VmcStats), _p]
    L.nqs_eloc_workspace_bytes.argtypes = [_p, _p, C.c_int64, C.POINTER(ElocOpts), C.c_int64,
                                           C.POINTER(C.c_size_t)]
    _lib = L
    return L


def check(code: int):
    if code != NQS_OK:
        raise NqsError(code, lib().nqs_last_error().decode())


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return C.c_void_p(t.data_ptr())


def _samples(s) -> torch.Tensor:
    if isinstance(s, np.ndarray):
        s = torch.from_numpy(np.ascontiguousarray(s).view(np.int64))
    s = s.reshape(-1, 2)
    if not s.is_cuda:
        s = s.cuda()
    return s.contiguous()


def opts(eps: float = 0.0, n_eps: int = 0, precision="f64", seed: int = 0, stream_id: int = 0,
         sample_base: int = 0, max_rows_per_pass: int = 0, resume: bool = True) -> ElocOpts:
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return ElocOpts(float(eps), int(n_eps), p, int(seed) & 0xFFFFFFFFFFFFFFFF,
                    int(stream_id) & 0xFFFFFFFFFFFFFFFF, int(sample_base), int(max_rows_per_pass),
                    0 if resume else ELOC_FULL_RECOMPUTE)


class Context:
    def __init__(self, device: int = 0):
        h = _p()
        check(lib().nqs_ctx_create(int(device), C.byref(h)))
        self.h = h
        self.device = device

    def fail_alloc_at(self, k: int):
        check(lib().nqs_ctx_fail_alloc_at(self.h, int(k)))

    def set_node_capacity(self, scale: float):
        check(lib().nqs_ctx_set_node_capacity(self.h, float(scale)))

    def pool_bytes(self):
        a, b = C.c_size_t(), C.c_size_t()
        check(lib().nqs_ctx_pool_bytes(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def pool_peak(self, reset: bool = False) -> int:
        a = C.c_size_t()
        check(lib().nqs_ctx_pool_peak(self.h, C.byref(a), 1 if reset else 0))
        return a.value

    def set_pool_limit(self, nbytes: int):
        check(lib().nqs_ctx_set_pool_limit(self.h, int(nbytes)))

    def close(self):
        if self.h:
            lib().nqs_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Instance:
    """Resident Hamiltonian: h (K x K) and eri (K^4, chemist) copied to HBM."""

    def __init__(self, ctx: Context, K: int, n_alpha: int, n_beta: int, h, eri, e_core: float = 0.0):
        h = np.ascontiguousarray(h, dtype=np.float64)
        eri = np.ascontiguousarray(eri, dtype=np.float64)
        assert h.shape == (K, K) and eri.shape == (K, K, K, K)
        out = _p()
        check(lib().nqs_instance_create(ctx.h, K, n_alpha, n_beta, h.ctypes.data_as(_p),
                                        eri.ctypes.data_as(_p), float(e_core), C.byref(out)))
        self.h = out
        self.ctx = ctx
        self.K, self.n_alpha, self.n_beta = K, n_alpha, n_beta
        self.n_conn = int(lib().nqs_instance_n_conn(out))

    def connected(self, samples):
        """(m [N, n_conn, 2] int64, H [N, n_conn], H_nn [N]) on the device."""
        s = _samples(samples)
        N = s.shape[0]
        m = torch.empty((N, self.n_conn, 2), dtype=torch.int64, device=s.device)
        hv = torch.empty((N, self.n_conn), dtype=torch.float64, device=s.device)
        hd = torch.empty(N, dtype=torch.float64, device=s.device)
        check(lib().nqs_connected(self.ctx.h, self.h, _ptr(s), N, _ptr(m), _ptr(hv), _ptr(hd), _p(_stream())))
        return m, hv, hd

    def close(self):
        if self.h:
            lib().nqs_instance_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ansatz:
    """BDG-RNN / MPS-RNN (+ cos-RBM or Ising-RBM correlator) layout; parameters
    bound from a device tensor."""

    def __init__(self, ctx: Context, K: int, n_alpha: int, n_beta: int, chi: int, parent_ptr, parent_idx,
                 n_hidden: int = 0, ising: bool = False, tensor: bool = False, cplx: bool = False):
        pp = np.ascontiguousarray(parent_ptr, dtype=np.int32)
        pi = np.ascontiguousarray(parent_idx, dtype=np.int32)
        if pi.size == 0:
            pi = np.zeros(1, dtype=np.int32)
        out = _p()
        check(lib().nqs_ansatz_create(ctx.h, K, n_alpha, n_beta, chi, pp.ctypes.data_as(_p),
                                      pi.ctypes.data_as(_p), n_hidden,
                                      (1 if ising else 0) | (ANSATZ_TENSOR if tensor else 0) |
                                      (ANSATZ_COMPLEX if cplx else 0), C.byref(out)))
        self.h = out
        self.ctx = ctx
        self.K, self.n_alpha, self.n_beta, self.chi, self.n_hidden = K, n_alpha, n_beta, chi, n_hidden
        self.ising = bool(ising) and n_hidden > 0
        self.tensor = bool(tensor)
        self.cplx = bool(cplx)
        self.n_params = int(lib().nqs_ansatz_n_params(out))
        # bind generation and a copy of the bound parameters: LogPsi.backward
        # uses them to take the gradient at its forward's parameters
        self.version = 0
        self._bound = None

    def bind(self, params):
        if isinstance(params, np.ndarray):
            params = torch.from_numpy(np.ascontiguousarray(params, dtype=np.float64))
        p = params.detach().to(dtype=torch.float64, device=f"cuda:{self.ctx.device}").contiguous()
        assert p.numel() == self.n_params
        self.version += 1
        self._bound = None
        check(lib().nqs_ansatz_bind_params(self.h, _ptr(p), _p(_stream())))
        self._bound = p.clone() if p.data_ptr() == params.data_ptr() else p
        return self

    def logpsi(self, samples, precision="f64"):
        s = _samples(samples)
        N = s.shape[0]
        la = torch.empty(N, dtype=torch.float64, device=s.device)
        sg = torch.empty(N, dtype=torch.int8, device=s.device)
        pr = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        check(lib().nqs_logpsi(self.ctx.h, self.h, _ptr(s), N, pr, _ptr(la), _ptr(sg), _p(_stream())))
        return la, sg

    def logpsi_phase(self, samples, precision="f64"):
        """(log|Psi|, phase of Psi in [-pi, pi]) as device float64 tensors."""
        s = _samples(samples)
        N = s.shape[0]
        la = torch.empty(N, dtype=torch.float64, device=s.device)
        ph = torch.empty(N, dtype=torch.float64, device=s.device)
        pr = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        check(lib().nqs_logpsi_phase(self.ctx.h, self.h, _ptr(s), N, pr, _ptr(la), _ptr(ph), _p(_stream())))
        return la, ph

    def vjp(self, samples, cot, precision="f64", grad: Optional[torch.Tensor] = None,
            cot_phase: Optional[torch.Tensor] = None):
        """grad += sum_n cot[n] d log|Psi(n)| (+ cot_phase[n] d phase(n)) / d theta."""
        s = _samples(samples)
        N = s.shape[0]
        c = cot.to(dtype=torch.float64, device=s.device).contiguous()
        cp = None if cot_phase is None else cot_phase.to(dtype=torch.float64, device=s.device).contiguous()
        if grad is None:
            grad = torch.zeros(self.n_params, dtype=torch.float64, device=s.device)
        pr = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        check(lib().nqs_logpsi_vjp_phase(self.ctx.h, self.h, _ptr(s), N, _ptr(c), _ptr(cp), pr, _ptr(grad),
                                         _p(_stream())))
        return grad

    def sample(self, n_draws: int, seed: int = 0, draw_base: int = 0, precision="f64",
               cap: Optional[int] = None, max_draws_per_pass: int = 0):
        """Exact autoregressive draws draw_base .. draw_base + n_draws - 1 from
        Phi^2 (counter-keyed: independent of how draws are split into calls),
        merged into unique ONVs; returns (samples [U, 2] int64 viewing the two
        uint64 words, counts [U], log|Phi| [U], sign Phi [U]) on the device."""
        n_draws = int(n_draws)
        cap = max(n_draws, 1) if cap is None else int(cap)
        dev = f"cuda:{self.ctx.device}"
        out = torch.empty((max(cap, 1), 2), dtype=torch.int64, device=dev)
        cnt = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
        la = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
        # complex parameters: Phi has a phase, not a sign (logpsi_phase gives it)
        sg = None if self.cplx else torch.empty(max(cap, 1), dtype=torch.int8, device=dev)
        nu = C.c_int64(0)
        pr = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        check(lib().nqs_sample(self.ctx.h, self.h, n_draws, int(seed) & 0xFFFFFFFFFFFFFFFF, int(draw_base), pr,
                               int(max_draws_per_pass), cap, _ptr(out), _ptr(cnt), _ptr(la), _ptr(sg), C.byref(nu),
                               _p(_stream())))
        u = min(int(nu.value), cap)
        return out[:u], cnt[:u], la[:u], (None if sg is None else sg[:u]), int(nu.value)

    def close(self):
        if self.h:
            lib().nqs_ansatz_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eloc(ctx: Context, inst: Instance, ans: Ansatz, samples, counts: Optional[torch.Tensor] = None,
         eps: float = 0.0, n_eps: int = 0, precision="f64", seed: int = 0, stream_id: int = 0,
         sample_base: int = 0, want_stats: bool = True, max_rows_per_pass: int = 0, resume: bool = True):
    """Semi-stochastic local energies; returns (dict of device tensors, stats dict or None).
    resume=False evaluates every amplitude row from site 0 (NQS_ELOC_FULL_RECOMPUTE)."""
    s = _samples(samples)
    N = s.shape[0]
    dev = s.device
    out = {
        "eloc": torch.empty(N, dtype=torch.float64, device=dev),
        "etnum": torch.empty(N, dtype=torch.float64, device=dev),
        "logabs": torch.empty(N, dtype=torch.float64, device=dev),
        "sign": torch.empty(N, dtype=torch.int8, device=dev),
        "fsq": torch.empty(N, dtype=torch.float64, device=dev),
    }
    c = None if counts is None else counts.to(dtype=torch.float64, device=dev).contiguous()
    o = opts(eps, n_eps, precision, seed, stream_id, sample_base, max_rows_per_pass, resume)
    st = ElocStats()
    check(lib().nqs_eloc(ctx.h, inst.h, ans.h, _ptr(s), _ptr(c), N, C.byref(o), _ptr(out["eloc"]),
                         _ptr(out["etnum"]), _ptr(out["logabs"]), _ptr(out["sign"]), _ptr(out["fsq"]),
                         C.byref(st) if want_stats else None, _p(_stream())))
    return out, (st.to_dict() if want_stats else None)


def eloc_noalloc(ctx: Context, inst: Instance, ans: Ansatz, samples, out: Dict[str, torch.Tensor],
                 counts: Optional[torch.Tensor] = None, eps: float = 0.0, n_eps: int = 0, precision="f64",
                 seed: int = 0, stream_id: int = 0, sample_base: int = 0, max_rows_per_pass: int = 0,
                 resume: bool = True) -> Dict[str, torch.Tensor]:
    """nqs_eloc_noalloc: the local energies of eloc() with the library's
    workspace taken from its static device array (no device allocation by the
    library).  The caller passes the output tensors (device, length N: eloc,
    etnum, logabs, fsq float64 and sign int8; any may be missing), so this
    call allocates nothing on the device either."""
    s = _samples(samples)
    N = s.shape[0]
    c = None if counts is None else counts.to(dtype=torch.float64, device=s.device).contiguous()
    o = opts(eps, n_eps, precision, seed, stream_id, sample_base, max_rows_per_pass, resume)
    check(lib().nqs_eloc_noalloc(ctx.h, inst.h, ans.h, _ptr(s), _ptr(c), N, C.byref(o), _ptr(out.get("eloc")),
                                 _ptr(out.get("etnum")), _ptr(out.get("logabs")), _ptr(out.get("sign")),
                                 _ptr(out.get("fsq")), _p(_stream())))
    return out


def eloc_complex(ctx: Context, inst: Instance, ans: Ansatz, samples, counts: Optional[torch.Tensor] = None,
                 eps: float = 0.0, n_eps: int = 0, precision="f64", seed: int = 0, stream_id: int = 0,
                 sample_base: int = 0, want_stats: bool = True, max_rows_per_pass: int = 0, resume: bool = True):
    """Local energies with complex amplitudes (nqs_eloc_complex): eloc and
    etnum as complex128 device tensors, logabs, phase, fsq; and the stats dict."""
    s = _samples(samples)
    N = s.shape[0]
    dev = s.device
    f = {k: torch.empty(N, dtype=torch.float64, device=dev)
         for k in ("er", "ei", "tr", "ti", "logabs", "phase", "fsq")}
    c = None if counts is None else counts.to(dtype=torch.float64, device=dev).contiguous()
    o = opts(eps, n_eps, precision, seed, stream_id, sample_base, max_rows_per_pass, resume)
    st = ElocStats()
    check(lib().nqs_eloc_complex(ctx.h, inst.h, ans.h, _ptr(s), _ptr(c), N, C.byref(o), _ptr(f["er"]),
                                 _ptr(f["ei"]), _ptr(f["tr"]), _ptr(f["ti"]), _ptr(f["logabs"]), _ptr(f["phase"]),
                                 _ptr(f["fsq"]), C.byref(st) if want_stats else None, _p(_stream())))
    out = dict(eloc=torch.complex(f["er"], f["ei"]), etnum=torch.complex(f["tr"], f["ti"]), logabs=f["logabs"],
               phase=f["phase"], fsq=f["fsq"])
    return out, (st.to_dict() if want_stats else None)


def vmc_step(ctx: Context, inst: Instance, ans: Ansatz, params: torch.Tensor, adam_m: torch.Tensor,
             adam_v: torch.Tensor, step: int, n_draws: int, sample_seed: int = 0, draw_base: int = 0,
             max_draws_per_pass: int = 0, eps: float = 0.0, n_eps: int = 0, precision="f64", seed: int = 0,
             stream_id: int = 0, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
             adam_eps: float = 1e-8, weight_decay: float = 0.0, grad: Optional[torch.Tensor] = None):
    """One VMC step (see nqs_vmc_step in include/nqs.h): params, adam_m, adam_v
    (device float64 [n_params]) are updated in place and the ansatz re-bound.
    Returns the stats dict."""
    for t in (params, adam_m, adam_v) + ((grad,) if grad is not None else ()):
        assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous() and t.numel() == ans.n_params
    o = VmcOpts(int(n_draws), int(sample_seed) & 0xFFFFFFFFFFFFFFFF, int(draw_base), int(max_draws_per_pass),
                opts(eps, n_eps, precision, seed, stream_id), float(lr), float(beta1), float(beta2),
                float(adam_eps), float(weight_decay), int(step))
    st = VmcStats()
    ans.version += 1
    ans._bound = None
    check(lib().nqs_vmc_step(ctx.h, inst.h, ans.h, C.byref(o), _ptr(params), _ptr(adam_m), _ptr(adam_v),
                             _ptr(grad), C.byref(st), _p(_stream())))
    ans._bound = params.detach().clone()   # the step re-bound the ansatz to the updated parameters
    return st.to_dict()


def rows(ctx: Context, inst: Instance, samples, eps: float = 0.0, n_eps: int = 0, seed: int = 0,
         stream_id: int = 0, sample_base: int = 0, cap: Optional[int] = None):
    """Row list of the local-energy computation (see nqs_rows in include/nqs.h)."""
    s = _samples(samples)
    N = s.shape[0]
    dev = s.device
    o = opts(eps, n_eps, "f64", seed, stream_id, sample_base)
    row_ptr = torch.empty(N + 1, dtype=torch.int64, device=dev)
    n_det = torch.empty(N, dtype=torch.int64, device=dev)
    Q = torch.empty(N, dtype=torch.int64, device=dev)
    nr = C.c_int64()
    if cap is None:
        check(lib().nqs_rows(ctx.h, inst.h, _ptr(s), N, C.byref(o), 0, _ptr(row_ptr), _ptr(n_det), _ptr(Q),
                             None, None, None, C.byref(nr), _p(_stream())))
        cap = nr.value
    rank = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
    coef = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
    m = torch.empty((max(cap, 1), 2), dtype=torch.int64, device=dev)
    check(lib().nqs_rows(ctx.h, inst.h, _ptr(s), N, C.byref(o), cap, _ptr(row_ptr), _ptr(n_det), _ptr(Q),
                         _ptr(rank), _ptr(coef), _ptr(m), C.byref(nr), _p(_stream())))
    R = nr.value
    return dict(row_ptr=row_ptr, n_det=n_det, Q=Q, rank=rank[:R], coef=coef[:R], m=m[:R], n_rows=R)


def workspace_bytes(inst: Instance, ans: Ansatz, N: int, n_rows: int = 0, eps=0.0, n_eps=0, precision="f64",
                    max_rows_per_pass: int = 0, resume: bool = True) -> int:
    b = C.c_size_t()
    o = opts(eps, n_eps, precision, max_rows_per_pass=max_rows_per_pass, resume=resume)
    check(lib().nqs_eloc_workspace_bytes(inst.h, ans.h, int(N), C.byref(o), int(n_rows), C.byref(b)))
    return b.value


class LogPsi(torch.autograd.Function):
    """log|Psi(n)| with a backward pass through the hand-written adjoint kernel.

    forward(params, samples, ans, precision) -> log|Psi| [N] (float64); the
    gradient with respect to params is sum_n g_n d log|Psi(n)| / d theta."""

    @staticmethod
    def forward(ctx_, params, samples, ans: Ansatz, precision="f64"):
        ans.bind(params)
        la, _ = ans.logpsi(samples, precision)
        ctx_.ans = ans
        ctx_.precision = precision
        ctx_.version = ans.version
        ctx_.save_for_backward(_samples(samples), params)
        return la

    @staticmethod
    def backward(ctx_, g):
        s, params = ctx_.saved_tensors
        ans = ctx_.ans
        if ans.version == ctx_.version:
            return ans.vjp(s, g.contiguous(), ctx_.precision), None, None, None
        # the ansatz was bound to other parameters after this forward: take the
        # gradient at the forward's parameters, then restore the newer binding
        current = ans._bound
        ans.bind(params)
        try:
            grad = ans.vjp(s, g.contiguous(), ctx_.precision)
        finally:
            if current is not None:
                ans.bind(current)
        return grad, None, None, None


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------

class Request(C.Structure):
    _fields_ = [("inst", _p), ("ans", _p), ("samples", _p), ("N", C.c_int64), ("opts", ElocOpts),
                ("eloc", _p), ("etnum", _p), ("logabs", _p), ("sign", _p), ("fsq", _p),
                ("t_arrival", C.c_double), ("user_tag", C.c_uint64)]


class Completion(C.Structure):
    _fields_ = [("ticket", C.c_int64), ("user_tag", C.c_uint64), ("status", C.c_int), ("pad", C.c_int32),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_end", C.c_double),
                ("footprint", C.c_size_t), ("stats", ElocStats), ("message", C.c_char * 256)]


class ServeStatus(C.Structure):
    _fields_ = [("budget", C.c_size_t), ("reserved", C.c_size_t), ("peak_reserved", C.c_size_t),
                ("in_flight", C.c_int32), ("peak_in_flight", C.c_int32), ("queued", C.c_int64),
                ("skips", C.c_int64)]


def _serve_lib():
    L = lib()
    if not getattr(L, "_serve_ready", False):
        L.nqs_monotonic_seconds.restype = C.c_double
        L.nqs_serve_create.argtypes = [_p, C.c_int, C.c_size_t, C.c_int32, C.POINTER(_p)]
        L.nqs_serve_destroy.argtypes = [_p]
        L.nqs_serve_submit.argtypes = [_p, C.POINTER(Request), C.POINTER(C.c_int64)]
        L.nqs_serve_footprint.argtypes = [_p, C.POINTER(Request), C.POINTER(C.c_size_t)]
        L.nqs_serve_poll.argtypes = [_p, C.POINTER(Completion)]
        L.nqs_serve_wait.argtypes = [_p, C.c_double, C.POINTER(Completion)]
        L.nqs_serve_info.argtypes = [_p, C.POINTER(ServeStatus)]
        L._serve_ready = True
    return L


def monotonic() -> float:
    return _serve_lib().nqs_monotonic_seconds()


class Server:
    """Continuous-batching server over a context: n_slots concurrent requests
    (one device stream each) admitted by exact device-memory footprint within
    budget_bytes.  Requests keep their tensors alive until completion."""

    def __init__(self, ctx: Context, n_slots: int, budget_bytes: int, max_rows_per_pass: int):
        L = _serve_lib()
        h = _p()
        check(L.nqs_serve_create(ctx.h, int(n_slots), int(budget_bytes), int(max_rows_per_pass), C.byref(h)))
        self.h = h
        self.ctx = ctx
        self._live = {}

    def _request(self, inst, ans, samples, out, eps, n_eps, precision, seed, stream_id, t_arrival, tag):
        s = _samples(samples)
        r = Request(inst.h, ans.h, _ptr(s), s.shape[0], opts(eps, n_eps, precision, seed, stream_id),
                    _ptr(out["eloc"]), _ptr(out["etnum"]), _ptr(out["logabs"]), _ptr(out["sign"]),
                    _ptr(out["fsq"]), float(t_arrival), int(tag))
        return r, s

    def submit(self, inst: Instance, ans: Ansatz, samples, eps=0.0, n_eps=0, precision="f64", seed=0,
               stream_id=0, t_arrival=0.0, tag=0) -> int:
        s = _samples(samples)
        N = s.shape[0]
        dev = s.device
        out = {"eloc": torch.empty(N, dtype=torch.float64, device=dev),
               "etnum": torch.empty(N, dtype=torch.float64, device=dev),
               "logabs": torch.empty(N, dtype=torch.float64, device=dev),
               "sign": torch.empty(N, dtype=torch.int8, device=dev),
               "fsq": torch.empty(N, dtype=torch.float64, device=dev)}
        r, s = self._request(inst, ans, s, out, eps, n_eps, precision, seed, stream_id, t_arrival, tag)
        torch.cuda.current_stream().synchronize()   # inputs are complete before another stream reads them
        t = C.c_int64()
        check(_serve_lib().nqs_serve_submit(self.h, C.byref(r), C.byref(t)))
        self._live[t.value] = (s, out)
        return t.value

    def footprint(self, inst, ans, samples, eps=0.0, n_eps=0, precision="f64") -> int:
        s = _samples(samples)
        dummy = {k: None for k in ("eloc", "etnum", "logabs", "sign", "fsq")}
        r, _ = self._request(inst, ans, s, dummy, eps, n_eps, precision, 0, 0, 0.0, 0)
        b = C.c_size_t()
        check(_serve_lib().nqs_serve_footprint(self.h, C.byref(r), C.byref(b)))
        return b.value

    def _done(self, c: Completion):
        s, out = self._live.pop(c.ticket)
        return dict(ticket=c.ticket, tag=c.user_tag, status=c.status, t_submit=c.t_submit, t_start=c.t_start,
                    t_end=c.t_end, footprint=c.footprint, stats=c.stats.to_dict(),
                    message=c.message.decode(), out=out)

    def poll(self):
        c = Completion()
        rc = _serve_lib().nqs_serve_poll(self.h, C.byref(c))
        if rc == NQS_EBUSY:
            return None
        check(rc)
        return self._done(c)

    def wait(self, timeout_s: float = 60.0):
        c = Completion()
        rc = _serve_lib().nqs_serve_wait(self.h, float(timeout_s), C.byref(c))
        if rc == NQS_EBUSY:
            return None
        check(rc)
        return self._done(c)

    def info(self) -> Dict[str, int]:
        st = ServeStatus()
        check(_serve_lib().nqs_serve_info(self.h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in st._fields_}

    def close(self):
        if self.h:
            _serve_lib().nqs_serve_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
