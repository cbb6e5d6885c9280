"""The stated per-sample error bound of the reduced-precision local energies
(derivation in the module docstring of test_gpu_precision_bounds.py).

Bond contractions with unit roundoff u leave every state within a relative
error kappa = 8 u and every log|Phi| within L = 8 K u: u = 2^-24 for FP32,
2^-8 for BF16 (8 significant bits), 2^-15 for the split BF16 form (each
operand as hi + lo BF16 parts, three products per MFMA step: the dropped
lo.lo product and the parts' representation error are each below 2^-16 of a
product); the correlator's cos theta is evaluated in FP32 on both paths from
an FP64 theta, within a relative error u_f (1 + |theta|), u_f = 2^-22 (the
rounding of theta to FP32, the FP32 cosine's own error below 1.9 x 2^-24,
and one FP64 product rounding per factor).  The oracle turns this into a bound per
sample (oracle.eloc(..., bounds=BOUNDS(K), u_f=U_F)["ebound"]), summing over
the terms of E_loc their |term| times how far the term can move."""
import numpy as np

U = {"f32": 2.0 ** -24, "bf16": 2.0 ** -8, "bf16x3": 2.0 ** -15}
U_F = 2.0 ** -22
KAPPA_F = 8 * U_F
COLS = ("f32", "bf16", "bf16x3")   # column order of the oracle's ebound


def kappa(prec):
    return 8 * U[prec]


def log_bound(prec, K):
    return 8 * K * U[prec]


def bounds(K):
    return tuple((log_bound(p, K), kappa(p)) for p in COLS)


def stated_bound(prec, ref):
    """Bound per sample from an oracle.eloc result computed with bounds(K), U_F."""
    return ref["ebound"][:, COLS.index(prec)]
