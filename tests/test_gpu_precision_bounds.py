"""Reduced-precision local energies against the FP64 oracle at the benchmark's
full sizes, in the launch configuration the benchmark times (whole batch in
one call, samples drawn from Phi^2 with their counts).

Stated bound, per sample n.  The bond contractions (unit roundoff u: FP32
2^-24, BF16 2^-8, split BF16 2^-15; tests/bounds.py) leave every carried state within a relative error
kappa = 8 u and every log|Phi| within L = 8 K u; the correlator's cos theta
is evaluated in FP32 from an FP64 theta on both paths, within a relative error
u_f (1 + |theta|), u_f = 2^-22.  Then each term x = coef Psi(m)/Psi(n) of
E_loc(n) moves by at most |x| (e^delta - 1), delta = 2 L + u_f (s(m) + s(n))
with s = sum_k (1 + |theta_k|) / |cos theta_k| (the ratio's log error), plus
2 |x| where its sign can flip: a sign margin |w.h + c| / (||w|| ||h|| + |c|)
of the row or of the sample below kappa, or a correlator margin
|cos theta| / (1 + |theta|) of the row below kappa_f = 8 u_f (plus
2 kappa_f / margin |x| there, as |cos theta| itself may grow).  H_nn is exact.
Summing gives |E_P(n) - E(n)| <= ebound(n) (oracle.eloc with bounds, u_f).
The premises are checked row by row on blocks of samples: |d log|Psi(m)|| <=
L + u_f s(m), and equal signs wherever no margin is below its kappa.  A sample
whose own correlator margin is below kappa_f has no bound (f(n) may be near a
zero); the tests count those (none on these batches).
"""
import functools

import numpy as np
import pytest
import torch

import oracle
from bounds import KAPPA_F, U_F, bounds, kappa, log_bound, stated_bound
from phi2 import batch

pytestmark = pytest.mark.gpu

SEED = 4242


@pytest.fixture(scope="module")
def nqs():
    from paper_2507_19276_amd import nqs as N
    N.lib()
    return N


@pytest.fixture(scope="module")
def ctx(nqs):
    c = nqs.Context(0)
    yield c
    c.close()


_obj = {}


def objects(nqs, ctx, name):
    if name not in _obj:
        w, smp, cnt, _ = batch(name)
        inst = nqs.Instance(ctx, w.K, w.n_alpha, w.n_beta, w.h, w.eri, w.e_core)
        ans = nqs.Ansatz(ctx, w.K, w.n_alpha, w.n_beta, w.chi, w.parent_ptr, w.parent_idx, w.n_hidden)
        ans.bind(w.params)
        _obj[name] = (w, smp, cnt, inst, ans)
    return _obj[name]


@functools.lru_cache(maxsize=4)
def oracle_block(name, n):
    """The oracle on the first n samples of the batch with the draws of the
    GPU call below (draw counters = batch positions)."""
    w, smp, cnt, _ = batch(name)
    ref = oracle.eloc(w.K, w.n_alpha, w.n_beta, w.h, w.eri, w.chi, w.parent_ptr, w.parent_idx, w.n_hidden,
                      w.params, smp[:n], eps=w.eps, n_eps=w.n_eps, seed=SEED, stream=0, bounds=bounds(w.K), u_f=U_F)
    amp = oracle.amplitudes(w.K, w.chi, w.n_alpha, w.n_beta, w.parent_ptr, w.parent_idx, w.n_hidden, w.params,
                            smp[:n])
    ref["corr_sens"] = amp["corr_sens"]
    return ref


def gpu_full(nqs, ctx, name, prec):
    w, smp, cnt, inst, ans = objects(nqs, ctx, name)
    out, st = nqs.eloc(ctx, inst, ans, smp, counts=torch.from_numpy(cnt.astype(np.float64)), eps=w.eps,
                       n_eps=w.n_eps, precision=prec, seed=SEED, stream_id=0)
    return {k: v.cpu().numpy() for k, v in out.items()}, st


def check_bound(w, got, ref, prec, n):
    L, kap = log_bound(prec, w.K), kappa(prec)
    ok = ref["margin_f"] >= KAPPA_F
    assert ok.all(), f"{(~ok).sum()} samples with a correlator within kappa_f of a zero"
    dE = np.abs(got["eloc"][:n] - ref["eloc"])
    bound = stated_bound(prec, ref)
    ratio = dE / bound
    print(f"{w.name} {prec}: |dE|/bound max {ratio.max():.3e} p99 {np.quantile(ratio, .99):.3e}; "
          f"|dE|/S p50 {np.median(dE / ref['sabs']):.2e} max {(dE / ref['sabs']).max():.2e}; "
          f"bound/S p50 {np.median(bound / ref['sabs']):.2e}")
    assert np.all(dE <= bound), (prec, int(np.argmax(ratio)), float(ratio.max()))
    dl = np.abs(got["logabs"][:n] - ref["logabs"])
    assert np.all(dl <= L + U_F * ref["corr_sens"]), (prec, float(dl.max()))
    # the sample's own sign: equal wherever its FP64 margins are >= kappa
    sure = (ref["margin_phi"] >= kap) & ok
    assert np.array_equal(got["sign"][:n][sure], ref["sign"][sure])


@pytest.mark.parametrize("prec", ["f32", "bf16", "bf16x3"])
def test_c2_every_sample_within_bound(nqs, ctx, prec):
    """All 4096 samples of the K = 20 chain batch."""
    w, smp, _, _, _ = objects(nqs, ctx, "c2")
    ref = oracle_block("c2", len(smp))
    got, st = gpu_full(nqs, ctx, "c2", prec)
    check_bound(w, got, ref, prec, len(smp))


@pytest.mark.parametrize("prec", ["f32", "bf16", "bf16x3"])
def test_c3_block_within_bound(nqs, ctx, prec):
    """The first 96 samples of the K = 50 batch (cos-RBM, chi = 32), the whole
    16384-sample batch evaluated in one call."""
    w, smp, _, _, _ = objects(nqs, ctx, "c3")
    ref = oracle_block("c3", 96)
    got, st = gpu_full(nqs, ctx, "c3", prec)
    check_bound(w, got, ref, prec, 96)


@pytest.mark.parametrize("name,n", [("c2", 24), ("c3", 2)])
def test_row_premises(nqs, ctx, name, n):
    """Every amplitude row of the first n samples (their deterministic and
    drawn determinants): |d log|Psi|| <= L + u_f s(m), and equal signs
    wherever no margin is below its kappa; in FP64 the rows match the oracle
    within 1e-12."""
    w, smp, _, inst, ans = objects(nqs, ctx, name)
    r = nqs.rows(ctx, inst, smp[:n], eps=w.eps, n_eps=w.n_eps, seed=SEED, stream_id=0)
    m = r["m"].cpu().numpy().view(np.uint64)
    ref = oracle.amplitudes(w.K, w.chi, w.n_alpha, w.n_beta, w.parent_ptr, w.parent_idx, w.n_hidden, w.params, m)
    la64, sg64 = ans.logpsi(r["m"], "f64")
    assert np.abs(la64.cpu().numpy() - ref["logabs"]).max() < 1e-12
    assert np.array_equal(sg64.cpu().numpy(), ref["sign"])
    okf = ref["margin_f"] >= KAPPA_F
    for prec in ("f32", "bf16", "bf16x3"):
        L, kap = log_bound(prec, w.K), kappa(prec)
        la, sg = ans.logpsi(r["m"], prec)
        la, sg = la.cpu().numpy(), sg.cpu().numpy()
        dl = np.abs(la - ref["logabs"])
        flips = sg != ref["sign"]
        sure = (ref["margin_phi"] >= kap) & okf
        print(f"{name} rows {len(m)} {prec}: |dlog| max {dl[okf].max():.3e} (L {L:.3e}); sign flips "
              f"{flips.sum()}, rows with a margin below kappa {(~sure).sum()}, largest Phi margin of a flipped "
              f"row {ref['margin_phi'][flips].max() if flips.any() else 0:.3e}")
        assert np.all(dl[okf] <= L + U_F * ref["corr_sens"][okf])
        assert not np.any(flips & sure)
