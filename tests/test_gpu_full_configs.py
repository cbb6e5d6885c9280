"""GPU parity at the full sizes of the larger configurations (K=50 NN+NNN
chi=32 with the cos-RBM correlator, 16384 samples; dense K=20 NN+NNN chi=64,
8192 samples, N_eps=1000; 3x3x2 lattice K=18 chi=64, 8192 samples), in the
launch configuration the configuration benchmark times: the whole batch in
one call, rows resumed from the nodes of their first changes.

A contiguous block of 16 samples is checked one by one against the FP64
oracle (which takes the block's position in the batch as the draw counter
base); all samples are checked for properties that hold at any size (finite
local energies, nonzero sign, row counts).  Bars: FP64 as everywhere (local
energies 1e-10 relative to max(|E|, 1e-3 RMS E), log|Psi| 1e-12 absolute);
FP32 within the bounds stated below.
"""
import numpy as np
import pytest

import oracle
from paper_2507_19276_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def rel_err(got, ref):
    tau = 1e-3 * np.sqrt(np.mean(ref ** 2))
    return np.abs(got - ref) / np.maximum(np.abs(ref), tau)


@pytest.mark.parametrize("name", ["c3", "c4a", "c4b"])
def test_full_size_sampled(nqs, ctx, name):
    """FP64: the 16 sampled outputs at the FP64 bars.  FP32 (bond
    contractions in FP32 MFMA; Hamiltonian elements, ratios and sums in FP64):
    log|Psi| carries ~K FP32 roundings of log P per sample, stated bound 1e-4
    absolute for K <= 50; local energies median relative error <= 1e-4 and
    every one within 1e-2 (a sample whose terms cancel amplifies the
    roundoff); the batch energy of all samples within 0.05 of its standard
    error of the FP64 batch energy.  Measured: log|Psi| max 2.4e-5 / 5.2e-7 /
    3.6e-7, E_loc median 1.4e-6 / 2.7e-7 / 2.7e-7 and max 1.5e-4 / 4.2e-4 /
    1.3e-6 (K=50 / dense K=20 / lattice), batch energy within 1e-3 SE."""
    w = W.make_workload(name)
    inst = nqs.Instance(ctx, w.K, w.n_alpha, w.n_beta, w.h, w.eri, w.e_core)
    ans = nqs.Ansatz(ctx, w.K, w.n_alpha, w.n_beta, w.chi, w.parent_ptr, w.parent_idx, w.n_hidden)
    ans.bind(w.params)
    k0 = int(np.random.default_rng(7).integers(0, w.n_samples - 16))
    ref = oracle.eloc(w.K, w.n_alpha, w.n_beta, w.h, w.eri, w.chi, w.parent_ptr, w.parent_idx, w.n_hidden,
                      w.params, w.samples[k0:k0 + 16], eps=w.eps, n_eps=w.n_eps, seed=w.seed, stream=1,
                      sample_base=k0)
    res = {}
    for prec in ("f64", "f32"):
        out, st = nqs.eloc(ctx, inst, ans, w.samples, eps=w.eps, n_eps=w.n_eps, precision=prec, seed=w.seed,
                           stream_id=1)
        got = {k: v.cpu().numpy() for k, v in out.items()}
        assert np.isfinite(got["eloc"]).all() and np.all(got["sign"] != 0)
        assert st["n_rows"] > w.n_samples
        res[prec] = (got, st)
    g64, st64 = res["f64"]
    blk = slice(k0, k0 + 16)
    assert rel_err(g64["eloc"][blk], ref["eloc"]).max() <= 1e-10
    assert rel_err(g64["etnum"][blk], ref["etnum"]).max() <= 1e-10
    assert np.abs(g64["logabs"][blk] - ref["logabs"]).max() < 1e-12
    assert np.array_equal(g64["sign"][blk], ref["sign"])
    np.testing.assert_allclose(g64["fsq"][blk], ref["fsq"], rtol=1e-12)
    g32, st32 = res["f32"]
    assert st32["n_rows"] == st64["n_rows"]
    e = rel_err(g32["eloc"][blk], ref["eloc"])
    dl = np.abs(g32["logabs"][blk] - ref["logabs"])
    fsq, el = g64["fsq"], g64["eloc"]
    se = np.sqrt((fsq ** 2 * (el - st64["E"]) ** 2).sum()) / fsq.sum()
    print("%s f32: logabs err max %.2e | E_loc rel err p50 %.2e max %.2e | dE/SE %.2e"
          % (name, dl.max(), np.median(e), e.max(), abs(st32["E"] - st64["E"]) / se))
    assert dl.max() <= 1e-4
    assert np.median(e) <= 1e-4 and e.max() <= 1e-2
    assert abs(st32["E"] - st64["E"]) <= 0.05 * se
