"""GPU parity at the largest system the sample layout holds: K = 64 spatial
orbitals (128 spin orbitals, both words of the interleaved ONV full), chain
integrals, NN+NNN BDG-RNN chi = 16, eps = 1e-2, N_eps = 100.  K > 30 also
takes the node level keyed by the first change alone (the pair table does not
fit the LDS).  Samples: random ones at half filling and off it, and the two
extremes of the half-filled sector (every electron in the upper 32 orbitals,
so the low word is empty, and every one in the lower 32).
"""
import numpy as np
import pytest

import oracle
from paper_2507_19276_amd import workloads as W

pytestmark = pytest.mark.gpu

K, CHI, EPS, NEPS, SEED = 64, 16, 1e-2, 100, 5


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


@pytest.fixture(scope="module")
def system():
    h, eri = W.chain_integrals(K, 424242)
    pp, pi = W.graph_nn_nnn(K)
    params = W.ansatz_params(K, CHI, pp, pi, 0, 424243)
    return h, eri, pp, pi, params


def samples_for(na, nb):
    s = W.random_onvs(K, na, nb, 6, 424244 + na)
    if na == nb == 32:
        top = W.onv_from_occ(K, range(32, 64), range(32, 64))
        bottom = W.onv_from_occ(K, range(32), range(32))
        s = np.concatenate([np.asarray([top, bottom], dtype=np.uint64), s])
    return s


def rel_err(got, ref):
    tau = 1e-3 * np.sqrt(np.mean(ref ** 2))
    return np.abs(got - ref) / np.maximum(np.abs(ref), tau)


@pytest.mark.parametrize("na,nb", [(32, 32), (20, 30)])
def test_k64_eloc(nqs, ctx, system, na, nb):
    """FP64 at the FP64 bars; resumed rows bit-identical to full recompute in
    FP64 and FP32; FP32 log|Psi| within 1e-4 and E_loc median 1e-4 (the
    bounds of the larger configurations); BF16 log|Psi| median within 1e-2."""
    h, eri, pp, pi, params = system
    s = samples_for(na, nb)
    inst = nqs.Instance(ctx, K, na, nb, h, eri, 0.0)
    ans = nqs.Ansatz(ctx, K, na, nb, CHI, pp, pi, 0)
    ans.bind(params)
    ref = oracle.eloc(K, na, nb, h, eri, CHI, pp, pi, 0, params, s, eps=EPS, n_eps=NEPS, seed=SEED, stream=1)
    kw = dict(eps=EPS, n_eps=NEPS, seed=SEED, stream_id=1)
    out, st = nqs.eloc(ctx, inst, ans, s, precision="f64", **kw)
    got = {k: v.cpu().numpy() for k, v in out.items()}
    assert rel_err(got["eloc"], ref["eloc"]).max() <= 1e-10
    assert rel_err(got["etnum"], ref["etnum"]).max() <= 1e-10
    assert np.abs(got["logabs"] - ref["logabs"]).max() < 1e-12
    assert np.array_equal(got["sign"], ref["sign"])
    assert st["n_det_rows"] == ref["n_det"].sum()
    assert st["n_draw_rows"] == ref["n_uniq"].sum()
    for prec in ("f64", "f32"):
        a, _ = nqs.eloc(ctx, inst, ans, s, precision=prec, **kw)
        b, _ = nqs.eloc(ctx, inst, ans, s, precision=prec, resume=False, **kw)
        for k in ("eloc", "etnum", "logabs", "sign"):
            assert np.array_equal(a[k].cpu().numpy(), b[k].cpu().numpy()), (prec, k)
        if prec == "f32":
            dl = np.abs(a["logabs"].cpu().numpy() - ref["logabs"])
            e = rel_err(a["eloc"].cpu().numpy(), ref["eloc"])
            assert dl.max() <= 1e-4 and np.median(e) <= 1e-4
    o16, _ = nqs.eloc(ctx, inst, ans, s, precision="bf16", **kw)
    assert np.isfinite(o16["eloc"].cpu().numpy()).all()
    assert np.median(np.abs(o16["logabs"].cpu().numpy() - ref["logabs"])) <= 1e-2


def test_k64_connected_bitexact(nqs, ctx, system):
    """All 1,542,656 connected determinants of the two extreme samples (and
    one random one), their Hamiltonian elements and diagonals, bit for bit."""
    h, eri, pp, pi, params = system
    s = samples_for(32, 32)[:3]
    inst = nqs.Instance(ctx, K, 32, 32, h, eri, 0.0)
    m, hv, hd = inst.connected(s)
    m, hv, hd = m.cpu().numpy().view(np.uint64), hv.cpu().numpy(), hd.cpu().numpy()
    assert np.array_equal(hd, oracle.hdiag(K, 32, 32, h, eri, s))
    for k in range(len(s)):
        rm, rh = oracle.connected(K, 32, 32, h, eri, s[k])
        assert len(rm) == 1542656
        assert np.array_equal(m[k], rm) and np.array_equal(hv[k], rh)
