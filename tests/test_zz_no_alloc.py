"""The allocation-free local energy (nqs_eloc_noalloc, for callers that
cannot allocate device memory) through the C ABI: bit for bit the results of
nqs_eloc on two calls in a row, the second with a smaller input; the
context's pool neither grows nor is touched; a call needing more than the
static workspace fails with NQS_ENOMEM and a message, and the next call
still works."""
import numpy as np
import pytest
import torch

from paper_2507_19276_amd import workloads as W

pytestmark = pytest.mark.gpu

NAMES = ("eloc", "etnum", "logabs", "sign", "fsq")


@pytest.fixture(scope="module")
def env():
    from paper_2507_19276_amd import nqs
    nqs.lib()
    ctx = nqs.Context(0)
    w = W.make_workload("c2", n_samples=160)
    inst = nqs.Instance(ctx, w.K, w.n_alpha, w.n_beta, w.h, w.eri, w.e_core)
    ans = nqs.Ansatz(ctx, w.K, w.n_alpha, w.n_beta, w.chi, w.parent_ptr, w.parent_idx, w.n_hidden)
    ans.bind(w.params)
    yield nqs, ctx, w, inst, ans
    ctx.close()


def _outputs(N):
    f = lambda: torch.full((N,), float("nan"), dtype=torch.float64, device="cuda")
    return {"eloc": f(), "etnum": f(), "logabs": f(), "fsq": f(),
            "sign": torch.zeros(N, dtype=torch.int8, device="cuda")}


def test_noalloc_matches_eloc_twice(env):
    nqs, ctx, w, inst, ans = env
    kw = dict(eps=w.eps, n_eps=w.n_eps, seed=w.seed, stream_id=2, max_rows_per_pass=300_000)
    for N, prec in ((160, "f32"), (48, "f64")):
        smp = torch.from_numpy(w.samples[:N].view(np.int64)).cuda()
        ref, st = nqs.eloc(ctx, inst, ans, smp, precision=prec, **kw)
        assert st["n_passes"] > 1 or N < 160
        out = _outputs(N)
        torch.cuda.synchronize()
        before = ctx.pool_bytes()
        ctx.pool_peak(reset=True)
        peak0 = ctx.pool_peak()
        nqs.eloc_noalloc(ctx, inst, ans, smp, out, precision=prec, **kw)
        torch.cuda.synchronize()
        assert ctx.pool_bytes() == before and ctx.pool_peak() == peak0
        for k in NAMES:
            assert np.array_equal(ref[k].cpu().numpy(), out[k].cpu().numpy(), equal_nan=True), (N, prec, k)


def test_noalloc_rejects_beyond_static_size(env):
    nqs, ctx, w, inst, ans = env
    big = W.make_workload("c2")           # 4096 samples, ~31 M rows in one pass: far beyond 256 MiB
    smp = torch.from_numpy(big.samples.view(np.int64)).cuda()
    with pytest.raises(nqs.NqsError) as e:
        nqs.eloc_noalloc(ctx, inst, ans, smp, _outputs(len(smp)), eps=w.eps, n_eps=w.n_eps, precision="f32",
                         seed=1)
    assert e.value.code == nqs.NQS_ENOMEM and "static workspace" in str(e.value)
    small = torch.from_numpy(w.samples[:20].view(np.int64)).cuda()
    ref, _ = nqs.eloc(ctx, inst, ans, small, eps=w.eps, n_eps=w.n_eps, precision="f64", seed=3)
    out = _outputs(20)
    nqs.eloc_noalloc(ctx, inst, ans, small, out, eps=w.eps, n_eps=w.n_eps, precision="f64", seed=3)
    assert np.array_equal(ref["eloc"].cpu().numpy(), out["eloc"].cpu().numpy())
