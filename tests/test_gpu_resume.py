"""Resumed amplitude rows.  FP64/FP32 rows start at their third changed site
from a node shared by the rows with the same first two changes (itself
resumed from the sample); BF16 rows at their first changed site from their
sample's stored state.  The autoregressive conditionals at a site see only
the occupations below it, so every result must be bit-identical to evaluating
every row from site 0, on every workload, with and without row passes; and
the executed site count must match the count from the row list."""
import numpy as np
import pytest

import oracle
from paper_2507_19276_amd import workloads as W

pytestmark = pytest.mark.gpu

NAMES = ("eloc", "etnum", "logabs", "sign", "fsq")


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


_cache = {}


def setup(nqs, ctx, name, n):
    key = (name, n)
    if key not in _cache:
        w = W.make_workload(name, n_samples=n)
        inst = nqs.Instance(ctx, w.K, w.n_alpha, w.n_beta, w.h, w.eri, w.e_core)
        ans = nqs.Ansatz(ctx, w.K, w.n_alpha, w.n_beta, w.chi, w.parent_ptr, w.parent_idx, w.n_hidden)
        ans.bind(w.params)
        _cache[key] = (w, inst, ans)
    return _cache[key]


def first_changed_sites(m, s, K):
    """First site where row m differs from its sample s (K when equal)."""
    out = np.full(len(m), K, dtype=np.int64)
    for k in range(len(m)):
        x = (int(m[k, 0]) ^ int(s[0])) | ((int(m[k, 1]) ^ int(s[1])) << 64)
        if x:
            out[k] = ((x & -x).bit_length() - 1) // 2
    return out


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "bf16x3"])
@pytest.mark.parametrize("name,n", [("c1", None), ("c2", 200), ("c3", 24), ("c4a", 24), ("c4b", 40)])
def test_resume_bit_identical(nqs, ctx, name, n, prec):
    w, inst, ans = setup(nqs, ctx, name, n)
    kw = dict(eps=w.eps, n_eps=w.n_eps, precision=prec, seed=w.seed, stream_id=5)
    full, st_full = nqs.eloc(ctx, inst, ans, w.samples, resume=False, **kw)
    res, st_res = nqs.eloc(ctx, inst, ans, w.samples, **kw)
    for k in NAMES:
        assert np.array_equal(full[k].cpu().numpy(), res[k].cpu().numpy(), equal_nan=True), (name, prec, k)
    assert st_full["n_rows"] == st_res["n_rows"]
    assert st_full["n_site_rows"] == st_full["n_rows"] * w.K
    assert st_res["n_site_rows"] < st_full["n_site_rows"]


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "bf16x3"])
def test_resume_with_passes(nqs, ctx, prec):
    """Several passes: each pass sorts its own rows; results are unchanged."""
    w, inst, ans = setup(nqs, ctx, "c2", 200)
    kw = dict(eps=w.eps, n_eps=w.n_eps, precision=prec, seed=w.seed, stream_id=6)
    full, _ = nqs.eloc(ctx, inst, ans, w.samples, resume=False, **kw)
    many, st = nqs.eloc(ctx, inst, ans, w.samples, max_rows_per_pass=100_000, **kw)
    assert st["n_passes"] > 1
    for k in NAMES:
        assert np.array_equal(full[k].cpu().numpy(), many[k].cpu().numpy(), equal_nan=True), (prec, k)


@pytest.mark.parametrize("name,n,scale", [("c2", 64, 0.05), ("c3", 8, 0.3)])
def test_node_capacity_fallback(nqs, ctx, name, n, scale):
    """Whole samples past a node storage capacity get no nodes and their rows
    resume at their first changed site from the sample: the results stay
    bit-identical to evaluating every row from site 0, and the site count lies
    between that of full node coverage and that of full recompute."""
    w, inst, ans = setup(nqs, ctx, name, n)
    for prec in ("f64", "f32"):
        kw = dict(eps=w.eps, n_eps=w.n_eps, precision=prec, seed=w.seed, stream_id=3)
        full, st_full = nqs.eloc(ctx, inst, ans, w.samples, resume=False, **kw)
        _, st_all = nqs.eloc(ctx, inst, ans, w.samples, **kw)
        ctx.set_node_capacity(scale)
        try:
            part, st_part = nqs.eloc(ctx, inst, ans, w.samples, **kw)
        finally:
            ctx.set_node_capacity(1.0)
        for k in NAMES:
            assert np.array_equal(full[k].cpu().numpy(), part[k].cpu().numpy(), equal_nan=True), (name, prec, k)
        assert st_all["n_site_rows"] < st_part["n_site_rows"] < st_full["n_site_rows"], (name, prec)


def changed_sites(m, s, K):
    """Sites (ascending) where row m differs from its sample s."""
    out = []
    for k in range(len(m)):
        x = (int(m[k, 0]) ^ int(s[0])) | ((int(m[k, 1]) ^ int(s[1])) << 64)
        out.append(sorted({b // 2 for b in range(128) if (x >> b) & 1}))
    return out


def site_state(w0, w1, i):
    v = (int(w0) | (int(w1) << 64)) >> (2 * i)
    return v & 3


@pytest.mark.parametrize("name,n", [("c2", 64), ("c3", 6)])
def test_site_count_matches_changed_sites(nqs, ctx, name, n):
    """Executed site evaluations: the samples' pass (N K), then for FP32/FP64
    one node per (sample, first changed site and state there, second changed
    site and state there) from its first changed site to the largest third
    changed site of its rows, and every row from its third changed site on;
    for BF16 (no node level; measured: nodes do not pay for its cheaper sites)
    every row from its first changed site on.  Counted here from the row list
    of the same call.  K = 50 spans both ONV words and the compact pair keys
    of large K (a node split in two would still give the same bits, but not
    this count)."""
    w, inst, ans = setup(nqs, ctx, name, n)
    kw = dict(eps=w.eps, n_eps=w.n_eps, seed=w.seed, stream_id=7)
    r = nqs.rows(ctx, inst, w.samples, **kw)
    rp = r["row_ptr"].cpu().numpy()
    m = r["m"].cpu().numpy().view(np.uint64)
    K = w.K
    two = one = lvl1 = w.n_samples * K
    for s in range(w.n_samples):
        rows = m[rp[s]:rp[s + 1]]
        ch = changed_sites(rows, w.samples[s], K)
        assert ch[0] == []            # the sample's own row
        nodes, nodes1 = {}, {}
        for k, c in enumerate(ch[1:], start=1):
            one += K - c[0]
            c2 = c[1] if len(c) > 1 else K
            s2 = site_state(rows[k, 0], rows[k, 1], c2) if c2 < K else 0
            c3 = c[2] if len(c) > 2 else K
            key = (c[0], site_state(rows[k, 0], rows[k, 1], c[0]), c2, s2)
            nodes[key] = max(nodes.get(key, 0), c3)
            two += K - c3
            key1 = key[:2]
            nodes1[key1] = max(nodes1.get(key1, 0), c2)
            lvl1 += K - c2
        two += sum(e - key[0] for key, e in nodes.items())
        lvl1 += sum(e - key[0] for key, e in nodes1.items())
    _, st = nqs.eloc(ctx, inst, ans, w.samples, precision="f32", **kw)
    assert st["n_site_rows"] == two
    _, st = nqs.eloc(ctx, inst, ans, w.samples, precision="bf16", **kw)
    assert st["n_site_rows"] == one
    assert two < lvl1 < one


def test_resume_matches_oracle_f64(nqs, ctx):
    """The resumed FP64 path against the oracle at the FP64 bar."""
    w, inst, ans = setup(nqs, ctx, "c4b", 16)
    out, _ = nqs.eloc(ctx, inst, ans, w.samples, eps=w.eps, n_eps=w.n_eps, precision="f64", seed=w.seed,
                      stream_id=2)
    ref = oracle.eloc(w.K, w.n_alpha, w.n_beta, w.h, w.eri, w.chi, w.parent_ptr, w.parent_idx, w.n_hidden,
                      w.params, w.samples, eps=w.eps, n_eps=w.n_eps, seed=w.seed, stream=2)
    el = out["eloc"].cpu().numpy()
    tau = 1e-3 * np.sqrt(np.mean(ref["eloc"] ** 2))
    assert (np.abs(el - ref["eloc"]) / np.maximum(np.abs(ref["eloc"]), tau)).max() <= 1e-10
