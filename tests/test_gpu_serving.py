"""Serving form: continuous batching of local-energy requests from several
resident instances; each result is the same alone and in the mix, served
results match the FP64 oracle (FP64 at its bar, FP32 and BF16 within the
stated per-sample bound), admission never exceeds the device-memory budget,
failures stay contained."""
import numpy as np
import pytest
import torch

import oracle
from bounds import U_F, bounds, stated_bound
from paper_2507_19276_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nqs():
    from paper_2507_19276_amd import nqs as N
    N.lib()
    return N


@pytest.fixture(scope="module")
def env(nqs):
    ctx = nqs.Context(0)
    specs = [s for s in W.serving_instances()
             if (s["K"], s["chi"]) in ((12, 16), (20, 32), (36, 16), (50, 64), (36, 64))]
    objs = []
    for s in specs:
        inst = nqs.Instance(ctx, s["K"], s["n_alpha"], s["n_beta"], s["h"], s["eri"])
        ans = nqs.Ansatz(ctx, s["K"], s["n_alpha"], s["n_beta"], s["chi"], s["parent_ptr"], s["parent_idx"], 0)
        ans.bind(s["params"])
        objs.append((s, inst, ans))
    yield ctx, objs


def _requests(objs, n_req, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_req):
        i = int(rng.integers(len(objs)))
        s, inst, ans = objs[i]
        N = int(rng.integers(16, 200)) if s["K"] == 50 else int(rng.integers(32, 700))
        smp = W.random_onvs(s["K"], s["n_alpha"], s["n_beta"], N, seed * 100 + k)
        out.append(dict(i=i, samples=torch.from_numpy(smp.view(np.int64)).cuda(), seed=1000 + k,
                        prec="bf16" if k % 2 else "f32"))
    return out


def test_results_identical_alone_and_in_mix(nqs, env):
    ctx, objs = env
    reqs = _requests(objs, 14, 1)
    max_rows = 200_000
    alone = []
    for r in reqs:
        s, inst, ans = objs[r["i"]]
        out, _ = nqs.eloc(ctx, inst, ans, r["samples"], eps=1e-2, n_eps=100, precision=r["prec"], seed=r["seed"],
                          max_rows_per_pass=max_rows)
        alone.append({k: v.clone() for k, v in out.items()})
    srv = nqs.Server(ctx, n_slots=4, budget_bytes=6 << 30, max_rows_per_pass=max_rows)
    tickets = {}
    for k, r in enumerate(reqs):
        s, inst, ans = objs[r["i"]]
        t = srv.submit(inst, ans, r["samples"], eps=1e-2, n_eps=100, precision=r["prec"], seed=r["seed"], tag=k)
        tickets[t] = k
    got = {}
    while len(got) < len(reqs):
        c = srv.wait(120.0)
        assert c is not None, "timed out waiting for a completion"
        assert c["status"] == 0, c["message"]
        got[tickets[c["ticket"]]] = c["out"]
    info = srv.info()
    srv.close()
    assert info["peak_in_flight"] >= 2, "requests should overlap"
    for k in range(len(reqs)):
        for name in ("eloc", "etnum", "logabs", "sign", "fsq"):
            a, b = alone[k][name].cpu().numpy(), got[k][name].cpu().numpy()
            assert np.array_equal(a, b, equal_nan=True), (k, name)


def test_admission_respects_budget(nqs, env):
    ctx, objs = env
    reqs = _requests(objs, 12, 2)
    max_rows = 100_000
    srv = nqs.Server(ctx, n_slots=4, budget_bytes=1 << 30, max_rows_per_pass=max_rows)
    fps = []
    for r in reqs:
        s, inst, ans = objs[r["i"]]
        fps.append(srv.footprint(inst, ans, r["samples"], eps=1e-2, n_eps=100, precision=r["prec"]))
    budget = max(fps) + sorted(fps)[len(fps) // 2]   # room for the largest plus a median one
    srv.close()
    ctx.pool_peak(reset=True)
    srv = nqs.Server(ctx, n_slots=4, budget_bytes=budget, max_rows_per_pass=max_rows)
    for k, r in enumerate(reqs):
        s, inst, ans = objs[r["i"]]
        srv.submit(inst, ans, r["samples"], eps=1e-2, n_eps=100, precision=r["prec"], seed=r["seed"], tag=k)
    done = 0
    while done < len(reqs):
        c = srv.wait(120.0)
        assert c is not None and c["status"] == 0, (c or {}).get("message")
        done += 1
    info = srv.info()
    srv.close()
    assert info["peak_reserved"] <= budget
    assert ctx.pool_peak() <= budget
    assert info["reserved"] == 0 and info["in_flight"] == 0


def test_forced_allocation_failure_is_contained(nqs, env):
    ctx, objs = env
    reqs = _requests(objs, 6, 3)
    srv = nqs.Server(ctx, n_slots=2, budget_bytes=4 << 30, max_rows_per_pass=100_000)
    ctx.fail_alloc_at(5)
    for k, r in enumerate(reqs):
        s, inst, ans = objs[r["i"]]
        srv.submit(inst, ans, r["samples"], eps=1e-2, n_eps=100, precision="f32", seed=r["seed"], tag=k)
    statuses = []
    while len(statuses) < len(reqs):
        c = srv.wait(120.0)
        assert c is not None
        statuses.append(c["status"])
    info = srv.info()
    srv.close()
    assert statuses.count(nqs.NQS_ENOMEM) == 1 and statuses.count(0) == len(reqs) - 1
    assert info["reserved"] == 0


def test_oversized_request_rejected(nqs, env):
    ctx, objs = env
    s, inst, ans = objs[-1]
    smp = torch.from_numpy(W.random_onvs(s["K"], s["n_alpha"], s["n_beta"], 64, 5).view(np.int64)).cuda()
    srv = nqs.Server(ctx, n_slots=1, budget_bytes=1 << 20, max_rows_per_pass=100_000)
    with pytest.raises(nqs.NqsError) as e:
        srv.submit(inst, ans, smp, eps=1e-2, n_eps=100)
    assert e.value.code == nqs.NQS_ENOMEM
    srv.close()


@pytest.mark.parametrize("prec", ["f64", "bf16"])
def test_passes_and_footprint_bound(nqs, env, prec):
    """Row passes change nothing in the results, and the pool never holds more
    than the stated footprint of the call."""
    ctx, objs = env
    s, inst, ans = objs[1]
    smp = torch.from_numpy(W.random_onvs(s["K"], s["n_alpha"], s["n_beta"], 900, 9).view(np.int64)).cuda()
    one, st1 = nqs.eloc(ctx, inst, ans, smp, eps=1e-2, n_eps=100, precision=prec, seed=3)
    ctx.pool_bytes()
    ctx.pool_peak(reset=True)
    base, _ = ctx.pool_bytes()
    many, st2 = nqs.eloc(ctx, inst, ans, smp, eps=1e-2, n_eps=100, precision=prec, seed=3,
                         max_rows_per_pass=20_000)
    peak = ctx.pool_peak() - base
    bound = nqs.workspace_bytes(inst, ans, 900, eps=1e-2, n_eps=100, precision=prec, max_rows_per_pass=20_000)
    assert st2["n_passes"] > 1 and st1["n_passes"] == 1
    assert peak <= bound, (peak, bound)
    for name in ("eloc", "etnum", "logabs", "sign", "fsq"):
        assert np.array_equal(one[name].cpu().numpy(), many[name].cpu().numpy()), name


def _serve_all(nqs, ctx, objs, reqs, n_slots=4, budget=8 << 30, max_rows=200_000):
    srv = nqs.Server(ctx, n_slots=n_slots, budget_bytes=budget, max_rows_per_pass=max_rows)
    tickets = {}
    for k, r in enumerate(reqs):
        s, inst, ans = r["obj"] if "obj" in r else objs[r["i"]]
        t = srv.submit(inst, ans, r["samples"], eps=1e-2, n_eps=100, precision=r["prec"], seed=r["seed"], tag=k)
        tickets[t] = k
    got = {}
    while len(got) < len(reqs):
        c = srv.wait(180.0)
        assert c is not None, "timed out waiting for a completion"
        got[tickets[c["ticket"]]] = c
    info = srv.info()
    srv.close()
    return got, info


def test_served_results_match_oracle(nqs, env):
    """Requests of every precision over the K = 12, 20, 36 and 50 instances,
    BF16 at chi = 64 on K = 36 and K = 50 among them, served concurrently; the
    first samples of each request against the oracle with the request's own
    draws (request-local draw counters)."""
    ctx, objs = env
    pick = {(s["K"], s["chi"]): i for i, (s, _, _) in enumerate(objs)}
    plan = [((12, 16), "f64", 300), ((20, 32), "f32", 200), ((36, 64), "bf16", 120), ((50, 64), "bf16", 64),
            ((36, 64), "f32", 90), ((50, 64), "f64", 48), ((12, 16), "bf16", 400), ((20, 32), "f64", 150)]
    reqs = []
    for k, (key, prec, n) in enumerate(plan):
        s, _, _ = objs[pick[key]]
        smp = W.random_onvs(s["K"], s["n_alpha"], s["n_beta"], n, 7000 + k)
        reqs.append(dict(i=pick[key], samples=torch.from_numpy(smp.view(np.int64)).cuda(), smp=smp,
                         seed=3000 + k, prec=prec))
    got, info = _serve_all(nqs, ctx, objs, reqs)
    assert info["peak_in_flight"] >= 2
    for k, r in enumerate(reqs):
        c = got[k]
        assert c["status"] == 0, c["message"]
        s, _, _ = objs[r["i"]]
        nb = 3 if s["K"] >= 36 else 6
        ref = oracle.eloc(s["K"], s["n_alpha"], s["n_beta"], s["h"], s["eri"], s["chi"], s["parent_ptr"],
                          s["parent_idx"], 0, s["params"], r["smp"][:nb], eps=1e-2, n_eps=100, seed=r["seed"],
                          stream=0, bounds=bounds(s["K"]), u_f=U_F)
        el = c["out"]["eloc"].cpu().numpy()[:nb]
        dE = np.abs(el - ref["eloc"])
        if r["prec"] == "f64":
            tau = 1e-3 * np.sqrt(np.mean(ref["eloc"] ** 2))
            assert np.all(dE <= 1e-10 * np.maximum(np.abs(ref["eloc"]), tau)), (k, dE)
        else:
            bound = stated_bound(r["prec"], ref)
            print(f"request {k} K={s['K']} chi={s['chi']} {r['prec']}: |dE|/bound {(dE / bound).max():.3e}")
            assert np.all(dE <= bound), (k, dE, bound)


def test_unsupported_request_in_the_mix(nqs, env):
    """A BF16 request on a tensor-RNN ansatz (not supported in BF16) fails
    alone with EUNSUPPORTED before queuing any work; the valid requests served
    around it are bit-identical to running them alone."""
    ctx, objs = env
    s0, inst0, _ = objs[0]
    tens = nqs.Ansatz(ctx, s0["K"], s0["n_alpha"], s0["n_beta"], 16, s0["parent_ptr"], s0["parent_idx"], 0,
                      tensor=True)
    tens.bind(W.ansatz_params(s0["K"], 16, s0["parent_ptr"], s0["parent_idx"], 0, 99, tensor=True))
    reqs = _requests(objs, 8, 4)
    bad = W.random_onvs(s0["K"], s0["n_alpha"], s0["n_beta"], 500, 77)
    reqs.insert(3, dict(obj=(s0, inst0, tens), samples=torch.from_numpy(bad.view(np.int64)).cuda(), seed=5,
                        prec="bf16"))
    alone = {}
    for k, r in enumerate(reqs):
        if "obj" in r:
            continue
        s, inst, ans = objs[r["i"]]
        out, _ = nqs.eloc(ctx, inst, ans, r["samples"], eps=1e-2, n_eps=100, precision=r["prec"], seed=r["seed"],
                          max_rows_per_pass=200_000)
        alone[k] = {n: v.clone() for n, v in out.items()}
    got, _ = _serve_all(nqs, ctx, objs, reqs)
    assert got[3]["status"] == nqs.NQS_EUNSUPPORTED
    for k, a in alone.items():
        assert got[k]["status"] == 0, got[k]["message"]
        for name in ("eloc", "etnum", "logabs", "sign", "fsq"):
            assert np.array_equal(a[name].cpu().numpy(), got[k]["out"][name].cpu().numpy(), equal_nan=True), (k, name)
    tens.close()
