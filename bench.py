"""Throughput of the semi-stochastic local energy on one MI355X.

Default: one step = one nqs_eloc call over the whole synthetic batch of the
K = 50 workload (50 spatial orbitals, 25a+25b, chain-like integrals with decay
length 2, BDG-RNN on the nearest + next-nearest neighbour graph with chi = 32,
cos-RBM correlator with 100 hidden units, 16384 distinct samples drawn exactly
from Phi^2 with their counts, eps = 1e-2, N_eps = 100): enumerate every
connected determinant, screen, draw, evaluate the amplitude of every row and
the correlator, reduce.  Integrals, parameters and samples are resident in HBM
before the timed region (the samples are drawn on the GPU by nqs_sample
beforehand); outputs stay on the device.  The headline precision is FP64, the
paper's (Sec. 3); FP32, BF16 and split-BF16 (hi + lo parts, three MFMA
products) bond contractions are timed alongside.  The
same is reported for the K = 20 chain workload (chi = 16, 4096 samples,
eps = 1e-3, N_eps = 64).

Equal energy error: on the K = 20 batch and a 256-sample block of the K = 50
batch, the batch energy sum c Etilde / sum c |f|^2 of every precision over 8
draw seeds against the same samples' exact energy (eps = 0, FP64); where a
precision's error exceeds the FP64 path's, the FP64 N_eps that matches it and
the throughput ratio there.

The CPU-baseline leg runs the FP64 oracle (built for the host CPU) on a block
of the K = 50 batch with the draws of one GPU call and reports the GPU error
per precision against it, with the stated per-sample bound of each precision.

--workload c2: the K = 20 chain workload as the headline instead.
--next / --serve / --configs / --speedups: see their functions.

Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import tempfile
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0}   # MI355X dense MFMA, TFLOP/s
# error model of the stated per-sample bounds (the GPU tests hold the
# derivation): bond contractions with unit roundoff u keep states within a
# relative error 8 u and log|Phi| within 8 K u; cos theta of the correlator
# is evaluated in FP32 within a relative error U_F (1 + |theta|)
UNIT_ROUNDOFF = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "bf16": 2.0 ** -8, "bf16x3": 2.0 ** -15}
U_F = 2.0 ** -22
# HBM bytes per launch of the headline row amplitude kernel, from the
# FETCH_SIZE / WRITE_SIZE counters (copy-calibrated) recorded in profiles/;
# valid only for the kernel source they were taken on (first 16 hex digits of
# the sha256 of psi.hip followed by device.h) and for that workload.
MEASURED_TRAFFIC = {
    ("c3", "f64"): {"sha16": "a5dfbc82a9b3c72e", "bytes_per_launch": 73.490e9 + 3.728e9},
}
KERNEL_SOURCES = ("psi.hip", "device.h")
WORKLOAD_TEXT = {
    "c2": "chain K=20 10a+10b, BDG-RNN chain chi=16, 4096 distinct samples drawn from Phi^2, eps=1e-3, N_eps=64",
    "c3": "chain-like K=50 25a+25b, BDG-RNN NN+NNN chi=32 x cos-RBM N_h=100, 16384 distinct samples drawn "
          "from Phi^2, eps=1e-2, N_eps=100",
}


def kernel_sha16():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2507_19276_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload, prec):
    rec = MEASURED_TRAFFIC.get((workload, prec))
    if rec is None or rec["sha16"] != kernel_sha16():
        return None
    return rec["bytes_per_launch"]


def phi2_batch(nqs, workloads, ans, w):
    """The workload's batch: distinct ONVs drawn exactly from Phi^2 on the GPU
    (nqs_sample, FP64, counter-keyed), with their counts; topped up with
    uniform valid ONVs only if the draws held fewer distinct ONVs."""
    import numpy as np
    import torch
    seed = w.seed + workloads.PHI2_SEED_OFFSET

    def draw(n):
        s, c, _, _, _ = ans.sample(n, seed=seed, precision="f64")
        return s, c

    s, c, n = workloads.draw_until_unique(draw, w.n_samples)
    smp = s.cpu().numpy().view(np.uint64)
    cnt = c.cpu().numpy()
    smp, cnt, added = workloads.top_up(smp, cnt, w.K, w.n_alpha, w.n_beta, w.n_samples, seed)
    dev = torch.from_numpy(np.ascontiguousarray(smp).view(np.int64)).cuda()
    return dev, torch.from_numpy(cnt.astype(np.float64)).cuda(), n, added, seed


def setup_workload(nqs, workloads, ctx, name):
    w = workloads.make_workload(name)
    inst = nqs.Instance(ctx, w.K, w.n_alpha, w.n_beta, w.h, w.eri, w.e_core)
    ans = nqs.Ansatz(ctx, w.K, w.n_alpha, w.n_beta, w.chi, w.parent_ptr, w.parent_idx, w.n_hidden)
    ans.bind(w.params)
    samples, counts, n_draws, added, sseed = phi2_batch(nqs, workloads, ans, w)
    return dict(w=w, inst=inst, ans=ans, samples=samples, counts=counts, n_draws=n_draws, added=added,
                sample_seed=sseed)


def time_precisions(nqs, ctx, W, precs, steps, warmup, full_recompute=False, ref_seed=None):
    """steps timed nqs_eloc calls per precision (after warmup); per-call stage
    times from the library's device events; one extra call with ref_seed keeps
    its outputs (for the oracle comparison)."""
    import numpy as np
    import torch
    w = W["w"]
    N = w.n_samples
    res, keep = {}, {}

    def step(k, prec):
        return nqs.eloc(ctx, W["inst"], W["ans"], W["samples"], counts=W["counts"], eps=w.eps, n_eps=w.n_eps,
                        precision=prec, seed=w.seed + k, stream_id=0, resume=not full_recompute)

    for prec in precs:
        for k in range(warmup):
            step(k, prec)
        torch.cuda.synchronize()
        sts = []
        t0 = time.perf_counter()
        for k in range(steps):
            _, st = step(1000 + k, prec)
            sts.append(st)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        mean = {k: float(np.mean([st[k] for st in sts])) for k in
                ("ms_enumerate", "ms_draw", "ms_rows", "ms_amplitude", "ms_reduce", "ms_psi", "psi_flops", "n_rows",
                 "n_site_rows", "n_det_rows", "n_draw_rows")}
        res[prec] = {"value": steps * N / dt, "ms_per_step": dt / steps * 1e3, "stats": mean, "E": sts[-1]["E"]}
        print(f"# {w.name} {prec}: {steps} steps in {dt:.3f} s ({dt / steps * 1e3:.2f} ms/step), "
              f"rows/step {mean['n_rows']:.0f}, row amplitude kernel {mean['ms_psi']:.3f} ms",
              file=sys.stderr, flush=True)
        if ref_seed is not None:
            out, st = nqs.eloc(ctx, W["inst"], W["ans"], W["samples"], counts=W["counts"], eps=w.eps,
                               n_eps=w.n_eps, precision=prec, seed=ref_seed, stream_id=0)
            keep[prec] = {k: v.cpu().numpy() for k, v in out.items()}
    return res, keep


def equal_error(nqs, ctx, W, precs, n_sub, seeds=8, max_rows=16_000_000):
    """Batch energy of each precision over `seeds` draw seeds against the exact
    energy of the same samples (eps = 0, FP64), on the first n_sub samples of
    the batch.  Where a precision's RMS error over the seeds exceeds the FP64
    path's, the FP64 N_eps with the same expected RMS error (the draw variance
    scales as 1/N_eps, Sec. 2.4) is timed and checked, and the throughput ratio
    at that N_eps is given."""
    import numpy as np
    import torch
    w = W["w"]
    smp = W["samples"][:n_sub]
    cnt = W["counts"][:n_sub]
    kw = dict(counts=cnt, stream_id=5, max_rows_per_pass=max_rows)
    _, st = nqs.eloc(ctx, W["inst"], W["ans"], smp, eps=0.0, n_eps=0, precision="f64", **kw)
    E_ex = st["E"]

    def run(prec, n_eps, reps=seeds):
        Es, ts = [], []
        for s in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = nqs.eloc(ctx, W["inst"], W["ans"], smp, eps=w.eps, n_eps=n_eps, precision=prec,
                             seed=777 + s, **kw)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            Es.append(st["E"])
        d = np.array(Es) - E_ex
        return {"n_eps": n_eps, "mean_error": float(d.mean()), "se_of_mean": float(d.std(ddof=1) / math.sqrt(reps)),
                "rms_error": float(np.sqrt(np.mean(d ** 2))), "local_energies_per_s": n_sub / float(np.median(ts))}

    out = {"samples": n_sub, "seeds": seeds, "E_exact_f64_eps0": E_ex, "eps": w.eps}
    for prec in precs:
        out[prec] = run(prec, w.n_eps)
    r64 = out["f64"]["rms_error"]
    for prec in precs:
        if prec == "f64":
            continue
        rp = out[prec]["rms_error"]
        if rp <= r64 or r64 == 0.0:
            out[prec]["at_equal_error"] = {"vs": "f64 at the same N_eps",
                                           "speedup": out[prec]["local_energies_per_s"]
                                           / out["f64"]["local_energies_per_s"]}
            continue
        n_match = max(1, int(round(w.n_eps * (r64 / rp) ** 2)))
        m = run("f64", n_match)
        out[prec]["at_equal_error"] = {"vs": f"f64 at N_eps={n_match}", "f64": m,
                                       "speedup": out[prec]["local_energies_per_s"] / m["local_energies_per_s"]}
    return out


def cpu_baseline(W, keep, seed, n_sub, threads):
    """The FP64 oracle, built for this host, on the first n_sub samples with the
    draws of the GPU call that used `seed`; returns the baseline record and the
    GPU error against it per precision (with the stated bound)."""
    import numpy as np
    import oracle
    from oracle import build as oracle_build
    native = os.path.join(tempfile.mkdtemp(prefix="oracle_native_"), "liboracle.so")
    try:
        oracle_build.build(native=True, out=native)
        oracle.use_library(native)
        build = "g++ -O3 -march=native (host build)"
    except Exception as e:   # fall back to the shipped x86-64-v3 build
        build = f"shipped x86-64-v3 build ({type(e).__name__})"
    w = W["w"]
    smp = W["samples"][:n_sub].cpu().numpy().view(np.uint64)
    cols = ("f32", "bf16", "bf16x3")
    bounds = tuple((8.0 * w.K * UNIT_ROUNDOFF[p], 8.0 * UNIT_ROUNDOFF[p]) for p in cols)
    t0 = time.perf_counter()
    ref = oracle.eloc(w.K, w.n_alpha, w.n_beta, w.h, w.eri, w.chi, w.parent_ptr, w.parent_idx, w.n_hidden,
                      w.params, smp, eps=w.eps, n_eps=w.n_eps, seed=seed, stream=0, nthreads=threads,
                      bounds=bounds, u_f=U_F)
    dt = time.perf_counter() - t0
    rec = {"value": n_sub / dt, "unit": "local energies/s", "cores": threads, "kind": "oracle",
           "sample": f"the first {n_sub} of the {w.n_samples} samples of the benchmark batch ({w.name}), with the "
                     f"draws of one GPU call; FP64 oracle, {build}, {dt:.1f} s"}
    e_ref = ref["eloc"]
    tau = 1e-3 * float(np.sqrt(np.mean(e_ref ** 2)))
    errs = {}
    for prec, out in keep.items():
        el = out["eloc"][:n_sub]
        dE = np.abs(el - e_ref)
        r = dE / np.maximum(np.abs(e_ref), tau)
        rec_p = {"p50": float(np.median(r)), "p99": float(np.quantile(r, 0.99)), "max": float(r.max()),
                 "dE_over_S_max": float((dE / ref["sabs"]).max())}
        if prec in cols:
            bound = ref["ebound"][:, cols.index(prec)]
            ok = ref["margin_f"] >= 8 * U_F      # a correlator this close to a zero has no bound
            rec_p["bound_ratio_max"] = float((dE[ok] / bound[ok]).max()) if ok.any() else None
            rec_p["bound_over_S_p50"] = float(np.median(bound / ref["sabs"]))
            rec_p["samples_without_bound"] = int((~ok).sum())
        errs[prec] = rec_p
    return rec, errs


def run_eloc_bench(args):
    import numpy as np
    import torch
    from paper_2507_19276_amd import nqs, workloads

    torch.cuda.set_device(0)
    ctx = nqs.Context(0)
    if args.copy_calibration_mib:
        nbytes = args.copy_calibration_mib << 20
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"# copy calibration: {nbytes} bytes read, {nbytes} bytes written", file=sys.stderr)
    precs = list(dict.fromkeys(args.precisions.split(",")))
    head_prec = precs[0]
    head_name = args.workload
    other = "c2" if head_name == "c3" else "c3"
    ref_seed = 424242
    Wh = setup_workload(nqs, workloads, ctx, head_name)
    print(f"# {head_name}: {Wh['w'].n_samples} distinct samples from {Wh['n_draws']} draws of Phi^2 "
          f"({Wh['added']} topped up)", file=sys.stderr, flush=True)
    results, keep = time_precisions(nqs, ctx, Wh, precs, args.steps, args.warmup, args.full_recompute,
                                    ref_seed=None if args.no_cpu_baseline else ref_seed)
    N = Wh["w"].n_samples
    head = results[head_prec]
    hs = head["stats"]
    achieved = hs["psi_flops"] / (hs["ms_psi"] * 1e-3) / 1e12
    peak = PEAKS[head_prec]
    wh = Wh["w"]
    line = {
        "metric": "local energies/sec at fixed bond dim D",
        "value": head["value"],
        "unit": "local energies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head_prec,
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[head_name], "global_batch": N, "precision": head_prec,
                   "samples_from": f"{Wh['n_draws']} exact draws of Phi^2 (nqs_sample, seed {Wh['sample_seed']}), "
                                   f"{Wh['added']} topped up"},
        "rows_per_step": hs["n_rows"],
        "site_rows_per_step": hs["n_site_rows"],
        "by_precision": {p: {"value": r["value"], "ms_per_step": r["ms_per_step"],
                             "row_kernel_ms": r["stats"]["ms_psi"],
                             "row_kernel_tflops": r["stats"]["psi_flops"] / r["stats"]["ms_psi"] / 1e9,
                             "row_kernel_frac_of_peak": r["stats"]["psi_flops"] / r["stats"]["ms_psi"] / 1e9
                             / PEAKS[p],
                             "stages_ms": {k: r["stats"][k] for k in ("ms_enumerate", "ms_draw", "ms_rows",
                                                                       "ms_amplitude", "ms_reduce")},
                             "H_elements_per_s_enumerate": N * int(Wh["inst"].n_conn)
                             / (r["stats"]["ms_enumerate"] * 1e-3),
                             "batch_energy": r["E"]} for p, r in results.items()},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": args.traffic_bytes if args.traffic_bytes else measured_traffic(head_name, head_prec),
                     "kernel": "k_psi_mt (row amplitude kernel: bond contractions and conditionals)",
                     "flops_per_launch": hs["psi_flops"], "ms_per_launch": hs["ms_psi"],
                     "kernel_sha16": kernel_sha16()},
    }
    if not args.headline_only:
        Wo = setup_workload(nqs, workloads, ctx, other)
        ro, _ = time_precisions(nqs, ctx, Wo, precs, max(2, args.steps // 2), 1)
        line[other] = {"workload": WORKLOAD_TEXT[other],
                       "by_precision": {p: {"value": r["value"], "ms_per_step": r["ms_per_step"],
                                            "row_kernel_ms": r["stats"]["ms_psi"],
                                            "row_kernel_frac_of_peak": r["stats"]["psi_flops"]
                                            / r["stats"]["ms_psi"] / 1e9 / PEAKS[p]}
                                        for p, r in ro.items()}}
        eq = {}
        for Wx, n_sub in ((Wh, 256 if head_name == "c3" else Wh["w"].n_samples),
                          (Wo, 256 if other == "c3" else Wo["w"].n_samples)):
            eq[Wx["w"].name] = equal_error(nqs, ctx, Wx, precs, n_sub)
            print(f"# equal error {Wx['w'].name}: " + ", ".join(
                f"{p} rms {eq[Wx['w'].name][p]['rms_error']:.3e}" for p in precs), file=sys.stderr, flush=True)
        line["equal_energy_error"] = eq
        del Wo
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        rec, errs = cpu_baseline(Wh, keep, ref_seed, 256 if head_name == "c3" else Wh["w"].n_samples, threads)
        line["cpu_baseline"] = rec
        line["eloc_error_vs_fp64_oracle"] = errs
    print(json.dumps(line), flush=True)


def run_serve_bench(args):
    import numpy as np
    import torch
    from paper_2507_19276_amd import nqs, workloads

    torch.cuda.set_device(0)
    ctx = nqs.Context(0)
    objs, pools = [], []
    for k, s in enumerate(workloads.serving_instances()):
        inst = nqs.Instance(ctx, s["K"], s["n_alpha"], s["n_beta"], s["h"], s["eri"])
        ans = nqs.Ansatz(ctx, s["K"], s["n_alpha"], s["n_beta"], s["chi"], s["parent_ptr"], s["parent_idx"], 0)
        ans.bind(s["params"])
        objs.append((s, inst, ans))
        pool = workloads.random_onvs(s["K"], s["n_alpha"], s["n_beta"], 16384, 500 + k)
        pools.append(torch.from_numpy(pool.view(np.int64)).cuda().contiguous())
    eps, n_eps, prec = 1e-2, 100, "bf16"
    # capacity: per-sample service time of every instance, one request at a time
    tps = []
    for (s, inst, ans), pool in zip(objs, pools):
        n = 2048
        nqs.eloc(ctx, inst, ans, pool[:n], eps=eps, n_eps=n_eps, precision=prec, seed=1, max_rows_per_pass=args.max_rows)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nqs.eloc(ctx, inst, ans, pool[:n], eps=eps, n_eps=n_eps, precision=prec, seed=2, max_rows_per_pass=args.max_rows)
        torch.cuda.synchronize()
        tps.append((time.perf_counter() - t0) / n)
    reqs = workloads.serving_requests(args.requests, 1.0, len(objs), seed=20250725)
    mean_service = float(np.mean([r["n"] * tps[r["instance"]] for r in reqs]))
    capacity = 1.0 / mean_service
    lam = args.load * capacity
    print(f"# serving: capacity {capacity:.2f} req/s (serial), arrival rate {lam:.2f} req/s", file=sys.stderr, flush=True)
    gaps = np.random.default_rng(7).exponential(1.0 / lam, args.requests)
    t_arr = np.cumsum(gaps) - gaps[0]
    srv = nqs.Server(ctx, n_slots=args.slots, budget_bytes=args.budget_gib << 30, max_rows_per_pass=args.max_rows)
    rng = np.random.default_rng(11)
    total = {"n": 0}
    lat, qd, nsamp = [], [], []
    done = threading.Event()

    def collector():
        got = 0
        while got < args.requests:
            c = srv.wait(300.0)
            if c is None:
                break
            if c["status"] != 0:
                print("# request failed:", c["message"], file=sys.stderr)
            lat.append(c["t_end"] - c["t_submit"])
            qd.append(c["t_start"] - c["t_submit"])
            nsamp.append(c["stats"]["n_samples"])
            got += 1
        done.set()

    th = threading.Thread(target=collector)
    th.start()
    t_base = nqs.monotonic() + 0.05
    for k, r in enumerate(reqs):
        s, inst, ans = objs[r["instance"]]
        off = int(rng.integers(0, 16384 - r["n"] + 1))
        smp = pools[r["instance"]][off:off + r["n"]]
        target = t_base + t_arr[k]
        while nqs.monotonic() < target:
            time.sleep(min(0.002, max(0.0, target - nqs.monotonic())))
        srv.submit(inst, ans, smp, eps=eps, n_eps=n_eps, precision=prec, seed=r["seed"], t_arrival=target, tag=k)
    done.wait()
    th.join()
    t_end = nqs.monotonic()
    info = srv.info()
    srv.close()
    makespan = t_end - t_base
    lat_ms = np.array(lat) * 1e3
    line = {
        "metric": "serving: total local energies/s with p50/p99 request latency",
        "value": float(np.sum(nsamp)) / makespan,
        "unit": "local energies/s",
        "n_gpus": 1,
        "steps": args.requests,
        "warmup": 0,
        "ms_per_step": makespan / args.requests * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": "serving: 12 instances norb {12,20,36,50} x chi {16,32,64}, half filling, "
                               "NN+NNN BDG-RNN, eps=1e-2, N_eps=100, batch log-uniform 256-16384",
                   "requests": args.requests, "arrival_rate_hz": lam, "load": args.load,
                   "slots": args.slots, "budget_gib": args.budget_gib, "max_rows_per_pass": args.max_rows},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                       "max": float(lat_ms.max()), "mean": float(lat_ms.mean())},
        "queue_delay_ms": {"p50": float(np.percentile(qd, 50) * 1e3), "p99": float(np.percentile(qd, 99) * 1e3)},
        "capacity_req_per_s_serial": capacity,
        "peak_in_flight": info["peak_in_flight"],
        "peak_reserved_gib": info["peak_reserved"] / 2 ** 30,
        "completed": len(lat),
    }
    print(json.dumps(line), flush=True)


def run_next_bench(args):
    """The paths beyond the local energy of the BDG-RNN: exact sampling, the
    Ising-RBM correlator, the BDG-TensorRNN and one VMC step, each timed on its
    own synthetic workload (chain K=20, 10a+10b) with a roofline of its
    dominant kernel.  One JSON line."""
    import numpy as np
    import torch
    from paper_2507_19276_amd import nqs, workloads

    torch.cuda.set_device(0)
    ctx = nqs.Context(0)

    def make(name):
        w = workloads.make_workload(name)
        inst = nqs.Instance(ctx, w.K, w.n_alpha, w.n_beta, w.h, w.eri, w.e_core)
        ans = nqs.Ansatz(ctx, w.K, w.n_alpha, w.n_beta, w.chi, w.parent_ptr, w.parent_idx, w.n_hidden,
                         ising=w.ising, tensor=w.tensor, cplx=w.cplx)
        ans.bind(w.params)
        s = torch.from_numpy(w.samples.view(np.int64)).cuda().contiguous()
        return w, inst, ans, s

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, r

    out = {}
    # exact sampling (k_psi_mt in sampling mode + radix-sort merge), chain chi=16
    w, inst, ans, s = make("c2")
    site_flops = 8.0 * w.chi * w.chi * float(w.parent_ptr[-1])   # per draw, all sites
    samp = {}
    for prec in ("f32", "f64"):
        nd = 10_000_000
        dt, r = timed(lambda: ans.sample(nd, seed=3, precision=prec), 3)
        fl = nd * site_flops / dt / 1e12
        samp[prec] = {"draws": nd, "ms": dt * 1e3, "draws_per_s": nd / dt, "unique": r[4],
                      "roofline": {"bound": "mfma", "achieved": fl, "peak": PEAKS[prec], "unit": "TFLOP/s",
                                   "frac": fl / PEAKS[prec],
                                   "note": "whole call (draws and unique merge) against the contraction flops"}}
        print(f"# sampler {prec}: {nd / dt:.3e} draws/s", file=sys.stderr, flush=True)
    out["sampler_chain_K20_chi16"] = samp
    # Ising-RBM correlator, N_h = 80, 4096 samples
    w, inst, ans, s = make("c2i")
    kw = dict(eps=w.eps, n_eps=w.n_eps, precision="f32", stream_id=0)
    dt, (o, st) = timed(lambda: nqs.eloc(ctx, inst, ans, s, seed=w.seed, **kw), 5)
    # table reads of the row update: theta, up to 4 E entries and 6 S pairs per hidden unit (FP32)
    byts = st["n_rows"] * w.n_hidden * 11 * 4
    gbs = byts / (st["ms_reduce"] * 1e-3) / 1e9
    out["ising_rbm_chain_K20_nh80"] = {
        "local_energies_per_s": w.n_samples / dt, "ms_per_step": dt * 1e3, "rows": st["n_rows"],
        "correlator_and_reduce_ms": st["ms_reduce"], "amplitude_ms": st["ms_amplitude"],
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0,
                     "kernel": "k_ising_rows<float,float>",
                     "note": "table bytes read per row (reused from L2), over the correlator and reduce stage"}}
    print(f"# ising: {w.n_samples / dt:.0f} E_loc/s, correlator stage {st['ms_reduce']:.2f} ms", file=sys.stderr,
          flush=True)
    # BDG-TensorRNN, NN+NNN chi=16 (chi' = 7), 4096 samples
    w, inst, ans, s = make("c2t")
    tens = {}
    for prec in ("f32", "f64"):
        kw = dict(eps=w.eps, n_eps=w.n_eps, precision=prec, stream_id=0)
        dt, (o, st) = timed(lambda: nqs.eloc(ctx, inst, ans, s, seed=w.seed, **kw), 3)
        fl = st["psi_flops"] / (st["ms_psi"] * 1e-3) / 1e12
        tens[prec] = {"local_energies_per_s": w.n_samples / dt, "ms_per_step": dt * 1e3,
                      "row_kernel_ms": st["ms_psi"], "site_rows": st["n_site_rows"],
                      "roofline": {"bound": "mfma", "achieved": fl, "peak": PEAKS[prec], "unit": "TFLOP/s",
                                   "frac": fl / PEAKS[prec],
                                   "kernel": f"k_psi_mt<{'float' if prec == 'f32' else 'double'},16,...,TN> (rows)",
                                   "flops_per_launch": st["psi_flops"],
                                   "note": "algorithmic flops (chi' = 7 unpadded) of the resumed rows"}}
        print(f"# tensor {prec}: {w.n_samples / dt:.0f} E_loc/s, row kernel {st['ms_psi']:.2f} ms, {fl:.2f} TFLOP/s",
              file=sys.stderr, flush=True)
    out["bdg_tensor_rnn_nnn_K20_chi16"] = tens
    # complex parameters, chain chi=16 complex units (the realified 32-unit state on MFMA), 4096 samples
    w, inst, ans, s = make("c2c")
    cx = {}
    for prec in ("f32", "f64"):
        kw = dict(eps=w.eps, n_eps=w.n_eps, precision=prec, stream_id=0)
        dt, (o, st) = timed(lambda: nqs.eloc_complex(ctx, inst, ans, s, seed=w.seed, **kw), 3)
        fl = st["psi_flops"] / (st["ms_psi"] * 1e-3) / 1e12
        cx[prec] = {"local_energies_per_s": w.n_samples / dt, "ms_per_step": dt * 1e3,
                    "row_kernel_ms": st["ms_psi"], "site_rows": st["n_site_rows"], "E_im": st["E_im"],
                    "roofline": {"bound": "mfma", "achieved": fl, "peak": PEAKS[prec], "unit": "TFLOP/s",
                                 "frac": fl / PEAKS[prec], "flops_per_launch": st["psi_flops"],
                                 "kernel": f"k_psi_mt<{'float' if prec == 'f32' else 'double'},32,...,CPLX>"}}
        print(f"# complex {prec}: {w.n_samples / dt:.0f} E_loc/s, row kernel {st['ms_psi']:.2f} ms, "
              f"{fl:.2f} TFLOP/s", file=sys.stderr, flush=True)
    p = torch.from_numpy(w.params.copy()).cuda()
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    steps = []
    for k in range(1, 4):
        t0 = time.perf_counter()
        st = nqs.vmc_step(ctx, inst, ans, p, m, v, k, n_draws=4096, sample_seed=k, draw_base=4096 * k,
                          eps=w.eps, n_eps=w.n_eps, precision="f32", seed=k, lr=1e-3)
        steps.append((time.perf_counter() - t0, st))
    cx["vmc_step_ms"] = float(np.mean([t for t, _ in steps[1:]])) * 1e3
    cx["vmc_stage_ms"] = {k: steps[-1][1][k] for k in ("ms_sample", "ms_eloc", "ms_grad", "ms_update")}
    out["complex_chain_K20_chi16"] = cx
    print(f"# complex vmc step: {cx['vmc_step_ms']:.2f} ms", file=sys.stderr, flush=True)
    # one VMC step (4096 draws, FP32 path), chain chi=16
    w, inst, ans, s = make("c2")
    p = torch.from_numpy(w.params.copy()).cuda()
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    steps = []
    for k in range(1, 5):
        t0 = time.perf_counter()
        st = nqs.vmc_step(ctx, inst, ans, p, m, v, k, n_draws=4096, sample_seed=k, draw_base=4096 * k,
                          eps=w.eps, n_eps=w.n_eps, precision="f32", seed=k, lr=1e-3)
        steps.append((time.perf_counter() - t0, st))
    dt = float(np.mean([t for t, _ in steps[1:]]))
    last = steps[-1][1]
    out["vmc_step_chain_K20_chi16"] = {"ms_per_step": dt * 1e3, "n_unique": last["n_unique"],
                                       "stage_ms": {k: last[k] for k in ("ms_sample", "ms_eloc", "ms_grad",
                                                                          "ms_update")},
                                       "E": [st["E"] for _, st in steps]}
    print(f"# vmc step: {dt * 1e3:.2f} ms", file=sys.stderr, flush=True)
    line = {
        "metric": "next rows: exact sampling, Ising-RBM, BDG-TensorRNN and complex-parameter local energies, "
                  "VMC step",
        "value": out["sampler_chain_K20_chi16"]["f32"]["draws_per_s"],
        "unit": "draws/s (FP32 sampler; the other figures in the sub-objects)",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": out["sampler_chain_K20_chi16"]["f32"]["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "chain K=20 10a+10b: c2 (chain chi=16), c2i (+Ising-RBM N_h=80), "
                               "c2t (NN+NNN BDG-TensorRNN chi=16), c2c (chain, complex chi=16)"},
        **out,
    }
    print(json.dumps(line), flush=True)


def run_configs_bench(args):
    """The other synthetic configurations at one GPU: K=50 with the cos-RBM
    (BF16 against FP32 and FP64), the dense K=20 and the 3x3x2 lattice K=18 at
    chi=64 (FP32 and FP64 local energies, FP32 and FP64 gradients of 8192
    samples).  Per precision: throughput, stage times, the row kernel against
    its MFMA peak, and the batch energy against the FP64 GPU path in units of its
    sampling standard error (equal energy error).  One JSON line."""
    import numpy as np
    import torch
    from paper_2507_19276_amd import nqs, workloads

    torch.cuda.set_device(0)
    ctx = nqs.Context(0)
    out = {}
    plan = {"c3": ("bf16", "f32", "f64"), "c4a": ("f32", "f64"), "c4b": ("f32", "f64")}
    for name, precs in plan.items():
        w = workloads.make_workload(name)
        inst = nqs.Instance(ctx, w.K, w.n_alpha, w.n_beta, w.h, w.eri, w.e_core)
        ans = nqs.Ansatz(ctx, w.K, w.n_alpha, w.n_beta, w.chi, w.parent_ptr, w.parent_idx, w.n_hidden)
        ans.bind(w.params)
        s = torch.from_numpy(w.samples.view(np.int64)).cuda().contiguous()
        res, energies = {}, {}
        for prec in precs:
            kw = dict(eps=w.eps, n_eps=w.n_eps, precision=prec, seed=w.seed, stream_id=0)
            nqs.eloc(ctx, inst, ans, s, **kw)
            torch.cuda.synchronize()
            reps = 2
            t0 = time.perf_counter()
            for _ in range(reps):
                o, st = nqs.eloc(ctx, inst, ans, s, **kw)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            el = o["eloc"].cpu().numpy()
            f2 = o["fsq"].cpu().numpy()
            ok = np.isfinite(el)
            E = float(st["E"])
            # standard error of the |f|^2-weighted mean (a self-normalised estimator):
            # sqrt(sum w^2 (E_loc - E)^2) / sum w, and its effective sample count
            wf = f2[ok]
            se = float(np.sqrt((wf ** 2 * (el[ok] - E) ** 2).sum()) / wf.sum())
            ess = float(wf.sum() ** 2 / (wf ** 2).sum())
            energies[prec] = (E, se)
            fl = st["psi_flops"] / (st["ms_psi"] * 1e-3) / 1e12
            res[prec] = {"local_energies_per_s": w.n_samples / dt, "ms_per_step": dt * 1e3, "rows": st["n_rows"],
                         "site_rows": st["n_site_rows"], "E": E, "sampling_se": se, "effective_samples": ess,
                         "stage_ms": {k: st[k] for k in ("ms_enumerate", "ms_draw", "ms_rows", "ms_amplitude",
                                                          "ms_reduce", "ms_psi")},
                         "roofline": {"bound": "mfma", "achieved": fl, "peak": PEAKS[prec], "unit": "TFLOP/s",
                                      "frac": fl / PEAKS[prec], "flops_per_launch": st["psi_flops"],
                                      "kernel": "row amplitude kernel"}}
            print(f"# {name} {prec}: {w.n_samples / dt:.0f} E_loc/s, {st['n_rows']} rows, row kernel "
                  f"{st['ms_psi']:.1f} ms at {fl:.1f} TFLOP/s", file=sys.stderr, flush=True)
        E64, se64 = energies["f64"]
        for prec in precs:
            res[prec]["energy_error_in_se_vs_f64_gpu"] = abs(energies[prec][0] - E64) / se64
        if name in ("c4a", "c4b"):
            g = torch.randn(w.n_samples, dtype=torch.float64, device="cuda")
            for prec in ("f32", "f64"):
                ans.vjp(s, g, prec)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ans.vjp(s, g, prec)
                torch.cuda.synchronize()
                res[f"vjp_{prec}_ms"] = (time.perf_counter() - t0) * 1e3
                print(f"# {name} vjp {prec}: {res[f'vjp_{prec}_ms']:.1f} ms", file=sys.stderr, flush=True)
        res["workload"] = {"K": w.K, "n_alpha": w.n_alpha, "n_beta": w.n_beta, "chi": w.chi, "n_hidden": w.n_hidden,
                           "samples": w.n_samples, "eps": w.eps, "n_eps": w.n_eps}
        out[name] = res
        del inst, ans
    line = {
        "metric": "local energies/sec at fixed bond dim D on the other configurations",
        "value": out["c3"]["bf16"]["local_energies_per_s"], "unit": "local energies/s (c3, BF16; the rest below)",
        "n_gpus": 1, "steps": 2, "warmup": 1, "ms_per_step": out["c3"]["bf16"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "c3 K=50 NN+NNN chi=32 cos-RBM N_h=100 16384 samples; c4a K=20 15a+15b dense "
                               "NN+NNN chi=64 8192 samples; c4b K=18 3x3x2 lattice chi=64 8192 samples"},
        **out,
    }
    print(json.dumps(line), flush=True)


def run_speedups_bench(args):
    """Exact against semi-stochastic local energies (Sec. 3: every connected
    determinant as a deterministic row, eps = 0, against the screened set plus
    N_eps draws), FP64 as in the paper, on the hydrogen-chain stand-ins whose
    relative costs the paper reports: K = 16 / 32 / 48 with chi = 50 and
    2048 samples (eps = 0.01, N_eps = 100), and K = 50 with chi = 10.  The
    semi-stochastic side runs the 2048 samples in one call; the exact side runs
    a 64-sample subset of them (its rows per sample are the closed-form N_conn)
    in passes of at most 8 M rows, and both are reported per sample.  One JSON
    line."""
    import numpy as np
    import torch
    from paper_2507_19276_amd import nqs, workloads

    torch.cuda.set_device(0)
    ctx = nqs.Context(0)
    cases = [(16, 50), (32, 50), (48, 50), (50, 10)]
    res = []
    for K, chi in cases:
        h, eri = workloads.chain_integrals(K, 20250725 + 31 * K)
        pp, pi = workloads.graph_chain(K)
        params = workloads.ansatz_params(K, chi, pp, pi, 0, 20250725 + 31 * K + 1)
        na = nb = K // 2
        smp = workloads.random_onvs(K, na, nb, 2048, 20250725 + 31 * K + 2)
        inst = nqs.Instance(ctx, K, na, nb, h, eri, 0.0)
        ans = nqs.Ansatz(ctx, K, na, nb, chi, pp, pi, 0)
        ans.bind(params)
        one = {}
        for mode, eps, n_eps, n in (("semi", 0.01, 100, 2048), ("exact", 0.0, 0, 64)):
            s = torch.from_numpy(smp[:n].view(np.int64)).cuda().contiguous()
            kw = dict(eps=eps, n_eps=n_eps, precision="f64", seed=7, stream_id=0, max_rows_per_pass=8_000_000)
            nqs.eloc(ctx, inst, ans, s, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            o, st = nqs.eloc(ctx, inst, ans, s, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            one[mode] = {"samples": n, "rows_per_sample": st["n_rows"] / n, "ms_per_sample": dt * 1e3 / n,
                         "amplitude_ms_per_sample": st["ms_amplitude"] / n, "E_loc_mean": float(o["eloc"].mean())}
            print(f"# K={K} chi={chi} {mode}: {st['n_rows'] / n:.0f} rows/sample, {dt * 1e3 / n:.4f} ms/sample",
                  file=sys.stderr, flush=True)
        res.append({"K": K, "chi": chi, "graph": "chain", **one,
                    "time_ratio": one["exact"]["ms_per_sample"] / one["semi"]["ms_per_sample"],
                    "amplitude_time_ratio": one["exact"]["amplitude_ms_per_sample"]
                    / one["semi"]["amplitude_ms_per_sample"],
                    "rows_ratio": one["exact"]["rows_per_sample"] / one["semi"]["rows_per_sample"]})
    line = {"metric": "exact / semi-stochastic local-energy time per sample", "unit": "ratio", "n_gpus": 1,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": "hydrogen-chain stand-ins: chain integrals, chain BDG-RNN, half filling, "
                                   "eps=0.01, N_eps=100 against eps=0"},
            "paper_context": {"psi_evaluation_speedup_K16_32_48_chi50": [43, 418, 1359],
                              "eloc_cost_fraction_K50_chi10": 0.0005},
            "cases": res}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precisions", default="f64,f32,bf16,bf16x3",
                    help="comma list; the first is the headline")
    ap.add_argument("--workload", default="c3", choices=("c2", "c3"),
                    help="headline workload: c3 (K=50, chi=32, cos-RBM, 16384 samples) or c2 (K=20, chi=16)")
    ap.add_argument("--headline-only", action="store_true",
                    help="skip the second workload and the equal-energy-error study")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--full-recompute", action="store_true",
                    help="evaluate every amplitude row from site 0 (no resumption at the first changed site)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device copy of this size first (scales PMC byte counters)")
    ap.add_argument("--traffic-bytes", type=float, default=None,
                    help="HBM bytes per amplitude-kernel launch from rocprofv3 PMC counters")
    ap.add_argument("--serve", action="store_true")
    ap.add_argument("--next", action="store_true",
                    help="time the sampler, the Ising-RBM, BDG-TensorRNN and complex paths and one VMC step")
    ap.add_argument("--configs", action="store_true",
                    help="time the K=50, dense K=20 and lattice K=18 configurations per precision")
    ap.add_argument("--speedups", action="store_true",
                    help="exact against semi-stochastic local energies on the hydrogen-chain stand-ins (FP64)")
    ap.add_argument("--requests", type=int, default=500)
    ap.add_argument("--load", type=float, default=0.8)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gib", type=int, default=64)
    ap.add_argument("--max-rows", type=int, default=4_000_000)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(samples would be sharded across GPUs with one scalar all-reduce)", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        run_serve_bench(args)
    elif args.next:
        run_next_bench(args)
    elif args.configs:
        run_configs_bench(args)
    elif args.speedups:
        run_speedups_bench(args)
    else:
        run_eloc_bench(args)


if __name__ == "__main__":
    main()
