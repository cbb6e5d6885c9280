"""Throughput of the semi-stochastic local energy on one MI355X.

One step = one nqs_eloc call over the whole synthetic batch of the chain
workload (K = 20 spatial orbitals, 10a+10b, chain BDG-RNN chi = 16, 4096 unique
samples, eps = 1e-3, N_eps = 64): enumerate every connected determinant,
screen, draw, evaluate the amplitude of every row, reduce.  Inputs (integrals,
parameters, samples) are resident in HBM before the timed region.

Prints one JSON line (see the design doc for the fields).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "c2"


def algorithmic_flops_per_row(chi, parent_ptr):
    # 4 candidates x chi outputs x (d_i chi) inputs x 2 flops, summed over sites
    return 8 * chi * chi * int(parent_ptr[-1])


def cpu_baseline(w, n_sub, eps, n_eps, seed):
    import numpy as np
    import oracle
    threads = os.cpu_count() or 1
    sub = w.samples[:n_sub]
    t0 = time.perf_counter()
    oracle.eloc(w.K, w.n_alpha, w.n_beta, w.h, w.eri, w.chi, w.parent_ptr, w.parent_idx, w.n_hidden,
                w.params, sub, eps=eps, n_eps=n_eps, seed=seed, stream=0, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": n_sub / dt, "unit": "local energies/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_sub} of {w.n_samples} samples of the same workload, FP64 oracle, "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="f32", choices=["f64", "f32", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=4096)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(samples would be sharded across GPUs with one scalar all-reduce)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2507_19276_amd import nqs, workloads

    torch.cuda.set_device(0)
    w = workloads.make_workload(WORKLOAD)
    ctx = nqs.Context(0)
    inst = nqs.Instance(ctx, w.K, w.n_alpha, w.n_beta, w.h, w.eri, w.e_core)
    ans = nqs.Ansatz(ctx, w.K, w.n_alpha, w.n_beta, w.chi, w.parent_ptr, w.parent_idx, w.n_hidden)
    ans.bind(w.params)
    samples = torch.from_numpy(w.samples.view(np.int64)).cuda().contiguous()
    N = w.n_samples

    def step(k, prec):
        return nqs.eloc(ctx, inst, ans, samples, eps=w.eps, n_eps=w.n_eps, precision=prec,
                        seed=w.seed + k, stream_id=0)

    results = {}
    for prec in dict.fromkeys([args.precision, "f64", "f32", "bf16"]):
        for k in range(args.warmup):
            step(k, prec)
        torch.cuda.synchronize()
        psi_ms, rows = [], []
        t0 = time.perf_counter()
        for k in range(args.steps):
            out, st = step(1000 + k, prec)
            psi_ms.append(st["ms_amplitude"])
            rows.append(st["n_rows"])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        results[prec] = dict(dt=dt, psi_ms=float(np.mean(psi_ms)), rows=float(np.mean(rows)), st=st)
        print(f"# {prec}: {args.steps} steps in {dt:.3f} s, rows/step {np.mean(rows):.0f}, "
              f"amplitude kernel {np.mean(psi_ms):.3f} ms", file=sys.stderr, flush=True)

    head = results[args.precision]
    value = args.steps * N / head["dt"]
    flops = algorithmic_flops_per_row(w.chi, w.parent_ptr) * head["rows"]
    achieved = flops / (head["psi_ms"] * 1e-3) / 1e12
    peak = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}[args.precision]
    line = {
        "metric": "local energies/sec at fixed bond dim D",
        "value": value,
        "unit": "local energies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["dt"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": "chain K=20 10a+10b, BDG-RNN chain chi=16, 4096 unique samples, "
                               "eps=1e-3, N_eps=64", "global_batch": N, "precision": args.precision},
        "rows_per_step": head["rows"],
        "by_precision": {p: {"value": args.steps * N / r["dt"], "amplitude_ms": r["psi_ms"]}
                         for p, r in results.items()},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": "k_psi (bond contractions)"},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_samples, w.eps, w.n_eps, w.seed)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
