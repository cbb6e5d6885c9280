"""Sample batches drawn exactly from Phi^2 with the oracle's counter-keyed
sampler: the same rule as the benchmark's batch (which the library's sampler
draws bit for bit alike, tests/test_gpu_sampler.py), so parity tests at full
size see the benchmark's inputs without taking them from the HIP path."""
import functools

import numpy as np

import oracle
from paper_2507_19276_amd import workloads as W


@functools.lru_cache(maxsize=8)
def batch(name: str):
    """(workload, samples uint64 [N, 2] ascending, counts int64 [N], draws)."""
    w = W.make_workload(name)
    seed = w.seed + W.PHI2_SEED_OFFSET

    def draw(n):
        return oracle.sample_unique(w.K, w.chi, w.n_alpha, w.n_beta, w.parent_ptr, w.parent_idx, w.params, seed, n)

    u, c, n = W.draw_until_unique(draw, w.n_samples)
    u, c, _ = W.top_up(u, c, w.K, w.n_alpha, w.n_beta, w.n_samples, seed)
    return w, u, c, n
