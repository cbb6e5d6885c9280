"""GPU VMC step (sampling, local energies, reweighted gradient of Sec. 2.3
Eq. (19), AdamW) against the oracle's step on the same seeds: FP64 energy at
1e-10 relative, gradient at 1e-9 of its largest entry; the AdamW update
against the oracle's AdamW applied to the GPU's own gradient and state
(1e-13 relative, 1e-15 of the largest moment: only the rounding of the
update itself differs, and b1 m + (1 - b1) g may cancel), and the
parameters against the oracle's step within 1e-6 of the learning rate (AdamW
divides each gradient entry by its own magnitude, so a small entry's relative
error, not the FP64 bar on the largest, sets this); and a short optimisation
that lowers the exact energy of a small sector."""
import numpy as np
import pytest
import torch

import oracle
from bruteforce import dense_hamiltonian, int_to_words
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


def make(nqs, ctx, name):
    w = W.make_workload(name, n_samples=16)
    inst = nqs.Instance(ctx, w.K, w.n_alpha, w.n_beta, w.h, w.eri, w.e_core)
    ans = nqs.Ansatz(ctx, w.K, w.n_alpha, w.n_beta, w.chi, w.parent_ptr, w.parent_idx, w.n_hidden, ising=w.ising)
    ans.bind(w.params)
    return w, inst, ans


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("name,n_draws", [("c1", 2000), ("c1i", 2000), ("c2", 96), ("c2i", 64)])
def test_two_steps_match_oracle_f64(nqs, ctx, name, n_draws):
    w, inst, ans = make(nqs, ctx, name)
    hp = dict(lr=2e-2, beta1=0.9, beta2=0.999, adam_eps=1e-8, weight_decay=1e-3)
    p = dev(w.params)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    g = torch.zeros_like(p)
    rp, rm, rv = w.params.copy(), np.zeros(w.params.size), np.zeros(w.params.size)
    for step in (1, 2):
        kw = dict(n_draws=n_draws, sample_seed=77 + step, draw_base=step * n_draws)
        p0, m0, v0 = p.cpu().numpy(), m.cpu().numpy(), v.cpu().numpy()
        st = nqs.vmc_step(ctx, inst, ans, p, m, v, step, eps=w.eps, n_eps=w.n_eps, precision="f64", seed=w.seed,
                          stream_id=3, grad=g, **kw, **hp)
        ref = oracle.vmc_step(w.K, w.n_alpha, w.n_beta, w.h, w.eri, w.chi, w.parent_ptr, w.parent_idx, w.n_hidden,
                              rp, rm, rv, step, n_draws, kw["sample_seed"], kw["draw_base"], eps=w.eps,
                              n_eps=w.n_eps, eloc_seed=w.seed, stream=3, lr=hp["lr"], beta1=hp["beta1"],
                              beta2=hp["beta2"], adam_eps=hp["adam_eps"], weight_decay=hp["weight_decay"],
                              ising=w.ising)
        assert st["n_unique"] == len(ref["samples"])
        assert abs(st["E"] - ref["E"]) <= 1e-10 * max(1.0, abs(ref["E"]))
        gg = g.cpu().numpy()
        assert np.abs(gg - ref["grad"]).max() <= 1e-9 * np.abs(ref["grad"]).max() + 1e-12
        assert abs(st["grad_norm"] - np.linalg.norm(ref["grad"])) <= 1e-9 * np.linalg.norm(ref["grad"])
        ep, em, ev = oracle.adamw(p0, gg, m0, v0, step, hp["lr"], hp["beta1"], hp["beta2"], hp["adam_eps"],
                                  hp["weight_decay"])
        np.testing.assert_allclose(p.cpu().numpy(), ep, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(m.cpu().numpy(), em, rtol=1e-13, atol=1e-15 * np.abs(em).max())
        np.testing.assert_allclose(v.cpu().numpy(), ev, rtol=1e-13, atol=1e-15 * np.abs(ev).max())
        assert np.abs(p.cpu().numpy() - ref["params"]).max() <= 1e-6 * hp["lr"]
        rp, rm, rv = ref["params"], ref["m"], ref["v"]


def test_step_rebinds_the_ansatz(nqs, ctx):
    w, inst, ans = make(nqs, ctx, "c2")
    p = dev(w.params)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    nqs.vmc_step(ctx, inst, ans, p, m, v, 1, n_draws=64, sample_seed=1, eps=w.eps, n_eps=w.n_eps, precision="f32",
                 seed=w.seed, lr=1e-2)
    fresh = nqs.Ansatz(ctx, w.K, w.n_alpha, w.n_beta, w.chi, w.parent_ptr, w.parent_idx, w.n_hidden)
    fresh.bind(p)
    for prec in ("f64", "f32"):
        a, sa = ans.logpsi(w.samples, prec)
        b, sb = fresh.logpsi(w.samples, prec)
        assert torch.equal(a, b) and torch.equal(sa, sb)


def test_f32_step_close_to_f64(nqs, ctx):
    """FP32 sampling, amplitudes and adjoint: the same draws up to boundary
    cases, and a gradient within the FP32 adjoint bound (1e-3 of its largest
    entry) plus the statistical effect of a few changed draws."""
    res = {}
    for prec in ("f64", "f32"):
        w, inst, ans = make(nqs, ctx, "c1i")
        p = dev(w.params)
        m, v, g = torch.zeros_like(p), torch.zeros_like(p), torch.zeros_like(p)
        st = nqs.vmc_step(ctx, inst, ans, p, m, v, 1, n_draws=4000, sample_seed=9, precision=prec, seed=w.seed,
                          lr=1e-2, grad=g)
        res[prec] = (st, g.cpu().numpy())
    (s64, g64), (s32, g32) = res["f64"], res["f32"]
    assert abs(s64["E"] - s32["E"]) <= 1e-4 * abs(s64["E"])
    assert np.abs(g64 - g32).max() <= 2e-3 * np.abs(g64).max()


def test_optimisation_lowers_the_exact_energy(nqs, ctx):
    """40 FP64 steps on the K=6 (3a, 3b) sector with the Ising-RBM correlator:
    the exact energy <Psi|H|Psi>/<Psi|Psi> (dense H over the sector) drops and
    stays above the FCI ground state."""
    w, inst, ans = make(nqs, ctx, "c1i")
    basis, H = dense_hamiltonian(w.h, w.eri, w.n_alpha, w.n_beta)
    keys = np.array([int_to_words(int(b)) for b in basis], dtype=np.uint64)
    E0 = np.linalg.eigvalsh(H)[0]

    def exact(params):
        a = oracle.amplitudes(w.K, w.chi, w.n_alpha, w.n_beta, w.parent_ptr, w.parent_idx, w.n_hidden, params, keys,
                              ising=True)
        psi = a["sign"] * np.exp(a["logabs"])
        return psi @ H @ psi / (psi @ psi)

    p = dev(w.params)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    e_start = exact(w.params)
    for step in range(1, 41):
        nqs.vmc_step(ctx, inst, ans, p, m, v, step, n_draws=4000, sample_seed=1000 + step,
                     draw_base=4000 * step, precision="f64", seed=step, lr=2e-2)
    e_end = exact(p.cpu().numpy())
    print(f"exact energy {e_start:.6f} -> {e_end:.6f} (FCI {E0:.6f})")
    assert e_end >= E0 - 1e-9
    assert e_start - e_end >= 0.3 * (e_start - E0)


def test_bad_arguments(nqs, ctx):
    w, inst, ans = make(nqs, ctx, "c1")
    p = dev(w.params)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    with pytest.raises(nqs.NqsError):
        nqs.vmc_step(ctx, inst, ans, p, m, v, 0, n_draws=10)
    with pytest.raises(nqs.NqsError):
        nqs.vmc_step(ctx, inst, ans, p, m, v, 1, n_draws=0)
    with pytest.raises(nqs.NqsError):
        nqs.vmc_step(ctx, inst, ans, p, m, v, 1, n_draws=10, beta1=1.0)
