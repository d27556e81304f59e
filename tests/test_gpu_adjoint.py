"""GPU adjoint (mm_adjoint) against the oracle's reverse-mode gradient, and
its own consistency: independence of the checkpoint spacing, the state left
unchanged, central differences of the HIP forward path, autograd."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as A
from tests import test_oracle_adjoint as OA

pytestmark = pytest.mark.gpu


def _gpu(ckpt, steps=OA.STEPS, fixed_iter=0, eps=None, Ms=None, inner=0):
    import paper_2103_12819_amd as mm
    e0, sig, ms0, alpha, m0, prof, E, H = OA._materials()
    dt = W.cfl_dt(0.9, *OA.D)
    sim = mm.Sim(OA.N, OA.D, dt, eps_r=e0 if eps is None else eps, sigma=sig,
                 Ms=ms0 if Ms is None else Ms, alpha=alpha, m0_dir=m0, H0=(2e4, 0.0, 1.2e5),
                 source=(2, prof, 3e12, 1 / 3e12, 1e-12), tol=1e-13, max_iter=50, fixed_iter=fixed_iter)
    sim.set_fields(E=E, H=H)
    pid = sim.add_probe(1, 0, OA.I0)
    sim.enable_adjoint(ckpt, inner)
    sim.step(steps)
    return sim, pid


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def oracle_grads():
    return A.loss_and_gradients(OA._make, OA.STEPS, OA.I0)


def test_gradient_matches_oracle_adjoint(oracle_grads):
    L, ge_o, gm_o = oracle_grads
    sim, pid = _gpu(ckpt=OA.STEPS)
    _, Lg = sim.probe(pid)
    ge, gm = sim.adjoint(pid)
    assert abs(Lg - L) <= 1e-12 * abs(L)
    assert _rel(ge, ge_o) <= 1e-10, _rel(ge, ge_o)
    assert _rel(gm, gm_o) <= 1e-10, _rel(gm, gm_o)


def test_checkpoint_spacing_does_not_change_the_gradient():
    """Single-level spacings 10, 3, 1 and two-level (outer, inner) spacings
    (10, 3), (10, 1), (4, 3) give bit-identical gradients."""
    sims = [_gpu(ckpt=k) for k in (OA.STEPS, 3, 1)]
    sims += [_gpu(ckpt=k, inner=q) for k, q in ((OA.STEPS, 3), (OA.STEPS, 1), (4, 3))]
    grads = [s.adjoint(p) for s, p in sims]
    for g in grads[1:]:
        assert np.array_equal(g[0], grads[0][0]) and np.array_equal(g[1], grads[0][1])


def test_state_is_restored_and_stepping_continues():
    sim, pid = _gpu(ckpt=4)
    before = [sim.field(n) for n in ("Ex", "Hy", "Mxz", "Mzy")]
    series, S = sim.probe(pid)
    sim.adjoint(pid)
    after = [sim.field(n) for n in ("Ex", "Hy", "Mxz", "Mzy")]
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    s2, S2 = sim.probe(pid)
    assert np.array_equal(series, s2) and S == S2
    ref, _ = _gpu(ckpt=4, steps=OA.STEPS + 3)
    sim.step(3)
    assert np.array_equal(sim.field("Ez"), ref.field("Ez"))


def test_central_differences_of_the_hip_forward():
    sim, pid = _gpu(ckpt=5, fixed_iter=4)
    _, L = sim.probe(pid)
    ge, gm = sim.adjoint(pid)
    e0, _, ms0, *_ = OA._materials()
    rng = np.random.default_rng(9)
    cells = [tuple(c) for c in np.argwhere(ms0 > 0)]
    for idx in [cells[i] for i in rng.choice(len(cells), 4, replace=False)]:
        for which, g, base in (("eps", ge, e0), ("ms", gm, ms0)):
            h = 1e-6 * base[idx]
            vals = []
            for sgn in (1, -1):
                p = base.copy()
                p[idx] += sgn * h
                s2, p2 = _gpu(ckpt=5, fixed_iter=4, **({"eps": p} if which == "eps" else {"Ms": p}))
                vals.append(s2.probe(p2)[1])
                s2.close()
            fd = (vals[0] - vals[1]) / (2 * h)
            floor = 1e3 * 2.220446049250313e-16 * abs(L) / h
            assert abs(fd - g[idx]) <= 1e-6 * abs(g[idx]) + floor, (which, idx, fd, g[idx])


def test_autograd_function():
    import torch
    import paper_2103_12819_amd as mm
    cfg = W.design128(seed=0, steps=30, n=(32, 16, 8))
    eps = torch.tensor(cfg.eps_r, dtype=torch.float64, requires_grad=True)
    ms = torch.tensor(cfg.Ms, dtype=torch.float64, requires_grad=True)
    L = mm.FluxLoss.apply(eps, ms, cfg, cfg.steps, 0, "fp64", 10)
    (2.0 * L).backward()
    sim = mm.from_config(cfg)
    sim.enable_adjoint(10)
    sim.step(cfg.steps)
    ge, gm = sim.adjoint(0)
    assert np.allclose(eps.grad.numpy(), 2.0 * ge, rtol=0, atol=0)
    assert np.allclose(ms.grad.numpy(), 2.0 * gm, rtol=0, atol=0)
    assert float(np.abs(ge).max()) > 0 and float(np.abs(gm).max()) > 0


def test_second_adjoint_call_after_more_steps():
    """mm_adjoint, three more steps, mm_adjoint again: the second gradient
    equals that of a fresh run of the longer horizon (the context's work
    buffers are reused, the iterate log grown if needed)."""
    sim, pid = _gpu(ckpt=4, inner=3)
    sim.adjoint(pid)
    sim.step(3)
    g2 = sim.adjoint(pid)
    ref, rp = _gpu(ckpt=4, inner=3, steps=OA.STEPS + 3)
    gr = ref.adjoint(rp)
    assert np.array_equal(g2[0], gr[0]) and np.array_equal(g2[1], gr[1])
