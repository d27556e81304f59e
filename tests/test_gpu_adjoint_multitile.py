"""GPU adjoint against the oracle's reverse-mode gradient on a grid with
several bulk tiles in x and y (96 x 12 x 10: two tiles of 64 columns in x,
three of 4 rows in y), magnetic faces in some tiles only (so both near tiles
and far tiles, which take the fused two-half-step pass inside a run, are
recomputed by the adjoint), a lossy dielectric background, a soft port
source, a flux plane in a far tile, 30 steps and two-level checkpoints
(every 10 steps, 3 inside a segment) as well as single-level ones.

Bar: the loss within 1e-12 and both gradients (eps_r, Ms cell maps) within
1e-10 normwise relative of the oracle's (the bar of the single-tile case).
"""
import numpy as np
import pytest

import workloads as W
from oracle import Simulation
from oracle import adjoint as A

pytestmark = pytest.mark.gpu
N = (96, 12, 10)
D = (1e-6, 1.2e-6, 0.9e-6)
I0 = 70
STEPS = 30


def _materials():
    rng = np.random.default_rng(21)
    shp = (N[2], N[1], N[0])
    eps = rng.uniform(1.0, 4.0, shp)
    sig = rng.uniform(0.0, 5e3, shp)
    Ms = np.zeros(shp)
    Ms[2:7, 1:5, 34:62] = rng.uniform(1e5, 1.8e5, (5, 4, 28))
    alpha = np.where(Ms > 0, rng.uniform(0.01, 0.05, shp), 0.0)
    m0 = np.zeros((3,) + shp)
    m0[0], m0[1], m0[2] = 0.3, -0.2, 1.0
    prof = np.zeros(W.edge_shape(N, (False,) * 3, 2))
    prof[:, 1:N[1], 4] = 1e11 * np.sin(np.pi * np.arange(1, N[1]) / N[1])[None, :]
    E, H = W.random_fields(W.Config("a", N, D, 1.0, 0), seed=5, amp_e=3e5, amp_h=3e3)
    return eps, sig, Ms, alpha, m0, prof, E, H


def _oracle():
    e0, sig, ms0, alpha, m0, prof, E, H = _materials()
    sim = Simulation(N, D, W.cfl_dt(0.9, *D), eps_r=e0, sigma=sig, Ms=ms0, alpha=alpha, m0_dir=m0,
                     H0=(2e4, 0.0, 1.2e5), source=(2, prof, 3e12, 1 / 3e12, 1e-12), tol=1e-13, max_iter=50)
    sim.set_fields(E=E, H=H)
    return sim


def _gpu(ckpt, inner):
    import paper_2103_12819_amd as mm
    e0, sig, ms0, alpha, m0, prof, E, H = _materials()
    sim = mm.Sim(N, D, W.cfl_dt(0.9, *D), eps_r=e0, sigma=sig, Ms=ms0, alpha=alpha, m0_dir=m0,
                 H0=(2e4, 0.0, 1.2e5), source=(2, prof, 3e12, 1 / 3e12, 1e-12), tol=1e-13, max_iter=50)
    sim.set_fields(E=E, H=H)
    pid = sim.add_probe(1, 0, I0)
    sim.enable_adjoint(ckpt, inner)
    sim.step(STEPS)
    return sim, pid


@pytest.fixture(scope="module")
def oracle_grads():
    return A.loss_and_gradients(_oracle, STEPS, I0)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("ckpt,inner", [(10, 3), (STEPS, 0)])
def test_multitile_gradient_matches_oracle(oracle_grads, ckpt, inner):
    L, ge_o, gm_o = oracle_grads
    print(f"multi-tile adjoint {N} {STEPS} steps, checkpoints {ckpt}/{inner}", flush=True)
    sim, pid = _gpu(ckpt, inner)
    lay = sim.tiles()
    assert lay["near_tiles"] > 0 and lay["far_tiles"] > 0, lay
    _, Lg = sim.probe(pid)
    ge, gm = sim.adjoint(pid)
    sim.close()
    assert abs(Lg - L) <= 1e-12 * abs(L), (Lg, L)
    assert _rel(ge, ge_o) <= 1e-10, _rel(ge, ge_o)
    assert _rel(gm, gm_o) <= 1e-10, _rel(gm, gm_o)
