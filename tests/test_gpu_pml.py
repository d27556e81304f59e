"""The open boundary (split-field PML, Sec. 3.2.3) on the HIP path.

* Parity with the oracle (FP64 at the 1e-12 bar, FP32 at 1e-4) on a grid
  with layers on five faces, a dielectric / mu_r map, a soft source, a small
  magnet away from the layers (near, far and layer tiles together) and
  probes, from a random start.
* Splitting the run into calls of any length gives the same bits (the layer
  tiles take every half step; the far tiles keep their fused pass).
* The normal-incidence reflection bar of the oracle pin, on the GPU.
"""
import numpy as np
import pytest

import workloads as W
from tests import parity_util as PU
from tests import test_oracle_pml as OP

pytestmark = pytest.mark.gpu


def _cfg(steps=30):
    n = (140, 20, 24)
    d = (1e-6, 1.2e-6, 0.9e-6)
    shp = (n[2], n[1], n[0])
    rng = np.random.default_rng(17)
    Ms = np.zeros(shp)
    Ms[9:14, 7:12, 60:76] = 1.3e5
    m0 = np.zeros((3,) + shp)
    m0[0], m0[2] = 0.2, 1.0
    prof = np.zeros(W.edge_shape(n, (False,) * 3, 1))
    prof[10, 2:18, 20] = 1e11
    cfg = W.Config("pmlbox", n, d, W.cfl_dt(0.9, *d), steps, eps_r=rng.uniform(1, 3, shp),
                   mu_r=np.where(Ms > 0, 1.0, rng.uniform(1, 1.5, shp)), Ms=Ms,
                   alpha=np.where(Ms > 0, 0.02, 0.0), gamma=np.full(shp, W.GAMMA_E), m0_dir=m0,
                   H0=(0, 0, 8e4), tol=1e-11)
    cfg.source = W.Source(1, prof, 20e12, 1 / 20e12, 1e-13)
    cfg.pml = ((8, 10, 0, 4, 5, 5), 1e-6, 3)
    PU.with_random_start(cfg, seed=3, amp_e=1e5, amp_h=3e2)
    F = W.FIELD_ID
    cfg.probes = [W.Probe(1, 0, 30), W.Probe(1, 0, 134), W.Probe(0, F["Ey"], 133, 10, 12),
                  W.Probe(0, F["Hz"], 3, 5, 20), W.Probe(0, F["Bz"], 70, 9, 11)]
    return cfg


def test_layout_has_layer_tiles():
    import paper_2103_12819_amd as mm
    sim = mm.from_config(_cfg())
    t = sim.tiles()
    sim.close()
    assert t["pml_tiles"] > 0 and t["near_tiles"] > 0 and t["far_tiles"] > 0, t


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-4)])
def test_parity_with_layers(precision, tol):
    cfg = _cfg()
    ref, sim, ref0 = PU.run_pair(cfg, cfg.steps, precision=precision)
    PU.compare(ref, sim, ref0, tol, check_iters=precision == "fp64", dev_tol=None if precision == "fp64" else tol)


def test_call_boundaries_with_layers():
    import paper_2103_12819_amd as mm
    outs = []
    for chunks in ([24], [1] * 24, [5, 11, 8]):
        cfg = _cfg(steps=24)
        sim = mm.from_config(cfg)
        for c in chunks:
            sim.step(c)
        outs.append([sim.field(nm) for nm in PU.E_H] + [sim.probe(p)[0] for p in range(len(cfg.probes))])
        sim.close()
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert np.array_equal(a, b)


def _gpu_line(nx, pml, steps, xs=40, xp=150):
    import paper_2103_12819_amd as mm
    d = (1e-6, 1e-4, 1e-4)
    dt = W.cfl_dt(0.9, *d)
    prof = np.zeros(W.edge_shape((nx, 1, 1), (False, True, True), 2))
    prof[0, 0, xs] = 1e12
    f0 = 15e12
    sim = mm.Sim((nx, 1, 1), d, dt, source=(2, prof, f0, 1 / f0, 3 / f0), periodic=(False, True, True),
                 pml=((0, OP.PML[0], 0, 0, 0, 0), OP.PML[1], OP.PML[2]) if pml else None)
    pid = sim.add_probe(0, W.FIELD_ID["Ez"], xp, 0, 0)
    sim.step(steps)
    s, _ = sim.probe(pid)
    sim.close()
    return s


def test_normal_incidence_reflection_on_the_gpu():
    a = _gpu_line(200, True, 420)
    ref = _gpu_line(900, False, 420)
    bare = _gpu_line(200, False, 420)
    r = np.max(np.abs(a - ref)) / np.max(np.abs(bare - ref))
    assert r < 1e-3, r
