"""The fused Faraday pass of the tiles away from magnetic material.

Within one mm_step call the far tiles take Step 3 of step n and Step 1 of
step n+1 (both with curl E^{n+1}) in one pass, and the probes of level n+1
read those tiles through the half step they have not stored yet.  Each half
step is the same rounded operation as in a separate pass, so splitting a run
into calls of any length must give bit-identical fields and probe series,
and the probes in far tiles must match the oracle like all others.
"""
import numpy as np
import pytest

import workloads as W
from tests import parity_util as PU

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


def _far_probe_config(steps=24):
    """192x16x12 grid, a small magnet near the x = 0 corner (4 near tiles of
    36), lossy dielectric, a mu_r map, and probes of every kind in far tiles."""
    n = (192, 16, 12)
    d = (1e-6, 1.1e-6, 0.9e-6)
    shp = (n[2], n[1], n[0])
    rng = np.random.default_rng(31)
    Ms = np.zeros(shp)
    Ms[2:6, 2:6, 8:24] = 1.5e5
    m0 = np.zeros((3,) + shp)
    m0[0], m0[2] = 0.3, 1.0
    cfg = W.Config("farprobe", n, d, W.cfl_dt(0.9, *d), steps, eps_r=rng.uniform(1, 4, shp),
                   sigma=rng.uniform(0, 1e3, shp), mu_r=rng.uniform(1, 1.5, shp), Ms=Ms,
                   alpha=np.where(Ms > 0, 0.02, 0.0), gamma=np.full(shp, W.GAMMA_E), m0_dir=m0,
                   H0=(0.0, 2e3, 9e4), tol=1e-11)
    PU.with_random_start(cfg, seed=5, amp_e=2e5, amp_h=4e3)
    F = W.FIELD_ID
    cfg.probes = [W.Probe(1, 0, 150), W.Probe(1, 0, 64), W.Probe(0, F["Hz"], 130, 9, 7),
                  W.Probe(0, F["By"], 100, 3, 9), W.Probe(0, F["Hx"], 128, 5, 5),
                  W.Probe(0, F["Hy"], 63, 15, 11), W.Probe(0, F["Bz"], 20, 4, 4),
                  W.Probe(0, F["Ex"], 140, 8, 6)]
    return cfg


def test_tile_split_of_the_far_probe_grid():
    import paper_2103_12819_amd as mm
    cfg = _far_probe_config()
    sim = mm.from_config(cfg)
    t = sim.tiles()
    sim.close()
    assert t["tiles"] == 36 and t["near_tiles"] == 4 and t["far_tiles"] == 32, t
    assert t["near_cells"] + t["far_cells"] == cfg.cells


def test_probes_in_far_tiles_match_the_oracle():
    cfg = _far_probe_config()
    ref, sim, ref0 = PU.run_pair(cfg, cfg.steps)
    PU.compare(ref, sim, ref0, TOL64)


def _run(cfg, chunks, precision):
    import paper_2103_12819_amd as mm
    sim = mm.from_config(cfg, precision=precision)
    for n in chunks:
        sim.step(n)
    out = [sim.field(nm) for nm in PU.E_H + PU.M_NAMES]
    out += [sim.probe(p)[0] for p in range(len(cfg.probes))]
    out.append(sim.stats())
    sim.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("which", ["farprobe", "filter_crop", "ragged_periodic"])
def test_call_boundaries_do_not_change_the_result(which, precision):
    if which == "farprobe":
        cfg = _far_probe_config(steps=20)
    elif which == "filter_crop":
        cfg = W.filter_crop(seed=0, steps=20)
    else:
        n, d = (70, 9, 10), (1e-6, 1.3e-6, 0.9e-6)
        shp = (n[2], n[1], n[0])
        rng = np.random.default_rng(3)
        Ms = np.zeros(shp)
        Ms[1:3, 1:3, 5:9] = 1.2e5
        m0 = np.zeros((3,) + shp)
        m0[2] = 1.0
        cfg = W.Config("ragged", n, d, W.cfl_dt(0.9, *d), 20, periodic=(True, False, True),
                       eps_r=rng.uniform(1, 3, shp), sigma=rng.uniform(0, 1e3, shp),
                       mu_r=rng.uniform(1, 2, shp), Ms=Ms, alpha=np.where(Ms > 0, 0.01, 0.0),
                       gamma=np.full(shp, W.GAMMA_E), m0_dir=m0, H0=(0, 0, 8e4), tol=1e-11)
        PU.with_random_start(cfg, seed=4, amp_e=1e5, amp_h=2e3)
        cfg.probes = [W.Probe(1, 0, 60), W.Probe(0, W.FIELD_ID["Hz"], 66, 8, 9)]
    one = _run(cfg, [20], precision)
    for chunks in ([1] * 20, [3, 1, 9, 7]):
        other = _run(cfg, chunks, precision)
        for a, b in zip(one, other):
            assert np.array_equal(a, b)


def test_material_id_mode_is_chosen_by_the_number_of_materials():
    """Few distinct (eps_r, sigma) pairs: byte ids + table; a smooth random
    eps_r map: the dense maps.  Parity of both paths is covered by the
    filter-crop and ragged-grid tests."""
    import paper_2103_12819_amd as mm
    a = mm.from_config(W.filter_crop(seed=0, steps=1))
    b = mm.from_config(W.design128(seed=0, steps=1, n=(64, 32, 16)))   # 2048 random cells
    try:
        assert 2 <= a.tiles()["materials"] <= 256
        assert b.tiles()["materials"] == 0
    finally:
        a.close()
        b.close()
