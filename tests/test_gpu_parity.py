"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bar (FP64): normwise relative L2 <= 1e-12 for E, H, M (nine components) and
normal B, and for every probe series and probe integral; the deviation
M - M0 within the same bar or, when M barely moves, within ~1000 ulps of |M|;
equal iteration counts for every sub-step.
"""
import numpy as np
import pytest

import workloads as W
from tests import parity_util as PU

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


def _mm():
    import paper_2103_12819_amd as mm
    return mm


def test_slab64_full_run_fp64():
    """The 64x16x16 slab configuration, all 200 steps."""
    cfg = W.slab64(steps=200)
    ref, sim, ref0 = PU.run_pair(cfg, cfg.steps)
    errs, info = PU.compare(ref, sim, ref0, TOL64)
    print("slab64", errs, info)


def test_slab64_random_start_exercises_iterations():
    cfg = PU.with_random_start(W.slab64(steps=30), seed=4, amp_e=1e6, amp_h=2e4)
    ref, sim, ref0 = PU.run_pair(cfg, cfg.steps)
    PU.compare(ref, sim, ref0, TOL64)
    assert max(ref.iters) >= 3


@pytest.mark.parametrize("per", [(True, True, True), (True, False, True), (False, True, False)])
def test_periodic_axes_ragged_grid(per):
    """Grid sizes that are not multiples of the 64 x 4 tile, with some axes
    periodic; magnets, conductivity and mu_r all present."""
    n = (70, 7, 5)
    d = (1e-6, 1.3e-6, 0.9e-6)
    shp = (n[2], n[1], n[0])
    rng = np.random.default_rng(8)
    Ms = np.zeros(shp)
    Ms[1:4, 2:6, 20:50] = 1.4e5
    m0 = np.zeros((3,) + shp)
    m0[0], m0[2] = 0.2, 1.0
    cfg = W.Config("ragged", n, d, W.cfl_dt(0.9, *d), 15, periodic=per,
                   eps_r=rng.uniform(1, 5, shp), sigma=rng.uniform(0, 2e3, shp),
                   mu_r=rng.uniform(1, 2, shp), Ms=Ms, alpha=rng.uniform(0.001, 0.05, shp),
                   gamma=np.full(shp, W.GAMMA_E), m0_dir=m0, H0=(1e4, -5e3, 8e4), tol=1e-11)
    PU.with_random_start(cfg, seed=2, amp_e=1e5, amp_h=3e3)
    cfg.probes = [W.Probe(1, 0, 35), W.Probe(0, W.FIELD_ID["Myx"], 30, 3, 2),
                  W.Probe(0, W.FIELD_ID["By"], 30, 3, 2), W.Probe(0, W.FIELD_ID["Bx"], 5, 1, 1)]
    ref, sim, ref0 = PU.run_pair(cfg, cfg.steps)
    PU.compare(ref, sim, ref0, TOL64)


def test_waveguide_shrunk_with_port_source():
    cfg = W.waveguide256(seed=1, steps=120, n=(96, 24, 16))
    ref, sim, ref0 = PU.run_pair(cfg, cfg.steps)
    PU.compare(ref, sim, ref0, TOL64)


def test_filter_crop_short_run():
    """The 128x64x64 crop (lossy dielectric boxes, ferrite bar on the floor)
    for 40 steps: several tiles in every direction."""
    cfg = W.filter_crop(seed=0, steps=40)
    ref, sim, ref0 = PU.run_pair(cfg, cfg.steps)
    PU.compare(ref, sim, ref0, TOL64)


def test_iterations_beyond_the_enqueued_launches():
    """A tight tolerance needs more iterations than the launches enqueued from
    the recent history, so hm_finish completes them (its barrier path)."""
    cfg = PU.with_random_start(W.slab64(steps=6), seed=12, amp_e=3e6, amp_h=5e4)
    cfg.tol = 1e-15
    ref, sim, ref0 = PU.run_pair(cfg, cfg.steps)
    PU.compare(ref, sim, ref0, TOL64)
    assert max(ref.iters) >= 4


def test_fixed_iteration_mode_matches():
    cfg = PU.with_random_start(W.slab64(steps=10), seed=6, amp_e=1e6, amp_h=2e4)
    ref, sim, ref0 = PU.run_pair(cfg, cfg.steps, fixed_iter=2)
    PU.compare(ref, sim, ref0, TOL64)
    assert set(sim.stats().tolist()) == {2}


def test_degenerate_grids():
    """One-cell axes, a fully magnetic box and a box without magnets."""
    mm = _mm()
    for n, per, ms in [((1, 1, 1), (False,) * 3, 1e5), ((3, 1, 2), (True, True, False), 1e5),
                       ((6, 5, 4), (False,) * 3, 0.0), ((4, 4, 4), (True,) * 3, 1.2e5)]:
        d = (1e-6,) * 3
        shp = (n[2], n[1], n[0])
        m0 = np.zeros((3,) + shp)
        m0[1], m0[2] = 0.5, 1.0
        cfg = W.Config("deg", n, d, W.cfl_dt(0.9, *d), 6, periodic=per, Ms=np.full(shp, ms),
                       alpha=np.full(shp, 0.01), m0_dir=m0, H0=(0, 0, 1e5), tol=1e-12)
        PU.with_random_start(cfg, seed=1, amp_e=1e4, amp_h=1e3)
        ref, sim, ref0 = PU.run_pair(cfg, cfg.steps)
        PU.compare(ref, sim, ref0, TOL64, probes=False)
        sim.close()


def test_gauss_law_for_B_holds_at_full_waveguide_size():
    """Full 256x64x64 waveguide, 200 steps: the per-cell flux of B is
    unchanged (a property that holds at any size), |M| = Ms on every face."""
    mm = _mm()
    cfg = W.waveguide256(seed=0, steps=200)
    PU.with_random_start(cfg, seed=3, amp_e=1e4, amp_h=1e2)
    sim = mm.from_config(cfg)

    def divB():
        B = [sim.field(nm) for nm in ("Bx", "By", "Bz")]      # host layout [k][j][i]
        d = cfg.d
        return ((B[0][:, :, 1:] - B[0][:, :, :-1]) / d[0] + (B[1][:, 1:, :] - B[1][:, :-1, :]) / d[1]
                + (B[2][1:, :, :] - B[2][:-1, :, :]) / d[2]), max(float(np.max(np.abs(b))) for b in B)

    d0, bmax = divB()
    sim.step(cfg.steps)
    d1, _ = divB()
    assert np.max(np.abs(d1 - d0)) < 1e-11 * bmax / cfg.d[0]
    Ms_face = 1.4e5
    for f in "xyz":
        m = [sim.field("M" + f + c) for c in "xyz"]
        nrm = np.sqrt(m[0] ** 2 + m[1] ** 2 + m[2] ** 2)
        mag = nrm > 0
        vals = nrm[mag]
        # interface faces carry Ms/2, interior faces Ms
        ok = np.minimum(np.abs(vals - Ms_face), np.abs(vals - Ms_face / 2)) < 1e-9 * Ms_face
        assert ok.all()


def test_nonconvergence_is_reported_and_stepping_continues():
    mm = _mm()
    cfg = PU.with_random_start(W.slab64(steps=3), seed=2, amp_e=1e6, amp_h=2e4)
    cfg.tol = 1e-30
    cfg.max_iter = 2
    sim = mm.from_config(cfg)
    sim.step(3)
    with pytest.raises(mm.MMError) as ei:
        sim.sync()
    assert ei.value.status == -4
    sim.sync()          # the sticky word was cleared
    assert list(sim.stats()) == [2] * 6


def test_nonfinite_field_is_reported():
    mm = _mm()
    cfg = W.slab64(steps=2)
    sim = mm.from_config(cfg)
    ex = sim.field("Hx")
    ex[8, 8, 32] = np.nan
    sim.set_field("Hx", ex)
    sim.step(2)
    with pytest.raises(mm.MMError) as ei:
        sim.sync()
    assert ei.value.status == -5


def test_two_runs_are_bitwise_identical():
    mm = _mm()
    cfg = PU.with_random_start(W.slab64(steps=25), seed=9, amp_e=1e6, amp_h=1e4)
    outs = []
    for _ in range(2):
        sim = mm.from_config(cfg)
        sim.step(cfg.steps)
        outs.append([sim.field(nm) for nm in PU.E_H + PU.M_NAMES] + [sim.probe(0)[0]])
        sim.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
