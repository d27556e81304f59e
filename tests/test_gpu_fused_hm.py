"""The fused H-M sub-step (hm_fused + hm_more) against the FP64 oracle and
against the per-iteration launches, on grids small enough for the oracle.

`fused=1` forces the fused form on grids where the automatic choice would
take the per-iteration launches (it is automatic from 2^18 magnetic faces).
Every case checks:
  * parity with the oracle at the FP64 bar of the HIP path (normwise 1e-12
    for E, H, the nine M components, normal B, every probe series and
    integral; equal iteration counts), and
  * bitwise equality with the same run on the per-iteration launches
    (fused=-1): fields, probes, iteration counts;
  * that the fused kernels really ran (launch counts of the profile classes:
    no hm_finish / hm_commit launch, one hm_fused per sub-step).
Cases: iteration counts of 1, 2-3 and above 3 (the recompute path of
hm_more), fixed counts 1-3, periodic and PEC axes on ragged grids with
conductivity and mu_r, a port source with flux probes across several calls
(near tiles held in the second buffer while far tiles lag), FP32, degenerate
grids, non-convergence and non-finite reporting, the adjoint.
"""
import numpy as np
import pytest

import workloads as W
from tests import parity_util as PU

pytestmark = pytest.mark.gpu
TOL64 = 1e-12
NAMES = PU.E_H + PU.M_NAMES


def _mm():
    import paper_2103_12819_amd as mm
    return mm


def _run(cfg, steps, precision="fp64", fixed_iter=0, fused=1, calls=None, profile=False):
    mm = _mm()
    sim = mm.from_config(cfg, precision=precision, fixed_iter=fixed_iter, fused=fused)
    if profile:
        sim.profile(True)
    for n in (calls or [steps]):
        sim.step(n)
    prof = sim.profile_read() if profile else None
    return sim, prof


def _same(a, b, nprobes):
    for nm in NAMES:
        x, y = a.field(nm), b.field(nm)
        assert np.array_equal(x, y), (nm, float(np.max(np.abs(x - y))))
    assert list(a.stats()) == list(b.stats())
    for pid in range(nprobes):
        s1, S1 = a.probe(pid)
        s0, S0 = b.probe(pid)
        assert np.array_equal(s1, s0) and S1 == S0, pid


def _check(cfg, steps=None, fixed_iter=0, calls=None, precision="fp64", oracle=True):
    steps = cfg.steps if steps is None else steps
    print(f"fused case {cfg.name} {cfg.n} {precision} fixed={fixed_iter} calls={calls}", flush=True)
    fz, prof = _run(cfg, steps, precision, fixed_iter, 1, calls, profile=True)
    lg, _ = _run(cfg, steps, precision, fixed_iter, -1, calls)
    subs = 2 * steps
    assert prof["hm_pre"][1] == subs, prof          # hm_fused, once per sub-step
    assert prof["hm_step"][1] == subs, prof         # hm_more
    assert prof["hm_finish"][1] == 0 and prof["hm_commit"][1] == 0, prof
    _same(fz, lg, len(cfg.probes))
    if oracle:
        from oracle import from_config as oracle_from_config
        ref = oracle_from_config(cfg, fixed_iter=fixed_iter)
        ref0 = oracle_from_config(cfg, fixed_iter=fixed_iter, with_probes=False)
        ref.step(steps)
        PU.compare(ref, fz, ref0, TOL64)
    it = fz.stats()
    fz.close()
    lg.close()
    return it


def test_slab64_full_run():
    it = _check(W.slab64(steps=200))
    assert set(it.tolist()) <= {1, 2, 3}


def test_random_start_first_count_mispredicted():
    """The first sub-step predicts 1 iteration and needs 3: hm_more's
    recompute path; the later ones are done by hm_fused alone."""
    cfg = PU.with_random_start(W.slab64(steps=30), seed=4, amp_e=1e6, amp_h=2e4)
    it = _check(cfg)
    assert it[0] >= 2 and max(it) >= 3


def test_tight_tolerance_recompute_path():
    cfg = PU.with_random_start(W.slab64(steps=6), seed=12, amp_e=3e6, amp_h=5e4)
    cfg.tol = 1e-15
    it = _check(cfg)
    assert max(it) >= 4


@pytest.mark.parametrize("k", [1, 2, 3])
def test_fixed_counts(k):
    cfg = PU.with_random_start(W.slab64(steps=10), seed=6, amp_e=1e6, amp_h=2e4)
    it = _check(cfg, fixed_iter=k)
    assert set(it.tolist()) == {k}


@pytest.mark.parametrize("per", [(True, True, True), (True, False, True), (False, True, False)])
def test_ragged_grids_periodic_and_pec(per):
    n = (70, 7, 5)
    d = (1e-6, 1.3e-6, 0.9e-6)
    shp = (n[2], n[1], n[0])
    rng = np.random.default_rng(8)
    Ms = np.zeros(shp)
    Ms[1:4, 2:6, 20:50] = 1.4e5
    Ms[0:2, 0:3, 60:70] = 1.1e5           # reaches the x end (wraps when periodic)
    m0 = np.zeros((3,) + shp)
    m0[0], m0[2] = 0.2, 1.0
    cfg = W.Config("ragged", n, d, W.cfl_dt(0.9, *d), 15, periodic=per,
                   eps_r=rng.uniform(1, 5, shp), sigma=rng.uniform(0, 2e3, shp),
                   mu_r=rng.uniform(1, 2, shp), Ms=Ms, alpha=rng.uniform(0.001, 0.05, shp),
                   gamma=np.full(shp, W.GAMMA_E), m0_dir=m0, H0=(1e4, -5e3, 8e4), tol=1e-11)
    PU.with_random_start(cfg, seed=2, amp_e=1e5, amp_h=3e3)
    cfg.probes = [W.Probe(1, 0, 35), W.Probe(0, W.FIELD_ID["Myx"], 30, 3, 2),
                  W.Probe(0, W.FIELD_ID["By"], 30, 3, 2), W.Probe(0, W.FIELD_ID["Bx"], 5, 1, 1)]
    _check(cfg)


def test_waveguide_port_across_calls():
    cfg = W.waveguide256(seed=1, steps=120, n=(96, 24, 16))
    _check(cfg, calls=[1, 37, 2, 80])
    # one call against several: the run boundaries do not change a bit
    a, _ = _run(cfg, 120, fused=1)
    b, _ = _run(cfg, 120, fused=1, calls=[1, 37, 2, 80])
    _same(a, b, len(cfg.probes))


def test_filter_crop_short_run():
    _check(W.filter_crop(seed=0, steps=40))


def test_fp32_matches_the_per_iteration_launches_bitwise():
    cfg = PU.with_random_start(W.slab64(steps=25), seed=7, amp_e=1e6, amp_h=2e4)
    _check(cfg, precision="fp32", oracle=False)
    cfg = W.waveguide256(seed=1, steps=60, n=(96, 24, 16))
    _check(cfg, precision="fp32", oracle=False, calls=[30, 30])


def test_degenerate_grids():
    for n, per, ms in [((1, 1, 1), (False,) * 3, 1e5), ((3, 1, 2), (True, True, False), 1e5),
                       ((4, 4, 4), (True,) * 3, 1.2e5), ((2, 9, 3), (False, True, True), 1e5)]:
        d = (1e-6,) * 3
        shp = (n[2], n[1], n[0])
        m0 = np.zeros((3,) + shp)
        m0[1], m0[2] = 0.5, 1.0
        cfg = W.Config("deg", n, d, W.cfl_dt(0.9, *d), 6, periodic=per, Ms=np.full(shp, ms),
                       alpha=np.full(shp, 0.01), m0_dir=m0, H0=(0, 0, 1e5), tol=1e-12)
        PU.with_random_start(cfg, seed=1, amp_e=1e4, amp_h=1e3)
        mm = _mm()
        if mm.from_config(cfg, fused=1).info()["n_mag"] == 0:
            continue
        _check(cfg)


def test_nonconvergence_and_nonfinite_are_reported():
    mm = _mm()
    cfg = PU.with_random_start(W.slab64(steps=3), seed=2, amp_e=1e6, amp_h=2e4)
    cfg.tol = 1e-30
    cfg.max_iter = 2
    sim = mm.from_config(cfg, fused=1)
    sim.step(3)
    with pytest.raises(mm.MMError) as ei:
        sim.sync()
    assert ei.value.status == -4
    sim.sync()
    assert list(sim.stats()) == [2] * 6
    cfg = W.slab64(steps=2)
    sim = mm.from_config(cfg, fused=1)
    hx = sim.field("Hx")
    hx[8, 8, 32] = np.nan
    sim.set_field("Hx", hx)
    sim.step(2)
    with pytest.raises(mm.MMError) as ei:
        sim.sync()
    assert ei.value.status == -5


@pytest.mark.parametrize("inner", [0, 3])
def test_adjoint_with_a_fused_forward_run(inner):
    """The adjoint recomputes the steps it reverses with the per-iteration
    launches (they log every iterate); with two-level checkpoints its first
    recompute, which only lays down the inner checkpoints, runs the chained
    forward form, fused here.  Either way the gradients are the same bits."""
    mm = _mm()
    cfg = W.design128(seed=0, steps=30, n=(32, 16, 8))
    out = []
    for fz in (1, -1):
        sim = mm.from_config(cfg, fused=fz)
        sim.enable_adjoint(10, inner)
        sim.step(cfg.steps)
        out.append(sim.adjoint(0))
        sim.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_noalloc_entry_point_with_the_fused_form():
    mm = _mm()
    cfg = PU.with_random_start(W.slab64(steps=20), seed=3, amp_e=1e6, amp_h=2e4)
    a = mm.from_config(cfg, fused=1)
    a.step(20)
    b = mm.from_config(cfg, fused=1)
    b.step(4)
    assert b._lib.mm_step_noalloc(b._ctx, 16) == 0
    _same(a, b, len(cfg.probes))
