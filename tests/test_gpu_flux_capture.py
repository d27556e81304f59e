"""The flux-plane capture: inside one mm_step call the far tiles' fused pass
stores E and H at level n+1 on the flux planes, and the flux probe then reads
that capture for far tiles and the fields for near tiles (Sec. 5.2: the
Poynting flux through a plane of nodes).

Grid: the waveguide shrunk to 192 x 16 x 12 with its ferrite slab
(x in [48, 144), y in [0, 4)) and a random start, so every plane carries
flux at once.  Planes at x = 64 (node column in the second 64-wide tile
column, its x - 1 faces in the first; near tiles on the slab's rows, far
tiles above them) and x = 150 (in the third tile column).

Each case checks
  * that the capture ran or not as the plane set allows (one flux launch
    after the far tiles' pass in every step that lags, counted in the
    profile class of the probes),
  * bitwise equality with the same run taken one step per call (no step
    lags, so no capture and no reconstructed half step), fields, probes and
    iteration counts, and
  * parity with the oracle at the FP64 bar (normwise 1e-12).
With three planes two share a tile column, so the capture is off and the
probe reconstructs the far tiles' half step itself.
"""
import numpy as np
import pytest

import workloads as W
from tests import parity_util as PU

pytestmark = pytest.mark.gpu
TOL64 = 1e-12
STEPS = 40


def _cfg(planes):
    cfg = W.waveguide256(seed=1, steps=STEPS, n=(192, 16, 12))
    PU.with_random_start(cfg, seed=4, amp_e=1e5, amp_h=3e2)
    cfg.probes = [W.Probe(1, 0, x) for x in planes] + [W.Probe(0, W.FIELD_ID["Hy"], 70, 10, 6)]
    return cfg


def _run(cfg, precision, calls, fused):
    import paper_2103_12819_amd as mm
    sim = mm.from_config(cfg, precision=precision, fused=fused)
    sim.profile(True)
    for n in calls:
        sim.step(n)
    return sim, sim.profile_read()


def _same(a, b, nprobes):
    for nm in PU.E_H + PU.M_NAMES:
        x, y = a.field(nm), b.field(nm)
        assert np.array_equal(x, y), (nm, float(np.max(np.abs(x - y))))
    assert list(a.stats()) == list(b.stats())
    for pid in range(nprobes):
        s1, S1 = a.probe(pid)
        s0, S0 = b.probe(pid)
        assert np.array_equal(s1, s0) and S1 == S0, pid


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("fused", [1, -1])
@pytest.mark.parametrize("planes,captured", [((64, 150), True), ((64, 100, 150), False)])
def test_flux_capture_matches_unlagged_steps(planes, captured, fused, precision):
    cfg = _cfg(planes)
    print(f"flux capture case planes={planes} fused={fused} {precision}", flush=True)
    one, prof = _run(cfg, precision, [STEPS], fused)
    # probe launches: one per step, plus one per lagging step when captured
    expect = STEPS + (STEPS - 1 if captured else 0)
    assert prof["probes"][1] == expect, prof["probes"]
    per, _ = _run(cfg, precision, [1] * STEPS, fused)
    _same(one, per, len(cfg.probes))
    s, _ = one.probe(0)
    assert np.max(np.abs(s)) > 0
    if precision == "fp64" and fused == 1:
        from oracle import from_config as oracle_from_config
        ref = oracle_from_config(cfg)
        ref0 = oracle_from_config(cfg, with_probes=False)
        ref.step(STEPS)
        PU.compare(ref, one, ref0, TOL64)
    one.close()
    per.close()
