"""Long runs against stored oracle results, FP64 and the FP32 bulk mode.

The oracle takes 25 min (the 128 x 64 x 64 crop of the filter grid, 1000
steps) and about 2 h (the 256 x 64 x 64 waveguide, 2000 steps) for these
runs, so its results are stored in tests/golden/ by make_oracle_runs.py
(which runs the oracle alone): every iteration count, every probe series
and integral as exact hexadecimal floats, and per field (E, H, the nine M
components) the SHA-256 of its FP64 values with a seeded sample of values.

FP64 (the benchmark's launch form: one mm_step call for the whole course):
  * every sub-step's iteration count equals the oracle's,
  * every probe series and integral within 1e-12 (normwise relative; in
    practice the same bits),
  * every field has the oracle's SHA-256: bit for bit at the end.
FP32 bulk mode, same course: since the FP64 run matched the oracle bit for
bit, its fields are the oracle's; the FP32 run's normwise relative L2 error
against them is the error against the oracle, required <= 1e-4 (the stated
FP32 bar) for E, H and M - M0, and for every probe series and integral
(compared with the stored oracle values directly).
"""
import gzip
import hashlib
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from tests import parity_util as PU

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
TOL64, TOL32 = 1e-12, 1e-4
FIELDS = PU.E_H + PU.M_NAMES


def _golden(name):
    path = os.path.join(HERE, "golden", f"{name}_oracle.json.gz")
    if not os.path.exists(path):
        pytest.skip(f"stored oracle run {path} not written yet")
    with gzip.open(path, "rt") as fh:
        return json.load(fh)


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(np.asarray(a, dtype=np.float64) + 0.0).tobytes()).hexdigest()


def _series(gold, pid):
    p = gold["probes"][pid]
    return np.array([float.fromhex(v) for v in p["series"]]), float.fromhex(p["sum"])


def _probe_errs(sim, gold, dt):
    errs = {}
    for pid in range(len(gold["probes"])):
        s_ref, S_ref = _series(gold, pid)
        s, S = sim.probe(pid)
        errs[f"probe{pid}"] = PU.rel_l2(s, s_ref)
        scale = max(abs(S_ref), dt * float(np.sum(np.abs(s_ref))), 1e-300)
        errs[f"sum{pid}"] = abs(S - S_ref) / scale
    return errs


def _run(cfg, precision):
    import paper_2103_12819_amd as mm
    print(f"long run {cfg.name} {cfg.n} {precision} {cfg.steps} steps", flush=True)
    sim = mm.from_config(cfg, precision=precision)
    sim.step(cfg.steps)
    return sim


def _check_fp64(cfg, gold):
    sim = _run(cfg, "fp64")
    assert list(sim.stats()) == gold["iters"]
    errs = _probe_errs(sim, gold, cfg.dt)
    report = {}
    for q, nm in enumerate(FIELDS):
        a = sim.field(nm)
        ref = gold["fields"][nm]
        idx = np.array(ref["sample_idx"])
        samp = np.array([float.fromhex(v) for v in ref["sample"]])
        got = a.reshape(-1)[idx]
        report[nm] = (_digest(a) == ref["sha256"], float(np.max(np.abs(got - samp))),
                      abs(float(np.linalg.norm(a)) - float.fromhex(ref["norm"])) / max(float.fromhex(ref["norm"]), 1e-300))
    print("probes", {k: f"{v:.1e}" for k, v in errs.items()})
    print("fields (same bits, max |diff| on the sample, rel. change of the norm)", report)
    assert all(v <= TOL64 for v in errs.values()), errs
    assert all(r[0] for r in report.values()), report
    return sim


def _check_fp32(cfg, gold, sim64):
    import paper_2103_12819_amd as mm
    sim = _run(cfg, "fp32")
    m0 = mm.from_config(cfg)
    M0 = {n: m0.field(n) for n in PU.M_NAMES}
    m0.close()
    errs = {
        "E": PU.normwise([sim.field(n) for n in ("Ex", "Ey", "Ez")], [sim64.field(n) for n in ("Ex", "Ey", "Ez")]),
        "H": PU.normwise([sim.field(n) for n in ("Hx", "Hy", "Hz")], [sim64.field(n) for n in ("Hx", "Hy", "Hz")]),
        "M-M0": PU.normwise([sim.field(n) - M0[n] for n in PU.M_NAMES],
                            [sim64.field(n) - M0[n] for n in PU.M_NAMES]),
    }
    errs.update(_probe_errs(sim, gold, cfg.dt))
    print("fp32 vs oracle", {k: f"{v:.2e}" for k, v in errs.items()})
    assert all(math.isfinite(v) and v <= TOL32 for v in errs.values()), errs
    assert errs["E"] > 1e-9     # FP32 is really in use
    sim.close()
    return errs


def test_filter_crop_1000_steps_fp64_and_fp32():
    """The 128 x 64 x 64 crop of the filter grid for its full 1000 steps: the
    port pulse crosses the crop and M precesses (iteration counts 3)."""
    gold = _golden("filter_crop")
    cfg = W.filter_crop(seed=0, steps=gold["steps"])
    sim64 = _check_fp64(cfg, gold)
    _check_fp32(cfg, gold, sim64)
    sim64.close()


def test_waveguide256_2000_steps_fp64_and_fp32():
    """The 256 x 64 x 64 waveguide for its full 2000 steps: flux planes at
    x = 32 and x = 224, point probes of E_z, H_y and M."""
    gold = _golden("waveguide256")
    cfg = W.waveguide256(seed=0, steps=gold["steps"])
    sim64 = _check_fp64(cfg, gold)
    _check_fp32(cfg, gold, sim64)
    sim64.close()
