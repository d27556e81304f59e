"""FP32 bulk mode against the FP64 oracle.

E, H and the cell maps are stored and updated in FP32; M, the LLG solve, the
sub-step residual and the probe accumulators stay FP64.  The stated bar is a
normwise relative L2 error <= 1e-4 for E, H, M - M0 and every probe series
and integral (FP32 rounding is ~6e-8 per operation; the bar leaves room for
its growth over a few hundred steps).  Iteration counts may differ from the
FP64 reference by rounding near the tolerance, so they are not compared.
"""
import pytest

import workloads as W
from tests import parity_util as PU

pytestmark = pytest.mark.gpu
TOL32 = 1e-4


def _check(cfg, steps):
    ref, sim, ref0 = PU.run_pair(cfg, steps, precision="fp32")
    errs, info = PU.compare(ref, sim, ref0, TOL32, check_iters=False, dev_tol=TOL32)
    print(cfg.name, {k: f"{v:.2e}" for k, v in errs.items()})
    return errs


def test_fp32_slab64_random_start():
    cfg = PU.with_random_start(W.slab64(steps=100), seed=4, amp_e=1e6, amp_h=2e4)
    errs = _check(cfg, cfg.steps)
    # FP32 is really in use: the error is far above FP64 round-off
    assert errs["E"] > 1e-10


def test_fp32_waveguide_shrunk():
    cfg = W.waveguide256(seed=1, steps=150, n=(96, 24, 16))
    _check(cfg, cfg.steps)


def test_fp32_filter_crop():
    cfg = W.filter_crop(seed=0, steps=20)
    _check(cfg, cfg.steps)
