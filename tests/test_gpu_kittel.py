"""The Kittel slab resonance (Sec. 5.2.2; set-up in tests/kittel_case.py) on
the HIP path: the probed M_y series matches the oracle's at a coarse grid,
and at finer grids than the oracle can afford the frequency converges at
first order to the formula, its Richardson extrapolation within 1e-4."""
import numpy as np
import pytest

import workloads as W
from oracle import from_config
from tests import kittel_case as K

pytestmark = pytest.mark.gpu


def _gpu_series(Nx, n):
    import paper_2103_12819_amd as mm
    cfg, ic = K.config(Nx, n)
    cfg.probes = [W.Probe(0, W.FIELD_ID["Mzy"], ic, 0, 0)]
    sim = mm.from_config(cfg)
    sim.step(cfg.steps)
    series, _ = sim.probe(0)
    iters = sim.stats()
    sim.close()
    return cfg, series, iters


def test_kittel_series_matches_the_oracle():
    cfg, ic = K.config(16, 4)
    ref = from_config(cfg, with_probes=False)
    ys = []
    for _ in range(cfg.steps):
        ref.step(1)
        ys.append(float(ref.M[2][1][ic, 0, 0]))
    _, series, iters = _gpu_series(16, 4)
    ys = np.array(ys)
    assert np.linalg.norm(series - ys) <= 1e-12 * np.linalg.norm(ys)
    assert list(iters) == list(ref.iters)


def test_kittel_frequency_converges_on_the_gpu():
    fk = K.kittel_slab(0.25)
    f = []
    for Nx in (64, 128, 256):
        cfg, series, _ = _gpu_series(Nx, Nx // 4)
        f.append(K.frequency(series, cfg.dt))
    err = [(v - fk) / fk for v in f]
    print(err)
    for a, b in zip(err, err[1:]):
        assert 1.8 < a / b < 2.2, err
    rich = 2 * f[-1] - f[-2]
    assert abs(rich - fk) / fk < 1e-4, (rich, fk)
