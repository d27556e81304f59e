"""Pin of the coupled E-H-M loop of the oracle by the Kittel slab resonance
(Sec. 5.2.2; set-up and expected value in tests/kittel_case.py).

Runs the oracle at three resolutions of the same box (the slab always a
quarter of it) and at two for a half-filled box: the error must fall at
first order (the face-averaged interface) and the first-order Richardson
extrapolation must meet the formula to 2e-4."""
import pytest

from oracle import from_config
from tests import kittel_case as K


def _oracle_frequency(Nx, n):
    cfg, ic = K.config(Nx, n)
    sim = from_config(cfg, with_probes=False)
    ys = []
    for _ in range(cfg.steps):
        sim.step(1)
        ys.append(float(sim.M[2][1][ic, 0, 0]))
    return K.frequency(ys, cfg.dt)


def test_paper_example_value():
    """The SI form of the thin-film formula with the paper's YIG values gives
    the 10.25 GHz the paper states."""
    assert abs(K.kittel_thin_film() - 10.25e9) < 0.01e9


@pytest.mark.parametrize("fill,sizes", [(0.25, (16, 32, 64)), (0.5, (16, 32))])
def test_slab_resonance_converges_to_kittel(fill, sizes):
    fk = K.kittel_slab(fill)
    f = [_oracle_frequency(Nx, int(fill * Nx)) for Nx in sizes]
    err = [(v - fk) / fk for v in f]
    print(fill, err)
    assert all(-2e-2 < e < 0 for e in err)
    for a, b in zip(err, err[1:]):
        assert 1.8 < a / b < 2.2, err
    rich = 2 * f[-1] - f[-2]
    assert abs(rich - fk) / fk < 2e-4, (rich, fk)
