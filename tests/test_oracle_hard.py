"""Pins of the oracle's hard sources (Sec. 3.2) and surface current (Sec. 5.2.1).

At Courant number 1 on a line (one cell across, periodic transverse axes)
the Yee scheme is exact: a discrete wave moves one cell per step without
dispersion.  Hence a hard source's waveform must arrive unchanged m cells
away m steps later, with the plane-wave ratio |E| = eta0 |H| when the source
holds H.  These identities fix the time level each hard value takes
(t^{n+1} for E after Step 2; t^{n+1/2} and t^{n+1} for H after Steps 1 and
3), the sign and the plane of the surface current, to the 1e-9 level.
The line is long enough that nothing returns from its walls inside the
window.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import Simulation
from oracle.yee_llg import EPS0, MU0, waveform

ETA = math.sqrt(MU0 / EPS0)
F0 = 15e12
TP, T0 = 1 / F0, 3 / F0
STEPS = 200
DIST = (1, 5, 40, 120)


def _line_x(nx):
    d = (1e-6, 1e2, 1e2)
    return d, W.cfl_dt(1.0, *d)


def test_courant_number_is_one():
    d, dt = _line_x(10)
    S = dt / (d[0] * math.sqrt(MU0 * EPS0))
    assert abs(S - 1) < 1e-12


def test_hard_e_source_is_transported_exactly():
    nx, x0, A = 700, 330, 2.0
    d, dt = _line_x(nx)
    prof = np.zeros(W.edge_shape((nx, 1, 1), (False, True, True), 2))
    prof[0, 0, x0] = A
    sim = Simulation((nx, 1, 1), d, dt, periodic=(False, True, True), hard_sources=[(2, prof, F0, TP, T0)])
    err = 0.0
    for n in range(1, STEPS + 1):
        sim.step(1)
        assert sim.E[2][x0, 0, 0] == A * waveform(n * dt, F0, TP, T0)
        for m in DIST:
            want = A * waveform((n - m) * dt, F0, TP, T0) if n > m else 0.0
            err = max(err, abs(sim.E[2][x0 + m, 0, 0] - want), abs(sim.E[2][x0 - m, 0, 0] - want))
    assert err < 1e-9 * A, err


def test_hard_h_source_is_transported_exactly():
    """Hy held on the face of cell x0; E_z at node x0 + m (m - 1/2 cells
    away) carries -eta0 Hy of the right-going wave, +eta0 Hy on the left."""
    nx, x0, A = 700, 330, 3.0
    d, dt = _line_x(nx)
    prof = np.zeros(W.face_shape((nx, 1, 1), (False, True, True), 1))
    prof[0, 0, x0] = A
    sim = Simulation((nx, 1, 1), d, dt, periodic=(False, True, True), hard_sources=[(4, prof, F0, TP, T0)])
    err = 0.0
    for n in range(1, STEPS + 1):
        sim.step(1)
        assert sim.H[1][x0, 0, 0] == A * waveform(n * dt, F0, TP, T0)      # held at t^{n+1}
        for m in DIST:
            g = A * waveform((n - m + 0.5) * dt, F0, TP, T0) if n >= m else 0.0
            err = max(err, abs(sim.E[2][x0 + m, 0, 0] + ETA * g), abs(sim.E[2][x0 + 1 - m, 0, 0] - ETA * g))
    assert err < 1e-9 * ETA * A, err


@pytest.mark.parametrize("side", [0, 1])
def test_surface_current_launches_minus_eta_js(side):
    """J_s along y on a z wall: n x H = J_s with n into the domain gives
    H_x = -J_s at the high wall and +J_s at the low wall, and the wave
    leaving the wall has E_y = -eta0 J_s (delayed by the distance to the
    held faces, half a cell inside the wall)."""
    nz, A = 400, 5.0
    d = (1e2, 1e2, 1e-6)
    dt = W.cfl_dt(1.0, *d)
    J = np.zeros(W.edge_shape((1, 1, nz), (True, True, False), 1))
    wall = nz if side == 1 else 0
    J[wall, 0, 0] = A
    sim = Simulation((1, 1, nz), d, dt, periodic=(True, True, False))
    sim.add_surface_current(2, side, 1, J, F0, TP, T0)
    held = nz - 1 if side == 1 else 0
    err = 0.0
    for n in range(1, STEPS + 1):
        sim.step(1)
        assert sim.H[0][0, 0, held] == (-A if side == 1 else A) * waveform(n * dt, F0, TP, T0)
        for m in DIST:
            g = A * waveform((n - m + 0.5) * dt, F0, TP, T0) if n >= m else 0.0
            k = nz - m if side == 1 else m
            err = max(err, abs(sim.E[1][0, 0, k] + ETA * g))
    assert err < 1e-9 * ETA * A, err


def test_support_is_the_bounding_box_of_the_profile():
    """Entries inside the box with a zero profile are held at zero; entries
    outside it evolve; PEC-pinned entries stay zero."""
    n = (12, 10, 8)
    d = (1e-6, 1e-6, 1e-6)
    dt = W.cfl_dt(0.9, *d)
    prof = np.zeros(W.edge_shape(n, (False,) * 3, 1))    # Ey: (9, 10, 13) host layout
    prof[3, 2, 4] = 1.0
    prof[5, 6, 7] = -2.0                                   # box z 3..5, y 2..6, x 4..7
    soft = np.zeros(W.edge_shape(n, (False,) * 3, 2))
    soft[2, 5, 2] = 1e12
    sim = Simulation(n, d, dt, source=(2, soft, F0, TP, T0), hard_sources=[(1, prof, F0, TP, T0)])
    sim.step(15)
    Ey = sim.field("Ey")
    g = waveform(15 * dt, F0, TP, T0)
    assert Ey[3, 2, 4] == g and Ey[5, 6, 7] == -2.0 * g
    assert np.all(Ey[3:6, 2:7, 4:8][prof[3:6, 2:7, 4:8] == 0] == 0)
    outside = np.ones_like(Ey, dtype=bool)
    outside[3:6, 2:7, 4:8] = False
    assert np.count_nonzero(Ey[outside]) > 100


def test_rejections():
    n = (16, 8, 8)
    d = (1e-6, 1e-6, 1e-6)
    dt = W.cfl_dt(0.9, *d)
    shp = (n[2], n[1], n[0])
    Ms = np.zeros(shp)
    Ms[3:5, 3:5, 6:10] = 1e5
    hx = np.zeros(W.face_shape(n, (False,) * 3, 0))
    hx[4, 4, 8] = 1.0                                     # an evolving magnetic x face
    with pytest.raises(ValueError):
        Simulation(n, d, dt, Ms=Ms, hard_sources=[(3, hx, F0, TP, T0)])
    ez = np.zeros(W.edge_shape(n, (False,) * 3, 2))
    ez[3, 4, 2] = 1.0                                     # node x = 2 inside a 3-cell x layer
    with pytest.raises(ValueError):
        Simulation(n, d, dt, pml=((3, 0, 0, 0, 0, 0), 1e-6, 3), hard_sources=[(2, ez, F0, TP, T0)])
    ez[3, 4, 2] = 0.0
    ez[3, 4, 3] = 1.0                                     # node x = 3: the layer's inner face
    Simulation(n, d, dt, pml=((3, 0, 0, 0, 0, 0), 1e-6, 3), hard_sources=[(2, ez, F0, TP, T0)])
    with pytest.raises(ValueError):
        Simulation(n, d, dt, hard_sources=[(2, np.zeros_like(ez), F0, TP, T0)])
