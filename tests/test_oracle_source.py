"""Pins of the oracle's soft current source (Sec. 2, Ampere's law with a
source current; Sec. 5.2.1, the pulse), independent of its code.

At Courant number 1 on a line (one cell across, periodic transverse axes)
the Yee equations can be followed by hand.  A soft injection s into E_z at
node x0 (the update adds -(dt/eps0) J there) leaves, one level later, +s at
x0; the next H update turns it into -s, +s on the faces beside it, and so
on: inside its light cone the field of one injection alternates in sign
from level to level, and it moves one cell per step.  Summed over the
injections s_p = -(dt/eps0) A g(t^{p+1/2}) of steps p = 0, 1, ..., the field
at node x0 +- m after step N is therefore

    E_z = a_{N-1-m},   a_p = s_p - a_{p-1},   a_{-1} = 0,

the same on both sides.  For a pulse that varies slowly over a step,
a_{N-1-m} is s / 2 at t^N - m dt to second order in the step: with
dt/eps0 = eta0 dx at Courant number 1 this is the continuum field of a
current sheet, E = -eta0 J_s / 2 with J_s = J dx, radiated equally both ways
and retarded by the travel time.  These fix the time level the source enters at
(t^{n+1/2}), its sign, the factor dt/eps0 and its support.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import Simulation
from oracle.yee_llg import EPS0, MU0, waveform

ETA = math.sqrt(MU0 / EPS0)
NX, X0, AMP = 700, 330, 2.0
DIST = (0, 1, 5, 40, 120)


def _line():
    d = (1e-6, 1e2, 1e2)
    return d, W.cfl_dt(1.0, *d)


def _run(f0, steps, amp=AMP, t_shift=0.0, nx=NX, x0=X0):
    """The oracle's E_z at x0 +- m after every step, for a soft source of
    amplitude `amp` at x0 (a planted mistake may shift the pulse in time)."""
    d, dt = _line()
    tp, t0 = 1 / f0, 3 / f0
    prof = np.zeros(W.edge_shape((nx, 1, 1), (False, True, True), 2))
    prof[0, 0, x0] = amp
    sim = Simulation((nx, 1, 1), d, dt, periodic=(False, True, True), source=(2, prof, f0, tp, t0 + t_shift))
    out = np.zeros((steps, len(DIST), 2))
    for n in range(steps):
        sim.step(1)
        for q, m in enumerate(DIST):
            out[n, q, 0] = sim.E[2][x0 + m, 0, 0]
            out[n, q, 1] = sim.E[2][x0 - m, 0, 0]
    return out, d, dt


def _expected(f0, steps, dt):
    """a_p of the hand derivation, from the pulse alone."""
    tp, t0 = 1 / f0, 3 / f0
    s = np.array([-(dt / EPS0) * AMP * waveform((p + 0.5) * dt, f0, tp, t0) for p in range(steps)])
    a = np.zeros(steps)
    prev = 0.0
    for p in range(steps):
        a[p] = s[p] - prev
        prev = a[p]
    want = np.zeros((steps, len(DIST), 2))
    for n in range(steps):          # after step n + 1
        for q, m in enumerate(DIST):
            p = n - m
            if p >= 0:
                want[n, q, :] = a[p]
    return want, s, a


def _rel_err(got, want):
    return float(np.max(np.abs(got - want)) / np.max(np.abs(want)))


def test_soft_source_field_follows_the_discrete_recursion():
    f0, steps = 15e12, 200
    got, _, dt = _run(f0, steps)
    want, _, _ = _expected(f0, steps, dt)
    assert _rel_err(got, want) < 1e-9


def test_soft_source_radiates_half_the_sheet_field_each_way():
    # a pulse of 100 steps per carrier period, delayed to start at e^{-12.5} of
    # its peak (a pulse switched on abruptly leaves a level-to-level
    # alternation, the undamped Nyquist mode at Courant number 1), on a line
    # long enough that nothing returns inside the window
    f0, steps, nx, x0 = 3e12, 850, 2000, 1000
    d, dt = _line()
    delay = 2 / f0
    got, d, dt = _run(f0, steps, t_shift=delay, nx=nx, x0=x0)
    assert abs(dt / EPS0 - ETA * d[0]) < 1e-12 * ETA * d[0]
    m = DIST.index(40)
    right = got[40:, m, 0]          # E_z at x0 + 40 after steps 41..
    left = got[40:, m, 1]
    # the continuum sheet field at level N = n + 1, 40 cells (40 steps) away:
    # -eta0 J dx / 2 times the pulse at t^N - 40 dt
    sheet = -0.5 * ETA * d[0] * AMP * np.array(
        [waveform((n + 1 - 40) * dt, f0, 1 / f0, 3 / f0 + delay) for n in range(40, steps)])
    assert np.array_equal(right, left)
    # second order in the step: (omega dt)^2 / 8 = 5e-4 here
    assert float(np.max(np.abs(right - sheet)) / np.max(np.abs(sheet))) < 2e-3
    # and the sign: E opposite to J where the pulse peaks
    k = int(np.argmax(np.abs(sheet)))
    assert np.sign(right[k]) == np.sign(sheet[k]) != 0


@pytest.mark.parametrize("plant", ["time level t^n", "sign of J", "factor 2"])
def test_planted_source_mistakes_fail(plant):
    f0, steps = 15e12, 200
    _, dt = _line()
    if plant == "time level t^n":
        got, _, dt = _run(f0, steps, t_shift=0.5 * _line()[1])    # g(t^n) in place of g(t^{n+1/2})
    elif plant == "sign of J":
        got, _, dt = _run(f0, steps, amp=-AMP)
    else:
        got, _, dt = _run(f0, steps, amp=2 * AMP)
    want, _, _ = _expected(f0, steps, dt)
    assert _rel_err(got, want) > 1e-3
