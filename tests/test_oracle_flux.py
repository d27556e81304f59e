"""Pin of the oracle's Poynting-flux probe against a closed form.

On a line along x (one periodic cell across y and z) at Courant number 1
the Yee leapfrog transports a discrete wave exactly: with a right-going
E^n_i = F(i - n), the leapfrog half-level field is H^{n+1/2}_{i+1/2} =
+-F(i - n)/eta0, and H at the integer level n (the mean of its two
neighbouring half levels, since each half step of Sec. 3.2.2 applies half
the Faraday increment) is

    E_z wave:  H_y^n_{i+1/2} = -(E_i + E_{i+1}) / (2 eta0),
    E_y wave:  H_z^n_{i+1/2} = +(E_i + E_{i+1}) / (2 eta0),

with both signs reversed for a left-going wave E^n_i = F(i + n).  The flux
through the node plane x = i0, with H averaged from the two cells beside
the plane, is therefore fixed by the analytic profile alone:

    P^n = s dy dz / (4 eta0) sum_pol E_i0 (E_{i0-1} + 2 E_i0 + E_{i0+1}),

s = +1 (right-going) or -1 (left-going), every E evaluated from F.  The
test starts the oracle from these fields at n = 0 and compares its probe
series and its time integral with this expression; three mistakes planted
in subclasses of the oracle (the sign of the E_z H_y term, H averaged from
the wrong side of the plane, the wrong face area) must fail it.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import Simulation
from oracle.yee_llg import EPS0, MU0

ETA = math.sqrt(MU0 / EPS0)
NX, I0, STEPS = 400, 230, 150
D = (1e-6, 3e-6, 5e-6)
PER = (False, True, True)


def _profiles():
    """Two smooth, oscillating pulses (one per polarisation), as functions of
    the (possibly fractional) node position."""
    Fz = lambda x: 7e4 * np.exp(-((x - 150.0) / 14.0) ** 2) * np.cos(0.31 * x)
    Fy = lambda x: -4e4 * np.exp(-((x - 165.0) / 9.0) ** 2) * np.cos(0.47 * x + 0.3)
    return Fy, Fz


def _setup(sim_cls, direction):
    """A simulation on the x line holding a travelling wave of both
    polarisations at level 0 (direction +1: right-going, -1: left-going)."""
    n = (NX, 1, 1)
    # dy, dz do not enter the transport (no variation across), but Courant
    # number 1 along x needs the transverse terms of the CFL sum gone: take
    # the step from dx alone.
    dt = D[0] * math.sqrt(MU0 * EPS0)
    sim = sim_cls(n, D, dt, periodic=PER)
    Fy, Fz = _profiles()
    x = np.arange(NX + 1, dtype=float)
    xs = x if direction > 0 else x[::-1]           # left-going: mirror the pulse
    Ey_n, Ez_n = Fy(xs), Fz(xs)
    E = [np.zeros(W.edge_shape(n, PER, c)) for c in range(3)]
    H = [np.zeros(W.face_shape(n, PER, f)) for f in range(3)]
    E[1][0, 0, :] = Ey_n
    E[2][0, 0, :] = Ez_n
    s = float(direction)
    H[1][0, 0, :] = -s * (Ez_n[:-1] + Ez_n[1:]) / (2 * ETA)
    H[2][0, 0, :] = s * (Ey_n[:-1] + Ey_n[1:]) / (2 * ETA)
    sim.set_fields(E, H)
    pid = sim.add_probe(1, i=I0)
    return sim, pid, dt, (Ey_n, Ez_n)


def _closed_form(direction, dt):
    """P^n for n = 1..STEPS and S = sum_n dt P^n from the analytic profiles."""
    Fy, Fz = _profiles()
    s = float(direction)
    P = []
    for n in range(1, STEPS + 1):
        tot = 0.0
        for F in (Fy, Fz):
            if direction > 0:
                e = lambda i: F(i - n)
            else:
                e = lambda i: F((NX - i) - n)         # mirrored pulse moving left
            tot += e(I0) * (e(I0 - 1) + 2.0 * e(I0) + e(I0 + 1))
        P.append(s * D[1] * D[2] * tot / (4.0 * ETA))
    P = np.array(P)
    S = 0.0
    for v in P:
        S += dt * v
    return P, S


def _pin_error(sim_cls, direction):
    sim, pid, dt, _ = _setup(sim_cls, direction)
    sim.step(STEPS)
    P, S = _closed_form(direction, dt)
    got = sim.probe_series(pid)
    scale = float(np.max(np.abs(P)))
    return float(np.max(np.abs(got - P))) / scale, abs(sim.probe_integral(pid) - S) / abs(S)


@pytest.mark.parametrize("direction", [1, -1])
def test_flux_matches_closed_form(direction):
    err_series, err_sum = _pin_error(Simulation, direction)
    assert err_series < 1e-12, err_series
    assert err_sum < 1e-12, err_sum


def test_flux_window_sees_the_pulse():
    """The probe plane lies on the pulse's path: the flux is not trivially
    small, and it has the sign of the propagation direction."""
    for direction in (1, -1):
        _, pid, dt, _ = _setup(Simulation, direction)
        P, S = _closed_form(direction, dt)
        assert np.max(np.abs(P)) > 1e-6
        assert S * direction > 0


class _SignOfEzHy(Simulation):
    def flux_x(self, i0):
        dy, dz = self.d[1], self.d[2]
        im1 = (i0 - 1) % self.n[0]
        hz = 0.5 * (self.H[2][im1] + self.H[2][i0])
        hy = 0.5 * (self.H[1][im1] + self.H[1][i0])
        return dy * dz * (np.sum(self.E[1][i0] * hz) + np.sum(self.E[2][i0] * hy))


class _WrongSide(Simulation):
    def flux_x(self, i0):
        dy, dz = self.d[1], self.d[2]
        hz = 0.5 * (self.H[2][i0] + self.H[2][i0 + 1])
        hy = 0.5 * (self.H[1][i0] + self.H[1][i0 + 1])
        return dy * dz * (np.sum(self.E[1][i0] * hz) - np.sum(self.E[2][i0] * hy))


class _WrongArea(Simulation):
    def flux_x(self, i0):
        dx, dy = self.d[0], self.d[1]
        im1 = (i0 - 1) % self.n[0]
        hz = 0.5 * (self.H[2][im1] + self.H[2][i0])
        hy = 0.5 * (self.H[1][im1] + self.H[1][i0])
        return dx * dy * (np.sum(self.E[1][i0] * hz) - np.sum(self.E[2][i0] * hy))


@pytest.mark.parametrize("mutant", [_SignOfEzHy, _WrongSide, _WrongArea])
def test_planted_mistakes_fail_the_pin(mutant):
    err_series, _ = _pin_error(mutant, 1)
    assert err_series > 1e-3, (mutant.__name__, err_series)
