"""Pins of the oracle's first-order scheme (Sec. 3.2.1, scheme=1).

* Macrospin without damping: with E = 0 and H + M conserved per face,
  H_eff = A - M for the fixed vector A = H0 + H(0) + M(0), so one explicit
  half step adds (dt/2) mu0 gamma (M x A), perpendicular to M, and N(M)
  brings |M| back.  About A this is exact: the azimuth advances by
  atan(eps) and tan(theta) grows by sqrt(1 + eps^2) per half step, with
  eps = mu0 |gamma| |A| dt / 2 (the explicit step's well-known spiral away
  from the axis).  A wrong step length (dt instead of dt/2), a lost 1/(1 +
  alpha^2) or a wrong sign fails it.
* Damped macrospin against the analytic Landau-Lifshitz solution: first
  order in time (error halves with dt).
* The H update of eq:H_update keeps the per-cell flux of B, as in the
  second-order scheme.
"""
import math

import numpy as np

import workloads as W
from oracle import Simulation
from oracle.yee_llg import MU0 as O_MU0
from tests import pin_helpers as P

GAMMA = -1.759e11


def _macrospin(dt, alpha=0.0, n=(2, 2, 2), Ms=1.4e5, H0=(0.0, 0.0, 5e4), Hinit=(1e3, -2e3, 0.0),
               tilt_deg=30.0):
    shp = (n[2], n[1], n[0])
    th = math.radians(tilt_deg)
    m0 = np.zeros((3,) + shp)
    m0[0] = math.sin(th)
    m0[2] = math.cos(th)
    sim = Simulation(n, (1.0, 1.0, 1.0), dt, Ms=np.full(shp, Ms), alpha=np.full(shp, alpha),
                     gamma=np.full(shp, GAMMA), m0_dir=m0, H0=H0, periodic=(True,) * 3, scheme=1)
    sim.set_fields(H=[np.full(W.face_shape(n, (True,) * 3, c), Hinit[c]) for c in range(3)])
    M0 = np.array([Ms * math.sin(th), 0.0, Ms * math.cos(th)])
    A = np.array(H0) + np.array(Hinit) + M0
    return sim, M0, A


def _frame(A):
    a = A / np.linalg.norm(A)
    e1 = np.cross(a, [0.0, 1.0, 0.0])
    e1 /= np.linalg.norm(e1)
    return a, e1, np.cross(a, e1)


def _angles(M, A):
    a, e1, e2 = _frame(A)
    m = M / np.linalg.norm(M)
    return math.acos(np.clip(np.dot(m, a), -1, 1)), math.atan2(np.dot(m, e2), np.dot(m, e1))


def _vector(Ms, th, ph, A):
    a, e1, e2 = _frame(A)
    return Ms * (math.cos(th) * a + math.sin(th) * (math.cos(ph) * e1 + math.sin(ph) * e2))


def test_undamped_macrospin_explicit_spiral():
    dt = 1e-12
    sim, M0, A = _macrospin(dt)
    nsteps = 30
    sim.step(nsteps)
    eps = O_MU0 * abs(GAMMA) * np.linalg.norm(A) * dt / 2
    th0, ph0 = _angles(M0, A)
    nh = 2 * nsteps
    th = math.atan(math.tan(th0) * (1 + eps**2) ** (nh / 2))
    ph = ph0 + nh * math.atan(eps)
    expect = _vector(np.linalg.norm(M0), th, ph, A)
    for f in range(3):
        got = np.array([sim.M[f][c][0, 0, 0] for c in range(3)])
        assert np.allclose(got, expect, rtol=0, atol=1e-9 * np.linalg.norm(M0)), (f, got, expect)
    # the spiral really moved theta (so the test sees the explicit step)
    assert th - th0 > 1e-3
    Hinit = (1e3, -2e3, 0.0)
    for f in range(3):
        assert np.allclose(sim.H[f] + sim.M[f][f], Hinit[f] + M0[f], rtol=0, atol=1e-8 * np.linalg.norm(M0))
        assert np.all(sim.E[f] == 0.0)
    assert set(sim.iters) == {1}


def test_damped_macrospin_first_order_in_time():
    alpha = 0.1
    T = 2.0e-10
    errs = []
    for nsteps in (200, 400, 800):
        dt = T / nsteps
        sim, M0, A = _macrospin(dt, alpha=alpha)
        sim.step(nsteps)
        w = O_MU0 * abs(GAMMA) * np.linalg.norm(A)
        th0, ph0 = _angles(M0, A)
        th = 2 * math.atan(math.tan(th0 / 2) * math.exp(-alpha * w * T / (1 + alpha**2)))
        ph = ph0 + w * T / (1 + alpha**2)
        exact = _vector(np.linalg.norm(M0), th, ph, A)
        got = np.array([sim.M[1][c][0, 0, 0] for c in range(3)])
        errs.append(np.linalg.norm(got - exact) / np.linalg.norm(M0))
    r1 = math.log2(errs[0] / errs[1])
    r2 = math.log2(errs[1] / errs[2])
    assert errs[0] < 5e-2
    assert 0.9 < r1 < 1.1 and 0.9 < r2 < 1.1, (errs, r1, r2)


def test_gauss_law_for_B_first_order():
    n = (12, 6, 6)
    per = (False, True, False)
    d = (1e-6,) * 3
    cfg = W.Config("gb1", n, d, W.cfl_dt(0.9, *d), 0, periodic=per)
    shp = (n[2], n[1], n[0])
    rng = np.random.default_rng(7)
    Ms = np.zeros(shp)
    Ms[1:5, 1:5, 3:9] = 1.2e5
    mu_r = rng.uniform(1, 2, shp)
    m0 = np.zeros((3,) + shp)
    m0[1], m0[2] = 0.4, 1.0
    sim = Simulation(n, d, cfg.dt, Ms=Ms, alpha=np.full(shp, 0.05), mu_r=mu_r,
                     eps_r=rng.uniform(1, 4, shp), m0_dir=m0, H0=(0, 2e4, 6e4), periodic=per, scheme=1)
    E, H = W.random_fields(cfg, seed=3, amp_e=1e6, amp_h=3e3)
    sim.set_fields(E=E, H=H)

    def B():
        out = []
        for f, nm in enumerate(("Hx", "Hy", "Hz")):
            Hf = P.ijk(sim.field(nm))
            Mn = P.ijk(sim.field("M" + "xyz"[f] + "xyz"[f]))
            Ms_f = P.face_mean(Ms, n, per, f)
            out.append(np.where(Ms_f > 0, P.MU0 * (Hf + Mn), P.MU0 * P.face_mean(mu_r, n, per, f) * Hf))
        return out

    b0 = B()
    div0 = P.div_faces(b0, n, d, per)
    scale = np.max(np.abs(b0[0])) / d[0]
    sim.step(5)
    div1 = P.div_faces(B(), n, d, per)
    assert np.max(np.abs(div1 - div0)) < 1e-12 * scale
