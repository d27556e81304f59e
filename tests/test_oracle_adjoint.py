"""Pins of the oracle's reverse-mode gradient (oracle/adjoint.py).

* Complex step: running the forward oracle with eps_r + i h v (or Ms + i h v)
  gives Im(L)/h = dL/dp . v to machine precision, an exact directional
  derivative that shares nothing with the reverse sweep.
* Dot-product test of one step in state space: <J v, w> from a complex-step
  JVP equals <v, J^T w> from step_vjp for random v (E, H, M) and w.
* Central finite differences with h = 1e-6 relative on single cells, in
  fixed-iteration mode (with the stopping test a +-h run can take one more
  or one fewer iteration in some sub-step, a jump the derivative does not
  see).  Their bar is 1e-6 relative plus the difference quotient's own
  rounding floor, 1e3 * eps * |L| / h.
* A single-cell complex step, which has no such floor.
"""
import numpy as np
import pytest

import workloads as W
from oracle import Simulation
from oracle import adjoint as A

N = (12, 6, 5)
D = (1e-6, 1.2e-6, 0.9e-6)
I0 = 9
STEPS = 10


def _materials():
    rng = np.random.default_rng(0)
    shp = (N[2], N[1], N[0])
    eps = rng.uniform(1.0, 4.0, shp)
    sig = rng.uniform(0.0, 5e3, shp)
    Ms = np.zeros(shp)
    Ms[1:4, 1:5, 3:9] = rng.uniform(1e5, 1.8e5, (3, 4, 6))
    alpha = np.where(Ms > 0, rng.uniform(0.01, 0.05, shp), 0.0)
    m0 = np.zeros((3,) + shp)
    m0[0], m0[1], m0[2] = 0.3, -0.2, 1.0
    prof = np.zeros(W.edge_shape(N, (False,) * 3, 2))
    prof[:, 1:N[1], 2] = 1e11 * np.sin(np.pi * np.arange(1, N[1]) / N[1])[None, :]
    E, H = W.random_fields(W.Config("a", N, D, 1.0, 0), seed=3, amp_e=3e5, amp_h=3e3)
    return eps, sig, Ms, alpha, m0, prof, E, H


def _make(eps=None, Ms=None, dtype=np.float64, fixed_iter=0):
    e0, sig, ms0, alpha, m0, prof, E, H = _materials()
    dt = W.cfl_dt(0.9, *D)
    sim = Simulation(N, D, dt, eps_r=e0 if eps is None else eps, sigma=sig,
                     Ms=ms0 if Ms is None else Ms, alpha=alpha, m0_dir=m0,
                     H0=(2e4, 0.0, 1.2e5), source=(2, prof, 3e12, 1 / 3e12, 1e-12),
                     tol=1e-13, max_iter=50, fixed_iter=fixed_iter, dtype=dtype)
    sim.set_fields(E=E, H=H)
    return sim


def _loss(sim):
    L = 0.0
    for _ in range(STEPS):
        sim.step(1)
        L = L + sim.dt * sim.flux_x(I0)
    return L


@pytest.fixture(scope="module")
def grads():
    L, g_eps, g_ms = A.loss_and_gradients(_make, STEPS, I0)
    return L, g_eps, g_ms


def _complex_step(v_eps=None, v_ms=None, h=1e-30):
    e0, _, ms0, *_ = _materials()
    eps = e0 + (1j * h * v_eps if v_eps is not None else 0)
    ms = ms0 + (1j * h * v_ms if v_ms is not None else 0)
    sim = _make(eps=eps.astype(complex), Ms=ms.astype(complex), dtype=np.complex128)
    return float(np.imag(_loss(sim))) / h


def test_gradient_eps_matches_complex_step(grads):
    L, g_eps, _ = grads
    rng = np.random.default_rng(11)
    v = rng.standard_normal(g_eps.shape)
    cs = _complex_step(v_eps=v)
    ad = float(np.sum(g_eps * v))
    assert abs(ad - cs) <= 1e-10 * abs(cs), (ad, cs)
    assert abs(cs) > 0


def test_gradient_Ms_matches_complex_step(grads):
    L, _, g_ms = grads
    e0, _, ms0, *_ = _materials()
    rng = np.random.default_rng(12)
    v = np.where(ms0 > 0, rng.standard_normal(ms0.shape) * 1e4, 0.0)
    cs = _complex_step(v_ms=v)
    ad = float(np.sum(g_ms * v))
    assert abs(ad - cs) <= 1e-10 * abs(cs), (ad, cs)
    assert abs(cs) > 0


def test_gradient_central_differences():
    L, g_eps, g_ms = A.loss_and_gradients(lambda: _make(fixed_iter=4), STEPS, I0)
    e0, _, ms0, *_ = _materials()
    rng = np.random.default_rng(5)
    cells = [tuple(c) for c in np.argwhere(ms0 > 0)]
    picks = [cells[i] for i in rng.choice(len(cells), 3, replace=False)]
    for idx in picks:
        for which in ("eps", "ms"):
            base = e0 if which == "eps" else ms0
            h = 1e-6 * base[idx]
            vals = []
            for sgn in (1, -1):
                p = base.copy()
                p[idx] += sgn * h
                sim = _make(eps=p, fixed_iter=4) if which == "eps" else _make(Ms=p, fixed_iter=4)
                vals.append(float(_loss(sim)))
            fd = (vals[0] - vals[1]) / (2 * h)
            ad = (g_eps if which == "eps" else g_ms)[idx]
            floor = 1e3 * 2.220446049250313e-16 * abs(L) / h
            assert abs(fd - ad) <= 1e-6 * abs(ad) + floor, (which, idx, fd, ad, floor)
            assert abs(fd - ad) <= 1e-2 * abs(ad), (which, idx, fd, ad)


def test_single_cell_complex_step(grads):
    L, g_eps, g_ms = grads
    e0, _, ms0, *_ = _materials()
    idx = tuple(np.argwhere(ms0 > 0)[7])
    for which, g, base in (("eps", g_eps, e0), ("ms", g_ms, ms0)):
        v = np.zeros_like(base)
        v[idx] = 1.0
        cs = _complex_step(v_eps=v) if which == "eps" else _complex_step(v_ms=v)
        assert abs(g[idx] - cs) <= 1e-9 * abs(cs), (which, g[idx], cs)


def test_step_vjp_dot_product():
    """<J v, w> = <v, J^T w> for one step, J the Jacobian of (E, H, M)^n ->
    (E, H, M)^{n+1} at a random state."""
    rng = np.random.default_rng(21)
    sim = _make()
    # random tangent on the interior entries and on the evolving faces' M
    vE = [np.where(sim.e_interior[c], rng.standard_normal(sim.E[c].shape), 0.0) * 1e3 for c in range(3)]
    vH = [np.where(sim.h_interior[f], rng.standard_normal(sim.H[f].shape), 0.0) * 10 for f in range(3)]
    vM = [[np.where(sim.evolve[f], rng.standard_normal(sim.H[f].shape), 0.0) * 10 for _ in range(3)]
          for f in range(3)]
    h = 1e-30
    simc = _make(dtype=np.complex128)
    for c in range(3):
        simc.E[c] = simc.E[c] + 1j * h * vE[c]
        simc.H[c] = simc.H[c] + 1j * h * vH[c]
        for q in range(3):
            simc.M[c][q] = simc.M[c][q] + 1j * h * vM[c][q]
    simc.step(1)
    jE = [np.imag(a) / h for a in simc.E]
    jH = [np.imag(a) / h for a in simc.H]
    jM = [[np.imag(v) / h for v in simc.M[f]] for f in range(3)]
    # random cotangent
    wE = [rng.standard_normal(a.shape) for a in jE]
    wH = [rng.standard_normal(a.shape) for a in jH]
    wM = [[rng.standard_normal(v.shape) for v in jM[f]] for f in range(3)]
    lhs = (sum(np.sum(jE[c] * np.where(sim.e_interior[c], wE[c], 0)) for c in range(3))
           + sum(np.sum(jH[c] * np.where(sim.h_interior[c], wH[c], 0)) for c in range(3))
           + sum(np.sum(jM[f][q] * wM[f][q]) for f in range(3) for q in range(3)))
    tape = []
    sim.step(1, tape=tape)
    z = [np.zeros(sim.edge_shape(c)) for c in range(3)]
    zf = [np.zeros(sim.face_shape(f)) for f in range(3)]
    eb, hb, mb = A.step_vjp(sim, tape[0], wE, wH, wM, A.edge_coef_derivs(sim), z,
                            [a.copy() for a in zf], [a.copy() for a in zf])
    rhs = (sum(np.sum(vE[c] * eb[c]) for c in range(3)) + sum(np.sum(vH[c] * hb[c]) for c in range(3))
           + sum(np.sum(vM[f][q] * mb[f][q]) for f in range(3) for q in range(3)))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs)), (lhs, rhs)
