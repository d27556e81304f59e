"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test targets a different part of the scheme, so that a plausible
mistake (a dropped term, a wrong sign or index, a transposed operand, a
full instead of a half step) fails at least one of them:

* macrospin closed form (trapezoidal LLG = Cayley rotation; sign of gamma,
  closed-form solve, N(M), H + M bookkeeping);
* damped macrospin against the analytic LLG solution, second order in dt;
* PEC cavity eigenmode against the Yee dispersion relation (exact);
* modified discrete energy of the lossless leapfrog (curl adjointness, the
  H half steps, the eps/mu weights);
* discrete Gauss laws for B (H-M coupling of eq:Faraday2) and D;
* |M| = Ms after renormalisation;
* the converged sub-step against an independent 3x3 solve of eq:llg_tra3;
* PEC reflection coefficient -1 (Sec. 3.2.3);
* the time-step convention against the printed waveguide dt (Sec. 5.2.1).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import Simulation, from_config
from oracle.yee_llg import MU0 as O_MU0
from tests import pin_helpers as P

GAMMA = -1.759e11


def _uniform_periodic(n=(4, 4, 4), d=(1.0, 1.0, 1.0), dt=1e-12, Ms=1.4e5, alpha=0.0,
                      H0=(0.0, 0.0, 5e4), Hinit=(1e3, -2e3, 0.0), tilt_deg=30.0,
                      tol=1e-14):
    nx, ny, nz = n
    shp = (nz, ny, nx)
    th = math.radians(tilt_deg)
    m0 = np.zeros((3,) + shp)
    m0[0] = math.sin(th)
    m0[2] = math.cos(th)
    sim = Simulation(n, d, dt, Ms=np.full(shp, Ms), alpha=np.full(shp, alpha),
                     gamma=np.full(shp, GAMMA), m0_dir=m0, H0=H0,
                     periodic=(True, True, True), tol=tol, max_iter=60)
    H = [np.full(W.face_shape(n, (True,) * 3, c), Hinit[c]) for c in range(3)]
    sim.set_fields(H=H)
    M0 = np.array([Ms * math.sin(th), 0.0, Ms * math.cos(th)])
    A = np.array(H0) + np.array(Hinit) + M0
    return sim, M0, A


def test_macrospin_is_exact_cayley_rotation():
    """alpha = 0, uniform periodic box: E stays 0, H + M is conserved per face,
    so H_eff = A - M with A = H0 + H(0) + M(0) fixed and M x H_eff = M x A.
    The trapezoid is then a Cayley map: each half step rotates M about A by
    exactly 2*atan(mu0*|gamma|*|A|*dt/4), right-handed for gamma < 0."""
    dt = 1e-12
    sim, M0, A = _uniform_periodic(dt=dt)
    nsteps = 40
    sim.step(nsteps)
    phi = 2.0 * math.atan(O_MU0 * abs(GAMMA) * np.linalg.norm(A) * dt / 4.0)
    expect = P.rotate(M0, A, 2 * nsteps * phi)
    for f in range(3):
        got = np.array([sim.M[f][c][0, 0, 0] for c in range(3)])
        assert np.allclose(got, expect, rtol=0, atol=1e-9 * np.linalg.norm(M0)), (f, got, expect)
        # every face of the family carries the same value
        for c in range(3):
            assert np.ptp(sim.M[f][c]) < 1e-9 * np.linalg.norm(M0)
    # H + M conserved on each family's normal component; E identically zero
    Hinit = (1e3, -2e3, 0.0)
    for f in range(3):
        assert np.allclose(sim.H[f] + sim.M[f][f], Hinit[f] + M0[f], rtol=0, atol=1e-8 * np.linalg.norm(M0))
        assert np.all(sim.E[f] == 0.0)


def test_macrospin_rotation_sense_for_positive_gamma_flips():
    """With a positive gyromagnetic ratio the same closed form rotates the
    other way (signed-gamma reading of eq:llg_tra5/6)."""
    dt = 1e-12
    n = (2, 2, 2)
    sim, M0, A = _uniform_periodic(n=n, dt=dt)
    sim.gamma_f = [np.abs(g) for g in sim.gamma_f]
    sim.step(10)
    phi = 2.0 * math.atan(O_MU0 * abs(GAMMA) * np.linalg.norm(A) * dt / 4.0)
    expect = P.rotate(M0, A, -20 * phi)
    got = np.array([sim.M[0][c][0, 0, 0] for c in range(3)])
    assert np.allclose(got, expect, atol=1e-9 * np.linalg.norm(M0))


def _damped_angles(M, A):
    a = A / np.linalg.norm(A)
    m = M / np.linalg.norm(M)
    theta = math.acos(np.clip(np.dot(m, a), -1, 1))
    # azimuth in a fixed frame perpendicular to A
    e1 = np.cross(a, [0.0, 1.0, 0.0])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(a, e1)
    phi = math.atan2(np.dot(m, e2), np.dot(m, e1))
    return theta, phi


def test_damped_macrospin_second_order_in_time():
    """alpha > 0: uniform M precesses and relaxes about the fixed A with
    tan(theta/2) = tan(theta0/2) exp(-alpha w t / (1+alpha^2)) and
    dphi/dt = w / (1+alpha^2), w = mu0 |gamma| |A| (the Landau-Lifshitz form
    eq:LLG_scalar of the Gilbert equation).  The trapezoidal sub-steps are
    second order: halving dt divides the error at a fixed time by ~4."""
    alpha = 0.1
    T = 2.0e-10
    errs = []
    for nsteps in (100, 200, 400):
        dt = T / nsteps
        sim, M0, A = _uniform_periodic(n=(2, 2, 2), dt=dt, alpha=alpha, tol=1e-15)
        sim.step(nsteps)
        w = O_MU0 * abs(GAMMA) * np.linalg.norm(A)
        th0, ph0 = _damped_angles(M0, A)
        th = 2 * math.atan(math.tan(th0 / 2) * math.exp(-alpha * w * T / (1 + alpha**2)))
        ph = ph0 + w * T / (1 + alpha**2)
        # build the exact vector in the same frame
        a = A / np.linalg.norm(A)
        e1 = np.cross(a, [0.0, 1.0, 0.0])
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(a, e1)
        Ms = np.linalg.norm(M0)
        exact = Ms * (math.cos(th) * a + math.sin(th) * (math.cos(ph) * e1 + math.sin(ph) * e2))
        got = np.array([sim.M[1][c][0, 0, 0] for c in range(3)])
        errs.append(np.linalg.norm(got - exact) / Ms)
    r1 = math.log2(errs[0] / errs[1])
    r2 = math.log2(errs[1] / errs[2])
    assert errs[0] < 1e-2
    assert 1.9 < r1 < 2.1 and 1.9 < r2 < 2.1, (errs, r1, r2)


@pytest.mark.parametrize("orient", [0, 1, 2])
def test_pec_cavity_mode_follows_yee_dispersion(orient):
    """PEC box, uniform eps_r and mu_r, no magnets.  The field component along
    `orient`, uniform along that axis and sin(m pi a/Na) sin(p pi b/Nb) across,
    is an eigenvector of the discrete curl-curl; with H(0) = 0 the
    H1/2-E-H1/2 scheme gives E^n = cos(n theta) E^0 exactly, with
    sin(theta/2) = (c dt / 2) sqrt((2/da)^2 sin^2(m pi/2Na) + (2/db)^2 sin^2(p pi/2Nb))."""
    n = [6, 6, 6]
    n[orient] = 3
    n[(orient + 1) % 3] = 8
    n[(orient + 2) % 3] = 6
    n = tuple(n)
    d = (1e-3, 1.3e-3, 0.8e-3)
    eps_r, mu_r = 2.5, 1.5
    dt = W.cfl_dt(0.9, *d)
    shp = (n[2], n[1], n[0])
    sim = Simulation(n, d, dt, eps_r=np.full(shp, eps_r), mu_r=np.full(shp, mu_r))
    ua, ub = (orient + 1) % 3, (orient + 2) % 3
    m, p = 2, 1
    ext = W.edge_shape(n, (False,) * 3, orient)            # host layout (z, y, x)
    grids = np.meshgrid(np.arange(ext[2]), np.arange(ext[1]), np.arange(ext[0]), indexing="ij")
    coords = {0: grids[0].transpose(2, 1, 0), 1: grids[1].transpose(2, 1, 0), 2: grids[2].transpose(2, 1, 0)}
    mode = np.sin(m * math.pi * coords[ua] / n[ua]) * np.sin(p * math.pi * coords[ub] / n[ub])
    E = [np.zeros(W.edge_shape(n, (False,) * 3, c)) for c in range(3)]
    E[orient] = mode
    sim.set_fields(E=E)
    c = 1.0 / math.sqrt(P.MU0 * mu_r * P.EPS0 * eps_r)
    lam = ((2 / d[ua]) * math.sin(m * math.pi / (2 * n[ua]))) ** 2 + \
          ((2 / d[ub]) * math.sin(p * math.pi / (2 * n[ub]))) ** 2
    theta = 2 * math.asin(c * dt / 2 * math.sqrt(lam))
    for step in range(1, 31):
        sim.step(1)
        got = sim.field(["Ex", "Ey", "Ez"][orient])
        exp = math.cos(step * theta) * mode
        assert np.max(np.abs(got - exp)) < 1e-12 * (1 + step), (step, np.max(np.abs(got - exp)))
        for cc in range(3):
            if cc != orient:
                assert np.max(np.abs(sim.E[cc])) == 0.0


def _energy(sim, eps_e, mu_f, d, per):
    dV = d[0] * d[1] * d[2]
    E = [P.ijk(sim.field(nm)) for nm in ("Ex", "Ey", "Ez")]
    H = [P.ijk(sim.field(nm)) for nm in ("Hx", "Hy", "Hz")]
    curl = P.curl_E_faces(E, sim.n, d, per)
    we = sum(0.5 * np.sum(eps_e[c] * E[c] ** 2) for c in range(3))
    wh = sum(0.5 * np.sum(mu_f[c] * H[c] ** 2) for c in range(3))
    corr = sum((sim.dt**2 / 8.0) * np.sum(curl[c] ** 2 / mu_f[c]) for c in range(3))
    return dV * (we + wh - corr), dV * (we + wh)


@pytest.mark.parametrize("per", [(False, False, False), (True, False, True)])
def test_modified_energy_is_conserved_in_lossless_cavity(per):
    """Lossless leapfrog conserves W = 1/2 sum eps|E^n|^2 + 1/2 sum mu|H^n|^2
    - dt^2/8 sum |curl E^n|^2 / mu (H^n is the mean of the two half-step H),
    with eps/mu the 4-cell / 2-cell means computed independently here."""
    n = (5, 4, 3)
    d = (1e-3, 0.7e-3, 1.2e-3)
    rng = np.random.default_rng(3)
    shp = (n[2], n[1], n[0])
    eps_r = rng.uniform(1, 4, shp)
    mu_r = rng.uniform(1, 2, shp)
    dt = W.cfl_dt(0.9, *d)
    sim = Simulation(n, d, dt, eps_r=eps_r, mu_r=mu_r, periodic=per)
    cfg = W.Config("t", n, d, dt, 0, periodic=per)
    E, H = W.random_fields(cfg, seed=5)
    sim.set_fields(E=E, H=H)
    eps_e = [P.eps_edges(eps_r, n, per, c) for c in range(3)]
    mu_f = [P.MU0 * P.face_mean(mu_r, n, per, f) for f in range(3)]
    w0, plain0 = _energy(sim, eps_e, mu_f, d, per)
    plains = []
    for _ in range(40):
        sim.step(1)
        w, plain = _energy(sim, eps_e, mu_f, d, per)
        assert abs(w - w0) < 1e-12 * abs(w0), (w, w0)
        plains.append(plain)
    # the plain energy is not conserved (it oscillates), so the pin has teeth
    assert np.ptp(plains) > 1e-6 * plain0


def _B_faces(sim, cfgMs, mu_r, per):
    Bs = []
    for f, nm in enumerate(("Hx", "Hy", "Hz")):
        H = P.ijk(sim.field(nm))
        Mn = P.ijk(sim.field("M" + "xyz"[f] + "xyz"[f]))
        Ms_f = P.face_mean(cfgMs, sim.n, per, f)
        mu_f = P.MU0 * P.face_mean(mu_r, sim.n, per, f)
        Bs.append(np.where(Ms_f > 0, P.MU0 * (H + Mn), mu_f * H))
    return Bs


@pytest.mark.parametrize("per", [(False, False, False), (False, True, True)])
def test_gauss_law_for_B_is_invariant(per):
    """The H update is H + M_n = H^s + M^s_n - (dt/2mu0) curl E on magnetic
    faces and mu H = mu H^s - (dt/2) curl E elsewhere, so the per-cell flux
    of B is unchanged to round-off (div curl = 0), at every iterate."""
    n = (16, 8, 8)
    cfg = W.Config("gb", n, (1e-6,) * 3, W.cfl_dt(0.9, 1e-6, 1e-6, 1e-6), 0, periodic=per)
    shp = (n[2], n[1], n[0])
    rng = np.random.default_rng(11)
    Ms = np.zeros(shp)
    Ms[2:6, 2:6, 4:12] = 1.4e5
    mu_r = rng.uniform(1, 3, shp)
    m0 = np.zeros((3,) + shp)
    m0[0] = 0.3
    m0[2] = 1.0
    sim = Simulation(n, cfg.d, cfg.dt, Ms=Ms, alpha=np.full(shp, 0.02), mu_r=mu_r,
                     eps_r=rng.uniform(1, 5, shp), sigma=rng.uniform(0, 1e3, shp),
                     m0_dir=m0, H0=(1e4, 0, 5e4), periodic=per, tol=1e-12)
    E, H = W.random_fields(cfg, seed=2, amp_e=1e6, amp_h=3e3)
    sim.set_fields(E=E, H=H)
    d = cfg.d
    div0 = P.div_faces(_B_faces(sim, Ms, mu_r, per), n, d, per)
    scale = np.max(np.abs(_B_faces(sim, Ms, mu_r, per)[0])) / d[0]
    for _ in range(6):
        sim.step(1)
    assert max(sim.iters) > 2          # the H-M iteration was exercised
    div1 = P.div_faces(_B_faces(sim, Ms, mu_r, per), n, d, per)
    assert np.max(np.abs(div1 - div0)) < 1e-12 * scale


def test_gauss_law_for_D_is_invariant_without_charges():
    """sigma = 0 and no source: the node divergence of eps E is unchanged."""
    n = (6, 5, 4)
    d = (1e-6, 1.5e-6, 1e-6)
    shp = (n[2], n[1], n[0])
    rng = np.random.default_rng(4)
    eps_r = rng.uniform(1, 10, shp)
    Ms = np.zeros(shp)
    Ms[1:3, 1:4, 2:4] = 1.75e5
    dt = W.cfl_dt(0.9, *d)
    sim = Simulation(n, d, dt, eps_r=eps_r, Ms=Ms, alpha=np.full(shp, 0.01),
                     H0=(0, 0, 1e5), tol=1e-12)
    cfg = W.Config("gd", n, d, dt, 0)
    E, H = W.random_fields(cfg, seed=9, amp_e=1e5, amp_h=1e3)
    sim.set_fields(E=E, H=H)
    per = (False,) * 3
    eps_e = [P.eps_edges(eps_r, n, per, c) for c in range(3)]

    def divD():
        Es = [P.ijk(sim.field(nm)) for nm in ("Ex", "Ey", "Ez")]
        return P.div_edges([eps_e[c] * Es[c] for c in range(3)], n, d, per)

    d0 = divD()
    scale = P.EPS0 * 10 * 1e5 / 1e-6
    sim.step(8)
    assert np.max(np.abs(divD() - d0)[1:-1, 1:-1, 1:-1]) < 1e-12 * scale
    # with conductivity the divergence decays: the pin has teeth
    sim2 = Simulation(n, d, dt, eps_r=eps_r, sigma=np.full(shp, 1e5))
    sim2.set_fields(E=E, H=H)
    Es = [P.ijk(sim2.field(nm)) for nm in ("Ex", "Ey", "Ez")]
    d0b = P.div_edges([eps_e[c] * Es[c] for c in range(3)], n, d, per)
    sim2.step(4)
    Es = [P.ijk(sim2.field(nm)) for nm in ("Ex", "Ey", "Ez")]
    d1b = P.div_edges([eps_e[c] * Es[c] for c in range(3)], n, d, per)
    assert np.max(np.abs(d1b - d0b)) > 1e-6 * scale


def test_magnetisation_magnitude_is_Ms_on_every_face():
    cfg = W.slab64(steps=40)
    sim = from_config(cfg)
    E, H = W.random_fields(cfg, seed=1, amp_e=1e5, amp_h=5e3)
    sim.set_fields(E=E, H=H)
    sim.step(20)
    for f in range(3):
        m = sim.M[f]
        nrm = np.sqrt(m[0] ** 2 + m[1] ** 2 + m[2] ** 2)
        mag = sim.Ms_f[f] > 0
        assert np.max(np.abs(nrm[mag] - sim.Ms_f[f][mag]) / sim.Ms_f[f][mag]) < 1e-14
        assert np.all(nrm[~mag] == 0)


def test_converged_substep_solves_the_trapezoid():
    """After a sub-step, every evolving face satisfies eq:llg_tra3 with
    H_eff^{n+1/2} built from the output H: the direction of M^{n+1/2} equals
    that of the solution x of x + x x (-k H' + (alpha/Ms) M^n) = M^n + k M^n x H^n,
    solved here by a dense 3x3 linear solve (not the closed form)."""
    cfg = W.slab64(steps=0)
    sim = from_config(cfg, with_probes=False)
    sim.tol = 1e-15
    E, H = W.random_fields(cfg, seed=7, amp_e=1e7, amp_h=2e4)
    sim.set_fields(E=E, H=H)
    Hs = [a.copy() for a in sim.H]
    Ms0 = [[v.copy() for v in sim.M[f]] for f in range(3)]
    sim.hm_substep(sim.curl_E(sim.E))
    assert sim.iters[-1] >= 3
    rng = np.random.default_rng(0)
    dt = sim.dt

    def heff(Hl, f, i, j, k):
        # four-point means of the transverse components, written out
        out = np.zeros(3)
        for c in range(3):
            if c == f:
                out[c] = Hl[f][i, j, k]
            else:
                p = [i, j, k]
                s = 0.0
                for df in (-1, 0):
                    for dc in (0, 1):
                        q = list(p)
                        q[f] += df
                        q[c] += dc
                        s += Hl[c][tuple(q)]
                out[c] = s / 4.0
        return out + np.array(sim.H0)

    for f in range(3):
        idx = np.argwhere(sim.evolve[f])
        for t in rng.choice(len(idx), size=min(12, len(idx)), replace=False):
            i, j, k = idx[t]
            Mn = np.array([Ms0[f][c][i, j, k] for c in range(3)])
            Mh = np.array([sim.M[f][c][i, j, k] for c in range(3)])
            Hn = heff(Hs, f, i, j, k)
            Hh = heff(sim.H, f, i, j, k)
            kap = P.MU0 * GAMMA * dt / 4.0
            Ms = sim.Ms_f[f][i, j, k]
            alpha = sim.alpha_f[f][i, j, k]
            v = -kap * Hh + (alpha / Ms) * Mn
            rhs = Mn + kap * np.cross(Mn, Hn)
            # x + x x v = rhs  ->  (I + [.] x v) x = rhs ; x x v = -[v]x x
            Vx = np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]])
            x = np.linalg.solve(np.eye(3) - Vx, rhs)
            x *= Ms / np.linalg.norm(x)
            assert np.allclose(Mh, x, rtol=0, atol=1e-12 * Ms), (f, i, j, k, Mh, x)


def test_pec_reflection_coefficient_is_minus_one():
    """A right-going E_y/H_z pulse hits the PEC wall at x = nx and comes back
    with E_y inverted (Sec. 3.2.3)."""
    n = (240, 2, 2)
    d = (1e-6,) * 3
    dt = W.cfl_dt(0.9, *d)
    sim = Simulation(n, d, dt, periodic=(False, True, True))
    x_nodes = np.arange(n[0] + 1)
    x_cells = np.arange(n[0]) + 0.5
    x0, w = 120.0, 8.0
    eta = math.sqrt(P.MU0 / P.EPS0)
    ey = np.exp(-((x_nodes - x0) / w) ** 2)
    hz = np.exp(-((x_cells - x0) / w) ** 2) / eta
    E = [np.zeros(W.edge_shape(n, (False, True, True), c)) for c in range(3)]
    H = [np.zeros(W.face_shape(n, (False, True, True), c)) for c in range(3)]
    E[1][:, :, :] = ey[None, None, :]
    H[2][:, :, :] = hz[None, None, :]
    sim.set_fields(E=E, H=H)
    # travel to the wall (120 cells) and back to x0: 240 cells of path
    steps = int(round(240 * d[0] / (3e8 * dt)))
    sim.step(steps)
    got = P.ijk(sim.field("Ey"))[:, 0, 0]
    mirror = np.exp(-((x_nodes - x0) / w) ** 2)
    r = float(np.dot(got, mirror) / np.dot(mirror, mirror))
    assert abs(r + 1.0) < 0.03, r
    assert got[-1] == 0.0


def test_time_step_convention_matches_printed_waveguide_dt():
    """512 x 4 x 512 cells over W = 14.95 mm, h = 10.16 mm, L = 500 mm at CFL
    0.8 gives dt = 77.8796 fs in Sec. 5.2.1; the vacuum-CFL convention
    dt = CFL / (c sqrt(sum 1/d^2)) reproduces it to 1.4e-5."""
    dt = W.cfl_dt(0.8, 14.95e-3 / 512, 10.16e-3 / 4, 0.5 / 512)
    assert abs(dt - 77.87961902e-15) / 77.87961902e-15 < 2e-5
    # the min-spacing convention is clearly worse
    alt = 0.8 * (14.95e-3 / 512) / 3e8
    assert abs(alt - 77.87961902e-15) > 10 * abs(dt - 77.87961902e-15)


def test_wall_entries_stay_zero_and_interior_is_updated():
    cfg = W.slab64(steps=0)
    sim = from_config(cfg, with_probes=False)
    E, H = W.random_fields(cfg, seed=3, amp_e=1e3, amp_h=10.0)
    sim.set_fields(E=E, H=H)
    before = [sim.field(nm).copy() for nm in ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")]
    sim.step(1)
    nx, ny, nz = cfg.n
    after = [sim.field(nm) for nm in ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")]
    # tangential E on the walls (host layout [k][j][i])
    assert np.all(after[0][[0, -1], :, :] == 0) and np.all(after[0][:, [0, -1], :] == 0)
    assert np.all(after[1][[0, -1], :, :] == 0) and np.all(after[1][:, :, [0, -1]] == 0)
    assert np.all(after[2][:, [0, -1], :] == 0) and np.all(after[2][:, :, [0, -1]] == 0)
    # normal H on the walls
    assert np.all(after[3][:, :, [0, -1]] == 0)
    assert np.all(after[4][:, [0, -1], :] == 0)
    assert np.all(after[5][[0, -1], :, :] == 0)
    # every interior entry changed
    assert np.all(after[0][1:-1, 1:-1, :] != before[0][1:-1, 1:-1, :])
    assert np.all(after[3][:, :, 1:-1] != before[3][:, :, 1:-1])
