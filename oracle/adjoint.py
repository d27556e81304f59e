"""Reverse mode of the oracle's coupled step (FP64).

TEST INFRASTRUCTURE ONLY (imported by the tests; the product path never
calls it).

The loss is the time-integrated Poynting flux through the node plane
x = i0, L = sum_{n=1}^{N} dt P^n, with P as in the forward oracle.  The
gradient is taken with respect to the cell maps eps_r and Ms by exact
reverse-mode differentiation of the computation the forward oracle performs
(the paper has no adjoint):

  * each H-M sub-step is reversed iteration by iteration, replaying the
    iterates recorded on the tape (the stopping rule is piecewise constant
    and contributes nothing);
  * the E update (Sec. 3.2.1 Step 2) is reversed as a linear map in E and H
    plus the derivatives of ca, cb with respect to the edge eps;
  * the parameter chain runs through the 4-cell edge mean of eps_r and,
    for Ms, through the face mean Ms_f (renormalisation target and alpha/Ms)
    and the initial face magnetisation (mean of Ms*m0 renormalised to Ms_f).
    Which faces are magnetic is a discrete choice and is held fixed, as are
    the alpha/gamma face values (means over the magnetic cells).

Every transpose below is written from the forward operator it reverses.
"""
from __future__ import annotations

import numpy as np

from .yee_llg import (EPS0, MU0, _sl, cross, dot, s_down, s_up, to_host, vacus_solve,
                      waveform)


# --------------------------------------------------------------------------
# transposes of the staggered difference / pair-sum operators
# --------------------------------------------------------------------------

def d_up_T(g, ax, per):
    """Transpose of d_up (nodes -> cells, a[m+1] - a[m])."""
    if per:
        return np.roll(g, 1, axis=ax) - g
    shp = list(g.shape)
    shp[ax] += 1
    out = np.zeros(shp, dtype=g.dtype)
    out[_sl(ax, slice(0, -1))] -= g
    out[_sl(ax, slice(1, None))] += g
    return out


def d_down_T(g, ax, per):
    """Transpose of d_down (cells -> nodes, a[m] - a[m-1], wall nodes 0)."""
    if per:
        return g - np.roll(g, -1, axis=ax)
    gi = g.copy()
    gi[_sl(ax, 0)] = 0.0
    gi[_sl(ax, -1)] = 0.0
    return gi[_sl(ax, slice(0, -1))] - gi[_sl(ax, slice(1, None))]


def s_up_T(g, ax, per):
    """Transpose of s_up (nodes -> cells, a[m] + a[m+1])."""
    if per:
        return g + np.roll(g, 1, axis=ax)
    shp = list(g.shape)
    shp[ax] += 1
    out = np.zeros(shp, dtype=g.dtype)
    out[_sl(ax, slice(0, -1))] += g
    out[_sl(ax, slice(1, None))] += g
    return out


def s_down_T(g, ax, per, clamp=False):
    """Transpose of s_down (cells -> nodes, a[m-1] + a[m]; wall nodes 0, or
    2 * inside value with clamp)."""
    if per:
        return g + np.roll(g, -1, axis=ax)
    gi = g.copy()
    gi[_sl(ax, 0)] = 0.0
    gi[_sl(ax, -1)] = 0.0
    out = gi[_sl(ax, slice(0, -1))] + gi[_sl(ax, slice(1, None))]
    if clamp:
        out[_sl(ax, 0)] += 2.0 * g[_sl(ax, 0)]
        out[_sl(ax, -1)] += 2.0 * g[_sl(ax, -1)]
    return out


def curl_E_T(sim, Cb):
    """Transpose of Simulation.curl_E: face cotangents -> edge cotangents."""
    dx, dy, dz = sim.d
    px, py, pz = sim.per
    Eb = [np.zeros(sim.edge_shape(c)) for c in range(3)]
    # cx = d_up(E2, y)/dy - d_up(E1, z)/dz ; cy = d_up(E0, z)/dz - d_up(E2, x)/dx ;
    # cz = d_up(E1, x)/dx - d_up(E0, y)/dy
    Eb[2] += d_up_T(Cb[0], 1, py) / dy
    Eb[1] -= d_up_T(Cb[0], 2, pz) / dz
    Eb[0] += d_up_T(Cb[1], 2, pz) / dz
    Eb[2] -= d_up_T(Cb[1], 0, px) / dx
    Eb[1] += d_up_T(Cb[2], 0, px) / dx
    Eb[0] -= d_up_T(Cb[2], 1, py) / dy
    return Eb


def curl_H_T(sim, Eb):
    """Transpose of Simulation.curl_H: edge cotangents -> face cotangents."""
    dx, dy, dz = sim.d
    px, py, pz = sim.per
    Hb = [np.zeros(sim.face_shape(c)) for c in range(3)]
    # cx = d_down(H2, y)/dy - d_down(H1, z)/dz ; cy = d_down(H0, z)/dz - d_down(H2, x)/dx ;
    # cz = d_down(H1, x)/dx - d_down(H0, y)/dy
    Hb[2] += d_down_T(Eb[0], 1, py) / dy
    Hb[1] -= d_down_T(Eb[0], 2, pz) / dz
    Hb[0] += d_down_T(Eb[1], 2, pz) / dz
    Hb[2] -= d_down_T(Eb[1], 0, px) / dx
    Hb[1] += d_down_T(Eb[2], 0, px) / dx
    Hb[0] -= d_down_T(Eb[2], 1, py) / dy
    return Hb


def transverse_T(sim, g, f, c):
    """Transpose of Simulation.transverse(H, f, c) = 0.25 s_up(s_down(H_c, f), c)."""
    return 0.25 * s_down_T(s_up_T(g, c, sim.per[c]), f, sim.per[f])


def vacus_vjp(a, b, x, xb):
    """Cotangents of a and b for x = (b + (a.b) a - a x b) / (1 + |a|^2)."""
    D = 1.0 + dot(a, a)
    ub = [xb[c] / D for c in range(3)]
    a_ub = dot(a, ub)
    a_b = dot(a, b)
    x_xb = dot(x, xb)
    axu = cross(a, ub)
    uxb = cross(ub, b)
    bb = [ub[c] + a[c] * a_ub + axu[c] for c in range(3)]
    ab = [b[c] * a_ub + a_b * ub[c] + uxb[c] - 2.0 * a[c] * x_xb / D for c in range(3)]
    return ab, bb


# --------------------------------------------------------------------------
# reverse of one H-M sub-step
# --------------------------------------------------------------------------

def substep_vjp(sim, tr, Hb_out, Mb_out):
    """Given cotangents of the sub-step outputs (H' on all faces, M' per
    family), return cotangents of its inputs H^s, M^s and C (curl E at the
    faces), and of the face Ms (through N(M)) and of alpha/Ms."""
    h = 0.5 * sim.dt
    Hs, Ms0, C, Hprevs = tr["Hs"], tr["Ms0"], tr["C"], tr["Hprevs"]
    R = len(Hprevs)
    zf = lambda f: np.zeros(sim.face_shape(f))
    Hb_s = [zf(f) for f in range(3)]
    Mb_s = [[zf(f) for _ in range(3)] for f in range(3)]
    Cb = [zf(f) for f in range(3)]
    Msf_b = [zf(f) for f in range(3)]
    aoms_b = [zf(f) for f in range(3)]
    kap, aoms, He_s, b, d = [], [], [], [], []
    for f in range(3):
        k = MU0 * sim.gamma_f[f] * sim.dt / 4.0
        mag = sim.mag[f]
        with np.errstate(divide="ignore", invalid="ignore"):
            ao = np.where(mag, sim.alpha_f[f] / np.where(mag, sim.Ms_f[f], 1.0), 0.0)
        He = sim.H_eff(Hs, f)
        mxh = cross(Ms0[f], He)
        kap.append(k)
        aoms.append(ao)
        He_s.append(He)
        b.append([Ms0[f][c] + k * mxh[c] for c in range(3)])
        d.append([ao * Ms0[f][c] for c in range(3)])
    qb = [zf(f) for f in range(3)]
    bb = [[zf(f) for _ in range(3)] for f in range(3)]
    db = [[zf(f) for _ in range(3)] for f in range(3)]
    Hnm_b = [zf(f) for f in range(3)]
    Hb = [a.copy() for a in Hb_out]
    Mb = []
    for f in range(3):
        ev = sim.evolve[f]
        # faces that do not evolve keep M = M^s through the sub-step
        for c in range(3):
            Mb_s[f][c] += np.where(ev, 0.0, Mb_out[f][c])
        Mb.append([np.where(ev, Mb_out[f][c], 0.0) for c in range(3)])
    for r in range(R, 0, -1):
        Hprev = Hprevs[r - 1]
        Hb_prev = [zf(f) for f in range(3)]
        for f in range(3):
            ev = sim.evolve[f]
            # H^{(r)} = q - M^{(r)}_f on evolving faces, the one-shot value elsewhere
            qb[f] += np.where(ev, Hb[f], 0.0)
            Mb[f][f] = Mb[f][f] - np.where(ev, Hb[f], 0.0)
            Hnm_b[f] += np.where(ev, 0.0, Hb[f])
            # M^{(r)} = N(x), x = V(a, b), a = kappa H_eff(H^{(r-1)}) - d
            He = sim.H_eff(Hprev, f)
            a = [kap[f] * He[c] - d[f][c] for c in range(3)]
            x = vacus_solve(a, b[f])
            nrm = np.sqrt(dot(x, x))
            safe = np.where(ev, nrm, 1.0)
            xh = [np.where(ev, x[c] / safe, 0.0) for c in range(3)]
            m_b = [np.where(ev, Mb[f][c], 0.0) for c in range(3)]
            Msf_b[f] += dot(m_b, xh)
            sc = np.where(ev, sim.Ms_f[f] / safe, 0.0)
            pr = dot(xh, m_b)
            xb = [sc * (m_b[c] - xh[c] * pr) for c in range(3)]
            ab, bbr = vacus_vjp(a, b[f], x, xb)
            for c in range(3):
                bb[f][c] += np.where(ev, bbr[c], 0.0)
                db[f][c] -= np.where(ev, ab[c], 0.0)
            heb = [np.where(ev, kap[f] * ab[c], 0.0) for c in range(3)]
            for c in range(3):
                if c == f:
                    Hb_prev[f] += heb[f]
                else:
                    Hb_prev[c] += transverse_T(sim, heb[c], f, c)
        Hb = Hb_prev
        Mb = [[zf(f) for _ in range(3)] for f in range(3)]
    # H^{(0)} = H^s is what iteration 1 read
    for f in range(3):
        Hb_s[f] += Hb[f]
    # iteration-invariant parts
    for f in range(3):
        ev = sim.evolve[f]
        interior = sim.h_interior[f]
        # q = H^s + M^s_f - (h/mu0) C
        qe = np.where(ev, qb[f], 0.0)
        Hb_s[f] += qe
        Mb_s[f][f] += qe
        Cb[f] += -(h / MU0) * qe
        # one-shot value: H^s - (h/mu_f) C on interior faces, H^s on walls
        Hb_s[f] += Hnm_b[f]
        Cb[f] += np.where(interior, -(h / sim.mu_f[f]) * Hnm_b[f], 0.0)
        # b = M^s + kappa M^s x H_eff^s
        bf = [np.where(ev, bb[f][c], 0.0) for c in range(3)]
        hxb = cross(He_s[f], bf)
        for c in range(3):
            Mb_s[f][c] += bf[c] + kap[f] * hxb[c]
        bxm = cross(bf, Ms0[f])
        heb = [kap[f] * bxm[c] for c in range(3)]
        for c in range(3):
            if c == f:
                Hb_s[f] += heb[f]
            else:
                Hb_s[c] += transverse_T(sim, heb[c], f, c)
        # d = (alpha/Ms) M^s
        dfb = [np.where(ev, db[f][c], 0.0) for c in range(3)]
        for c in range(3):
            Mb_s[f][c] += aoms[f] * dfb[c]
        aoms_b[f] += dot(dfb, Ms0[f])
    return Hb_s, Mb_s, Cb, Msf_b, aoms_b


# --------------------------------------------------------------------------
# loss and full reverse sweep
# --------------------------------------------------------------------------

def flux_vjp(sim, E, H, i0, w):
    """Cotangents of w * P(E, H) at the node plane x = i0."""
    dx, dy, dz = sim.d
    im1 = (i0 - 1) % sim.n[0]
    i0m = i0 % sim.n[0]
    Eb = [np.zeros(sim.edge_shape(c)) for c in range(3)]
    Hb = [np.zeros(sim.face_shape(c)) for c in range(3)]
    s = w * dy * dz
    hz = 0.5 * (H[2][im1] + H[2][i0m])
    hy = 0.5 * (H[1][im1] + H[1][i0m])
    Eb[1][i0] += s * hz
    Hb[2][im1] += s * 0.5 * E[1][i0]
    Hb[2][i0m] += s * 0.5 * E[1][i0]
    Eb[2][i0] -= s * hy
    Hb[1][im1] -= s * 0.5 * E[2][i0]
    Hb[1][i0m] -= s * 0.5 * E[2][i0]
    return Eb, Hb


def edge_eps_sigma(sim, c):
    t1, t2 = [a for a in range(3) if a != c]
    per = sim.per
    eps_e = EPS0 * (0.25 * s_down(s_down(sim.eps_r, t1, per[t1]), t2, per[t2]))
    sig_e = 0.25 * s_down(s_down(sim.sigma, t1, per[t1]), t2, per[t2])
    return eps_e, sig_e


def run_with_tape(sim, nsteps, i0):
    """Forward run recording the tape; returns (L, tape)."""
    tape = []
    L = 0.0
    for _ in range(nsteps):
        sim.step(1, tape=tape)
        L += sim.dt * sim.flux_x(i0)
    return L, tape


def step_vjp(sim, rec, Eb, Hb, Mb, coef, epse_b, Msf_b, aoms_b):
    """Reverse of one step n -> n+1 recorded in `rec`: cotangents of
    (E, H, M)^{n+1} -> cotangents of (E, H, M)^n; parameter cotangents are
    accumulated into epse_b (edge eps), Msf_b (face Ms) and aoms_b (alpha/Ms)."""
    dt = sim.dt
    Eb = [np.where(sim.e_interior[c], Eb[c], 0.0) for c in range(3)]
    Hb = [np.where(sim.h_interior[c], Hb[c], 0.0) for c in range(3)]
    # Step 3
    Hh, Mh, Cb, ms_b, ao_b = substep_vjp(sim, rec["tr3"], Hb, Mb)
    for f in range(3):
        Msf_b[f] += ms_b[f]
        aoms_b[f] += ao_b[f]
    cE = curl_E_T(sim, Cb)
    Ebi = [np.where(sim.e_interior[c], Eb[c] + cE[c], 0.0) for c in range(3)]
    # Step 2: E' = ca E + cb (curl H^{n+1/2} - J g)
    CH = sim.curl_H(rec["tr3"]["Hs"])
    t_half = (rec["n"] + 0.5) * dt
    for c in range(3):
        rhs = CH[c]
        if sim.src is not None and sim.src[0] == c:
            _, prof, f0, Tp, t0 = sim.src
            rhs = rhs - prof * waveform(t_half, f0, Tp, t0)
        dca, dcb = coef[c]
        epse_b[c] += Ebi[c] * (rec["E0"][c] * dca + rhs * dcb)
    cH = curl_H_T(sim, [sim.cb[c] * Ebi[c] for c in range(3)])
    for f in range(3):
        Hh[f] = Hh[f] + cH[f]
    En = [sim.ca[c] * Ebi[c] for c in range(3)]
    # Step 1
    H0b, M0b, Cb1, ms_b, ao_b = substep_vjp(sim, rec["tr1"], Hh, Mh)
    for f in range(3):
        Msf_b[f] += ms_b[f]
        aoms_b[f] += ao_b[f]
    cE = curl_E_T(sim, Cb1)
    Eb = [np.where(sim.e_interior[c], En[c] + cE[c], 0.0) for c in range(3)]
    Hb = [np.where(sim.h_interior[f], H0b[f], 0.0) for f in range(3)]
    return Eb, Hb, M0b


def edge_coef_derivs(sim):
    """d ca / d eps_e and d cb / d eps_e on every edge (0 on walls):
    ca = (eps/dt - sigma/2)/D, cb = 1/D, D = eps/dt + sigma/2."""
    dt = sim.dt
    out = []
    for c in range(3):
        eps_e, sig_e = edge_eps_sigma(sim, c)
        with np.errstate(divide="ignore", invalid="ignore"):
            Dn = eps_e / dt + sig_e / 2.0
            dca = np.where(sim.e_interior[c], (sig_e / dt) / (Dn * Dn), 0.0)
            dcb = np.where(sim.e_interior[c], -(1.0 / dt) / (Dn * Dn), 0.0)
        out.append((dca, dcb))
    return out


def reverse(sim, tape, i0, M0_state):
    """Gradients of L = sum dt P^n (P at x = i0) with respect to the eps_r and
    Ms cell maps, in host layout.  `sim` is the simulation after the forward
    run (its materials are used); M0_state is its initial face M."""
    dt = sim.dt
    per = sim.per
    Eb = [np.zeros(sim.edge_shape(c)) for c in range(3)]
    Hb = [np.zeros(sim.face_shape(c)) for c in range(3)]
    Mb = [[np.zeros(sim.face_shape(f)) for _ in range(3)] for f in range(3)]
    epse_b = [np.zeros(sim.edge_shape(c)) for c in range(3)]
    Msf_b = [np.zeros(sim.face_shape(f)) for f in range(3)]
    aoms_b = [np.zeros(sim.face_shape(f)) for f in range(3)]
    coef = edge_coef_derivs(sim)
    for rec in reversed(tape):
        gE, gH = flux_vjp(sim, rec["E1"], rec["H1"], i0, dt)
        Eb = [Eb[c] + gE[c] for c in range(3)]
        Hb = [Hb[c] + gH[c] for c in range(3)]
        Eb, Hb, Mb = step_vjp(sim, rec, Eb, Hb, Mb, coef, epse_b, Msf_b, aoms_b)
    # ---- parameter chains -------------------------------------------------
    eps_b = np.zeros(sim.n)
    for c in range(3):
        t1, t2 = [a for a in range(3) if a != c]
        g = EPS0 * 0.25 * np.where(sim.e_interior[c], epse_b[c], 0.0)
        eps_b += s_down_T(s_down_T(g, t2, per[t2]), t1, per[t1])
    Ms_b = np.zeros(sim.n)
    m0 = sim.m0_dir
    for f in range(3):
        mag = sim.mag[f]
        ev = sim.evolve[f]
        Msf = sim.Ms_f[f]
        with np.errstate(divide="ignore", invalid="ignore"):
            gtot = Msf_b[f] + aoms_b[f] * np.where(mag, -sim.alpha_f[f] / (Msf * Msf), 0.0)
        # initial face magnetisation M0_f = v Ms_f / |v|, v = mean of Ms * m0
        v = [0.5 * s_down(sim.Ms_c * m0[c], f, per[f], clamp=True) for c in range(3)]
        nv = np.sqrt(dot(v, v))
        safe = np.where(mag, nv, 1.0)
        vh = [np.where(mag, v[c] / safe, 0.0) for c in range(3)]
        mb0 = [np.where(ev, Mb[f][c], 0.0) for c in range(3)]
        gtot = gtot + dot(mb0, vh)
        pr = dot(vh, mb0)
        vb = [np.where(mag, (Msf / safe) * (mb0[c] - vh[c] * pr), 0.0) for c in range(3)]
        for c in range(3):
            Ms_b += m0[c] * (0.5 * s_down_T(vb[c], f, per[f], clamp=True))
        Ms_b += 0.5 * s_down_T(np.where(mag, gtot, 0.0), f, per[f], clamp=True)
    # cells with Ms = 0 are not magnetic: the model has no derivative there
    Ms_b = np.where(np.real(sim.Ms_c) > 0, Ms_b, 0.0)
    return to_host(eps_b), to_host(Ms_b)


def loss_and_gradients(make_sim, nsteps, i0):
    """L and (dL/d eps_r, dL/d Ms) for a freshly built simulation."""
    sim = make_sim()
    M0_state = [[v.copy() for v in sim.M[f]] for f in range(3)]
    L, tape = run_with_tape(sim, nsteps, i0)
    g_eps, g_ms = reverse(sim, tape, i0, M0_state)
    return float(np.real(L)), g_eps, g_ms
