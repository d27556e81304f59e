"""FP64 reference of the coupled Maxwell-LLG time step.

TEST INFRASTRUCTURE ONLY.  This module is imported by the tests, by the
smoke check and by the CPU-baseline leg of the benchmark; the product path
(the HIP library and its binding) never calls it and shares no code with it.

Method: Yao, Jambunathan, Zeng & Nonaka, "A Massively Parallel Time-Domain
Coupled Electrodynamics-Micromagnetics Solver".
  * Sec. 2: Ampere (eq:Ampere) with J = sigma E + J_src; Faraday in magnetic
    regions with B = mu0 (H + M) (eq:Faraday2) and with mu elsewhere
    (eq:Faraday3); LLG in Gilbert form without the extra torque (eq:LLG);
    H_eff = H_EM + H0; |M| = Ms.
  * Sec. 3.1: Yee grid, normal H on faces, tangential E/J on edges, all three
    M components on every face; transverse H on a face from a four-point
    average; materials given at cell centres and averaged to edges/faces;
    M initialised at cell centres and averaged to faces.
  * Sec. 3.2: H half step, E full step, H half step; renormalisation N(M).
  * Sec. 3.2.1 Step 2 (E update with sigma, eps and J at n+1/2).
  * Sec. 3.2.2: second-order H-M sub-step: trapezoidal LLG (eq:llg_tra1-3),
    closed-form solve (eq:llg_tra4-6), H from Faraday (eq:iterate_H),
    iterated until the domain-wide max of |dM|/Ms drops below tol; faces
    with Ms = 0 take the plain Faraday update with mu.
  * Sec. 3.2.3: periodic and PEC boundaries.
  * Sec. 3.2.3 (pml=...): the open boundary, a split-field perfectly
    matched layer (Berenger) whose split parts take the macroscopic update
    and are damped before and after it (the two-step time-centred form the
    paper uses), with a graded damping rate matched for E and H.
  * Sec. 3.2 (hard_sources=...): hard sources, a field component overwritten
    with a prescribed waveform after each of its updates (E after Step 2,
    H after each Faraday half step, on faces that do not evolve M).
  * Sec. 3.2.1 Steps 1 and 3 (scheme=1): the first-order scheme, an
    explicit step of the LLG in Landau-Lifshitz form (eq:LLG_scalar, with
    gamma_L = gamma / (1 + alpha^2)) then N(M) and eq:H_update /
    eq:H_update2; read with dt/2 for each half step.

Readings where the paper is silent or ambiguous (each one is listed in the
design notes): the residual is the max over magnetic faces and components of
|M^r_c - M^{r-1}_c| / Ms_f with a strict "<" test; the iteration is Jacobi
(every face lags its neighbours by one iterate, H^{r=0} = H^s everywhere and
non-magnetic faces hold their one-shot Faraday value from r = 1 on); the
closed form is used with signed gamma (kappa = mu0*gamma*dt/4), identical to
the printed |gamma| form for gamma < 0; edges average the 4 adjacent cells
and faces the 2 adjacent cells (clamped at PEC walls); alpha and gamma on a
face average over its magnetic neighbour cells only; magnetic faces lying on
a PEC wall are not evolved; the soft current enters Step 2 at t^{n+1/2};
a hard source holds on the bounding box of its profile's nonzero interior
entries and takes g(t^{n+1}) after Step 2 (E), g(t^{n+1/2}) after Step 1 and
g(t^{n+1}) after Step 3 (H), an H source replacing the non-magnetic Faraday
value before the iterations read it.

Arrays are indexed [i, j, k] internally; inputs and outputs use the host
layout of the library (x fastest, numpy shape (nz', ny', nx')).
"""
from __future__ import annotations

import math

import numpy as np

MU0 = 1.25663706212e-6
EPS0 = 8.8541878128e-12


class NonConvergence(RuntimeError):
    pass


# --------------------------------------------------------------------------
# staggered index helpers (Sec. 3.1)
# --------------------------------------------------------------------------

def _sl(ax, s):
    idx = [slice(None)] * 3
    idx[ax] = s
    return tuple(idx)


def d_up(a, ax, per):
    """Forward difference nodes -> cells along `ax`: a[m+1] - a[m]."""
    if per:
        return np.roll(a, -1, axis=ax) - a
    return a[_sl(ax, slice(1, None))] - a[_sl(ax, slice(0, -1))]


def d_down(a, ax, per):
    """Backward difference cells -> nodes along `ax`: a[m] - a[m-1].
    On PEC axes the two wall nodes get 0 (never used)."""
    if per:
        return a - np.roll(a, 1, axis=ax)
    shp = list(a.shape)
    shp[ax] += 1
    out = np.zeros(shp, dtype=np.result_type(a, np.float64))
    out[_sl(ax, slice(1, -1))] = a[_sl(ax, slice(1, None))] - a[_sl(ax, slice(0, -1))]
    return out


def s_down(a, ax, per, clamp=False):
    """Pair sum cells -> nodes along `ax`: a[m-1] + a[m].  On PEC axes the wall
    nodes get 0, or twice the inside value with clamp=True."""
    if per:
        return np.roll(a, 1, axis=ax) + a
    shp = list(a.shape)
    shp[ax] += 1
    out = np.zeros(shp, dtype=np.result_type(a, np.float64))
    out[_sl(ax, slice(1, -1))] = a[_sl(ax, slice(0, -1))] + a[_sl(ax, slice(1, None))]
    if clamp:
        out[_sl(ax, 0)] = 2.0 * a[_sl(ax, 0)]
        out[_sl(ax, -1)] = 2.0 * a[_sl(ax, -1)]
    return out


def s_up(a, ax, per):
    """Pair sum nodes -> cells along `ax`: a[m] + a[m+1]."""
    if per:
        return a + np.roll(a, -1, axis=ax)
    return a[_sl(ax, slice(0, -1))] + a[_sl(ax, slice(1, None))]


def to_ijk(a, dtype=np.float64):
    return np.asarray(a, dtype=dtype).transpose(2, 1, 0)


def to_host(a):
    return np.ascontiguousarray(a.transpose(2, 1, 0))


def cross(a, b):
    return [a[1] * b[2] - a[2] * b[1],
            a[2] * b[0] - a[0] * b[2],
            a[0] * b[1] - a[1] * b[0]]


def dot(a, b):
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]


def vacus_solve(a, b):
    """Closed-form solution x of x + a x x = b (eq:llg_tra4):
    x = (b + (a.b) a - a x b) / (1 + |a|^2)."""
    ab = dot(a, b)
    axb = cross(a, b)
    den = 1.0 + dot(a, a)
    return [(b[c] + ab * a[c] - axb[c]) / den for c in range(3)]


def renormalise(m, Ms):
    """N(M) = M * (Ms / |M|)  (Sec. 3.2).  |M| is written as sqrt(M.M) (no
    conjugation), so the function is analytic and complex-step derivatives
    pass through it."""
    nrm = np.sqrt(dot(m, m))
    pos = np.real(nrm) > 0
    with np.errstate(invalid="ignore", divide="ignore"):
        s = np.where(pos, Ms / np.where(pos, nrm, 1.0), 0.0)
    return [m[c] * s for c in range(3)]


def waveform(t, f0, Tp, t0):
    """Gaussian-modulated sinusoid of the pulse equation in Sec. 5.2.1.  The
    square of t - t0 is the rounded product (a power through libm pow is not
    always correctly rounded)."""
    d = t - t0
    return math.exp(-(d * d) / (2.0 * Tp * Tp)) * math.cos(2.0 * math.pi * f0 * t)


# --------------------------------------------------------------------------
# the simulation
# --------------------------------------------------------------------------

class Simulation:
    """Second-order coupled scheme (Sec. 3.2.2) on a uniform Yee grid.

    Parameters mirror the library's mm_init: grid size `n`, spacings `d`,
    time step `dt`, cell-centred material maps (host layout, None -> default),
    uniform bias `H0`, optional soft source (comp, profile, f0, Tp, t0),
    per-axis periodic flags, sub-step tolerance / iteration cap, and
    `fixed_iter` (> 0: exactly that many iterations per sub-step), and
    `scheme` (2: the iterative second-order sub-step; 1: the first-order
    scheme of Sec. 3.2.1, one explicit update per sub-step), and `pml`:
    None, or (cells, R0, order) with cells = (x_lo, x_hi, y_lo, y_hi, z_lo,
    z_hi) layer thicknesses on PEC axes, the normal-incidence reflection
    target R0 of the grading and its polynomial order.
    `hard_sources`: a list of (field, profile, f0, Tp, t0) hard sources
    (field 0-2: Ex, Ey, Ez; 3-5: Hx, Hy, Hz; see add_hard_source).
    `dtype` complex128 runs the same arithmetic on complex numbers (all
    decisions use real parts), for complex-step derivatives in the tests.
    """

    def __init__(self, n, d, dt, eps_r=None, sigma=None, mu_r=None, Ms=None,
                 alpha=None, gamma=None, m0_dir=None, H0=(0.0, 0.0, 0.0),
                 source=None, periodic=(False, False, False), tol=1e-10,
                 max_iter=100, fixed_iter=0, raise_on_noconv=False, dtype=np.float64, scheme=2,
                 pml=None, hard_sources=()):
        self.dtype = np.dtype(dtype)
        assert scheme in (1, 2)
        self.scheme = int(scheme)
        self.n = tuple(int(v) for v in n)
        self.d = tuple(float(v) for v in d)
        self.dt = float(dt)
        self.per = tuple(bool(p) for p in periodic)
        self.tol = float(tol)
        self.max_iter = int(max_iter)
        self.fixed_iter = int(fixed_iter)
        self.raise_on_noconv = raise_on_noconv
        self.H0 = tuple(float(v) for v in H0)
        nx, ny, nz = self.n
        shp = (nx, ny, nz)

        def cmap(a, default):
            if a is None:
                return np.full(shp, float(default), dtype=self.dtype)
            a = to_ijk(a, self.dtype)
            assert a.shape == shp
            return a

        self.eps_r = cmap(eps_r, 1.0)
        self.sigma = cmap(sigma, 0.0)
        self.mu_r = cmap(mu_r, 1.0)
        self.Ms_c = cmap(Ms, 0.0)
        self.alpha_c = cmap(alpha, 0.0)
        self.gamma_c = cmap(gamma, -1.759e11)
        if m0_dir is None:
            m0 = [np.zeros(shp), np.zeros(shp), np.ones(shp)]
        else:
            m0 = [to_ijk(np.asarray(m0_dir)[c]) for c in range(3)]
        self.m0_dir = m0
        self._prepare(m0)
        self._prepare_pml(pml)

        # fields on the Yee grid (Sec. 3.1)
        self.E = [np.zeros(self.edge_shape(c), dtype=self.dtype) for c in range(3)]
        self.H = [np.zeros(self.face_shape(c), dtype=self.dtype) for c in range(3)]
        self.src = None
        if source is not None:
            comp, prof, f0, Tp, t0 = source
            prof = to_ijk(prof, self.dtype)
            assert prof.shape == self.edge_shape(comp)
            self.src = (int(comp), prof * self.e_interior[comp], float(f0), float(Tp), float(t0))
        self.hard = []           # (field, support mask, profile, f0, Tp, t0)
        for hs in hard_sources:
            self.add_hard_source(*hs)
        self.step_count = 0
        self._t_sub = 0.0        # time level the current sub-step ends at (hard H sources)
        self._E_for_C = None     # the E whose curl the current sub-step uses (for the PML split)
        self.iters = []          # iterations used by every sub-step, in order
        self.noconv = False
        self.nonfinite = False
        self.probes = []

    # ---- extents ---------------------------------------------------------
    def nodes(self, ax):
        return self.n[ax] if self.per[ax] else self.n[ax] + 1

    def edge_shape(self, c):
        return tuple(self.n[a] if a == c else self.nodes(a) for a in range(3))

    def face_shape(self, c):
        return tuple(self.nodes(a) if a == c else self.n[a] for a in range(3))

    def _node_interior(self, ax, length):
        m = np.ones(length, dtype=bool)
        if not self.per[ax]:
            m[0] = False
            m[-1] = False
        return m

    # ---- hard sources (Sec. 3.2) ------------------------------------------
    def add_hard_source(self, field, profile, f0, Tp, t0):
        """Hard source on component `field` (0-2: Ex, Ey, Ez; 3-5: Hx, Hy, Hz):
        after every update of that component, the entries inside the bounding
        box of the nonzero interior entries of `profile` (host layout, the
        component's staggered extent) are set to profile * g(t), g the pulse
        of Sec. 5.2.1.  Interior means not pinned by a PEC wall; pinned
        entries inside the box stay zero.  H sources may not hold evolving
        magnetic faces, and no source may reach into an open-boundary layer."""
        field = int(field)
        assert 0 <= field < 6
        c = field % 3
        is_e = field < 3
        shp = self.edge_shape(c) if is_e else self.face_shape(c)
        prof = to_ijk(profile, self.dtype)
        assert prof.shape == shp
        interior = self.e_interior[c] if is_e else self.h_interior[c]
        nz = np.argwhere((prof != 0) & interior)
        if len(nz) == 0:
            raise ValueError("a hard source needs a nonzero interior profile entry")
        lo, hi = nz.min(axis=0), nz.max(axis=0) + 1
        box = np.zeros(shp, dtype=bool)
        box[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] = True
        mask = box & interior
        if not is_e and np.any(mask & self.evolve[c]):
            raise ValueError("a hard H source may not hold evolving magnetic faces")
        if self.pml_cells is not None:
            for a in range(3):
                lo_t, hi_t = self.pml_cells[2 * a], self.pml_cells[2 * a + 1]
                # positions along axis a in cells: cell centres where the
                # component is cell-centred, nodes elsewhere
                cell_axis = (a == c) if is_e else (a != c)
                pos = np.arange(shp[a]) + (0.5 if cell_axis else 0.0)
                bad = ((lo_t > 0) & (pos < lo_t)) | ((hi_t > 0) & (pos > self.n[a] - hi_t))
                if np.any(bad[lo[a]:hi[a]]):
                    raise ValueError("a hard source may not reach into an open-boundary layer")
        self.hard.append((field, mask, prof, float(f0), float(Tp), float(t0)))

    def add_surface_current(self, axis, side, comp, profile, f0, Tp, t0):
        """Surface current J_s (A/m) along `comp` on the PEC wall normal to
        `axis` at its low (side 0) or high (side 1) end (Sec. 5.2.1): the
        boundary condition n x H = J_s, n the unit normal into the domain,
        fixes the tangential H at the wall to J_s x n.  It is held, as a hard
        source, on the tangential-H faces half a cell inside the wall.
        `profile`: host layout on component `comp`'s edge array; the entries
        on the wall plane are used."""
        axis, side, comp = int(axis), int(side), int(comp)
        assert axis != comp and not self.per[axis] and side in (0, 1)
        h = 3 - axis - comp
        # e_comp x n, n = -e_axis at the high wall, +e_axis at the low wall
        perm = {(0, 1, 2): 1, (1, 2, 0): 1, (2, 0, 1): 1, (0, 2, 1): -1, (2, 1, 0): -1, (1, 0, 2): -1}
        sign = perm[(comp, axis, h)] * (1 if side == 0 else -1)
        J = to_ijk(profile, self.dtype)
        assert J.shape == self.edge_shape(comp)
        Hp = np.zeros(self.face_shape(h), dtype=self.dtype)
        wall_node = 0 if side == 0 else self.n[axis]
        first_cell = 0 if side == 0 else self.n[axis] - 1
        src = [slice(None)] * 3
        dst = [slice(None)] * 3
        src[axis] = wall_node
        dst[axis] = first_cell
        Hp[tuple(dst)] = sign * J[tuple(src)]
        self.add_hard_source(3 + h, to_host(Hp), f0, Tp, t0)

    def _apply_hard(self, arr, field, t):
        for fid, mask, prof, f0, Tp, t0 in self.hard:
            if fid == field:
                arr = np.where(mask, prof * waveform(t, f0, Tp, t0), arr)
        return arr

    # ---- init: materials to edges and faces (Sec. 3.1) -------------------
    def _prepare(self, m0):
        per = self.per
        dt = self.dt
        # interior masks: tangential E and normal H on PEC walls stay zero
        self.e_interior = []
        for c in range(3):
            shp = self.edge_shape(c)
            m = np.ones(shp, dtype=bool)
            for a in range(3):
                if a != c:
                    line = self._node_interior(a, shp[a])
                    m &= line.reshape([-1 if b == a else 1 for b in range(3)])
            self.e_interior.append(m)
        self.h_interior = []
        for f in range(3):
            shp = self.face_shape(f)
            line = self._node_interior(f, shp[f])
            self.h_interior.append(np.broadcast_to(
                line.reshape([-1 if b == f else 1 for b in range(3)]), shp).copy())

        # edges: eps and sigma as the mean of the 4 adjacent cells
        self.ca, self.cb = [], []
        for c in range(3):
            t1, t2 = [a for a in range(3) if a != c]
            eps_e = EPS0 * (0.25 * s_down(s_down(self.eps_r, t1, per[t1]), t2, per[t2]))
            sig_e = 0.25 * s_down(s_down(self.sigma, t1, per[t1]), t2, per[t2])
            with np.errstate(divide="ignore", invalid="ignore"):
                den = eps_e / dt + sig_e / 2.0
                ca = (eps_e / dt - sig_e / 2.0) / den
                cb = 1.0 / den
            im = self.e_interior[c]
            self.ca.append(np.where(im, ca, 0.0))
            self.cb.append(np.where(im, cb, 0.0))

        # faces: Ms as the mean of the 2 adjacent cells, mu likewise; alpha and
        # gamma over the magnetic neighbour cells only; M0 as the mean of the
        # cell-centred M0 = Ms * m0_dir, renormalised to Ms_f
        mag_c = (np.real(self.Ms_c) > 0).astype(np.float64)
        self.Ms_f, self.mu_f, self.alpha_f, self.gamma_f = [], [], [], []
        self.mag, self.evolve, self.M = [], [], []
        for f in range(3):
            Msf = 0.5 * s_down(self.Ms_c, f, per[f], clamp=True)
            muf = MU0 * (0.5 * s_down(self.mu_r, f, per[f], clamp=True))
            cnt = s_down(mag_c, f, per[f], clamp=True)
            with np.errstate(divide="ignore", invalid="ignore"):
                af = np.where(cnt > 0, s_down(self.alpha_c * mag_c, f, per[f], clamp=True)
                              / np.where(cnt > 0, cnt, 1.0), 0.0)
                gf = np.where(cnt > 0, s_down(self.gamma_c * mag_c, f, per[f], clamp=True)
                              / np.where(cnt > 0, cnt, 1.0), 0.0)
            mag = np.real(Msf) > 0
            Mf = [0.5 * s_down(self.Ms_c * m0[c], f, per[f], clamp=True) for c in range(3)]
            nrm = np.sqrt(dot(Mf, Mf))
            if np.any(mag & (np.abs(nrm) == 0)):
                raise ValueError("initial magnetisation averages to zero on a magnetic face")
            Mf = [np.where(mag, v, 0.0) for v in renormalise(Mf, Msf)]
            self.Ms_f.append(Msf)
            self.mu_f.append(muf)
            self.alpha_f.append(af)
            self.gamma_f.append(gf)
            self.mag.append(mag)
            self.evolve.append(mag & self.h_interior[f])
            self.M.append(Mf)

    # ---- field access ------------------------------------------------------
    def set_fields(self, E=None, H=None):
        """Set E and/or H from host-layout arrays; PEC-wall entries are zeroed."""
        if E is not None:
            for c in range(3):
                self.E[c] = np.where(self.e_interior[c], to_ijk(E[c], self.dtype), 0.0)
        if H is not None:
            for f in range(3):
                self.H[f] = np.where(self.h_interior[f], to_ijk(H[f], self.dtype), 0.0)

    def field(self, name):
        """Host-layout copy of a field: Ex..Hz, M<family><comp> (e.g. 'Myz'), Bx..Bz."""
        names = {"Ex": ("E", 0), "Ey": ("E", 1), "Ez": ("E", 2),
                 "Hx": ("H", 0), "Hy": ("H", 1), "Hz": ("H", 2)}
        if name in names:
            k, c = names[name]
            return to_host((self.E if k == "E" else self.H)[c])
        if name[0] == "M":
            f = "xyz".index(name[1])
            c = "xyz".index(name[2])
            return to_host(self.M[f][c])
        if name[0] == "B":
            f = "xyz".index(name[1])
            return to_host(self.B_normal(f))
        raise KeyError(name)

    def B_normal(self, f):
        """Normal B on the faces of family f: mu0 (H + M_n) on magnetic faces,
        mu_f H elsewhere (Sec. 2)."""
        return np.where(self.mag[f], MU0 * (self.H[f] + self.M[f][f]), self.mu_f[f] * self.H[f])

    # ---- discrete operators (Sec. 3.1) ------------------------------------
    def curl_E(self, E):
        """Curl of E at the faces (normal components)."""
        dx, dy, dz = self.d
        px, py, pz = self.per
        cx = d_up(E[2], 1, py) / dy - d_up(E[1], 2, pz) / dz
        cy = d_up(E[0], 2, pz) / dz - d_up(E[2], 0, px) / dx
        cz = d_up(E[1], 0, px) / dx - d_up(E[0], 1, py) / dy
        return [cx, cy, cz]

    def curl_H(self, H):
        """Curl of H at the edges (tangential components)."""
        dx, dy, dz = self.d
        px, py, pz = self.per
        cx = d_down(H[2], 1, py) / dy - d_down(H[1], 2, pz) / dz
        cy = d_down(H[0], 2, pz) / dz - d_down(H[2], 0, px) / dx
        cz = d_down(H[1], 0, px) / dx - d_down(H[0], 1, py) / dy
        return [cx, cy, cz]

    def transverse(self, H, f, c):
        """Component c of H at the faces of family f (c != f): mean of the four
        nearest values, paired along f first and then along c."""
        return 0.25 * s_up(s_down(H[c], f, self.per[f]), c, self.per[c])

    def H_eff(self, H, f):
        """H_eff = H_EM + H0 on the faces of family f (Sec. 2)."""
        out = []
        for c in range(3):
            hc = H[f] if c == f else self.transverse(H, f, c)
            out.append(hc + self.H0[c])
        return out

    # ---- open boundary: split-field PML (Sec. 3.2.3) ------------------------
    # Component c of E (or H) splits into the part driven by the positive
    # term of its curl, P (derivative along axis p), and the rest (axis m):
    #   E: x: p = y, m = z;  y: p = z, m = x;  z: p = x, m = y  (same for H).
    # P is stored; the full field stays in E / H.  In the layer each part takes
    # the macroscopic update and is multiplied by exp(-kappa dt/2) before and
    # after it (E, a full step) or by exp(-kappa dt/4) (H, each half step),
    # kappa(depth) = kappa_max (depth / L)^order along the part's axis,
    # kappa_max = -(order + 1) c ln(R0) / (2 L).  kappa is a rate (sigma/eps
    # for E, sigma*/mu for H), so the layer is matched in any non-magnetic
    # material.  Entries with kappa = 0 for both parts take the plain update.
    PM = ((1, 2), (2, 0), (0, 1))

    def _prepare_pml(self, pml):
        self.pml = None
        self.pml_cells = None
        if pml is None:
            return
        cells, R0, order = pml
        cells = tuple(int(v) for v in cells)
        if not any(cells):
            return
        self.pml_cells = cells
        c0 = 299792458.0
        node_k, cent_k = [], []
        for a in range(3):
            lo, hi = cells[2 * a], cells[2 * a + 1]
            n = self.n[a]
            if (lo or hi) and self.per[a]:
                raise ValueError("a PML needs a PEC (non-periodic) axis")
            xn = np.arange(n + 1, dtype=np.float64)     # node positions (cells)
            xc = np.arange(n, dtype=np.float64) + 0.5    # cell-centre positions
            kn, kc = np.zeros(n + 1), np.zeros(n)
            for thick, depth_n, depth_c in ((lo, lo - xn, lo - xc), (hi, xn - (n - hi), xc - (n - hi))):
                if thick <= 0:
                    continue
                L = thick * self.d[a]
                kmax = -(order + 1) * c0 * math.log(R0) / (2.0 * L)
                kn = kn + np.where(depth_n > 0, kmax * (np.clip(depth_n, 0, None) / thick) ** order, 0.0)
                kc = kc + np.where(depth_c > 0, kmax * (np.clip(depth_c, 0, None) / thick) ** order, 0.0)
            node_k.append(kn if not self.per[a] else kn[:n])
            cent_k.append(kc)
        dt = self.dt

        def bcast(v, ax):
            return v.reshape([-1 if b == ax else 1 for b in range(3)])
        # E_c lives on nodes along its transverse axes; H_f on cell centres
        self.pml = {"dE": [], "dH": [], "onE": [], "onH": [], "PE": [], "PH": []}
        for c in range(3):
            p, m = self.PM[c]
            kp = np.broadcast_to(bcast(node_k[p], p), self.edge_shape(c))
            km = np.broadcast_to(bcast(node_k[m], m), self.edge_shape(c))
            self.pml["dE"].append((np.exp(-kp * dt / 2.0), np.exp(-km * dt / 2.0)))
            self.pml["onE"].append((kp > 0) | (km > 0))
            self.pml["PE"].append(np.zeros(self.edge_shape(c), dtype=self.dtype))
            kp = np.broadcast_to(bcast(cent_k[p], p), self.face_shape(c))
            km = np.broadcast_to(bcast(cent_k[m], m), self.face_shape(c))
            self.pml["dH"].append((np.exp(-kp * dt / 4.0), np.exp(-km * dt / 4.0)))
            on = (kp > 0) | (km > 0)
            self.pml["onH"].append(on)
            self.pml["PH"].append(np.zeros(self.face_shape(c), dtype=self.dtype))
            if np.any(on & self.mag[c]):
                raise ValueError("magnetic faces inside the PML are not supported (Sec. 3.2.3)")

    def _curl_terms_H(self, H, c):
        """The two terms of (curl H)_c at the edges: T_p - T_m."""
        p, m = self.PM[c]
        return (d_down(H[3 - c - p], p, self.per[p]) / self.d[p],
                d_down(H[3 - c - m], m, self.per[m]) / self.d[m])

    def _curl_terms_E(self, E, f):
        """The two terms of (curl E)_f at the faces: T_p - T_m."""
        p, m = self.PM[f]
        return (d_up(E[3 - f - p], p, self.per[p]) / self.d[p],
                d_up(E[3 - f - m], m, self.per[m]) / self.d[m])

    def _pml_h(self, Hs, Hplain, f, h, E):
        """H of family f after a half step with the layer: the plain update
        outside it, the split update inside."""
        if self.pml is None:
            return Hplain
        assert E is not None, "with a PML, sub-steps run through step()"
        on = self.pml["onH"][f] & self.h_interior[f]
        if not on.any():
            return Hplain
        dp, dm = self.pml["dH"][f]
        Tp, Tm = self._curl_terms_E(E, f)
        P = self.pml["PH"][f]
        Mpart = Hs[f] - P
        cf = h / self.mu_f[f]
        Pn = dp * (dp * P - cf * Tp)
        Mn = dm * (dm * Mpart + cf * Tm)
        self.pml["PH"][f] = np.where(on, Pn, P)
        return np.where(on, Pn + Mn, Hplain)

    # ---- Step 1 / Step 3 of the first-order scheme (Sec. 3.2.1) -----------
    def hm_substep_first_order(self, C):
        """M^{new} = N(M + (dt/2) [mu0 gamma_L M x H_eff + (alpha mu0 gamma_L / Ms)
        M x (M x H_eff)]) with H_eff from the current H, then
        H^{new} = H + M_n - M^{new}_n - (dt / 2 mu0) curl E; faces with Ms = 0
        take the plain Faraday update with mu."""
        h = 0.5 * self.dt
        Hs = [a.copy() for a in self.H]
        Mn_all, Hn_all = [], []
        for f in range(3):
            ev = self.evolve[f]
            M = self.M[f]
            He = self.H_eff(Hs, f)
            gL = self.gamma_f[f] / (1.0 + self.alpha_f[f] ** 2)
            k1 = MU0 * gL
            with np.errstate(divide="ignore", invalid="ignore"):
                k2 = np.where(self.mag[f], self.alpha_f[f] * MU0 * gL / np.where(self.mag[f], self.Ms_f[f], 1.0), 0.0)
            mxh = cross(M, He)
            mxmxh = cross(M, mxh)
            Mt = [M[c] + h * (k1 * mxh[c] + k2 * mxmxh[c]) for c in range(3)]
            Mn = renormalise(Mt, self.Ms_f[f])
            Mn = [np.where(ev, Mn[c], M[c]) for c in range(3)]
            q = Hs[f] + M[f] - (h / MU0) * C[f]
            H_nonmag = np.where(self.h_interior[f], Hs[f] - (h / self.mu_f[f]) * C[f], Hs[f])
            H_nonmag = self._pml_h(Hs, H_nonmag, f, h, self._E_for_C)
            H_nonmag = self._apply_hard(H_nonmag, 3 + f, self._t_sub)
            Hn_all.append(np.where(ev, q - Mn[f], H_nonmag))
            Mn_all.append(Mn)
        self.H = Hn_all
        self.M = Mn_all
        self.iters.append(1)

    # ---- Step 1 / Step 3: the iterative H-M sub-step (Sec. 3.2.2) ----------
    def hm_substep(self, C, trace=None):
        """One H-M sub-step from the current (H, M) with face curl C.  With a
        dict `trace`, records its inputs and the iterate H^{(r-1)} read by each
        iteration r (what the reverse sweep replays)."""
        if self.scheme == 1:
            assert trace is None, "the reverse sweep covers the second-order scheme only"
            return self.hm_substep_first_order(C)
        h = 0.5 * self.dt
        Hs = [a.copy() for a in self.H]
        Ms0 = [[v.copy() for v in self.M[f]] for f in range(3)]
        H_nonmag, q, b, dvec, kappa = [], [], [], [], []
        for f in range(3):
            # faces with Ms = 0: Faraday with the local mu (eq:Faraday3)
            H_nonmag.append(self._apply_hard(
                self._pml_h(Hs, np.where(self.h_interior[f], Hs[f] - (h / self.mu_f[f]) * C[f], Hs[f]),
                            f, h, self._E_for_C), 3 + f, self._t_sub))
            # iteration-invariant parts of eq:llg_tra5/6 and eq:iterate_H
            kap = MU0 * self.gamma_f[f] * self.dt / 4.0
            He = self.H_eff(Hs, f)
            mxh = cross(Ms0[f], He)
            b.append([Ms0[f][c] + kap * mxh[c] for c in range(3)])
            with np.errstate(divide="ignore", invalid="ignore"):
                aoms = np.where(self.mag[f], self.alpha_f[f] / np.where(self.mag[f], self.Ms_f[f], 1.0), 0.0)
            dvec.append([aoms * Ms0[f][c] for c in range(3)])
            kappa.append(kap)
            q.append(Hs[f] + Ms0[f][f] - (h / MU0) * C[f])
        Hprev, Mprev = Hs, Ms0
        if trace is not None:
            trace["Hs"] = [a.copy() for a in Hs]
            trace["Ms0"] = [[v.copy() for v in Ms0[f]] for f in range(3)]
            trace["C"] = [a.copy() for a in C]
            trace["Hprevs"] = []
        r = 0
        limit = self.fixed_iter if self.fixed_iter > 0 else self.max_iter
        converged = False
        while r < limit:
            r += 1
            if trace is not None:
                trace["Hprevs"].append(Hprev)
            Hr, Mr = [], []
            parts = [0.0]
            for f in range(3):
                ev = self.evolve[f]
                He = self.H_eff(Hprev, f)
                a = [kappa[f] * He[c] - dvec[f][c] for c in range(3)]
                Mt = vacus_solve(a, b[f])
                Mn = renormalise(Mt, self.Ms_f[f])
                Mn = [np.where(ev, Mn[c], Mprev[f][c]) for c in range(3)]
                Hn = np.where(ev, q[f] - Mn[f], H_nonmag[f])
                if ev.any():
                    with np.errstate(invalid="ignore"):
                        for c in range(3):
                            parts.append(float(np.max(np.abs(Mn[c] - Mprev[f][c])[ev]
                                                      / np.abs(self.Ms_f[f][ev]))))
                Hr.append(Hn)
                Mr.append(Mn)
            # np.max propagates NaN, so a non-finite iterate shows up here
            res = float(np.max(np.array(parts)))
            Hprev, Mprev = Hr, Mr
            if not math.isfinite(res):
                self.nonfinite = True
                break
            if self.fixed_iter <= 0 and res < self.tol:
                converged = True
                break
        if self.fixed_iter <= 0 and not converged:
            self.noconv = True
            if self.raise_on_noconv:
                raise NonConvergence(f"sub-step did not converge in {self.max_iter} iterations")
        self.H = Hprev
        self.M = Mprev
        self.iters.append(r)

    # ---- Step 2: E update (Sec. 3.2.1) -------------------------------------
    def e_update(self):
        CH = self.curl_H(self.H)
        t_half = (self.step_count + 0.5) * self.dt
        for c in range(3):
            rhs = CH[c]
            if self.src is not None and self.src[0] == c:
                comp, prof, f0, Tp_, t0 = self.src
                rhs = rhs - prof * waveform(t_half, f0, Tp_, t0)
            Eplain = np.where(self.e_interior[c], self.ca[c] * self.E[c] + self.cb[c] * rhs, 0.0)
            if self.pml is not None and self.pml["onE"][c].any():
                on = self.pml["onE"][c] & self.e_interior[c]
                dp, dm = self.pml["dE"][c]
                Tp, Tm = self._curl_terms_H(self.H, c)
                rp = Tp
                if self.src is not None and self.src[0] == c:
                    rp = Tp - prof * waveform(t_half, f0, Tp_, t0)
                P = self.pml["PE"][c]
                Mpart = self.E[c] - P
                Pn = dp * (self.ca[c] * (dp * P) + self.cb[c] * rp)
                Mn = dm * (self.ca[c] * (dm * Mpart) - self.cb[c] * Tm)
                self.pml["PE"][c] = np.where(on, Pn, P)
                Eplain = np.where(on, Pn + Mn, Eplain)
            self.E[c] = self._apply_hard(Eplain, c, (self.step_count + 1.0) * self.dt)

    # ---- one full step n -> n+1 --------------------------------------------
    def step(self, nsteps=1, tape=None):
        """Advance `nsteps` steps.  With a list `tape`, appends per step the
        states and sub-step traces the reverse sweep needs."""
        for _ in range(nsteps):
            rec = None
            if tape is not None:
                rec = {"n": self.step_count, "E0": [a.copy() for a in self.E], "tr1": {}, "tr3": {}}
            if rec is not None and self.hard:
                raise ValueError("the reverse sweep does not cover hard sources")
            self._E_for_C = self.E
            self._t_sub = (self.step_count + 0.5) * self.dt
            self.hm_substep(self.curl_E(self.E), trace=None if rec is None else rec["tr1"])  # Step 1
            self.e_update()                                                                  # Step 2
            self._E_for_C = self.E
            self._t_sub = (self.step_count + 1.0) * self.dt
            self.hm_substep(self.curl_E(self.E), trace=None if rec is None else rec["tr3"])  # Step 3
            self.step_count += 1
            if rec is not None:
                rec["E1"] = [a.copy() for a in self.E]
                rec["H1"] = [a.copy() for a in self.H]
                tape.append(rec)
            self._record_probes()

    # ---- probes -------------------------------------------------------------
    def add_probe(self, kind, field=0, i=0, j=0, k=0):
        """kind 0: sample of field id `field` at staggered index (i, j, k) every
        step; kind 1: Poynting flux P through the node plane x = i every step."""
        self.probes.append({"kind": int(kind), "field": int(field), "i": int(i),
                            "j": int(j), "k": int(k), "series": []})
        return len(self.probes) - 1

    def flux_x(self, i0):
        """P = dy dz sum_{j,k} [Ey Hz - Ez Hy] on the node plane x = i0, with
        H_z, H_y averaged to the plane from the two adjacent cells."""
        dx, dy, dz = self.d
        im1 = (i0 - 1) % self.n[0]
        hz = 0.5 * (self.H[2][im1] + self.H[2][i0 % self.n[0]])
        hy = 0.5 * (self.H[1][im1] + self.H[1][i0 % self.n[0]])
        s = np.sum(self.E[1][i0] * hz) - np.sum(self.E[2][i0] * hy)
        return dy * dz * s

    def point_value(self, field, i, j, k):
        if field < 3:
            return self.E[field][i, j, k]
        if field < 6:
            return self.H[field - 3][i, j, k]
        if field < 15:
            f, c = divmod(field - 6, 3)
            return self.M[f][c][i, j, k]
        return self.B_normal(field - 15)[i, j, k]

    def _record_probes(self):
        for p in self.probes:
            if p["kind"] == 1:
                p["series"].append(self.flux_x(p["i"]))
            else:
                p["series"].append(self.point_value(p["field"], p["i"], p["j"], p["k"]))

    def probe_series(self, pid):
        return np.array(self.probes[pid]["series"], dtype=self.dtype)

    def probe_integral(self, pid):
        """S = sum_n dt * P^n, accumulated in step order."""
        s = 0.0
        for v in self.probes[pid]["series"]:
            s += self.dt * v
        return s


def from_config(cfg, fixed_iter=0, with_probes=True, **kw):
    """Build a Simulation from a workloads.Config."""
    src = None
    if cfg.source is not None:
        s = cfg.source
        src = (s.comp, s.profile, s.f0, s.Tp, s.t0)
    hard = [(h.field, h.profile, h.f0, h.Tp, h.t0) for h in cfg.hard_sources]
    sim = Simulation(cfg.n, cfg.d, cfg.dt, eps_r=cfg.eps_r, sigma=cfg.sigma,
                     mu_r=cfg.mu_r, Ms=cfg.Ms, alpha=cfg.alpha, gamma=cfg.gamma,
                     m0_dir=cfg.m0_dir, H0=cfg.H0, source=src, periodic=cfg.periodic,
                     tol=cfg.tol, max_iter=cfg.max_iter, fixed_iter=fixed_iter,
                     **({"pml": cfg.pml} if cfg.pml is not None else {}),
                     **({"hard_sources": hard} if hard else {}), **kw)
    for sc in cfg.surface_currents:
        sim.add_surface_current(sc.axis, sc.side, sc.comp, sc.profile, sc.f0, sc.Tp, sc.t0)
    if cfg.E_init is not None or cfg.H_init is not None:
        sim.set_fields(cfg.E_init, cfg.H_init)
    if with_probes:
        for p in cfg.probes:
            sim.add_probe(p.kind, p.field, p.i, p.j, p.k)
    return sim
