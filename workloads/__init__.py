"""Seeded synthetic inputs for the coupled Maxwell-LLG step.

This module is the only code shared by the FP64 oracle and the HIP path: it
builds cell-centred material maps, source profiles and probe lists, and holds
none of the method's arithmetic (no averaging to edges or faces, no update
formulas, no waveform evaluation).  Every array uses the library's host
layout: C-contiguous float64, x fastest, i.e. numpy shape (nz, ny, nx) for a
cell map and the staggered extent for an edge profile.

Geometry follows the paper's validation problems (Sec. 5): PEC-walled
waveguides with a thin ferrite (YIG-like) slab, a bias field along the slab
and a Gaussian-modulated sinusoidal current (Sec. 5.2.1, the pulse equation),
scaled to micrometre cells.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# Physical constants shared by the configuration recipes only (the time-step
# convention and the bias field in A/m).  Each implementation carries its own
# copy for its arithmetic.
C0 = 299792458.0
MU0 = 1.25663706212e-6
GAMMA_E = -1.759e11          # gyromagnetic ratio of the electron, rad/(s*T), Sec. 2


def cfl_dt(cfl: float, dx: float, dy: float, dz: float) -> float:
    """Time step for a Courant number `cfl` based on the vacuum light speed.

    Convention read from Sec. 5.1 / 5.2.1: dt = CFL / (c * sqrt(1/dx^2 + 1/dy^2 + 1/dz^2)).
    """
    return cfl / (C0 * math.sqrt(1.0 / dx**2 + 1.0 / dy**2 + 1.0 / dz**2))


@dataclass
class Source:
    comp: int                    # 0: Jx, 1: Jy, 2: Jz
    profile: np.ndarray          # J0 * p on that component's edge array (A/m^2)
    f0: float
    Tp: float
    t0: float


@dataclass
class HardSource:
    field: int                   # 0-2: Ex, Ey, Ez; 3-5: Hx, Hy, Hz
    profile: np.ndarray          # amplitude (V/m or A/m) on that component's array
    f0: float
    Tp: float
    t0: float


@dataclass
class SurfaceCurrent:
    axis: int                    # normal of the PEC wall
    side: int                    # 0: low end, 1: high end of that axis
    comp: int                    # direction of J_s
    profile: np.ndarray          # J_s (A/m) on component comp's edge array (wall plane used)
    f0: float
    Tp: float
    t0: float


@dataclass
class Probe:
    kind: int                    # 0: point sample, 1: x-plane Poynting flux
    field: int = 0               # see FIELD_NAMES
    i: int = 0
    j: int = 0
    k: int = 0


FIELD_NAMES = ["Ex", "Ey", "Ez", "Hx", "Hy", "Hz",
               "Mxx", "Mxy", "Mxz", "Myx", "Myy", "Myz", "Mzx", "Mzy", "Mzz",
               "Bx", "By", "Bz"]
FIELD_ID = {n: i for i, n in enumerate(FIELD_NAMES)}


@dataclass
class Config:
    name: str
    n: tuple                     # (nx, ny, nz)
    d: tuple                     # (dx, dy, dz)
    dt: float
    steps: int
    periodic: tuple = (False, False, False)
    eps_r: Optional[np.ndarray] = None
    sigma: Optional[np.ndarray] = None
    mu_r: Optional[np.ndarray] = None
    Ms: Optional[np.ndarray] = None
    alpha: Optional[np.ndarray] = None
    gamma: Optional[np.ndarray] = None
    m0_dir: Optional[np.ndarray] = None     # (3, nz, ny, nx)
    H0: tuple = (0.0, 0.0, 0.0)
    source: Optional[Source] = None
    probes: list = field(default_factory=list)
    tol: float = 1e-10
    max_iter: int = 100
    # initial fields (ABI layout, staggered extents); None -> zero
    E_init: Optional[list] = None
    H_init: Optional[list] = None
    pml: Optional[tuple] = None          # open boundary: (cells[6], R0, order)
    hard_sources: list = field(default_factory=list)       # HardSource entries
    surface_currents: list = field(default_factory=list)   # SurfaceCurrent entries

    @property
    def cells(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]


def edge_shape(n, periodic, comp):
    """(nz', ny', nx') extent of the edge array of component `comp`."""
    ext = []
    for ax in range(3):
        if ax == comp:
            ext.append(n[ax])
        else:
            ext.append(n[ax] if periodic[ax] else n[ax] + 1)
    return (ext[2], ext[1], ext[0])


def face_shape(n, periodic, comp):
    """(nz', ny', nx') extent of the face array normal to `comp`."""
    ext = []
    for ax in range(3):
        if ax == comp:
            ext.append(n[ax] if periodic[ax] else n[ax] + 1)
        else:
            ext.append(n[ax])
    return (ext[2], ext[1], ext[0])


def _cell(n, value):
    return np.full((n[2], n[1], n[0]), float(value))


def _box(arr, x, y, z, value):
    arr[z[0]:z[1], y[0]:y[1], x[0]:x[1]] = value


def _dir_z(n):
    m = np.zeros((3, n[2], n[1], n[0]))
    m[2] = 1.0
    return m


def _line_source_y(n, i, k, J0, f0):
    prof = np.zeros(edge_shape(n, (False,) * 3, 1))
    prof[k, :, i] = J0
    return Source(comp=1, profile=prof, f0=f0, Tp=1.0 / f0, t0=3.0 / f0)


def _port_source_z(n, i, J0, f0):
    """TE10-like port: Jz edges on the node plane x = i, profile sin(pi*j/ny)."""
    prof = np.zeros(edge_shape(n, (False,) * 3, 2))
    j = np.arange(n[1] + 1)
    prof[:, :, i] = J0 * np.sin(np.pi * j / n[1])[None, :]
    prof[:, 0, i] = 0.0
    prof[:, n[1], i] = 0.0
    return Source(comp=2, profile=prof, f0=f0, Tp=1.0 / f0, t0=3.0 / f0)


def slab64(steps: int = 200) -> Config:
    """64x16x16 PEC box with a centred 16x8x8 ferrite slab and a Jy line source."""
    n = (64, 16, 16)
    d = (1e-6,) * 3
    Ms = _cell(n, 0.0)
    _box(Ms, (24, 40), (4, 12), (4, 12), 1.4e5)
    alpha = _cell(n, 0.0)
    _box(alpha, (24, 40), (4, 12), (4, 12), 0.005)
    cfg = Config(name="slab64", n=n, d=d, dt=cfl_dt(0.9, *d), steps=steps,
                 eps_r=_cell(n, 1.0), sigma=_cell(n, 0.0), mu_r=_cell(n, 1.0),
                 Ms=Ms, alpha=alpha, gamma=_cell(n, GAMMA_E), m0_dir=_dir_z(n),
                 H0=(0.0, 0.0, 5e4), tol=1e-10)
    cfg.source = _line_source_y(n, 8, 8, 1e13, 10e9)
    cfg.probes = [Probe(1, 0, 48), Probe(0, FIELD_ID["Ey"], 32, 8, 8),
                  Probe(0, FIELD_ID["Mzx"], 32, 8, 8), Probe(0, FIELD_ID["Bz"], 32, 8, 8)]
    return cfg


def waveguide256(seed: int = 0, steps: int = 2000, n=(256, 64, 64)) -> Config:
    """PEC rectangular guide with a ferrite slab on the floor and a TE10-like port.

    The slab spans x in [nx/4, 3nx/4), y in [0, ny/4) and all z; alpha is i.i.d.
    U[0.001, 0.01] per cell from `seed`; eps_r = 13 in the slab (YIG, Sec. 5.2.2).
    `n` may be shrunk for tests; the geometry scales with it.
    """
    nx, ny, nz = n
    d = (2e-6,) * 3
    rng = np.random.default_rng(seed)
    xs, ys = (nx // 4, 3 * nx // 4), (0, ny // 4)
    Ms = _cell(n, 0.0)
    _box(Ms, xs, ys, (0, nz), 1.4e5)
    alpha = _cell(n, 0.0)
    a = rng.uniform(0.001, 0.01, size=(nz, ys[1] - ys[0], xs[1] - xs[0]))
    alpha[:, ys[0]:ys[1], xs[0]:xs[1]] = a
    eps = _cell(n, 1.0)
    _box(eps, xs, ys, (0, nz), 13.0)
    cfg = Config(name=f"waveguide{nx}", n=n, d=d, dt=cfl_dt(0.9, *d), steps=steps,
                 eps_r=eps, sigma=_cell(n, 0.0), mu_r=_cell(n, 1.0), Ms=Ms,
                 alpha=alpha, gamma=_cell(n, GAMMA_E), m0_dir=_dir_z(n),
                 H0=(0.0, 0.0, 0.2 / MU0), tol=1e-10)
    cfg.source = _port_source_z(n, 8 * nx // 256 if nx >= 64 else 2, 1e9, 1.5e12)
    p1, p2 = nx // 8, 7 * nx // 8
    cfg.probes = [Probe(1, 0, p1), Probe(1, 0, p2),
                  Probe(0, FIELD_ID["Ez"], p1, ny // 2, nz // 2),
                  Probe(0, FIELD_ID["Hy"], p2, ny // 2, nz // 2),
                  Probe(0, FIELD_ID["Myx"], nx // 2, ny // 8, nz // 2)]
    return cfg


def _random_boxes(rng, n, count, side_lo, side_hi, eps, sigma):
    for _ in range(count):
        s = rng.integers(side_lo, side_hi + 1, size=3)
        o = [rng.integers(0, max(1, n[a] - s[a] + 1)) for a in range(3)]
        e = rng.uniform(1.0, 10.0)
        g = rng.uniform(0.0, 1e3)
        sl = (slice(o[2], o[2] + s[2]), slice(o[1], o[1] + s[1]), slice(o[0], o[0] + s[0]))
        eps[sl] = e
        sigma[sl] = g


def filter512(seed: int = 0, steps: int = 1000, n=(512, 256, 256)) -> Config:
    """Tunable-filter-like grid: two ferrite bars plus seeded dielectric/lossy boxes.

    Bars (scaled with n): x in [nx/4, 3nx/4), z in [3nz/8, 5nz/8); bar A at
    y in [0, ny/8) with Ms = 1.4e5, bar B at y in [7ny/8, ny) with Ms = 1.75e5;
    alpha 0.0051 and eps_r 13 (YIG, Sec. 5.2.2).  Sixteen boxes with sides
    U{n/32 .. n/8} carry eps_r U[1,10] and sigma U[0,1e3] S/m; the ferrite wins
    overlaps.
    """
    nx, ny, nz = n
    d = (2e-6,) * 3
    rng = np.random.default_rng(seed)
    eps = _cell(n, 1.0)
    sig = _cell(n, 0.0)
    lo = max(2, min(n) // 16)
    hi = max(lo, min(n) // 4)
    _random_boxes(rng, n, 16, lo, hi, eps, sig)
    Ms = _cell(n, 0.0)
    alpha = _cell(n, 0.0)
    xs, zs = (nx // 4, 3 * nx // 4), (3 * nz // 8, 5 * nz // 8)
    for ys, ms in (((0, ny // 8), 1.4e5), ((7 * ny // 8, ny), 1.75e5)):
        _box(Ms, xs, ys, zs, ms)
        _box(alpha, xs, ys, zs, 0.0051)
        _box(eps, xs, ys, zs, 13.0)
        _box(sig, xs, ys, zs, 0.0)
    cfg = Config(name=f"filter{nx}", n=n, d=d, dt=cfl_dt(0.9, *d), steps=steps,
                 eps_r=eps, sigma=sig, mu_r=_cell(n, 1.0), Ms=Ms, alpha=alpha,
                 gamma=_cell(n, GAMMA_E), m0_dir=_dir_z(n), H0=(0.0, 0.0, 0.2 / MU0),
                 tol=1e-10)
    cfg.source = _port_source_z(n, max(2, 8 * nx // 512), 1e9, 2e12)
    cfg.probes = [Probe(1, 0, nx // 8), Probe(1, 0, 7 * nx // 8),
                  Probe(0, FIELD_ID["Ez"], nx // 2, ny // 2, nz // 2),
                  Probe(0, FIELD_ID["Myx"], nx // 2, ny // 16, nz // 2)]
    return cfg


def filter_crop(seed: int = 0, steps: int = 1000) -> Config:
    """The 128x64x64 crop of the filter grid, x in [192,320), y in [0,64),
    z in [96,160), run as its own PEC problem with its own port at local x = 8."""
    full = filter512(seed=seed, steps=steps)
    sl = (slice(96, 160), slice(0, 64), slice(192, 320))
    n = (128, 64, 64)
    cfg = Config(name="filter_crop128", n=n, d=full.d, dt=full.dt, steps=steps,
                 eps_r=np.ascontiguousarray(full.eps_r[sl]),
                 sigma=np.ascontiguousarray(full.sigma[sl]),
                 mu_r=np.ascontiguousarray(full.mu_r[sl]),
                 Ms=np.ascontiguousarray(full.Ms[sl]),
                 alpha=np.ascontiguousarray(full.alpha[sl]),
                 gamma=np.ascontiguousarray(full.gamma[sl]),
                 m0_dir=np.ascontiguousarray(full.m0_dir[(slice(None),) + sl]),
                 H0=full.H0, tol=full.tol)
    cfg.source = _port_source_z(n, 8, 1e9, 2e12)
    cfg.probes = [Probe(1, 0, 16), Probe(1, 0, 112), Probe(0, FIELD_ID["Myx"], 64, 8, 32)]
    return cfg


def _smooth_field(rng, shape, sigma_cells=3.0):
    from scipy.ndimage import gaussian_filter
    u = rng.uniform(0.0, 1.0, size=shape)
    s = gaussian_filter(u, sigma=sigma_cells, mode="reflect")
    return (s - s.min()) / (s.max() - s.min())


def design128(seed: int = 0, steps: int = 4000, n=(128, 64, 64)) -> Config:
    """Waveguide with a smooth random eps_r in [1,4] and Ms in [1e5,1.8e5] over a
    design region x in [nx/4, 3nx/4), y in [0, ny/2), z in [3nz/8, 5nz/8)."""
    nx, ny, nz = n
    d = (2e-6,) * 3
    rng = np.random.default_rng(seed)
    xs, ys, zs = (nx // 4, 3 * nx // 4), (0, ny // 2), (3 * nz // 8, 5 * nz // 8)
    shp = (zs[1] - zs[0], ys[1] - ys[0], xs[1] - xs[0])
    e = 1.0 + 3.0 * _smooth_field(rng, shp)
    m = 1e5 + 0.8e5 * _smooth_field(rng, shp)
    eps = _cell(n, 1.0)
    Ms = _cell(n, 0.0)
    alpha = _cell(n, 0.0)
    eps[zs[0]:zs[1], ys[0]:ys[1], xs[0]:xs[1]] = e
    Ms[zs[0]:zs[1], ys[0]:ys[1], xs[0]:xs[1]] = m
    alpha[zs[0]:zs[1], ys[0]:ys[1], xs[0]:xs[1]] = 0.005
    cfg = Config(name=f"design{nx}", n=n, d=d, dt=cfl_dt(0.9, *d), steps=steps,
                 eps_r=eps, sigma=_cell(n, 0.0), mu_r=_cell(n, 1.0), Ms=Ms,
                 alpha=alpha, gamma=_cell(n, GAMMA_E), m0_dir=_dir_z(n),
                 H0=(0.0, 0.0, 0.2 / MU0), tol=1e-10)
    cfg.source = _port_source_z(n, max(2, 8 * nx // 128), 1e9, 1.5e12)
    cfg.probes = [Probe(1, 0, nx - max(2, 8 * nx // 128))]
    return cfg


def scale1024(seed: int = 0, steps: int = 500, n=(1024, 512, 512)) -> Config:
    """Large grid: three ferrite inclusions (Ms U[1e5,2e5], alpha U[0.001,0.02],
    eps_r 13) at seeded non-overlapping positions plus 64 seeded dielectric boxes."""
    nx, ny, nz = n
    d = (2e-6,) * 3
    rng = np.random.default_rng(seed)
    eps = _cell(n, 1.0).astype(np.float64)
    sig = _cell(n, 0.0)
    lo = max(2, min(n) // 16)
    hi = max(lo, min(n) // 4)
    _random_boxes(rng, n, 64, lo, hi, eps, sig)
    Ms = _cell(n, 0.0)
    alpha = _cell(n, 0.0)
    bx, by, bz = nx // 8, ny // 8, nz // 8
    slots = [(a, b, c) for a in range(1, 7) for b in range(0, 7) for c in range(0, 7)]
    pick = rng.choice(len(slots), size=3, replace=False)
    for p in pick:
        a, b, c = slots[p]
        ms = rng.uniform(1e5, 2e5)
        al = rng.uniform(0.001, 0.02)
        box = ((a * bx, a * bx + bx), (b * by, b * by + by), (c * bz, c * bz + bz))
        _box(Ms, *box, ms)
        _box(alpha, *box, al)
        _box(eps, *box, 13.0)
        _box(sig, *box, 0.0)
    cfg = Config(name=f"scale{nx}", n=n, d=d, dt=cfl_dt(0.9, *d), steps=steps,
                 eps_r=eps, sigma=sig, mu_r=_cell(n, 1.0), Ms=Ms, alpha=alpha,
                 gamma=_cell(n, GAMMA_E), m0_dir=_dir_z(n), H0=(0.0, 0.0, 0.2 / MU0),
                 tol=1e-10)
    cfg.source = _port_source_z(n, max(2, 8 * nx // 512), 1e9, 2e12)
    # loss plane between the port and the inclusions: within 500 steps the
    # pulse (about 0.5 cells per step) reaches it, not the far end of the grid
    cfg.probes = [Probe(1, 0, max(2, 3 * nx // 32))]
    return cfg


def air_waveguide(steps: int = 80000, pml_cells: int = 64, source: str = "soft") -> Config:
    """The air-filled X-band waveguide of Sec. 5.2.1: W = 14.95 mm (x),
    h = 10.16 mm (y), L = 500 mm (z) on 512 x 4 x 512 cells, PEC side walls,
    PEC at the z = +L/2 end and an open boundary (PML of `pml_cells` cells)
    at z = -L/2; CFL 0.8.  The TE10 excitation ~ sin(pi x / W) carries the
    modulated Gaussian pulse (f0 = 10.5 GHz, Tp = 1/f0, peak at 3 Tp):
    source "soft", a current sheet Jy one cell inside the PEC end; source
    "surface", the surface current J_s,y (A/m) on the PEC end wall itself, as
    in the paper.  Ey is sampled along the centre line x = W/2, all z nodes;
    with the surface current also Hx, all z cells (probes 513 on): holding
    H at the wall leaves the evanescent Ey smaller than Hx by the modal wave
    impedance omega mu0 / alpha (~0.4 ohm at 7.5 GHz)."""
    W_, h_, L_ = 14.95e-3, 10.16e-3, 500e-3
    n = (512, 4, 512)
    d = (W_ / n[0], h_ / n[1], L_ / n[2])
    cfg = Config(name="airwg", n=n, d=d, dt=cfl_dt(0.8, *d), steps=steps)
    prof = np.zeros(edge_shape(n, (False,) * 3, 1))
    xi = np.arange(n[0] + 1) * d[0]
    f0 = 10.5e9
    if source == "soft":
        prof[n[2] - 1, :, :] = np.sin(np.pi * xi / W_)[None, :]
        cfg.source = Source(1, prof, f0, 1.0 / f0, 3.0 / f0)
    elif source == "surface":
        prof[n[2], :, :] = np.sin(np.pi * xi / W_)[None, :]
        cfg.surface_currents = [SurfaceCurrent(2, 1, 1, prof, f0, 1.0 / f0, 3.0 / f0)]
    else:
        raise ValueError(source)
    cfg.pml = ((0, 0, 0, 0, pml_cells, 0), 1e-6, 3.0)
    cfg.probes = [Probe(0, FIELD_ID["Ey"], n[0] // 2, n[1] // 2, k) for k in range(n[2] + 1)]
    if source == "surface":
        cfg.probes += [Probe(0, FIELD_ID["Hx"], n[0] // 2, n[1] // 2, k) for k in range(n[2])]
    return cfg


def tunable_filter(steps: int = 320000, pml_cells: int = 64, gap: int = 16, n=(1024, 4, 512),
                   source: str = "surface") -> Config:
    """The magnetically tunable filter of Sec. 5.2.2: the waveguide of
    air_waveguide() with a YIG slab 0.45 mm thick against the x = 0 side
    wall, over the full height and along the guide (Ms = 1.3926e5 A/m,
    alpha = 0.0051, eps_r = 13), bias H0 = 2.2998e5 A/m along y, M along y;
    1024 x 4 x 512 cells, CFL 0.8.  The slab stops `gap` cells short of the
    open layer at z = -L/2 (magnetic material inside the layer is not
    supported).  320,000 steps are 12.5 ns, four decay times of the damped
    precession (1 / (alpha omega) ~ 3 ns): the spectrum has settled.
    Drive as in air_waveguide(): "surface", the paper's surface current on
    the PEC end (the held wall faces may not be magnetic, so the slab's
    magnetisation stops one cell short of that end; its permittivity does
    not), or "soft", the current sheet one cell inside it."""
    W_, h_, L_ = 14.95e-3, 10.16e-3, 500e-3
    d = (W_ / n[0], h_ / n[1], L_ / n[2])
    cfg = Config(name="mtf", n=n, d=d, dt=cfl_dt(0.8, *d), steps=steps)
    shp = (n[2], n[1], n[0])
    t = int(round(0.45e-3 / d[0]))
    eps = np.ones(shp)
    Ms = np.zeros(shp)
    alpha = np.zeros(shp)
    z0 = pml_cells + gap
    eps[z0:, :, :t] = 13.0
    Ms[z0:, :, :t] = 1.3926e5
    alpha[z0:, :, :t] = 0.0051
    m0 = np.zeros((3,) + shp)
    m0[1] = 1.0
    cfg.eps_r, cfg.Ms, cfg.alpha = eps, Ms, alpha
    cfg.gamma = np.full(shp, GAMMA_E)
    cfg.m0_dir = m0
    cfg.H0 = (0.0, 2.2998e5, 0.0)
    cfg.tol = 1e-10
    prof = np.zeros(edge_shape(n, (False,) * 3, 1))
    xi = np.arange(n[0] + 1) * d[0]
    f0 = 10.5e9
    if source == "soft":
        prof[n[2] - 1, :, :] = np.sin(np.pi * xi / W_)[None, :]
        cfg.source = Source(1, prof, f0, 1.0 / f0, 3.0 / f0)
    elif source == "surface":
        prof[n[2], :, :] = np.sin(np.pi * xi / W_)[None, :]
        cfg.surface_currents = [SurfaceCurrent(2, 1, 1, prof, f0, 1.0 / f0, 3.0 / f0)]
        Ms[-1] = 0.0
        alpha[-1] = 0.0
    else:
        raise ValueError(source)
    cfg.pml = ((0, 0, 0, 0, pml_cells, 0), 1e-6, 3.0)
    cfg.probes = [Probe(0, FIELD_ID["Ey"], n[0] // 2, n[1] // 2, k) for k in range(n[2] + 1)]
    return cfg


def convergence_cube(N: int, side: float = 0.2, tol: float = 1e-6) -> Config:
    """The coupled convergence problem of Sec. 5.1 on an N^3 grid.

    Fully periodic cube of edge `side` centred on the origin; cosine E and H
    of eq:convergeE / eq:convergeH (amplitudes 1e6 V/m and 1e6/(120 pi)
    A/m, wavenumber 20 pi) at their Yee locations; Gaussian bumps
    g = exp(-1000 r^2) at cell centres in sigma = 0.1 g, eps_r = 1 + g,
    Ms = 1e4 (1 + g), alpha = 0.5 (1 + g), gamma = -1.759e11 (1 + g);
    M along x, no bias; CFL 0.9 on the vacuum light speed; 5 N / 32 steps,
    so every resolution reaches the same time.
    """
    d = (side / N,) * 3
    xn = np.arange(N) * d[0] - side / 2        # node coordinates
    xc = xn + d[0] / 2                          # cell-centre coordinates
    X, Y, Z = np.meshgrid(xc, xc, xc, indexing="ij")
    g = np.exp(-1000.0 * (X**2 + Y**2 + Z**2))
    host = lambda a: np.ascontiguousarray(a.transpose(2, 1, 0))
    m0 = np.zeros((3, N, N, N))
    m0[0] = 1.0
    cfg = Config(name=f"conv{N}", n=(N, N, N), d=d, dt=cfl_dt(0.9, *d), steps=5 * N // 32,
                 periodic=(True, True, True), eps_r=host(1 + g), sigma=host(0.1 * g),
                 Ms=host(1e4 * (1 + g)), alpha=host(0.5 * (1 + g)),
                 gamma=host(GAMMA_E * (1 + g)), m0_dir=m0, tol=tol)
    k = 20 * math.pi
    e0, h0 = 1e6, 1e6 / (120 * math.pi)
    ones = np.ones((N, N, N))
    # (i, j, k)-indexed placements, then host layout
    Ex = e0 * np.cos(k * xn)[None, None, :] * ones      # cos(20 pi z), z at nodes
    Ey = e0 * np.cos(k * xn)[:, None, None] * ones      # cos(20 pi x), x at nodes
    Ez = e0 * np.cos(k * xn)[None, :, None] * ones      # cos(20 pi y), y at nodes
    Hx = h0 * np.cos(k * xc)[None, :, None] * ones      # cos(20 pi y), y at cell centres
    Hy = h0 * np.cos(k * xc)[None, None, :] * ones      # cos(20 pi z), z at cell centres
    Hz = h0 * np.cos(k * xc)[:, None, None] * ones      # cos(20 pi x), x at cell centres
    cfg.E_init = [host(a) for a in (Ex, Ey, Ez)]
    cfg.H_init = [host(a) for a in (Hx, Hy, Hz)]
    return cfg


def random_fields(cfg: Config, seed: int, amp_e: float = 1.0, amp_h: float = 1.0):
    """Seeded random E and H on every staggered entry (the solvers zero the
    PEC-wall entries themselves).  Returns (E_list, H_list) in ABI layout."""
    rng = np.random.default_rng(seed)
    E = [amp_e * rng.standard_normal(edge_shape(cfg.n, cfg.periodic, c)) for c in range(3)]
    H = [amp_h * rng.standard_normal(face_shape(cfg.n, cfg.periodic, c)) for c in range(3)]
    return E, H


CONFIGS = {
    "slab64": slab64,
    "waveguide256": waveguide256,
    "filter512": filter512,
    "filter_crop128": filter_crop,
    "design128": design128,
    "scale1024": scale1024,
}
