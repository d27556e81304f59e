"""Hard sources (Sec. 3.2) and the surface current (Sec. 5.2.1) on the HIP path.

* Parity with the oracle (FP64 at the 1e-12 bar, FP32 at 1e-4, iteration
  counts equal) on two grids with an E hard source, an H hard source on the
  non-magnetic faces that a magnet's H_eff reads (the iterations must see the
  held value), a surface current on a PEC wall, a soft source, near, far and
  layer tiles, and probes; from a random start.
* Splitting a run into calls of any length gives the same bits (the tiles
  of an H source leave the fused far pass).
* The exact transport at Courant number 1 through the library: the
  waveform of each source arrives m cells away m steps later.
* Rejections through the C ABI.
* The air-filled waveguide of Sec. 5.2.1 driven, as in the paper, by the
  surface current on its PEC end: the attenuation below cutoff within 2 %
  of theory and the cutoff within 0.5 %, fitted on Hx of the TE10 mode
  (same alpha as Ey).  With H held at the wall, the evanescent Ey is the
  modal wave impedance omega mu0 / alpha (~0.4 ohm at 7.5 GHz) times Hx,
  against ~900 ohm in the propagating band, so below cutoff it sits under
  the spectral leakage of an unwindowed transform; Hx does not.
"""
import math

import numpy as np
import pytest

import workloads as W
from tests import parity_util as PU
from tests import test_gpu_waveguide as WG

pytestmark = pytest.mark.gpu
F0 = 20e12
ETA = math.sqrt(1.25663706212e-6 / 8.8541878128e-12)


def _sources(cfg, n):
    """E hard on Ez, H hard on the Hy faces of the cell column beside the
    magnet's x = 60 side (read by the magnetic x faces there), a surface
    current Jz on the y = 0 wall."""
    ez = np.zeros(W.edge_shape(n, cfg.periodic, 2))
    ez[12, 8:13, 100] = np.linspace(1e3, 3e3, 5)
    hy = np.zeros(W.face_shape(n, cfg.periodic, 1))
    hy[9:14, 8:12, 59] = 40.0
    hy[11, 9, 59] = 0.0                     # held at zero inside the box
    js = np.zeros(W.edge_shape(n, cfg.periodic, 2))
    js[8:16, 0, 30:51] = 25.0
    cfg.hard_sources = [W.HardSource(2, ez, F0, 1 / F0, 3 / F0), W.HardSource(4, hy, F0, 1 / F0, 2 / F0)]
    cfg.surface_currents = [W.SurfaceCurrent(1, 0, 2, js, F0, 1 / F0, 2.5 / F0)]


def _cfg(steps=30, pml=True):
    n = (140, 20, 24)
    d = (1e-6, 1.2e-6, 0.9e-6)
    shp = (n[2], n[1], n[0])
    rng = np.random.default_rng(23)
    Ms = np.zeros(shp)
    Ms[9:14, 7:12, 60:76] = 1.3e5
    m0 = np.zeros((3,) + shp)
    m0[0], m0[2] = 0.2, 1.0
    prof = np.zeros(W.edge_shape(n, (False,) * 3, 1))
    prof[10, 2:18, 20] = 1e11
    cfg = W.Config("hardbox", n, d, W.cfl_dt(0.9, *d), steps, eps_r=rng.uniform(1, 3, shp),
                   mu_r=np.where(Ms > 0, 1.0, rng.uniform(1, 1.5, shp)), Ms=Ms,
                   alpha=np.where(Ms > 0, 0.02, 0.0), gamma=np.full(shp, W.GAMMA_E), m0_dir=m0,
                   H0=(0, 0, 8e4), tol=1e-11)
    cfg.source = W.Source(1, prof, F0, 1 / F0, 1e-13)
    if pml:
        cfg.pml = ((8, 10, 0, 4, 5, 5), 1e-6, 3)
    PU.with_random_start(cfg, seed=8, amp_e=1e5, amp_h=3e2)
    _sources(cfg, n)
    F = W.FIELD_ID
    cfg.probes = [W.Probe(0, F["Ez"], 100, 10, 12), W.Probe(0, F["Ez"], 104, 10, 12),
                  W.Probe(0, F["Hy"], 58, 9, 11), W.Probe(0, F["Ey"], 40, 1, 11),
                  W.Probe(0, F["Hx"], 40, 0, 11), W.Probe(1, 0, 110)]
    return cfg


def test_h_source_tiles_leave_the_fused_pass():
    """Without layers the surface current's faces (y = 0, x 30-50) lie in a
    far tile of the plain grid."""
    import paper_2103_12819_amd as mm
    cfg = _cfg(pml=False)
    base = mm.from_config(cfg, with_probes=False)
    cfg.hard_sources, cfg.surface_currents = [], []
    plain = mm.from_config(cfg, with_probes=False)
    a, b = base.tiles(), plain.tiles()
    base.close()
    plain.close()
    assert a["near_tiles"] > b["near_tiles"] and a["tiles"] == b["tiles"], (a, b)
    assert a["near_tiles"] + a["far_tiles"] == b["near_tiles"] + b["far_tiles"]


@pytest.mark.parametrize("pml", [True, False])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-4)])
def test_parity_with_hard_sources(precision, tol, pml):
    cfg = _cfg(pml=pml)
    ref, sim, ref0 = PU.run_pair(cfg, cfg.steps, precision=precision)
    PU.compare(ref, sim, ref0, tol, check_iters=precision == "fp64", dev_tol=None if precision == "fp64" else tol)
    # the held entries hold exactly their value (FP64)
    if precision == "fp64":
        from oracle.yee_llg import waveform
        g = waveform(cfg.steps * cfg.dt, F0, 1 / F0, 3 / F0)
        assert sim.field("Ez")[12, 10, 100] == ref.field("Ez")[12, 10, 100] == 2e3 * g
        assert sim.field("Hy")[11, 9, 59] == 0.0


def test_call_boundaries_with_hard_sources():
    import paper_2103_12819_amd as mm
    outs = []
    for chunks in ([24], [1] * 24, [7, 2, 15]):
        cfg = _cfg(steps=24)
        sim = mm.from_config(cfg)
        for c in chunks:
            sim.step(c)
        outs.append([sim.field(nm) for nm in PU.E_H + PU.M_NAMES] + [sim.probe(p)[0] for p in range(len(cfg.probes))])
        sim.close()
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert np.array_equal(a, b)


def _line(kind):
    """A 700-cell line at Courant number 1 (11 tiles of 64 along it) with one
    source; returns the sampled series at distances 1, 5, 40, 120 and the
    expected ones."""
    import paper_2103_12819_amd as mm
    from oracle.yee_llg import waveform
    Tp, t0, steps, A = 1 / 15e12, 3 / 15e12, 200, 2.0
    dist = (1, 5, 40, 120)
    if kind == "surface":
        n, d, per = (1, 1, 400), (1e2, 1e2, 1e-6), (True, True, False)
    else:
        n, d, per = (700, 1, 1), (1e-6, 1e2, 1e2), (False, True, True)
    dt = W.cfl_dt(1.0, *d)
    sim = mm.Sim(n, d, dt, periodic=per)
    x0 = 330
    F = W.FIELD_ID
    if kind == "E":
        prof = np.zeros(W.edge_shape(n, per, 2))
        prof[0, 0, x0] = A
        sim.add_hard_source(2, prof, 15e12, Tp, t0)
        pts = [sim.add_probe(0, F["Ez"], x0 + m, 0, 0) for m in dist]
        want = lambda q, m: A * waveform((q - m) * dt, 15e12, Tp, t0) if q > m else 0.0  # noqa: E731
    elif kind == "H":
        prof = np.zeros(W.face_shape(n, per, 1))
        prof[0, 0, x0] = A
        sim.add_hard_source(4, prof, 15e12, Tp, t0)
        pts = [sim.add_probe(0, F["Ez"], x0 + m, 0, 0) for m in dist]
        want = lambda q, m: -ETA * A * waveform((q - m + 0.5) * dt, 15e12, Tp, t0) if q >= m else 0.0  # noqa: E731
    else:
        J = np.zeros(W.edge_shape(n, per, 1))
        J[n[2], 0, 0] = A
        sim.add_surface_current(2, 1, 1, J, 15e12, Tp, t0)
        pts = [sim.add_probe(0, F["Ey"], 0, 0, n[2] - m) for m in dist]
        want = lambda q, m: -ETA * A * waveform((q - m + 0.5) * dt, 15e12, Tp, t0) if q >= m else 0.0  # noqa: E731
    sim.step(steps)
    got = np.array([sim.probe(p)[0] for p in pts])
    sim.close()
    exp = np.array([[want(q, m) for q in range(1, steps + 1)] for m in dist])
    return got, exp


@pytest.mark.parametrize("kind", ["E", "H", "surface"])
def test_exact_transport_at_courant_number_one(kind):
    got, exp = _line(kind)
    scale = np.max(np.abs(exp))
    assert scale > 0
    assert np.max(np.abs(got - exp)) < 1e-9 * scale, np.max(np.abs(got - exp)) / scale


def test_rejections():
    import paper_2103_12819_amd as mm
    cfg = _cfg(steps=2)
    n = cfg.n
    bad_h = np.zeros(W.face_shape(n, cfg.periodic, 0))
    bad_h[11, 9, 64] = 1.0                  # an evolving magnetic x face
    in_layer = np.zeros(W.edge_shape(n, cfg.periodic, 2))
    in_layer[12, 10, 3] = 1.0               # node x = 3 inside the 8-cell x layer
    zero = np.zeros(W.edge_shape(n, cfg.periodic, 2))
    for field, prof in ((3, bad_h), (2, in_layer), (2, zero)):
        sim = mm.from_config(cfg, with_probes=False)
        with pytest.raises(mm.MMError, match="MM_EINVAL"):
            sim.add_hard_source(field, prof, F0, 1 / F0, 0.0)
        sim.close()
    ok = np.zeros(W.edge_shape(n, cfg.periodic, 2))
    ok[12, 10, 100] = 1.0
    sim = mm.from_config(cfg, with_probes=False)
    for _ in range(5):                       # with the three of the config: 8 = MM_MAX_HARD
        sim.add_hard_source(2, ok, F0, 1 / F0, 0.0)
    with pytest.raises(mm.MMError, match="MM_EINVAL"):
        sim.add_hard_source(2, ok, F0, 1 / F0, 0.0)
    sim.close()
    sim = mm.from_config(cfg, with_probes=False)
    sim.step(1)
    with pytest.raises(mm.MMError, match="MM_ESTATE"):
        sim.add_hard_source(2, ok, F0, 1 / F0, 0.0)
    sim.close()
    cfg.pml, cfg.mu_r = None, None           # otherwise admissible for the adjoint
    sim = mm.from_config(cfg, with_probes=False)
    with pytest.raises(mm.MMError, match="MM_EINVAL"):
        sim.enable_adjoint(10)
    sim.close()
    cfg.hard_sources, cfg.surface_currents = [], []
    sim = mm.from_config(cfg, with_probes=False)
    sim.enable_adjoint(10)
    with pytest.raises(mm.MMError, match="MM_EINVAL"):
        sim.add_hard_source(2, ok, F0, 1 / F0, 0.0)
    with pytest.raises(mm.MMError, match="MM_EINVAL"):
        sim.add_surface_current(2, 0, 2, ok, F0, 1 / F0, 0.0)    # comp == axis
    sim.close()


@pytest.fixture(scope="module")
def surface_spectrum():
    import paper_2103_12819_amd as mm
    cfg = W.air_waveguide(source="surface")
    sim = mm.from_config(cfg)
    sim.step(cfg.steps)
    nz = cfg.n[2]
    series = np.array([sim.probe(p)[0] for p in range(nz + 1, 2 * nz + 1)])     # Hx, z cells
    sim.close()
    spec = np.abs(np.fft.rfft(series, axis=1))
    freqs = np.fft.rfftfreq(series.shape[1], cfg.dt)
    z = (np.arange(series.shape[0]) + 0.5) * cfg.d[2]
    return cfg, spec, freqs, z


def test_waveguide_driven_by_the_surface_current(surface_spectrum):
    cfg, spec, freqs, z = surface_spectrum
    for f in np.arange(7.5e9, 9.61e9, 0.3e9):
        fb, a = WG._alpha_fit(spec, freqs, z, f, cfg.n[2])
        th = WG._alpha_theory(fb)
        print(f"{fb / 1e9:.3f} GHz alpha {a:.2f} theory {th:.2f} 1/m")
        assert abs(a - th) <= 0.02 * th, (fb, a, th)
    fs, a2 = [], []
    for f in np.arange(7.5e9, 9.61e9, 0.15e9):
        fb, a = WG._alpha_fit(spec, freqs, z, f, cfg.n[2])
        fs.append(fb)
        a2.append(a * a)
    slope, icpt = np.polyfit(np.array(fs) ** 2, np.array(a2), 1)
    fc = math.sqrt(-icpt / slope)
    print("cutoff", fc / 1e9)
    assert abs(fc - WG.C0 / (2 * WG.WIDTH)) <= 0.005 * WG.C0 / (2 * WG.WIDTH), fc
