"""The Kittel slab (ferromagnetic resonance of a uniformly biased slab).

Sec. 5.2.2 quotes Kittel's thin-slab resonance with the YIG values of its
tunable filter: H0 = 2890 Oe and 4 pi Ms = 1750 G, i.e. H0 = 2.2998e5 A/m and
Ms = 1.3926e5 A/m in SI, 10.25 GHz.

Set-up: a box periodic on all axes whose fields vary only along x (one cell
in y and z, so the 1-D Courant limit applies), a slab of n cells normal to
x filling the fraction n/Nx of the box, bias H0 along z (in the slab's
plane), no damping, M tilted by a small angle towards y.  For a box much
smaller than the wavelength the uniform precession sees two demagnetising
factors: N_x = 1 (B_x cannot change along x) and N_y = n/Nx (the mean of
B_y over the periodic box is conserved), so

    f = (mu0 |gamma| / 2 pi) sqrt((H0 + Ms) (H0 + (n/Nx) Ms)),

which tends to the thin-film formula as n/Nx -> 0.  The face-averaged Ms
of the Yee discretisation (Sec. 3.1) smears each interface over a face,
so on a grid the frequency approaches this value at first order in 1/n.
"""
import math

import numpy as np

import workloads as W

MU0 = 1.25663706212e-6
GAMMA = -1.759e11
H0 = 2890.0 * 1e3 / (4 * math.pi)      # 2890 Oe in A/m
MS = 1750.0 * 1e3 / (4 * math.pi)      # 4 pi Ms = 1750 G, Ms in A/m
BOX = 3.2e-4                           # box length (m), ~1/80 of the wavelength
THETA = math.radians(0.1)


def kittel_slab(fill):
    return MU0 * abs(GAMMA) / (2 * math.pi) * math.sqrt((H0 + MS) * (H0 + fill * MS))


def kittel_thin_film():
    return MU0 * abs(GAMMA) / (2 * math.pi) * math.sqrt(H0 * (H0 + MS))


def config(Nx, n, periods=1.0):
    """Config of an Nx x 1 x 1 box with a centred slab of n cells and enough
    steps for `periods` periods (plus a margin); also returns the probed face
    index along x (a z-normal face at the slab centre)."""
    d = BOX / Nx
    D = (d, 100 * d, 100 * d)
    shp = (1, 1, Nx)
    Ms = np.zeros(shp)
    x0 = (Nx - n) // 2
    Ms[:, :, x0:x0 + n] = MS
    m0 = np.zeros((3,) + shp)
    m0[1], m0[2] = math.sin(THETA), math.cos(THETA)
    dt = W.cfl_dt(0.9, *D)
    steps = int(periods / (kittel_slab(n / Nx) * dt)) + 20
    cfg = W.Config(f"kittel{Nx}", (Nx, 1, 1), D, dt, steps, periodic=(True, True, True),
                   Ms=Ms, alpha=np.zeros(shp), gamma=np.full(shp, GAMMA), m0_dir=m0,
                   H0=(0.0, 0.0, H0), tol=1e-10)
    return cfg, x0 + n // 2


def frequency(series, dt):
    """Frequency of a sampled cosine from its zero crossings about the
    mid-range (linear interpolation between samples)."""
    y = np.asarray(series) - 0.5 * (np.max(series) + np.min(series))
    t = (np.arange(len(y)) + 1) * dt
    zc = []
    for q in range(1, len(y)):
        if (y[q - 1] < 0 <= y[q]) or (y[q - 1] > 0 >= y[q]):
            zc.append(t[q - 1] + (t[q] - t[q - 1]) * (-y[q - 1]) / (y[q] - y[q - 1]))
    assert len(zc) >= 2
    half = (zc[-1] - zc[0]) / (len(zc) - 1)
    return 1.0 / (2 * half)
