"""The air-filled X-band waveguide of Sec. 5.2.1 on the HIP path (FP64).

The full run of the paper: 512 x 4 x 512 cells, 80,000 steps at CFL 0.8, an
open boundary (PML) at one end.  Ey is sampled along the centre line; its
spectrum at each z gives the attenuation constant alpha(f) from the decay
away from the source (a least-squares fit of log|Ey| against z, in place of
the paper's ESPRIT).  Theory: alpha = Im sqrt((omega/c)^2 - (pi/W)^2), zero
above the TE10 cutoff c/(2W) = 10.03 GHz.

Checks: alpha within 2 % of theory from 7.5 to 9.6 GHz (measured: within
0.8 %); near zero above 10.4 GHz; the cutoff recovered from the fitted
alpha^2 (linear in f^2 below cutoff) within 0.5 % of 10.03 GHz (measured:
10.006 GHz).
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
C0 = 299792458.0
WIDTH = 14.95e-3


def _alpha_theory(f):
    k2 = (math.pi / WIDTH) ** 2 - (2 * math.pi * f / C0) ** 2
    return math.sqrt(k2) if k2 > 0 else 0.0


@pytest.fixture(scope="module")
def spectrum():
    import paper_2103_12819_amd as mm
    cfg = W.air_waveguide()
    sim = mm.from_config(cfg)
    sim.step(cfg.steps)
    series = np.array([sim.probe(p)[0] for p in range(len(cfg.probes))])
    sim.close()
    spec = np.abs(np.fft.rfft(series, axis=1))
    freqs = np.fft.rfftfreq(series.shape[1], cfg.dt)
    z = np.arange(series.shape[0]) * cfg.d[2]
    return cfg, spec, freqs, z


def _alpha_fit(spec, freqs, z, f, nz):
    """Decay constant of |Ey(f, z)| away from the source sheet (at z node
    nz - 1), fitted where the evanescent field stands well above the spectral
    leakage of the propagating part: from two cells below the sheet down to
    30 % of that value, at most 20 cells."""
    b = int(np.argmin(np.abs(freqs - f)))
    a = spec[:, b]
    top = nz - 2
    ks = []
    for k in range(top, top - 20, -1):
        if a[k] < 0.3 * a[top]:
            break
        ks.append(k)
    slope = np.polyfit(z[ks], np.log(a[ks]), 1)[0]
    return freqs[b], slope               # log|E| grows towards the source: slope = alpha


def test_attenuation_below_cutoff_follows_theory(spectrum):
    cfg, spec, freqs, z = spectrum
    for f in np.arange(7.5e9, 9.61e9, 0.3e9):
        fb, a = _alpha_fit(spec, freqs, z, f, cfg.n[2])
        th = _alpha_theory(fb)
        print(f"{fb / 1e9:.3f} GHz alpha {a:.2f} theory {th:.2f} 1/m")
        assert abs(a - th) <= 0.02 * th, (fb, a, th)


def test_no_attenuation_above_cutoff(spectrum):
    cfg, spec, freqs, z = spectrum
    ref = _alpha_theory(9e9)
    for f in np.arange(10.4e9, 12.6e9, 0.3e9):
        fb, a = _alpha_fit(spec, freqs, z, f, cfg.n[2])
        print(f"{fb / 1e9:.3f} GHz alpha {a:.3f} 1/m")
        assert abs(a) < 0.05 * ref, (fb, a)


def test_cutoff_frequency(spectrum):
    cfg, spec, freqs, z = spectrum
    fs, a2 = [], []
    for f in np.arange(7.5e9, 9.61e9, 0.15e9):
        fb, a = _alpha_fit(spec, freqs, z, f, cfg.n[2])
        fs.append(fb)
        a2.append(a * a)
    # alpha^2 = (pi/W)^2 - (2 pi f / c)^2 is linear in f^2; its zero is the cutoff
    slope, icpt = np.polyfit(np.array(fs) ** 2, np.array(a2), 1)
    fc = math.sqrt(-icpt / slope)
    print("cutoff", fc / 1e9)
    assert abs(fc - C0 / (2 * WIDTH)) <= 0.005 * C0 / (2 * WIDTH), fc
