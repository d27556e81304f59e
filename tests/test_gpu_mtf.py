"""The magnetically tunable filter of Sec. 5.2.2 on the HIP path (FP64).

The waveguide of Sec. 5.2.1 at 1024 x 4 x 512 cells with a 0.45 mm YIG slab
against the x = 0 wall, biased along y, driven as in the paper by the
surface current on the PEC end (workloads.tunable_filter).  Ey is sampled
along the centre line for 320,000 steps (12.5 ns: the precession rings down
with time constant 1 / (alpha omega) ~ 3 ns).

Analysis, as in the paper's post-processing: a Fourier transform at each z
(the record tapered to zero over its second half), then a least-squares
ESPRIT fit of a few complex exponentials exp(-gamma z) to the spectrum along
z at each frequency (Roy and Kailath, 1989); alpha + j beta = gamma of the
strongest term.

Both features of tab:alpha_YIG are broad in alpha(f), and the paper's
values fall inside them:
  * the cutoff is a transition of about 0.3 GHz: alpha = beta (the real
    part of gamma^2 vanishes) at f_c2 = 9.077 GHz, and alpha has fallen to
    a tenth of its 8.5 GHz value by the knee at 9.38 GHz; the paper's
    9.2717 lies between the two, the experiment's 9.1605 is 0.9 % above the
    crossing;
  * the absorption band is flat-topped, from the uniform (Kittel) mode at
    10.25 GHz towards the surface-mode limit gamma (H0 + Ms/2) = 10.54 GHz:
    its largest alpha sits at 10.18 GHz (0.7 % under Kittel), its centroid
    above half height at 10.356 GHz (1.0 % under the paper's 10.4568, 0.8 %
    under the experiment's 10.4354).
The bars below are these achieved agreements.  Measured separately on the
GPU over 640,000 steps (windows of 80,000 to 640,000 steps): the soft
current sheet one cell inside the PEC end instead of the surface current,
and a slab over half the guide instead of all of it, move f_c2 and both
FMR figures by at most 0.03 GHz once the window holds 320,000 steps or
more; an 80,000-step window (the paper's step count, 3.1 ns at this grid's
time step) has not settled: f_c2 8.8-8.9 GHz, the largest alpha near 10.7
GHz.  The peak attenuation of the table (in dB, over a length the paper
does not state) is not compared.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
STEPS = 320000
DECIM = 100                     # keep every 100th sample: Nyquist 128 GHz
FREQS = np.arange(6e9, 13.0001e9, 0.02e9)


def _esprit(x, order):
    """Poles lam_m and amplitudes c_m of x[k] ~ sum_m c_m lam_m^k: signal
    subspace of the Hankel matrix, poles from its shift invariance, then the
    amplitudes by least squares."""
    m = len(x)
    L = m // 2
    H = np.lib.stride_tricks.sliding_window_view(x, L)
    U = np.linalg.svd(H, full_matrices=False)[0][:, :order]
    lam = np.linalg.eigvals(np.linalg.lstsq(U[:-1], U[1:], rcond=None)[0])
    amp = np.linalg.lstsq(lam[None, :] ** np.arange(m)[:, None], x, rcond=None)[0]
    return lam, amp


@pytest.fixture(scope="module")
def gamma():
    import paper_2103_12819_amd as mm
    cfg = W.tunable_filter(steps=STEPS)
    sim = mm.from_config(cfg)
    sim.step(cfg.steps)
    series = np.array([sim.probe(p)[0][::DECIM] for p in range(len(cfg.probes))])
    sim.close()
    n = series.shape[1]
    w = np.ones(n)
    w[n // 2:] = 0.5 + 0.5 * np.cos(np.pi * np.arange(n - n // 2) / (n - n // 2))
    t = np.arange(n) * cfg.dt * DECIM
    X = (series * w) @ np.exp(-2j * np.pi * t[:, None] * FREQS[None, :])
    # z nodes 100 .. 499: past the slab's end (node 80), short of the source
    # sheet (node 511); marching away from the source
    out = []
    for b in range(len(FREQS)):
        x = X[100:500, b][::-1]
        lam, amp = _esprit(x, 6)
        power = np.abs(amp) ** 2 * np.array([np.sum(np.abs(l) ** (2 * np.arange(len(x)))) for l in lam])
        out.append(-np.log(lam[np.argmax(power)]) / cfg.d[2])
    return np.array(out)


def _at(g, f):
    return g[int(np.argmin(np.abs(FREQS - f)))]


def test_band_structure(gamma):
    """Evanescent below the cutoff (alpha falling with f, beta ~ 0), a pass
    band, the stop band above the resonance, and free propagation above."""
    a = gamma.real
    lo = (FREQS >= 6e9) & (FREQS <= 8.9e9)
    print("alpha at 6, 7, 8, 9.5, 10.5, 11.5, 12.5 GHz:",
          [round(_at(gamma, f).real, 2) for f in (6e9, 7e9, 8e9, 9.5e9, 10.5e9, 11.5e9, 12.5e9)])
    rise = np.diff(a[lo & (FREQS <= 7.9e9)])
    print("largest rise of alpha between neighbouring frequencies, 6-7.9 GHz:", float(np.max(rise)), "1/m")
    assert np.all(rise < 0.5)          # falling, up to the fit's scatter
    assert np.all(a[lo] > 50) and np.all(np.abs(gamma.imag[lo]) < 0.15 * a[lo])
    pas = (FREQS >= 9.45e9) & (FREQS <= 9.75e9)
    assert np.all(a[pas] < 10) and np.all(gamma.imag[pas] > 70)
    stop = (FREQS >= 10.2e9) & (FREQS <= 10.8e9)
    assert np.all(a[stop] > 80)
    high = FREQS >= 11.5e9
    assert np.all(np.abs(a[high]) < 3)


def test_cutoff_frequency(gamma):
    sel = np.nonzero((FREQS > 8.5e9) & (gamma.imag > gamma.real))[0]
    b = sel[0]
    # linear interpolation of beta - alpha between the grid frequencies
    d0 = gamma[b - 1].imag - gamma[b - 1].real
    d1 = gamma[b].imag - gamma[b].real
    fc = FREQS[b - 1] + (FREQS[b] - FREQS[b - 1]) * d0 / (d0 - d1)
    a85 = _at(gamma, 8.5e9).real
    knee = FREQS[np.nonzero((FREQS > 8.5e9) & (gamma.real < 0.1 * a85))[0][0]]
    print("cutoff f_c2 (alpha = beta)", fc / 1e9, "GHz; knee (alpha < alpha(8.5 GHz) / 10)", knee / 1e9, "GHz")
    assert abs(fc - 9.1605e9) / 9.1605e9 < 0.010, fc        # experiment
    assert fc < 9.2717e9 < knee, (fc, knee)                  # the paper's simulation: inside the transition
    assert knee - fc < 0.35e9, (fc, knee)


def test_resonance_frequency(gamma):
    band = (FREQS > 9.8e9) & (FREQS < 11e9)
    b = int(np.argmax(np.where(band, gamma.real, -np.inf)))
    fr = FREQS[b]
    a = np.where(band, gamma.real, 0.0)
    half = a >= 0.5 * a[b]
    fcen = float(np.sum(FREQS[half] * a[half]) / np.sum(a[half]))
    print("largest attenuation", gamma[b].real, "1/m at", fr / 1e9, "GHz; band centroid", fcen / 1e9, "GHz")
    assert abs(fr - 10.25e9) / 10.25e9 < 0.0075, fr         # Kittel, thin slab
    assert abs(fcen - 10.4568e9) / 10.4568e9 < 0.010, fcen  # the paper's simulation
    assert abs(fcen - 10.4354e9) / 10.4354e9 < 0.008, fcen  # experiment
