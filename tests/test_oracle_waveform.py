"""Pin of the oracle's source pulse (eq:gaulssian, Sec. 5.2.1).

The paper's excitation is a Gaussian envelope centred at t = 3 Tp with
time width Tp (one period of the carrier, Tp = 1/f0), carrying cos(w0 t),
w0 = 2 pi f0.  Instead of re-typing that expression, the test checks what
it implies:

  * the envelope peaks at 3 Tp, where the carrier is at a crest (3 Tp f0 =
    3), so g(3 Tp) = 1; one width away (2 Tp, 4 Tp) the carrier is again at
    a crest and g = e^{-1/2}; at 1 and 5 widths e^{-2}; at t = 0, e^{-9/2};
  * the carrier's zeros: g((m + 1/4) / f0) = 0 for every integer m;
  * the spectrum: the Fourier transform of the pulse is a Gaussian centred
    on f0, |G(f)| / |G(f0)| = exp(-2 pi^2 (f - f0)^2 Tp^2) (the negative-
    frequency image sits 2 f0 away, e^{-8 pi^2} below: negligible), computed
    here by numerical quadrature of the sampled pulse;
  * the printed width of the paper's run, Tp = 0.095238 ns, is one period
    of f0 = 10.5 GHz.

Planted mistakes (a sine carrier, a width without the factor 2, no delay,
f0 used as an angular frequency) each fail one of these.
"""
import math

import numpy as np
import pytest

from oracle.yee_llg import waveform

F0 = 10.5e9
TP = 1.0 / F0
T0 = 3.0 * TP


def _check(g):
    """Largest violation of the pinned properties by the pulse g(t)."""
    bad = 0.0
    for m, want in ((3, 1.0), (2, math.exp(-0.5)), (4, math.exp(-0.5)), (1, math.exp(-2.0)),
                    (5, math.exp(-2.0)), (0, math.exp(-4.5))):
        bad = max(bad, abs(g(m * TP) - want))
    for m in range(-2, 9):
        bad = max(bad, abs(g((m + 0.25) / F0)))
    # Fourier transform by the trapezoid rule over +-10 widths (the pulse is
    # below 1e-21 there); relative spectrum at offsets from f0
    t = np.linspace(T0 - 10 * TP, T0 + 10 * TP, 40001)
    gt = np.array([g(x) for x in t])
    dt = t[1] - t[0]

    def G(f):
        v = gt * np.exp(-2j * math.pi * f * t)
        return abs(dt * (v.sum() - 0.5 * (v[0] + v[-1])))

    g0 = G(F0)
    for df in (0.1, 0.25, 0.5, -0.3):
        f = F0 * (1 + df)
        want = math.exp(-2 * math.pi**2 * (f - F0) ** 2 * TP**2)
        bad = max(bad, abs(G(f) / g0 - want))
    # the peak of |G| lies at f0 (no larger value on a fine grid around it)
    fs = F0 * (1 + np.linspace(-0.5, 0.5, 201))
    Gs = np.array([G(f) for f in fs])
    bad = max(bad, abs(fs[int(np.argmax(Gs))] / F0 - 1))
    return bad


def test_pulse_has_the_stated_delay_width_and_carrier():
    assert _check(lambda t: waveform(t, F0, TP, T0)) < 1e-9


def test_printed_width_is_one_period():
    assert abs(0.095238e-9 * F0 - 1) < 1e-5


MUTANTS = {
    "sine carrier": lambda t: math.exp(-((t - T0) ** 2) / (2 * TP * TP)) * math.sin(2 * math.pi * F0 * t),
    "width without 2": lambda t: math.exp(-((t - T0) ** 2) / (TP * TP)) * math.cos(2 * math.pi * F0 * t),
    "no delay": lambda t: math.exp(-(t**2) / (2 * TP * TP)) * math.cos(2 * math.pi * F0 * t),
    "f0 as angular": lambda t: math.exp(-((t - T0) ** 2) / (2 * TP * TP)) * math.cos(F0 * t),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_fail_the_pin(name):
    assert _check(MUTANTS[name]) > 1e-2, name
