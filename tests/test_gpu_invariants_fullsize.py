"""Invariants of the method checked at full size, where the oracle cannot run:
the 512 x 256 x 256 filter grid (FP64) after the benchmark's course of 610
steps and the 1024 x 512 x 512 grid (FP32 bulk mode) after 450 steps.

* Gauss law for B (Sec. 3.2.2, eq:iterate_H): per cell, the sum over its
  faces of normal B (mu0 (H + M_n) on magnetic faces, mu0 mu_r H elsewhere)
  is unchanged, because each sub-step changes H + M_n by -(dt/2 mu0) curl E
  and the discrete divergence of a discrete curl vanishes.
* Gauss law for D (Sec. 3.2.1, Step 2): at every interior node whose six
  edges carry no conductivity and no source current, the divergence of
  eps_e E is unchanged (eps_e: the 4-cell mean of eps_r times eps0).
* |M| = Ms_f on every magnetic face (the renormalisation of Sec. 3.2; Ms_f
  the 2-cell mean of the cell map, so interface faces carry Ms/2).
Bars: FP64 1e-10 of the field's own scale (max |B| / dx, max |D| / dx; the
changes accumulate rounding only); FP32 bulk mode 1e-4 for the two Gauss
laws (FP32 storage rounds E and H at every half step); |M| to 1e-13
relative in both (M is FP64 in both modes).
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
EPS0 = 8.8541878128e-12
MU0 = 1.25663706212e-6


def _div_B(sim, d):
    Bx, By, Bz = (sim.field(n) for n in ("Bx", "By", "Bz"))      # host layout [k][j][i]
    scale = max(float(np.max(np.abs(b))) for b in (Bx, By, Bz)) / min(d)
    div = np.empty((Bx.shape[0], By.shape[1] - 1, Bx.shape[2] - 1))
    for k in range(div.shape[0]):                               # plane by plane: bounded temporaries
        div[k] = ((Bx[k, :, 1:] - Bx[k, :, :-1]) / d[0] + (By[k, 1:, :] - By[k, :-1, :]) / d[1]
                  + (Bz[k + 1] - Bz[k]) / d[2])
    return div, scale


def _edge_mean4(cell, axis):
    """Mean of the 4 cells around the interior edges along `axis` (host
    layout [k][j][i]), on the interior nodes of the two other axes."""
    c = cell
    if axis == 0:     # x-edges (i+1/2, j, k): cells j-1..j, k-1..k
        return 0.25 * ((c[:-1, :-1, :] + c[:-1, 1:, :]) + (c[1:, :-1, :] + c[1:, 1:, :]))
    if axis == 1:     # y-edges: cells i-1..i, k-1..k
        return 0.25 * ((c[:-1, :, :-1] + c[:-1, :, 1:]) + (c[1:, :, :-1] + c[1:, :, 1:]))
    return 0.25 * ((c[:, :-1, :-1] + c[:, :-1, 1:]) + (c[:, 1:, :-1] + c[:, 1:, 1:]))


def _div_D(sim, cfg):
    """Divergence of eps_e E on the interior nodes (nz-1, ny-1, nx-1), the
    mask of nodes whose six edges are lossless and source-free, and the
    scale max |D| / dx."""
    d = cfg.d
    nx, ny, nz = cfg.n
    Ex, Ey, Ez = (sim.field(n) for n in ("Ex", "Ey", "Ez"))
    Dx = EPS0 * _edge_mean4(cfg.eps_r, 0) * Ex[1:-1, 1:-1, :]      # (nz-1, ny-1, nx)
    Dy = EPS0 * _edge_mean4(cfg.eps_r, 1) * Ey[1:-1, :, 1:-1]      # (nz-1, ny, nx-1)
    Dz = EPS0 * _edge_mean4(cfg.eps_r, 2) * Ez[:, 1:-1, 1:-1]      # (nz, ny-1, nx-1)
    del Ex, Ey, Ez
    scale = max(float(np.max(np.abs(a))) for a in (Dx, Dy, Dz)) / min(d)
    div = ((Dx[:, :, 1:] - Dx[:, :, :-1]) / d[0] + (Dy[:, 1:, :] - Dy[:, :-1, :]) / d[1]
           + (Dz[1:] - Dz[:-1]) / d[2])
    del Dx, Dy, Dz
    sx = _edge_mean4(cfg.sigma, 0) > 0
    sy = _edge_mean4(cfg.sigma, 1) > 0
    sz = _edge_mean4(cfg.sigma, 2) > 0
    bad = (sx[:, :, 1:] | sx[:, :, :-1]) | (sy[:, 1:, :] | sy[:, :-1, :]) | (sz[1:] | sz[:-1])
    src = cfg.source
    if src is not None:
        p = np.abs(src.profile) > 0                                # on the source component's edges
        if src.comp == 0:
            e = p[1:-1, 1:-1, :]
            bad |= e[:, :, 1:] | e[:, :, :-1]
        elif src.comp == 1:
            e = p[1:-1, :, 1:-1]
            bad |= e[:, 1:, :] | e[:, :-1, :]
        else:
            e = p[:, 1:-1, 1:-1]
            bad |= e[1:] | e[:-1]
    return div, ~bad, scale


def _face_Ms(cfg, f):
    """2-cell mean of the Ms map on the faces of family f (host layout),
    clamped at the PEC walls."""
    c = cfg.Ms
    ax = 2 - f                                                     # numpy axis of the face normal
    lo = np.concatenate([np.take(c, [0], axis=ax), c], axis=ax)
    hi = np.concatenate([c, np.take(c, [-1], axis=ax)], axis=ax)
    return 0.5 * (lo + hi)


def _check_M(sim, cfg):
    worst = 0.0
    for f in range(3):
        m = [sim.field("M" + "xyz"[f] + c) for c in "xyz"]
        nrm = np.sqrt(m[0] ** 2 + m[1] ** 2 + m[2] ** 2)
        del m
        ms = _face_Ms(cfg, f)
        mag = ms > 0
        assert np.array_equal(nrm > 0, mag), f
        worst = max(worst, float(np.max(np.abs(nrm[mag] - ms[mag]) / ms[mag])))
    return worst


def _run(cfg, precision, steps, tol_gauss):
    import paper_2103_12819_amd as mm
    print(f"invariants {cfg.name} {cfg.n} {precision}: {steps} steps", flush=True)
    sim = mm.from_config(cfg, precision=precision, with_probes=False)
    b0, _ = _div_B(sim, cfg.d)
    dd0, mask, _ = _div_D(sim, cfg)
    sim.step(steps)
    b1, sb = _div_B(sim, cfg.d)
    dB = float(np.max(np.abs(b1 - b0))) / sb
    del b0, b1
    dd1, _, sd = _div_D(sim, cfg)
    dD = float(np.max(np.abs((dd1 - dd0)[mask]))) / sd
    frac = float(np.mean(mask))
    del dd0, dd1, mask
    dM = _check_M(sim, cfg)
    sim.close()
    print(f"  div B change / scale {dB:.2e}, div D change / scale {dD:.2e} on {100 * frac:.1f} % of nodes, "
          f"max | |M| - Ms | / Ms {dM:.2e}", flush=True)
    assert sb > 0 and sd > 0 and frac > 0.1
    assert dB <= tol_gauss and dD <= tol_gauss and dM <= 1e-13, (dB, dD, dM)


def test_filter512_fp64_after_the_benchmark_course():
    _run(W.filter512(seed=0), "fp64", 610, 1e-10)


@pytest.mark.timeout(900)
def test_scale1024_fp32_after_450_steps():
    _run(W.scale1024(seed=0), "fp32", 450, 1e-4)
