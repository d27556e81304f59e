"""The coupled convergence problem of Sec. 5.1, set up for the oracle.

Fully periodic cube of side L = 0.1 m centred on the origin; cosine E and H
fields of eq:convergeE / eq:convergeH placed at their Yee locations;
Gaussian bumps in sigma, eps, Ms, alpha and gamma at cell centres; Mx = Ms,
no bias; CFL 0.9 on the vacuum light speed; runs of 5 * N/32 steps reach the
same physical time.  Errors follow the paper: mean absolute difference
between a run and the next finer one restricted to the coarse locations
(4 fine faces per coarse face, 2 fine edges per coarse edge).
"""
import math

import numpy as np

import workloads as W
from oracle import from_config

L = 0.1


def build(N, tol=1e-6, side=L, scheme=2):
    """`side` is the edge length of the periodic cube centred on the origin."""
    return from_config(W.convergence_cube(N, side=side, tol=tol), with_probes=False, scheme=scheme)


def run(N, side=L, scheme=2, steps=None):
    """Fields after `steps` steps (default 5 N / 32, the paper's common time)."""
    sim = build(N, side=side, scheme=scheme)
    sim.step(5 * N // 32 if steps is None else steps)
    out = {}
    for nm in ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz"):
        out[nm] = sim.field(nm).transpose(2, 1, 0)
    for f in "xyz":
        for c in "xyz":
            out["M" + f + c] = sim.field("M" + f + c).transpose(2, 1, 0)
    return out


def restrict_edge(a, comp):
    """Mean of the 2 fine edges along `comp` under each coarse edge."""
    sl0 = [slice(0, None, 2)] * 3
    sl1 = [slice(0, None, 2)] * 3
    sl1[comp] = slice(1, None, 2)
    return 0.5 * (a[tuple(sl0)] + a[tuple(sl1)])


def restrict_face(a, fam):
    """Mean of the 4 fine faces covering each coarse face of family `fam`."""
    u, v = [ax for ax in range(3) if ax != fam]
    acc = 0.0
    for du in (0, 1):
        for dv in (0, 1):
            sl = [slice(0, None, 2)] * 3
            sl[u] = slice(du, None, 2)
            sl[v] = slice(dv, None, 2)
            acc = acc + a[tuple(sl)]
    return 0.25 * acc


def l1_error(coarse, fine):
    err = {}
    for nm, a in coarse.items():
        if nm[0] == "E":
            r = restrict_edge(fine[nm], "xyz".index(nm[1]))
        else:
            r = restrict_face(fine[nm], "xyz".index(nm[1]))
        err[nm] = float(np.mean(np.abs(r - a)))
    return err
