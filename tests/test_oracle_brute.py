"""Brute force on tiny grids: one full step of the oracle (non-magnetic) against
scalar loops that spell out every neighbour index of the Yee updates.

The loops follow Sec. 3.1 (E on edges, H on faces, curls as differences of
the two neighbouring samples, eps and sigma on an edge the mean of its four
cells, mu on a face the mean of its two cells, clamped at a PEC wall) and
Sec. 3.2.1 (H half step, E step with the time-centred conductivity term, H
half step), written per entry with explicit index arithmetic and no array
shifts, so a shifted, transposed or sign-flipped index set in the oracle's
vectorised helpers shows up entry by entry.  3 x 2 x 2 and 2 x 3 x 2 grids,
PEC and periodic axes, anisotropic spacings, random fields and materials.
"""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import Simulation
from oracle.yee_llg import EPS0, MU0


def _brute_step(n, d, dt, per, eps_r, sigma, mu_r, E, H):
    """One step from E, H (lists of [i, j, k] arrays) by scalar loops."""
    nx, ny, nz = n
    N = [n[a] if per[a] else n[a] + 1 for a in range(3)]

    def wrap(v, a):
        return v % n[a] if per[a] else v

    def cell(arr, i, j, k):
        # clamp at a PEC wall, wrap on a periodic axis
        q = [i, j, k]
        for a in range(3):
            q[a] = q[a] % n[a] if per[a] else min(max(q[a], 0), n[a] - 1)
        return arr[q[0], q[1], q[2]]

    def edge_interior(c, q):
        return all(per[a] or (0 < q[a] < n[a]) for a in range(3) if a != c)

    def face_interior(f, q):
        return per[f] or (0 < q[f] < n[f])

    def mu_face(f, q):
        lo = list(q)
        lo[f] -= 1
        return MU0 * 0.5 * (cell(mu_r, *lo) + cell(mu_r, *q))

    def coef_edge(c, q):
        t1, t2 = [a for a in range(3) if a != c]
        vals_e, vals_s = [], []
        for s1, s2 in ((1, 1), (0, 1), (1, 0), (0, 0)):
            p = list(q)
            p[t1] -= s1
            p[t2] -= s2
            vals_e.append(cell(eps_r, *p))
            vals_s.append(cell(sigma, *p))
        ee = EPS0 * 0.25 * sum(vals_e)
        se = 0.25 * sum(vals_s)
        den = ee / dt + se / 2
        return (ee / dt - se / 2) / den, 1.0 / den

    def curl_e(Ea, f, i, j, k):
        dx, dy, dz = d
        if f == 0:
            return ((Ea[2][i, wrap(j + 1, 1), k] - Ea[2][i, j, k]) / dy
                    - (Ea[1][i, j, wrap(k + 1, 2)] - Ea[1][i, j, k]) / dz)
        if f == 1:
            return ((Ea[0][i, j, wrap(k + 1, 2)] - Ea[0][i, j, k]) / dz
                    - (Ea[2][wrap(i + 1, 0), j, k] - Ea[2][i, j, k]) / dx)
        return ((Ea[1][wrap(i + 1, 0), j, k] - Ea[1][i, j, k]) / dx
                - (Ea[0][i, wrap(j + 1, 1), k] - Ea[0][i, j, k]) / dy)

    def curl_h(Ha, c, i, j, k):
        dx, dy, dz = d
        if c == 0:
            return ((Ha[2][i, j, k] - Ha[2][i, wrap(j - 1, 1), k]) / dy
                    - (Ha[1][i, j, k] - Ha[1][i, j, wrap(k - 1, 2)]) / dz)
        if c == 1:
            return ((Ha[0][i, j, k] - Ha[0][i, j, wrap(k - 1, 2)]) / dz
                    - (Ha[2][i, j, k] - Ha[2][wrap(i - 1, 0), j, k]) / dx)
        return ((Ha[1][i, j, k] - Ha[1][wrap(i - 1, 0), j, k]) / dx
                - (Ha[0][i, j, k] - Ha[0][i, wrap(j - 1, 1), k]) / dy)

    def h_half(Hin, Ea):
        Hout = [a.copy() for a in Hin]
        for f in range(3):
            for q in itertools.product(*[range(s) for s in Hin[f].shape]):
                if face_interior(f, q):
                    Hout[f][q] = Hin[f][q] - (0.5 * dt / mu_face(f, q)) * curl_e(Ea, f, *q)
        return Hout

    Hh = h_half(H, E)
    E1 = [a.copy() for a in E]
    for c in range(3):
        for q in itertools.product(*[range(s) for s in E[c].shape]):
            if edge_interior(c, q):
                ca, cb = coef_edge(c, q)
                E1[c][q] = ca * E[c][q] + cb * curl_h(Hh, c, *q)
    H1 = h_half(Hh, E1)
    return E1, H1


@pytest.mark.parametrize("n,per", [((3, 2, 2), (False, False, False)), ((2, 3, 2), (True, False, True)),
                                   ((3, 2, 2), (False, True, False)), ((2, 2, 3), (True, True, True))])
def test_one_step_matches_scalar_loops(n, per):
    rng = np.random.default_rng(sum(n) + 7 * sum(per))
    d = (1.1e-6, 0.8e-6, 1.3e-6)
    dt = W.cfl_dt(0.9, *d)
    shp = (n[2], n[1], n[0])
    eps_r = rng.uniform(1, 5, shp)
    sigma = rng.uniform(0, 2e4, shp)
    mu_r = rng.uniform(1, 3, shp)
    sim = Simulation(n, d, dt, eps_r=eps_r, sigma=sigma, mu_r=mu_r, periodic=per)
    E0 = [rng.normal(0, 1e4, W.edge_shape(n, per, c)) for c in range(3)]
    H0 = [rng.normal(0, 30, W.face_shape(n, per, c)) for c in range(3)]
    sim.set_fields(E0, H0)
    E_in = [a.copy() for a in sim.E]          # [i, j, k], PEC entries zeroed
    H_in = [a.copy() for a in sim.H]
    sim.step(1)
    to_ijk = lambda a: np.ascontiguousarray(a.transpose(2, 1, 0))  # noqa: E731
    E1, H1 = _brute_step(n, d, dt, per, to_ijk(eps_r), to_ijk(sigma), to_ijk(mu_r), E_in, H_in)
    for c in range(3):
        scale_e = np.max(np.abs(E1[c])) + 1e-300
        scale_h = np.max(np.abs(H1[c])) + 1e-300
        assert np.max(np.abs(sim.E[c] - E1[c])) <= 1e-13 * scale_e, ("E", c)
        assert np.max(np.abs(sim.H[c] - H1[c])) <= 1e-13 * scale_h, ("H", c)
        assert np.count_nonzero(E1[c]) > 0 and np.count_nonzero(H1[c]) > 0
