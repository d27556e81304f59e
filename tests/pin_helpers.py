"""Independent plain-loop helpers used by the oracle pins.

These are written from the definitions (discrete divergence, energy weights,
rotation formulas) with explicit loops over small grids; they do not call
the oracle's operators, so a mistake in the oracle's vectorised indexing
shows up as a disagreement.
"""
import math

import numpy as np

MU0 = 1.25663706212e-6
EPS0 = 8.8541878128e-12


def rotate(v, axis, angle):
    """Rodrigues rotation of vector v about unit `axis` by `angle` (right-handed)."""
    k = np.asarray(axis, float) / np.linalg.norm(axis)
    v = np.asarray(v, float)
    return (v * math.cos(angle) + np.cross(k, v) * math.sin(angle)
            + k * np.dot(k, v) * (1.0 - math.cos(angle)))


def cell_at(a, i, j, k, n, per):
    """Cell value with periodic wrap / PEC clamp (clamp only used at walls)."""
    idx = []
    for v, nn, p in zip((i, j, k), n, per):
        if p:
            v %= nn
        else:
            v = min(max(v, 0), nn - 1)
        idx.append(v)
    # host layout: a[k, j, i]
    return a[idx[2], idx[1], idx[0]]


def eps_edges(eps_r, n, per, comp):
    """eps0 * mean of the four cells sharing each edge of component `comp`
    (ijk-indexed output on the edge extent)."""
    nx, ny, nz = n
    ext = [n[a] if (a == comp or per[a]) else n[a] + 1 for a in range(3)]
    out = np.zeros(ext)
    t = [a for a in range(3) if a != comp]
    for i in range(ext[0]):
        for j in range(ext[1]):
            for k in range(ext[2]):
                s = 0.0
                for d1 in (-1, 0):
                    for d2 in (-1, 0):
                        p = [i, j, k]
                        p[t[0]] += d1
                        p[t[1]] += d2
                        s += cell_at(eps_r, p[0], p[1], p[2], n, per)
                out[i, j, k] = EPS0 * s / 4.0
    return out


def face_mean(cmap, n, per, fam):
    """Mean of the two cells sharing each face of family `fam` (ijk-indexed)."""
    ext = [(n[a] if per[a] else n[a] + 1) if a == fam else n[a] for a in range(3)]
    out = np.zeros(ext)
    for i in range(ext[0]):
        for j in range(ext[1]):
            for k in range(ext[2]):
                p = [i, j, k]
                q = list(p)
                q[fam] -= 1
                out[i, j, k] = 0.5 * (cell_at(cmap, *p, n, per) + cell_at(cmap, *q, n, per))
    return out


def ijk(a):
    return np.asarray(a).transpose(2, 1, 0)


def div_faces(B, n, d, per):
    """Per-cell divergence of a face-normal field B = (Bx, By, Bz) (ijk arrays)."""
    nx, ny, nz = n
    out = np.zeros((nx, ny, nz))
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                ip = (i + 1) % B[0].shape[0]
                jp = (j + 1) % B[1].shape[1]
                kp = (k + 1) % B[2].shape[2]
                out[i, j, k] = ((B[0][ip, j, k] - B[0][i, j, k]) / d[0]
                                + (B[1][i, jp, k] - B[1][i, j, k]) / d[1]
                                + (B[2][i, j, kp] - B[2][i, j, k]) / d[2])
    return out


def div_edges(D, n, d, per):
    """Per-node divergence of an edge field D = (Dx, Dy, Dz) (ijk arrays)."""
    ext = [n[a] if per[a] else n[a] + 1 for a in range(3)]
    out = np.zeros(ext)
    for i in range(ext[0]):
        for j in range(ext[1]):
            for k in range(ext[2]):
                s = 0.0
                for ax, arr in enumerate(D):
                    p = [i, j, k]
                    q = [i, j, k]
                    q[ax] -= 1
                    hi = arr[tuple(p)] if p[ax] < arr.shape[ax] else 0.0
                    if q[ax] < 0:
                        lo = arr[tuple(q)] if per[ax] else 0.0
                    else:
                        lo = arr[tuple(q)]
                    s += (hi - lo) / d[ax]
                out[i, j, k] = s
    return out


def curl_E_faces(E, n, d, per):
    """Curl of E at faces by explicit loops (ijk arrays in and out)."""
    ext = lambda f: [(n[a] if per[a] else n[a] + 1) if a == f else n[a] for a in range(3)]
    out = [np.zeros(ext(f)) for f in range(3)]

    def ge(c, i, j, k):
        a = E[c]
        p = [i, j, k]
        for ax in range(3):
            if per[ax]:
                p[ax] %= a.shape[ax]
        return a[tuple(p)]

    for f in range(3):
        o = out[f]
        u, v = (f + 1) % 3, (f + 2) % 3
        for i in range(o.shape[0]):
            for j in range(o.shape[1]):
                for k in range(o.shape[2]):
                    p = [i, j, k]
                    pu = list(p)
                    pu[u] += 1
                    pv = list(p)
                    pv[v] += 1
                    o[i, j, k] = ((ge(v, *pu) - ge(v, *p)) / d[u]
                                  - (ge(u, *pv) - ge(u, *p)) / d[v])
    return out
