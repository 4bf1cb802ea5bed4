"""Independent brute-force evaluator for tiny grids (test helper).

Written separately from the oracle: voxel membership is decided by comparing
each point's voxel coordinate against every voxel's bounds (lo <= u < lo+1, no
floor), variances are exact rationals (fractions.Fraction), and MI comes from
sklearn's mutual_info_score on the contingency table.  Only the rotation
matrix is taken as an input (it is pinned on its own against scipy).
"""
from __future__ import annotations

from fractions import Fraction
import math

import numpy as np
from sklearn.metrics import mutual_info_score


def voxel_coords(P, origin, voxel, R=None, t=(0.0, 0.0, 0.0)):
    x, y, z = (np.asarray(P[a], np.float64) for a in range(3))
    s = 1.0 / voxel
    if R is None:
        w = [x, y, z]
    else:
        w = [(R[r][0] * x + R[r][1] * y) + R[r][2] * z for r in range(3)]
    c = [(t[a] - origin[a]) * s for a in range(3)]
    return [w[a] * s + c[a] for a in range(3)]


def voxel_table(P, origin, dims, voxel, R=None, t=(0.0, 0.0, 0.0)):
    """{(ix, iy, iz): [q values]} by enumeration over every voxel."""
    u = voxel_coords(P, origin, voxel, R, t)
    finite = np.isfinite(u[0]) & np.isfinite(u[1]) & np.isfinite(u[2])
    table = {}
    for iz in range(dims[2]):
        mz = finite & (u[2] >= iz) & (u[2] < iz + 1)
        for iy in range(dims[1]):
            my = mz & (u[1] >= iy) & (u[1] < iy + 1)
            for ix in range(dims[0]):
                m = my & (u[0] >= ix) & (u[0] < ix + 1)
                if m.any():
                    q = np.floor((u[2][m] - iz) * 1048576.0).astype(np.int64)
                    table[(ix, iy, iz)] = [int(v) for v in q]
    return table


def count_bin(n, edges):
    return sum(1 for e in edges if n >= int(e))


def zvar_bin(qs, edges):
    if not qs:
        return 0
    n = len(qs)
    mean = Fraction(sum(qs), n)
    var = Fraction(sum(q * q for q in qs), n) - mean * mean
    return 1 + sum(1 for e in edges if var >= int(e))


def bins_of(table, key, kind, edges):
    """kind "count" / "zvar" with that feature's edges; "joint" with the pair
    (count edges, z-variance edges): the occupied voxel's two bins numbered
    row-major over the occupied bins (count bins 1.., z-variance bins 1..),
    after the empty voxel's 0."""
    qs = table.get(key, [])
    if kind == "count":
        return count_bin(len(qs), edges)
    if kind == "zvar":
        return zvar_bin(qs, edges)
    if not qs:
        return 0
    ce, ze = edges
    n_z_occupied = len(ze) + 1
    return 1 + (count_bin(len(qs), ce) - 1) * n_z_occupied + (zvar_bin(qs, ze) - 1)


def box_of(table, dims):
    if not table:
        return [dims[0], dims[1], dims[2]], [-1, -1, -1]
    keys = np.array(list(table.keys()))
    return list(keys.min(axis=0)), list(keys.max(axis=0))


def evaluate(A, B, origin, dims, voxel, R, t, kind, nb, edges):
    """(hist [nb][nb], overlap lo/hi, MI) for one pose."""
    ta = voxel_table(A, origin, dims, voxel)
    tb = voxel_table(B, origin, dims, voxel, R, t)
    alo, ahi = box_of(ta, dims)
    blo, bhi = box_of(tb, dims)
    lo = [max(alo[a], blo[a], 0) for a in range(3)]
    hi = [min(ahi[a], bhi[a], dims[a] - 1) for a in range(3)]
    H = np.zeros((nb, nb), np.int64)
    if all(lo[a] <= hi[a] for a in range(3)):
        for iz in range(lo[2], hi[2] + 1):
            for iy in range(lo[1], hi[1] + 1):
                for ix in range(lo[0], hi[0] + 1):
                    key = (ix, iy, iz)
                    H[bins_of(ta, key, kind, edges), bins_of(tb, key, kind, edges)] += 1
    mi = 0.0 if H.sum() == 0 else float(mutual_info_score(None, None, contingency=H))
    return H, lo, hi, mi


NEAR_FACE_M = Fraction(1, 100000)


def near_face_count(B, origin, dims, voxel, R, t, lo, hi):
    """B points inside the overlap box [lo, hi] (voxel indices) whose distance
    to the nearest face of their voxel is under 1e-5 m, from exact rationals:
    the float32 coordinates, the entries of R and t and the voxel size are
    converted exactly, the voxel coordinate (R p + t - origin) / voxel is
    formed without rounding, and the voxel is its floor (no floating point
    decides anything here)."""
    if any(lo[a] > hi[a] for a in range(3)):
        return 0
    vox = Fraction(float(voxel))
    Rq = [[Fraction(float(R[r][c])) for c in range(3)] for r in range(3)]
    tq = [Fraction(float(t[a])) for a in range(3)]
    oq = [Fraction(float(origin[a])) for a in range(3)]
    P = np.asarray(B, np.float32)
    count = 0
    for i in range(P.shape[1]):
        p = [float(P[a, i]) for a in range(3)]
        if not all(math.isfinite(v) for v in p):
            continue
        pq = [Fraction(v) for v in p]
        near, inside = False, True
        for a in range(3):
            u = (sum(Rq[a][b] * pq[b] for b in range(3)) + tq[a] - oq[a]) / vox
            iu = math.floor(u)
            if not (lo[a] <= iu <= hi[a] and 0 <= iu < dims[a]):
                inside = False
                break
            fr = u - iu
            if min(fr, 1 - fr) * vox < NEAR_FACE_M:
                near = True
        if inside and near:
            count += 1
    return count
