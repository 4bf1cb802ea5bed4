"""Plain FP64 CPU oracle for mutual-information scan alignment.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  The product library never imports,
links or calls anything here, and nothing here imports the product package.

The arithmetic lives in ``mi_oracle.c`` (compiled with gcc, no FP contraction);
this module only marshals numpy arrays.  Every function cites the part of the
paper (Mehta, McBride, Pandey, arXiv 1709.06948) that it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mi_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

FEAT_COUNT = 1
FEAT_ZVAR = 2
FEAT_JOINT = 4
NSTATS = 11
STATS_FIELDS = ("lo_x", "lo_y", "lo_z", "hi_x", "hi_y", "hi_z", "n_overlap", "n_in_grid",
                "n_out_of_grid", "n_nonfinite", "n_near_face")


def build(force: bool = False) -> str:
    """Compile mi_oracle.c with gcc (plain -O2, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Grid(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("dims", C.c_int32 * 3), ("voxel", C.c_double),
                ("features", C.c_uint32), ("nb_count", C.c_int32),
                ("count_edges", C.POINTER(C.c_uint32)), ("nb_zvar", C.c_int32),
                ("zvar_edges", C.POINTER(C.c_uint64))]


_lib = None


def _L():
    global _lib
    if _lib is None:
        lib = C.CDLL(build())
        dp, fp, i64p, u32p, u64p, u8p, i32p = (C.POINTER(C.c_double), C.POINTER(C.c_float),
                                               C.POINTER(C.c_int64), C.POINTER(C.c_uint32),
                                               C.POINTER(C.c_uint64), C.POINTER(C.c_uint8),
                                               C.POINTER(C.c_int32))
        gp = C.POINTER(_Grid)
        lib.mio_pose_matrix.argtypes = [dp, dp]
        lib.mio_default_count_edges.argtypes = [C.c_int32, u32p]
        lib.mio_default_count_edges.restype = C.c_int
        lib.mio_default_zvar_edges.argtypes = [C.c_double, C.c_int32, u64p]
        lib.mio_default_zvar_edges.restype = C.c_int
        lib.mio_mi_from_hist.argtypes = [u32p, C.c_int32]
        lib.mio_mi_from_hist.restype = C.c_double
        lib.mio_entropies_from_hist.argtypes = [u32p, C.c_int32, dp]
        lib.mio_scan_features.argtypes = [gp, fp, C.c_int64, dp, u32p, u64p, u64p, u8p, i32p, i64p]
        lib.mio_scan_features.restype = C.c_int
        lib.mio_eval_poses.argtypes = [gp, fp, C.c_int64, fp, C.c_int64, dp, C.c_int64, dp, u32p,
                                       i64p, C.c_int32]
        lib.mio_eval_poses.restype = C.c_int
        lib.mio_argmax.argtypes = [dp, C.c_int64]
        lib.mio_argmax.restype = C.c_int64
        lib.mio_grid_poses.argtypes = [dp, dp, i32p, dp]
        lib.mio_grid_poses.restype = C.c_int64
        lib.mio_align_c2f.argtypes = [gp, fp, C.c_int64, fp, C.c_int64, dp, dp, i32p, C.c_int32,
                                      C.c_double, C.c_int32, dp, dp, dp, C.c_int32]
        lib.mio_weighted.argtypes = [dp, C.c_int64, C.c_int32, dp, dp]
        lib.mio_align_c2f.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class Grid:
    """Voxel grid R_v over scan A's frame plus the feature description
    (Sec. III-A; Sec. IV uses R_v = 1 m).  Features: bitmask of FEAT_COUNT
    (number of points, MI-N), FEAT_ZVAR (variance of z, MI-VARZ) and
    FEAT_JOINT (the pair of the two bins as one value), at most two of them;
    the joint feature bins its parts with nb_count and nb_zvar."""

    def __init__(self, origin, dims, voxel, features=FEAT_COUNT, nb_count=16, nb_zvar=32,
                 count_edges=None, zvar_edges=None):
        self.origin = tuple(float(v) for v in origin)
        self.dims = tuple(int(v) for v in dims)
        self.voxel = float(voxel)
        self.features = int(features)
        self.nb_count = int(nb_count)
        self.nb_zvar = int(nb_zvar)
        L = _L()
        if count_edges is None:
            count_edges = np.zeros(max(self.nb_count - 1, 1), np.uint32)
            if L.mio_default_count_edges(self.nb_count, _ptr(count_edges, C.c_uint32)):
                raise ValueError("bad nb_count")
        if zvar_edges is None:
            zvar_edges = np.zeros(max(self.nb_zvar - 2, 1), np.uint64)
            if (self.features & (FEAT_ZVAR | FEAT_JOINT)) and self.nb_zvar >= 3 and \
                    L.mio_default_zvar_edges(self.voxel, self.nb_zvar, _ptr(zvar_edges, C.c_uint64)):
                raise ValueError("bad nb_zvar / voxel for default z-variance edges")
        self.count_edges = np.ascontiguousarray(count_edges, np.uint32)
        self.zvar_edges = np.ascontiguousarray(zvar_edges, np.uint64)
        g = _Grid()
        g.origin[:] = self.origin
        g.dims[:] = self.dims
        g.voxel = self.voxel
        g.features = self.features
        g.nb_count = self.nb_count
        g.count_edges = _ptr(self.count_edges, C.c_uint32)
        g.nb_zvar = self.nb_zvar
        g.zvar_edges = _ptr(self.zvar_edges, C.c_uint64)
        self._g = g

    @property
    def V(self) -> int:
        return self.dims[0] * self.dims[1] * self.dims[2]

    @property
    def feature_list(self):
        out = []
        if self.features & FEAT_COUNT:
            out.append((FEAT_COUNT, self.nb_count))
        if self.features & FEAT_ZVAR:
            out.append((FEAT_ZVAR, self.nb_zvar))
        if self.features & FEAT_JOINT:
            out.append((FEAT_JOINT, 1 + (self.nb_count - 1) * (self.nb_zvar - 1)))
        return out


def _soa(points) -> np.ndarray:
    p = np.ascontiguousarray(points, dtype=np.float32)
    if p.ndim != 2 or p.shape[0] != 3:
        raise ValueError("points must be float32 SoA [3, n]")
    return p


def pose_matrix(eta) -> np.ndarray:
    """R of pose eta = [tx,ty,tz,roll,pitch,yaw] as Rz(yaw) Ry(pitch) Rx(roll)
    (Sec. I parameterisation; Sec. III-A rigid transform T)."""
    e = np.ascontiguousarray(eta, np.float64)
    R = np.zeros(9, np.float64)
    _L().mio_pose_matrix(_ptr(e, C.c_double), _ptr(R, C.c_double))
    return R.reshape(3, 3)


def mi_from_hist(H) -> float:
    """Eq. 2 with Eqs. 3-5 on a joint histogram (rows = A bins, cols = B bins)."""
    H = np.ascontiguousarray(H, np.uint32)
    return float(_L().mio_mi_from_hist(_ptr(H, C.c_uint32), H.shape[0]))


def entropies_from_hist(H):
    """(H(X), H(Y), H(X,Y)) of Eqs. 3-5 for a joint histogram."""
    H = np.ascontiguousarray(H, np.uint32)
    out = np.zeros(3, np.float64)
    _L().mio_entropies_from_hist(_ptr(H, C.c_uint32), H.shape[0], _ptr(out, C.c_double))
    return tuple(out)


def scan_features(grid: Grid, points, eta=None):
    """Voxel-point mapping and per-voxel feature map of one scan (Alg. 1
    initialisation; with eta the scan is first moved by the pose, as in the
    Alg. 1 loop).  Returns dict with cnt, s1, s2 (dense [V]), bins [nfeat][V],
    box (lo[3], hi[3]) and counters (in, out, nonfinite, occupied)."""
    p = _soa(points)
    V = grid.V
    nf = len(grid.feature_list)
    cnt = np.zeros(V, np.uint32)
    s1 = np.zeros(V, np.uint64)
    s2 = np.zeros(V, np.uint64)
    bins = np.zeros((nf, V), np.uint8)
    box = np.zeros(6, np.int32)
    ctr = np.zeros(4, np.int64)
    e = None if eta is None else np.ascontiguousarray(eta, np.float64)
    rc = _L().mio_scan_features(C.byref(grid._g), _ptr(p, C.c_float), p.shape[1],
                                None if e is None else _ptr(e, C.c_double),
                                _ptr(cnt, C.c_uint32), _ptr(s1, C.c_uint64), _ptr(s2, C.c_uint64),
                                _ptr(bins, C.c_uint8), _ptr(box, C.c_int32), _ptr(ctr, C.c_int64))
    if rc:
        raise ValueError(f"mio_scan_features failed ({rc})")
    return dict(cnt=cnt, s1=s1, s2=s2, bins=bins, box=box, counters=ctr)


def eval_poses(grid: Grid, A, B, poses, want_hist=False, want_stats=False, nthreads=0):
    """MI (Eq. 2) of every candidate pose (Alg. 1 loop body per pose).
    Returns (mi [nfeat][K], hists list per feature [K][nb][nb] or None,
    stats [K][11] or None)."""
    A = _soa(A)
    B = _soa(B)
    P = np.ascontiguousarray(poses, np.float64).reshape(-1, 6)
    K = P.shape[0]
    fl = grid.feature_list
    mi = np.zeros((len(fl), K), np.float64)
    htot = sum(K * nb * nb for _, nb in fl)
    hist = np.zeros(htot, np.uint32) if want_hist else None
    stats = np.zeros((K, NSTATS), np.int64) if want_stats else None
    rc = _L().mio_eval_poses(C.byref(grid._g), _ptr(A, C.c_float), A.shape[1], _ptr(B, C.c_float),
                             B.shape[1], _ptr(P, C.c_double), K, _ptr(mi, C.c_double),
                             None if hist is None else _ptr(hist, C.c_uint32),
                             None if stats is None else _ptr(stats, C.c_int64), int(nthreads))
    if rc:
        raise RuntimeError(f"mio_eval_poses failed ({rc})")
    hists = None
    if want_hist:
        hists, off = [], 0
        for _, nb in fl:
            hists.append(hist[off:off + K * nb * nb].reshape(K, nb, nb))
            off += K * nb * nb
    return mi, hists, stats


def argmax(mi) -> int:
    """Smallest pose index within 1e-12 of the maximum MI (Eq. 1 over a finite set)."""
    m = np.ascontiguousarray(mi, np.float64)
    return int(_L().mio_argmax(_ptr(m, C.c_double), m.shape[0]))


def weighted(mi, weights) -> np.ndarray:
    """Weighted objective w0 * MI_0 + w1 * MI_1 of every pose (products rounded,
    then the sum), for mi [nfeat][K]."""
    m = np.ascontiguousarray(mi, np.float64)
    w = np.ascontiguousarray(weights, np.float64).reshape(2)
    out = np.zeros(m.shape[1], np.float64)
    _L().mio_weighted(_ptr(m, C.c_double), m.shape[1], m.shape[0], _ptr(w, C.c_double),
                      _ptr(out, C.c_double))
    return out


def grid_poses(center, half, samples) -> np.ndarray:
    """Pose grid of one coarse-to-fine level (row-major, yaw fastest)."""
    c = np.ascontiguousarray(center, np.float64)
    h = np.ascontiguousarray(half, np.float64)
    s = np.ascontiguousarray(samples, np.int32)
    K = int(np.prod(s))
    P = np.zeros((K, 6), np.float64)
    _L().mio_grid_poses(_ptr(c, C.c_double), _ptr(h, C.c_double), _ptr(s, C.c_int32),
                        _ptr(P, C.c_double))
    return P


def align_c2f(grid: Grid, A, B, init, half, samples, levels, shrink, feature_slot=0, nthreads=0,
              weights=None):
    """Coarse-to-fine grid maximisation of Eq. 1 (stand-in for the Sec. III-B
    search) for feature slot feature_slot, or of the weighted objective when
    weights (w0, w1) are given.  Returns (pose[6], objective at that pose)."""
    A = _soa(A)
    B = _soa(B)
    i0 = np.ascontiguousarray(init, np.float64)
    h0 = np.ascontiguousarray(half, np.float64)
    s = np.ascontiguousarray(samples, np.int32)
    out = np.zeros(6, np.float64)
    best = np.zeros(1, np.float64)
    w = None if weights is None else np.ascontiguousarray(weights, np.float64).reshape(2)
    slot = -1 if w is not None else int(feature_slot)
    rc = _L().mio_align_c2f(C.byref(grid._g), _ptr(A, C.c_float), A.shape[1], _ptr(B, C.c_float),
                            B.shape[1], _ptr(i0, C.c_double), _ptr(h0, C.c_double),
                            _ptr(s, C.c_int32), int(levels), float(shrink), slot,
                            None if w is None else _ptr(w, C.c_double),
                            _ptr(out, C.c_double), _ptr(best, C.c_double), int(nthreads))
    if rc:
        raise RuntimeError(f"mio_align_c2f failed ({rc})")
    return out, float(best[0])


# --------------------------------------------------------------- simplex search

NM_REFLECT, NM_EXPAND, NM_CONTRACT, NM_SHRINK = 1.0, 2.0, 0.5, 0.5


def nelder_mead(f, x0, steps, max_iter, ftol, xtol):
    """Nelder-Mead simplex minimisation of f (Sec. III-B: a simplex of N+1
    points improved by reflecting, expanding, contracting or shrinking; the
    method of the cited Nelder & Mead paper with its usual coefficients
    1, 2, 1/2, 1/2).  Vertex 0 is x0, vertex i is x0 + steps[i-1] along axis
    i-1.  Vertices are kept ordered by f, ties by age (stable sort).  Each
    iteration reflects the worst vertex through the centroid of the others;
    a reflection better than the best is tried expanded; one that is no better
    than the second worst is contracted (outside if it beats the worst, else
    inside), and a failed contraction shrinks every vertex halfway towards the
    best.  Stops after max_iter iterations, or when every vertex is within
    xtol (max norm) of the best and every value within ftol of the best.
    f takes a list of points and returns their values (so a caller may batch).
    Returns (best point, best value, iterations)."""
    x0 = np.asarray(x0, np.float64)
    n = x0.size
    simplex = [x0.copy()]
    for i in range(n):
        v = x0.copy()
        v[i] = v[i] + steps[i]
        simplex.append(v)
    values = list(f(simplex))
    it = 0
    while True:
        order = sorted(range(n + 1), key=lambda k: values[k])  # stable
        simplex = [simplex[k] for k in order]
        values = [values[k] for k in order]
        best, worst = values[0], values[n]
        spread_x = max(float(np.max(np.abs(simplex[k] - simplex[0]))) for k in range(1, n + 1))
        spread_f = max(abs(values[k] - best) for k in range(1, n + 1))
        if it >= max_iter or (spread_x <= xtol and spread_f <= ftol):
            return simplex[0], values[0], it
        it += 1
        centroid = simplex[0].copy()
        for k in range(1, n):
            centroid = centroid + simplex[k]
        centroid = centroid / n
        xw = simplex[n]
        xr = centroid + NM_REFLECT * (centroid - xw)
        xe = centroid + NM_EXPAND * (xr - centroid)
        xoc = centroid + NM_CONTRACT * (xr - centroid)
        xic = centroid + NM_CONTRACT * (xw - centroid)
        fr, fe, foc, fic = f([xr, xe, xoc, xic])
        second = values[n - 1]
        if fr < best:
            if fe < fr:
                simplex[n], values[n] = xe, fe
            else:
                simplex[n], values[n] = xr, fr
            continue
        if fr < second:
            simplex[n], values[n] = xr, fr
            continue
        if fr < worst:
            if foc <= fr:
                simplex[n], values[n] = xoc, foc
                continue
        elif fic < worst:
            simplex[n], values[n] = xic, fic
            continue
        shrunk = [simplex[0] + NM_SHRINK * (simplex[k] - simplex[0]) for k in range(1, n + 1)]
        fs = list(f(shrunk))
        simplex = [simplex[0]] + shrunk
        values = [values[0]] + fs


def align_nelder_mead(grid: Grid, A, B, init, steps, max_iter, ftol, xtol, feature_slot=0,
                      nthreads=0, weights=None):
    """Alg. 1 with the Nelder-Mead update of Sec. III-B: maximise Eq. 1 (MI of
    feature slot `feature_slot`, or the weighted objective when weights are
    given) over the pose from T_o = init.  Returns (pose[6], objective,
    iterations)."""
    def cost(points):
        mi, _, _ = eval_poses(grid, A, B, np.asarray(points), nthreads=nthreads)
        obj = mi[feature_slot] if weights is None else weighted(mi, weights)
        return [-float(v) for v in obj]
    x, v, it = nelder_mead(cost, init, steps, max_iter, ftol, xtol)
    return x, -v, it
