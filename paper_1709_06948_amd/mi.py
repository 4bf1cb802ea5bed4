"""Python binding of libmi355.so (include/mi.h): argument marshalling only.

Every step of the hot path runs in the library's HIP kernels; torch provides
device memory (workspaces, inputs, outputs) and the current HIP stream.
Importing this module loads the native library and raises if it is missing:
there is no CPU fallback.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import functools
import inspect
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmi355.so")

MI_OK, MI_E_INVALID, MI_E_WORKSPACE, MI_E_DEVICE, MI_E_UNSUPPORTED = 0, -1, -2, -3, -4
FEAT_COUNT, FEAT_ZVAR, FEAT_JOINT = 1, 2, 4
SLOT_WEIGHTED = -1         # searches maximise w0 * MI_0 + w1 * MI_1
EVAL_NEAR_FACE = 1
EVAL_PER_POSE = 2          # force per-pose bucketing
EVAL_SHARED_FRAMES = 4     # force shared rotated frames
MAX_POINTS = 1 << 20

STATS_DTYPE = np.dtype([("lo", "<i4", 3), ("hi", "<i4", 3), ("n_overlap", "<i8"),
                        ("n_in_grid", "<i8"), ("n_out_of_grid", "<i8"), ("n_nonfinite", "<i8"),
                        ("n_near_face", "<i8")])
assert STATS_DTYPE.itemsize == 64


class MIError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


class _GridDesc(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("dims", C.c_int32 * 3), ("voxel", C.c_double),
                ("features", C.c_uint32), ("nbins_count", C.c_int32),
                ("count_edges", C.POINTER(C.c_uint32)), ("nbins_zvar", C.c_int32),
                ("zvar_edges", C.POINTER(C.c_uint64))]


class _C2F(C.Structure):
    _fields_ = [("half_range", C.c_double * 6), ("samples", C.c_int32 * 6), ("levels", C.c_int32),
                ("shrink", C.c_double), ("feature_slot", C.c_int32), ("weight", C.c_double * 2)]


class _Profile(C.Structure):
    _fields_ = [("frames_ms", C.c_double), ("eval_ms", C.c_double), ("plain_ms", C.c_double),
                ("frame_launches", C.c_int64), ("eval_launches", C.c_int64),
                ("plain_poses", C.c_int64), ("poses", C.c_int64), ("point_poses", C.c_int64)]


class _WorkItem(C.Structure):
    _fields_ = [("ref", C.c_void_p), ("xyz_b", C.c_void_p), ("n_b", C.c_int64),
                ("poses", C.POINTER(C.c_double)), ("K", C.c_int64), ("mi_out", C.c_void_p),
                ("argmax_out", C.c_void_p), ("hist_out", C.c_void_p), ("stats_out", C.c_void_p)]


class _NMDesc(C.Structure):
    _fields_ = [("step", C.c_double * 6), ("max_iter", C.c_int32), ("ftol", C.c_double),
                ("xtol", C.c_double), ("feature_slot", C.c_int32), ("weight", C.c_double * 2)]


class _ServerDesc(C.Structure):
    _fields_ = [("arena", C.c_void_p), ("arena_bytes", C.c_size_t), ("step_bytes", C.c_size_t),
                ("max_active", C.c_int32)]


class _Request(C.Structure):
    _fields_ = [("grid", _GridDesc), ("xyz_a", C.c_void_p), ("n_a", C.c_int64),
                ("xyz_b", C.c_void_p), ("n_b", C.c_int64), ("init", C.c_double * 6),
                ("search", _C2F)]


class _RequestState(C.Structure):
    _fields_ = [("state", C.c_int32), ("levels_done", C.c_int32), ("status", C.c_int32),
                ("pad", C.c_int32), ("pose", C.c_double * 6), ("mi", C.c_double),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]


class _Tuning(C.Structure):
    _fields_ = [("waves", C.c_int32), ("hash_bytes", C.c_int32), ("hist_copies", C.c_int32),
                ("stripe_rows", C.c_int32), ("wgs_per_cu", C.c_int32)]


class _AutotuneReport(C.Structure):
    _fields_ = [("best", _Tuning), ("best_ms", C.c_double), ("start_ms", C.c_double),
                ("tried", C.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m "
                          "paper_1709_06948_amd.build` (there is no fallback path)")
    L = C.CDLL(LIB_PATH)
    vp, i64, u32, sz, st = C.c_void_p, C.c_int64, C.c_uint32, C.c_size_t, C.c_int32
    dp = C.POINTER(C.c_double)
    sig = {
        "mi_status_str": ([st], C.c_char_p),
        "mi_last_error": ([], C.c_char_p),
        "mi_tuning_set": ([C.POINTER(_Tuning)], st),
        "mi_profile_enable": ([st], st),
        "mi_profile_read": ([C.POINTER(_Profile)], st),
        "mi_tuning_get": ([C.POINTER(_Tuning)], st),
        "mi_grid_create": ([C.POINTER(_GridDesc), C.POINTER(vp)], st),
        "mi_grid_destroy": ([vp], None),
        "mi_grid_edges": ([vp, C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)], st),
        "mi_pose_to_matrix": ([dp, dp], st),
        "mi_features_ref_workspace": ([vp, i64, C.POINTER(sz)], sz),
        "mi_features_ref": ([vp, vp, i64, vp, sz, vp, C.POINTER(vp)], st),
        "mi_ref_destroy": ([vp], None),
        "mi_ref_resident_bytes": ([vp], sz),
        "mi_ref_move": ([vp, vp, sz, vp], st),
        "mi_ref_bins": ([vp, st, C.POINTER(vp)], st),
        "mi_ref_summary": ([vp, vp, C.POINTER(C.c_int32), C.POINTER(C.c_int64)], st),
        "mi_eval_poses_workspace": ([vp, i64, dp, i64, u32, sz], sz),
        "mi_eval_poses": ([vp, vp, i64, dp, i64, u32, vp, vp, vp, vp, vp, sz, vp], st),
        "mi_eval_poses_static": ([vp, vp, i64, dp, i64, u32, vp, vp, vp, vp, vp], st),
        "mi_calibrate_launch": ([st, i64, vp, i64, vp, dp], st),
        "mi_eval_poses_plain_workspace": ([vp, i64, i64], sz),
        "mi_eval_poses_plain": ([vp, vp, i64, dp, i64, u32, vp, vp, vp, vp, vp, sz, vp], st),
        "mi_plan_create": ([vp, i64, dp, i64, u32, vp, sz, sz, vp, C.POINTER(vp)], st),
        "mi_plan_execute": ([vp, vp, vp, vp, vp, vp, vp], st),
        "mi_plan_destroy": ([vp], None),
        "mi_plan_launch": ([vp, C.POINTER(_Tuning), C.POINTER(C.c_int32)], st),
        "mi_server_info": ([vp, C.POINTER(sz), C.POINTER(sz)], st),
        "mi_batch_workspace": ([C.POINTER(_WorkItem), i64, u32, sz], sz),
        "mi_batch_create": ([C.POINTER(_WorkItem), i64, u32, vp, sz, sz, vp, C.POINTER(vp)], st),
        "mi_batch_execute": ([vp, vp], st),
        "mi_eval_batch": ([C.POINTER(_WorkItem), i64, u32, vp, sz, vp], st),
        "mi_autotune_workspace": ([C.POINTER(_WorkItem), i64, u32, i64], sz),
        "mi_autotune": ([C.POINTER(_WorkItem), i64, u32, i64, vp, sz, vp,
                         C.POINTER(_AutotuneReport)], st),
        "mi_autotune_cached": ([C.POINTER(_WorkItem), i64, u32, i64, vp, sz, vp, C.c_char_p,
                                C.POINTER(_AutotuneReport)], st),
        "mi_tuning_cache_key": ([C.c_char_p, u32, st, st, i64, i64, C.c_char_p, sz], st),
        "mi_tuning_cache_get": ([C.c_char_p, C.c_char_p, C.POINTER(_Tuning),
                                 C.POINTER(C.c_int32)], st),
        "mi_tuning_cache_put": ([C.c_char_p, C.c_char_p, C.POINTER(_Tuning)], st),
        "mi_align_nm_workspace": ([vp, i64, C.c_int32], sz),
        "mi_align_nelder_mead": ([vp, vp, i64, dp, C.c_int32, C.POINTER(_NMDesc), dp, dp,
                                  C.POINTER(C.c_int32), vp, sz, vp], st),
        "mi_server_create": ([C.POINTER(_ServerDesc), vp, C.POINTER(vp)], st),
        "mi_server_submit": ([vp, C.POINTER(_Request), C.POINTER(i64)], st),
        "mi_server_step": ([vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)], st),
        "mi_server_poll": ([vp, i64, C.POINTER(_RequestState)], st),
        "mi_server_release": ([vp, i64], st),
        "mi_server_destroy": ([vp], None),
        "mi_align_workspace": ([vp, i64, C.POINTER(_C2F)], sz),
        "mi_align_coarse_to_fine": ([vp, vp, i64, dp, C.POINTER(_C2F), dp, dp, vp, sz, vp], st),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


_lib = _load()
EXPORTED = ("mi_status_str", "mi_last_error", "mi_tuning_set", "mi_tuning_get",
            "mi_profile_enable", "mi_profile_read", "mi_grid_create",
            "mi_grid_destroy", "mi_grid_edges", "mi_pose_to_matrix", "mi_features_ref_workspace",
            "mi_features_ref", "mi_ref_destroy", "mi_ref_resident_bytes", "mi_ref_move", "mi_ref_bins",
            "mi_ref_summary",
            "mi_eval_poses_workspace", "mi_eval_poses", "mi_eval_poses_plain_workspace",
            "mi_eval_poses_plain", "mi_plan_create", "mi_plan_execute", "mi_plan_destroy",
            "mi_plan_launch", "mi_server_info",
            "mi_batch_workspace", "mi_batch_create", "mi_batch_execute", "mi_eval_batch",
            "mi_autotune_workspace", "mi_autotune", "mi_autotune_cached",
            "mi_tuning_cache_key", "mi_tuning_cache_get", "mi_tuning_cache_put",
            "mi_align_workspace", "mi_align_coarse_to_fine", "mi_align_nm_workspace",
            "mi_align_nelder_mead", "mi_server_create",
            "mi_server_submit", "mi_server_step", "mi_server_poll", "mi_server_release",
            "mi_server_destroy")


def lib():
    return _lib


def _check(status: int, where: str):
    if status != MI_OK:
        raise MIError(status, where, (_lib.mi_last_error() or b"").decode())


def _dptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _on(stream):
    """Make `stream` current for torch's allocations and copies, so that they
    are ordered with the library calls issued on it and the caching allocator
    reuses their memory only after that stream's work."""
    return torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()


def _stream_ordered(fn):
    """Run a wrapper whose allocations and copies feed one library call under
    _on(its `stream` argument)."""
    sig = inspect.signature(fn)

    @functools.wraps(fn)
    def run(*args, **kw):
        with _on(sig.bind(*args, **kw).arguments.get("stream")):
            return fn(*args, **kw)
    return run


def _used_on(stream, *tensors):
    """Tensors made on another stream and used by work on `stream`: tell the
    caching allocator not to reuse them before that work ends."""
    if stream is None or stream == torch.cuda.current_stream():
        return
    for t in tensors:
        if t is not None:
            t.record_stream(stream)


def _dev_points(xyz) -> torch.Tensor:
    if not isinstance(xyz, torch.Tensor):
        xyz = torch.from_numpy(np.ascontiguousarray(xyz, np.float32))
    if xyz.dim() != 2 or xyz.shape[0] != 3:
        raise ValueError("points must be SoA [3, n]")
    return xyz.to(device="cuda", dtype=torch.float32).contiguous()


def _workspace(nbytes: int) -> torch.Tensor:
    # torch's caching allocator returns 256-byte-aligned blocks
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")
    assert t.data_ptr() % 256 == 0
    return t


def _poses(poses) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(poses, np.float64).reshape(-1, 6))


def status_str(s: int) -> str:
    return _lib.mi_status_str(s).decode()


# ------------------------------------------------------------------ tuning

def tuning_get() -> dict:
    t = _Tuning()
    _check(_lib.mi_tuning_get(C.byref(t)), "mi_tuning_get")
    return dict(waves=t.waves, hash_bytes=t.hash_bytes, hist_copies=t.hist_copies,
                stripe_rows=t.stripe_rows, wgs_per_cu=t.wgs_per_cu)


def tuning_set(waves: int, hash_bytes: int = 0, hist_copies: int = 1, stripe_rows: int = 16,
               wgs_per_cu: int = 0):
    t = _Tuning(int(waves), int(hash_bytes), int(hist_copies), int(stripe_rows), int(wgs_per_cu))
    _check(_lib.mi_tuning_set(C.byref(t)), "mi_tuning_set")


# --------------------------------------------------------------- profiling

def profile_enable(on: bool = True):
    _check(_lib.mi_profile_enable(1 if on else 0), "mi_profile_enable")


def profile_read() -> dict:
    p = _Profile()
    _check(_lib.mi_profile_read(C.byref(p)), "mi_profile_read")
    return {name: getattr(p, name) for name, _ in _Profile._fields_}


# ------------------------------------------------------------------ grid

class Grid:
    """mi_grid: the voxel grid R_v and the features (Sec. III-A)."""

    def __init__(self, origin, dims, voxel, features=FEAT_COUNT, nb_count=16, nb_zvar=32,
                 count_edges=None, zvar_edges=None):
        d = _GridDesc()
        d.origin[:] = [float(v) for v in origin]
        d.dims[:] = [int(v) for v in dims]
        d.voxel = float(voxel)
        d.features = int(features)
        d.nbins_count = int(nb_count)
        d.nbins_zvar = int(nb_zvar)
        self._ce = None if count_edges is None else np.ascontiguousarray(count_edges, np.uint32)
        self._ze = None if zvar_edges is None else np.ascontiguousarray(zvar_edges, np.uint64)
        d.count_edges = None if self._ce is None else self._ce.ctypes.data_as(C.POINTER(C.c_uint32))
        d.zvar_edges = None if self._ze is None else self._ze.ctypes.data_as(C.POINTER(C.c_uint64))
        h = C.c_void_p()
        _check(_lib.mi_grid_create(C.byref(d), C.byref(h)), "mi_grid_create")
        self._h = h
        self.origin = tuple(d.origin)
        self.dims = tuple(d.dims)
        self.voxel = d.voxel
        self.features = d.features
        self.nb_count = d.nbins_count
        self.nb_zvar = d.nbins_zvar

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mi_grid_destroy(self._h)
            self._h = None

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

    @property
    def nf(self):
        return len(self.feature_list)

    def edges(self):
        ce = np.zeros(64, np.uint32)
        ze = np.zeros(64, np.uint64)
        _check(_lib.mi_grid_edges(self._h, ce.ctypes.data_as(C.POINTER(C.c_uint32)),
                                  ze.ctypes.data_as(C.POINTER(C.c_uint64))), "mi_grid_edges")
        return ce[:max(self.nb_count - 1, 0)], ze[:max(self.nb_zvar - 2, 0)]


def pose_to_matrix(eta) -> np.ndarray:
    e = np.ascontiguousarray(eta, np.float64)
    rt = np.zeros(12, np.float64)
    _check(_lib.mi_pose_to_matrix(e.ctypes.data_as(C.POINTER(C.c_double)),
                                  rt.ctypes.data_as(C.POINTER(C.c_double))), "mi_pose_to_matrix")
    return rt.reshape(3, 4)


# ------------------------------------------------------------- reference

class Ref:
    """mi_ref: scan A's resident feature map (Alg. 1 initialisation)."""

    def __init__(self, grid: Grid, xyz_a, stream=None, compact=True):
        """compact: once built, move the reference into a workspace of just
        its resident size (mi_ref_move), so that the worst-case workspace it
        was built in goes back to torch's allocator."""
        self.grid = grid
        with _on(stream):
            self.xyz_a = _dev_points(xyz_a)
            n = self.xyz_a.shape[1]
            pers = C.c_size_t()
            nbytes = _lib.mi_features_ref_workspace(grid._h, n, C.byref(pers))
            self.ws = _workspace(nbytes)
            self.persistent_bytes = pers.value
            h = C.c_void_p()
            _check(_lib.mi_features_ref(grid._h, _dptr(self.xyz_a), n, _dptr(self.ws),
                                        self.ws.numel(), _stream(stream), C.byref(h)),
                   "mi_features_ref")
        self._h = h
        # the bytes of the workspace the reference keeps (its tables as laid out
        # for this scan A; persistent_bytes is the most they could take)
        self.resident_bytes = _lib.mi_ref_resident_bytes(h)
        if compact and self.resident_bytes < self.ws.numel():
            with _on(stream):
                ws = _workspace(self.resident_bytes)
                _check(_lib.mi_ref_move(h, _dptr(ws), ws.numel(), _stream(stream)),
                       "mi_ref_move")
                # the old block is reused only by work ordered after the copy
                self.ws = ws

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mi_ref_destroy(self._h)
            self._h = None

    def bins(self, feature_slot: int) -> torch.Tensor:
        p = C.c_void_p()
        _check(_lib.mi_ref_bins(self._h, int(feature_slot), C.byref(p)), "mi_ref_bins")
        off = p.value - self.ws.data_ptr()
        V = self.grid.dims[0] * self.grid.dims[1] * self.grid.dims[2]
        return self.ws[off:off + V]

    def summary(self, stream=None):
        box = np.zeros(6, np.int32)
        ctr = np.zeros(4, np.int64)
        _check(_lib.mi_ref_summary(self._h, _stream(stream),
                                   box.ctypes.data_as(C.POINTER(C.c_int32)),
                                   ctr.ctypes.data_as(C.POINTER(C.c_int64))), "mi_ref_summary")
        return box, ctr


# ------------------------------------------------------------- evaluate

def _outputs(grid: Grid, K: int, want_hist: bool, want_stats: bool, want_argmax: bool):
    mi = torch.empty((grid.nf, K), dtype=torch.float64, device="cuda")
    am = torch.empty(grid.nf, dtype=torch.int64, device="cuda") if want_argmax else None
    hist = None
    if want_hist:
        tot = sum(K * nb * nb for _, nb in grid.feature_list)
        hist = torch.empty(max(tot, 1), dtype=torch.int32, device="cuda")
    stats = torch.empty(max(K, 1) * 64, dtype=torch.uint8, device="cuda") if want_stats else None
    return mi, am, hist, stats


def _unpack(grid: Grid, K: int, mi, am, hist, stats):
    out = {"mi": mi, "argmax": am}
    if hist is not None:
        hs, off = [], 0
        for _, nb in grid.feature_list:
            hs.append(hist[off:off + K * nb * nb].view(K, nb, nb))
            off += K * nb * nb
        out["hist"] = hs
    if stats is not None:
        out["stats_raw"] = stats
    return out


def stats_to_numpy(stats_raw: torch.Tensor, K: int) -> np.ndarray:
    return stats_raw[:K * 64].cpu().numpy().view(STATS_DTYPE)


@_stream_ordered
def eval_poses(ref: Ref, xyz_b, poses, flags=0, want_hist=False, want_stats=False,
               want_argmax=True, stream=None, frame_budget=0):
    """mi_eval_poses: MI per feature of every pose (Eqs. 1-5)."""
    xb = _dev_points(xyz_b)
    P = _poses(poses)
    K = P.shape[0]
    pp = P.ctypes.data_as(C.POINTER(C.c_double))
    nbytes = _lib.mi_eval_poses_workspace(ref._h, xb.shape[1], pp, K, flags, frame_budget)
    mi, am, hist, stats = _outputs(ref.grid, K, want_hist, want_stats, want_argmax)
    # a rejected pose set sizes to 0; the call itself then reports why
    ws = _workspace(nbytes)
    _check(_lib.mi_eval_poses(ref._h, _dptr(xb), xb.shape[1], pp, K, flags, _dptr(mi), _dptr(am),
                              _dptr(hist), _dptr(stats), _dptr(ws), ws.numel(), _stream(stream)),
           "mi_eval_poses")
    out = _unpack(ref.grid, K, mi, am, hist, stats)
    out["_keep"] = (xb, ws)
    return out


def calibrate_launch(kind: int, size: int, scratch: torch.Tensor, stream=None) -> float:
    """mi_calibrate_launch: launches one roofline microbenchmark kernel on the
    stream and returns its operation count (the caller times it)."""
    ops = C.c_double(0.0)
    _check(_lib.mi_calibrate_launch(int(kind), int(size), _dptr(scratch), scratch.numel() *
                                    scratch.element_size(), _stream(stream), C.byref(ops)),
           "mi_calibrate_launch")
    return ops.value


@_stream_ordered
def eval_poses_static(ref: Ref, xyz_b, poses, flags=0, want_hist=False, want_stats=False,
                      want_argmax=True, stream=None):
    """mi_eval_poses_static: mi_eval_poses on the library's static device
    scratch (no workspace; the call allocates no device memory)."""
    xb = _dev_points(xyz_b)
    P = _poses(poses)
    K = P.shape[0]
    pp = P.ctypes.data_as(C.POINTER(C.c_double))
    mi, am, hist, stats = _outputs(ref.grid, K, want_hist, want_stats, want_argmax)
    _check(_lib.mi_eval_poses_static(ref._h, _dptr(xb), xb.shape[1], pp, K, flags, _dptr(mi),
                                     _dptr(am), _dptr(hist), _dptr(stats), _stream(stream)),
           "mi_eval_poses_static")
    out = _unpack(ref.grid, K, mi, am, hist, stats)
    out["_keep"] = (xb,)
    return out


@_stream_ordered
def eval_poses_plain(ref: Ref, xyz_b, poses, flags=0, want_hist=False, want_stats=False,
                     want_argmax=True, stream=None):
    """mi_eval_poses_plain: the per-pose stage sequence (same results)."""
    xb = _dev_points(xyz_b)
    P = _poses(poses)
    K = P.shape[0]
    nbytes = _lib.mi_eval_poses_plain_workspace(ref._h, xb.shape[1], K)
    ws = _workspace(nbytes)
    mi, am, hist, stats = _outputs(ref.grid, K, want_hist, want_stats, want_argmax)
    _check(_lib.mi_eval_poses_plain(ref._h, _dptr(xb), xb.shape[1],
                                    P.ctypes.data_as(C.POINTER(C.c_double)), K, flags, _dptr(mi),
                                    _dptr(am), _dptr(hist), _dptr(stats), _dptr(ws), ws.numel(),
                                    _stream(stream)), "mi_eval_poses_plain")
    out = _unpack(ref.grid, K, mi, am, hist, stats)
    out["_keep"] = (xb, ws)
    return out


class Plan:
    """mi_plan: pose tables uploaded once; execute() only launches kernels
    (capturable in a HIP graph)."""

    @_stream_ordered
    def __init__(self, ref: Ref, n_b: int, poses, flags=0, stream=None, frame_budget=0):
        self.ref = ref
        P = _poses(poses)
        self.K = P.shape[0]
        self.n_b = int(n_b)
        pp = P.ctypes.data_as(C.POINTER(C.c_double))
        nbytes = _lib.mi_eval_poses_workspace(ref._h, self.n_b, pp, self.K, flags, frame_budget)
        # a rejected pose set sizes to 0; mi_plan_create then reports why
        self.ws = _workspace(nbytes)
        h = C.c_void_p()
        _check(_lib.mi_plan_create(ref._h, self.n_b, pp, self.K, flags, _dptr(self.ws),
                                   self.ws.numel(), frame_budget, _stream(stream), C.byref(h)),
               "mi_plan_create")
        self._h = h

    def execute(self, xyz_b: torch.Tensor, mi: torch.Tensor, argmax=None, hist=None, stats=None,
                stream=None):
        _used_on(stream, self.ws)
        _check(_lib.mi_plan_execute(self._h, _dptr(xyz_b), _dptr(mi), _dptr(argmax), _dptr(hist),
                                    _dptr(stats), _stream(stream)), "mi_plan_execute")

    def launch(self) -> dict:
        """mi_plan_launch: the tuning the plan runs under (auto hash resolved)
        and the LDS bytes of one evaluator workgroup."""
        t, lds = _Tuning(), C.c_int32()
        _check(_lib.mi_plan_launch(self._h, C.byref(t), C.byref(lds)), "mi_plan_launch")
        return dict(waves=t.waves, hash_bytes=t.hash_bytes, hist_copies=t.hist_copies,
                    stripe_rows=t.stripe_rows, wgs_per_cu=t.wgs_per_cu, lds_bytes=lds.value)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mi_plan_destroy(self._h)
            self._h = None


class WorkItem:
    """One scan pair and pose set of a batch, with its device outputs."""

    def __init__(self, ref: Ref, xyz_b, poses, want_hist=False, want_stats=False,
                 want_argmax=True):
        self.ref = ref
        self.xyz_b = _dev_points(xyz_b)
        self.poses = _poses(poses)
        self.K = self.poses.shape[0]
        self.mi, self.argmax, self.hist_raw, self.stats_raw = _outputs(
            ref.grid, self.K, want_hist, want_stats, want_argmax)

    def _c(self) -> _WorkItem:
        return _WorkItem(self.ref._h, _dptr(self.xyz_b), self.xyz_b.shape[1],
                         self.poses.ctypes.data_as(C.POINTER(C.c_double)), self.K,
                         _dptr(self.mi), _dptr(self.argmax), _dptr(self.hist_raw),
                         _dptr(self.stats_raw))

    def results(self) -> dict:
        return _unpack(self.ref.grid, self.K, self.mi, self.argmax, self.hist_raw, self.stats_raw)


def _items_array(items):
    arr = (_WorkItem * max(len(items), 1))()
    for i, it in enumerate(items):
        arr[i] = it._c()
    return arr


class Batch:
    """mi_batch_*: the poses of many scan pairs in one schedule; execute()
    only launches kernels (capturable in a HIP graph)."""

    @_stream_ordered
    def __init__(self, items, flags=0, stream=None, frame_budget=0):
        self.items = list(items)
        arr = _items_array(self.items)
        nbytes = _lib.mi_batch_workspace(arr, len(self.items), flags, frame_budget)
        if nbytes == 0:
            raise MIError(MI_E_INVALID, "mi_batch_workspace", _lib.mi_last_error().decode())
        self.ws = _workspace(nbytes)
        h = C.c_void_p()
        _check(_lib.mi_batch_create(arr, len(self.items), flags, _dptr(self.ws), self.ws.numel(),
                                    frame_budget, _stream(stream), C.byref(h)), "mi_batch_create")
        self._h = h

    def execute(self, stream=None):
        _used_on(stream, self.ws, *[t for it in self.items
                                    for t in (it.xyz_b, it.mi, it.argmax, it.hist_raw,
                                              it.stats_raw)])
        _check(_lib.mi_batch_execute(self._h, _stream(stream)), "mi_batch_execute")

    def launch(self) -> dict:
        """mi_plan_launch: the tuning the plan runs under (auto hash resolved)
        and the LDS bytes of one evaluator workgroup."""
        t, lds = _Tuning(), C.c_int32()
        _check(_lib.mi_plan_launch(self._h, C.byref(t), C.byref(lds)), "mi_plan_launch")
        return dict(waves=t.waves, hash_bytes=t.hash_bytes, hist_copies=t.hist_copies,
                    stripe_rows=t.stripe_rows, wgs_per_cu=t.wgs_per_cu, lds_bytes=lds.value)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mi_plan_destroy(self._h)
            self._h = None


@_stream_ordered
def eval_batch(items, flags=0, stream=None):
    """mi_eval_batch: create, execute and release a batch in one call."""
    items = list(items)
    arr = _items_array(items)
    nbytes = _lib.mi_batch_workspace(arr, len(items), flags, 0)
    if nbytes == 0:
        raise MIError(MI_E_INVALID, "mi_batch_workspace", _lib.mi_last_error().decode())
    ws = _workspace(nbytes)
    _check(_lib.mi_eval_batch(arr, len(items), flags, _dptr(ws), ws.numel(), _stream(stream)),
           "mi_eval_batch")
    return ws


@_stream_ordered
def autotune(items, flags=0, max_poses=4096, stream=None, cache=None) -> dict:
    """mi_autotune: time candidate tunings on a sample of the workload and make
    the fastest current.  Returns the chosen tuning and the timings.  cache: a
    tuning-cache file (mi_autotune_cached): a tuning cached for this workload's
    key is made current without timing (tried = 0); else the result is stored."""
    items = list(items)
    arr = _items_array(items)
    nbytes = _lib.mi_autotune_workspace(arr, len(items), flags, int(max_poses))
    if nbytes == 0:
        raise MIError(MI_E_INVALID, "mi_autotune_workspace", _lib.mi_last_error().decode())
    ws = _workspace(nbytes)
    rep = _AutotuneReport()
    if cache is None:
        _check(_lib.mi_autotune(arr, len(items), flags, int(max_poses), _dptr(ws), ws.numel(),
                                _stream(stream), C.byref(rep)), "mi_autotune")
    else:
        _check(_lib.mi_autotune_cached(arr, len(items), flags, int(max_poses), _dptr(ws),
                                       ws.numel(), _stream(stream), os.fsencode(cache),
                                       C.byref(rep)), "mi_autotune_cached")
    b = rep.best
    return dict(best=dict(waves=b.waves, hash_bytes=b.hash_bytes, hist_copies=b.hist_copies,
                          stripe_rows=b.stripe_rows, wgs_per_cu=b.wgs_per_cu),
                best_ms=rep.best_ms, start_ms=rep.start_ms, tried=rep.tried)


def tuning_cache_key(arch: str, features: int, nb0: int, nb1: int, n_b: int, voxels: int) -> str:
    """mi_tuning_cache_key (host only)."""
    buf = C.create_string_buffer(256)
    _check(_lib.mi_tuning_cache_key(arch.encode(), int(features), int(nb0), int(nb1), int(n_b),
                                    int(voxels), buf, len(buf)), "mi_tuning_cache_key")
    return buf.value.decode()


def tuning_cache_get(path, key: str):
    """mi_tuning_cache_get (host only): the cached tuning as a dict, or None."""
    t = _Tuning()
    found = C.c_int32(0)
    _check(_lib.mi_tuning_cache_get(os.fsencode(path), key.encode(), C.byref(t), C.byref(found)),
           "mi_tuning_cache_get")
    if not found.value:
        return None
    return dict(waves=t.waves, hash_bytes=t.hash_bytes, hist_copies=t.hist_copies,
                stripe_rows=t.stripe_rows, wgs_per_cu=t.wgs_per_cu)


def tuning_cache_put(path, key: str, tuning: dict):
    """mi_tuning_cache_put (host only)."""
    t = _Tuning(int(tuning["waves"]), int(tuning["hash_bytes"]), int(tuning["hist_copies"]),
                int(tuning["stripe_rows"]), int(tuning["wgs_per_cu"]))
    _check(_lib.mi_tuning_cache_put(os.fsencode(path), key.encode(), C.byref(t)),
           "mi_tuning_cache_put")


def _objective(d, feature_slot, weights):
    if weights is None:
        d.feature_slot = int(feature_slot)
    else:
        d.feature_slot = SLOT_WEIGHTED
        d.weight[:] = [float(v) for v in weights]


@_stream_ordered
def align_coarse_to_fine(ref: Ref, xyz_b, init, half_range, samples, levels, shrink,
                         feature_slot=0, stream=None, weights=None):
    """mi_align_coarse_to_fine: shrinking grid search for Eq. 1 from T_o, on
    one feature slot or, given weights (w0, w1), on w0 * MI_0 + w1 * MI_1."""
    xb = _dev_points(xyz_b)
    d = _c2f_desc(half_range, samples, levels, shrink, feature_slot, weights)
    nbytes = _lib.mi_align_workspace(ref._h, xb.shape[1], C.byref(d))
    if nbytes == 0:
        raise MIError(MI_E_INVALID, "mi_align_workspace", "bad arguments")
    ws = _workspace(nbytes)
    i0 = np.ascontiguousarray(init, np.float64)
    out = np.zeros(6, np.float64)
    best = np.zeros(1, np.float64)
    _check(_lib.mi_align_coarse_to_fine(ref._h, _dptr(xb), xb.shape[1],
                                        i0.ctypes.data_as(C.POINTER(C.c_double)), C.byref(d),
                                        out.ctypes.data_as(C.POINTER(C.c_double)),
                                        best.ctypes.data_as(C.POINTER(C.c_double)), _dptr(ws),
                                        ws.numel(), _stream(stream)), "mi_align_coarse_to_fine")
    return out, float(best[0])


@_stream_ordered
def align_nelder_mead(ref: Ref, xyz_b, starts, step, max_iter, ftol, xtol, feature_slot=0,
                      stream=None, weights=None):
    """mi_align_nelder_mead: simplex search for Eq. 1 (Sec. III-B) from one or
    more starts, the simplexes advancing together in batched evaluations.
    Returns (pose[6], MI, iterations per start)."""
    xb = _dev_points(xyz_b)
    S = np.ascontiguousarray(np.asarray(starts, np.float64).reshape(-1, 6))
    d = _NMDesc()
    d.step[:] = [float(v) for v in step]
    d.max_iter = int(max_iter)
    d.ftol = float(ftol)
    d.xtol = float(xtol)
    _objective(d, feature_slot, weights)
    nbytes = _lib.mi_align_nm_workspace(ref._h, xb.shape[1], S.shape[0])
    if nbytes == 0:
        raise MIError(MI_E_INVALID, "mi_align_nm_workspace", _lib.mi_last_error().decode())
    ws = _workspace(nbytes)
    out = np.zeros(6, np.float64)
    best = np.zeros(1, np.float64)
    iters = np.zeros(S.shape[0], np.int32)
    _check(_lib.mi_align_nelder_mead(ref._h, _dptr(xb), xb.shape[1],
                                     S.ctypes.data_as(C.POINTER(C.c_double)), S.shape[0],
                                     C.byref(d), out.ctypes.data_as(C.POINTER(C.c_double)),
                                     best.ctypes.data_as(C.POINTER(C.c_double)),
                                     iters.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(ws),
                                     ws.numel(), _stream(stream)), "mi_align_nelder_mead")
    return out, float(best[0]), iters


# ------------------------------------------------------------- serving

REQ_QUEUED, REQ_ACTIVE, REQ_DONE, REQ_FAILED = 0, 1, 2, 3


def _c2f_desc(half_range, samples, levels, shrink, feature_slot, weights=None) -> _C2F:
    d = _C2F()
    d.half_range[:] = [float(v) for v in half_range]
    d.samples[:] = [int(v) for v in samples]
    d.levels = int(levels)
    d.shrink = float(shrink)
    _objective(d, feature_slot, weights)
    return d


class Server:
    """mi_server: continuous batching of coarse-to-fine alignments over one
    device arena (torch-allocated here) and one stream."""

    def __init__(self, arena_bytes: int, max_active: int, step_bytes: int = 0, stream=None):
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        with _on(self.stream):
            self.arena = _workspace(arena_bytes)
        d = _ServerDesc(_dptr(self.arena).value, self.arena.numel(), int(step_bytes),
                        int(max_active))
        h = C.c_void_p()
        _check(_lib.mi_server_create(C.byref(d), _stream(self.stream), C.byref(h)),
               "mi_server_create")
        self._h = h

    def submit(self, origin, dims, voxel, xyz_a, xyz_b, init, half_range, samples, levels,
               shrink, features=FEAT_COUNT, nb_count=16, nb_zvar=32, feature_slot=0,
               weights=None) -> int:
        A = np.ascontiguousarray(xyz_a, np.float32)
        B = np.ascontiguousarray(xyz_b, np.float32)
        q = _Request()
        q.grid.origin[:] = [float(v) for v in origin]
        q.grid.dims[:] = [int(v) for v in dims]
        q.grid.voxel = float(voxel)
        q.grid.features = int(features)
        q.grid.nbins_count = int(nb_count)
        q.grid.nbins_zvar = int(nb_zvar)
        q.xyz_a = A.ctypes.data
        q.n_a = A.shape[1]
        q.xyz_b = B.ctypes.data
        q.n_b = B.shape[1]
        q.init[:] = [float(v) for v in init]
        q.search = _c2f_desc(half_range, samples, levels, shrink, feature_slot, weights)
        rid = C.c_int64()
        _check(_lib.mi_server_submit(self._h, C.byref(q), C.byref(rid)), "mi_server_submit")
        return rid.value

    def step(self):
        na, nq = C.c_int32(), C.c_int32()
        _check(_lib.mi_server_step(self._h, C.byref(na), C.byref(nq)), "mi_server_step")
        return na.value, nq.value

    def poll(self, rid: int) -> dict:
        st = _RequestState()
        _check(_lib.mi_server_poll(self._h, int(rid), C.byref(st)), "mi_server_poll")
        return dict(state=st.state, levels_done=st.levels_done, status=st.status,
                    pose=np.array(st.pose[:]), mi=st.mi, t_submit=st.t_submit,
                    t_admit=st.t_admit, t_done=st.t_done)

    def release(self, rid: int):
        _check(_lib.mi_server_release(self._h, int(rid)), "mi_server_release")

    def info(self) -> dict:
        """mi_server_info: bytes of the request heap in all and free now."""
        tot, free = C.c_size_t(), C.c_size_t()
        _check(_lib.mi_server_info(self._h, C.byref(tot), C.byref(free)), "mi_server_info")
        return dict(heap_bytes=tot.value, heap_free=free.value)

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mi_server_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()
