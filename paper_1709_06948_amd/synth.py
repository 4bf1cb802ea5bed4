"""Seeded synthetic inputs for scan alignment.

This module only makes inputs: scenes, scans (float32 SoA [3, n]) and pose
sets.  It holds none of the alignment method's arithmetic (no voxelization,
features, histograms or MI), so both the HIP library's tests and the CPU
oracle's tests can draw from it.

The paper evaluates on vehicle-lidar scan pairs (Ford Campus, KITTI) with 1 m
voxels (Sec. IV).  Those datasets are not available, so these generators stand
in for them with scenes of the same kind: a ground plane with box-shaped
buildings/cars and thin poles, either sampled uniformly on visible surfaces or
ray-cast by a simulated 64-ring spinning scanner.

Seeds: base 170906948; workload c uses base + c, its pair/request j uses
base + 1000*c + j.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 170906948
NOISE_SIGMA = 0.02


def seed_for(config: int, item: int | None = None) -> int:
    return BASE_SEED + config if item is None else BASE_SEED + 1000 * config + item


# ----------------------------------------------------------------- geometry

def _rot(roll: float, pitch: float, yaw: float) -> np.ndarray:
    """Rotation used to *place* the second scan: yaw about z, then pitch about y,
    then roll about x applied first (z-y-x intrinsic), built from elementary
    rotations in numpy.  Only used to synthesise data."""
    c, s = math.cos, math.sin
    rx = np.array([[1, 0, 0], [0, c(roll), -s(roll)], [0, s(roll), c(roll)]])
    ry = np.array([[c(pitch), 0, s(pitch)], [0, 1, 0], [-s(pitch), 0, c(pitch)]])
    rz = np.array([[c(yaw), -s(yaw), 0], [s(yaw), c(yaw), 0], [0, 0, 1]])
    return rz @ ry @ rx


def to_frame(points_world: np.ndarray, eta) -> np.ndarray:
    """Express world (= scan A frame) points in the frame of a sensor placed at
    pose eta = [tx,ty,tz,roll,pitch,yaw]: p_B = R^T (p - t)."""
    R = _rot(eta[3], eta[4], eta[5])
    t = np.asarray(eta[:3], np.float64).reshape(3, 1)
    return R.T @ (points_world - t)


@dataclass
class Scene:
    half_extent: float
    boxes: np.ndarray                 # [nb, 6]: xmin, ymin, zmin, xmax, ymax, zmax
    cyls: np.ndarray                  # [nc, 4]: cx, cy, r, h
    meta: dict = field(default_factory=dict)


def make_box_scene(rng: np.random.Generator, half_extent=30.0, n_boxes=30, n_cyl=10,
                   edge=(0.5, 5.0), cyl_r=0.15, cyl_h=(3.0, 7.0), keep_clear=()) -> Scene:
    """Ground plane z=0 with axis-aligned boxes (every edge U[edge]) standing on it
    and vertical cylinders (radius cyl_r, height U[cyl_h])."""
    boxes = []
    while len(boxes) < n_boxes:
        w, d, h = rng.uniform(edge[0], edge[1], 3)
        cx, cy = rng.uniform(-half_extent + w / 2, half_extent - w / 2), \
            rng.uniform(-half_extent + d / 2, half_extent - d / 2)
        if any(abs(cx - kx) < w / 2 + 2.0 and abs(cy - ky) < d / 2 + 2.0 for kx, ky in keep_clear):
            continue
        boxes.append([cx - w / 2, cy - d / 2, 0.0, cx + w / 2, cy + d / 2, h])
    cyls = []
    while len(cyls) < n_cyl:
        cx, cy = rng.uniform(-half_extent + 1, half_extent - 1, 2)
        if any(math.hypot(cx - kx, cy - ky) < 2.0 for kx, ky in keep_clear):
            continue
        cyls.append([cx, cy, cyl_r, rng.uniform(cyl_h[0], cyl_h[1])])
    return Scene(half_extent, np.array(boxes, np.float64).reshape(-1, 6),
                 np.array(cyls, np.float64).reshape(-1, 4))


def _inside_any_box(p: np.ndarray, boxes: np.ndarray, skip: np.ndarray | None = None,
                    eps=1e-9) -> np.ndarray:
    """True where point p[:, i] lies strictly inside a box other than skip[i]."""
    n = p.shape[1]
    hidden = np.zeros(n, bool)
    for bi, b in enumerate(boxes):
        m = ((p[0] > b[0] + eps) & (p[0] < b[3] - eps) & (p[1] > b[1] + eps) & (p[1] < b[4] - eps)
             & (p[2] > b[2] + eps) & (p[2] < b[5] - eps))
        if skip is not None:
            m &= skip != bi
        hidden |= m
    return hidden


def sample_surfaces(scene: Scene, n: int, rng: np.random.Generator) -> np.ndarray:
    """n points uniform (by area) on the visible surfaces of the scene: ground not
    covered by a footprint, box tops and sides, cylinder sides and tops.
    Returns float64 [3, n] without noise."""
    H = scene.half_extent
    patches = []  # (kind, index, area)
    patches.append(("ground", -1, (2 * H) ** 2))
    for i, b in enumerate(scene.boxes):
        w, d, h = b[3] - b[0], b[4] - b[1], b[5] - b[2]
        patches += [("top", i, w * d), ("sx0", i, d * h), ("sx1", i, d * h), ("sy0", i, w * h),
                    ("sy1", i, w * h)]
    for i, c in enumerate(scene.cyls):
        patches += [("cside", i, 2 * math.pi * c[2] * c[3]), ("ctop", i, math.pi * c[2] ** 2)]
    areas = np.array([a for _, _, a in patches])
    prob = areas / areas.sum()
    out = []
    have = 0
    while have < n:
        m = int((n - have) * 1.6) + 64
        which = rng.choice(len(patches), size=m, p=prob)
        pts = np.zeros((3, m))
        owner = np.full(m, -1)
        u, v = rng.random(m), rng.random(m)
        for pi in np.unique(which):
            sel = which == pi
            kind, idx, _ = patches[pi]
            uu, vv = u[sel], v[sel]
            if kind == "ground":
                pts[:, sel] = [(uu * 2 - 1) * H, (vv * 2 - 1) * H, 0.0 * uu]
            elif kind in ("top", "sx0", "sx1", "sy0", "sy1"):
                b = scene.boxes[idx]
                owner[sel] = idx
                if kind == "top":
                    pts[:, sel] = [b[0] + uu * (b[3] - b[0]), b[1] + vv * (b[4] - b[1]), b[5] + 0 * uu]
                elif kind in ("sx0", "sx1"):
                    x = b[0] if kind == "sx0" else b[3]
                    pts[:, sel] = [x + 0 * uu, b[1] + uu * (b[4] - b[1]), b[2] + vv * (b[5] - b[2])]
                else:
                    y = b[1] if kind == "sy0" else b[4]
                    pts[:, sel] = [b[0] + uu * (b[3] - b[0]), y + 0 * uu, b[2] + vv * (b[5] - b[2])]
            elif kind == "cside":
                c = scene.cyls[idx]
                a = uu * 2 * math.pi
                pts[:, sel] = [c[0] + c[2] * np.cos(a), c[1] + c[2] * np.sin(a), vv * c[3]]
            else:
                c = scene.cyls[idx]
                a, r = uu * 2 * math.pi, c[2] * np.sqrt(vv)
                pts[:, sel] = [c[0] + r * np.cos(a), c[1] + r * np.sin(a), c[3] + 0 * uu]
        keep = ~_inside_any_box(pts, scene.boxes, owner)
        ground = which == 0
        if ground.any():
            g = pts[:, ground]
            cov = np.zeros(g.shape[1], bool)
            for b in scene.boxes:
                cov |= (g[0] > b[0]) & (g[0] < b[3]) & (g[1] > b[1]) & (g[1] < b[4])
            for c in scene.cyls:
                cov |= (g[0] - c[0]) ** 2 + (g[1] - c[1]) ** 2 < c[2] ** 2
            k = keep[ground]
            k &= ~cov
            keep[ground] = k
        pts = pts[:, keep]
        out.append(pts)
        have += pts.shape[1]
    return np.concatenate(out, axis=1)[:, :n]


def add_noise(p: np.ndarray, rng: np.random.Generator, sigma=NOISE_SIGMA) -> np.ndarray:
    return p + rng.normal(0.0, sigma, size=p.shape)


def as_soa32(p: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(p, dtype=np.float32)


# ------------------------------------------------------------- workloads

@dataclass
class Pair:
    """A scan pair: A in its own frame, B in its own frame, and the true pose
    eta_gt that maps B into A (p_A = R p_B + t)."""
    A: np.ndarray          # float32 [3, nA]
    B: np.ndarray          # float32 [3, nB]
    eta_gt: np.ndarray     # float64 [6]: tx, ty, tz, roll, pitch, yaw (rad)
    origin: tuple
    dims: tuple
    voxel: float
    meta: dict = field(default_factory=dict)


def tiny_pair(seed=None, n_a=20000, n_b=20000, crop=0.70) -> Pair:
    """Single scan pair of the tiny plain workload: 60x60x8 m scene, 30 boxes,
    10 poles, 20k points per scan on visible surfaces, sigma 0.02 m; B resampled,
    cropped to a window of 70% of the scene area and moved by a true pose with
    tx,ty U[-2,2] m, tz U[-0.2,0.2] m, yaw U[-10,10] deg, roll/pitch U[-2,2] deg.
    Grid: origin (-32,-32,-1), 64x64x10 voxels of 1 m."""
    rng = np.random.default_rng(seed_for(1) if seed is None else seed)
    scene = make_box_scene(rng, 30.0, 30, 10)
    A = add_noise(sample_surfaces(scene, n_a, rng), rng)
    Bw = sample_surfaces(scene, n_b, rng)
    side = 60.0 * math.sqrt(crop)
    x0, y0 = rng.uniform(-30.0, 30.0 - side, 2)
    inside = (Bw[0] >= x0) & (Bw[0] < x0 + side) & (Bw[1] >= y0) & (Bw[1] < y0 + side)
    Bw = Bw[:, inside]
    d2r = math.pi / 180.0
    eta = np.array([rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(-0.2, 0.2),
                    rng.uniform(-2, 2) * d2r, rng.uniform(-2, 2) * d2r, rng.uniform(-10, 10) * d2r])
    B = add_noise(to_frame(Bw, eta), rng)
    return Pair(as_soa32(A), as_soa32(B), eta, (-32.0, -32.0, -1.0), (64, 64, 10), 1.0,
                dict(window=(x0, y0, side)))


def tiny_search_poses() -> np.ndarray:
    """11 x 11 x 11 exhaustive search over x, y in [-2, 2] m (0.4 m) and yaw in
    [-10, 10] deg (2 deg); z, roll, pitch = 0.  Row-major (x, y, yaw)."""
    xs = np.linspace(-2.0, 2.0, 11)
    yaws = np.deg2rad(np.linspace(-10.0, 10.0, 11))
    P = np.zeros((11 ** 3, 6))
    k = 0
    for x in xs:
        for y in xs:
            for w in yaws:
                P[k] = [x, y, 0, 0, 0, w]
                k += 1
    return P


def grid8_poses(n=8) -> np.ndarray:
    """n^6 candidate poses: tx,ty in +-2 m, tz in +-0.2 m, roll,pitch in +-2 deg,
    yaw in +-10 deg, n nodes per axis including endpoints; row-major with yaw
    fastest (n^3 distinct rotations x n^3 translations)."""
    d2r = math.pi / 180.0
    axes = [np.linspace(-2, 2, n), np.linspace(-2, 2, n), np.linspace(-0.2, 0.2, n),
            np.linspace(-2, 2, n) * d2r, np.linspace(-2, 2, n) * d2r, np.linspace(-10, 10, n) * d2r]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.reshape(-1) for m in mesh], axis=1)


# ------------------------------------------------------------ ray casting

def _ray_hits(origin: np.ndarray, dirs: np.ndarray, scene: Scene, rmax: float) -> np.ndarray:
    """Nearest hit distance of each ray with the ground plane, the boxes and the
    vertical cylinders (inf for no hit within rmax)."""
    n = dirs.shape[1]
    best = np.full(n, np.inf)
    dz = dirs[2]
    with np.errstate(divide="ignore", invalid="ignore"):
        tg = -origin[2] / dz
    tg[(dz >= 0) | ~np.isfinite(tg)] = np.inf
    best = np.minimum(best, tg)
    inv = np.where(dirs == 0, 1e300, 1.0 / np.where(dirs == 0, 1.0, dirs))
    for b in scene.boxes:
        t1 = (b[:3].reshape(3, 1) - origin.reshape(3, 1)) * inv
        t2 = (b[3:].reshape(3, 1) - origin.reshape(3, 1)) * inv
        tmin = np.minimum(t1, t2).max(axis=0)
        tmax = np.maximum(t1, t2).min(axis=0)
        hit = (tmax >= np.maximum(tmin, 0.0)) & (tmin > 1e-6)
        best = np.where(hit & (tmin < best), tmin, best)
    dx, dy = dirs[0], dirs[1]
    a = dx * dx + dy * dy
    for c in scene.cyls:
        ox, oy = origin[0] - c[0], origin[1] - c[1]
        bq = 2 * (ox * dx + oy * dy)
        cq = ox * ox + oy * oy - c[2] ** 2
        disc = bq * bq - 4 * a * cq
        ok = (disc >= 0) & (a > 0)
        with np.errstate(invalid="ignore", divide="ignore"):
            t = (-bq - np.sqrt(np.where(ok, disc, 0))) / (2 * np.where(a > 0, a, 1))
        z = origin[2] + t * dirs[2]
        hit = ok & (t > 1e-6) & (z >= 0) & (z <= c[3])
        best = np.where(hit & (t < best), t, best)
    best[best > rmax] = np.inf
    return best


def raycast_scan(scene: Scene, eta, rng: np.random.Generator, rings=64, elev=(-24.8, 2.0),
                 az_step=0.2, rmax=80.0, sensor_h=1.8) -> np.ndarray:
    """Simulated spinning scanner on a vehicle at pose eta (world frame): rings
    evenly spaced over elev (deg), one beam every az_step deg, range <= rmax,
    sensor sensor_h above the vehicle origin.  Returns points in the vehicle
    frame (float64 [3, n]) with N(0, 0.02^2) noise per coordinate."""
    el = np.deg2rad(np.linspace(elev[0], elev[1], rings))
    az = np.deg2rad(np.arange(0.0, 360.0, az_step))
    E, A = np.meshgrid(el, az, indexing="ij")
    d_local = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)]).reshape(3, -1)
    R = _rot(eta[3], eta[4], eta[5])
    t = np.asarray(eta[:3], np.float64)
    origin = t + R @ np.array([0.0, 0.0, sensor_h])
    dirs = R @ d_local
    r = _ray_hits(origin, dirs, scene, rmax)
    ok = np.isfinite(r)
    pw = origin.reshape(3, 1) + dirs[:, ok] * r[ok]
    return add_noise(to_frame(pw, eta), rng)


def urban_scene(rng: np.random.Generator, half_extent=80.0, n_boxes=150, n_poles=50,
                keep_clear=((0.0, 0.0),)) -> Scene:
    """160 x 160 m plane with 200 objects: boxes (footprint 1-12 m, height 1-8 m)
    and poles (radius 0.15-0.3 m, height 3-8 m)."""
    boxes = []
    while len(boxes) < n_boxes:
        w, d = rng.uniform(1.0, 12.0, 2)
        h = rng.uniform(1.0, 8.0)
        cx, cy = rng.uniform(-half_extent + 6, half_extent - 6, 2)
        if any(abs(cx - kx) < w / 2 + 4.0 and abs(cy - ky) < d / 2 + 4.0 for kx, ky in keep_clear):
            continue
        boxes.append([cx - w / 2, cy - d / 2, 0.0, cx + w / 2, cy + d / 2, h])
    poles = []
    while len(poles) < n_poles:
        cx, cy = rng.uniform(-half_extent + 1, half_extent - 1, 2)
        if any(math.hypot(cx - kx, cy - ky) < 3.0 for kx, ky in keep_clear):
            continue
        poles.append([cx, cy, rng.uniform(0.15, 0.3), rng.uniform(3.0, 8.0)])
    return Scene(half_extent, np.array(boxes).reshape(-1, 6), np.array(poles).reshape(-1, 4))


def urban_pair(seed=None, max_offset=5.0, max_yaw_deg=15.0) -> Pair:
    """Single realistic pair: two 64-ring scans (elevation -24.8..+2 deg, 0.2 deg
    azimuth, range <= 80 m, ~115k points each, sigma 0.02 m) of a 160x160 m urban
    scene, the second taken from an offset of up to max_offset m and
    max_yaw_deg deg of yaw (plus tz in +-0.1 m and roll/pitch in +-1 deg).
    Grid: origin (-80,-80,-1), 320x320x20 voxels of 0.5 m."""
    rng = np.random.default_rng(seed_for(2) if seed is None else seed)
    d2r = math.pi / 180.0
    rad, ang = rng.uniform(0, max_offset), rng.uniform(0, 2 * math.pi)
    eta = np.array([rad * math.cos(ang), rad * math.sin(ang), rng.uniform(-0.1, 0.1),
                    rng.uniform(-1, 1) * d2r, rng.uniform(-1, 1) * d2r,
                    rng.uniform(-max_yaw_deg, max_yaw_deg) * d2r])
    scene = urban_scene(rng, keep_clear=((0.0, 0.0), (eta[0], eta[1])))
    A = raycast_scan(scene, np.zeros(6), rng)
    B = raycast_scan(scene, eta, rng)
    return Pair(as_soa32(A), as_soa32(B), eta, (-80.0, -80.0, -1.0), (320, 320, 20), 0.5)


@dataclass
class DisplacedSet:
    """One reference scan A and query scans B of the same scene taken from
    other poses: B[i] is expressed in its own frame and eta_gt[i] maps it
    into A's frame."""
    A: np.ndarray                      # float32 [3, nA]
    B: list                            # float32 [3, nB_i] each
    eta_gt: np.ndarray                 # float64 [n, 6]
    origin: tuple
    dims: tuple
    voxel: float
    study: str                         # "translation" or "rotation"
    levels: np.ndarray                 # the initial-error level of each query (m or deg)


def displaced_scans(seed=None, study="translation", levels=None, az_step=0.4) -> DisplacedSet:
    """Stand-in for the accuracy protocol of Sec. IV (Figs. 4, 5): a reference
    scan A at the origin of a ray-cast urban scene and query scans B from poses
    whose offset from A is the initial error the alignment starts with (it
    starts from the identity).

    study "translation": B at distance d in levels (default 1..10 m) along a
    seeded heading, with yaw U[-2, 2] deg, roll/pitch U[-1, 1] deg, tz U[-0.1, 0.1] m.
    study "rotation": yaw offsets of levels (default 2..20 deg in steps of 2,
    seeded sign) with a translation below 5 m (distance U[0, 5] m).
    Scans: 64 rings over -24.8..+2 deg, az_step deg azimuth, range <= 80 m.
    Grid: origin (-80,-80,-1), 160x160x10 voxels of 1 m, the resolution of the
    paper's experiments."""
    rng = np.random.default_rng(seed_for(6) if seed is None else seed)
    d2r = math.pi / 180.0
    if study == "translation":
        lv = np.arange(1.0, 11.0) if levels is None else np.asarray(levels, np.float64)
        etas = []
        for d in lv:
            ang = rng.uniform(0, 2 * math.pi)
            etas.append([d * math.cos(ang), d * math.sin(ang), rng.uniform(-0.1, 0.1),
                         rng.uniform(-1, 1) * d2r, rng.uniform(-1, 1) * d2r,
                         rng.uniform(-2, 2) * d2r])
    elif study == "rotation":
        lv = np.arange(2.0, 22.0, 2.0) if levels is None else np.asarray(levels, np.float64)
        etas = []
        for a in lv:
            d, ang = rng.uniform(0, 5.0), rng.uniform(0, 2 * math.pi)
            sign = 1.0 if rng.uniform() < 0.5 else -1.0
            etas.append([d * math.cos(ang), d * math.sin(ang), rng.uniform(-0.1, 0.1),
                         rng.uniform(-1, 1) * d2r, rng.uniform(-1, 1) * d2r, sign * a * d2r])
    else:
        raise ValueError("study must be 'translation' or 'rotation'")
    etas = np.array(etas, np.float64)
    scene = urban_scene(rng, keep_clear=((0.0, 0.0),) + tuple((e[0], e[1]) for e in etas))
    A = raycast_scan(scene, np.zeros(6), rng, az_step=az_step)
    B = [as_soa32(raycast_scan(scene, e, rng, az_step=az_step)) for e in etas]
    return DisplacedSet(as_soa32(A), B, etas, (-80.0, -80.0, -1.0), (160, 160, 10), 1.0, study, lv)


def surface_poses(center, half_xy=10.0, step_xy=0.25, half_yaw_deg=30.0, step_yaw_deg=0.25):
    """Pose sets of the cost-surface plots of Fig. 6: a (tx, ty) grid of
    +-half_xy m around center with every other parameter at center (row-major,
    ty fastest), and a heading sweep of +-half_yaw_deg around center's yaw.
    Returns (xy poses [nx*ny, 6], the x and y node values, yaw poses [n, 6],
    yaw node values in rad)."""
    c = np.asarray(center, np.float64)
    n = int(round(2 * half_xy / step_xy)) + 1
    xs = c[0] + np.linspace(-half_xy, half_xy, n)
    ys = c[1] + np.linspace(-half_xy, half_xy, n)
    P = np.repeat(c.reshape(1, 6), n * n, axis=0)
    P[:, 0] = np.repeat(xs, n)
    P[:, 1] = np.tile(ys, n)
    m = int(round(2 * half_yaw_deg / step_yaw_deg)) + 1
    yaws = c[5] + np.deg2rad(np.linspace(-half_yaw_deg, half_yaw_deg, m))
    Y = np.repeat(c.reshape(1, 6), m, axis=0)
    Y[:, 5] = yaws
    return P, xs, ys, Y, yaws


def level_poses(center, half, samples) -> np.ndarray:
    """A pose grid around center (per axis samples[a] values spanning
    +-half[a]), row-major with the last axis fastest -- used to draw sample
    poses of a search level as inputs."""
    axes = [np.array([center[a]]) if samples[a] == 1 else
            np.linspace(center[a] - half[a], center[a] + half[a], int(samples[a])) for a in range(6)]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.reshape(-1) for m in mesh], axis=1)


def urban_c2f_params():
    """3-level coarse-to-fine search of 5^6 poses per level: level-0 half-ranges
    (5, 5, 0.5 m, 2, 2, 15 deg), shrink 4x per level."""
    d2r = math.pi / 180.0
    half = np.array([5.0, 5.0, 0.5, 2 * d2r, 2 * d2r, 15 * d2r])
    return dict(half=half, samples=np.array([5, 5, 5, 5, 5, 5], np.int32), levels=3, shrink=4.0)


# --------------------------------------------------- uneven batch / serving

VOXEL_DIMS = {0.25: (640, 640, 40), 0.5: (320, 320, 20), 1.0: (160, 160, 10)}


def surface_pair(rng: np.random.Generator, n_points: int, voxel: float, half_extent=80.0,
                 crop=0.70, prior_range=(3.0, 3.0, 0.2, 2.0, 2.0, 10.0)) -> Pair:
    """Surface-sampled pair over a 160x160x10 m scene (the tiny workload's recipe
    scaled to the larger area: boxes and poles in proportion), n_points per
    scan, B cropped to 70% of the area and moved by a true pose within
    prior_range (m, m, m, deg, deg, deg)."""
    area_scale = (half_extent / 30.0) ** 2
    scene = make_box_scene(rng, half_extent, int(30 * area_scale), int(10 * area_scale))
    A = add_noise(sample_surfaces(scene, n_points, rng), rng)
    Bw = sample_surfaces(scene, int(n_points / crop), rng)
    side = 2 * half_extent * math.sqrt(crop)
    x0, y0 = rng.uniform(-half_extent, half_extent - side, 2)
    inside = (Bw[0] >= x0) & (Bw[0] < x0 + side) & (Bw[1] >= y0) & (Bw[1] < y0 + side)
    Bw = Bw[:, inside][:, :n_points]
    d2r = math.pi / 180.0
    pr = prior_range
    eta = np.array([rng.uniform(-pr[0], pr[0]), rng.uniform(-pr[1], pr[1]), rng.uniform(-pr[2], pr[2]),
                    rng.uniform(-pr[3], pr[3]) * d2r, rng.uniform(-pr[4], pr[4]) * d2r,
                    rng.uniform(-pr[5], pr[5]) * d2r])
    B = add_noise(to_frame(Bw, eta), rng)
    dims = VOXEL_DIMS[voxel]
    origin = (-half_extent, -half_extent, -1.0)
    return Pair(as_soa32(A), as_soa32(B), eta, origin, dims, voxel)


def uneven_pair(j, seed=None, n_range=(10_000, 300_000), voxels=(0.25, 0.5, 1.0),
                poses_per_pair=4096):
    """Pair j of the uneven batch: (Pair, poses[P, 6]).  Each pair has its own
    seed, so pairs can be generated independently (in parallel)."""
    d2r = math.pi / 180.0
    rng = np.random.default_rng(seed_for(4, j) if seed is None else seed + j)
    n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
    voxel = float(rng.choice(voxels))
    pair = surface_pair(rng, n, voxel)
    prior = pair.eta_gt + np.array([rng.normal(0, 0.5), rng.normal(0, 0.5), 0.0, 0.0, 0.0,
                                    rng.normal(0, 2 * d2r)])
    span = np.array([3.0, 3.0, 0.2, 2 * d2r, 2 * d2r, 10 * d2r])
    poses = prior + rng.uniform(-1, 1, (poses_per_pair, 6)) * span
    return pair, poses


def uneven_batch(n_pairs=64, seed=None, n_range=(10_000, 300_000), voxels=(0.25, 0.5, 1.0),
                 poses_per_pair=4096):
    """Uneven batch: per-pair point counts log-uniform in n_range, voxel size
    drawn from voxels, and poses_per_pair candidates uniform within +-3 m (x,y),
    +-0.2 m (z), +-10 deg yaw, +-2 deg roll/pitch of a seeded prior near the
    true pose.  Returns a list of (Pair, poses[P, 6])."""
    return [uneven_pair(j, seed, n_range, voxels, poses_per_pair) for j in range(n_pairs)]


def serving_requests(rate_hz: float, n_requests: int, seed=None, n_range=(20_000, 250_000),
                     voxels=(0.5, 1.0)):
    """Poisson arrivals at rate_hz: returns (arrival times [s], request specs).
    Each spec holds the point count and voxel size of a surface-sampled pair;
    make_request() materialises it."""
    rng = np.random.default_rng(seed_for(5) if seed is None else seed)
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    t = np.cumsum(gaps) - gaps[0]
    specs = []
    for j in range(n_requests):
        n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        specs.append(dict(index=j, n_points=n, voxel=float(rng.choice(voxels)),
                          seed=seed_for(5, j)))
    return t, specs


def make_request(spec) -> Pair:
    rng = np.random.default_rng(spec["seed"])
    return surface_pair(rng, spec["n_points"], spec["voxel"])
