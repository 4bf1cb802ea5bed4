"""GPU parity on degenerate and maximum-size inputs, through the C ABI,
against the CPU oracle: the largest scan B the z-variance feature accepts,
every point in one voxel, a one-voxel grid, the fewest bins, identical
points, and the size limit's error."""
import sys

import numpy as np
import pytest
import torch

import oracle as O

pytestmark = pytest.mark.gpu

MI_TOL = 1e-6


@pytest.fixture(scope="module")
def M():
    from paper_1709_06948_amd import mi
    return mi


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _compare(M, kw, A, B, poses, label, flags_extra=(0,)):
    og = O.Grid(**kw)
    mg = M.Grid(**kw)
    ref = M.Ref(mg, A)
    omi, oh, ost = O.eval_poses(og, A, B, poses, want_hist=True, want_stats=True)
    K = len(poses)
    forms = [("plain", None)] + [(f"batched/{e}", e) for e in flags_extra]
    for name, extra in forms:
        if extra is None:
            r = M.eval_poses_plain(ref, B, poses, flags=M.EVAL_NEAR_FACE, want_hist=True,
                                   want_stats=True)
        else:
            r = M.eval_poses(ref, B, poses, flags=M.EVAL_NEAR_FACE | extra, want_hist=True,
                             want_stats=True)
        torch.cuda.synchronize()
        gmi = r["mi"].cpu().numpy()
        for f in range(mg.nf):
            gh = r["hist"][f].cpu().numpy().astype(np.int64).reshape(K, -1)
            assert np.array_equal(gh, oh[f].reshape(K, -1).astype(np.int64)), (label, name, f)
            assert np.max(np.abs(gmi[f] - omi[f])) <= MI_TOL, (label, name, f)
        st = M.stats_to_numpy(r["stats_raw"], K)
        for i, field in enumerate(("n_overlap", "n_in_grid", "n_out_of_grid", "n_nonfinite",
                                   "n_near_face")):
            assert np.array_equal(st[field], ost[:, 6 + i]), (label, name, field)


def test_largest_scan_b_with_z_variance(M):
    """n_b = 2^20 - 1, the most the packed (n << 44 | S1) sums accept, over a
    small grid so that voxels hold thousands of points each."""
    rng = np.random.default_rng(1)
    n = (1 << 20) - 1
    B = np.stack([rng.uniform(0, 8, n), rng.uniform(0, 8, n), rng.uniform(0, 4, n)]).astype(
        np.float32)
    A = np.stack([rng.uniform(0, 8, 50_000), rng.uniform(0, 8, 50_000),
                  rng.uniform(0, 4, 50_000)]).astype(np.float32)
    kw = dict(origin=(0.0, 0.0, 0.0), dims=(8, 8, 4), voxel=1.0, features=3, nb_count=64,
              nb_zvar=64, count_edges=np.arange(1, 64, dtype=np.uint32) * 256)
    poses = np.array([[0, 0, 0, 0, 0, 0], [0.5, -0.25, 0.1, 0.01, -0.02, 0.3]])
    _say("n_b = 2^20 - 1")
    _compare(M, kw, A, B, poses, "max-n", flags_extra=(M.EVAL_SHARED_FRAMES, M.EVAL_PER_POSE))


def test_size_limit_is_an_error(M):
    kw = dict(origin=(0.0, 0.0, 0.0), dims=(4, 4, 4), voxel=1.0, features=2, nb_zvar=8)
    mg = M.Grid(**kw)
    ref = M.Ref(mg, np.zeros((3, 10), np.float32))
    B = torch.zeros((3, 1 << 20), dtype=torch.float32, device="cuda")
    with pytest.raises(M.MIError) as e:
        M.eval_poses(ref, B, np.zeros((1, 6)))
    assert e.value.status == M.MI_E_UNSUPPORTED


def test_every_point_in_one_voxel(M):
    rng = np.random.default_rng(2)
    A = (np.array([[2.5], [2.5], [1.5]]) + rng.uniform(-0.4, 0.4, (3, 5000))).astype(np.float32)
    B = (np.array([[2.5], [2.5], [1.5]]) + rng.uniform(-0.4, 0.4, (3, 7000))).astype(np.float32)
    kw = dict(origin=(0.0, 0.0, 0.0), dims=(5, 5, 3), voxel=1.0, features=3, nb_count=16,
              nb_zvar=16)
    poses = np.array([[0, 0, 0, 0, 0, 0], [1.0, 0, 0, 0, 0, 0], [0.2, 0.1, 0.05, 0, 0, 0.05]])
    _compare(M, kw, A, B, poses, "one-voxel-cloud",
             flags_extra=(M.EVAL_SHARED_FRAMES, M.EVAL_PER_POSE))


def test_one_voxel_grid_and_fewest_bins(M):
    rng = np.random.default_rng(3)
    A = rng.uniform(0, 1, (3, 40)).astype(np.float32)
    B = rng.uniform(-0.5, 1.5, (3, 60)).astype(np.float32)
    kw = dict(origin=(0.0, 0.0, 0.0), dims=(1, 1, 1), voxel=1.0, features=3, nb_count=2,
              nb_zvar=3)
    poses = np.array([[0, 0, 0, 0, 0, 0], [0.3, 0.3, 0.3, 0, 0, 0], [2.0, 0, 0, 0, 0, 0]])
    _compare(M, kw, A, B, poses, "1x1x1", flags_extra=(M.EVAL_SHARED_FRAMES, M.EVAL_PER_POSE))


def test_identical_points_and_single_pose(M):
    A = np.tile(np.array([[1.25], [3.75], [0.5]], np.float32), (1, 300))
    B = np.tile(np.array([[1.25], [3.75], [0.5]], np.float32), (1, 200))
    kw = dict(origin=(0.0, 0.0, 0.0), dims=(6, 6, 2), voxel=1.0, features=3, nb_count=8,
              nb_zvar=8)
    _compare(M, kw, A, B, np.zeros((1, 6)), "identical-points",
             flags_extra=(M.EVAL_SHARED_FRAMES, M.EVAL_PER_POSE))


def test_coarse_to_fine_level_size_limit(M):
    """A level of 2^31 or more poses is rejected before any allocation."""
    kw = dict(origin=(0.0, 0.0, 0.0), dims=(4, 4, 4), voxel=1.0, features=1, nb_count=4)
    mg = M.Grid(**kw)
    A = np.random.default_rng(5).uniform(0, 4, (3, 100)).astype(np.float32)
    ref = M.Ref(mg, A)
    with pytest.raises(M.MIError) as e:
        M.align_coarse_to_fine(ref, A, np.zeros(6), [1.0] * 6, [1024, 1024, 1024, 2, 1, 1], 1,
                               2.0)
    assert e.value.status == M.MI_E_INVALID
    pose, best = M.align_coarse_to_fine(ref, A, np.zeros(6), [1.0] * 6, [2, 2, 1, 1, 1, 3], 1, 2.0)
    assert np.all(np.isfinite(pose)) and np.isfinite(best)
