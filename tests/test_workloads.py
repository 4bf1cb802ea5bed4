"""CPU checks of the accuracy and cost-surface workload generators (the
protocol of Sec. IV and Fig. 6 on synthetic stand-ins): the query scans sit
at the requested initial errors, the true pose brings B onto A's scene, and
the oracle scores the true pose above displaced ones."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1709_06948_amd import synth

D2R = math.pi / 180.0


@pytest.fixture(scope="module")
def trans():
    return synth.displaced_scans(study="translation", levels=[1.0, 4.0, 9.0])


def test_translation_study_offsets(trans):
    D = trans
    assert D.dims == (160, 160, 10) and D.voxel == 1.0
    assert np.allclose(np.linalg.norm(D.eta_gt[:, :2], axis=1), [1.0, 4.0, 9.0], atol=1e-12)
    assert np.all(np.abs(D.eta_gt[:, 2]) <= 0.1)
    assert np.all(np.abs(D.eta_gt[:, 3:5]) <= 1 * D2R) and np.all(np.abs(D.eta_gt[:, 5]) <= 2 * D2R)
    for B in D.B:
        assert B.dtype == np.float32 and B.shape[0] == 3 and B.shape[1] > 20_000


def test_rotation_study_headings():
    D = synth.displaced_scans(study="rotation", levels=[4.0, 16.0])
    assert np.allclose(np.abs(D.eta_gt[:, 5]) / D2R, [4.0, 16.0], atol=1e-9)
    assert np.all(np.linalg.norm(D.eta_gt[:, :2], axis=1) < 5.0)


def test_true_pose_maps_b_onto_a(trans):
    """p_A = R p_B + t with the generator's rotation: B's points then lie on
    the same surfaces as A's (most within 0.3 m of an A point in the plane)."""
    D = trans
    A = D.A.astype(np.float64)
    from scipy.spatial import cKDTree
    tree = cKDTree(A.T)
    for B, g in zip(D.B, D.eta_gt):
        Bw = synth._rot(g[3], g[4], g[5]) @ B.astype(np.float64) + g[:3].reshape(3, 1)
        d, _ = tree.query(Bw.T[::20])
        assert np.median(d) < 0.3, np.median(d)


def test_surface_pose_layout():
    c = np.array([0.4, -6.0, 0.05, 0.01, -0.01, 0.48])
    P, xs, ys, Y, yaws = synth.surface_poses(c, half_xy=1.0, step_xy=0.5, half_yaw_deg=2.0,
                                             step_yaw_deg=1.0)
    assert P.shape == (25, 6) and Y.shape == (5, 6)
    assert np.allclose(xs, c[0] + np.array([-1, -0.5, 0, 0.5, 1]))
    assert np.array_equal(P[1, :2], [xs[0], ys[1]])          # ty fastest
    assert np.array_equal(P[12], c)                           # the centre node is the pose
    assert np.array_equal(P[:, 2:], np.repeat(c[2:].reshape(1, 4), 25, axis=0))
    assert np.allclose(Y[:, 5], c[5] + np.deg2rad([-2, -1, 0, 1, 2]))
    assert np.array_equal(Y[:, :5], np.repeat(c[:5].reshape(1, 5), 5, axis=0))


def test_oracle_prefers_the_true_pose(trans):
    """On the 1 m query, the oracle's MI (z-variance) is highest at the true
    pose among it and poses 2 m / 5 deg away from it."""
    D = trans
    g = D.eta_gt[0]
    grid = O.Grid(D.origin, D.dims, D.voxel, features=3, nb_count=32, nb_zvar=32)
    P = [g, g + [2, 0, 0, 0, 0, 0], g + [0, -2, 0, 0, 0, 0], g + [0, 0, 0, 0, 0, 5 * D2R],
         g + [-2, 2, 0, 0, 0, -5 * D2R]]
    mi, _, _ = O.eval_poses(grid, D.A, D.B[0], np.array(P))
    assert mi[1, 0] > mi[1, 1:].max()
