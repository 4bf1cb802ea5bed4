"""GPU tests of the accuracy and cost-surface workloads (Sec. IV protocol,
Fig. 6) on synthetic displaced scans at 1 m voxels: sampled surface poses
against the CPU oracle, and the simplex search from the identity recovering
nearby queries."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_1709_06948_amd import synth

pytestmark = pytest.mark.gpu

D2R = math.pi / 180.0
STEP = [8.0, 8.0, 1.0, 0.1, 0.1, 0.8]   # the paper's initial simplex


@pytest.fixture(scope="module")
def M():
    from paper_1709_06948_amd import mi
    return mi


@pytest.fixture(scope="module")
def D():
    return synth.displaced_scans(study="translation", levels=[1.0, 2.0, 3.0, 6.0])


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_surface_samples_match_oracle(M, D):
    g = D.eta_gt[3]
    P, xs, ys, Y, yaws = synth.surface_poses(g)
    rng = np.random.default_rng(0)
    Ps = np.concatenate([P[rng.choice(len(P), 10, replace=False)], Y[rng.choice(len(Y), 4,
                                                                                   replace=False)],
                         g.reshape(1, 6)])
    kw = dict(origin=D.origin, dims=D.dims, voxel=D.voxel, features=3, nb_count=32, nb_zvar=32)
    ref = M.Ref(M.Grid(**kw), D.A)
    _say("surface samples", len(Ps))
    r = M.eval_poses(ref, D.B[3], Ps, want_hist=True)
    torch.cuda.synchronize()
    omi, oh, _ = O.eval_poses(O.Grid(**kw), D.A, D.B[3], Ps, want_hist=True)
    for f in range(2):
        assert np.array_equal(r["hist"][f].cpu().numpy().astype(np.int64), oh[f].astype(np.int64))
        assert np.max(np.abs(r["mi"][f].cpu().numpy() - omi[f])) <= 1e-6


@pytest.mark.parametrize("i", [0, 1, 2])
def test_simplex_search_recovers_nearby_queries(M, D, i):
    """Four starts around the identity, MI-VARZ: queries 1-3 m away are
    recovered to within one voxel (1 m) and 2 deg, the workload's success rule."""
    grid = M.Grid(D.origin, D.dims, D.voxel, features=3, nb_count=32, nb_zvar=32)
    ref = M.Ref(grid, D.A)
    starts = np.array([[0, 0, 0, 0, 0, 0], [4, 4, 0, 0, 0, 0.3], [-4, 4, 0, 0, 0, -0.3],
                       [0, -5, 0, 0, 0, 0]], np.float64)
    pose, best, it = M.align_nelder_mead(ref, D.B[i], starts, STEP, 400, 1e-7, 1e-3,
                                         feature_slot=1)
    g = D.eta_gt[i]
    et = float(np.linalg.norm(pose[:3] - g[:3]))
    er = float(np.linalg.norm(pose[3:] - g[3:]) / D2R)
    _say("query", D.levels[i], "m: error", round(et, 3), "m", round(er, 3), "deg, iterations", it)
    assert et < 1.0 and er < 2.0
