"""GPU tests of the searches built on the evaluator: the simplex search of
Sec. III-B (mi_align_nelder_mead) against the CPU oracle's, several starts
advancing together, and recovery of the true pose on the urban pair.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_1709_06948_amd import synth

pytestmark = pytest.mark.gpu

D2R = math.pi / 180.0
STEP = [1.0, 1.0, 0.1, 0.03, 0.03, 0.2]


@pytest.fixture(scope="module")
def M():
    from paper_1709_06948_amd import mi
    return mi


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("seed,features,slot", [(0, 1, 0), (2, 3, 1)])
def test_nelder_mead_matches_oracle(M, seed, features, slot):
    p = synth.tiny_pair() if seed == 0 else synth.tiny_pair(seed=synth.seed_for(1, seed))
    kw = dict(origin=p.origin, dims=p.dims, voxel=p.voxel, features=features, nb_count=16,
              nb_zvar=32)
    og = O.Grid(**kw)
    mg = M.Grid(**kw)
    ref = M.Ref(mg, p.A)
    _say("simplex search, tiny pair seed", seed, "features", features)
    pose, best, iters = M.align_nelder_mead(ref, p.B, np.zeros(6), STEP, 80, 1e-9, 1e-4,
                                            feature_slot=slot)
    opose, obest, oit = O.align_nelder_mead(og, p.A, p.B, np.zeros(6), STEP, 80, 1e-9, 1e-4,
                                            feature_slot=slot)
    assert int(iters[0]) == oit
    assert np.max(np.abs(pose - opose)) <= 1e-9, (pose, opose)
    assert abs(best - obest) <= 1e-6


def test_nelder_mead_starts_advance_independently(M):
    p = synth.tiny_pair()
    mg = M.Grid(p.origin, p.dims, p.voxel, features=1, nb_count=16)
    ref = M.Ref(mg, p.A)
    starts = np.array([[0, 0, 0, 0, 0, 0], [1.0, -1.0, 0, 0, 0, 0.1], [-1.5, 0.5, 0, 0, 0, -0.1]])
    pose, best, iters = M.align_nelder_mead(ref, p.B, starts, STEP, 60, 1e-9, 1e-4)
    singles = [M.align_nelder_mead(ref, p.B, s, STEP, 60, 1e-9, 1e-4) for s in starts]
    for i, (sp, sb, si) in enumerate(singles):
        assert int(iters[i]) == int(si[0]), i
    k = int(np.argmax([sb for _, sb, _ in singles]))
    assert np.array_equal(pose, singles[k][0]) and best == singles[k][1]


def test_urban_true_pose_is_the_mi_maximum_and_is_recovered(M):
    """On the urban pair, MI (both features) is larger at the true pose than
    anywhere on a local x-y and heading scan around it, and a coarse-to-fine
    grid fine enough for the MI basin (7,7,5,5,5,9 nodes, 4 levels, shrink 3)
    recovers the pose to 0.1 m / 0.25 deg.  (The benchmark's 5^6 grid with a
    2.5 m / 7.5 deg first step is wider than the basin and does not.)"""
    pair = synth.urban_pair()
    c2f = synth.urban_c2f_params()
    mg = M.Grid(pair.origin, pair.dims, pair.voxel, features=3, nb_count=32, nb_zvar=32)
    ref = M.Ref(mg, pair.A)
    g = pair.eta_gt
    xs = np.linspace(-2, 2, 17)
    P = [g] + [[g[0] + dx, g[1] + dy, *g[2:]] for dx in xs for dy in xs if dx or dy]
    P += [[*g[:5], g[5] + d * D2R] for d in np.linspace(-10, 10, 41) if d]
    r = M.eval_poses(ref, pair.B, np.array(P))
    mi_np = r["mi"].cpu().numpy()
    for f in range(2):
        assert mi_np[f, 0] > mi_np[f, 1:].max(), f
    og = O.Grid(pair.origin, pair.dims, pair.voxel, features=3, nb_count=32, nb_zvar=32)
    omi, _, _ = O.eval_poses(og, pair.A, pair.B, np.array([g]))
    assert np.max(np.abs(omi[:, 0] - mi_np[:, 0])) <= 1e-6
    for slot in range(2):
        pose, _ = M.align_coarse_to_fine(ref, pair.B, np.zeros(6), c2f["half"], [7, 7, 5, 5, 5, 9],
                                         4, 3.0, feature_slot=slot)
        err = np.abs(pose - g)
        _say("finer coarse-to-fine, feature", slot, "error", np.round(err, 4))
        assert err[:3].max() <= 0.1 and err[3:].max() <= 0.25 * D2R


def test_urban_ground_truth_over_ten_seeds(M):
    """Ground-truth recovery on 10 seeded urban pairs (second scan up to 5 m /
    15 deg away), both searches starting from the identity with the same
    level-0 ranges.  A finer grid search (7,7,5,5,5,9 nodes, 6 levels, shrink
    2) recovers the true pose within 0.1 m and 0.25 deg per parameter on at
    least 9 of 10.  The configured 5^6, 3-level, shrink-4 search lands within
    0.2 m (translation norm) and 1 deg (rotation norm) of the truth on at
    least 8 of 10: the oracle's calibration of it on these seeds gives 8 (the
    other two are 2.7-4.5 m away, in another MI basin).  Sampled poses of the
    finer search's last level are checked against the oracle."""
    c2f = synth.urban_c2f_params()
    h = np.asarray(c2f["half"])
    fine_ok = grid_ok = 0
    for j in range(10):
        pair = synth.urban_pair(seed=synth.seed_for(2, j))
        mg = M.Grid(pair.origin, pair.dims, pair.voxel, features=3, nb_count=32, nb_zvar=32)
        ref = M.Ref(mg, pair.A)
        g = pair.eta_gt
        fine, _ = M.align_coarse_to_fine(ref, pair.B, np.zeros(6), h, [7, 7, 5, 5, 5, 9], 6, 2.0,
                                         feature_slot=1)
        coarse, _ = M.align_coarse_to_fine(ref, pair.B, np.zeros(6), h, c2f["samples"],
                                           int(c2f["levels"]), c2f["shrink"], feature_slot=1)
        ef, ec = np.abs(fine - g), np.abs(coarse - g)
        f_ok = ef[:3].max() <= 0.1 and ef[3:].max() <= 0.25 * D2R
        c_ok = np.linalg.norm(ec[:3]) <= 0.2 and np.linalg.norm(ec[3:]) <= 1.0 * D2R
        fine_ok += f_ok
        grid_ok += c_ok
        _say("seed", j, "finer search error", np.round(ef, 4), f_ok, "| configured", np.round(ec, 3),
             c_ok)
        if j < 2:
            # the finer search's last level around its result, sampled against the oracle
            hl = h / 2.0 ** 5
            P = synth.level_poses(fine, hl, [7, 7, 5, 5, 5, 9])
            sel = np.random.default_rng(j).choice(len(P), 12, replace=False)
            r = M.eval_poses(ref, pair.B, P[sel])
            og = O.Grid(pair.origin, pair.dims, pair.voxel, features=3, nb_count=32, nb_zvar=32)
            omi, _, _ = O.eval_poses(og, pair.A, pair.B, P[sel])
            assert np.max(np.abs(omi - r["mi"].cpu().numpy())) <= 1e-6
    assert fine_ok >= 9, fine_ok
    assert grid_ok >= 8, grid_ok
