"""GPU tests of the binding on a stream other than torch's current one: the
reference, single-call evaluation, a plan, a batch and a search issued on a
side stream give the same results as on the default stream (allocations and
copies of the binding follow the stream the library calls run on)."""
import math
import sys

import numpy as np
import pytest
import torch

from paper_1709_06948_amd import synth

pytestmark = pytest.mark.gpu

D2R = math.pi / 180.0


@pytest.fixture(scope="module")
def M():
    from paper_1709_06948_amd import mi
    return mi


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_side_stream_equals_default_stream(M):
    p = synth.tiny_pair()
    grid = M.Grid(p.origin, p.dims, p.voxel, features=3, nb_count=16, nb_zvar=32)
    poses = synth.level_poses(np.zeros(6), np.array([1.0, 1.0, 0.1, 1 * D2R, 1 * D2R, 5 * D2R]),
                              [3, 3, 2, 2, 2, 5])
    K = len(poses)
    _say("default stream, K =", K)
    ref0 = M.Ref(grid, p.A)
    r0 = M.eval_poses(ref0, p.B, poses, want_hist=True)
    torch.cuda.synchronize()
    mi0 = r0["mi"].cpu().numpy()
    h0 = [h.cpu().numpy() for h in r0["hist"]]
    c2f0 = M.align_coarse_to_fine(ref0, p.B, np.zeros(6), [1.0, 1.0, 0.1, D2R, D2R, 5 * D2R],
                                  [3, 3, 3, 3, 3, 3], 2, 3.0, feature_slot=1)

    s = torch.cuda.Stream()
    _say("side stream")
    ref1 = M.Ref(grid, p.A, stream=s)
    r1 = M.eval_poses(ref1, p.B, poses, want_hist=True, stream=s)
    B_dev = torch.from_numpy(p.B).cuda()
    plan = M.Plan(ref1, B_dev.shape[1], poses, stream=s)
    with torch.cuda.stream(s):
        out = torch.empty((grid.nf, K), dtype=torch.float64, device="cuda")
    torch.cuda.current_stream().synchronize()   # B_dev's copy, made on the default stream
    plan.execute(B_dev, out, stream=s)
    item = M.WorkItem(ref1, p.B, poses, want_hist=True)
    torch.cuda.current_stream().synchronize()   # the item's inputs and outputs
    batch = M.Batch([item], stream=s)
    batch.execute(stream=s)
    c2f1 = M.align_coarse_to_fine(ref1, p.B, np.zeros(6), [1.0, 1.0, 0.1, D2R, D2R, 5 * D2R],
                                  [3, 3, 3, 3, 3, 3], 2, 3.0, feature_slot=1, stream=s)
    s.synchronize()
    assert np.array_equal(r1["mi"].cpu().numpy(), mi0)
    for f in range(grid.nf):
        assert np.array_equal(r1["hist"][f].cpu().numpy(), h0[f]), f
    assert np.array_equal(out.cpu().numpy(), mi0)
    res = item.results()
    assert np.array_equal(res["mi"].cpu().numpy(), mi0)
    for f in range(grid.nf):
        assert np.array_equal(res["hist"][f].cpu().numpy(), h0[f]), f
    assert np.array_equal(c2f1[0], c2f0[0]) and c2f1[1] == c2f0[1]
