"""mi_eval_poses_static (the entry point without a workspace) against
mi_eval_poses, through the C ABI: two calls in a row, the second with a
smaller input, on the shared-frame form and on the per-pose form (whose
buckets for a ~115k-point scan are more than the static scratch holds for
every resident workgroup, so the call runs fewer)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _same(a, b, want_hist=True):
    for f in range(len(a["mi"])):
        ma, mb = a["mi"][f].cpu().numpy(), b["mi"][f].cpu().numpy()
        assert np.max(np.abs(ma - mb)) <= 1e-6
        assert int(a["argmax"][f].item()) == int(b["argmax"][f].item())
        if want_hist:
            assert np.array_equal(a["hist"][f].cpu().numpy(), b["hist"][f].cpu().numpy())
    sa, sb = a["stats_raw"].cpu().numpy(), b["stats_raw"].cpu().numpy()
    assert sa.shape == sb.shape and np.array_equal(sa, sb)


def test_static_scratch_equals_workspace_two_calls_shrinking():
    from paper_1709_06948_amd import mi, synth
    p = synth.tiny_pair()
    grid = mi.Grid(p.origin, p.dims, p.voxel, features=3, nb_count=16, nb_zvar=32)
    ref = mi.Ref(grid, p.A)
    rng = np.random.default_rng(7)
    P1 = np.concatenate([rng.uniform(-2, 2, (300, 2)), rng.uniform(-0.2, 0.2, (300, 1)),
                         np.zeros((300, 2)), np.repeat(rng.uniform(-0.17, 0.17, (30, 1)), 10, 0)],
                        axis=1)
    B1 = p.B
    B2 = np.ascontiguousarray(p.B[:, : p.B.shape[1] // 3])
    P2 = P1[:40]
    for B, P in ((B1, P1), (B2, P2)):
        print(f"static vs workspace: tiny pair, {B.shape[1]} points, {len(P)} poses", flush=True)
        s = mi.eval_poses_static(ref, B, P, flags=mi.EVAL_NEAR_FACE, want_hist=True, want_stats=True)
        w = mi.eval_poses(ref, B, P, flags=mi.EVAL_NEAR_FACE, want_hist=True, want_stats=True)
        torch.cuda.synchronize()
        _same(s, w)


def test_static_scratch_per_pose_form_large_scan_two_calls():
    from paper_1709_06948_amd import mi, synth
    p = synth.urban_pair()
    grid = mi.Grid(p.origin, p.dims, p.voxel, features=3, nb_count=32, nb_zvar=32)
    ref = mi.Ref(grid, p.A)
    rng = np.random.default_rng(8)
    d2r = np.pi / 180
    P1 = p.eta_gt + rng.uniform(-1, 1, (96, 6)) * np.array([2, 2, 0.2, 2 * d2r, 2 * d2r, 5 * d2r])
    P2 = P1[:24]
    B2 = np.ascontiguousarray(p.B[:, ::2])
    for B, P in ((p.B, P1), (B2, P2)):
        print(f"static vs workspace, per-pose form: urban pair, {B.shape[1]} points, {len(P)} poses",
              flush=True)
        s = mi.eval_poses_static(ref, B, P, flags=mi.EVAL_PER_POSE, want_hist=True, want_stats=True)
        w = mi.eval_poses(ref, B, P, flags=mi.EVAL_PER_POSE, want_hist=True, want_stats=True)
        torch.cuda.synchronize()
        _same(s, w)


def test_static_scratch_rejects_oversized_sets():
    from paper_1709_06948_amd import mi, synth
    p = synth.urban_pair()
    grid = mi.Grid(p.origin, p.dims, p.voxel, features=1, nb_count=32)
    ref = mi.Ref(grid, p.A)
    # a scan whose single rotated frame (24 bytes per point) exceeds the static
    # scratch is rejected on the host, before any launch, with a clear error
    print("static scratch: oversized frame rejected", flush=True)
    big = np.zeros((3, 12_000_000), np.float32)
    big[0] = np.linspace(-70, 70, big.shape[1], dtype=np.float32)
    with pytest.raises(mi.MIError) as e:
        mi.eval_poses_static(ref, big, np.zeros((1, 6)), flags=mi.EVAL_SHARED_FRAMES)
    assert e.value.status == mi.MI_E_UNSUPPORTED
    assert "static scratch" in str(e.value)
