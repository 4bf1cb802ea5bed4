"""GPU parity of batches: many scan pairs of uneven size, grid and voxel size
evaluated in one schedule through the C ABI (mi_batch_* / mi_eval_batch).

Each item's histograms, overlap boxes and counts must equal the CPU oracle's
bit for bit and its MI be within 1e-6; and every item's results must be
identical to those of the same item evaluated alone.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_1709_06948_amd import synth

pytestmark = pytest.mark.gpu

MI_TOL = 1e-6


@pytest.fixture(scope="module")
def M():
    from paper_1709_06948_amd import mi
    return mi


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _grid_kw(pair, features, nb):
    return dict(origin=pair.origin, dims=pair.dims, voxel=pair.voxel, features=features,
                nb_count=nb, nb_zvar=nb)


def _check_item(M, og, grid, A, B, poses, res, label):
    omi, oh, ost = O.eval_poses(og, A, B, poses, want_hist=True, want_stats=True)
    torch.cuda.synchronize()
    K = len(poses)
    gmi = res["mi"].cpu().numpy()
    for f in range(grid.nf):
        gh = res["hist"][f].cpu().numpy().astype(np.int64).reshape(K, -1)
        bad = np.flatnonzero(np.any(gh != oh[f].reshape(K, -1).astype(np.int64), axis=1))
        assert bad.size == 0, f"{label} feature {f}: histograms differ at poses {bad[:10]}"
        d = np.max(np.abs(gmi[f] - omi[f])) if K else 0.0
        assert d <= MI_TOL, f"{label} feature {f}: max |dMI| = {d}"
        if res["argmax"] is not None and K:
            assert int(res["argmax"][f].item()) == O.argmax(omi[f]), label
    st = M.stats_to_numpy(res["stats_raw"], K)
    assert np.array_equal(st["lo"], ost[:, 0:3]) and np.array_equal(st["hi"], ost[:, 3:6]), label
    for i, name in enumerate(("n_overlap", "n_in_grid", "n_out_of_grid", "n_nonfinite",
                              "n_near_face")):
        assert np.array_equal(st[name], ost[:, 6 + i]), (label, name)


def _same(a, b, grid, label):
    torch.cuda.synchronize()
    assert torch.equal(a["mi"], b["mi"]), label
    for f in range(grid.nf):
        assert torch.equal(a["hist"][f], b["hist"][f]), (label, f)
    if a["argmax"] is not None:
        assert torch.equal(a["argmax"], b["argmax"]), label


def _mixed_pairs(n_pairs=5, K=48, seed=11):
    """Small uneven pairs: 6k-30k points, voxels 0.5 / 1.0 m, both feature
    sets, random 6-DOF poses around each true pose plus a shared-rotation
    block (so some frames serve several poses)."""
    out = []
    d2r = math.pi / 180.0
    for j in range(n_pairs):
        rng = np.random.default_rng(seed * 1000 + j)
        n = int(rng.integers(6_000, 30_000))
        voxel = (0.5, 1.0)[j % 2]
        pair = synth.surface_pair(rng, n, voxel, half_extent=40.0)
        span = np.array([2.0, 2.0, 0.2, 2 * d2r, 2 * d2r, 8 * d2r])
        rand = pair.eta_gt + rng.uniform(-1, 1, (K // 2, 6)) * span
        shared = np.repeat(rand[:1], K - K // 2, axis=0)
        shared[:, :3] += rng.uniform(-1, 1, (K - K // 2, 3)) * span[:3]
        poses = np.concatenate([rand, shared])
        features = (3, 1, 2)[j % 3]
        nb = (32, 16, 24)[j % 3]
        out.append((pair, poses, features, nb))
    return out


def test_batch_matches_oracle_and_single_items(M):
    items, keep = [], []
    for j, (pair, poses, features, nb) in enumerate(_mixed_pairs()):
        kw = _grid_kw(pair, features, nb)
        mg = M.Grid(**kw)
        ref = M.Ref(mg, pair.A)
        items.append(M.WorkItem(ref, pair.B, poses, want_hist=True, want_stats=True))
        keep.append((O.Grid(**kw), mg, ref, pair, poses))
    _say("batch of", len(items), "pairs,", sum(it.K for it in items), "poses")
    b = M.Batch(items, flags=M.EVAL_NEAR_FACE)
    b.execute()
    torch.cuda.synchronize()
    for j, (it, (og, mg, ref, pair, poses)) in enumerate(zip(items, keep)):
        _say("item", j, "n_b", pair.B.shape[1], "voxel", pair.voxel, "features", mg.features)
        res = it.results()
        _check_item(M, og, mg, pair.A, pair.B, poses, res, f"item {j}")
        alone = M.eval_poses(ref, pair.B, poses, flags=M.EVAL_NEAR_FACE, want_hist=True,
                             want_stats=True)
        _same(res, alone, mg, f"item {j} alone vs in batch")


def test_batch_chunked_frames_and_graph_replay(M):
    pairs = _mixed_pairs(n_pairs=3, K=40, seed=23)
    items, grids = [], []
    for pair, poses, features, nb in pairs:
        mg = M.Grid(**_grid_kw(pair, features, nb))
        ref = M.Ref(mg, pair.A)
        items.append(M.WorkItem(ref, pair.B, poses, want_hist=True, want_stats=True))
        grids.append((mg, ref, pair, poses))
    whole = M.Batch(items, flags=M.EVAL_NEAR_FACE)
    whole.execute()
    torch.cuda.synchronize()
    base = [dict(mi=it.mi.clone(), argmax=it.argmax.clone(),
                 hist=[h.clone() for h in it.results()["hist"]]) for it in items]
    # a frame budget of ~3 frames forces many chunks across pair boundaries
    small = M.Batch(items, flags=M.EVAL_NEAR_FACE, frame_budget=3 * 30_000 * 24)
    for it in items:
        it.mi.fill_(-1.0)
    small.execute()
    torch.cuda.synchronize()
    for j, (it, (mg, _, _, _)) in enumerate(zip(items, grids)):
        _same(it.results(), base[j], mg, f"chunked item {j}")
    # capture the whole batch in a graph and replay it with eager work between
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        whole.execute(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        whole.execute()
    for rep in range(3):
        for it in items:
            it.mi.fill_(-2.0)
            it.hist_raw.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for j, (it, (mg, _, _, _)) in enumerate(zip(items, grids)):
            _same(it.results(), base[j], mg, f"graph replay {rep} item {j}")


def test_uneven_batch_sampled_against_oracle(M):
    """The uneven-batch workload's recipe (log-uniform points, voxel sizes
    0.25 / 0.5 / 1 m, grids up to 640x640x40, count + z-variance at 32 bins)
    on 6 pairs with 4096 poses each; every pose's MI is checked against a
    sample evaluated by the oracle."""
    work = synth.uneven_batch(n_pairs=6, n_range=(10_000, 60_000), poses_per_pair=4096)
    items, keep = [], []
    for pair, poses in work:
        kw = _grid_kw(pair, 3, 32)
        mg = M.Grid(**kw)
        ref = M.Ref(mg, pair.A)
        items.append(M.WorkItem(ref, pair.B, poses, want_hist=True, want_stats=True))
        keep.append((O.Grid(**kw), mg, pair, poses))
    M.Batch(items, flags=M.EVAL_NEAR_FACE).execute()
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    for j, (it, (og, mg, pair, poses)) in enumerate(zip(items, keep)):
        sel = np.sort(rng.choice(len(poses), 12, replace=False))
        _say("uneven item", j, "n_b", pair.B.shape[1], "voxel", pair.voxel, "dims", pair.dims)
        res = it.results()
        sub = dict(mi=res["mi"][:, sel], argmax=None,
                   hist=[h[sel] for h in res["hist"]],
                   stats_raw=torch.from_numpy(
                       M.stats_to_numpy(res["stats_raw"], len(poses))[sel].view(np.uint8).copy()
                   ).cuda())
        _check_item(M, og, mg, pair.A, pair.B, poses[sel], sub, f"uneven item {j}")


def test_batch_errors_name_the_item(M):
    pair = synth.tiny_pair()
    mg = M.Grid(pair.origin, pair.dims, pair.voxel, features=1, nb_count=16)
    ref = M.Ref(mg, pair.A)
    good = M.WorkItem(ref, pair.B, synth.grid8_poses(2)[:8])
    bad_poses = np.zeros((4, 6))
    bad_poses[2, 4] = np.nan
    bad = M.WorkItem(ref, pair.B, bad_poses)
    with pytest.raises(M.MIError) as e:
        M.eval_batch([good, bad])
    assert "work item 1" in str(e.value) or e.value.status == M.MI_E_INVALID
    # an empty batch and items without poses are valid no-ops
    M.eval_batch([])
    M.eval_batch([M.WorkItem(ref, pair.B, np.zeros((0, 6)))])
    torch.cuda.synchronize()


def test_autotune_changes_speed_only(M):
    pair = synth.tiny_pair()
    mg = M.Grid(pair.origin, pair.dims, pair.voxel, features=3, nb_count=32, nb_zvar=32)
    ref = M.Ref(mg, pair.A)
    P = synth.grid8_poses(4)
    orig = M.tuning_get()
    try:
        before = M.WorkItem(ref, pair.B, P, want_hist=True)
        M.Batch([before]).execute()
        torch.cuda.synchronize()
        rep = M.autotune([before], max_poses=1024)
        _say("autotune", rep)
        assert rep["tried"] >= 10
        assert 0 < rep["best_ms"] <= rep["start_ms"]
        assert M.tuning_get() == rep["best"]
        after = M.WorkItem(ref, pair.B, P, want_hist=True)
        M.Batch([after]).execute()
        _same(after.results(), before.results(), mg, "autotuned vs default")
    finally:
        M.tuning_set(**orig)


def test_autotune_through_the_cache(M, tmp_path):
    """mi_autotune_cached: the first call times the candidates and stores the
    best tuning under the workload's key; the second finds it, makes it
    current without timing anything, and the results stay bit-identical."""
    pair = synth.tiny_pair()
    mg = M.Grid(pair.origin, pair.dims, pair.voxel, features=3, nb_count=32, nb_zvar=32)
    ref = M.Ref(mg, pair.A)
    P = synth.grid8_poses(4)
    cache = str(tmp_path / "tuning.json")
    orig = M.tuning_get()
    try:
        before = M.WorkItem(ref, pair.B, P, want_hist=True)
        M.Batch([before]).execute()
        torch.cuda.synchronize()
        first = M.autotune([before], max_poses=1024, cache=cache)
        M.tuning_set(**orig)
        second = M.autotune([before], max_poses=1024, cache=cache)
        _say("cached autotune", first["tried"], second)
        assert first["tried"] >= 10 and second["tried"] == 0
        assert second["best"] == first["best"] == M.tuning_get()
        key = M.tuning_cache_key(torch.cuda.get_device_properties(0).gcnArchName, 3, 32, 32,
                                 pair.B.shape[1], int(np.prod(mg.dims)))
        assert M.tuning_cache_get(cache, key) == first["best"]
        after = M.WorkItem(ref, pair.B, P, want_hist=True)
        M.Batch([after]).execute()
        _same(after.results(), before.results(), mg, "cached tuning vs default")
    finally:
        M.tuning_set(**orig)


def test_auto_hash_survives_a_tuning_round_trip(M):
    # hash_bytes = 0 is the auto size (66 KiB, or 60 KiB where 66 would leave
    # one workgroup per CU); a get / set round trip keeps it, so a large
    # z-variance grid (0.25 m, 640 x 640 x 40) still gets the fitting size.
    rng = np.random.default_rng(5)
    pair = synth.surface_pair(rng, 30_000, 0.25)
    mg = M.Grid(pair.origin, pair.dims, pair.voxel, features=3, nb_count=32, nb_zvar=32)
    assert tuple(mg.dims) == (640, 640, 40)
    ref = M.Ref(mg, pair.A)
    P = pair.eta_gt + rng.uniform(-0.05, 0.05, (64, 6))
    orig = M.tuning_get()
    try:
        assert orig["hash_bytes"] == 0, orig
        item = M.WorkItem(ref, pair.B, P)
        before = M.Batch([item]).launch()
        M.tuning_set(**M.tuning_get())
        assert M.tuning_get()["hash_bytes"] == 0
        after = M.Batch([item]).launch()
        _say("launch", before)
        assert before == after
        assert before["hash_bytes"] in (60 * 1024, 66 * 1024)
        assert before["lds_bytes"] <= 80 * 1024
        # an explicit size is used as given
        M.tuning_set(**dict(orig, hash_bytes=66 * 1024))
        assert M.Batch([item]).launch()["hash_bytes"] == 66 * 1024
    finally:
        M.tuning_set(**orig)
