"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Histograms, overlap boxes and point counts must be bit-exact; MI within 1e-6
absolute (the stated tolerance; in practice ~1e-15 since the histograms are
identical); argmax identical under the smallest-index-within-1e-12 rule.
"""
import json
import math
import os
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_1709_06948_amd import synth

pytestmark = pytest.mark.gpu

MI_TOL = 1e-6
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def M():
    from paper_1709_06948_amd import mi
    return mi


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _grids(M, **kw):
    okw = dict(kw)
    return O.Grid(**okw), M.Grid(**kw)


def _oracle(og, A, B, poses):
    return O.eval_poses(og, A, B, poses, want_hist=True, want_stats=True)


def _check(M, og, mg, A, B, poses, res, K=None, label=""):
    omi, oh, ost = _oracle(og, A, B, poses)
    torch.cuda.synchronize()
    K = len(poses)
    gmi = res["mi"].cpu().numpy()
    for f, (_, nb) in enumerate(mg.feature_list):
        gh = res["hist"][f].cpu().numpy().astype(np.int64)
        bad = np.flatnonzero(np.any(gh.reshape(K, -1) != oh[f].reshape(K, -1).astype(np.int64), axis=1))
        assert bad.size == 0, f"{label} feature {f}: histograms differ at poses {bad[:10]}"
        d = np.max(np.abs(gmi[f] - omi[f])) if K else 0.0
        assert d <= MI_TOL, f"{label} feature {f}: max |dMI| = {d}"
        if res["argmax"] is not None and K:
            assert int(res["argmax"][f].item()) == O.argmax(omi[f]), label
    if "stats_raw" in res:
        st = M.stats_to_numpy(res["stats_raw"], K)
        assert np.array_equal(st["lo"], ost[:, 0:3]) and np.array_equal(st["hi"], ost[:, 3:6])
        for i, name in enumerate(("n_overlap", "n_in_grid", "n_out_of_grid", "n_nonfinite",
                                  "n_near_face")):
            assert np.array_equal(st[name], ost[:, 6 + i]), (label, name)
    return omi


def _both_paths(M, og, mg, A, B, poses, label):
    ref = M.Ref(mg, A)
    # batched evaluator: automatic choice, then each way of feeding it forced
    for extra, name in ((0, "batched"), (M.EVAL_SHARED_FRAMES, "frames"),
                        (M.EVAL_PER_POSE, "per-pose")):
        r1 = M.eval_poses(ref, B, poses, flags=M.EVAL_NEAR_FACE | extra, want_hist=True,
                          want_stats=True)
        _check(M, og, mg, A, B, poses, r1, label=label + "/" + name)
    r2 = M.eval_poses_plain(ref, B, poses, flags=M.EVAL_NEAR_FACE, want_hist=True,
                            want_stats=True)
    _check(M, og, mg, A, B, poses, r2, label=label + "/plain")


# ------------------------------------------------------------ reference

def test_ref_features_bit_exact(M):
    p = synth.tiny_pair()
    kw = dict(origin=p.origin, dims=p.dims, voxel=p.voxel, features=3, nb_count=16, nb_zvar=32)
    og, mg = _grids(M, **kw)
    _say("ref features: tiny pair A", p.A.shape)
    ref = M.Ref(mg, p.A)
    o = O.scan_features(og, p.A)
    box, ctr = ref.summary()
    assert np.array_equal(box, o["box"]) and np.array_equal(ctr, o["counters"])
    for f in range(2):
        assert np.array_equal(ref.bins(f).cpu().numpy(), o["bins"][f])


# --------------------------------------------------------- tiny workload

def test_tiny_exhaustive_search_count16(M):
    p = synth.tiny_pair()
    P = synth.tiny_search_poses()
    kw = dict(origin=p.origin, dims=p.dims, voxel=p.voxel, features=1, nb_count=16)
    og, mg = _grids(M, **kw)
    _say("tiny 11^3 search, count 16 bins, K =", len(P))
    _both_paths(M, og, mg, p.A, p.B, P, "tiny-count16")


@pytest.mark.parametrize("seed", [0, 1])
def test_tiny_random_6dof_both_features(M, seed):
    p = synth.tiny_pair(seed=synth.seed_for(1, 50 + seed))
    rng = np.random.default_rng(seed)
    K = 301   # ragged: not a multiple of the 8 XCD slots
    P = np.concatenate([rng.uniform(-2.5, 2.5, (K, 2)), rng.uniform(-0.3, 0.3, (K, 1)),
                        rng.uniform(-0.05, 0.05, (K, 2)), rng.uniform(-0.25, 0.25, (K, 1))], 1)
    kw = dict(origin=p.origin, dims=p.dims, voxel=p.voxel, features=3, nb_count=32, nb_zvar=32)
    og, mg = _grids(M, **kw)
    _say("tiny random 6-DOF both features seed", seed)
    _both_paths(M, og, mg, p.A, p.B, P, f"tiny-6dof-{seed}")


# ------------------------------------------------------------ hand cases

def _hand_cases():
    with open(os.path.join(GOLDEN, "hand_cases.json")) as fh:
        return json.load(fh)["cases"]


@pytest.mark.parametrize("case", _hand_cases(), ids=lambda c: c["name"])
def test_hand_cases_gpu(M, case):
    gd = case["grid"]
    mg = M.Grid(gd["origin"], gd["dims"], gd["voxel"], features=1, nb_count=gd["nb_count"])
    A = np.array(case["A"], np.float32)
    B = np.array(case["B"], np.float32)
    _say("hand case", case["name"])
    ref = M.Ref(mg, A)
    for fn in (M.eval_poses, M.eval_poses_plain):
        r = fn(ref, B, np.array([case["pose"]]), want_hist=True, want_stats=True)
        torch.cuda.synchronize()
        nb = gd["nb_count"]
        want = np.zeros((nb, nb), np.int64)
        for a, b, c in case["hist_nonzero"]:
            want[a, b] = c
        assert np.array_equal(r["hist"][0][0].cpu().numpy().astype(np.int64), want)
        st = M.stats_to_numpy(r["stats_raw"], 1)
        assert list(st["lo"][0]) + list(st["hi"][0]) == case["overlap"]
        assert abs(r["mi"][0, 0].item() - case["mi"]) < 1e-12


# ------------------------------------------------- brute-force-sized grids

def _tiny_cloud(rng, n):
    P = rng.uniform(-0.5, 4.5, (3, n))
    P[:, 0] = [1.0, 2.0, 1.0]
    P[:, 1] = [0.0, 0.0, 0.0]
    P[:, 2] = [4.0, 1.0, 1.0]
    P[:, 3] = [-0.25, 1.5, 1.5]
    P[:, 4] = [3.0, 3.0, 3.0]
    P[:, 5] = [np.nan, 1.0, 1.0]
    return P.astype(np.float32)


@pytest.mark.parametrize("seed", range(3))
def test_small_grids_faces_and_outside(M, seed):
    rng = np.random.default_rng(100 + seed)
    A = _tiny_cloud(rng, 60)
    B = _tiny_cloud(rng, 50)
    poses = np.array([[0, 0, 0, 0, 0, 0], [1.0, 0, 0, 0, 0, 0], [0.5, -0.5, 0.25, 0, 0, 0.2],
                      [0, 0, 0, 0.1, -0.1, -0.4], [7.0, 0, 0, 0, 0, 0], [-1.0, -1.0, -1.0, 0, 0, 0]])
    kw = dict(origin=(0.0, 0.0, 0.0), dims=(4, 4, 4), voxel=1.0, features=3, nb_count=5, nb_zvar=8)
    og, mg = _grids(M, **kw)
    _say("4x4x4 grid seed", seed)
    _both_paths(M, og, mg, A, B, poses, f"4x4x4-{seed}")


# -------------------------------------------------------------- edge cases

def test_edge_cases(M):
    p = synth.tiny_pair()
    kw = dict(origin=p.origin, dims=p.dims, voxel=p.voxel, features=3, nb_count=16, nb_zvar=32)
    og, mg = _grids(M, **kw)
    P = np.array([[0, 0, 0, 0, 0, 0], [300.0, 0, 0, 0, 0, 0], [0, 0, -50.0, 0, 0, 0]])
    _say("edge: empty B")
    _both_paths(M, og, mg, p.A, np.zeros((3, 0), np.float32), P, "empty-B")
    _say("edge: all-NaN B")
    nanB = np.full((3, 17), np.nan, np.float32)
    _both_paths(M, og, mg, p.A, nanB, P, "nan-B")
    _say("edge: empty A")
    _both_paths(M, og, mg, np.zeros((3, 0), np.float32), p.B, P, "empty-A")
    _say("edge: single pose, single point")
    _both_paths(M, og, mg, p.A, p.B[:, :1].copy(), P[:1], "one-point")
    _say("edge: points on voxel faces")
    face = np.stack(np.meshgrid(np.arange(-5, 5, 1.0), np.arange(-5, 5, 1.0), [0.0, 1.0, 2.0],
                                indexing="ij")).reshape(3, -1).astype(np.float32)
    _both_paths(M, og, mg, face, face, np.array([[0, 0, 0, 0, 0, 0], [1.0, 2.0, 0, 0, 0, 0]]),
                "faces")


def test_custom_edges(M):
    """Caller-given bin edges: count edges that are not 1..nb-1 (so the binary
    search runs) and z-variance edges with repeats and a zero edge."""
    p = synth.tiny_pair()
    ce = np.array([1, 2, 3, 5, 8, 13, 21, 34], np.uint32)
    ze = np.array([0, 0, 5, 100, 100, 1_000, 100_000, 10_000_000, 1_000_000_000, 10 ** 11],
                  np.uint64)
    kw = dict(origin=p.origin, dims=p.dims, voxel=p.voxel, features=3, nb_count=9, nb_zvar=12,
              count_edges=ce, zvar_edges=ze)
    og, mg = _grids(M, **kw)
    rng = np.random.default_rng(7)
    K = 97
    P = np.concatenate([rng.uniform(-2, 2, (K, 2)), rng.uniform(-0.2, 0.2, (K, 1)),
                        rng.uniform(-0.03, 0.03, (K, 2)), rng.uniform(-0.2, 0.2, (K, 1))], 1)
    _say("custom edges")
    _both_paths(M, og, mg, p.A, p.B, P, "custom-edges")


def test_zero_poses(M):
    p = synth.tiny_pair()
    mg = M.Grid(p.origin, p.dims, p.voxel, features=1, nb_count=16)
    ref = M.Ref(mg, p.A)
    r = M.eval_poses(ref, p.B, np.zeros((0, 6)), want_argmax=False)
    torch.cuda.synchronize()
    assert r["mi"].shape == (1, 0)


# ------------------------------------------------- execution-form equality

def test_chunked_frames_and_tuning_variants_identical(M):
    p = synth.tiny_pair()
    kw = dict(origin=p.origin, dims=p.dims, voxel=p.voxel, features=3, nb_count=32, nb_zvar=32)
    mg = M.Grid(**kw)
    ref = M.Ref(mg, p.A)
    P = synth.grid8_poses(4)            # 4096 poses, 64 distinct rotations
    base = M.eval_poses(ref, p.B, P, want_hist=True)
    torch.cuda.synchronize()
    bh = [h.cpu().numpy() for h in base["hist"]]
    bmi = base["mi"].cpu().numpy()
    orig = M.tuning_get()
    try:
        for waves, hb, hc, sr, pw in [(4, 98304, 1, 8, 0), (8, 49152, 2, 4, 0),
                                      (2, 36864, 1, 16, 0), (16, 98304, 4, 1, 0),
                                      (1, 65536, 1, 3, 0), (1, 8192, 2, 62, 0),
                                      (3, 16384, 2, 40, 0), (8, 49152, 2, 8, 1),
                                      (4, 24576, 1, 8, 3), (16, 98304, 2, 16, 1)]:
            # the last three run a persistent grid: workgroups loop over poses
            _say("tuning", waves, hb, hc, sr, pw)
            M.tuning_set(waves, hb, hc, sr, pw)
            r = M.eval_poses(ref, p.B, P, want_hist=True)
            torch.cuda.synchronize()
            for f in range(2):
                assert np.array_equal(r["hist"][f].cpu().numpy(), bh[f])
            assert np.array_equal(r["mi"].cpu().numpy(), bmi)
    finally:
        M.tuning_set(**orig)
    _say("chunked frames")
    plan = M.Plan(ref, p.B.shape[1], P, frame_budget=3 * 1024 * 1024)
    xb = torch.from_numpy(p.B).cuda()
    mi_t = torch.empty((2, len(P)), dtype=torch.float64, device="cuda")
    tot = sum(len(P) * nb * nb for _, nb in mg.feature_list)
    hist = torch.empty(tot, dtype=torch.int32, device="cuda")
    plan.execute(xb, mi_t, hist=hist)
    torch.cuda.synchronize()
    assert np.array_equal(mi_t.cpu().numpy(), bmi)
    n0 = len(P) * 32 * 32
    assert np.array_equal(hist[:n0].cpu().numpy().reshape(bh[0].shape), bh[0])


def test_plan_graph_replay(M):
    p = synth.tiny_pair()
    mg = M.Grid(p.origin, p.dims, p.voxel, features=3, nb_count=16, nb_zvar=32)
    ref = M.Ref(mg, p.A)
    P = synth.tiny_search_poses()
    xb = torch.from_numpy(p.B).cuda()
    plan = M.Plan(ref, xb.shape[1], P)
    eager = torch.empty((2, len(P)), dtype=torch.float64, device="cuda")
    am_e = torch.empty(2, dtype=torch.int64, device="cuda")
    plan.execute(xb, eager, am_e)
    torch.cuda.synchronize()
    out = torch.zeros_like(eager)
    am = torch.zeros_like(am_e)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.execute(xb, out, am, stream=s)     # warm-up outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.execute(xb, out, am)
    for rep in range(3):
        out.zero_()
        am.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _say("graph replay", rep)
        assert torch.equal(out, eager) and torch.equal(am, am_e)
        junk = torch.randn(1000, device="cuda").sum().item()   # eager work between replays
        assert math.isfinite(junk)


# ------------------------------------------------------------ urban pair

@pytest.fixture(scope="module")
def urban():
    return synth.urban_pair()


def test_urban_pair_sampled_poses(M, urban):
    p = urban
    kw = dict(origin=p.origin, dims=p.dims, voxel=p.voxel, features=3, nb_count=32, nb_zvar=32)
    og, mg = _grids(M, **kw)
    c2f = synth.urban_c2f_params()
    full = O.grid_poses(np.zeros(6), c2f["half"], c2f["samples"])       # level-0 grid
    rng = np.random.default_rng(9)
    idx = np.sort(rng.choice(len(full), 12, replace=False))
    P = np.concatenate([full[idx], p.eta_gt[None, :]])
    _say("urban pair sampled poses", len(P), "A", p.A.shape, "B", p.B.shape)
    _both_paths(M, og, mg, p.A, p.B, P, "urban")


def test_urban_full_level_sampled_against_oracle(M, urban):
    # the full 5^6 level in one launch; the oracle checks a sample of it
    p = urban
    kw = dict(origin=p.origin, dims=p.dims, voxel=p.voxel, features=3, nb_count=32, nb_zvar=32)
    og, mg = _grids(M, **kw)
    c2f = synth.urban_c2f_params()
    P = O.grid_poses(np.zeros(6), c2f["half"], c2f["samples"])
    ref = M.Ref(mg, p.A)
    _say("urban full level", len(P))
    r = M.eval_poses(ref, p.B, P, want_hist=True, want_stats=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    idx = np.sort(rng.choice(len(P), 10, replace=False))
    omi, oh, _ = O.eval_poses(og, p.A, p.B, P[idx], want_hist=True)
    for f in range(2):
        gh = r["hist"][f][torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.int64)
        assert np.array_equal(gh, oh[f].astype(np.int64))
        assert np.max(np.abs(r["mi"][f].cpu().numpy()[idx] - omi[f])) <= MI_TOL
    # properties that hold at any size, on every pose of the level (Eqs. 2-5,
    # overlap step of Alg. 1): histogram mass = |O| from the pose's overlap
    # box, and 0 <= MI <= min(H(X), H(Y)) with the marginal entropies of each
    # pose's own histogram
    st = M.stats_to_numpy(r["stats_raw"], len(P))
    ext = np.clip(st["hi"] - st["lo"] + 1, 0, None)
    nO = torch.from_numpy(np.prod(ext.astype(np.int64), axis=1)).cuda()
    assert torch.equal(torch.from_numpy(st["n_overlap"]).cuda(), nO)
    assert torch.all(nO > 0)

    def ent(c, N):
        p = c.to(torch.float64) / N[:, None]
        return -(torch.where(p > 0, p * torch.log(p), torch.zeros_like(p))).sum(dim=1)

    for f, (_, nb) in enumerate(mg.feature_list):
        H = r["hist"][f].to(torch.int64)
        mass = H.sum(dim=(1, 2))
        assert torch.equal(mass, nO), f"feature {f}: mass differs from |O|"
        N = mass.to(torch.float64)
        hx, hy = ent(H.sum(dim=2), N), ent(H.sum(dim=1), N)
        m = r["mi"][f]
        assert torch.all(m >= -1e-12)
        assert torch.all(m <= torch.minimum(hx, hy) + 1e-12)


def test_coarse_to_fine_matches_oracle(M):
    p = synth.tiny_pair()
    kw = dict(origin=p.origin, dims=p.dims, voxel=p.voxel, features=2, nb_zvar=32)
    og, mg = _grids(M, **kw)
    half = np.array([2.0, 2.0, 0.2, math.radians(2), math.radians(2), math.radians(10)])
    samples = np.array([3, 3, 3, 3, 3, 3], np.int32)
    _say("coarse-to-fine 3 levels of 3^6")
    ref = M.Ref(mg, p.A)
    pose, best = M.align_coarse_to_fine(ref, p.B, np.zeros(6), half, samples, 3, 3.0, 0)
    opose, obest = O.align_c2f(og, p.A, p.B, np.zeros(6), half, samples, 3, 3.0, 0)
    assert np.array_equal(pose, opose)
    assert abs(best - obest) <= MI_TOL
