"""GPU tests of the serving loop (mi_server_* through the C ABI).

Each request's result from the server, with other requests of different
sizes in flight and admitted at different times, must be bit-identical to
the same alignment run alone by mi_align_coarse_to_fine; one request is also
checked against the CPU oracle's coarse-to-fine search.  Admission follows
arrival order, the slot count and the arena budget.
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


@pytest.fixture(scope="module")
def M():
    from paper_1709_06948_amd import mi
    return mi


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _requests(n, seed=3, n_range=(8_000, 40_000)):
    """Surface-sampled pairs over an 80 x 80 m area, 0.5 or 1 m voxels, both
    features, searches of 3 levels x 3^6 poses around a prior."""
    out = []
    for j in range(n):
        rng = np.random.default_rng(seed * 100 + j)
        npts = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        voxel = (0.5, 1.0)[j % 2]
        pair = synth.surface_pair(rng, npts, voxel, half_extent=40.0,
                                  prior_range=(2.0, 2.0, 0.1, 1.0, 1.0, 6.0))
        dims = (int(80 / voxel), int(80 / voxel), int(10 / voxel))
        init = pair.eta_gt + np.array([rng.normal(0, 0.4), rng.normal(0, 0.4), 0, 0, 0,
                                       rng.normal(0, 1.5 * D2R)])
        out.append(dict(origin=(-40.0, -40.0, -1.0), dims=dims, voxel=voxel, A=pair.A, B=pair.B,
                        init=init, half=(1.5, 1.5, 0.15, 1.5 * D2R, 1.5 * D2R, 4.0 * D2R),
                        samples=(3, 3, 3, 3, 3, 3), levels=3, shrink=3.0,
                        feature_slot=j % 2))
    return out


def _submit(srv, q):
    return srv.submit(q["origin"], q["dims"], q["voxel"], q["A"], q["B"], q["init"], q["half"],
                      q["samples"], q["levels"], q["shrink"], features=3, nb_count=32,
                      nb_zvar=32, feature_slot=q["feature_slot"])


def _alone(M, q):
    g = M.Grid(q["origin"], q["dims"], q["voxel"], features=3, nb_count=32, nb_zvar=32)
    ref = M.Ref(g, q["A"])
    return M.align_coarse_to_fine(ref, q["B"], q["init"], q["half"], q["samples"], q["levels"],
                                  q["shrink"], feature_slot=q["feature_slot"])


def _drain(srv, ids, max_steps=200):
    for _ in range(max_steps):
        na, nq = srv.step()
        if na == 0 and nq == 0:
            break
    out = {i: srv.poll(i) for i in ids}
    return out


def test_results_in_the_mix_equal_alone(M):
    qs = _requests(6)
    srv = M.Server(arena_bytes=6 << 30, max_active=8)
    ids = []
    # staggered arrivals: requests join while others are between levels
    ids += [_submit(srv, qs[0]), _submit(srv, qs[1])]
    srv.step()
    ids += [_submit(srv, qs[2]), _submit(srv, qs[3])]
    srv.step()
    ids.append(_submit(srv, qs[4]))
    srv.step()
    ids.append(_submit(srv, qs[5]))
    res = _drain(srv, ids)
    for j, (q, rid) in enumerate(zip(qs, ids)):
        r = res[rid]
        _say("request", j, "n_b", q["B"].shape[1], "voxel", q["voxel"], "state", r["state"],
             "levels", r["levels_done"], "mi", r["mi"])
        assert r["state"] == M.REQ_DONE and r["levels_done"] == 3, r
        pose, best = _alone(M, q)
        assert np.array_equal(r["pose"], pose), (j, r["pose"], pose)
        assert r["mi"] == best, (j, r["mi"], best)
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
        srv.release(rid)
    srv.close()


def test_server_request_matches_oracle_search(M):
    q = _requests(2, seed=9, n_range=(6_000, 12_000))[1]   # 1 m voxels: 80 x 80 x 10
    q["levels"] = 2
    srv = M.Server(arena_bytes=1 << 30, max_active=2)
    rid = _submit(srv, q)
    r = _drain(srv, [rid])[rid]
    assert r["state"] == M.REQ_DONE
    og = O.Grid(q["origin"], q["dims"], q["voxel"], features=3, nb_count=32, nb_zvar=32)
    opose, omi = O.align_c2f(og, q["A"], q["B"], q["init"], q["half"], q["samples"], q["levels"],
                             q["shrink"], feature_slot=q["feature_slot"])
    assert np.array_equal(r["pose"], np.asarray(opose)), (r["pose"], opose)
    assert abs(r["mi"] - omi) <= 1e-6
    srv.close()


def test_admission_by_slots_and_budget(M):
    qs = _requests(5, seed=21)
    # two slots: never more than two requests in flight
    srv = M.Server(arena_bytes=4 << 30, max_active=2)
    ids = [_submit(srv, q) for q in qs]
    seen_active = 0
    for _ in range(100):
        na, nq = srv.step()
        seen_active = max(seen_active, na)
        if na == 0 and nq == 0:
            break
    assert seen_active <= 2
    res = {i: srv.poll(i) for i in ids}
    assert all(r["state"] == M.REQ_DONE for r in res.values())
    admits = [res[i]["t_admit"] for i in ids]
    assert admits == sorted(admits), "admission must follow arrival order"
    srv.close()
    # a budget that holds one 0.5 m request (~146 MB of reference features)
    # at a time: the second 0.5 m request waits until the first is done
    srv = M.Server(arena_bytes=(160 << 20) + (256 << 20), step_bytes=256 << 20, max_active=8)
    ids = [_submit(srv, q) for q in qs[:3]]
    res = _drain(srv, ids)
    for j, i in enumerate(ids):
        assert res[i]["state"] == M.REQ_DONE, (j, res[i])
        pose, best = _alone(M, qs[j])
        assert np.array_equal(res[i]["pose"], pose) and res[i]["mi"] == best
    assert qs[0]["voxel"] == qs[2]["voxel"] == 0.5
    assert res[ids[2]]["t_admit"] >= res[ids[0]]["t_done"]
    srv.close()


def test_oversized_request_is_rejected(M):
    q = _requests(1, seed=4)[0]
    srv = M.Server(arena_bytes=64 << 20, step_bytes=32 << 20, max_active=2)
    with pytest.raises(M.MIError) as e:
        _submit(srv, q)
    assert e.value.status == M.MI_E_UNSUPPORTED
    na, nq = srv.step()
    assert (na, nq) == (0, 0)
    srv.close()


def test_failing_and_degenerate_requests_leave_the_others_unchanged(M):
    # Failure isolation: in a mix of six, one request fails at its first level
    # (a grid 1000 voxels tall, more than a brick's voxel hash can hold: the
    # evaluator rejects it as unsupported), one has an all-NaN scan B (every
    # point skipped: MI = 0 at every pose) and one an empty scan A (empty
    # overlap everywhere).  The other three must finish bit-identical to their
    # runs alone, the degenerate ones must equal theirs alone too, and every
    # arena block must be back once the server is idle.
    qs = _requests(3, seed=31)
    nan_q = dict(qs[0])
    nan_q["B"] = np.full_like(qs[0]["B"], np.nan)
    empty_q = dict(qs[1])
    empty_q["A"] = np.zeros((3, 0), np.float32)
    tall = dict(qs[2])
    tall.update(origin=(-1.0, -1.0, -1.0), dims=(8, 8, 1000), voxel=0.25)
    srv = M.Server(arena_bytes=4 << 30, max_active=8)
    info0 = srv.info()
    assert info0["heap_free"] == info0["heap_bytes"]
    order = [qs[0], tall, nan_q, qs[1], empty_q, qs[2]]
    ids = [_submit(srv, q) for q in order[:3]]
    srv.step()
    ids += [_submit(srv, q) for q in order[3:]]
    res = _drain(srv, ids)
    for j, (q, rid) in enumerate(zip(order, ids)):
        r = res[rid]
        _say("request", j, "state", r["state"], "status", r["status"], "mi", r["mi"])
        if q is tall:
            assert r["state"] == M.REQ_FAILED and r["status"] == M.MI_E_UNSUPPORTED, r
            continue
        assert r["state"] == M.REQ_DONE and r["levels_done"] == 3, r
        pose, best = _alone(M, q)
        assert np.array_equal(r["pose"], pose), (j, r["pose"], pose)
        assert r["mi"] == best, (j, r["mi"], best)
        if q is nan_q or q is empty_q:
            assert r["mi"] == 0.0
    info = srv.info()
    assert info["heap_free"] == info["heap_bytes"], info
    for rid in ids:
        srv.release(rid)
    srv.close()
