"""The C ABI on the CPU: the library loads, exports every symbol that
include/mi.h declares, and its host-only calls (validation, pose matrix, bin
edges, error paths) behave.  No kernel is launched here."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1709_06948_amd import mi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "mi.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mi_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 20
    lib = C.CDLL(mi.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(mi.EXPORTED) <= set(names)


@pytest.mark.parametrize("seed", range(30))
def test_pose_matrix_bitwise_equals_oracle(seed):
    rng = np.random.default_rng(seed)
    eta = np.concatenate([rng.uniform(-10, 10, 3), rng.uniform(-math.pi, math.pi, 3)])
    rt = mi.pose_to_matrix(eta)
    assert np.array_equal(rt[:, :3], O.pose_matrix(eta))
    assert np.array_equal(rt[:, 3], eta[:3])


@pytest.mark.parametrize("vox", [0.25, 0.5, 1.0, 0.3])
@pytest.mark.parametrize("nb", [3, 16, 32, 64])
def test_default_edges_equal_oracle(vox, nb):
    g = mi.Grid((0, 0, 0), (4, 4, 4), vox, features=mi.FEAT_COUNT | mi.FEAT_ZVAR, nb_count=nb,
                nb_zvar=nb)
    og = O.Grid((0, 0, 0), (4, 4, 4), vox, features=O.FEAT_COUNT | O.FEAT_ZVAR, nb_count=nb,
                nb_zvar=nb)
    ce, ze = g.edges()
    assert np.array_equal(ce, og.count_edges) and np.array_equal(ze, og.zvar_edges)


@pytest.mark.parametrize("bad", [
    dict(dims=(0, 4, 4)), dict(dims=(65536, 65536, 2)), dict(voxel=0.0), dict(voxel=float("nan")),
    dict(features=0), dict(features=8), dict(features=7), dict(features=4, nb_count=10, nb_zvar=10),
    dict(features=4, nb_zvar=1), dict(nb_count=1), dict(nb_count=65),
    dict(features=2, nb_zvar=2), dict(features=2, voxel=0.005),
    dict(count_edges=[0, 1, 2]), dict(count_edges=[3, 2, 5]),
    dict(origin=(float("inf"), 0, 0)),
])
def test_grid_validation(bad):
    kw = dict(origin=(0, 0, 0), dims=(4, 4, 4), voxel=1.0, features=1, nb_count=4, nb_zvar=8)
    kw.update(bad)
    with pytest.raises(mi.MIError) as e:
        mi.Grid(**kw)
    assert e.value.status == mi.MI_E_INVALID


@pytest.mark.parametrize("features,nbc,nbz,slots", [
    (4, 8, 9, [(4, 57)]), (5, 8, 2, [(1, 8), (4, 8)]), (6, 2, 16, [(2, 16), (4, 16)]),
    (3, 16, 32, [(1, 16), (2, 32)])])
def test_joint_feature_slots(features, nbc, nbz, slots):
    """Slots follow count, z-variance, joint; the joint feature has
    1 + (nbc - 1)(nbz - 1) bins; both sides agree on the slots and edges."""
    g = mi.Grid((0, 0, 0), (4, 4, 4), 1.0, features=features, nb_count=nbc, nb_zvar=nbz)
    og = O.Grid((0, 0, 0), (4, 4, 4), 1.0, features=features, nb_count=nbc, nb_zvar=nbz)
    assert g.feature_list == slots == og.feature_list
    ce, ze = g.edges()
    assert np.array_equal(ce, og.count_edges[:nbc - 1])
    if nbz >= 3:
        assert np.array_equal(ze, og.zvar_edges[:nbz - 2])


def test_status_strings():
    for s in (0, -1, -2, -3, -4):
        assert mi.status_str(s)
    assert mi.status_str(7) == "unknown status"
