"""Host-side checks of the C ABI (no GPU): the shared library loads and
exports every entry point declared in include/octmg.h, the host tree
planner builds the same tree as the oracle (uniform and adaptive, 2:1
balance), and invalid descriptors are rejected with OCTMG_ERR_INVALID."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2205_09411_amd import octmg
from paper_2205_09411_amd import workloads as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "octmg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(octmg_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(octmg.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding covers the whole header
    assert sorted(octmg.exported_names()) == names


GEOMS = {
    "mms2d": lambda: W.mms2d().geom,
    "mms3d_16": lambda: W.mms3d(max_level=4).geom,
    "spheres_amr": lambda: W.spheres(n_spheres=6, max_level=5, block_n=8, seed=9).geom,
    "spheres_amr16": lambda: W.spheres(n_spheres=20, max_level=5, block_n=16).geom,
    "cylinder": lambda: W.cylinder(max_level=3).geom,
    # sharp shapes refined near the interface: the host refinement predicate
    # evaluates the shape (with its + - * / cube root) like the oracle
    "heart_amr2d": lambda: W.Geometry(dim=2, block_n=8, max_level=5, lsf_kind=W.LSF_HEART,
                                      lsf_params=np.array([0.5, 0.5, 0.5, 4.0, 0.0]), refine_kind=W.REFINE_NEAR_INTERFACE,
                                      refine_width=2.0 + np.sqrt(3) / 2, w_min=4e-3),
    "astroid_amr3d": lambda: W.Geometry(dim=3, block_n=8, max_level=4, lsf_kind=W.LSF_ASTROID,
                                        lsf_params=np.array([0.0, 0.0, 0.5, 4.0, 0.5]),
                                        refine_kind=W.REFINE_NEAR_INTERFACE, refine_width=2.0 + np.sqrt(3) / 2,
                                        w_min=8e-3),
}


@pytest.mark.parametrize("name", sorted(GEOMS))
def test_host_tree_matches_oracle(orc, name):
    geom = GEOMS[name]()
    plan = octmg.plan_levels(geom)
    o = orc.Oracle(geom)
    assert len(plan) == o.n_levels
    for il, p in enumerate(plan):
        info = o.level_info(il)
        assert (p["n"], p["Nb"], p["nblocks"], p["nleaf"]) == (info["n"], info["Nb"], info["nblocks"], info["nleaf"])
        pos, leaf = octmg.plan_blocks(geom, il)
        opos, oleaf = o.block_positions(il)
        assert np.array_equal(pos, opos) and np.array_equal(leaf, oleaf)


def test_adaptive_plan_is_adaptive():
    plan = octmg.plan_levels(GEOMS["spheres_amr16"]())
    leaf_levels = [i for i, p in enumerate(plan) if p["nleaf"] > 0]
    assert len(leaf_levels) >= 2


@pytest.mark.parametrize("field,value", [("dim", 4), ("block_n", 12), ("max_level", 0), ("coarse_n", 4),
                                         ("eps_tol", 0.0), ("lsf_kind", 9), ("lsf_kind", 8), ("neumann_faces", 64),
                                         ("uniform_level", 9)])
def test_invalid_descriptor_rejected(field, value):
    """lsf_kind 8 is OCTMG_LSF_CALLBACK, invalid without a function."""
    geom = W.mms3d(max_level=2).geom
    setattr(geom, field, value)
    with pytest.raises(octmg.OctmgError) as e:
        octmg.plan_levels(geom)
    assert e.value.status == octmg.ERR_INVALID


def test_callback_tree_matches_builtin(orc):
    """A level set given as a host function (OCTMG_LSF_CALLBACK) that
    restates a built-in union of spheres gives the same refined tree as the
    built-in kind and the oracle (the refinement test evaluates f at block
    centres on the host)."""
    import copy
    import math
    geom = GEOMS["spheres_amr16"]()
    P = [float(v) for v in geom.lsf_params]
    calls = [0]

    def f(x, y, z):
        calls[0] += 1
        best = 0.0
        for m in range(len(P) // 4):
            ex, ey, ez = x - P[4 * m], y - P[4 * m + 1], z - P[4 * m + 2]
            v = math.sqrt(ex * ex + ey * ey + ez * ez) - P[4 * m + 3]
            if m == 0 or v < best:
                best = v
        return best
    g = copy.copy(geom)
    g.lsf_kind, g.lsf_fn = octmg.LSF_CALLBACK, f
    plan_cb, plan = octmg.plan_levels(g), octmg.plan_levels(geom)
    assert calls[0] > 0 and plan_cb == plan
    for il in range(len(plan)):
        a, b = octmg.plan_blocks(g, il), octmg.plan_blocks(geom, il)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
