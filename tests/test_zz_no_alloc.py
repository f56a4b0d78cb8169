"""octmg_solve_noalloc (one FP64 solve whose fields live in the library's
fixed device array, no allocation) against octmg_solve on a state: two
calls in a row, the second on a smaller geometry, each with the same
solution bit for bit, the same cycles and residuals; and a geometry too
large for the array is refused."""
import numpy as np
import pytest
import torch

from paper_2205_09411_amd import octmg
from paper_2205_09411_amd import workloads as W

pytestmark = pytest.mark.gpu


def with_state(w, G, g, iv, dv):
    S = octmg.State(G)
    S.set_boundary(iv, dv)
    S.set_rhs(g)
    rep = S.solve(rtol=1e-10, max_cycles=40, zero_start=True)
    return rep, S.get_solution()


def test_noalloc_equals_solve_two_calls():
    cases = [("spheres_amr (adaptive, 8^3 blocks)", W.spheres(n_spheres=5, max_level=5, block_n=8, seed=9)),
             ("mms3d 64^3 (16^3 blocks)", W.mms3d(max_level=3, block_n=16))]
    sizes = []
    for name, w in cases:
        print("noalloc solve:", name, flush=True)
        G = octmg.Geometry(w.geom)
        sizes.append(G.n_leaf)
        xyz, _ = G.leaf_coords()
        g = w.rhs(xyz)
        iv = w.iface_value(G.iface_points())
        dv = w.domain_value(G.domain_points())
        ref_rep, ref = with_state(w, G, g, iv, dv)
        dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
        phi = torch.full((G.n_leaf,), float("nan"), dtype=torch.float64, device="cuda")
        rep = G.solve_noalloc(dev(g), phi, dev(iv), dev(dv), rtol=1e-10, max_cycles=40)
        got = phi.cpu().numpy()
        assert rep.status == 0 and rep.cycles == ref_rep.cycles, (rep.cycles, ref_rep.cycles)
        assert rep.r0 == ref_rep.r0 and rep.r_final == ref_rep.r_final
        assert rep.per_rhs["status"][0] == 0 and rep.per_rhs["cycles"][0] == ref_rep.cycles
        assert np.array_equal(got, ref), np.abs(got - ref).max()
    assert sizes[1] < sizes[0]


def test_noalloc_refuses_too_large_geometry():
    w = W.mms3d(max_level=5)  # 256^3: about 460 MB of fields
    G = octmg.Geometry(w.geom)
    t = torch.zeros(G.n_leaf, dtype=torch.float64, device="cuda")
    with pytest.raises(octmg.OctmgError) as e:
        G.solve_noalloc(t, t.clone())
    assert e.value.status == octmg.ERR_INVALID and "too large" in str(e.value)
