"""The V-cycle's prolongation fused with the red half sweep after it
(launch option prolong_fused, the default) gives the same iterates bit for
bit as the two separate launches: uniform and adaptive trees (refinement
faces), 8^3 and 16^3 blocks, zero-flux faces, FP64 and mixed precision,
one and two post-smoothing steps, and several right-hand sides."""
import numpy as np
import pytest

from paper_2205_09411_amd import octmg
from paper_2205_09411_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    "mms3d_b16_64": lambda: W.mms3d(max_level=3, block_n=16),
    "mms3d_b8_32": lambda: W.mms3d(max_level=3, block_n=8),
    "cylinder_64": lambda: W.cylinder(max_level=3),
    "spheres_amr": lambda: W.spheres(n_spheres=5, max_level=5, block_n=8, seed=9),
    "spheres_amr16": lambda: W.spheres(n_spheres=8, max_level=5, block_n=16, seed=12),
    "electrodes_small": lambda: W.two_electrodes(max_level=5, uniform_level=3),
}


def state(w, G, fused, precision, n_rhs, n_up):
    S = octmg.State(G, n_rhs, precision)
    S.set_launch(prolong_fused=fused)
    S.set_smoothing(2, n_up)
    S.set_boundary_fn(w.iface_value, w.domain_value)
    xyz, _ = G.leaf_coords()
    g = w.rhs(xyz)
    S.set_rhs(np.stack([g * (1.0 + 0.5 * i) for i in range(n_rhs)]) if n_rhs > 1 else g)
    return S


@pytest.mark.parametrize("precision", [octmg.FP64, octmg.MIXED])
@pytest.mark.parametrize("name", sorted(CASES))
def test_fused_prolongation_bitwise(name, precision):
    w = CASES[name]()
    print("fused prolongation", name, precision, flush=True)
    G = octmg.Geometry(w.geom)
    for n_up, n_rhs in ((2, 1), (1, 2)):
        a = state(w, G, 1, precision, n_rhs, n_up)
        b = state(w, G, 0, precision, n_rhs, n_up)
        a.fmg(have_guess=False)
        b.fmg(have_guess=False)
        assert np.array_equal(a.get_solution(), b.get_solution()), (n_up, "fmg")
        for k in range(3):
            a.vcycle()
            b.vcycle()
            assert np.array_equal(a.get_solution(), b.get_solution()), (n_up, k)
        ra = a.solve(rtol=1e-10, max_cycles=40, zero_start=True)
        rb = b.solve(rtol=1e-10, max_cycles=40, zero_start=True)
        assert ra.cycles == rb.cycles and ra.r_final == rb.r_final
        assert np.array_equal(a.get_solution(), b.get_solution()), (n_up, "solve")
