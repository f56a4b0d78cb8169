"""The mixed-precision defect that leaves the FP32 correction's red cells as
its first red half sweep from zero would (launch option red_preset, the
default) gives the same iterates bit for bit as zeroing the correction and
running that half sweep: uniform 3D trees with 16^3 and 8^3 blocks, an
interface through cell centres, zero-flux faces, several right-hand sides,
pre-smoothing counts 1 to 3, eager launches and graphs, V-cycles and solves;
where it does not apply (adaptive trees, FMG corrections) the two settings
run the same launches."""
import numpy as np
import pytest

from paper_2205_09411_amd import octmg
from paper_2205_09411_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    "mms3d_b16_64": lambda: W.mms3d(max_level=3, block_n=16),
    "mms3d_b8_32": lambda: W.mms3d(max_level=3, block_n=8),
    "cylinder_64": lambda: W.cylinder(max_level=3),
    "through_centres_64": lambda: W.through_centres(),
    "electrodes_uniform": lambda: W.two_electrodes(max_level=4, uniform_level=4),
    "spheres_amr16": lambda: W.spheres(n_spheres=8, max_level=5, block_n=16, seed=12),
}


def state(w, G, preset, n_rhs, n_down, n_up):
    S = octmg.State(G, n_rhs, octmg.MIXED)
    S.set_launch(red_preset=preset)
    S.set_smoothing(n_down, n_up)
    S.set_boundary_fn(w.iface_value, w.domain_value)
    xyz, _ = G.leaf_coords()
    g = w.rhs(xyz)
    S.set_rhs(np.stack([g * (1.0 + 0.5 * i) for i in range(n_rhs)]) if n_rhs > 1 else g)
    return S


@pytest.mark.parametrize("name", sorted(CASES))
def test_red_preset_bitwise(name):
    w = CASES[name]()
    print("red preset", name, flush=True)
    G = octmg.Geometry(w.geom)
    for n_down, n_up, n_rhs in ((2, 2, 1), (1, 2, 3), (3, 1, 1)):
        a = state(w, G, 1, n_rhs, n_down, n_up)
        b = state(w, G, 0, n_rhs, n_down, n_up)
        for k in range(2):
            a.vcycle()
            b.vcycle()
            assert np.array_equal(a.get_solution(), b.get_solution()), (n_down, n_up, k)
        a.fmg(have_guess=True)
        b.fmg(have_guess=True)
        assert np.array_equal(a.get_solution(), b.get_solution()), (n_down, n_up, "fmg")
        for gm in (0, 1, 2):
            ra = a.solve(rtol=1e-10, max_cycles=30, zero_start=True, graph_mode=gm, raise_on_fail=False)
            rb = b.solve(rtol=1e-10, max_cycles=30, zero_start=True, graph_mode=gm, raise_on_fail=False)
            assert ra.cycles == rb.cycles and ra.r_final == rb.r_final, (n_down, n_up, gm)
            assert np.array_equal(a.get_solution(), b.get_solution()), (n_down, n_up, "solve", gm)
