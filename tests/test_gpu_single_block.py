"""The one-block 16^3 level (the level above the 8^3 coarsest grid) runs its
steps of a cycle in one workgroup per right-hand side, both colours resident
in LDS.  Its iterates must equal, bit for bit, those of the separate
launches (pair_max_blocks = 0 selects them): Dirichlet faces with face data
(FP64) and without (the FP32 correction equation), zero-flux faces,
smoothing counts other than (2, 2), V-cycles and FMG, several rhs; and,
with such counts, parity with the oracle."""
import numpy as np
import pytest

from paper_2205_09411_amd import octmg
from paper_2205_09411_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    # 64^3 in 16^3 blocks: levels 8^3, 16^3 (one block), 32^3, 64^3
    "mms3d_b16_64": lambda: W.mms3d(max_level=3, block_n=16),
    # zero flux on the four side faces, Dirichlet top and bottom, adaptive
    "electrodes_b16": lambda: W.two_electrodes(max_level=4, uniform_level=3, block_n=16),
}


def make_state(G, w, n_rhs, precision, pair_max):
    S = octmg.State(G, n_rhs, precision)
    S.set_launch(pair_max_blocks=pair_max)
    S.set_boundary_fn(w.iface_value, w.domain_value)
    xyz, _ = G.leaf_coords()
    g = w.rhs(xyz)
    S.set_rhs(np.stack([g * (1.0 + 0.5 * r) for r in range(n_rhs)]) if n_rhs > 1 else g)
    return S


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", [octmg.FP64, octmg.MIXED])
def test_single_block_equals_separate_launches(name, precision):
    print("single block", name, precision, flush=True)
    w = CASES[name]()
    G = octmg.Geometry(w.geom)
    info = G.level_info(1)
    assert info["nblocks"] == 1 and info["Nb"] == 16 and G.n_levels > 2
    n_rhs = 3 if precision == octmg.MIXED else 1
    for n_down, n_up in ((2, 2), (1, 3), (3, 0), (0, 1)):
        states = [make_state(G, w, n_rhs, precision, p) for p in (1 << 30, 0)]
        for S in states:
            S.set_smoothing(n_down, n_up)
        for k in range(2):
            for S in states:
                S.vcycle()
            a, b = (S.get_solution() for S in states)
            assert np.array_equal(a, b), (n_down, n_up, k)
        for S in states:
            S.fmg(have_guess=True)
        assert np.array_equal(states[0].get_solution(), states[1].get_solution()), (n_down, n_up, "fmg")
        for S in states:
            S.zero_solution()
            S.fmg(have_guess=False)
        assert np.array_equal(states[0].get_solution(), states[1].get_solution()), (n_down, n_up, "fmg0")
        if precision == octmg.FP64:
            na, nb = (S.residual_norm() for S in states)
            assert np.array_equal(na, nb)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("counts", [(1, 3), (3, 1)])
def test_single_block_oracle_parity(orc, name, counts):
    """With smoothing counts other than (2, 2), the path with the one-block
    kernel matches the oracle after every V-cycle and FMG (1e-10)."""
    n_down, n_up = counts
    print("single block oracle parity", name, counts, flush=True)
    w = CASES[name]()
    o = orc.setup_workload(w, n_down, n_up)
    G = octmg.Geometry(w.geom)
    S = octmg.State(G)
    S.set_smoothing(n_down, n_up)
    xo, _ = o.leaf_coords()
    S.set_boundary(w.iface_value(o.iface_points()) if G.n_iface else None, w.domain_value(o.domain_points()))
    S.set_rhs(w.rhs(xo))
    S.fmg(have_guess=False)
    o.fmg(have_guess=False)
    assert rel(S.get_solution(), o.get_solution()) < 1e-10
    for k in range(3):
        S.vcycle()
        o.vcycle()
        assert rel(S.get_solution(), o.get_solution()) < 1e-10, k
