"""Degenerate inputs of the oracle, against closed forms.

* An interface through cell centres (f = 0 exactly at a centre, Sec. 3.2):
  every link of such a cell brackets a root at t = 0, and bisection of the
  bracket [0, 1] halves towards 0 on each of its steps (the product
  f(a) f(x) is 0, never positive), so d is the smallest value the search can
  return, 2^-28 with 27 halvings for eps_tol = 1e-8, never 0.  All links of
  the cell are then cut, the row is c_ii phi_i = g_i - b_i with
  b_i = -c_ii phi_b, and because |g_i / c_ii| is far below the rounding unit
  the smoothed value is the boundary value exactly.
* No interface at all: no stencil record on any level, and the method is the
  textbook cell-centred FAS multigrid, exact on a linear solution.
"""
import numpy as np

from paper_2205_09411_amd import workloads as W


def test_interface_through_cell_centres(orc):
    w = W.through_centres()
    o = orc.setup_workload(w)
    xyz, _ = o.leaf_coords()
    on = (np.sqrt((xyz[:, 0] - 0.5) ** 2 + (xyz[:, 1] - 0.5) ** 2) - w.extra["radius"]) == 0
    assert on.sum() == 8 * 64  # eight mirror cells in each of the 64 z layers
    _, d, _ = o.records(o.n_levels - 1)
    assert d.min() == 2.0 ** -28
    # six links per such cell, less the 16 z links that leave the cube
    assert (d == 2.0 ** -28).sum() == 6 * on.sum() - 16
    assert (d[d != 2.0 ** -28] > 1e-3).all()  # no other link comes close
    o.zero_solution()
    o.vcycle()
    assert np.all(o.get_solution()[on] == 1.0)
    o.fmg(have_guess=True)
    assert np.all(o.get_solution()[on] == 1.0)


def test_no_interface(orc):
    w = W.no_interface()
    o = orc.setup_workload(w)
    assert all(o.level_info(il)["nrec"] == 0 for il in range(o.n_levels))
    assert len(o.iface_points()) == 0
    # a linear function is reproduced exactly (domain ghosts, transfers and
    # the standard stencil are exact on it)
    xyz, _ = o.leaf_coords()
    lin = lambda x: 0.3 + 1.5 * x[:, 0] - 0.7 * x[:, 1] + 0.2 * x[:, 2]
    o.set_boundary(np.zeros(0), lin(o.domain_points()))
    o.set_rhs(np.zeros(len(xyz)))
    o.zero_solution()
    for _ in range(30):
        o.vcycle()
    assert np.abs(o.get_solution() - lin(xyz)).max() < 1e-12
