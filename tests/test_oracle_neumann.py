"""Pins of the oracle's zero-flux (Neumann) domain faces, as used by the
two-electrode application of Sec. 4.3: the textbook cell-centred Laplacian
with mirror ghosts assembled with scipy, exactness for a solution that is
linear along the Dirichlet axis, a harmonic closed form with zero normal
derivative (second-order convergence), and the dense direct solve of the
assembled operator; then the application's field by face differences (exact
for linear phi, inside cells zeroed) and its FMG reduction."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from paper_2205_09411_amd import workloads as W

X_FACES, Y_FACES = 0b0011, 0b1100


def _converge(o, n):
    for _ in range(n):
        o.vcycle()


def test_textbook_laplacian_neumann_sides(orc):
    """No interface, zero flux on the x faces, Dirichlet on the y faces: the
    method reduces to the 5-point Laplacian whose x second difference has
    -1 (mirror ghost) instead of -3 (Dirichlet ghost) in its end rows."""
    geom = W.Geometry(dim=2, block_n=8, max_level=3, lsf_kind=W.LSF_NONE, lsf_params=np.zeros(0),
                      neumann_faces=X_FACES)
    o = orc.Oracle(geom)
    n, h = 32, 1.0 / 32
    bfun = lambda x: np.sin(3 * x[:, 0]) + np.cos(2 * x[:, 1])
    o.set_boundary(np.zeros(0), bfun(o.domain_points()))
    xyz, _ = o.leaf_coords()
    g = np.random.default_rng(6).standard_normal(len(xyz))
    o.set_rhs(g)
    _converge(o, 40)
    phi = o.get_solution()

    def second_difference(end):
        T = sp.diags([np.ones(n - 1), -2 * np.ones(n), np.ones(n - 1)], [-1, 0, 1]).tolil()
        T[0, 0] = T[n - 1, n - 1] = end
        return T.tocsr() / h ** 2

    Tx, Ty, I = second_difference(-1.0), second_difference(-3.0), sp.identity(n)
    A = sp.kron(I, Tx) + sp.kron(Ty, I)  # x fastest
    cc = (np.arange(n) + 0.5) * h
    idx = np.floor(xyz[:, 1] / h).astype(int) * n + np.floor(xyz[:, 0] / h).astype(int)
    rhs = np.zeros(n * n)
    rhs[idx] = g
    b = np.zeros((n, n))
    b[0, :] += 2 * bfun(np.stack([cc, np.zeros(n), 0 * cc], 1)) / h ** 2
    b[-1, :] += 2 * bfun(np.stack([cc, np.ones(n), 0 * cc], 1)) / h ** 2
    ref = spla.spsolve(A.tocsc(), rhs - b.reshape(-1))
    assert np.abs(phi - ref[idx]).max() < 1e-11 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("case", ["uniform3d", "adaptive3d", "adaptive2d"])
def test_linear_along_dirichlet_axis_exact(orc, case):
    """phi = 1 - 2z (2D: 1 - 2y) has zero flux through the side faces: with
    mirror ghosts on the sides, Dirichlet data at the remaining faces and on
    an interface, the fixed point is phi itself, including refinement
    boundaries that meet the zero-flux faces."""
    if case == "adaptive2d":
        geom = W.Geometry(dim=2, block_n=8, max_level=5, lsf_kind=W.LSF_SPHERES,
                          lsf_params=np.array([0.2, 0.5, 0, 0.08]), refine_kind=W.REFINE_NEAR_INTERFACE,
                          refine_width=1.0, w_min=4e-3, neumann_faces=X_FACES)
        lin = lambda x: 1.0 - 2.0 * x[:, 1]
    else:
        geom = W.Geometry(dim=3, block_n=8, max_level=3 if case == "uniform3d" else 4,
                          lsf_kind=W.LSF_SPHERES, lsf_params=np.array([0.15, 0.5, 0.5, 0.1]),
                          refine_kind=W.REFINE_NEAR_INTERFACE if case == "adaptive3d" else W.REFINE_UNIFORM,
                          refine_width=1.0, w_min=8e-3, neumann_faces=X_FACES | Y_FACES)
        lin = lambda x: 1.0 - 2.0 * x[:, 2]
    o = orc.Oracle(geom)
    if case != "uniform3d":
        assert o.adaptive
    o.set_boundary_fn(lin, lin)
    xyz, _ = o.leaf_coords()
    o.set_rhs(np.zeros(len(xyz)))
    _converge(o, 40)
    assert np.abs(o.get_solution() - lin(xyz)).max() < 1e-12


def _harmonic_neumann_errors(level):
    """phi = cos(pi x) exp(pi y) is harmonic with d phi/dx = 0 at x = 0, 1:
    zero flux on the x faces, Dirichlet phi on the y faces and a circle."""
    import oracle
    phi = lambda x: np.cos(math.pi * x[:, 0]) * np.exp(math.pi * x[:, 1])
    geom = W.Geometry(dim=2, block_n=8, max_level=level, lsf_kind=W.LSF_SPHERES,
                      lsf_params=np.array([0.55, 0.45, 0, 0.2]), w_min=4e-3, neumann_faces=X_FACES)
    o = oracle.Oracle(geom)
    o.set_boundary_fn(phi, phi)
    xyz, _ = o.leaf_coords()
    o.set_rhs(np.zeros(len(xyz)))
    o.solve(rtol=1e-11, max_cycles=40)
    e = o.get_solution() - phi(xyz)
    return np.abs(e).max(), math.sqrt((e ** 2).mean())


def test_second_order_with_zero_flux_faces(orc):
    errs = [_harmonic_neumann_errors(L) for L in (4, 5, 6)]
    for (a, b), (c, d) in zip(errs[:-1], errs[1:]):
        assert math.log2(a / c) > 1.8 and math.log2(b / d) > 1.8, errs


def test_dense_direct_solve_neumann(orc):
    """Multigrid fixed point = direct solve of the composite operator
    assembled by probing the residual, with zero-flux x faces."""
    geom = W.Geometry(dim=2, block_n=8, max_level=4, lsf_kind=W.LSF_SPHERES,
                      lsf_params=np.array([0.3, 0.6, 0, 0.09]), refine_kind=W.REFINE_NEAR_INTERFACE,
                      refine_width=0.5, w_min=4e-3, neumann_faces=X_FACES)
    o = orc.Oracle(geom)
    assert o.adaptive
    f = lambda x: np.sin(2 * x[:, 0]) + x[:, 1]
    o.set_boundary_fn(f, f)
    xyz, _ = o.leaf_coords()
    o.set_rhs(np.cos(3 * xyz[:, 0]) * xyz[:, 1])
    n = o.n_leaf
    r0 = o.leaf_residual(np.zeros(n))
    A = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, j] = r0 - o.leaf_residual(e)
    ref = np.linalg.solve(A, r0)
    o.zero_solution()
    _converge(o, 40)
    assert np.abs(o.get_solution() - ref).max() <= 1e-11 * np.abs(ref).max()


# ------------------------------------------------ two electrodes (Sec. 4.3)
def test_gradient_exact_for_linear_phi(orc):
    """For linear phi every face difference is exact: neighbour values and
    domain/refinement ghosts, and at cut links (phi_b - phi_i)/(d dx)
    with phi_b = phi(x0).  The cell gradient is the constant gradient."""
    grad = np.array([2.0, -3.0, 0.5])
    lin = lambda x: 1.0 + x[:, :3] @ grad
    geom = W.Geometry(dim=3, block_n=8, max_level=4, lsf_kind=W.LSF_SPHERES,
                      lsf_params=np.array([0.45, 0.55, 0.5, 0.2]), refine_kind=W.REFINE_NEAR_INTERFACE,
                      refine_width=1.0, w_min=8e-3)
    o = orc.Oracle(geom)
    assert o.adaptive
    o.set_boundary_fn(lin, lin)
    xyz, _ = o.leaf_coords()
    o.set_rhs(np.zeros(len(xyz)))
    _converge(o, 40)
    err = np.abs(o.gradient() - grad).max(axis=1)
    assert np.median(err) < 1e-10 and err.max() < 1e-6, (np.median(err), err.max())


def test_gradient_zero_flux_and_inside_cells(orc):
    """phi = 1 - 2z with zero flux on the sides: gradient (0, 0, -2) in every
    cell; with inside_zero the cut cells whose centre lies inside the
    interface report 0."""
    lin = lambda x: 1.0 - 2.0 * x[:, 2]
    geom = W.Geometry(dim=3, block_n=8, max_level=3, lsf_kind=W.LSF_SPHERES,
                      lsf_params=np.array([0.5, 0.5, 0.4, 0.18]), w_min=8e-3, neumann_faces=X_FACES | Y_FACES)
    o = orc.Oracle(geom)
    o.set_boundary_fn(lin, lin)
    xyz, _ = o.leaf_coords()
    o.set_rhs(np.zeros(len(xyz)))
    _converge(o, 40)
    g = o.gradient()
    err = np.abs(g - np.array([0.0, 0.0, -2.0])).max(axis=1)
    assert np.median(err) < 1e-10 and err.max() < 1e-6
    gz = o.gradient(inside_zero=True)
    r = np.linalg.norm(xyz - np.array([0.5, 0.5, 0.4]), axis=1)
    zeroed = np.all(gz == 0.0, axis=1)
    assert zeroed.any() and np.all(r[zeroed] < 0.18)  # only inside cells are zeroed
    assert np.array_equal(gz[~zeroed], g[~zeroed])
    # cut cells just outside keep their gradient
    assert np.all(~zeroed[(r > 0.18) & (r < 0.18 + 1.0 / 32)])


def test_two_electrode_fmg_reduction(orc):
    """Sec. 4.3: the residual drops by about 30-40 per FMG iteration on the
    paper's mesh; on a coarser mesh of the same problem (uniform 32^3,
    refined to 128^3 near the electrodes) the oracle's reduction is at least
    20 per iteration after the first."""
    w = W.two_electrodes(max_level=5, uniform_level=3)
    o = orc.setup_workload(w)
    assert o.adaptive
    xyz, _ = o.leaf_coords()
    r = [o.residual_max(phi_zero=True)]
    for k in range(4):
        o.fmg(have_guess=k > 0)
        r.append(o.residual_max())
    factors = [r[i] / r[i + 1] for i in range(1, 4)]
    assert min(factors) > 20, factors
    phi = o.get_solution()
    # electrode potentials: the rod at 1, the half sphere at 0, in between
    assert -0.01 < phi.min() and phi.max() < 1.01
