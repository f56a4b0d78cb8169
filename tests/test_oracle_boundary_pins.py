"""Pins of the oracle's domain-face handling in the transfers and of the
two-electrode level set, against closed forms.

Cell-centred tensor-product linear interpolation (Sec. 2.2 and Sec. 3.4:
standard (bi/tri)linear prolongation) reproduces every multilinear function
(a product of functions that are each linear in one coordinate) exactly.  A
coarse correction that vanishes on a Dirichlet face is odd across that face,
so the reflected ghost -e is its exact continuation; a correction that does
not depend on the normal coordinate of a zero-flux face is even across it,
so the mirrored ghost e is.  Prolongating such a correction must therefore
reproduce it exactly in the fine cells next to those faces -- with the sign
of the reflection wrong (or the face kind ignored) these cells are off by a
quarter of the ghost's error.

The rod-plus-sphere level set of the application (Sec. 4.3) is checked at
points built with known distances to the segment and to the sphere: beside
the segment (perpendicular offset), beyond both of its ends, and near the
half sphere.
"""
import numpy as np
import pytest

from paper_2205_09411_amd import workloads as W


def _centres(o, il, dim):
    """Global cell centres of every cell of level il, in the oracle's level
    order (block-major, x fastest within a block)."""
    info = o.level_info(il)
    nb_cells = info["Nb"]
    pos, _ = o.block_positions(il)
    loc = np.arange(nb_cells ** dim)
    h = 1.0 / info["n"]
    ix = (pos[:, None, 0] * nb_cells + loc[None, :] % nb_cells).reshape(-1)
    iy = (pos[:, None, 1] * nb_cells + (loc[None, :] // nb_cells) % nb_cells).reshape(-1)
    if dim == 3:
        iz = (pos[:, None, 2] * nb_cells + loc[None, :] // nb_cells ** 2).reshape(-1)
    else:
        iz = np.zeros_like(ix)
    idx = np.stack([ix, iy, iz], axis=1)
    x = (idx + 0.5) * h
    if dim == 2:
        x[:, 2] = 0.0
    return idx, x, info["n"]


def _prolong_correction(orc, geom, fn):
    """Put e = fn(coarse centres) as the correction phi_c - old_c on the
    level below the top, prolongate onto a zero top level, and return the
    fine values, the wanted fn(fine centres) and the fine cell indices."""
    o = orc.Oracle(geom)
    o.set_boundary(np.zeros(0), np.zeros(len(o.domain_points())))
    top = o.n_levels - 1
    _, xc, _ = _centres(o, top - 1, geom.dim)
    e = fn(xc)
    o.set_field(top - 1, o.FIELD_OLD, np.zeros_like(e))
    o.set_field(top - 1, o.FIELD_PHI, e)
    idx, xf, n = _centres(o, top, geom.dim)
    o.set_field(top, o.FIELD_PHI, np.zeros(len(xf)))
    o.prolong(top)
    return o.get_field(top, o.FIELD_PHI), fn(xf), idx, n


def _touches(idx, n, dim, lower, upper):
    """Cells whose face lies on a lower (index 0) or upper (n-1) domain face
    of the given axes."""
    m = np.zeros(len(idx), dtype=bool)
    for a in range(dim):
        if a in lower:
            m |= idx[:, a] == 0
        if a in upper:
            m |= idx[:, a] == n - 1
    return m


def _geom(dim, neumann=0):
    return W.Geometry(dim=dim, block_n=8, max_level=3, lsf_kind=W.LSF_NONE, lsf_params=np.zeros(0),
                      neumann_faces=neumann)


@pytest.mark.parametrize("dim", [2, 3])
def test_prolong_odd_reflection_at_dirichlet_faces(orc, dim):
    """A correction vanishing on the lower faces (e = x y [z]) and one
    vanishing on the upper faces (e = (1-x)(1-y)[(1-z)]) are prolongated
    exactly, also in the fine cells next to those faces, edges and corners
    (ghost -e across each outside axis)."""
    ax = range(dim)
    low = lambda x: np.prod([x[:, a] for a in ax], axis=0)
    high = lambda x: np.prod([1.0 - x[:, a] for a in ax], axis=0)
    for fn, exact_side in ((low, "lower"), (high, "upper")):
        got, want, idx, n = _prolong_correction(orc, _geom(dim), fn)
        other = _touches(idx, n, dim, lower=set() if exact_side == "lower" else set(ax),
                         upper=set(ax) if exact_side == "lower" else set())
        near = _touches(idx, n, dim, lower=set(ax) if exact_side == "lower" else set(),
                        upper=set(ax) if exact_side == "upper" else set()) & ~other
        assert near.sum() > 0
        err = np.abs(got - want)
        assert err[~other].max() < 1e-14, (exact_side, err[near].max())
        # the cells at the faces where e does not vanish are not exact: the
        # check above is not vacuous about which faces it covers
        assert err[other].max() > 1e-4


@pytest.mark.parametrize("dim", [2, 3])
def test_prolong_mirror_at_zero_flux_faces(orc, dim):
    """x faces zero-flux (ghost = inside value), the others Dirichlet: a
    correction that does not depend on x and vanishes on the lower (upper)
    Dirichlet faces is prolongated exactly, including the cells next to the
    zero-flux faces and the edges where the two kinds meet."""
    t = range(1, dim)
    low = lambda x: (1.0 + 0.0 * x[:, 0]) * np.prod([x[:, a] for a in t], axis=0)
    high = lambda x: (1.0 + 0.0 * x[:, 0]) * np.prod([1.0 - x[:, a] for a in t], axis=0)
    for fn, side in ((low, "lower"), (high, "upper")):
        got, want, idx, n = _prolong_correction(orc, _geom(dim, neumann=0b11), fn)
        other = _touches(idx, n, dim, lower=set(t) if side == "upper" else set(),
                         upper=set(t) if side == "lower" else set())
        xface = _touches(idx, n, dim, lower={0}, upper={0}) & ~other
        assert xface.sum() > 0
        err = np.abs(got - want)
        assert err[~other].max() < 1e-14, (side, err[xface].max())


def _multilinear(dim):
    if dim == 2:
        return lambda x: 0.3 + 0.5 * x[:, 0] - 0.2 * x[:, 1] + 1.1 * x[:, 0] * x[:, 1]
    return lambda x: (0.3 + 0.5 * x[:, 0] - 0.2 * x[:, 1] + 0.7 * x[:, 2] + 1.1 * x[:, 0] * x[:, 1]
                      - 0.6 * x[:, 1] * x[:, 2] + 0.4 * x[:, 0] * x[:, 2] + 0.9 * x[:, 0] * x[:, 1] * x[:, 2])


@pytest.mark.parametrize("dim", [2, 3])
def test_prolong_solution_mode_dirichlet_ghosts(orc, dim):
    """First interpolation of a nested iteration (coarse solution, not a
    correction): with Dirichlet ghosts 2 phi_b - phi_in on faces and linear
    extrapolation at edges and corners, a multilinear phi whose face values
    are given is reproduced exactly in every fine cell."""
    m = _multilinear(dim)
    o = orc.Oracle(_geom(dim))
    o.set_boundary(np.zeros(0), m(o.domain_points()))
    top = o.n_levels - 1
    _, xc, _ = _centres(o, top - 1, dim)
    o.set_field(top - 1, o.FIELD_PHI, m(xc))
    _, xf, _ = _centres(o, top, dim)
    o.set_field(top, o.FIELD_PHI, np.zeros(len(xf)))
    o.prolong(top, solution_mode=True)
    assert np.abs(o.get_field(top, o.FIELD_PHI) - m(xf)).max() < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_prolong_solution_mode_zero_flux_mirror(orc, dim):
    """Same with zero-flux x faces: a phi independent of x (multilinear in
    the other axes, Dirichlet values given on their faces) is reproduced
    exactly; the x ghosts are the mirror cells."""
    m0 = _multilinear(dim)
    m = lambda x: m0(np.concatenate([np.full((len(x), 1), 0.25), x[:, 1:]], axis=1))
    o = orc.Oracle(_geom(dim, neumann=0b11))
    o.set_boundary(np.zeros(0), m(o.domain_points()))
    top = o.n_levels - 1
    _, xc, _ = _centres(o, top - 1, dim)
    o.set_field(top - 1, o.FIELD_PHI, m(xc))
    _, xf, _ = _centres(o, top, dim)
    o.set_field(top, o.FIELD_PHI, np.zeros(len(xf)))
    o.prolong(top, solution_mode=True)
    assert np.abs(o.get_field(top, o.FIELD_PHI) - m(xf)).max() < 1e-13


# ----------------------------------------------------- two-electrode level set
def _perp_basis(u):
    """Two unit vectors orthogonal to the unit vector u and to each other."""
    t = np.array([1.0, 0.0, 0.0]) if abs(u[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    v = np.cross(u, t)
    v /= np.linalg.norm(v)
    return v, np.cross(u, v)


@pytest.mark.parametrize("tilt", [False, True])
def test_electrode_lsf_closed_form(orc, tilt):
    """f = min(distance to the segment - r_rod, distance to the sphere
    centre - r_sph).  Points are built with known distances: a point at
    axial parameter t in [0, 1] and perpendicular offset rho is rho from the
    segment; a point beyond an end, in the half space past that end, is its
    distance from that end point.  A tilted segment checks that no axis is
    assumed."""
    a = np.array([0.5, 0.5, 0.6])
    b = np.array([0.5, 0.5, 1.1]) if not tilt else np.array([0.62, 0.41, 1.05])
    r_rod, c, r_sph = 0.05, np.array([0.5, 0.5, 0.0]), 0.25
    geom = W.Geometry(dim=3, block_n=8, max_level=1, lsf_kind=W.LSF_ELECTRODES,
                      lsf_params=np.array([*a, *b, r_rod, *c, r_sph]))
    L = np.linalg.norm(b - a)
    u = (b - a) / L
    v, w = _perp_basis(u)
    rng = np.random.default_rng(7)
    pts, dist = [], []
    for _ in range(300):  # beside the segment
        t, rho, ang = rng.uniform(0, 1), rng.uniform(0, 0.3), rng.uniform(0, 2 * np.pi)
        pts.append(a + t * L * u + rho * (np.cos(ang) * v + np.sin(ang) * w))
        dist.append(rho)
    for end, sgn in ((b, 1.0), (a, -1.0)):  # beyond each end: a direction into that end's half space
        for _ in range(300):
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            if sgn * (d @ u) < 0:
                d = d - 2 * (d @ u) * u
            rho = rng.uniform(0, 0.3)
            pts.append(end + rho * d)
            dist.append(rho)
    pts, dist = np.array(pts), np.array(dist)
    sph = np.linalg.norm(pts - c, axis=1) - r_sph
    want = np.minimum(dist - r_rod, sph)
    got = np.array([orc.lsf_value(geom, p) for p in pts])
    assert np.abs(got - want).max() < 1e-14
    # near the half sphere, far from the rod, f is the sphere's distance
    q = []
    for _ in range(300):
        d = rng.normal(size=3)
        d[2] = abs(d[2])
        d /= np.linalg.norm(d)
        q.append(c + (r_sph + rng.uniform(-0.05, 0.05)) * d)
    q = np.array(q)
    got = np.array([orc.lsf_value(geom, p) for p in q])
    assert np.abs(got - (np.linalg.norm(q - c, axis=1) - r_sph)).max() < 1e-14
