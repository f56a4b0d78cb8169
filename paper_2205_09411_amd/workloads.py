"""Seeded synthetic workloads: geometry descriptions, right-hand sides and
boundary data for the multigrid solver and for its FP64 CPU oracle.

This module holds inputs only.  It contains none of the solver's arithmetic
(no stencils, no line search, no transfers): it turns seeds and closed-form
fields into the arrays both sides are fed.  Every generator is deterministic
(NumPy PCG64 ``default_rng``).

Workload shapes follow the paper's test problems (Sec. 4) and the scaled
workloads of this package:

* ``mms2d``   2D unit square, circle r=0.25 at (0.5,0.5), manufactured
              phi = sin(2 pi x) cos(3 pi y) + x^2, 8x8-cell blocks.
* ``mms3d``   3D unit cube, sphere r=0.3 at the centre, manufactured
              phi = exp(x) sin(pi y) cos(pi z), 16^3-cell blocks.
* ``spheres`` 3D union of seeded spheres (centres U[0.2,0.8]^3, radii
              U[0.03,0.1]), phi=1 on the spheres, 0 on the cube, g ~ N(0,1).
* ``cylinder``3D cylinder r=0.2 along z through (0.5,0.5), phi=0 on it and on
              the cube; right-hand sides are sums of seeded Gaussian sources.
* ``sphere_f1`` the convergence test of Sec. 4.1: domain of unit size centred
              at the origin, sphere of radius R, exact solutions of
              eq. (solution-sphere) imposed on the domain boundary.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# level-set kinds understood by both the library and the oracle
LSF_NONE = 0
LSF_SPHERES = 1      # union of spheres/circles: params [cx, cy, cz, r] * n
LSF_CYLINDER_Z = 2   # infinite cylinder along z: params [cx, cy, r]
# the sharp shapes of Sec. 4.2, params [cx, cy, cz, s, r0]: 2D p = s(x-cx),
# q = s(y-cy); 3D p = s(|(x-cx, y-cy)| - r0), q = s(z-cz)
LSF_SPHEROID, LSF_RHOMBUS, LSF_HEART, LSF_ASTROID = 3, 4, 5, 6
SHAPES = {"spheroid": LSF_SPHEROID, "rhombus": LSF_RHOMBUS, "heart": LSF_HEART, "astroid": LSF_ASTROID}
# two electrodes: rod around segment a-b plus a sphere, params
# [ax, ay, az, bx, by, bz, r_rod, cx, cy, cz, r_sphere]
LSF_ELECTRODES = 7

REFINE_UNIFORM = 0
REFINE_NEAR_INTERFACE = 1


@dataclass
class Geometry:
    """Plain description of a block octree and its level set."""
    dim: int
    block_n: int
    max_level: int
    lsf_kind: int
    lsf_params: np.ndarray
    lo: tuple = (0.0, 0.0, 0.0)
    refine_kind: int = REFINE_UNIFORM
    refine_width: float = 0.0
    eps_tol: float = 1e-8
    mask_factor: float = 1.5
    w_min: float = 0.0
    coarse_n: int = 8
    name: str = ""
    neumann_faces: int = 0   # bit f: zero-flux domain face f (x-, x+, y-, y+, z-, z+)
    uniform_level: int = 0   # levels <= this are complete; finer ones follow refine_kind

    @property
    def lsf_n(self) -> int:
        if self.lsf_kind == LSF_SPHERES:
            return len(self.lsf_params) // 4
        if self.lsf_kind in (LSF_CYLINDER_Z, LSF_SPHEROID, LSF_RHOMBUS, LSF_HEART, LSF_ASTROID, LSF_ELECTRODES):
            return 1
        return 0

    def finest_cells_per_dim(self) -> int:
        return self.block_n * (1 << (self.max_level - 1))


@dataclass
class Workload:
    geom: Geometry
    rhs: callable            # xyz[n,3] -> g[n]
    iface_value: callable    # xyz[n,3] -> phi_b[n]
    domain_value: callable   # xyz[n,3] -> phi_b[n]
    exact: callable = None   # xyz[n,3] -> phi[n] (closed form), if any
    notes: str = ""
    extra: dict = field(default_factory=dict)


# ---------------------------------------------------------------- closed forms
def _mms2d_phi(x):
    return np.sin(2 * np.pi * x[:, 0]) * np.cos(3 * np.pi * x[:, 1]) + x[:, 0] ** 2


def _mms2d_g(x):
    # Laplacian of _mms2d_phi, written out analytically
    return (-13.0 * np.pi ** 2 * np.sin(2 * np.pi * x[:, 0]) * np.cos(3 * np.pi * x[:, 1])
            + 2.0)


def _mms3d_phi(x):
    return np.exp(x[:, 0]) * np.sin(np.pi * x[:, 1]) * np.cos(np.pi * x[:, 2])


def _mms3d_g(x):
    return (1.0 - 2.0 * np.pi ** 2) * _mms3d_phi(x)


def mms2d(max_level: int = 4, block_n: int = 8, w_min: float = 4e-3) -> Workload:
    """2D manufactured problem: 64^2 cells (max_level 4) in 8^2 blocks."""
    g = Geometry(dim=2, block_n=block_n, max_level=max_level, lsf_kind=LSF_SPHERES,
                 lsf_params=np.array([0.5, 0.5, 0.0, 0.25]), w_min=w_min,
                 name=f"mms2d_{block_n * (1 << (max_level - 1))}")
    return Workload(g, _mms2d_g, _mms2d_phi, _mms2d_phi, exact=_mms2d_phi)


def mms3d(max_level: int = 5, block_n: int = 16, w_min: float = 8e-3) -> Workload:
    """3D manufactured problem: 256^3 cells (max_level 5) in 16^3 blocks."""
    g = Geometry(dim=3, block_n=block_n, max_level=max_level, lsf_kind=LSF_SPHERES,
                 lsf_params=np.array([0.5, 0.5, 0.5, 0.3]), w_min=w_min,
                 name=f"mms3d_{block_n * (1 << (max_level - 1))}")
    return Workload(g, _mms3d_g, _mms3d_phi, _mms3d_phi, exact=_mms3d_phi)


def sphere_params(n: int, seed: int) -> np.ndarray:
    """n spheres, centres U[0.2,0.8]^3, radii U[0.03,0.1] (seeded)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.2, 0.8, size=(n, 3))
    r = rng.uniform(0.03, 0.1, size=(n, 1))
    return np.concatenate([c, r], axis=1).reshape(-1)


def spheres(n_spheres: int = 20, max_level: int = 6, block_n: int = 16, seed: int = 3,
            g_seed: int = 31, adaptive: bool = True, refine_width: float = 2.0 + math.sqrt(3) / 2,
            w_min: float = 8e-3) -> Workload:
    """Union of seeded spheres; phi=1 on the spheres, 0 on the cube; g ~ N(0,1)."""
    geom = Geometry(dim=3, block_n=block_n, max_level=max_level, lsf_kind=LSF_SPHERES,
                    lsf_params=sphere_params(n_spheres, seed),
                    refine_kind=REFINE_NEAR_INTERFACE if adaptive else REFINE_UNIFORM,
                    refine_width=refine_width, w_min=w_min,
                    name=f"spheres{n_spheres}_L{max_level}_{'amr' if adaptive else 'uni'}")

    def rhs(x, _seed=g_seed):
        return np.random.default_rng(_seed).standard_normal(x.shape[0])

    return Workload(geom, rhs, lambda x: np.ones(x.shape[0]), lambda x: np.zeros(x.shape[0]))


def gaussian_params(seed: int, n_src: int = 8):
    """Amplitudes U[-1,1], widths U[0.02,0.05] and centres U[0.1,0.9]^3 of
    n_src Gaussian sources (seeded)."""
    rng = np.random.default_rng(seed)
    amp = rng.uniform(-1.0, 1.0, n_src)
    wid = rng.uniform(0.02, 0.05, n_src)
    cen = rng.uniform(0.1, 0.9, size=(n_src, 3))
    return amp, wid, cen


def gaussian_sources(x: np.ndarray, seed: int, n_src: int = 8) -> np.ndarray:
    """Sum of n_src Gaussians: g = sum A exp(-|x-c|^2 / (2 w^2)) with the
    parameters of gaussian_params(seed)."""
    amp, wid, cen = gaussian_params(seed, n_src)
    out = np.zeros(x.shape[0])
    for a, w, c in zip(amp, wid, cen):
        d2 = ((x[:, :3] - c) ** 2).sum(axis=1)
        out += a * np.exp(-d2 / (2.0 * w * w))
    return out


def cylinder(max_level: int = 4, block_n: int = 16, n_rhs: int = 64, seed0: int = 400,
             w_min: float = 8e-3) -> Workload:
    """Cylinder r=0.2 along z through (0.5,0.5); phi=0 on it and on the cube;
    n_rhs right-hand sides of 8 Gaussian sources each (seeds seed0+i)."""
    geom = Geometry(dim=3, block_n=block_n, max_level=max_level, lsf_kind=LSF_CYLINDER_Z,
                    lsf_params=np.array([0.5, 0.5, 0.2]), w_min=w_min,
                    name=f"cylinder_{block_n * (1 << (max_level - 1))}")

    def rhs(x, i=0):
        return gaussian_sources(x, seed0 + i)

    z = lambda x: np.zeros(x.shape[0])
    return Workload(geom, rhs, z, z, extra={"n_rhs": n_rhs, "seed0": seed0})


def no_interface(max_level: int = 3, block_n: int = 16) -> Workload:
    """The 3D manufactured problem without any interface (no level set):
    Dirichlet data on the cube only, standard stencils everywhere."""
    geom = Geometry(dim=3, block_n=block_n, max_level=max_level, lsf_kind=LSF_NONE, lsf_params=np.zeros(1),
                    name=f"no_interface_{block_n * (1 << (max_level - 1))}")
    return Workload(geom, _mms3d_g, _mms3d_phi, _mms3d_phi, exact=_mms3d_phi)


def through_centres(max_level: int = 3, block_n: int = 16, a: int = 12, b: int = 5) -> Workload:
    """Degenerate interface: a cylinder along z through (1/2, 1/2) whose
    radius is the distance of the finest-level cell centre (1/2 + (a + 1/2)
    dx, 1/2 + (b + 1/2) dx) from the axis, computed with the same operations
    as the level set, so that f = 0 exactly at the centres of that cell and
    its seven mirror images in every z layer; phi = 1 on the cylinder and 0 on
    the cube, Gaussian sources as rhs (seed 7)."""
    n = block_n * (1 << (max_level - 1))
    ex, ey = (a + 0.5) / n, (b + 0.5) / n
    r = float(np.sqrt(ex * ex + ey * ey))
    geom = Geometry(dim=3, block_n=block_n, max_level=max_level, lsf_kind=LSF_CYLINDER_Z,
                    lsf_params=np.array([0.5, 0.5, r]), w_min=8e-3, name=f"through_centres_{n}")
    return Workload(geom, lambda x: gaussian_sources(x, 7), lambda x: np.ones(x.shape[0]),
                    lambda x: np.zeros(x.shape[0]), extra={"radius": r, "on_interface": (a, b)})


def sphere_f1(dim: int = 3, max_level: int = 4, R: float = 0.25, block_n: int = 8,
              phi_b: float = 0.0, a: float = 1.0) -> Workload:
    """Sec. 4.1 convergence test: Laplace equation, f = |x| - R on a domain of
    unit size centred at the origin; the exact solution of eq.
    (solution-sphere) is imposed on the domain boundary, phi_b on the sphere."""
    geom = Geometry(dim=dim, block_n=block_n, max_level=max_level, lsf_kind=LSF_SPHERES,
                    lsf_params=np.array([0.0, 0.0, 0.0, R]), lo=(-0.5, -0.5, -0.5),
                    w_min=4e-3 if dim == 2 else 8e-3,
                    name=f"sphere_f1_{dim}d_{block_n * (1 << (max_level - 1))}")

    def exact(x):
        r = np.sqrt((x[:, :dim] ** 2).sum(axis=1))
        if dim == 2:
            return phi_b + a * np.log(r / R)
        return phi_b + a * (1.0 - R / r)

    return Workload(geom, lambda x: np.zeros(x.shape[0]), lambda x: np.full(x.shape[0], phi_b),
                    exact, exact=exact)


# 3D forms of the shapes: "ring" p = 4(sqrt(x^2 + y^2) - 0.5), q = 4(z - 0.5),
# the printed axisymmetric transform with the same x4 scale as in 2D (axis on
# the cube edge x = y = 0); "spindle" p = 4|(x, y) - (0.5, 0.5)|,
# q = 4(z - 0.5), the shape revolved about the cube's vertical centre line
SHAPE_3D = {"ring": [0.0, 0.0, 0.5, 4.0, 0.5], "spindle": [0.5, 0.5, 0.5, 4.0, 0.0]}


def sharp_shape(shape: str, dim: int = 2, max_level: int = 4, block_n: int = 8, form3d: str = "ring") -> Workload:
    """Sec. 4.2: Laplace equation on the unit square/cube, phi = 1 on the
    shape's boundary, 0 on the domain boundary, uniform grid, w_min = 4e-3
    (2D) or 8e-3 (3D); 2D shapes centred at 0.5 with scale 4, 3D forms as
    in SHAPE_3D."""
    prm = [0.5, 0.5, 0.5, 4.0, 0.0] if dim == 2 else SHAPE_3D[form3d]
    geom = Geometry(dim=dim, block_n=block_n, max_level=max_level, lsf_kind=SHAPES[shape],
                    lsf_params=np.array(prm), w_min=4e-3 if dim == 2 else 8e-3,
                    name=f"{shape}_{dim}d_{block_n * (1 << (max_level - 1))}" + ("" if dim == 2 else f"_{form3d}"))
    return Workload(geom, lambda x: np.zeros(x.shape[0]), lambda x: np.ones(x.shape[0]),
                    lambda x: np.zeros(x.shape[0]))


def two_electrodes(max_level: int = 7, uniform_level: int = 5, block_n: int = 8, refine_width: float = 1.0,
                   tip_z: float = 0.6) -> Workload:
    """Sec. 4.3: unit cube, phi = 1 on the top face and 0 on the bottom face,
    zero flux on the four sides; a rod electrode of radius 0.05 hanging from
    the top (segment (0.5, 0.5, tip_z)-(0.5, 0.5, 1.1)) at phi = 1 and a
    half sphere of radius 0.25 centred on the bottom face at phi = 0.
    Uniform to `uniform_level`, then refined near the electrodes to
    max_level (8^3 blocks: dx = 1/128 and 1/512 for 5 and 7); g = 0."""
    p = np.array([0.5, 0.5, tip_z, 0.5, 0.5, 1.1, 0.05, 0.5, 0.5, 0.0, 0.25])
    geom = Geometry(dim=3, block_n=block_n, max_level=max_level, lsf_kind=LSF_ELECTRODES, lsf_params=p,
                    refine_kind=REFINE_NEAR_INTERFACE, refine_width=refine_width, w_min=8e-3,
                    neumann_faces=0b001111, uniform_level=uniform_level,
                    name=f"two_electrodes_L{max_level}")

    def on_rod(x):
        ab = p[3:6] - p[0:3]
        t = np.clip(((x[:, :3] - p[0:3]) @ ab) / (ab @ ab), 0.0, 1.0)
        rod = np.linalg.norm(x[:, :3] - (p[0:3] + t[:, None] * ab), axis=1) - p[6]
        sph = np.linalg.norm(x[:, :3] - p[7:10], axis=1) - p[10]
        return np.abs(rod) < np.abs(sph)

    return Workload(geom, lambda x: np.zeros(x.shape[0]), lambda x: on_rod(x).astype(float),
                    lambda x: (x[:, 2] > 0.5).astype(float))


def neumann2d(max_level: int = 5) -> Workload:
    """2D, zero flux on the x faces: phi = cos(pi x) exp(pi y) (harmonic,
    d phi/dx = 0 at x = 0 and 1) on a circle and on the y faces, g = 0;
    8^2 blocks refined near the circle."""
    geom = Geometry(dim=2, block_n=8, max_level=max_level, lsf_kind=LSF_SPHERES,
                    lsf_params=np.array([0.55, 0.45, 0.0, 0.2]), refine_kind=REFINE_NEAR_INTERFACE,
                    refine_width=1.0, w_min=4e-3, neumann_faces=0b0011, name=f"neumann2d_L{max_level}")
    phi = lambda x: np.cos(np.pi * x[:, 0]) * np.exp(np.pi * x[:, 1])
    return Workload(geom, lambda x: np.zeros(x.shape[0]), phi, phi, exact=phi)


def serving_geometries(seed0: int = 500, counts=(1, 5, 10, 20)):
    """The four pre-built level sets of the serving stream: unions of
    {1, 5, 10, 20} seeded spheres."""
    return [sphere_params(n, seed0 + i) for i, n in enumerate(counts)]


def serving_stream(n_requests: int, rate_hz: float, seed: int = 510):
    """Poisson arrivals at a fixed rate: (arrival_time_s, size_level, geom_id,
    rhs_seed) per request; sizes uniform over 64^3, 128^3, 256^3 (max_level
    3, 4, 5 with 16^3 blocks)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    t = np.cumsum(gaps) - gaps[0]
    lv = rng.integers(3, 6, n_requests)
    gid = rng.integers(0, 4, n_requests)
    return [(float(t[i]), int(lv[i]), int(gid[i]), 10000 + i) for i in range(n_requests)]
