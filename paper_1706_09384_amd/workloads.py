"""Seeded synthetic inputs: point clouds, normals and right-hand sides.

This module only produces input data (coordinates, unit normals, random vectors
and the numeric parameters of each workload).  It contains none of the
H-matrix method's arithmetic, so both the library's tests and the CPU oracle
draw their inputs from it.

The paper's experiments use triangulated sphere meshes with material
mu = rho = 1, nu = 1/3 (so lambda = 2 mu and kappa_p = kappa_s / 2), see the
test problem definition of Section 7.1.  The meshes themselves are not
available, so point clouds of the same geometry scale, wavelength density and
size range stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict
from typing import Optional

import numpy as np

KERNEL_U = 0
KERNEL_T = 1

SPHERE_AREA = 4.0 * math.pi
CUBE_AREA = 24.0
# Surface area of the prolate spheroid with semi-axes (2, 1, 1):
# 2 pi b^2 (1 + a/(b e) asin e), e = sqrt(1 - b^2/a^2).
_E = math.sqrt(1.0 - 0.25)
SPHEROID_AREA = 2.0 * math.pi * (1.0 + 2.0 / _E * math.asin(_E))


def fibonacci_sphere(n: int) -> np.ndarray:
    """Fibonacci lattice on the unit sphere, (n, 3) float64, deterministic."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * (math.pi * (3.0 - math.sqrt(5.0)))
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def cube_surface(n: int, seed: int = 0):
    """Uniform points on the surface of [-1, 1]^3 and their outward normals.

    face ~ U{0..5} (face f lies at coordinate f//2 = -1 for even f, +1 for odd
    f), the two in-face coordinates ~ U(-1, 1).
    """
    rng = np.random.default_rng(seed)
    face = rng.integers(0, 6, size=n)
    uv = rng.uniform(-1.0, 1.0, size=(n, 2))
    axis = face // 2
    sign = np.where(face % 2 == 0, -1.0, 1.0)
    pts = np.empty((n, 3), dtype=np.float64)
    nrm = np.zeros((n, 3), dtype=np.float64)
    for a in range(3):
        others = [b for b in range(3) if b != a]
        sel = axis == a
        pts[sel, a] = sign[sel]
        pts[sel, others[0]] = uv[sel, 0]
        pts[sel, others[1]] = uv[sel, 1]
        nrm[sel, a] = sign[sel]
    return pts, nrm


def prolate_spheroid(n: int, seed: int = 0, semi=(2.0, 1.0, 1.0)):
    """Area-uniform points on the spheroid x^2/a^2 + y^2/b^2 + z^2/c^2 = 1.

    A direction u uniform on S^2 is mapped to (a u_x, b u_y, c u_z) and kept
    with probability sqrt(u_x^2/a^2 + u_y^2/b^2 + u_z^2/c^2) * min(a, b, c),
    the ratio of surface elements (rejection sampling).
    """
    a, b, c = semi
    rng = np.random.default_rng(seed)
    out = []
    got = 0
    while got < n:
        m = max(1024, 2 * (n - got))
        g = rng.standard_normal((m, 3))
        u = g / np.linalg.norm(g, axis=1, keepdims=True)
        w = np.sqrt(u[:, 0] ** 2 / a**2 + u[:, 1] ** 2 / b**2 + u[:, 2] ** 2 / c**2) * min(a, b, c)
        keep = rng.uniform(0.0, 1.0, size=m) < w
        p = u[keep] * np.array([a, b, c])
        out.append(p)
        got += p.shape[0]
    pts = np.concatenate(out, axis=0)[:n].copy()
    nrm = pts / np.array([a * a, b * b, c * c])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return pts, nrm


def complex_normal(rows: int, nrhs: int = 1, seed: int = 0) -> np.ndarray:
    """CN(0, 1) entries (g1 + i g2)/sqrt(2), shape (rows, nrhs), complex128."""
    g = np.random.default_rng(seed).standard_normal((2, rows, nrhs))
    return (g[0] + 1j * g[1]) / math.sqrt(2.0)


def uniform_ball(n: int, seed: int = 0, radius: float = 1.0) -> np.ndarray:
    """Uniform points inside a ball (small generic clouds for tests)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    r = radius * rng.uniform(0.0, 1.0, size=(n, 1)) ** (1.0 / 3.0)
    return g * r


@dataclass
class Workload:
    """One synthetic workload: the cloud plus every numeric parameter."""
    name: str
    n_points: int
    kernel: int
    omega: float
    lam: float = 2.0
    mu: float = 1.0
    rho: float = 1.0
    eta: float = 3.0
    eps: float = 1e-4
    leaf: int = 32
    self_re: float = 0.0
    self_im: float = 0.0
    nrhs: int = 1
    geometry: str = "sphere"
    seed: int = 0
    description: str = ""
    extra: dict = field(default_factory=dict)

    def points(self):
        """(points, normals or None) as float64 arrays of shape (n, 3)."""
        if self.geometry == "sphere":
            p = fibonacci_sphere(self.n_points)
            return p, (p.copy() if self.kernel == KERNEL_T else None)
        if self.geometry == "cube":
            p, nrm = cube_surface(self.n_points, self.seed)
            return p, (nrm if self.kernel == KERNEL_T else None)
        if self.geometry == "spheroid":
            p, nrm = prolate_spheroid(self.n_points, self.seed)
            return p, (nrm if self.kernel == KERNEL_T else None)
        raise ValueError(self.geometry)

    def rhs(self, nrhs: Optional[int] = None) -> np.ndarray:
        k = self.nrhs if nrhs is None else nrhs
        # A generator instance of its own, distinct from the one for points.
        return complex_normal(3 * self.n_points, k, seed=self.seed)

    def params(self) -> dict:
        return asdict(self)


def _u_self(area: float, n: int, mu: float = 1.0) -> float:
    # Self 3x3 block (1/(4 pi mu h)) I3 with h = sqrt(area / n).
    h = math.sqrt(area / n)
    return 1.0 / (4.0 * math.pi * mu * h)


def _t_self(area: float, n: int) -> float:
    # Free term 1/2 of the double-layer equation in the unweighted point
    # matrix (rows scaled by 1/w, w = area / n): n / (2 area).
    return n / (2.0 * area)


def plain_sphere_1k() -> Workload:
    """Plain complex128 method, 1,000 Fibonacci points on the unit sphere."""
    n = 1000
    return Workload("sphere1k_U_c128", n, KERNEL_U, omega=5.6, eps=1e-4, leaf=32,
                    self_re=1.0 / (4.0 * math.pi * 0.112), geometry="sphere",
                    description="U kernel, kappa_s=5.6, leaf 32, eta 3, eps 1e-4, complex128")


def precision_sphere_20k(eps: float = 1e-4) -> Workload:
    """Complex64 form, 20,000 Fibonacci points, kappa_s = 25."""
    n = 20000
    return Workload(f"sphere20k_U_c64_eps{eps:.0e}", n, KERNEL_U, omega=25.0, eps=eps, leaf=32,
                    self_re=_u_self(SPHERE_AREA, n), geometry="sphere",
                    description="U kernel, kappa_s=25, complex64 + FP64 recompression/refinement")


def batching_cube_100k(leaf: int = 32) -> Workload:
    """T kernel on 100,000 points on the cube surface, kappa_s * D = 4."""
    n = 100000
    return Workload(f"cube100k_T_leaf{leaf}", n, KERNEL_T, omega=4.0 / (2.0 * math.sqrt(3.0)),
                    eps=1e-4, leaf=leaf, self_re=_t_self(CUBE_AREA, n), geometry="cube",
                    description="T kernel with outward normals, low frequency")


def learned_spheroid_50k() -> Workload:
    """U kernel on 50,000 random points on the (2,1,1) prolate spheroid."""
    n = 50000
    return Workload("spheroid50k_U", n, KERNEL_U, omega=20.0, eps=1e-4, leaf=32,
                    self_re=_u_self(SPHEROID_AREA, n), geometry="spheroid",
                    description="U kernel, kappa_s=20, rank-model evaluation cloud")


def multirhs_sphere_200k() -> Workload:
    """T kernel on 200,000 Fibonacci points, kappa_s = 56, 64 right-hand sides."""
    n = 200000
    return Workload("sphere200k_T_64rhs", n, KERNEL_T, omega=56.0, eps=1e-4, leaf=64, nrhs=64,
                    self_re=_t_self(SPHERE_AREA, n), geometry="sphere",
                    description="T kernel with normals n = x, 64 CN(0,1) right-hand sides")


def small_sphere(n: int, kernel: int = KERNEL_U, omega: float = 5.6, leaf: int = 16,
                 eps: float = 1e-4, eta: float = 3.0) -> Workload:
    """Scaled-down sphere workload for parity tests (same density rule)."""
    self_re = _u_self(SPHERE_AREA, n) if kernel == KERNEL_U else _t_self(SPHERE_AREA, n)
    return Workload(f"sphere{n}", n, kernel, omega=omega, eps=eps, leaf=leaf, eta=eta,
                    self_re=self_re, geometry="sphere")


# Fixed density of points per S-wavelength (the paper's Section 8, Table table_corr):
# (DOFs N = 3 x mesh vertices, circular frequency omega) of its sphere meshes.
TABLE_CORR = [(7686, 8.25), (30726, 16.5), (122886, 33.0), (183099, 40.0), (490629, 66.0),
              (763638, 84.0), (985818, 92.0)]


def fixed_density_series() -> list:
    """(points, omega) pairs of the fixed-density sweep: N_c = N / 3 points at the
    paper's frequencies (10 points per S-wavelength on its meshes)."""
    return [(n // 3, w) for n, w in TABLE_CORR]


def sweep_sphere(n: int, omega: float, kernel: int = KERNEL_U, eps: float = 1e-4,
                 leaf: int = 32) -> Workload:
    """Fibonacci sphere of the frequency sweeps: unit sphere, material of Section 7.1,
    self blocks by the density rule of the other workloads."""
    w = small_sphere(n, kernel=kernel, omega=omega, leaf=leaf, eps=eps)
    w.name = f"sphere{n}_{'U' if kernel == KERNEL_U else 'T'}_w{omega:g}"
    return w


# ---------------------------------------------------------------- meshes
# The paper's sphere meshes (Section 7.1) have N_c = N / 3 = 2,562, 10,242 and
# 40,962 vertices (Table max_rank_frequency), the vertex counts 10 4^L + 2 of
# an icosahedron subdivided L = 4, 5, 6 times.


def icosphere(level: int, radius: float = 1.0):
    """Subdivided icosahedron on the sphere of the given radius.

    Returns (nodes (10 4^level + 2, 3) float64, tri (20 4^level, 3) int32):
    every subdivision splits each triangle into four at its edge midpoints,
    which are pushed out onto the sphere.  Triangles keep one orientation
    (counter-clockwise seen from outside).
    """
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t),
         (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
         (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
         (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    pts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    for _ in range(level):
        mid = {}

        def midpoint(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                m = pts[a] + pts[b]
                pts.append(m / np.linalg.norm(m))
                mid[key] = len(pts) - 1
            return mid[key]

        nf = []
        for a, b, c in f:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = nf
    return radius * np.array(pts), np.array(f, dtype=np.int32)


def p_wave(nodes: np.ndarray, omega: float, lam: float = 2.0, mu: float = 1.0, rho: float = 1.0,
           direction=(0.0, 0.0, 1.0)) -> np.ndarray:
    """Incident plane P wave u_inc(x) = d exp(i kappa_p d.x) sampled at the nodes,
    interleaved (3 n,) complex128 (the vertical incidence of Section 7.1: d = e_z)."""
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    kp = omega * math.sqrt(rho / (lam + 2.0 * mu))
    ph = np.exp(1j * kp * (nodes @ d))
    return (ph[:, None] * d[None, :]).ravel()


@dataclass
class Mesh:
    """A collocation workload: icosphere of the given level, the Section 7.1
    material, and the tree / tolerance parameters."""
    name: str
    level: int
    omega: float
    lam: float = 2.0
    mu: float = 1.0
    rho: float = 1.0
    eta: float = 3.0
    eps: float = 1e-4
    leaf: int = 100
    q_reg: int = 3
    q_sing: int = 6

    def mesh(self):
        return icosphere(self.level)

    @property
    def n_nodes(self) -> int:
        return 10 * 4**self.level + 2

    def rhs(self) -> np.ndarray:
        return p_wave(self.mesh()[0], self.omega, self.lam, self.mu, self.rho)


def bem_sphere(level: int, omega: float = 3.0, eps: float = 1e-4, leaf: int = 100,
               eta: float = 3.0) -> Mesh:
    """P1 collocation of the single-layer equation on the unit icosphere (Section 7.1:
    N_leaf = 100, eta-hat = 3, eps = 1e-4, mu = rho = 1, nu = 1/3)."""
    return Mesh(f"bem_sphere_L{level}_w{omega:g}", level, omega, eps=eps, leaf=leaf, eta=eta)


ALL = {
    "sphere1k": plain_sphere_1k,
    "sphere20k": precision_sphere_20k,
    "cube100k": batching_cube_100k,
    "spheroid50k": learned_spheroid_50k,
    "sphere200k": multirhs_sphere_200k,
}
