"""P1 collocation of the single-layer equation (Section 4) -- FP64 oracle.

TEST INFRASTRUCTURE: only the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of the benchmark may import this module.  It shares no code
with the library.

The boundary is a mesh of flat triangles E_e with vertices y_1 .. y_Nc, the
traction is approximated by continuous piecewise-linear hat functions v_j
(v_j(y_k) = delta_jk), and eq. EFIE is enforced at the vertices (collocation
points x_i = y_i).  The result is the 3 Nc x 3 Nc system of eq. discre_syst,
whose 3 x 3 block (i, j) is

    A_ij = sum over elements e with vertex j of  int_{E_e} U(x_i, y) v_j(y) dS(y).

Every element integral is a quadrature (readings of the design notes: the
paper names no rule):

* a collapsed (Duffy) Gauss-Legendre product rule on the triangle (c, c+1,
  c+2): y(s, t) = y_c + s (y_{c+1} - y_c) + s t (y_{c+2} - y_{c+1}) for
  (s, t) in [0, 1]^2, dS = s |(y_{c+1} - y_c) x (y_{c+2} - y_{c+1})| ds dt,
  q Gauss-Legendre points in each of s and t; the hat functions of the three
  vertices are the barycentric coordinates 1 - s, s (1 - t), s t;
* when x_i is a vertex of E_e the rule collapses onto x_i (c = that vertex),
  so the factor s of dS cancels the 1/|x_i - y| singularity of U, with
  q_sing points; otherwise it collapses onto the element's first vertex,
  with q_reg points.

With a single rule per element this is the factorised form the paper writes
for the single layer, A = U_w W V: U_w the Green's tensors between the
collocation points and all quadrature points, W the quadrature weights, V the
hat functions at the quadrature points -- except that the elements containing
x_i are integrated with their own rule.  ``collocation_matrix`` builds exactly
that: U W V over the regular rule, then, for every (x_i, element containing
x_i), the singular rule's integral in place of the regular one.
"""
from __future__ import annotations

import functools

import numpy as np

from . import KERNEL_U, Problem, dense, matvec_rows


@functools.lru_cache(maxsize=None)
def gauss01(q: int):
    """Gauss-Legendre nodes and weights on [0, 1] (q points, exact to degree 2q - 1)."""
    x, w = np.polynomial.legendre.leggauss(int(q))
    return 0.5 * (x + 1.0), 0.5 * w


@functools.lru_cache(maxsize=None)
def collapsed_rule(q: int):
    """(s, t, w) of the collapsed product rule, w = w_s w_t s (the Duffy factor)."""
    g, w = gauss01(q)
    s, t = np.meshgrid(g, g, indexing="ij")
    ws, wt = np.meshgrid(w, w, indexing="ij")
    return s.ravel(), t.ravel(), (ws * wt * s).ravel()


def element_rule(P: np.ndarray, tri: np.ndarray, e: int, c: int, q: int):
    """Quadrature points y (nq, 3), weights (nq,) including the surface Jacobian,
    and the three hat-function values (nq, 3) in the element's own vertex
    order, for the rule collapsed onto local vertex c."""
    v = tri[e]
    a, b, cc = P[v[c]], P[v[(c + 1) % 3]], P[v[(c + 2) % 3]]
    e1, e2 = b - a, cc - b
    two_area = np.linalg.norm(np.cross(e1, e2))
    s, t, w = collapsed_rule(q)
    y = a[None, :] + s[:, None] * e1[None, :] + (s * t)[:, None] * e2[None, :]
    lam_rot = np.stack([1.0 - s, s * (1.0 - t), s * t], axis=1)   # vertices c, c+1, c+2
    lam = np.empty_like(lam_rot)
    for k in range(3):
        lam[:, (c + k) % 3] = lam_rot[:, k]
    return y, w * two_area, lam


def element_integral(f, P, tri, e: int, c: int, q: int) -> np.ndarray:
    """[int_{E_e} f(y) v_k(y) dS]_k for the three vertices k of element e, with the
    rule collapsed onto local vertex c.  f maps (nq, 3) points to (nq, ...) values."""
    y, w, lam = element_rule(P, tri, e, c, q)
    fy = np.asarray(f(y))
    return np.einsum("q,qk,q...->k...", w, lam, fy)


def _u_rows(X, Y, omega, lam, mu, rho):
    """U(x, y) for all pairs, shape (3 nx, 3 ny) (eq. elasto_U)."""
    return dense(Problem(KERNEL_U, X, Y, None, omega, lam, mu, rho, same=False))


def _regular_points(P, tri, q):
    """All elements' regular-rule points, their weights and the sparse W V map
    as (point index, node, weight * hat value) triplets."""
    ys, ws, rows, cols, vals = [], [], [], [], []
    off = 0
    for e in range(tri.shape[0]):
        y, w, lam = element_rule(P, tri, e, 0, q)
        ys.append(y)
        ws.append(w)
        for k in range(3):
            rows.append(off + np.arange(len(w)))
            cols.append(np.full(len(w), tri[e, k]))
            vals.append(w * lam[:, k])
        off += len(w)
    return np.concatenate(ys), np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)


def _wv_dense(nq, nc, rows, cols, vals):
    """(nq, nc) matrix of weight x hat value (the scalar W V of Section 4)."""
    M = np.zeros((nq, nc))
    np.add.at(M, (rows, cols), vals)
    return M


def collocation_matrix(P: np.ndarray, tri: np.ndarray, omega: float, lam: float = 2.0,
                       mu: float = 1.0, rho: float = 1.0, q_reg: int = 3, q_sing: int = 6,
                       chunk: int = 96) -> np.ndarray:
    """Dense complex128 collocation matrix (3 Nc, 3 Nc), original node order,
    rows 3 i + a, columns 3 j + b."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    tri = np.asarray(tri)
    nc = P.shape[0]
    Yq, rows, cols, vals = _regular_points(P, tri, q_reg)
    WV = _wv_dense(Yq.shape[0], nc, rows, cols, vals)
    A = np.empty((3 * nc, 3 * nc), dtype=np.complex128)
    for i0 in range(0, nc, chunk):
        i1 = min(nc, i0 + chunk)
        nr = 3 * (i1 - i0)
        G = _u_rows(P[i0:i1], Yq, omega, lam, mu, rho).reshape(nr, -1, 3)
        # sum_q G[:, q, b] WV[q, j] -> block column (j, b)
        T = G.transpose(0, 2, 1).reshape(nr * 3, -1) @ WV
        A[3 * i0:3 * i1] = T.reshape(nr, 3, nc).transpose(0, 2, 1).reshape(nr, 3 * nc)
    _singular_fix(A, P, tri, omega, lam, mu, rho, q_reg, q_sing)
    return A


def _singular_fix(A, P, tri, omega, lam, mu, rho, q_reg, q_sing, rows=None):
    """Replace, for every element containing the collocation point x_i, the
    regular-rule integral by the singular one (rows: the i to treat, as a map
    i -> row offset in A; all rows when None)."""
    for e in range(tri.shape[0]):
        for c in range(3):
            i = int(tri[e, c])
            if rows is not None and i not in rows:
                continue
            r0 = 3 * (i if rows is None else rows[i])
            xi = P[i:i + 1]
            for rule_c, q, sign in ((c, q_sing, 1.0), (0, q_reg, -1.0)):
                y, w, hat = element_rule(P, tri, e, rule_c, q)
                G = _u_rows(xi, y, omega, lam, mu, rho).reshape(3, -1, 3)
                for k in range(3):
                    j = int(tri[e, k])
                    A[r0:r0 + 3, 3 * j:3 * j + 3] += sign * np.einsum("aqb,q->ab", G, w * hat[:, k])


def apply_rows(P, tri, p: np.ndarray, rows, omega: float, lam: float = 2.0, mu: float = 1.0,
               rho: float = 1.0, q_reg: int = 3, q_sing: int = 6) -> np.ndarray:
    """Rows 3 i + a (i in rows) of A p without storing A: U W V p on the regular
    rule, then the singular elements of those rows re-integrated."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    tri = np.asarray(tri)
    rows = np.asarray(rows, dtype=np.int64)
    nc = P.shape[0]
    Yq, qr, qc, qv = _regular_points(P, tri, q_reg)
    pn = np.asarray(p, dtype=np.complex128).reshape(nc, 3)
    f = np.zeros((Yq.shape[0], 3), dtype=np.complex128)   # W V p at the quadrature points
    np.add.at(f, qr, qv[:, None] * pn[qc])
    out = matvec_rows(Problem(KERNEL_U, P, Yq, None, omega, lam, mu, rho, same=False),
                      f.ravel(), rows=rows).reshape(len(rows), 3)
    pos = {int(i): k for k, i in enumerate(rows)}
    Ar = np.zeros((3 * len(rows), 3 * nc), dtype=np.complex128)
    _singular_fix(Ar, P, tri, omega, lam, mu, rho, q_reg, q_sing, rows=pos)
    return out.ravel() + Ar @ pn.ravel()


# ------------------------------------------------------------------ closed forms
def sphere_constant_density(R: float, omega: float, lam: float = 2.0, mu: float = 1.0,
                            rho: float = 1.0):
    """(sigma_n, sigma_t): the single layer of a constant vector density c on the
    sphere |y| = R, at a point x of the sphere, is sigma_n (x^.c) x^ + sigma_t
    (c - (x^.c) x^).

    With U = (1/mu)[G_s I + ks^-2 Hess(G_s - G_p)] and Phi_k(x) = int G_k(x - y)
    dS(y) = R sin(kR) e^{ik rho} / (k rho) for rho = |x| >= R, the Hessian of a
    radial f is f'' x^x^ + (f'/rho)(I - x^x^); Phi_s - Phi_p is twice
    continuously differentiable across the sphere, so its outside derivatives
    at rho = R give the values on the sphere.  omega = 0 is the Kelvin limit
    R (5 - 6 nu) / (6 mu (1 - nu)) in both directions.
    """
    if omega == 0.0:
        nu = lam / (2.0 * (lam + mu))
        v = R * (5.0 - 6.0 * nu) / (6.0 * mu * (1.0 - nu))
        return complex(v), complex(v)
    ks = omega * np.sqrt(rho / mu)
    kp = omega * np.sqrt(rho / (lam + 2.0 * mu))

    def derivs(k):
        al = R * np.sin(k * R) / k
        e = np.exp(1j * k * R)
        f0 = al * e / R
        f1 = al * e * (1j * k / R - 1.0 / R**2)
        f2 = al * e * (-k * k / R - 2j * k / R**2 + 2.0 / R**3)
        return f0, f1, f2

    s0, s1, s2 = derivs(ks)
    _, p1, p2 = derivs(kp)
    sig_n = (s0 + (s2 - p2) / ks**2) / mu
    sig_t = (s0 + (s1 - p1) / (R * ks**2)) / mu
    return complex(sig_n), complex(sig_t)


def inv_r_vertex(P3: np.ndarray) -> float:
    """int over the flat triangle (A, B, C) of 1 / |y - A| dS(y), in closed form:
    polar coordinates about A give int R(phi) dphi with R = h / cos(psi), psi the
    angle from the foot F of A on line BC, so the integral is
    h [asinh(tan psi)] = h (asinh(d_C / h) - asinh(d_B / h)), d the signed
    positions of B and C along BC measured from F."""
    a, b, c = (np.asarray(v, dtype=np.float64) for v in P3)
    u = (c - b) / np.linalg.norm(c - b)
    f = b + np.dot(a - b, u) * u
    h = np.linalg.norm(a - f)
    return float(h * (np.arcsinh(np.dot(c - f, u) / h) - np.arcsinh(np.dot(b - f, u) / h)))
