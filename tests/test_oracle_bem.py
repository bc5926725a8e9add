"""Pins of the oracle's P1 collocation of the single-layer equation (Section 4).

* The meshes: icospheres with the paper's vertex counts (Table
  max_rank_frequency: N = 3 N_c = 7,686, 30,726, 122,886), closed and
  consistently oriented.
* The element rule: exact for polynomials up to its degree on the reference
  triangle (closed-form monomial integrals), every hat function attached to
  its own vertex whichever vertex the rule collapses onto (the closed form
  of int lambda_k y dS), and the singular rule against the closed form of
  int 1/|y - A| dS over a triangle with vertex A.
* The assembled matrix: A (1 x c) is the single layer of a constant density,
  which on the sphere has a closed form at any frequency; the discrete value
  converges to it at the O(h^2) rate of the flat-triangle geometry.  The
  matrix equals the entry-by-entry definition (a gather over the elements of
  each node, written independently of the U W V form) on a small mesh.
"""
import math

import numpy as np
import pytest

from paper_1706_09384_amd import workloads as W


@pytest.fixture(scope="module")
def bem():
    from oracle import bem as b
    return b


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4, 5])
def test_icosphere_is_a_closed_oriented_sphere_mesh(level):
    P, T = W.icosphere(level)
    nv, nf = 10 * 4**level + 2, 20 * 4**level
    assert P.shape == (nv, 3) and T.shape == (nf, 3)
    assert np.allclose(np.linalg.norm(P, axis=1), 1.0, atol=1e-14)
    edges = {}
    for a, b, c in T:
        for u, v in ((a, b), (b, c), (c, a)):
            edges[(u, v)] = edges.get((u, v), 0) + 1
    assert all(n == 1 for n in edges.values())
    assert all((v, u) in edges for (u, v) in edges)          # every edge in two faces, opposite ways
    assert nv - len(edges) // 2 + nf == 2                     # Euler characteristic of a sphere
    a, b, c = P[T[:, 0]], P[T[:, 1]], P[T[:, 2]]
    assert (np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) > 0).all()   # outward


def test_paper_mesh_sizes():
    assert [3 * (10 * 4**L + 2) for L in (4, 5, 6)] == [7686, 30726, 122886]


@pytest.mark.parametrize("q", [1, 2, 3, 5])
def test_collapsed_rule_integrates_monomials(bem, q):
    """int over the reference triangle of x^a y^b = a! b! / (a + b + 2)!,
    exact for a + b <= 2q - 2."""
    s, t, w = bem.collapsed_rule(q)
    x, y = s * (1.0 - t), s * t     # collapse onto the origin of the reference triangle
    for a in range(2 * q - 1):
        for b in range(2 * q - 1 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs(np.sum(w * x**a * y**b) - exact) <= 1e-14
    if q <= 3:   # one degree higher is no longer exact
        a = 2 * q - 1
        assert abs(np.sum(w * x**a) - 1.0 / ((a + 1) * (a + 2))) > 1e-8


@pytest.mark.parametrize("c", [0, 1, 2])
def test_hat_functions_follow_their_vertices(bem, c):
    """int_T lambda_k y_a dS = (area / 12) (2 Y_k + sum_{l != k} Y_l)_a for every k,
    whatever vertex the rule collapses onto (a hat function attached to the
    wrong vertex fails this on a generic triangle)."""
    P = np.array([[0.3, -0.2, 0.1], [1.7, 0.4, -0.3], [0.2, 1.1, 0.9]])
    T = np.array([[0, 1, 2]])
    area = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
    got = bem.element_integral(lambda y: y, P, T, 0, c, 2)
    want = np.array([area / 12.0 * (P.sum(axis=0) + P[k]) for k in range(3)])
    assert np.allclose(got, want, rtol=0, atol=1e-14)
    tot = bem.element_integral(lambda y: np.ones(len(y)), P, T, 0, c, 2)
    assert np.allclose(tot, area / 3.0, rtol=1e-14)


@pytest.mark.parametrize("c", [0, 1, 2])
def test_singular_rule_against_closed_form(bem, c):
    P = np.array([[0.3, -0.2, 0.1], [1.7, 0.4, -0.3], [0.2, 1.1, 0.9]])
    T = np.array([[0, 1, 2]])
    A = P[c]
    exact = bem.inv_r_vertex([P[c], P[(c + 1) % 3], P[(c + 2) % 3]])
    for q, tol in ((6, 1e-5), (20, 1e-14)):
        got = bem.element_integral(lambda y: 1.0 / np.linalg.norm(y - A, axis=1), P, T, 0, c, q).sum()
        assert abs(got - exact) <= tol * exact
    # the regular rule (collapsed elsewhere) is visibly worse on this integrand
    other = (c + 1) % 3
    bad = bem.element_integral(lambda y: 1.0 / np.linalg.norm(y - A, axis=1), P, T, 0, other, 6).sum()
    assert abs(bad - exact) > 1e-4 * exact


def test_sphere_closed_form_itself(bem):
    """The closed form of the constant-density single layer, against a direct
    quadrature over the exact sphere (polar angle about the point, where the
    1/r of U is cancelled by sin theta), at omega = 3."""
    import oracle as orc
    from scipy.integrate import quad
    omega, R = 3.0, 1.0
    x = np.array([0.0, 0.0, R])
    sn, st = bem.sphere_constant_density(R, omega)

    def block(th, ph):
        y = R * np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
        return orc.green_block(0, x, y, omega=omega) * R * R * math.sin(th)

    # phi by the trapezoidal rule (periodic, spectrally accurate), theta adaptive
    nph = 32
    phs = 2 * math.pi * np.arange(nph) / nph
    S = np.zeros((3, 3), dtype=complex)
    for a, b in ((0, 0), (2, 2), (0, 1)):
        for part in (np.real, np.imag):
            f = lambda th: sum(part(block(th, ph)[a, b]) for ph in phs) * 2 * math.pi / nph
            v, _ = quad(f, 0.0, math.pi, limit=200, epsabs=1e-11)
            S[a, b] += v if part is np.real else 1j * v
    assert abs(S[0, 0] - st) <= 1e-8 * abs(st)     # tangential
    assert abs(S[2, 2] - sn) <= 1e-8 * abs(sn)     # normal
    assert abs(S[0, 1]) <= 1e-9


@pytest.mark.parametrize("omega", [0.0, 3.0])
def test_collocation_converges_to_sphere_closed_form(bem, omega):
    c = np.array([0.3, -0.5, 0.8])
    errs = []
    for level in (1, 2, 3):
        P, T = W.icosphere(level)
        rows = np.arange(0, P.shape[0], 5)
        y = bem.apply_rows(P, T, np.tile(c, P.shape[0]), rows, omega).reshape(-1, 3)
        sn, st = bem.sphere_constant_density(1.0, omega)
        xh = P[rows]
        ex = sn * (xh @ c)[:, None] * xh + st * (c[None, :] - (xh @ c)[:, None] * xh)
        errs.append(np.abs(y - ex).max() / np.abs(ex).max())
    assert errs[2] < 0.012
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5      # O(h^2)


def test_matrix_equals_entrywise_definition(bem):
    """Gather form: A_ij = sum_{e with vertex j} sum_q w_q v_j(y_q) U(x_i, y_q), the
    rule collapsed onto x_i when x_i is a vertex of e."""
    import oracle as orc
    P, T = W.icosphere(1)
    omega = 3.0
    A = bem.collocation_matrix(P, T, omega)
    elems = [[] for _ in range(P.shape[0])]
    for e in range(T.shape[0]):
        for k in range(3):
            elems[T[e, k]].append((e, k))
    rng = np.random.default_rng(1)
    for i, j in [(0, 0), (0, int(T[0, 1]))] + [tuple(rng.integers(0, P.shape[0], 2)) for _ in range(12)]:
        B = np.zeros((3, 3), dtype=complex)
        for e, k in elems[j]:
            loc = [kk for kk in range(3) if T[e, kk] == i]
            cc, q = (loc[0], 6) if loc else (0, 3)
            y, w, hat = bem.element_rule(P, T, e, cc, q)
            for qq in range(len(w)):
                B += w[qq] * hat[qq, k] * orc.green_block(0, P[i], y[qq], omega=omega)
        assert np.allclose(A[3 * i:3 * i + 3, 3 * j:3 * j + 3], B, rtol=1e-12, atol=1e-14 * np.abs(B).max())


def test_p_wave_rhs():
    P, _ = W.icosphere(1)
    b = W.p_wave(P, 3.0).reshape(-1, 3)
    assert np.allclose(b[:, :2], 0) and np.allclose(b[:, 2], np.exp(1.5j * P[:, 2]))


def test_rule_orders_converge(bem):
    """Raising the regular and singular orders changes the matrix less and less:
    the default (3, 6) is within 1e-3 of (8, 16) on a coarse mesh, and (5, 10)
    is closer still (a rule mis-assembled for one of the two cases would not
    converge)."""
    P, T = W.icosphere(1)
    ref = bem.collocation_matrix(P, T, 3.0, q_reg=8, q_sing=16)
    e = [np.abs(bem.collocation_matrix(P, T, 3.0, q_reg=qr, q_sing=qs) - ref).max() / np.abs(ref).max()
         for qr, qs in ((3, 6), (5, 10))]
    assert e[0] <= 1e-3 and e[1] <= 0.2 * e[0]
