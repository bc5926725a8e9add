"""Pins of the oracle's Green's tensors against what the paper and mathematics fix.

None of these re-types the oracle's closed form: each compares it with an
independent statement (finite-difference derivatives of the scalar Helmholtz
Green's function, the Navier equation, the textbook Kelvin solutions, the
traction operator of eq. elasto_T, exact symmetries and zero patterns).
"""
import math

import numpy as np
import pytest

LAM, MU, RHO = 2.0, 1.0, 1.0


def kappas(omega, lam=LAM, mu=MU, rho=RHO):
    return omega * math.sqrt(rho / mu), omega * math.sqrt(rho / (lam + 2 * mu))


def rand_pairs(rng, count, rmin, rmax):
    out = []
    for _ in range(count):
        x = rng.uniform(-1, 1, 3)
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        r = math.exp(rng.uniform(math.log(rmin), math.log(rmax)))
        out.append((x, x - r * d))
    return out


def helm_diff(y, x, ks, kp):
    """D(x) = G_ks - G_kp at distance |x - y|, G_k = e^{ikr}/(4 pi r)."""
    r = np.linalg.norm(x - y)
    return (np.exp(1j * ks * r) - np.exp(1j * kp * r)) / (4 * math.pi * r)


def fd_hessian(f, x, h):
    H = np.zeros((3, 3), dtype=np.complex128)
    E = np.eye(3)
    for a in range(3):
        for b in range(3):
            H[a, b] = (f(x + h * E[a] + h * E[b]) - f(x + h * E[a] - h * E[b])
                       - f(x - h * E[a] + h * E[b]) + f(x - h * E[a] - h * E[b])) / (4 * h * h)
    return H


@pytest.mark.parametrize("omega", [0.3, 5.6, 25.0])
def test_U_equals_derivative_form(orc, omega):
    """U = (1/mu)[G_ks I + ks^-2 Hess_x (G_ks - G_kp)] (eq. elasto_U), Hessian by FD."""
    ks, kp = kappas(omega)
    rng = np.random.default_rng(1)
    for x, y in rand_pairs(rng, 12, 0.02 / ks, 8.0 / ks):
        r = np.linalg.norm(x - y)
        Gs = np.exp(1j * ks * r) / (4 * math.pi * r)
        H = fd_hessian(lambda z: helm_diff(y, z, ks, kp), x, 5e-4 * min(r, 1.0 / ks))
        Ufd = (Gs * np.eye(3) + H / ks**2) / MU
        U = orc.green_block(0, x, y, None, omega, LAM, MU, RHO)
        assert np.linalg.norm(U - Ufd) <= 2e-5 * np.linalg.norm(Ufd), (ks * r)


def navier_residual(orc, x, y, omega, beta, h):
    """mu Lap u + (lam+mu) grad div u + rho w^2 u for u = U(., y) e_beta (eq. NE)."""
    E = np.eye(3)

    def u(z):
        return orc.green_block(0, z, y, None, omega, LAM, MU, RHO)[:, beta]

    u0 = u(x)
    lap = np.zeros(3, dtype=np.complex128)
    gd = np.zeros(3, dtype=np.complex128)
    for a in range(3):
        lap += (u(x + h * E[a]) - 2 * u0 + u(x - h * E[a])) / (h * h)
    # grad div u: d_a sum_c d_c u_c
    for a in range(3):
        for c in range(3):
            if a == c:
                gd[a] += (u(x + h * E[a])[c] - 2 * u0[c] + u(x - h * E[a])[c]) / (h * h)
            else:
                gd[a] += (u(x + h * E[a] + h * E[c])[c] - u(x + h * E[a] - h * E[c])[c]
                          - u(x - h * E[a] + h * E[c])[c] + u(x - h * E[a] - h * E[c])[c]) / (4 * h * h)
    res = MU * lap + (LAM + MU) * gd + RHO * omega**2 * u0
    return np.linalg.norm(res), RHO * omega**2 * np.linalg.norm(u0)


@pytest.mark.parametrize("omega", [2.0, 5.6])
def test_U_solves_navier(orc, omega):
    ks, _ = kappas(omega)
    rng = np.random.default_rng(2)
    for x, y in rand_pairs(rng, 6, 0.6 / ks, 6.0 / ks):
        r = np.linalg.norm(x - y)
        for beta in range(3):
            res, scale = navier_residual(orc, x, y, omega, beta, 1e-3 * min(r, 1.0 / ks))
            assert res <= 1e-4 * scale


def kelvin_U(x, y, lam=LAM, mu=MU):
    """Static Kelvin solution [(lam+3mu) I + (lam+mu) dh dh^T] / (8 pi mu (lam+2mu) r)."""
    d = x - y
    r = np.linalg.norm(d)
    dh = d / r
    return ((lam + 3 * mu) * np.eye(3) + (lam + mu) * np.outer(dh, dh)) / (8 * math.pi * mu * (lam + 2 * mu) * r)


def kelvin_T(x, y, n, lam=LAM, mu=MU):
    """Static traction kernel (Kelvin), written with Poisson's ratio nu.

    With r_i = (x_i - y_i)/r and dr/dn = -r.n (derivative in y along n(y)):
    T = -[dr/dn ((1-2nu) I + 3 r r^T) + (1-2nu)(n r^T - r n^T)] / (8 pi (1-nu) r^2).
    """
    nu = lam / (2 * (lam + mu))
    d = x - y
    r = np.linalg.norm(d)
    rh = d / r
    drdn = -rh @ n
    return -(drdn * ((1 - 2 * nu) * np.eye(3) + 3 * np.outer(rh, rh))
             + (1 - 2 * nu) * (np.outer(n, rh) - np.outer(rh, n))) / (8 * math.pi * (1 - nu) * r * r)


def test_U_static_kelvin_limit(orc):
    rng = np.random.default_rng(3)
    for omega in [1e-6, 1e-3]:
        for x, y in rand_pairs(rng, 8, 0.05, 3.0):
            ks, _ = kappas(omega)
            r = np.linalg.norm(x - y)
            U = orc.green_block(0, x, y, None, omega, LAM, MU, RHO)
            K = kelvin_U(x, y)
            assert np.linalg.norm(U.real - K) <= 4 * ks * r * np.linalg.norm(K) + 1e-14
    # Exactly omega = 0 reduces to the Kelvin solution to rounding.
    x, y = np.array([0.1, 0.2, 0.3]), np.array([-0.4, 0.5, 1.1])
    U0 = orc.green_block(0, x, y, None, 0.0, LAM, MU, RHO)
    assert np.allclose(U0, kelvin_U(x, y), rtol=1e-14, atol=0)


def test_T_static_kelvin_limit(orc):
    rng = np.random.default_rng(4)
    for x, y in rand_pairs(rng, 8, 0.05, 3.0):
        n = rng.standard_normal(3); n /= np.linalg.norm(n)
        T0 = orc.green_block(1, x, y, n, 0.0, LAM, MU, RHO)
        K = kelvin_T(x, y, n)
        assert np.linalg.norm(T0 - K) <= 1e-13 * np.linalg.norm(K)
        T1 = orc.green_block(1, x, y, n, 1e-5, LAM, MU, RHO)
        r = np.linalg.norm(x - y)
        assert np.linalg.norm(T1 - K) <= 4 * 1e-5 * r * np.linalg.norm(K) + 1e-12


def traction_fd(orc, x, y, n, omega, h):
    """Traction operator of eq. elasto_T applied in y to each column of U, by FD.

    t(u) = 2 mu du/dn + lam n div u + mu n x curl u, with u = U(x, .) e_beta.
    """
    E = np.eye(3)
    T = np.zeros((3, 3), dtype=np.complex128)
    for beta in range(3):
        def u(z):
            return orc.green_block(0, x, z, None, omega, LAM, MU, RHO)[:, beta]
        J = np.zeros((3, 3), dtype=np.complex128)       # J[a, s] = d u_a / d y_s
        for s in range(3):
            J[:, s] = (u(y + h * E[s]) - u(y - h * E[s])) / (2 * h)
        div = np.trace(J)
        curl = np.array([J[2, 1] - J[1, 2], J[0, 2] - J[2, 0], J[1, 0] - J[0, 1]])
        dn = J @ n
        T[:, beta] = 2 * MU * dn + LAM * n * div + MU * np.cross(n, curl)
    return T


@pytest.mark.parametrize("omega", [0.5, 5.6, 20.0])
def test_T_is_traction_of_U(orc, omega):
    ks, _ = kappas(omega)
    rng = np.random.default_rng(5)
    for x, y in rand_pairs(rng, 8, 0.05 / ks, 6.0 / ks):
        n = rng.standard_normal(3); n /= np.linalg.norm(n)
        r = np.linalg.norm(x - y)
        Tfd = traction_fd(orc, x, y, n, omega, 1e-4 * min(r, 1.0 / ks))
        T = orc.green_block(1, x, y, n, omega, LAM, MU, RHO)
        assert np.linalg.norm(T - Tfd) <= 1e-6 * np.linalg.norm(T)


def test_U_symmetries_exact(orc):
    rng = np.random.default_rng(6)
    for x, y in rand_pairs(rng, 20, 0.01, 5.0):
        U = orc.green_block(0, x, y, None, 5.6, LAM, MU, RHO)
        assert np.array_equal(U, U.T)
        assert np.array_equal(U, orc.green_block(0, y, x, None, 5.6, LAM, MU, RHO).T)


def test_planar_zero_pattern(orc):
    """Eq. FSplane: x_3 = y_3 and n = e_3 give the reducible zero pattern."""
    import json, os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "planar_pattern.json")))
    rng = np.random.default_rng(7)
    n = np.array([0.0, 0.0, 1.0])
    for _ in range(20):
        x = np.r_[rng.uniform(-1, 1, 2), 0.25]
        y = np.r_[rng.uniform(-1, 1, 2), 0.25]
        U = orc.green_block(0, x, y, None, 5.6, LAM, MU, RHO)
        T = orc.green_block(1, x, y, n, 5.6, LAM, MU, RHO)
        assert np.array_equal(U != 0, np.array(gold["U_nonzero"], bool))
        assert np.array_equal(T != 0, np.array(gold["T_nonzero"], bool))


def test_series_and_closed_branches_agree(orc):
    """The two evaluations of the radial functions coincide where both are accurate."""
    for q in [0.5, 0.3]:
        for a in np.linspace(0.1, 1.2, 23):
            s = orc.radial(a, q, "series")
            c = orc.radial(a, q, "closed")
            tol = 1e-15 / a**2 * 50 + 1e-15
            assert np.all(np.abs(s - c) <= tol * (1 + np.abs(s))), (a, np.abs(s - c))


def test_radial_static_values(orc):
    """a -> 0: A -> (1+q^2)/2, B -> (1-q^2)/2, aA' -> 0, aB' -> 0 (Kelvin)."""
    q = 0.5
    a = 1e-9
    v = orc.radial(a, q)
    assert abs(v[0] - (1 + q * q) / 2) < 2 * a
    assert abs(v[1] - (1 - q * q) / 2) < 2 * a
    assert abs(v[2]) < 2 * a and abs(v[3]) < 2 * a
