"""Pins of the appendix closed forms I_2^{mnq} (Appendix A)."""
import numpy as np
import pytest
from scipy import integrate

from oracle import closed_forms as C
from oracle import equilibrium as E
from oracle import gfunc as G
from oracle import quadrature as Q

POINTS = [("MJ", 1.1, 0.7, 0.31, -0.22), ("FD", 0.8, 1.6, -0.45, 0.12), ("BE", 1.3, 0.6, 0.05, 0.52)]


def _numeric_I2(stats, theta, z, ux, uy, nang=256):
    """Direct 2D integration of the definition: periodic trapezoid in phi (exponentially
    convergent), adaptive quadrature in p at every angle."""
    xi = {"MJ": 0.0, "FD": 1.0, "BE": -1.0}[stats]
    ga = 1.0 / np.sqrt(1 - ux * ux - uy * uy)
    phis = 2 * np.pi * np.arange(nang) / nang
    rad = np.zeros((nang, 6))
    for i, ph in enumerate(phis):
        a = ga * (1 - ux * np.cos(ph) - uy * np.sin(ph)) / theta
        for K in range(6):
            if xi == 0.0:
                fun = lambda p: p ** K * z * np.exp(-a * p)
            else:
                # exp(-a p) form: no overflow far out in p, where the integrand is zero
                fun = lambda p: p ** K * np.exp(-a * p) * z / (1.0 + xi * z * np.exp(-a * p))
            rad[i, K] = integrate.quad(fun, 0, np.inf, epsabs=0, epsrel=1e-13, limit=200)[0]
    out = {}
    for (m, n, q) in C.MONOMIALS:
        K = m + n + q
        out[(m, n, q)] = np.sum(rad[:, K] * np.cos(phis) ** n * np.sin(phis) ** q) * 2 * np.pi / nang
    return out


@pytest.mark.parametrize("stats,theta,z,ux,uy", POINTS)
def test_closed_forms_against_numerical_integration(stats, theta, z, ux, uy):
    g = G.g_all(stats, np.array(z))
    I = C.I2_all(theta, g, ux, uy)
    ref = _numeric_I2(stats, theta, z, ux, uy)
    for key in C.MONOMIALS:
        K = sum(key)
        scale = abs(I[(K, 0, 0)])  # same-degree energy-like moment sets the scale
        assert abs(I[key] - ref[key]) <= 1e-10 * scale, (key, I[key], ref[key])


@pytest.mark.parametrize("stats,theta,z,ux,uy", POINTS)
def test_cone_identities(stats, theta, z, ux, uy):
    """(p^0)^2 = (p^x)^2 + (p^y)^2 on the light cone: every monomial with a factor
    (p^0)^2 equals the sum of the two with (p^x)^2 and (p^y)^2 instead."""
    g = G.g_all(stats, np.array(z))
    I = C.I2_all(theta, g, ux, uy)
    n_checked = 0
    for (m, n, q) in C.MONOMIALS:
        if m >= 2:
            a, b = (m - 2, n + 2, q), (m - 2, n, q + 2)
            if a in I and b in I:
                assert abs(I[(m, n, q)] - I[a] - I[b]) <= 1e-13 * abs(I[(m + n + q, 0, 0)])
                n_checked += 1
    assert n_checked >= 20


@pytest.mark.parametrize("stats,theta,z,ux,uy", POINTS)
def test_lattice_equilibrium_reproduces_all_56(stats, theta, z, ux, uy):
    """Quadrature exactness of the equilibrium moments up to fifth order:
    sum_i f^eq_i phi(p_i) = I_2 for all 56 monomials of degree <= 5."""
    g = G.g_all(stats, np.array(z))
    feq = E.feq_lattice(stats, np.float64(theta), g, ux, uy)
    v = Q.vectors(stats)
    I = C.I2_all(theta, g, ux, uy)
    for (m, n, q) in C.MONOMIALS:
        s = np.sum(feq * v["p0"] ** m * v["px"] ** n * v["py"] ** q)
        scale = abs(I[(m + n + q, 0, 0)])
        assert abs(s - I[(m, n, q)]) <= 5e-13 * scale, ((m, n, q), s, I[(m, n, q)])


def test_degree_six_not_reproduced():
    stats, theta, z, ux, uy = POINTS[0][0], 1.1, 0.7, 0.31, -0.22
    g = G.g_all(stats, np.array(z))
    feq = E.feq_lattice(stats, np.float64(theta), g, ux, uy)
    v = Q.vectors(stats)
    # (p^0)^6 moment: exact value 6! g_7 theta^7 gamma^-7 int (1-u.v)^-7 dphi
    from scipy.special import factorial
    ga = 1 / np.sqrt(1 - ux * ux - uy * uy)
    ph = 2 * np.pi * np.arange(720) / 720
    ang = np.sum((1 - ux * np.cos(ph) - uy * np.sin(ph)) ** -7) * 2 * np.pi / 720
    exact = factorial(6) * z * theta ** 7 * ga ** -7 * ang
    s = np.sum(feq * v["p0"] ** 6)
    assert abs(s - exact) > 1e-6 * exact
