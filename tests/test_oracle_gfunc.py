"""Pins of g_nu(z) (Eq. gz-eq) and of the (n, eps) -> (theta, z) inversion
(Eqs. theta-eq, n-eps-eq)."""
import mpmath as mp
import numpy as np
import pytest

from oracle import gfunc as G


@pytest.mark.parametrize("stats", ["FD", "BE"])
def test_series_against_mpmath_polylog(stats):
    hi = 7.0 if stats == "FD" else G.LOG_ZC_BE
    zs = np.exp(np.linspace(-7.0, hi, 57))
    for nu in range(1, 7):
        a = G.g_vec(stats, nu, zs)
        b = np.array([float(G.g_mp(stats, nu, z)) for z in zs])
        np.testing.assert_allclose(a, b, rtol=2e-15)


def test_definition_by_quadrature():
    # g_nu(z) = Gamma(nu)^-1 int x^{nu-1}/(z^-1 e^x + xi) dx, directly
    with mp.workdps(25):
        for stats, xi in (("FD", 1), ("BE", -1)):
            for z in (0.3, 0.8):
                for nu in (1, 3, 6):
                    ref = mp.quad(lambda x: x ** (nu - 1) / (mp.exp(x) / z + xi), [0, 5, 20, mp.inf]) / mp.gamma(nu)
                    assert abs(G.g_vec(stats, nu, np.array(z)) - float(ref)) <= 2e-15 * float(ref)


def test_special_values():
    # FD at z = 1: g_nu(1) = eta(nu) = (1 - 2^{1-nu}) zeta(nu); g_1(1) = ln 2
    assert abs(G.g_vec("FD", 1, np.array(1.0)) - np.log(2.0)) < 1e-15
    for nu in range(2, 7):
        ref = (1 - 2.0 ** (1 - nu)) * float(mp.zeta(nu))
        assert abs(G.g_vec("FD", nu, np.array(1.0)) - ref) < 2e-15 * ref
    # MJ: g_nu(z) = z (with z carrying the normalisation)
    assert G.g_vec("MJ", 4, np.array(0.37)) == 0.37
    # BE: g_1(z) = -ln(1 - z)
    assert abs(G.g_vec("BE", 1, np.array(0.6)) + np.log(0.4)) < 2e-15
    # BE limit h -> zeta(2)^3/zeta(3)^2 as z -> 1
    lim = float(mp.zeta(2) ** 3 / mp.zeta(3) ** 2)
    assert 0 < lim - G.h_max_be() < 2e-3


@pytest.mark.parametrize("stats", ["MJ", "FD", "BE"])
def test_inversion_round_trip(stats):
    rng = np.random.default_rng(11)
    theta = 0.5 + rng.random(200)
    z = 0.05 + (0.9 if stats == "BE" else 3.0) * rng.random(200)
    if stats == "MJ":
        g2 = g3 = z
    else:
        g2, g3 = G.g_vec(stats, 2, z), G.g_vec(stats, 3, z)
    n = 2 * np.pi * theta ** 2 * g2
    eps = 4 * np.pi * theta ** 3 * g3
    th, zz, ok = G.invert_n_eps(stats, n, eps)
    assert ok.all()
    np.testing.assert_allclose(th, theta, rtol=4e-15)
    np.testing.assert_allclose(zz, z, rtol=2e-14)
    # n -> z at given theta
    np.testing.assert_allclose(G.z_from_n_theta(stats, n, theta), z, rtol=2e-14)


def test_h_increasing():
    for stats, hi in (("FD", 8.0), ("BE", G.LOG_ZC_BE)):
        s = np.linspace(-8, hi, 400)
        hv = G.h(stats, np.exp(s))
        assert np.all(np.diff(hv) > 0)


def test_be_beyond_condensation_flagged():
    n = np.array([1.0])
    # r = 2 n^3/(pi eps^2) above h(z_c) -> clamp and flag
    eps = np.sqrt(2 * n ** 3 / (np.pi * (G.h_max_be() * 1.01)))
    th, z, ok = G.invert_n_eps("BE", n, eps)
    assert not ok[0] and abs(z[0] - G.Z_C_BE) < 1e-12
