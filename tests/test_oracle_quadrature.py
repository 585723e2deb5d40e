"""Pins of the oracle's d2v72 quadrature (Sec. 2.4, Eq. quadrature-eq)."""
import mpmath as mp
import numpy as np
import pytest

from conftest import read_golden
from oracle import quadrature as Q


@pytest.mark.parametrize("stats,fname", [("MJ", "quadrature_mj.txt"), ("BE", "quadrature_be.txt")])
def test_printed_nodes_and_weights(stats, fname):
    p, w = Q.lattice(stats)
    for k, ps, ws in read_golden(fname):
        k = int(k) - 1
        # printed to 6-7 significant figures, some truncated rather than rounded
        # (BE w_2 = 0.55102865.. is printed 5.510286e-1): one unit in the last place
        dp = 1.0 * 10.0 ** -(len(ps.split(".")[1]))
        assert abs(p[k] - float(ps)) <= dp * 1.0001, (k, p[k], ps)
        mant, _, ex = ws.partition("e")
        dw = 1.0 * 10.0 ** (-(len(mant.split(".")[1])) + (int(ex) if ex else 0))
        assert abs(w[k] - float(ws)) <= dw * 1.0001, (k, w[k], ws)


def test_mj_is_gauss_laguerre():
    # e^-p/2pi weight: nodes are the Gauss-Laguerre nodes, per-vector weight = lambda/12
    x, lam = np.polynomial.laguerre.laggauss(6)
    p, w = Q.lattice("MJ")
    np.testing.assert_allclose(p, x, rtol=1e-13)
    np.testing.assert_allclose(w, lam / 12.0, rtol=1e-12)


def test_fd_weight_sum():
    # sum of per-vector weights over one direction = (2pi/12) int omega = (pi/6) ln 2
    _, w = Q.lattice("FD")
    assert abs(w.sum() - np.pi / 6 * np.log(2.0)) < 1e-14


@pytest.mark.parametrize("stats", Q.STATS)
def test_exact_up_to_degree_10(stats):
    """sum_i w_i (p^0)^m (p^x)^a (p^y)^b = int d^2p/p^0 omega (..) for m+a+b <= 10."""
    v = Q.vectors(stats)
    for deg in range(11):
        for a in range(deg + 1):
            for b in range(deg - a + 1):
                m = deg - a - b
                s = np.sum(v["w"] * v["p0"] ** m * v["px"] ** a * v["py"] ** b)
                ref = float(Q.continuous_monomial_integral(stats, m, a, b))
                scale = float(Q.continuous_monomial_integral(stats, deg, 0, 0))
                assert abs(s - ref) <= 1e-13 * scale, (stats, m, a, b, s, ref)


def test_not_exact_at_degree_12():
    # the rule has a limit: the 12-direction angular sum fails for cos^12
    v = Q.vectors("MJ")
    s = np.sum(v["w"] * v["px"] ** 12)
    ref = float(Q.continuous_monomial_integral("MJ", 0, 12, 0))
    assert abs(s - ref) > 1e-6 * abs(ref)


def test_directions_are_exact():
    assert Q.COS_DIR[3] == 0.0 and Q.SIN_DIR[0] == 0.0 and Q.COS_DIR[9] == 0.0
    np.testing.assert_allclose(Q.COS_DIR ** 2 + Q.SIN_DIR ** 2, 1.0, rtol=0, atol=2e-16)
    with mp.workdps(30):
        for n in range(12):
            assert abs(Q.COS_DIR[n] - float(mp.cos(mp.pi * n / 6))) < 1e-16
            assert abs(Q.SIN_DIR[n] - float(mp.sin(mp.pi * n / 6))) < 1e-16


@pytest.mark.parametrize("stats", Q.STATS)
def test_radial_moments_by_direct_integration(stats):
    """mu_k = int_0^inf omega(p) p^k dp for k = 0..12 (the moments the radial rule is
    built from) against direct numerical integration of the weight functions of
    Eqs. mj-w-eq, fd-w-eq and be-w-eq, not through their closed forms (factorials,
    the eta function, the polylogarithm)."""
    zc = Q.Z_C_BE
    with mp.workdps(40):
        weight = {"MJ": lambda p: mp.exp(-p) / (2 * mp.pi),
                  "FD": lambda p: 1 / (mp.exp(p) + 1),
                  "BE": lambda p: 1 / (mp.exp(p) / zc - 1)}[stats]
        # the BE weight peaks like 1/(p + 1e-7) at the origin: split the range there
        pts = [0, mp.mpf(10) ** -9, mp.mpf(10) ** -7, mp.mpf(10) ** -5, mp.mpf(10) ** -3, mp.mpf("0.1"), 1, 4, 10,
               25, 60, 150, mp.inf]
        for k in range(13):
            direct = mp.quad(lambda p: weight(p) * p ** k, pts)
            mu = Q.radial_moment(stats, k)
            assert abs(mu / direct - 1) < mp.mpf(10) ** -20, (stats, k, mu, direct)
