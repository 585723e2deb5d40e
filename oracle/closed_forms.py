"""Monomial integrals of the equilibrium (Appendix A, "Integrals used in the expansion").

Test infrastructure (see the package docstring): never used by the product path.

I_2^{mnq} = int d^2p/p^0 (p^0)^m (p^x)^n (p^y)^q f^eq,
f^eq = 1 / (z^-1 exp[p gamma (1 - v.u) / theta] + xi).

The table below restates the appendix's closed forms for all 56 monomials of
degree m + n + q <= 5.  Each is a polynomial in (u^x, u^y) times
theta^{K+1} g_{K+1}(z) gamma^K with K = m + n + q.  Arguments may be NumPy arrays
(vectorised over cells); ``g`` is the sequence [g_1, ..., g_6].
"""
import numpy as np

PI = np.pi


def _terms(th, g, ux, uy):
    u2 = ux * ux + uy * uy
    ga = 1.0 / np.sqrt(1.0 - u2)
    om = 1.0 - u2  # (1 - u^2)
    g1, g2, g3, g4, g5, g6 = g
    c1 = th * g1
    c2 = th ** 2 * g2 * ga
    c3 = th ** 3 * g3 * ga ** 2
    c4 = th ** 4 * g4 * ga ** 3
    c5 = th ** 5 * g5 * ga ** 4
    c6 = th ** 6 * g6 * ga ** 5
    x, y = ux, uy
    I = {}
    # degree 0..2
    I[(0, 0, 0)] = 2 * PI * c1
    I[(1, 0, 0)] = 2 * PI * c2
    I[(0, 1, 0)] = 2 * PI * c2 * x
    I[(0, 0, 1)] = 2 * PI * c2 * y
    I[(2, 0, 0)] = 2 * PI * c3 * (2 + u2)
    I[(0, 2, 0)] = 2 * PI * c3 * (om + 3 * x * x)
    I[(0, 0, 2)] = 2 * PI * c3 * (om + 3 * y * y)
    I[(1, 1, 0)] = 6 * PI * c3 * x
    I[(1, 0, 1)] = 6 * PI * c3 * y
    I[(0, 1, 1)] = 6 * PI * c3 * x * y
    # degree 3
    I[(3, 0, 0)] = 6 * PI * c4 * (2 + 3 * u2)
    I[(0, 3, 0)] = 6 * PI * c4 * (3 * om * x + 5 * x ** 3)
    I[(0, 0, 3)] = 6 * PI * c4 * (3 * om * y + 5 * y ** 3)
    I[(1, 2, 0)] = 6 * PI * c4 * (om + 5 * x * x)
    I[(1, 0, 2)] = 6 * PI * c4 * (om + 5 * y * y)
    I[(1, 1, 1)] = 6 * PI * c4 * (5 * x * y)
    I[(2, 0, 1)] = 6 * PI * c4 * (4 + u2) * y
    I[(2, 1, 0)] = 6 * PI * c4 * (4 + u2) * x
    I[(0, 2, 1)] = 6 * PI * c4 * (om + 5 * x * x) * y
    I[(0, 1, 2)] = 6 * PI * c4 * (om + 5 * y * y) * x
    # degree 4
    I[(4, 0, 0)] = 6 * PI * c5 * (8 + 24 * u2 + 3 * u2 ** 2)
    I[(0, 4, 0)] = 6 * PI * c5 * (3 + 3 * u2 ** 2 + 30 * x ** 2 + 35 * x ** 4 - 6 * u2 * (1 + 5 * x ** 2))
    I[(0, 0, 4)] = 6 * PI * c5 * (3 + 3 * u2 ** 2 + 30 * y ** 2 + 35 * y ** 4 - 6 * u2 * (1 + 5 * y ** 2))
    I[(2, 2, 0)] = 6 * PI * c5 * (4 - 3 * u2 - u2 ** 2 + 5 * x ** 2 * (6 + u2))
    I[(2, 0, 2)] = 6 * PI * c5 * (4 - 3 * u2 - u2 ** 2 + 5 * y ** 2 * (6 + u2))
    I[(0, 2, 2)] = 6 * PI * c5 * (om + 4 * om * u2 + 35 * x ** 2 * y ** 2)
    I[(0, 3, 1)] = 30 * PI * c5 * (3 * om + 7 * x ** 2) * x * y
    I[(0, 1, 3)] = 30 * PI * c5 * (3 * om + 7 * y ** 2) * x * y
    I[(2, 1, 1)] = 30 * PI * c5 * (6 + u2) * x * y
    I[(1, 3, 0)] = -30 * PI * c5 * x * (-3 + 3 * u2 - 7 * x ** 2)
    I[(1, 0, 3)] = -30 * PI * c5 * y * (-3 + 3 * u2 - 7 * y ** 2)
    I[(3, 1, 0)] = 30 * PI * c5 * (4 + 3 * u2) * x
    I[(3, 0, 1)] = 30 * PI * c5 * (4 + 3 * u2) * y
    I[(1, 2, 1)] = -30 * PI * c5 * (-1 + u2 - 7 * x ** 2) * y
    I[(1, 1, 2)] = -30 * PI * c5 * (-1 + u2 - 7 * y ** 2) * x
    # degree 5
    I[(5, 0, 0)] = 30 * PI * c6 * (8 + 40 * u2 + 15 * u2 ** 2)
    I[(0, 5, 0)] = 30 * PI * c6 * x * (15 * om ** 2 + 70 * x ** 2 * om + 63 * x ** 4)
    I[(0, 0, 5)] = 30 * PI * c6 * y * (15 * om ** 2 + 70 * y ** 2 * om + 63 * y ** 4)
    I[(2, 3, 0)] = 30 * PI * c6 * x * (18 - 3 * u2 ** 2 + 56 * x ** 2 + u2 * (-15 + 7 * x ** 2))
    I[(2, 0, 3)] = 30 * PI * c6 * y * (18 - 3 * u2 ** 2 + 56 * y ** 2 + u2 * (-15 + 7 * y ** 2))
    I[(0, 4, 1)] = 90 * PI * c6 * (om ** 2 + 14 * x ** 2 * om + 21 * x ** 4) * y
    I[(0, 1, 4)] = 90 * PI * c6 * (om ** 2 + 14 * y ** 2 * om + 21 * y ** 4) * x
    I[(2, 2, 1)] = -30 * PI * c6 * (-6 * om - u2 * om - 56 * x ** 2 + u2 * (-7 * x ** 2)) * y
    I[(2, 1, 2)] = -30 * PI * c6 * (-6 * om - u2 * om - 56 * y ** 2 + u2 * (-7 * y ** 2)) * x
    I[(0, 3, 2)] = -30 * PI * c6 * x * (x ** 2 * (-1 + 4 * u2 - 63 * y ** 2) + 3 * (-1 + (-5 + 6 * u2) * y ** 2))
    I[(0, 2, 3)] = -30 * PI * c6 * y * (y ** 2 * (-1 + 4 * u2 - 63 * x ** 2) + 3 * (-1 + (-5 + 6 * u2) * x ** 2))
    I[(4, 1, 0)] = 90 * PI * c6 * x * (8 + 12 * u2 + u2 ** 2)
    I[(4, 0, 1)] = 90 * PI * c6 * y * (8 + 12 * u2 + u2 ** 2)
    I[(1, 4, 0)] = 90 * PI * c6 * (om ** 2 + 14 * x ** 2 * om + 21 * x ** 4)
    I[(1, 0, 4)] = 90 * PI * c6 * (om ** 2 + 14 * y ** 2 * om + 21 * y ** 4)
    I[(3, 2, 0)] = -30 * PI * c6 * (-4 * om - 3 * u2 * om - 42 * x ** 2 + u2 * (-21 * x ** 2))
    I[(3, 0, 2)] = -30 * PI * c6 * (-4 * om - 3 * u2 * om - 42 * y ** 2 + u2 * (-21 * y ** 2))
    I[(1, 2, 2)] = -30 * PI * c6 * (-1 + u2 - 6 * u2 * om - 63 * x ** 2 * y ** 2)
    I[(1, 3, 1)] = -630 * PI * c6 * x * (-1 + u2 - 3 * x ** 2) * y
    I[(1, 1, 3)] = -630 * PI * c6 * y * (-1 + u2 - 3 * y ** 2) * x
    I[(3, 1, 1)] = 315 * PI * c6 * (2 + u2) * 2 * x * y
    return I


MONOMIALS = sorted(_terms(1.0, [1.0] * 6, 0.1, 0.2).keys(), key=lambda t: (sum(t), t))


def I2_all(theta, g, ux, uy):
    """Dict (m, n, q) -> I_2^{mnq} for all 56 monomials of degree <= 5."""
    return _terms(theta, g, ux, uy)


def I2(mnq, theta, g, ux, uy):
    return _terms(theta, g, ux, uy)[tuple(mnq)]
