"""d2v72 Gaussian quadrature (Sec. 2.4 "Gaussian Quadrature", Eq. quadrature-eq).

Test infrastructure (see the package docstring): never used by the product path.

The quadrature must reproduce  int d^2p/p^0 omega(p) p^{mu_1}..p^{mu_N}  for N <= 10.
With p^0 = |p| the measure d^2p/p^0 is dp dphi, so the rule separates into

* an angular part: the 12 roots phi_n = n pi/6 of sin(6 phi), each with weight
  2 pi / 12 (the 12-point rule integrates trigonometric polynomials of degree
  <= 11 exactly);
* a radial part: the 6 roots of R_6, the degree-6 orthogonal polynomial for the
  weight omega(p) on [0, inf), obtained by Gram-Schmidt on the monomials, with
  weights lambda_k fixed by the moment equations  sum_k lambda_k p_k^m = mu_m.

The per-vector weight is w_k = lambda_k * 2 pi / 12.  Vector index q = 6 n + k
(direction n = 0..11, shell k = 0..5); the paper's direction label is i = n + 1.
"""
from functools import lru_cache

import mpmath as mp
import numpy as np

DPS = 50
STATS = ("MJ", "FD", "BE")
Z_C_BE = mp.mpf(1) - mp.mpf(10) ** -7      # reference fugacity of the BE weight (Eq. be-w-eq)

# cos and sin of n pi / 6, written out exactly so that the axis directions stay
# pure shifts (a library cos(3 pi/6) is 6e-17, not 0).
_S3 = np.sqrt(3.0) / 2.0
COS_DIR = np.array([1.0, _S3, 0.5, 0.0, -0.5, -_S3, -1.0, -_S3, -0.5, 0.0, 0.5, _S3])
SIN_DIR = np.array([0.0, 0.5, _S3, 1.0, _S3, 0.5, 0.0, -0.5, -_S3, -1.0, -_S3, -0.5])
NDIR, NSHELL, Q = 12, 6, 72


def radial_moment(stats, k):
    """mu_k = int_0^inf omega(p) p^k dp for the weight functions of
    Eqs. mj-w-eq (e^-p / 2pi), fd-w-eq (1/(e^p+1)) and be-w-eq (1/(z_c^-1 e^p - 1))."""
    with mp.workdps(DPS):
        k = int(k)
        if stats == "MJ":
            return mp.factorial(k) / (2 * mp.pi)
        if stats == "FD":
            # int p^k/(e^p+1) = k! eta(k+1), eta the Dirichlet eta function (eta(1) = ln 2)
            return mp.factorial(k) * mp.altzeta(k + 1)
        if stats == "BE":
            # int p^k/(z^-1 e^p - 1) = k! Li_{k+1}(z)
            return mp.factorial(k) * mp.polylog(k + 1, Z_C_BE)
    raise ValueError(stats)


@lru_cache(maxsize=None)
def radial_rule(stats):
    """(p_k, lambda_k) for k = 1..6 as mpmath numbers: roots of R_6 and the weights
    solving the moment equations for m = 0..5."""
    with mp.workdps(DPS):
        mu = [radial_moment(stats, k) for k in range(13)]

        def inner(a, b):  # <a, b> = int omega a b dp for coefficient lists (ascending powers)
            return mp.fsum(ai * bj * mu[i + j] for i, ai in enumerate(a) for j, bj in enumerate(b))

        basis = []
        for d in range(7):  # Gram-Schmidt on 1, p, ..., p^6 -> monic orthogonal polynomials
            poly = [mp.mpf(0)] * d + [mp.mpf(1)]
            for prev in basis:
                c = inner(poly, prev) / inner(prev, prev)
                poly = [poly[i] - c * (prev[i] if i < len(prev) else 0) for i in range(len(poly))]
            basis.append(poly)
        r6 = basis[6]
        roots = mp.polyroots(list(reversed(r6)), maxsteps=400, extraprec=400)
        nodes = sorted(mp.re(r) for r in roots)
        vand = mp.matrix([[p ** m for p in nodes] for m in range(6)])
        lam = mp.lu_solve(vand, mp.matrix(mu[:6]))
        return nodes, [lam[i] for i in range(6)]


@lru_cache(maxsize=None)
def lattice(stats):
    """Float64 arrays (p_shell[6], w_shell[6]): radial nodes and per-vector weights."""
    nodes, lam = radial_rule(stats)
    with mp.workdps(DPS):
        w = [l * 2 * mp.pi / 12 for l in lam]
    return np.array([float(p) for p in nodes]), np.array([float(x) for x in w])


def vectors(stats):
    """Per-vector arrays over q = 6 n + k: p0 (=|p|), px, py, w, and the unit
    velocity (vx, vy) = (cos, sin) of the direction."""
    p, w = lattice(stats)
    n = np.repeat(np.arange(NDIR), NSHELL)
    k = np.tile(np.arange(NSHELL), NDIR)
    p0 = p[k]
    vx, vy = COS_DIR[n], SIN_DIR[n]
    return dict(p0=p0, px=p0 * vx, py=p0 * vy, w=w[k], vx=vx, vy=vy, n=n, k=k)


def angular_integral(a, b):
    """int_0^{2pi} cos^a(phi) sin^b(phi) dphi, exactly (mpmath): 2 B((a+1)/2, (b+1)/2)
    when a and b are both even, else 0."""
    if a % 2 or b % 2:
        return mp.mpf(0)
    with mp.workdps(DPS):
        return 2 * mp.beta(mp.mpf(a + 1) / 2, mp.mpf(b + 1) / 2)


def continuous_monomial_integral(stats, m, a, b):
    """int d^2p/p^0 omega(p) (p^0)^m (p^x)^a (p^y)^b = mu_{m+a+b} * int cos^a sin^b dphi."""
    with mp.workdps(DPS):
        return radial_moment(stats, m + a + b) * angular_integral(a, b)
