"""Generalised EDF integral g_nu(z) (Eq. gz-eq) and the inversions from the
macroscopic moments to (theta, z) (Eqs. theta-eq and n-eps-eq).

Test infrastructure (see the package docstring): never used by the product path.

g_nu(z) = Gamma(nu)^-1 int_0^inf x^{nu-1} / (z^-1 e^x + xi) dx, with xi = 0 (MJ),
+1 (FD), -1 (BE).  In closed form: MJ g_nu = z; FD g_nu = -Li_nu(-z);
BE g_nu = Li_nu(z).

Two evaluators:
* ``g_mp``   - mpmath's polylogarithm at 30 digits (the definition; slow);
* ``g_vec``  - FP64 NumPy, vectorised over cells, from three classical series of
  the polylogarithm in mu = ln z (coefficients eta(s), zeta(s) from mpmath):
    FD  mu <= -1 :  sum_k (-1)^{k+1} e^{k mu} / k^nu                (defining series)
        |mu| < 1 :  sum_k eta(nu-k) mu^k / k!                        (Taylor at z = 1)
        mu >= 1  :  sum_{j<=nu/2} 2 eta(2j) mu^{nu-2j}/(nu-2j)! - (-1)^nu g_nu(-mu)
                    (inversion formula of the polylogarithm for integer order)
    BE  mu <= -1 :  sum_k e^{k mu} / k^nu
        mu > -1  :  mu^{nu-1}/(nu-1)! (H_{nu-1} - ln(-mu)) + sum_{k != nu-1} zeta(nu-k) mu^k/k!
  ``g_vec`` is pinned against ``g_mp`` by the tests.

Reading for MJ: the paper writes the MJ distribution with z = 1 and a free
normalisation A.  Here A is carried by z, f^eq = z exp(-p.U/theta), so that
g_nu(z) = z for every nu and n, theta vary independently.

Inversion (n, eps) -> (theta, z): r = 2 n^3/(pi eps^2) equals h(z) = g_2^3/g_3^2
(theta cancels in Eq. n-eps-eq); h increases with z, so its root is found by
bisection on s = ln z to the last bit; then theta = (1/2)(g_2/g_3)(eps/n)
(Eq. theta-eq).
"""
from functools import lru_cache

import mpmath as mp
import numpy as np

DPS = 30
Z_C_BE = 1.0 - 1e-7
LOG_ZC_BE = float(mp.log(mp.mpf(1) - mp.mpf(10) ** -7))
NTERM_DIRECT = 64
NTERM_TAYLOR = 48


def g_mp(stats, nu, z):
    """g_nu(z) as an mpmath number (definition through the polylogarithm)."""
    with mp.workdps(DPS):
        z = mp.mpf(z)
        if stats == "MJ":
            return z
        if stats == "FD":
            return -mp.polylog(nu, -z)
        if stats == "BE":
            return mp.polylog(nu, z)
    raise ValueError(stats)


@lru_cache(maxsize=None)
def _coef(kind, nu):
    with mp.workdps(40):
        k = np.arange(NTERM_TAYLOR)
        if kind == "eta":
            return np.array([float(mp.altzeta(nu - int(j)) / mp.factorial(int(j))) for j in k])
        # zeta(nu - k)/k!, with the k = nu - 1 pole term removed
        out = []
        for j in k:
            j = int(j)
            out.append(0.0 if j == nu - 1 else float(mp.zeta(nu - j) / mp.factorial(j)))
        return np.array(out)


@lru_cache(maxsize=None)
def _harmonic(m):
    return float(sum(mp.mpf(1) / j for j in range(1, m + 1)))


def _poly(c, x):
    acc = np.zeros_like(x)
    for cj in c[::-1]:
        acc = acc * x + cj
    return acc


def _fd(nu, mu):
    mu = np.asarray(mu, dtype=np.float64)
    out = np.empty_like(mu)
    k = np.arange(1, NTERM_DIRECT + 1)
    lo, mid, hi = mu <= -1.0, np.abs(mu) < 1.0, mu >= 1.0
    if lo.any():
        e = np.exp(np.multiply.outer(mu[lo], k))
        out[lo] = (e * ((-1.0) ** (k + 1) / k ** float(nu))).sum(-1)
    if mid.any():
        out[mid] = _poly(_coef("eta", nu), mu[mid])
    if hi.any():
        m = mu[hi]
        with mp.workdps(30):
            poly = sum(2 * float(mp.altzeta(2 * j)) * m ** (nu - 2 * j) / float(mp.factorial(nu - 2 * j))
                       for j in range(nu // 2 + 1))
        out[hi] = poly - (-1) ** nu * _fd(nu, -m)
    return out


def _be(nu, mu):
    mu = np.asarray(mu, dtype=np.float64)
    out = np.empty_like(mu)
    k = np.arange(1, NTERM_DIRECT + 1)
    lo = mu <= -1.0
    hi = ~lo
    if lo.any():
        e = np.exp(np.multiply.outer(mu[lo], k))
        out[lo] = (e / k ** float(nu)).sum(-1)
    if hi.any():
        m = mu[hi]
        if np.any(m >= 0):
            raise ValueError("BE needs z < 1")
        sing = m ** (nu - 1) / float(mp.factorial(nu - 1)) * (_harmonic(nu - 1) - np.log(-m))
        out[hi] = sing + _poly(_coef("zeta", nu), m)
    return out


def g_vec(stats, nu, z):
    """g_nu(z) in FP64, vectorised (see module docstring)."""
    z = np.asarray(z, dtype=np.float64)
    if stats == "MJ":
        return z.copy()
    mu = np.log(z)
    if stats == "FD":
        return _fd(nu, mu)
    if stats == "BE":
        return _be(nu, mu)
    raise ValueError(stats)


def g_all(stats, z, nmax=6):
    """Array (nmax, ...) of g_1(z) .. g_nmax(z)."""
    return np.stack([g_vec(stats, nu, z) for nu in range(1, nmax + 1)])


def h(stats, z):
    return g_vec(stats, 2, z) ** 3 / g_vec(stats, 3, z) ** 2


def h_max_be():
    """h at the reference fugacity z_c = 1 - 1e-7 of the BE weight: the largest r
    that has a root below z_c."""
    return float(h("BE", np.array(Z_C_BE)))


def _bisect(fun, target, lo, hi, iters=200):
    """Bisection on s for an increasing fun(s) = target, elementwise, to the last bit."""
    lo = np.array(lo, dtype=np.float64)
    hi = np.array(hi, dtype=np.float64)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        done = (mid == lo) | (mid == hi)
        if done.all():
            break
        up = fun(mid) < target
        lo = np.where(up & ~done, mid, lo)
        hi = np.where(~up & ~done, mid, hi)
    flo, fhi = fun(lo), fun(hi)
    return np.where(np.abs(flo - target) <= np.abs(fhi - target), lo, hi)


def _bracket(stats):
    if stats == "FD":
        return -40.0, 40.0
    return -40.0, LOG_ZC_BE


def invert_n_eps(stats, n, eps):
    """(n, eps) -> (theta, z, ok), elementwise.  BE states with r >= h(z_c) have no
    root below the reference fugacity: z is clamped to z_c and ok is False."""
    n = np.asarray(n, dtype=np.float64)
    eps = np.asarray(eps, dtype=np.float64)
    ok = (n > 0) & (eps > 0)
    ns, es = np.where(ok, n, 1.0), np.where(ok, eps, 1.0)
    r = 2.0 * ns ** 3 / (np.pi * es ** 2)
    if stats == "MJ":
        return es / (2.0 * ns), r, ok
    lo, hi = _bracket(stats)
    if stats == "BE":
        over = r >= h_max_be()
        ok = ok & ~over
        r = np.where(over, h_max_be(), r)
    s = _bisect(lambda s: h(stats, np.exp(s)), r, np.full_like(r, lo), np.full_like(r, hi))
    z = np.exp(s)
    theta = 0.5 * g_vec(stats, 2, z) / g_vec(stats, 3, z) * es / ns
    return theta, z, ok


def z_from_n_theta(stats, n, theta):
    """Fugacity from (n, theta) through n = 2 pi theta^2 g_2(z) (Eq. n-eps-eq)."""
    n = np.asarray(n, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    target = n / (2.0 * np.pi * theta ** 2)
    if stats == "MJ":
        return target
    lo, hi = _bracket(stats)
    if stats == "BE" and np.any(target >= float(g_vec("BE", 2, np.array(Z_C_BE)))):
        raise ValueError("BE density above the condensation bound")
    s = _bisect(lambda s: g_vec(stats, 2, np.exp(s)), target, np.full_like(target, lo),
                np.full_like(target, hi))
    return np.exp(s)


def n_from_z_theta(stats, z, theta):
    """n = 2 pi theta^2 g_2(z) (Eq. n-eps-eq)."""
    return 2.0 * np.pi * np.asarray(theta) ** 2 * g_vec(stats, 2, z)
