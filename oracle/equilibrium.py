"""N-th order expansion of the equilibrium (Sec. 2.3, Eqs. expansion-eq and
projections-eq) sampled on the d2v72 lattice.

Test infrastructure (see the package docstring): never used by the product path.

Reading.  The paper's relativistic polynomials P^{i_1..i_N} (N <= 5) and
P^{i_1..i_M 0} (M <= 4) are orthonormal in the inner product
<a, b> = int d^2p/p^0 omega(p) a b  (Eq. ortho-eq) and the expansion
f^eq ~ omega * sum A P with A = int d^2p/p^0 f^eq P is therefore the orthogonal
projection of f^eq/omega onto their span V_N.  V_N is the space of polynomials of
degree <= N in (p^0, p^x, p^y) restricted to the light cone p^0 = |p|; it has
dimension (N+1)^2 and the monomials (p^0)^m (p^x)^n (p^y)^q with q <= 1 and
m + n + q <= N form a basis of it.  The projection does not depend on which basis
spans V_N, so the oracle uses this monomial basis:

    f^eq/omega  ~  sum_a c_a phi_a,   G c = m,
    G_ab = <phi_a, phi_b>               (continuous integrals, mpmath, 50 digits),
    m_a  = int d^2p/p^0 f^eq phi_a      (the appendix closed forms I_2^{mnq}).

On the lattice the expansion is sampled as f^eq_i = w_i sum_a c_a phi_a(p_i), i.e.
f^eq = M m with the 72 x (N+1)^2 matrix M = W Phi G^{-1}, built once in mpmath and
rounded to FP64.  Because the quadrature integrates degree <= 10 exactly, the
discrete moments sum_i f^eq_i phi(p_i) of every phi in V_N equal the continuous
ones (Eq. quadrature-eq).
"""
from functools import lru_cache

import mpmath as mp
import numpy as np

from . import closed_forms, quadrature

DPS = 50


def basis(order=5):
    """Monomial exponents (m, n, q) spanning V_order: q <= 1, m + n + q <= order."""
    out = []
    for deg in range(order + 1):
        for q in (0, 1):
            for n in range(deg - q + 1):
                m = deg - q - n
                out.append((m, n, q))
    return out


@lru_cache(maxsize=None)
def gram(stats, order=5):
    """Gram matrix <phi_a, phi_b> (mpmath matrix) from the exact continuous integrals."""
    bs = basis(order)
    with mp.workdps(DPS):
        G = mp.matrix(len(bs), len(bs))
        for a, (ma, na, qa) in enumerate(bs):
            for b, (mb, nb, qb) in enumerate(bs):
                G[a, b] = quadrature.continuous_monomial_integral(stats, ma + mb, na + nb, qa + qb)
        return G


@lru_cache(maxsize=None)
def projector(stats, order=5):
    """FP64 matrix M (72 x dim) with f^eq_i = sum_a M_ia m_a."""
    bs = basis(order)
    nodes, lam = quadrature.radial_rule(stats)
    with mp.workdps(DPS):
        Ginv = gram(stats, order) ** -1
        cosd = [mp.mpf(1), mp.sqrt(3) / 2, mp.mpf(1) / 2, mp.mpf(0), -mp.mpf(1) / 2, -mp.sqrt(3) / 2,
                -mp.mpf(1), -mp.sqrt(3) / 2, -mp.mpf(1) / 2, mp.mpf(0), mp.mpf(1) / 2, mp.sqrt(3) / 2]
        sind = [cosd[(n - 3) % 12] for n in range(12)]
        M = np.zeros((quadrature.Q, len(bs)))
        for n in range(12):
            for k in range(6):
                p = nodes[k]
                w = lam[k] * 2 * mp.pi / 12
                phi = [p ** m * (p * cosd[n]) ** a * (p * sind[n]) ** b for (m, a, b) in bs]
                for col in range(len(bs)):
                    M[6 * n + k, col] = float(w * mp.fsum(phi[r] * Ginv[r, col] for r in range(len(bs))))
        return M


def moments(theta, g, ux, uy, order=5):
    """Array (dim, ...) of the basis moments m_a from the appendix closed forms."""
    I = closed_forms.I2_all(theta, g, ux, uy)
    return np.stack([np.broadcast_to(I[t], np.shape(theta)) for t in basis(order)])


def feq_lattice(stats, theta, g, ux, uy, order=5):
    """Discrete equilibrium f^eq_i, shape (72,) + shape(theta)."""
    theta = np.asarray(theta, dtype=np.float64)
    m = moments(theta, g, ux, uy, order)
    M = projector(stats, order)
    return np.tensordot(M, m, axes=(1, 0))


def weight_function(stats, p):
    """omega(p) of Eqs. mj-w-eq, fd-w-eq, be-w-eq."""
    p = np.asarray(p, dtype=np.float64)
    if stats == "MJ":
        return np.exp(-p) / (2 * np.pi)
    if stats == "FD":
        return 1.0 / (np.exp(p) + 1.0)
    if stats == "BE":
        return 1.0 / (np.exp(p) / quadrature.Z_C_BE.__float__() - 1.0)
    raise ValueError(stats)


def feq_exact(stats, px, py, theta, z, ux, uy):
    """Unexpanded equilibrium 1/(z^-1 exp[p.U/theta] + xi) at momentum (px, py)."""
    p = np.hypot(px, py)
    ga = 1.0 / np.sqrt(1.0 - ux * ux - uy * uy)
    arg = (p * ga - ga * (px * ux + py * uy)) / theta
    if stats == "MJ":
        return z * np.exp(-arg)
    xi = 1.0 if stats == "FD" else -1.0
    return 1.0 / (np.exp(arg) / z + xi)


def feq_expanded_at(stats, px, py, theta, g, ux, uy, order):
    """Continuous N-th order expansion omega(p) sum_a c_a phi_a(p) at momentum (px, py)."""
    bs = basis(order)
    with mp.workdps(DPS):
        Ginv = gram(stats, order) ** -1
        Gi = np.array([[float(Ginv[r, c]) for c in range(len(bs))] for r in range(len(bs))])
    m = moments(np.float64(theta), g, ux, uy, order)
    c = Gi @ m
    p0 = np.hypot(px, py)
    phi = np.array([p0 ** a * px ** b * py ** q for (a, b, q) in bs])
    return weight_function(stats, p0) * float(phi @ c)
