"""Second, slower checker for tiny grids, built from routes other than the main
oracle's, used only to pin the main oracle (tests/test_oracle_bruteforce.py).

Test infrastructure (see the package docstring): never used by the product path.

Differences from ``oracle.lattice``:
* equilibrium: the projection onto V_5 in the harmonic basis p^k cos(j phi),
  p^k sin(j phi) (0 <= j <= k <= 5) instead of monomials, with the moments taken
  from the general one-dimensional form of the appendix,
      int dp dphi p^k T(phi) f^eq = k! g_{k+1}(z) theta^{k+1} gamma^{-(k+1)}
                                    int T(phi) (1 - u.v(phi))^{-(k+1)} dphi,
  whose angular integral is done numerically (periodic trapezoid rule, 720
  points, exponentially convergent for |u| < 1), not the closed-form list;
  the Gram matrix comes from the lattice sums and is inverted in mpmath;
* streaming: a dense interpolation matrix per direction assembled cell by cell;
* Landau frame: numpy.linalg.eig of T^alpha_beta, the eigenvector with the
  largest eigenvalue normalised to V^0 = 1;
* inversion: mpmath.findroot on z itself with the mpmath polylogarithm.
"""
from functools import lru_cache

import mpmath as mp
import numpy as np

from . import gfunc, quadrature

NANG = 720


def _harm_basis(order=5):
    return [(k, j, c) for k in range(order + 1) for j in range(k + 1) for c in ((0,) if j == 0 else (0, 1))]


@lru_cache(maxsize=None)
def _synth(stats, order=5):
    """72 x dim matrix S with f^eq_i = sum_b S_ib b_b (b: harmonic moments)."""
    nodes, lam = quadrature.radial_rule(stats)
    bs = _harm_basis(order)
    with mp.workdps(50):
        phis = [mp.pi * n / 6 for n in range(12)]
        rows = []
        wts = []
        for n in range(12):
            for k in range(6):
                p = nodes[k]
                rows.append([p ** kk * (mp.cos(j * phis[n]) if c == 0 else mp.sin(j * phis[n])) for (kk, j, c) in bs])
                wts.append(lam[k] * 2 * mp.pi / 12)
        Phi = mp.matrix(rows)
        W = mp.diag(wts)
        G = Phi.T * W * Phi
        S = W * Phi * G ** -1
        return np.array([[float(S[i, j]) for j in range(len(bs))] for i in range(72)])


def harmonic_moments(theta, g, ux, uy, order=5):
    """b = int dp dphi p^k T_jc(phi) f^eq, numerically in phi; arrays broadcast over cells."""
    phi = 2 * np.pi * np.arange(NANG) / NANG
    ux = np.asarray(ux, dtype=np.float64)[..., None]
    uy = np.asarray(uy, dtype=np.float64)[..., None]
    th = np.asarray(theta, dtype=np.float64)
    ga = 1.0 / np.sqrt(1.0 - ux * ux - uy * uy)
    den = 1.0 - ux * np.cos(phi) - uy * np.sin(phi)
    out = []
    for (k, j, c) in _harm_basis(order):
        trig = np.cos(j * phi) if c == 0 else np.sin(j * phi)
        ang = (trig * den ** (-(k + 1))).sum(-1) * (2 * np.pi / NANG)
        out.append(float(mp.factorial(k)) * g[k] * th ** (k + 1) * ga[..., 0] ** (-(k + 1)) * ang)
    return np.stack(out)


def feq(stats, theta, g, ux, uy):
    return np.tensordot(_synth(stats), harmonic_moments(theta, g, ux, uy), axes=(1, 0))


def _axis_src(i, d, L, lo, hi):
    s = i - d
    if s < 0:
        return s + L if lo == "periodic" else 0
    if s >= L:
        return s - L if hi == "periodic" else L - 1
    return s


@lru_cache(maxsize=None)
def _stream_mats(nx, ny, bc_key):
    bc = dict(bc_key)
    mats = []
    N = nx * ny
    for n in range(12):
        cx, cy = quadrature.COS_DIR[n], quadrature.SIN_DIR[n]
        sx, sy = int(np.sign(cx)), int(np.sign(cy))
        ax, ay = abs(cx), abs(cy)
        S = np.zeros((N, N))
        for y in range(ny):
            for x in range(nx):
                xb = _axis_src(x, sx, nx, bc["xlo"], bc["xhi"])
                yb = _axis_src(y, sy, ny, bc["ylo"], bc["yhi"])
                dst = y * nx + x
                for (xx, yy, wgt) in ((xb, yb, ax * ay), (x, yb, (1 - ax) * ay),
                                      (xb, y, ax * (1 - ay)), (x, y, (1 - ax) * (1 - ay))):
                    S[dst, yy * nx + xx] += wgt
        mats.append(S)
    return mats


def stream(fstar, bc):
    ny, nx = fstar.shape[1:]
    mats = _stream_mats(nx, ny, tuple(sorted(bc.items())))
    out = np.empty_like(fstar)
    for q in range(72):
        out[q] = (mats[q // 6] @ fstar[q].reshape(-1)).reshape(ny, nx)
    return out


def landau_eig(T):
    """eps, ux, uy per cell from numpy.linalg.eig of T^alpha_beta."""
    shp = T.shape[2:]
    eps, ux, uy = np.empty(shp), np.empty(shp), np.empty(shp)
    for idx in np.ndindex(shp):
        A = T[(slice(None), slice(None)) + idx].copy()
        A[:, 1:] *= -1.0
        lam, vec = np.linalg.eig(A)
        i = int(np.argmax(lam.real))
        v = vec[:, i].real
        v = v / v[0]
        eps[idx], ux[idx], uy[idx] = lam[i].real, v[1], v[2]
    return eps, ux, uy


def _invert(stats, n, eps):
    r = 2.0 * n ** 3 / (np.pi * eps ** 2)
    if stats == "MJ":
        return eps / (2 * n), r
    with mp.workdps(30):
        hz = lambda z: gfunc.g_mp(stats, 2, z) ** 3 / gfunc.g_mp(stats, 3, z) ** 2 - r
        z = mp.findroot(hz, (mp.mpf("0.001"), mp.mpf("0.999999") if stats == "BE" else mp.mpf(50)),
                        solver="bisect" if False else "anderson")
        theta = 0.5 * gfunc.g_mp(stats, 2, z) / gfunc.g_mp(stats, 3, z) * eps / n
        return float(theta), float(z)


def step(fstar, stats, tau, bc):
    """One periodic/open step with constant tau (no walls)."""
    v = quadrature.vectors(stats)
    f = stream(fstar, bc)
    pmu = np.stack([v["p0"], v["px"], v["py"]])
    N = np.tensordot(pmu, f, axes=(1, 0))
    T = np.einsum("aq,bq,qyx->abyx", pmu, pmu, f)
    eps, ux, uy = landau_eig(T)
    ga = 1.0 / np.sqrt(1.0 - ux ** 2 - uy ** 2)
    n = ga * (N[0] - ux * N[1] - uy * N[2])
    theta, z = np.empty_like(n), np.empty_like(n)
    for idx in np.ndindex(n.shape):
        theta[idx], z[idx] = _invert(stats, n[idx], eps[idx])
    if stats == "MJ":
        g = np.broadcast_to(z, (6,) + z.shape)
    else:
        g = np.empty((6,) + z.shape)
        for idx in np.ndindex(z.shape):
            for nu in range(1, 7):
                g[(nu - 1,) + idx] = float(gfunc.g_mp(stats, nu, z[idx]))
    fe = feq(stats, theta, g, ux, uy)
    vu = v["vx"][:, None, None] * ux + v["vy"][:, None, None] * uy
    return f - ga * (1.0 - vu) / tau * (f - fe)
