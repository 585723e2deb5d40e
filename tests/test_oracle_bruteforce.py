"""The main oracle against the brute-force checker on tiny grids (different routes:
harmonic basis with numerically integrated moments, dense interpolation matrices,
library eigen-solver, mpmath root finding)."""
import numpy as np
import pytest

from oracle import bruteforce as B
from oracle import gfunc as G
from oracle import lattice as L


@pytest.mark.parametrize("stats,nx,ny,nsteps,bc", [
    ("MJ", 8, 8, 10, "periodic"),
    ("MJ", 8, 8, 6, "open"),
    ("FD", 4, 4, 3, "periodic"),
    ("BE", 4, 4, 3, "open"),
])
def test_oracle_matches_bruteforce(stats, nx, ny, nsteps, bc):
    bcd = dict(xlo=bc, xhi=bc, ylo=bc, yhi=bc)
    p = L.Params(stats=stats, nx=nx, ny=ny, tau=0.8, bc=bcd)
    rng = np.random.default_rng(17)
    th = 1 + 0.2 * rng.random((ny, nx))
    ux = 0.1 * rng.standard_normal((ny, nx))
    uy = 0.1 * rng.standard_normal((ny, nx))
    z = 0.3 + 0.5 * rng.random((ny, nx))
    f = L.init_state(p, th, ux, uy, z=z)
    fb = B.feq(stats, th, G.g_all(stats, z), ux, uy)
    np.testing.assert_allclose(fb, f, rtol=0, atol=3e-13 * np.abs(f).max())
    a, b = f.copy(), f.copy()
    for _ in range(nsteps):
        a, _ = L.step(a, p)
        b = B.step(b, stats, 0.8, bcd)
    # populations: per shell relative to that shell's largest value; the outermost
    # shell (weight 1e-7 of the first) carries the largest rounding
    for k, tol in zip(range(6), (1e-13, 1e-13, 1e-13, 5e-13, 2e-12, 2e-11)):
        sl = slice(k, 72, 6)
        scale = np.abs(a[sl]).max()
        assert np.abs(a[sl] - b[sl]).max() <= tol * scale, k
    fa, fbb = L.fields(a, p), L.fields(b, p)
    for key in ("n", "eps", "theta", "z", "ux", "uy"):
        assert np.abs(fa[key] - fbb[key]).max() <= 1e-12 * np.abs(fbb[key]).max(), key
    for key in ("qx", "qy"):
        assert np.abs(fa[key] - fbb[key]).max() <= 1e-11 * np.abs(fbb[key]).max(), key
