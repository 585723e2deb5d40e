"""Invariants of the oracle's time step (Sec. 2.1 discrete equation, Sec. 2.4 streaming,
Eqs. eigen-eq, density-eq, conserv-eq)."""
import numpy as np
import pytest

from oracle import gfunc as G
from oracle import lattice as L
from oracle import quadrature as Q


def _random_state(stats, nx, ny, seed, amp=0.1):
    rng = np.random.default_rng(seed)
    p = L.Params(stats=stats, nx=nx, ny=ny, tau=0.9)
    th = 1 + amp * rng.random((ny, nx))
    ux = amp * rng.standard_normal((ny, nx))
    uy = amp * rng.standard_normal((ny, nx))
    z = 0.3 + 0.4 * rng.random((ny, nx))
    return p, L.init_state(p, th, ux, uy, z=z), (th, ux, uy, z)


@pytest.mark.parametrize("stats", Q.STATS)
def test_round_trip(stats):
    p, f, (th, ux, uy, z) = _random_state(stats, 7, 5, 1)
    mac = L.macroscopic(f, p)
    np.testing.assert_allclose(mac["theta"], th, rtol=1e-13)
    np.testing.assert_allclose(mac["z"], z, rtol=1e-12)
    np.testing.assert_allclose(mac["ux"], ux, atol=1e-14)
    np.testing.assert_allclose(mac["uy"], uy, atol=1e-14)
    n = G.n_from_z_theta(stats, z, th)
    np.testing.assert_allclose(mac["n"], n, rtol=1e-13)


@pytest.mark.parametrize("stats", Q.STATS)
def test_collision_conserves_N0_and_T0nu(stats):
    p, f0, _ = _random_state(stats, 9, 6, 2, amp=0.2)
    f = L.stream(f0, p)   # non-equilibrium populations
    mac = L.macroscopic(f, p)
    feq = L.equilibrium_state(p, mac["theta"], mac["g"], mac["ux"], mac["uy"])
    out = L.collide(f, feq, mac, L.relaxation_time(mac["theta"], p), stats)
    N0, T0 = L.moments(f, stats)
    N1, T1 = L.moments(out, stats)
    # AW conserves p_mu U^mu weighted moments; per cell the conserved ones are
    # U_mu N^mu ... the collision term integrates to zero against p^0 and p^0 p^nu
    d = out - f
    v = Q.vectors(stats)
    for wvec in (v["p0"], v["p0"] * v["p0"], v["p0"] * v["px"], v["p0"] * v["py"]):
        s = np.tensordot(wvec, d, axes=(0, 0))
        scale = np.tensordot(np.abs(wvec), np.abs(f), axes=(0, 0))
        assert np.max(np.abs(s) / scale) < 5e-14


def test_traceless():
    p, f, _ = _random_state("MJ", 6, 4, 3)
    _, T = L.moments(f, "MJ")
    tr = T[0, 0] - T[1, 1] - T[2, 2]
    assert np.max(np.abs(tr) / T[0, 0]) < 1e-14


def test_landau_against_eig():
    p, f0, _ = _random_state("FD", 5, 4, 4, amp=0.3)
    f = L.stream(f0, p)
    _, T = L.moments(f, "FD")
    eps, ux, uy, _ = L.landau(T)
    for idx in np.ndindex(eps.shape):
        A = T[(slice(None), slice(None)) + idx].copy()
        A[:, 1:] *= -1
        lam, vec = np.linalg.eig(A)
        i = np.argmax(lam.real)
        vv = vec[:, i].real / vec[0, i].real
        assert abs(lam[i].real - eps[idx]) < 1e-13 * eps[idx]
        assert abs(vv[1] - ux[idx]) < 1e-13 and abs(vv[2] - uy[idx]) < 1e-13


def test_streaming_conserves_each_population_periodic():
    p, f, _ = _random_state("BE", 8, 6, 5)
    s = L.stream(f, p)
    np.testing.assert_allclose(s.sum(axis=(1, 2)), f.sum(axis=(1, 2)), rtol=1e-14)


def test_axis_directions_are_permutations():
    p, f, _ = _random_state("MJ", 8, 6, 6)
    s = L.stream(f, p)
    for n in (0, 3, 6, 9):
        for k in range(6):
            q = 6 * n + k
            assert sorted(s[q].ravel().tolist()) == sorted(f[q].ravel().tolist())
    # direction 0 moves +x by one cell
    np.testing.assert_array_equal(s[0], np.roll(f[0], 1, axis=1))
    np.testing.assert_array_equal(s[6 * 3], np.roll(f[6 * 3], 1, axis=0))


def test_off_axis_stream_of_a_delta():
    """A single nonzero value in direction 1 (v = (sqrt3/2, 1/2)) spreads to the four
    cells downstream with weights |vx||vy|, (1-|vx|)|vy|, |vx|(1-|vy|), (1-|vx|)(1-|vy|)."""
    p = L.Params(stats="MJ", nx=6, ny=6)
    f = np.zeros((72, 6, 6))
    f[6, 2, 2] = 1.0
    s = L.stream(f, p)[6]
    a, b = np.sqrt(3) / 2, 0.5
    assert abs(s[3, 3] - a * b) < 1e-16 and abs(s[3, 2] - (1 - a) * b) < 1e-16
    assert abs(s[2, 3] - a * (1 - b)) < 1e-16 and abs(s[2, 2] - (1 - a) * (1 - b)) < 1e-16
    assert abs(s.sum() - 1) < 1e-15


@pytest.mark.parametrize("stats", Q.STATS)
def test_full_step_global_conservation(stats):
    p, f, _ = _random_state(stats, 8, 7, 7, amp=0.15)
    v = Q.vectors(stats)
    def tot(ff):
        return [np.tensordot(w, ff, axes=(0, 0)).sum() for w in (v["p0"], v["p0"] ** 2, v["p0"] * v["px"], v["p0"] * v["py"])]
    a = tot(f)
    for _ in range(3):
        f, _ = L.step(f, p)
    b = tot(f)
    for x, y in zip(a, b):
        assert abs(x - y) < 1e-13 * abs(a[1])


def test_riemann_mirror_symmetry():
    """Symmetric Riemann set-up (Sec. 3.1): n = 1 in L/4 < x < 3L/4, 0.1 elsewhere,
    periodic; the solution stays mirror-symmetric about the centre."""
    nx, ny = 32, 2
    p = L.Params(stats="MJ", nx=nx, ny=ny, tau=2.0)
    x = np.arange(nx)
    n = np.where((x > nx / 4) & (x < 3 * nx / 4), 1.0, 0.1)[None, :] * np.ones((ny, 1))
    f = L.init_state(p, np.ones((ny, nx)), 0.0, 0.0, n=n)
    for _ in range(20):
        f, _ = L.step(f, p)
    fl = L.fields(f, p)
    # mirror about x = nx/2: cell x <-> nx - x (x = 1..nx-1)
    m = fl["n"][0]
    np.testing.assert_allclose(m[1:], m[1:][::-1], rtol=1e-12)
    np.testing.assert_allclose(fl["ux"][0][1:], -fl["ux"][0][1:][::-1], atol=1e-13)
