"""The oracle reproduces the transport relations the paper measures (Sec. 3.2, Eq.
nu-ref-eq: nu = (tau - 0.2546)/4; Sec. 3.3, Eq. kappa-tau-eq: kappa = 1.5 tau g_3/g_2)
and not the Grad-theory values (nu = tau/5, kappa = 3 n tau/8), for Maxwell-Juttner.

Small grids (32^2 Taylor-Green, 64 x 2 Fourier flow) keep the CPU time to seconds;
the relations hold there to better than 1% (viscosity) and 0.1% (conductivity).
"""
import numpy as np
import pytest

from conftest import read_golden
from oracle import gfunc as G
from oracle import lattice as L

GOLD = {k: float(v) for k, v in read_golden("transport.txt")}


def taylor_green_nu(L_, tau, u0=0.05, stats="MJ"):
    p = L.Params(stats=stats, nx=L_, ny=L_, tau=tau)
    x = np.arange(L_)[None, :]
    y = np.arange(L_)[:, None]
    k = 2 * np.pi / L_
    ux = -u0 * np.cos(k * x) * np.sin(k * y)
    uy = u0 * np.sin(k * x) * np.cos(k * y)
    f = L.init_state(p, np.ones((L_, L_)), ux, uy, n=np.ones((L_, L_)))
    rate = 16 * np.pi ** 2 * (tau - GOLD["nu_offset"]) * GOLD["nu_slope"] / L_ ** 2
    nsteps = int(3 / rate)
    every = max(1, nsteps // 30)
    ts, sig = [], []
    for t in range(nsteps + 1):
        if t % every == 0 and t >= nsteps // 5:
            fl = L.fields(f, p)
            u2 = fl["ux"] ** 2 + fl["uy"] ** 2
            ts.append(t)
            sig.append(np.sqrt(((u2 - u2.mean()) ** 2).mean()))   # sigma_{u^2}, Eq. sigma-u2
        if t < nsteps:
            f, _ = L.step(f, p)
    slope = np.polyfit(ts, np.log(sig), 1)[0]
    return -slope * L_ ** 2 / (16 * np.pi ** 2)


@pytest.mark.slow
def test_taylor_green_viscosity():
    taus = (0.6, 0.8, 1.0)
    nus = [taylor_green_nu(32, t) for t in taus]
    for tau, nu in zip(taus, nus):
        paper = GOLD["nu_slope"] * (tau - GOLD["nu_offset"])
        grad = GOLD["grad_nu_slope"] * tau
        assert abs(nu / paper - 1) < 0.01, (tau, nu, paper)
        assert abs(nu / grad - 1) > 0.05, (tau, nu, grad)
    slope, icpt = np.polyfit(taus, nus, 1)
    assert abs(slope - 0.25) < 0.005


def fourier_kappa(nx, tau, dT=1e-3, nsteps=200, stats="MJ"):
    ny = 2
    p = L.Params(stats=stats, nx=nx, ny=ny, tau=tau,
                 bc=dict(xlo="wall", xhi="wall", ylo="periodic", yhi="periodic"),
                 theta_wall=dict(xlo=1 - dT / 2, xhi=1 + dT / 2))
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    f = L.init_state(p, (1 - dT / 2) + x * dT / (nx - 1), 0.0, 0.0, n=np.ones((ny, nx)))
    for _ in range(nsteps - 1):
        f, _ = L.step(f, p)
    fm = L.fields(f, p)
    f, _ = L.step(f, p)
    fl = L.fields(f, p)
    f, _ = L.step(f, p)
    fp = L.fields(f, p)
    gu = lambda d: d["ux"][0] / np.sqrt(1 - d["ux"][0] ** 2 - d["uy"][0] ** 2)
    T, ux = fl["theta"][0], fl["ux"][0]
    ga = 1 / np.sqrt(1 - ux ** 2 - fl["uy"][0] ** 2)
    # F(dT) of Eq. fdt-eq, with the time derivative by central differences
    F = -((1 + ux ** 2 * ga ** 2) * np.gradient(T)
          + T * ga * ((gu(fp) - gu(fm)) / 2 + ux * np.gradient(gu(fl))))
    m = slice(nx // 8, nx - nx // 8)
    g = G.g_all(stats, fl["z"][0])
    return fl["qx"][0][m].mean() / F[m].mean(), (g[2] / g[1])[m].mean(), fl["n"][0][m].mean()


@pytest.mark.slow
def test_fourier_conductivity():
    for tau in (0.8, 1.5):
        kappa, g32, n = fourier_kappa(64, tau)
        paper = GOLD["kappa_slope_mj"] * tau * g32
        grad = GOLD["grad_kappa_slope_mj"] * n * tau
        assert abs(kappa / paper - 1) < 1e-3, (tau, kappa, paper)
        assert abs(kappa / grad - 1) > 0.5


def kappa_anderson_witting(stats, n, z, tau):
    """First-order Chapman-Enskog conductivity of the Anderson-Witting equation for
    the massless 2-D gas, written out independently of the lattice: with
    delta f = -(tau / p.U) p^mu d_mu f_eq, the Euler equation for the acceleration and
    Gibbs-Duhem, the particle current in the Landau frame is
      N^x = pi tau theta F (2 g_2 - 3 g_1 g_3 / g_2),   F of Eq. fdt-eq,
    and q^x = -(3 theta g_3/g_2) N^x (Eq. heat-eq2), so
      kappa = (3/2) tau n (g_3/g_2)(3 g_1 g_3/g_2^2 - 2),   n = 2 pi theta^2 g_2.
    For MJ (g_nu = z) it is (3/2) n tau; at n = 1 the paper's kappa = 1.5 tau."""
    g = G.g_all(stats, np.array([z]))
    g1, g2, g3 = g[0][0], g[1][0], g[2][0]
    return 1.5 * tau * n * (g3 / g2) * (3 * g1 * g3 / g2 ** 2 - 2)


def fourier_kappa_state(nx, tau, stats, n0=None, z0=None, dT=1e-3, nsteps=200):
    """Fourier flow between fixed-temperature walls started from a uniform n0 (or z0):
    kappa = <q^x>/<F> over the interior, with the interior means of n and z."""
    ny = 2
    p = L.Params(stats=stats, nx=nx, ny=ny, tau=tau,
                 bc=dict(xlo="wall", xhi="wall", ylo="periodic", yhi="periodic"),
                 theta_wall=dict(xlo=1 - dT / 2, xhi=1 + dT / 2))
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    th = (1 - dT / 2) + x * dT / (nx - 1)
    if z0 is not None:
        f = L.init_state(p, th, 0.0, 0.0, z=np.full((ny, nx), z0))
    else:
        f = L.init_state(p, th, 0.0, 0.0, n=np.full((ny, nx), n0))
    for _ in range(nsteps - 1):
        f, _ = L.step(f, p)
    fm = L.fields(f, p)
    f, _ = L.step(f, p)
    fl = L.fields(f, p)
    f, _ = L.step(f, p)
    fp = L.fields(f, p)
    gu = lambda d: d["ux"][0] / np.sqrt(1 - d["ux"][0] ** 2 - d["uy"][0] ** 2)
    T, ux = fl["theta"][0], fl["ux"][0]
    ga = 1 / np.sqrt(1 - ux ** 2 - fl["uy"][0] ** 2)
    F = -((1 + ux ** 2 * ga ** 2) * np.gradient(T)
          + T * ga * ((gu(fp) - gu(fm)) / 2 + ux * np.gradient(gu(fl))))
    m = slice(nx // 8, nx - nx // 8)
    return fl["qx"][0][m].mean() / F[m].mean(), fl["n"][0][m].mean(), fl["z"][0][m].mean()


@pytest.mark.slow
@pytest.mark.parametrize("stats,n0", [("MJ", 2.0), ("FD", 1.0), ("BE", 1.0)])
def test_conductivity_is_the_anderson_witting_value(stats, n0):
    """Sec. 3.3 set-up at n0 = 1 (FD, BE) and n0 = 2 (MJ): the oracle's kappa equals the
    closed-form Anderson-Witting conductivity to 1e-5.  For FD and BE at n0 = 1 that is
    kappa g_2/g_3 = 1.416 tau and 1.596 tau, not the 1.5 tau printed with Eq.
    kappa-tau-eq; for MJ at n0 = 2 it is 3 tau, twice the printed value (which holds at
    n = 1 only)."""
    tau = 1.0
    kappa, n, z = fourier_kappa_state(64, tau, stats, n0=n0)
    ce = kappa_anderson_witting(stats, n, z, tau)
    g = G.g_all(stats, np.array([z]))
    a = kappa * g[1][0] / g[2][0] / tau
    print(f"  {stats} n={n:.5f} z={z:.5f}: kappa g2/g3 / tau = {a:.7f}, Anderson-Witting "
          f"{ce * g[1][0] / g[2][0] / tau:.7f}")
    assert abs(kappa / ce - 1) < 1e-5, (stats, kappa, ce)
    if stats == "MJ":
        assert abs(kappa / (1.5 * n * tau) - 1) < 1e-5
    else:
        assert abs(a - 1.5) > 0.05           # the printed FD/BE slope is not what the method gives


@pytest.mark.slow
@pytest.mark.parametrize("stats,z0", [("FD", 3.0), ("BE", 0.9)])
def test_conductivity_degenerate_states_approach_anderson_witting(stats, z0):
    """Far from the classical limit (FD z = 3, BE z = 0.9) the same relation holds once
    the start-up transient has passed: the gap falls from ~5e-3 after 200 steps to
    ~1e-3 after 600 on 64 x 2 (the two formulas 1.5 n g_1/g_3 and Anderson-Witting
    differ there by 0.7% and 4%)."""
    tau = 1.0
    k200, n, z = fourier_kappa_state(64, tau, stats, z0=z0, nsteps=200)
    k600, n6, z6 = fourier_kappa_state(64, tau, stats, z0=z0, nsteps=600)
    e200 = abs(k200 / kappa_anderson_witting(stats, n, z, tau) - 1)
    e600 = abs(k600 / kappa_anderson_witting(stats, n6, z6, tau) - 1)
    print(f"  {stats} z={z0}: |kappa/AW - 1| {e200:.2e} (200 steps), {e600:.2e} (600 steps)")
    assert e600 < 2e-3 and e600 < e200 / 3


def axial_shear_nu(L_, tau, nx=1, u0=1e-4):
    """Kinematic viscosity from the decay of a transverse shear wave u_x = u0 sin(2 pi y/L)
    whose wavevector lies along a lattice axis (periodic, MJ, n = theta = 1): projection
    of u_x on the mode, fitted over one e-folding time after a fifth of it."""
    p = L.Params(stats="MJ", nx=nx, ny=L_, tau=tau)
    s = np.sin(2 * np.pi * np.arange(L_) / L_)
    ux = u0 * s[:, None] * np.ones((1, nx))
    f = L.init_state(p, np.ones((L_, nx)), ux, 0 * ux, n=np.ones((L_, nx)))
    k2 = (2 * np.pi / L_) ** 2
    T = int(1.0 / ((tau - GOLD["nu_offset"]) * GOLD["nu_slope"] * k2))
    t_skip = max(20, T // 5)
    every = max(1, (T - t_skip) // 20)
    ts, amp = [], []
    for t in range(T + 1):
        if t >= t_skip and (t - t_skip) % every == 0:
            u = L.fields(f, p)["ux"][:, 0]
            ts.append(t)
            amp.append(np.dot(u, s) / np.dot(s, s))
        if t < T:
            f, _ = L.step(f, p)
    return -np.polyfit(ts, np.log(amp), 1)[0] / k2


@pytest.mark.slow
def test_axial_shear_viscosity_converges_above_the_diagonal_value():
    """tau = 3 (the Poiseuille runs of Sec. 3.4): shear waves with the wavevector along
    a lattice axis decay with a viscosity that converges like 1/L^2 to 0.697, 1.6%
    above Eq. nu-ref-eq's 0.6864, which the paper measured on Taylor-Green modes (whose
    wavevectors are diagonal).  The interpolated streaming is anisotropic."""
    tau = 3.0
    nus = [axial_shear_nu(L_, tau) for L_ in (64, 128, 256)]
    d1, d2 = nus[1] - nus[0], nus[2] - nus[1]
    limit = nus[2] + d2 / 3.0                      # Richardson, error ~ 1/L^2
    paper = GOLD["nu_slope"] * (tau - GOLD["nu_offset"])
    print(f"  axial nu(tau=3): L=64 {nus[0]:.6f}, 128 {nus[1]:.6f}, 256 {nus[2]:.6f}; limit {limit:.6f}; "
          f"Eq. nu-ref-eq {paper:.6f}")
    assert 0 < d2 < d1 / 3.5                       # second-order convergence
    assert abs(limit - 0.6972) < 5e-4
    assert limit / paper - 1 > 0.012
