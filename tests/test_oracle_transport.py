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
