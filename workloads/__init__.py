"""Seeded synthetic inputs for the lattice Boltzmann workloads.

Shared by the oracle-based tests and the GPU path; holds none of the method's
arithmetic: each function returns initial macroscopic fields (theta, u and either
n or z, as float64 tensors of shape (ny, nx)) and the run parameters.  Random
parameters come from numpy.random.default_rng(seed); fields are evaluated with
torch on the requested device.

Workloads (the paper uses formula-defined initial-value problems, no datasets):
* riemann          - shock tube (Sec. 3.1 set-up with a single discontinuity pair)
* taylor_green     - decaying vortex (Sec. 3.2)
* fourier          - heat conduction between fixed-temperature walls (Sec. 3.3)
* hotspot_fd       - Fermi-Dirac Gaussian hot spot with a seeded smooth fugacity
* hotspot_be       - Bose-Einstein field of 16 seeded Gaussian bumps
* hotspot_paper    - the paper's Maxwell-Juttner hot spot (Sec. 3.5)
* smooth_random    - seeded smooth random fields for parity tests
* fugacity_ramp    - fugacity across the whole range of a statistic along x
* batch_specs      - 64 uneven Taylor-Green and Fourier grids for sweeps
* poiseuille       - forced flow between plates (Sec. 3.4)
* shear_wave       - decaying transverse shear wave (u_x varying along y)
"""
import math

import numpy as np
import torch


def _grid(nx, ny, device):
    x = torch.arange(nx, dtype=torch.float64, device=device)[None, :].expand(ny, nx)
    y = torch.arange(ny, dtype=torch.float64, device=device)[:, None].expand(ny, nx)
    return x, y


def riemann(nx=1024, ny=4, tau=0.9, n_left=1.0, n_right=0.139, device="cpu"):
    """Left/right states at equal temperature theta = 1 and u = 0; for MJ the
    pressure n theta is 1.0 / 0.139.  x sides open, y periodic."""
    x, _ = _grid(nx, ny, device)
    n = torch.where(x < nx // 2, torch.full_like(x, n_left), torch.full_like(x, n_right))
    fields = dict(n=n.contiguous(), theta=torch.ones_like(x), ux=torch.zeros_like(x), uy=torch.zeros_like(x))
    params = dict(nx=nx, ny=ny, tau_mode="const", tau=tau, bc=("open", "open", "periodic", "periodic"))
    return params, fields


def taylor_green(L=512, u0=0.05, tau=0.8, device="cpu"):
    """u_x = -u0 cos(2 pi x/L) sin(2 pi y/L), u_y = u0 sin(2 pi x/L) cos(2 pi y/L), n = theta = 1, periodic."""
    x, y = _grid(L, L, device)
    k = 2 * math.pi / L
    ux = -u0 * torch.cos(k * x) * torch.sin(k * y)
    uy = u0 * torch.sin(k * x) * torch.cos(k * y)
    fields = dict(n=torch.ones_like(x), theta=torch.ones_like(x), ux=ux.contiguous(), uy=uy.contiguous())
    params = dict(nx=L, ny=L, tau_mode="const", tau=tau, bc=("periodic",) * 4)
    return params, fields


def fourier(nx=2048, ny=2, dT=1e-3, tau=1.0, device="cpu"):
    """theta linear between the walls theta_L = 1 - dT/2 (x = 0) and theta_R = 1 + dT/2
    (x = nx - 1), n = 1, u = 0; y periodic."""
    x, _ = _grid(nx, ny, device)
    th = (1 - dT / 2) + x * dT / (nx - 1)
    fields = dict(n=torch.ones_like(x), theta=th.contiguous(), ux=torch.zeros_like(x), uy=torch.zeros_like(x))
    params = dict(nx=nx, ny=ny, tau_mode="const", tau=tau, bc=("wall", "wall", "periodic", "periodic"),
                  theta_wall=(1 - dT / 2, 1 + dT / 2))
    return params, fields


def _smooth_field(nx, ny, rng, nmodes, kmax, device):
    """Sum of nmodes cosines with integer wavevectors |k| <= kmax and random phases,
    rescaled to [0, 1]."""
    x, y = _grid(nx, ny, device)
    s = torch.zeros_like(x)
    ks = [(a, b) for a in range(-kmax, kmax + 1) for b in range(0, kmax + 1)
          if 0 < a * a + b * b <= kmax * kmax and (b > 0 or a > 0)]
    pick = rng.choice(len(ks), size=nmodes, replace=False)
    for i in pick:
        a, b = ks[i]
        ph = rng.uniform(0, 2 * math.pi)
        s = s + torch.cos(2 * math.pi * (a * x / nx + b * y / ny) + ph)
    return (s - s.min()) / (s.max() - s.min())


def hotspot_fd(L=2048, seed=4, amp=0.3, sigma=64.0, device="cpu"):
    """theta = 1 + amp exp(-r^2 / 2 sigma^2) about the centre; z = 0.5 * 4^s with s a
    seeded smooth field in [0, 1] (so z in [0.5, 2]); u = 0; open boundaries;
    tau = 2/theta + 0.2546 (eta/s = 0.5, Sec. 3.5)."""
    rng = np.random.default_rng(seed)
    x, y = _grid(L, L, device)
    c = L / 2
    th = 1 + amp * torch.exp(-((x - c) ** 2 + (y - c) ** 2) / (2 * sigma ** 2))
    s = _smooth_field(L, L, rng, 8, 4, device)
    z = 0.5 * torch.pow(4.0, s)
    fields = dict(z=z.contiguous(), theta=th.contiguous(), ux=torch.zeros_like(x), uy=torch.zeros_like(x))
    params = dict(nx=L, ny=L, stats="FD", tau_mode="theta", tau_a=2.0, tau_b=0.2546, bc=("open",) * 4)
    return params, fields


def hotspot_be(L=8192, seed=5, nbumps=16, device="cpu"):
    """16 Gaussian bumps g_k (centres uniform on the grid, sigma_k ~ U[L/128, L/16]):
    theta = 1 + sum a_k g_k, a_k ~ U[-0.2, 0.3]; z = clip(0.55 + sum b_k g_k, 0.2, 0.9),
    b_k ~ U[-0.3, 0.3]; u = 0; open boundaries; tau = 2/theta + 0.2546."""
    rng = np.random.default_rng(seed)
    x, y = _grid(L, L, device)
    th = torch.ones_like(x)
    zz = torch.full_like(x, 0.55)
    for _ in range(nbumps):
        cx, cy = rng.uniform(0, L, size=2)
        sg = rng.uniform(L / 128, L / 16)
        a, b = rng.uniform(-0.2, 0.3), rng.uniform(-0.3, 0.3)
        g = torch.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * sg * sg))
        th = th + a * g
        zz = zz + b * g
    th = torch.clamp(th, min=0.5)
    fields = dict(z=torch.clamp(zz, 0.2, 0.9).contiguous(), theta=th.contiguous(),
                  ux=torch.zeros_like(x), uy=torch.zeros_like(x))
    params = dict(nx=L, ny=L, stats="BE", tau_mode="theta", tau_a=2.0, tau_b=0.2546, bc=("open",) * 4)
    return params, fields


def hotspot_paper(L=512, radius=32.0, theta_in=1.5, theta_out=0.5, device="cpu"):
    """Hot spot of Sec. 3.5: theta_in inside (x - L/2)^2 + (y - L/2)^2 <= radius^2,
    theta_out elsewhere, n = 1, u = 0, open boundaries, tau = 2/theta + 0.2546
    (eta/s = 0.5)."""
    x, y = _grid(L, L, device)
    inside = (x - L / 2) ** 2 + (y - L / 2) ** 2 <= radius ** 2
    th = torch.where(inside, torch.full_like(x, theta_in), torch.full_like(x, theta_out))
    fields = dict(n=torch.ones_like(x), theta=th.contiguous(), ux=torch.zeros_like(x), uy=torch.zeros_like(x))
    params = dict(nx=L, ny=L, stats="MJ", tau_mode="theta", tau_a=2.0, tau_b=0.2546, bc=("open",) * 4)
    return params, fields


def smooth_random(nx, ny, seed, stats="MJ", amp_theta=0.2, amp_u=0.15, device="cpu"):
    """Seeded smooth random theta in [1 - amp, 1 + amp], u of magnitude up to ~amp_u and
    z in [0.3, 0.9] (BE) or [0.3, 2.0] (MJ, FD) for parity tests."""
    rng = np.random.default_rng(seed)
    th = 1 - amp_theta + 2 * amp_theta * _smooth_field(nx, ny, rng, 4, 2, device)
    ux = amp_u * (2 * _smooth_field(nx, ny, rng, 4, 2, device) - 1)
    uy = amp_u * (2 * _smooth_field(nx, ny, rng, 4, 2, device) - 1)
    zhi = 0.9 if stats == "BE" else 2.0
    z = 0.3 + (zhi - 0.3) * _smooth_field(nx, ny, rng, 4, 2, device)
    return dict(z=z.contiguous(), theta=th.contiguous(), ux=ux.contiguous(), uy=uy.contiguous())


def fugacity_ramp(nx, ny, seed, stats="FD", amp_theta=0.1, amp_u=0.05, device="cpu"):
    """ln z swept along x across the statistic's range: FD from ln 1e-6 to ln 1e4
    (evenly in ln z); BE ln z = -exp(s) with s even from ln(-ln 1e-6) to ln(-ln 0.999),
    so that z approaches 1 on a logarithmic scale.  theta and u are seeded smooth
    fields of amplitude amp_theta about 1 and amp_u."""
    rng = np.random.default_rng(seed)
    x, _ = _grid(nx, ny, device)
    t = x / max(nx - 1, 1)
    if stats == "FD":
        mu = math.log(1e-6) + (math.log(1e4) - math.log(1e-6)) * t
    elif stats == "BE":
        s0, s1 = math.log(-math.log(1e-6)), math.log(-math.log(0.999))
        mu = -torch.exp(s0 + (s1 - s0) * t)
    else:
        raise ValueError("fugacity_ramp is for FD and BE")
    th = 1 - amp_theta + 2 * amp_theta * _smooth_field(nx, ny, rng, 4, 2, device)
    ux = amp_u * (2 * _smooth_field(nx, ny, rng, 4, 2, device) - 1)
    uy = amp_u * (2 * _smooth_field(nx, ny, rng, 4, 2, device) - 1)
    return dict(z=torch.exp(mu).contiguous(), theta=th.contiguous(), ux=ux.contiguous(), uy=uy.contiguous())


def batch_specs(seed=3, ngrids=64, steps=10000):
    """64 grid descriptions for a transport sweep: even index Taylor-Green (square,
    L a multiple of 16 in [64, 512], u0 = 0.05), odd index Fourier flow (nx, ny
    multiples of 16 in [64, 512], walls theta = 1 -/+ 5e-4); tau ~ U[0.55, 1.5].
    The walls hold dT = 1e-3, the paper's own scale (Sec. 3.3 uses 5e-4 .. 1.5e-3): under
    the wall rule (density and velocity extrapolated from the first fluid cell) the
    pressure difference between the walls accelerates the fluid uniformly, by about
    dT / (1.5 nx) per step, and with dT = 0.1 a 64-wide grid passes |u| = 0.5 within
    1000 steps and breaks down before 2000; with 1e-3 it stays below 0.07 over 10000."""
    rng = np.random.default_rng(seed)
    sizes = np.arange(64, 513, 16)
    specs = []
    for g in range(ngrids):
        tau = float(rng.uniform(0.55, 1.5))
        if g % 2 == 0:
            L = int(rng.choice(sizes))
            specs.append(dict(kind="taylor_green", nx=L, ny=L, tau=tau, u0=0.05))
        else:
            nx, ny = int(rng.choice(sizes)), int(rng.choice(sizes))
            specs.append(dict(kind="fourier", nx=nx, ny=ny, tau=tau, dT=1e-3))
    return specs


def poiseuille(L=32, nx=4, a=1e-8, tau=3.0, device="cpu"):
    """Plates at the wall rows y = 0 and y = L (ny = L + 1) with n = theta = 1, u = 0
    imposed; x periodic; fluid at rest with n = theta = 1; acceleration a along x;
    constant tau (Sec. 3.4 uses tau = 3, a = 1e-8)."""
    x, _ = _grid(nx, L + 1, device)
    one = torch.ones_like(x)
    fields = dict(n=one.clone(), theta=one.clone(), ux=torch.zeros_like(x), uy=torch.zeros_like(x))
    params = dict(nx=nx, ny=L + 1, tau_mode="const", tau=tau, force=(a, 0.0),
                  bc=("periodic", "periodic", "wall_neq", "wall_neq"), wall_n=1.0, wall_theta=1.0)
    return params, fields


def shear_wave(L=32, nx=4, u0=1e-4, tau=3.0, device="cpu"):
    """u_x = u0 sin(2 pi y / L), u_y = 0, n = theta = 1, periodic: its decay rate
    nu k^2 measures the shear viscosity for wavevectors along y."""
    _, y = _grid(nx, L, device)
    one = torch.ones_like(y)
    fields = dict(n=one.clone(), theta=one.clone(), ux=(u0 * torch.sin(2 * math.pi * y / L)).contiguous(),
                  uy=torch.zeros_like(y))
    params = dict(nx=nx, ny=L, tau_mode="const", tau=tau, bc=("periodic",) * 4)
    return params, fields
