"""One time step of the d2v72 relativistic lattice Boltzmann method, in FP64.

Test infrastructure (see the package docstring): never used by the product path.

State and order of operations (reading of the discrete Boltzmann equation, Sec. 2.1):
the stored state is the post-collision population f*.  A step is
  1. pull streaming with bilinear interpolation (Sec. 2.4),
  2. moments N^mu = sum f p^mu, T^{mu nu} = sum f p^mu p^nu,
  3. Landau frame: T^alpha_beta U^beta = eps U^alpha by the power method (Eq. eigen-eq),
  4. n = U_mu N^mu (Eq. density-eq),
  5. (n, eps) -> (theta, z) (Eqs. theta-eq, n-eps-eq),
  6. relaxation time: constant, or tau = a/theta + b (Sec. 3.2 uses a = 4 eta/s, b = 0.2546),
  7. equilibrium of order N on the lattice (Eq. expansion-eq),
  8. f* = f - gamma (1 - v.u) (f - f^eq) / tau  (Anderson-Witting, delta t = 1),
  9. wall cells (fixed temperature) are overwritten with f^eq(n_nb, theta_wall, u_nb).
The output fields of a state are the step's steps 1-5 plus the heat flux
q^a = (3 theta g_3/g_2)(n U^a - N^a) (Eq. heat-eq2).

Layout: f has shape (72, ny, nx), vector index q = 6 n + k (direction n, shell k),
cell (x, y) at integer coordinates x = 0..nx-1, y = 0..ny-1.

Boundary rules per side: 'periodic' (wrap), 'open' (a pull from outside the grid
takes the nearest cell of the grid: zero-gradient), 'wall' (fixed-temperature wall
cell on the edge column; x sides only; its own pull is clamped like 'open' and then
replaced in step 9), 'wall_neq' (y sides only: the edge row is a wall node whose
state is the equilibrium of an imposed (n, theta, u = 0) plus the non-equilibrium
part extrapolated from the nearest fluid row, Sec. 3.4; pulls clamp like 'open').

Forced flow (Sec. 3.4): with p.force = (a_x, a_y) the collision uses u + a tau.
"""
from dataclasses import dataclass, field

import numpy as np

from . import equilibrium, gfunc, quadrature

PM_TOL = 2.0 ** -50      # power-method stopping rule on max |delta u|
PM_MAXIT = 200


@dataclass
class Params:
    stats: str = "MJ"
    nx: int = 8
    ny: int = 8
    order: int = 5
    tau_mode: str = "const"     # 'const' | 'theta'
    tau: float = 1.0
    tau_a: float = 2.0          # tau = tau_a / theta + tau_b in 'theta' mode
    tau_b: float = 0.2546
    bc: dict = field(default_factory=lambda: dict(xlo="periodic", xhi="periodic",
                                                  ylo="periodic", yhi="periodic"))
    theta_wall: dict = field(default_factory=lambda: dict(xlo=1.0, xhi=1.0))
    force: tuple = (0.0, 0.0)   # constant acceleration (a_x, a_y), momentum update u + a tau
    wall_eq: dict = field(default_factory=lambda: dict(n=1.0, theta=1.0))   # 'wall_neq' sides, u = 0


def _src(idx, d, L, lo, hi):
    """Source coordinate idx - d along one axis under the boundary rules."""
    s = idx - d
    out = s.copy()
    low, high = s < 0, s >= L
    out[low] = (s[low] + L) if lo == "periodic" else 0
    out[high] = (s[high] - L) if hi == "periodic" else L - 1
    return out


def stream(fstar, p: Params):
    """Pull streaming (Sec. 2.4).  Axis directions (n = 0, 3, 6, 9; the paper's
    i = 1, 4, 7, 10) shift by one cell.  The others interpolate bilinearly at the
    departure point x - v from the four cells x, x - sgn(v_x), y, y - sgn(v_y):
    f_i(x,y) = f*(xb,yb)|vx||vy| + f*(x,yb)(1-|vx|)|vy| + f*(xb,y)|vx|(1-|vy|)
             + f*(x,y)(1-|vx|)(1-|vy|)."""
    ny, nx = fstar.shape[1:]
    xs, ys = np.arange(nx), np.arange(ny)
    out = np.empty_like(fstar)
    for n in range(12):
        cx, cy = quadrature.COS_DIR[n], quadrature.SIN_DIR[n]
        sx, sy = int(np.sign(cx)), int(np.sign(cy))
        ax, ay = abs(cx), abs(cy)
        xb = _src(xs, sx, nx, p.bc["xlo"], p.bc["xhi"])
        yb = _src(ys, sy, ny, p.bc["ylo"], p.bc["yhi"])
        blk = fstar[6 * n:6 * n + 6]
        if n % 3 == 0:   # axis direction: plain shift
            out[6 * n:6 * n + 6] = blk[:, yb][:, :, xb]
        else:
            out[6 * n:6 * n + 6] = (blk[:, yb][:, :, xb] * (ax * ay)
                                    + blk[:, yb][:, :, xs] * ((1 - ax) * ay)
                                    + blk[:, ys][:, :, xb] * (ax * (1 - ay))
                                    + blk * ((1 - ax) * (1 - ay)))
    return out


def moments(f, stats):
    """N^mu (3, ny, nx) and T^{mu nu} (3, 3, ny, nx) over the 72 vectors."""
    v = quadrature.vectors(stats)
    pmu = np.stack([v["p0"], v["px"], v["py"]])          # (3, 72)
    N = np.tensordot(pmu, f, axes=(1, 0))
    T = np.einsum("aq,bq,qyx->abyx", pmu, pmu, f)
    return N, T


def landau(T):
    """Power method on the mixed tensor T^alpha_beta = T^{alpha gamma} eta_{gamma beta},
    eta = diag(1, -1, -1), iterate normalised to V^0 = 1 from V = (1, 0, 0):
    V <- A V / (A V)^0.  Returns eps, ux, uy and the iteration count."""
    A = T.copy()
    A[:, 1:] *= -1.0
    shp = T.shape[2:]
    ux, uy = np.zeros(shp), np.zeros(shp)
    for it in range(1, PM_MAXIT + 1):
        av0 = A[0, 0] + A[0, 1] * ux + A[0, 2] * uy
        av1 = A[1, 0] + A[1, 1] * ux + A[1, 2] * uy
        av2 = A[2, 0] + A[2, 1] * ux + A[2, 2] * uy
        nx_, ny_ = av1 / av0, av2 / av0
        du = max(np.max(np.abs(nx_ - ux)), np.max(np.abs(ny_ - uy)))
        ux, uy = nx_, ny_
        if du <= PM_TOL:
            break
    eps = A[0, 0] + A[0, 1] * ux + A[0, 2] * uy
    return eps, ux, uy, it


def macroscopic(f, p: Params):
    """Steps 2-5 on pre-collision populations: dict of n, eps, theta, z, ux, uy,
    gamma, g (6, ...), N, flags."""
    N, T = moments(f, p.stats)
    eps, ux, uy, _ = landau(T)
    u2 = ux * ux + uy * uy
    ok = (u2 < 1.0) & (eps > 0)
    ga = 1.0 / np.sqrt(np.where(ok, 1.0 - u2, 1.0))
    n = ga * (N[0] - ux * N[1] - uy * N[2])
    ok &= n > 0
    theta, z, good = gfunc.invert_n_eps(p.stats, np.where(ok, n, 1.0), np.where(ok, eps, 1.0))
    ok &= good
    g = gfunc.g_all(p.stats, z)
    return dict(n=n, eps=eps, theta=theta, z=z, ux=ux, uy=uy, gamma=ga, g=g, N=N, ok=ok)


def relaxation_time(theta, p: Params):
    if p.tau_mode == "const":
        return np.full_like(theta, p.tau)
    return p.tau_a / theta + p.tau_b


def equilibrium_state(p: Params, theta, g, ux, uy):
    return equilibrium.feq_lattice(p.stats, theta, g, ux, uy, p.order)


def collide(f, feq, mac, tau, stats):
    """f* = f - gamma (1 - v.u) (f - f^eq) / tau (discrete AW equation, delta t = 1)."""
    v = quadrature.vectors(stats)
    vu = v["vx"][:, None, None] * mac["ux"] + v["vy"][:, None, None] * mac["uy"]
    om = mac["gamma"] * (1.0 - vu) / tau
    return f - om * (f - feq)


def _wall_feq(p: Params, mac, side):
    """f^eq(n_nb, theta_wall, u_nb) for the wall column of an x side, with n and u
    extrapolated at zeroth order from the first fluid column (Sec. 3.3)."""
    col = 1 if side == "xlo" else p.nx - 2
    n = mac["n"][:, col]
    ux, uy = mac["ux"][:, col], mac["uy"][:, col]
    th = np.full_like(n, p.theta_wall[side])
    g = gfunc.g_all(p.stats, gfunc.z_from_n_theta(p.stats, n, th))
    return equilibrium_state(p, th, g, ux, uy)


def forced(mac, tau, p: Params):
    """Momentum update of the forced flow (Sec. 3.4): the collision sees u + a tau
    (and its gamma) in place of the Landau velocity; theta, z and n are unchanged."""
    ax, ay = p.force
    if ax == 0.0 and ay == 0.0:
        return mac
    ux, uy = mac["ux"] + ax * tau, mac["uy"] + ay * tau
    return dict(mac, ux=ux, uy=uy, gamma=1.0 / np.sqrt(1.0 - (ux * ux + uy * uy)))


def _neq_wall_feq(p: Params):
    """f^eq at the imposed wall state (n, theta from p.wall_eq, u = 0), shape (72,)."""
    th = np.array(p.wall_eq["theta"], dtype=np.float64)
    z = gfunc.z_from_n_theta(p.stats, np.array(p.wall_eq["n"], dtype=np.float64), th)
    return equilibrium_state(p, th, gfunc.g_all(p.stats, z), 0.0, 0.0)


def step(fstar, p: Params):
    """One time step: returns (new post-collision state, macroscopic dict of this step).

    Walls with non-equilibrium extrapolation ('wall_neq', y sides, Sec. 3.4): the
    wall row's post-collision state is the equilibrium of the imposed wall state plus
    the post-collision non-equilibrium part f* - f^eq of the nearest fluid row."""
    f = stream(fstar, p)
    mac = macroscopic(f, p)
    tau = relaxation_time(mac["theta"], p)
    cm = forced(mac, tau, p)
    feq = equilibrium_state(p, cm["theta"], cm["g"], cm["ux"], cm["uy"])
    out = collide(f, feq, cm, tau, p.stats)
    for side, col in (("xlo", 0), ("xhi", p.nx - 1)):
        if p.bc[side] == "wall":
            out[:, :, col] = _wall_feq(p, mac, side)
    for side, row, nb in (("ylo", 0, 1), ("yhi", p.ny - 1, p.ny - 2)):
        if p.bc[side] == "wall_neq":
            out[:, row, :] = _neq_wall_feq(p)[:, None] + (out[:, nb, :] - feq[:, nb, :])
    return out, mac


def run(fstar, p: Params, nsteps):
    for _ in range(nsteps):
        fstar, _ = step(fstar, p)
    return fstar


def fields(fstar, p: Params):
    """Output fields of a state: n, eps, theta, z, ux, uy, qx, qy (moments of the
    pre-collision populations the next step would see)."""
    f = stream(fstar, p)
    mac = macroscopic(f, p)
    g2, g3 = mac["g"][1], mac["g"][2]
    hE = 3.0 * mac["theta"] * g3 / g2
    ga = mac["gamma"]
    qx = hE * (mac["n"] * ga * mac["ux"] - mac["N"][1])
    qy = hE * (mac["n"] * ga * mac["uy"] - mac["N"][2])
    return dict(n=mac["n"], eps=mac["eps"], theta=mac["theta"], z=mac["z"],
                ux=mac["ux"], uy=mac["uy"], qx=qx, qy=qy, ok=mac["ok"])


def noneq_tensors(fstar, p: Params):
    """Diagonal x components of the non-equilibrium tensors of ranks 2..5 (Eq.
    tensors-eq): {r: sum_i (f_i - f^eq_i) (p_i^x)^r}, for the pre-collision populations
    the next step would see and the equilibrium of order p.order at each cell's own
    (theta, z, u)."""
    f = stream(fstar, p)
    mac = macroscopic(f, p)
    feq = equilibrium_state(p, mac["theta"], mac["g"], mac["ux"], mac["uy"])
    px = quadrature.vectors(p.stats)["px"]
    d = f - feq
    return {r: np.tensordot(px ** r, d, axes=(0, 0)) for r in (2, 3, 4, 5)}


def init_state(p: Params, theta, ux, uy, n=None, z=None):
    """Initial post-collision state f* = f^eq from (n or z, theta, u)."""
    theta = np.asarray(theta, dtype=np.float64)
    ux = np.broadcast_to(np.asarray(ux, dtype=np.float64), theta.shape)
    uy = np.broadcast_to(np.asarray(uy, dtype=np.float64), theta.shape)
    if z is not None:
        zz = np.broadcast_to(np.asarray(z, dtype=np.float64), theta.shape)
    else:
        zz = gfunc.z_from_n_theta(p.stats, np.broadcast_to(np.asarray(n, dtype=np.float64), theta.shape), theta)
    g = gfunc.g_all(p.stats, zz)
    return equilibrium_state(p, theta, g, ux, uy)
