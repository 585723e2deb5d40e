"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

FP64 bars: tests/parity_bars.py (a base of about three times the short-run errors,
plus three times the per-step drift between two independent FP64 implementations of
the method, times the number of steps).
FP32 populations: bars from the 2^-24 storage rounding per step, amplified by the
inversion (theta, z) and by the cancellation in q = n U - N.
Edge cases: fugacities across every branch of the g_nu evaluation (FD 1e-6 .. 1e4, BE
1e-6 .. 0.999), the FD table-range flag, |u| up to 0.6, and the persistent batch
kernel.  Where one grid spans many decades of n, errors are taken cell by cell
(relative to the cell's own value) with the inversion's conditioning in the bar.
"""
import numpy as np
import pytest
import torch

import workloads
from conftest import same_bits
from oracle import gfunc as G
from oracle import lattice as L
from oracle import quadrature as Q
from parity_bars import field_bar, shell_bar

pytestmark = pytest.mark.gpu

FIELD_NAMES = ("n", "eps", "theta", "z", "ux", "uy", "qx", "qy")
FIELD_TOL_FP32 = dict(n=2e-6, eps=2e-6, theta=2e-6, z=5e-6, ux=2e-5, uy=2e-5, qx=2e-3, qy=2e-3)
FLOOR = dict(ux=("abs", 0.01), uy=("abs", 0.01), qx=("eps", 1e-3), qy=("eps", 1e-3))


@pytest.fixture(scope="module")
def rl():
    from paper_1709_09073_amd import rlbm
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return rlbm


def _oracle_params(params, stats):
    bcmap = dict(zip(("xlo", "xhi", "ylo", "yhi"), params.get("bc", ("periodic",) * 4)))
    tw = params.get("theta_wall", (1.0, 1.0))
    return L.Params(stats=stats, nx=params["nx"], ny=params["ny"], tau_mode=params.get("tau_mode", "const"),
                    tau=params.get("tau", 1.0), tau_a=params.get("tau_a", 2.0), tau_b=params.get("tau_b", 0.2546),
                    bc=bcmap, theta_wall=dict(xlo=tw[0], xhi=tw[1]))


def _oracle_init(op, fields):
    f = {k: v.cpu().numpy() for k, v in fields.items()}
    return L.init_state(op, f["theta"], f["ux"], f["uy"], n=f.get("n"), z=f.get("z"))


def _scale(k, b):
    ref = np.abs(b[k]).max()
    if k in FLOOR:
        kind, fl = FLOOR[k]
        ref = max(ref, fl if kind == "abs" else fl * np.abs(b["eps"]).max())
    return max(ref, 1e-300)


def _compare_fields(a, b, tol, ctx):
    for k, t in tol.items():
        err = np.abs(a[k] - b[k]).max() / _scale(k, b)
        print(f"  {ctx}: {k} err {err:.2e} (bar {t:.1e}, ratio {err / t:.2f})")
        assert err <= t, f"{ctx}: field {k} rel err {err:.3e} > {t:.1e}"


def _compare_pops(a, b, tols, ctx):
    for k, t in enumerate(tols):
        sl = slice(k, 72, 6)
        err = np.abs(a[sl] - b[sl]).max() / np.abs(b[sl]).max()
        print(f"  {ctx}: shell {k} err {err:.2e} (bar {t:.1e}, ratio {err / t:.2f})")
        assert err <= t, f"{ctx}: shell {k} rel err {err:.3e} > {t:.1e}"


def fp64_field_bars(k):
    return {name: field_bar(name, k) for name in FIELD_NAMES}


def fp64_shell_bars(k):
    return [shell_bar(s, k) for s in range(6)]


def _run(rl, stats, precision, params, fields, nsteps):
    params = dict(params, stats=stats, precision=precision)
    print(f"[parity] {stats} {precision} {params['nx']}x{params['ny']} bc={params.get('bc')} steps={nsteps}", flush=True)
    sim = rl.Sim(params, {k: v.cuda() for k, v in fields.items()})
    sim.step(nsteps)
    pops = sim.populations().double().cpu().numpy()
    flds = {k: v.cpu().numpy() for k, v in sim.fields().items()}
    sim.close()
    op = _oracle_params(params, stats)
    f = _oracle_init(op, fields)
    for _ in range(nsteps):
        f, _ = L.step(f, op)
    return pops, flds, f, L.fields(f, op)


CASES = [
    # stats, nx, ny, steps, bc, tau_mode
    ("MJ", 70, 13, 6, ("periodic",) * 4, "const"),
    ("MJ", 67, 9, 4, ("open",) * 4, "theta"),
    ("FD", 70, 13, 3, ("periodic",) * 4, "const"),
    ("FD", 66, 7, 3, ("open", "open", "periodic", "periodic"), "theta"),
    ("BE", 70, 13, 3, ("open",) * 4, "const"),
    ("BE", 65, 6, 2, ("periodic",) * 4, "theta"),
]


@pytest.mark.parametrize("stats,nx,ny,nsteps,bc,tau_mode", CASES)
def test_fp64_parity(rl, stats, nx, ny, nsteps, bc, tau_mode):
    fields = workloads.smooth_random(nx, ny, seed=nx * ny, stats=stats)
    params = dict(nx=nx, ny=ny, bc=bc, tau_mode=tau_mode, tau=0.85, tau_a=0.6, tau_b=0.6)
    pops, flds, fo, flo = _run(rl, stats, "fp64", params, fields, nsteps)
    ctx = f"{stats} fp64 {nx}x{ny} {bc[0]}"
    _compare_pops(pops, fo, fp64_shell_bars(nsteps), ctx)
    _compare_fields(flds, flo, fp64_field_bars(nsteps), ctx)


@pytest.mark.parametrize("stats", ["MJ", "FD", "BE"])
def test_fp64_init_parity(rl, stats):
    fields = workloads.smooth_random(33, 5, seed=5, stats=stats)
    params = dict(nx=33, ny=5)
    pops, flds, fo, flo = _run(rl, stats, "fp64", params, fields, 0)
    _compare_pops(pops, fo, fp64_shell_bars(0), f"{stats} init")
    _compare_fields(flds, flo, fp64_field_bars(0), f"{stats} init")


@pytest.mark.parametrize("stats", ["MJ", "FD", "BE"])
def test_fp64_walls(rl, stats):
    params, fields = workloads.fourier(nx=40, ny=4, dT=0.05, tau=0.9)
    pops, flds, fo, flo = _run(rl, stats, "fp64", params, fields, 4)
    _compare_pops(pops, fo, fp64_shell_bars(4), f"{stats} walls")
    _compare_fields(flds, flo, fp64_field_bars(4), f"{stats} walls")


@pytest.mark.parametrize("stats,nsteps", [("MJ", 8), ("FD", 3), ("BE", 3)])
def test_fp32_parity(rl, stats, nsteps):
    fields = workloads.smooth_random(70, 13, seed=3, stats=stats)
    params = dict(nx=70, ny=13, bc=("periodic",) * 4, tau=0.9)
    pops, flds, fo, flo = _run(rl, stats, "fp32", params, fields, nsteps)
    _compare_fields(flds, flo, FIELD_TOL_FP32, f"{stats} fp32")


@pytest.mark.parametrize("stats", ["MJ", "FD", "BE"])
def test_fp64_single_step_from_oracle_state(rl, stats):
    """One GPU step from a non-equilibrium state produced by the oracle (copied into
    the caller-owned population buffer) against the oracle's next step."""
    nx, ny = 69, 11
    fields = workloads.smooth_random(nx, ny, seed=21, stats=stats, amp_u=0.2)
    op = _oracle_params(dict(nx=nx, ny=ny, tau=0.7), stats)
    f = _oracle_init(op, fields)
    for _ in range(15):
        f, _ = L.step(f, op)
    print(f"[parity] {stats} single step from oracle state {nx}x{ny}", flush=True)
    sim = rl.Sim(dict(nx=nx, ny=ny, stats=stats, precision="fp64", tau=0.7), {k: v.cuda() for k, v in fields.items()})
    sim.set_populations(torch.from_numpy(f))
    sim.step(1)
    pops = sim.populations().cpu().numpy()
    flds = {k: v.cpu().numpy() for k, v in sim.fields().items()}
    sim.close()
    f1, _ = L.step(f, op)
    ref = L.fields(f1, op)
    _compare_pops(pops, f1, fp64_shell_bars(1), f"{stats} one step")
    _compare_fields(flds, ref, fp64_field_bars(1), f"{stats} one step")


def test_riemann_fp64_full_config(rl):
    """Shock tube MJ, 1024 x 4, FP64, tau = 0.9, 500 steps: the small configuration."""
    params, fields = workloads.riemann(nx=1024, ny=4, tau=0.9)
    pops, flds, fo, flo = _run(rl, "MJ", "fp64", params, fields, 500)
    _compare_pops(pops, fo, fp64_shell_bars(500), "riemann")
    _compare_fields(flds, flo, fp64_field_bars(500), "riemann")


def test_minimal_grid(rl):
    fields = workloads.smooth_random(2, 2, seed=9, stats="MJ", amp_u=0.05)
    params = dict(nx=2, ny=2)
    pops, flds, fo, flo = _run(rl, "MJ", "fp64", params, fields, 3)
    _compare_fields(flds, flo, fp64_field_bars(3), "2x2")


def test_domain_flag_be_condensation(rl):
    """A BE state beyond the condensation bound is clamped and reported."""
    nx, ny = 16, 4
    th = torch.ones((ny, nx), dtype=torch.float64)
    # n far above 2 pi theta^2 g_2(z_c) = 2 pi zeta(2)(1 - ...) ~ 10.3
    fields = dict(n=torch.full((ny, nx), 50.0, dtype=torch.float64), theta=th,
                  ux=torch.zeros_like(th), uy=torch.zeros_like(th))
    sim = rl.Sim(dict(nx=nx, ny=ny, stats="BE", precision="fp64"), {k: v.cuda() for k, v in fields.items()})
    assert sim.status() & rl.FLAG_CONDENSED
    with pytest.raises(rl.RlbmError):
        sim.sync()
    assert sim.status() == 0
    sim.close()


def test_deterministic(rl):
    fields = workloads.smooth_random(130, 17, seed=1, stats="FD")
    params = dict(nx=130, ny=17, stats="FD", precision="fp32")
    outs = []
    for _ in range(2):
        sim = rl.Sim(params, {k: v.cuda() for k, v in fields.items()})
        sim.step(5)
        outs.append(sim.state().cpu().clone())
        sim.close()
    assert same_bits(outs[0], outs[1])


def _cellwise(a, b):
    return np.abs(a - b) / np.abs(b)


@pytest.mark.parametrize("stats", ["FD", "BE"])
def test_fp64_fugacity_across_every_branch(rl, stats):
    """z swept across the range of the statistic (FD 1e-6 .. 1e4: the defining series
    below ln z = -12.125 and the Taylor tables above; BE 1e-6 .. 0.999: the series, the
    tables and the expansion about z = 1).  n spans many decades here, so fields are
    compared cell by cell against the cell's own value: n and eps to 2e-13 x steps;
    z and theta with the inversion's conditioning kappa = 1 / |3 g_1/g_2 - 2 g_2/g_3|
    (d ln z = kappa d ln r, d ln r = 3 d ln n - 2 d ln eps; FD at z = 1e4 has kappa ~ 35);
    populations on the scale w_k max_i |f_i/w_k| of their own cell."""
    nx, ny, nsteps = 64, 5, 3
    fields = workloads.fugacity_ramp(nx, ny, seed=7, stats=stats)
    params = dict(nx=nx, ny=ny, bc=("open", "open", "periodic", "periodic"), tau=0.9)
    pops, flds, fo, flo = _run(rl, stats, "fp64", params, fields, nsteps)
    g = G.g_all(stats, flo["z"])
    kappa = 1.0 / np.abs(3 * g[0] / g[1] - 2 * g[1] / g[2])
    base = 2e-13 * nsteps
    bars = dict(n=base, eps=base, z=base * (1 + 5 * kappa),
                theta=base * (2 + 5 * kappa * np.abs(g[0] / g[1] - g[1] / g[2])))
    for k, bar in bars.items():
        r = (_cellwise(flds[k], flo[k]) / bar).max()
        print(f"  {stats} z sweep: {k} worst cell error / bar {r:.3f}")
        assert r <= 1.0, (k, r)
    du = np.maximum(np.abs(flds["ux"] - flo["ux"]), np.abs(flds["uy"] - flo["uy"])).max()
    print(f"  {stats} z sweep: max |u - u_oracle| {du:.2e}")
    assert du <= base
    w = Q.vectors(stats)["w"][:, None, None]
    M = np.abs(fo / w).max(axis=0)
    r = (np.abs(pops - fo) / (w * M) / 1.5e-12).max()
    print(f"  {stats} z sweep: populations worst error / (1.5e-12 w_k M_cell) {r:.3f}")
    assert r <= 1.0


@pytest.mark.parametrize("stats", ["FD", "BE"])
def test_fp32_fugacity_across_every_branch(rl, stats):
    """The same z sweep with FP32 populations and the fixed Newton start (mu = 0 FD,
    ln 1/2 BE): the Newton iterates walk across many table centres, so the FP32
    inversion's row kept in registers between evaluations is replaced whenever the
    centre changes (a stale row would be off by orders of magnitude).  Bars from the
    2^-24 storage rounding of each step, cell by cell: n, eps 2e-6 x steps, z and theta
    with the conditioning kappa as above, u 2e-5 of max(|u|, 0.01), populations 1e-5 of
    w_k max_i |f_i/w_k| of their own cell."""
    nx, ny, nsteps = 64, 5, 3
    fields = workloads.fugacity_ramp(nx, ny, seed=7, stats=stats)
    params = dict(nx=nx, ny=ny, bc=("open", "open", "periodic", "periodic"), tau=0.9)
    pops, flds, fo, flo = _run(rl, stats, "fp32", params, fields, nsteps)
    g = G.g_all(stats, flo["z"])
    kappa = 1.0 / np.abs(3 * g[0] / g[1] - 2 * g[1] / g[2])
    base = 2e-6 * nsteps
    bars = dict(n=base, eps=base, z=base * (1 + 5 * kappa),
                theta=base * (2 + 5 * kappa * np.abs(g[0] / g[1] - g[1] / g[2])))
    for k, bar in bars.items():
        r = (_cellwise(flds[k], flo[k]) / bar).max()
        print(f"  {stats} fp32 z sweep: {k} worst cell error / bar {r:.3f}")
        assert r <= 1.0, (k, r)
    du = np.maximum(np.abs(flds["ux"] - flo["ux"]), np.abs(flds["uy"] - flo["uy"])).max()
    ubar = 2e-5 * max(np.abs(flo["ux"]).max(), np.abs(flo["uy"]).max(), 0.01)
    print(f"  {stats} fp32 z sweep: max |u - u_oracle| {du:.2e} (bar {ubar:.1e})")
    assert du <= ubar
    w = Q.vectors(stats)["w"][:, None, None]
    M = np.abs(fo / w).max(axis=0)
    r = (np.abs(pops - fo) / (w * M) / 1e-5).max()
    print(f"  {stats} fp32 z sweep: populations worst error / (1e-5 w_k M_cell) {r:.3f}")
    assert r <= 1.0


def test_fd_table_range_flag(rl):
    """FD fugacity beyond the tables (ln z > 12.125) is reported, not silently used."""
    nx, ny = 16, 4
    one = torch.ones((ny, nx), dtype=torch.float64)
    fields = dict(z=1e6 * one, theta=one.clone(), ux=0 * one, uy=0 * one)
    sim = rl.Sim(dict(nx=nx, ny=ny, stats="FD", precision="fp64"), {k: v.cuda() for k, v in fields.items()})
    assert sim.status() & rl.FLAG_RANGE
    with pytest.raises(rl.RlbmError):
        sim.sync()
    sim.close()


@pytest.mark.parametrize("stats", ["MJ", "FD", "BE"])
def test_fp64_large_velocity(rl, stats):
    """|u| up to 0.6: the Landau solve's start and the inversion away from the rest
    frame; tau = 1.3 keeps gamma (1 + |u|)/tau below 2."""
    nx, ny, nsteps = 67, 9, 4
    fields = workloads.smooth_random(nx, ny, seed=41, stats=stats, amp_u=0.45)
    umax = torch.sqrt(fields["ux"] ** 2 + fields["uy"] ** 2).max().item()
    print(f"  {stats}: max |u| at start {umax:.3f}")
    assert umax > 0.55
    params = dict(nx=nx, ny=ny, bc=("periodic",) * 4, tau=1.3)
    pops, flds, fo, flo = _run(rl, stats, "fp64", params, fields, nsteps)
    ctx = f"{stats} |u|<=0.6"
    _compare_pops(pops, fo, fp64_shell_bars(nsteps), ctx)
    _compare_fields(flds, flo, fp64_field_bars(nsteps), ctx)


@pytest.mark.parametrize("stats", ["MJ", "FD"])
def test_fp64_persistent_batch_kernel(rl, stats):
    """The persistent batch kernel (96 workgroups per XCD sweeping the tiles of uneven
    grids) against the oracle, every grid, every field and population."""
    specs = []
    for i, (nx, ny, bc) in enumerate([(40, 9, "periodic"), (33, 17, "open"), (70, 13, "periodic"), (16, 16, "open")]):
        f = workloads.smooth_random(nx, ny, seed=200 + i, stats=stats)
        specs.append((dict(nx=nx, ny=ny, stats=stats, precision="fp64", tau=0.7 + 0.1 * i, bc=(bc,) * 4), f))
    p, f = workloads.fourier(nx=48, ny=5, dT=0.02, tau=0.9)
    specs.append((dict(p, stats=stats, precision="fp64"), f))
    nsteps = 5
    b = rl.Batch([s[0] for s in specs], [{k: v.cuda() for k, v in s[1].items()} for s in specs])
    b.configure(32, 8, 96)
    b.step(nsteps)
    for i, (p, f) in enumerate(specs):
        print(f"[parity] persistent batch {stats} grid {i} {p['nx']}x{p['ny']}", flush=True)
        pops = rl.unpack_populations(b.state(i), "fp64", p["nx"], p["ny"]).cpu().numpy()
        flds = {k: v.cpu().numpy() for k, v in b.fields(i).items()}
        op = _oracle_params(p, stats)
        fo = _oracle_init(op, f)
        for _ in range(nsteps):
            fo, _ = L.step(fo, op)
        ctx = f"{stats} persistent grid {i}"
        _compare_pops(pops, fo, fp64_shell_bars(nsteps), ctx)
        _compare_fields(flds, L.fields(fo, op), fp64_field_bars(nsteps), ctx)
    b.close()
