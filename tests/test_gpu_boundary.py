"""The C ABI's outputs and error paths on the GPU: raw moments N^mu, T^{mu nu} against
the oracle, the check mode (RLBM_ENONFINITE from a non-finite population put in from the
host), the stability rejection at init, and the inversion counters after autotuning."""
import ctypes

import numpy as np
import pytest
import torch

import workloads
from oracle import lattice as L
from parity_bars import field_bar

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rl():
    from paper_1709_09073_amd import rlbm
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return rlbm


@pytest.mark.parametrize("stats,precision", [("MJ", "fp64"), ("FD", "fp64"), ("BE", "fp64"), ("FD", "fp32")])
def test_raw_moments_match_the_oracle(rl, stats, precision):
    """N^mu and T^{mu nu} of the populations the next step would see (streamed state),
    Sec. 2.4: FP64 to the FP64 parity bar of eps after three steps, relative to N^0 /
    T^00; FP32 populations to 2e-7."""
    nx, ny, nsteps = 37, 9, 3
    fields = workloads.smooth_random(nx, ny, seed=61, stats=stats)
    params = dict(nx=nx, ny=ny, stats=stats, precision=precision, tau=0.9, bc=("open",) * 4)
    sim = rl.Sim(params, {k: v.cuda() for k, v in fields.items()})
    sim.step(nsteps)
    got = {k: v.cpu().numpy() for k, v in sim.fields(names=rl.MOMENT_NAMES).items()}
    sim.close()
    op = L.Params(stats=stats, nx=nx, ny=ny, tau=0.9, bc=dict(xlo="open", xhi="open", ylo="open", yhi="open"))
    f0 = {k: v.numpy() for k, v in fields.items()}
    f = L.init_state(op, f0["theta"], f0["ux"], f0["uy"], z=f0["z"])
    for _ in range(nsteps):
        f, _ = L.step(f, op)
    N, T = L.moments(L.stream(f, op), stats)
    ref = dict(N0=N[0], Nx=N[1], Ny=N[2], T00=T[0, 0], T0x=T[0, 1], T0y=T[0, 2], Txx=T[1, 1], Txy=T[1, 2], Tyy=T[2, 2])
    bar = field_bar("eps", nsteps) if precision == "fp64" else 2e-7
    for k, v in ref.items():
        scale = np.abs(ref["N0" if k.startswith("N") else "T00"]).max()
        err = np.abs(got[k] - v).max() / scale
        print(f"  {stats} {precision}: {k} err {err:.2e} (bar {bar:.0e})")
        assert err <= bar, (k, err)
    # the tensor is traceless: T^00 = T^xx + T^yy
    assert np.abs(got["T00"] - got["Txx"] - got["Tyy"]).max() <= 4 * bar * np.abs(ref["T00"]).max()


@pytest.mark.parametrize("check", [True, False])
def test_nonfinite_population_reported(rl, check):
    """A NaN written into one population from the host: the next step reports
    RLBM_ENONFINITE, at once in check mode, at the next sync otherwise."""
    nx, ny = 24, 6
    fields = workloads.smooth_random(nx, ny, seed=3, stats="FD")
    sim = rl.Sim(dict(nx=nx, ny=ny, stats="FD", precision="fp64", tau=0.9, check=check),
                 {k: v.cuda() for k, v in fields.items()})
    sim.step(2)
    f = sim.populations()
    f[13, 3, 7] = float("nan")
    sim.set_populations(f)
    rc = rl.lib().rlbm_step(sim.ctx, 1)
    if check:
        assert rc == rl.RLBM_ENONFINITE
    else:
        assert rc == rl.RLBM_OK
        assert sim.status() & rl.FLAG_NONFINITE
        assert rl.lib().rlbm_sync(sim.ctx) == rl.RLBM_ENONFINITE
    assert sim.status() == 0          # reported once, then cleared
    sim.close()


def test_check_mode_passes_clean_steps(rl):
    fields = workloads.smooth_random(24, 6, seed=4, stats="BE")
    sim = rl.Sim(dict(nx=24, ny=6, stats="BE", precision="fp32", tau=0.9, check=True),
                 {k: v.cuda() for k, v in fields.items()})
    assert rl.lib().rlbm_step(sim.ctx, 70) == rl.RLBM_OK   # graph replay plus single launches
    sim.close()


def test_unstable_relaxation_rejected(rl):
    """tau <= gamma (1 + |u|)/2 somewhere in the initial state: rlbm_init returns
    RLBM_EINVAL and no context; a slightly larger tau is accepted."""
    nx, ny = 16, 4
    one = torch.ones((ny, nx), dtype=torch.float64)
    ux = 0 * one
    ux[2, 5] = 0.3                              # gamma (1 + 0.3)/2 = 0.6814
    fields = dict(n=one.clone(), theta=one.clone(), ux=ux, uy=0 * one)
    with pytest.raises(rl.RlbmError) as e:
        rl.Sim(dict(nx=nx, ny=ny, stats="MJ", precision="fp64", tau=0.68), {k: v.cuda() for k, v in fields.items()})
    assert e.value.code == rl.RLBM_EINVAL
    sim = rl.Sim(dict(nx=nx, ny=ny, stats="MJ", precision="fp64", tau=0.69), {k: v.cuda() for k, v in fields.items()})
    assert sim.status() == 0
    sim.close()
    # tau = tau_a / theta + tau_b: checked with each cell's own theta
    th = one.clone()
    th[1, 1] = 4.0                               # tau = 0.2/4 + 0.45 = 0.5 there
    fields = dict(n=one.clone(), theta=th, ux=0 * one, uy=0 * one)
    with pytest.raises(rl.RlbmError):
        rl.Sim(dict(nx=nx, ny=ny, stats="MJ", precision="fp32", tau_mode="theta", tau_a=0.2, tau_b=0.45),
               {k: v.cuda() for k, v in fields.items()})


def test_inversion_counters_after_autotune(rl):
    """After rlbm_autotune the counters restart: K steps give K x cells solves and
    between 1 and 10 Newton iterations per solve."""
    nx = ny = 64
    fields = workloads.smooth_random(nx, ny, seed=5, stats="FD")
    sim = rl.Sim(dict(nx=nx, ny=ny, stats="FD", precision="fp32", tau=0.9, collect_stats=True),
                 {k: v.cuda() for k, v in fields.items()})
    sim.step(3)
    sim.autotune(trial_steps=2)
    it0, so0 = sim.inversion_stats()
    assert it0 == 0 and so0 == 0
    sim.step(7)
    it, so = sim.inversion_stats()
    print(f"  after autotune + 7 steps: {it} iterations over {so} solves ({it / so:.2f} per solve)")
    assert so == 7 * nx * ny
    assert so <= it <= 10 * so
    sim.close()
