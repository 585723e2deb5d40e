"""Batched uneven grids (one persistent launch per step), graph replay of step chunks,
the tile autotuner, and the transport relations measured on the GPU path."""
import math

import numpy as np
import pytest
import torch

import workloads
from conftest import same_bits
from oracle import lattice as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rl():
    from paper_1709_09073_amd import rlbm
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return rlbm


def _grids(stats="MJ", precision="fp64"):
    out = []
    for i, (nx, ny, bc) in enumerate([(40, 9, "periodic"), (33, 17, "open"), (70, 13, "periodic"),
                                      (16, 16, "open"), (65, 6, "periodic")]):
        f = workloads.smooth_random(nx, ny, seed=100 + i, stats=stats)
        out.append((dict(nx=nx, ny=ny, stats=stats, precision=precision, tau=0.7 + 0.1 * i,
                         bc=(bc,) * 4), f))
    p, f = workloads.fourier(nx=48, ny=5, dT=0.02, tau=0.9)
    out.append((dict(p, stats=stats, precision=precision), f))
    return out


def test_batch_matches_single_grids(rl):
    grids = _grids()
    print("[batch] 6 uneven grids vs single-grid contexts, 10 steps", flush=True)
    b = rl.Batch([g[0] for g in grids], [{k: v.cuda() for k, v in g[1].items()} for g in grids])
    b.step(10)
    for i, (p, f) in enumerate(grids):
        s = rl.Sim(p, {k: v.cuda() for k, v in f.items()})
        s.step(10)
        a, c = b.state(i), s.state()
        err = (a - c).abs().max().item() / c.abs().max().item()
        assert err <= 1e-15, (i, err)
        s.close()
    b.close()


def test_batch_parity_with_oracle(rl):
    grids = _grids()[:2] + _grids()[-1:]
    b = rl.Batch([g[0] for g in grids], [{k: v.cuda() for k, v in g[1].items()} for g in grids])
    b.step(5)
    for i, (p, f) in enumerate(grids):
        op = L.Params(stats="MJ", nx=p["nx"], ny=p["ny"], tau=p["tau"],
                      bc=dict(zip(("xlo", "xhi", "ylo", "yhi"), p["bc"])),
                      theta_wall=dict(zip(("xlo", "xhi"), p.get("theta_wall", (1.0, 1.0)))))
        fo = L.init_state(op, f["theta"].numpy(), f["ux"].numpy(), f["uy"].numpy(),
                          n=f["n"].numpy() if "n" in f else None, z=f["z"].numpy() if "z" in f else None)
        for _ in range(5):
            fo, _ = L.step(fo, op)
        ref = L.fields(fo, op)
        got = {k: v.cpu().numpy() for k, v in b.fields(i).items()}
        for k in ("n", "eps", "theta"):
            err = np.abs(got[k] - ref[k]).max() / np.abs(ref[k]).max()
            assert err <= 1e-12, (i, k, err)
    b.close()


def test_graph_replay_matches_eager(rl):
    """Runs of >= 64 steps replay captured 32-step graphs; every replay block is checked
    against eager single-step launches, with eager work and syncs in between."""
    p, f = workloads.smooth_random(50, 11, seed=7, stats="FD"), None
    params = dict(nx=50, ny=11, stats="FD", precision="fp32", tau=0.8)
    a = rl.Sim(params, {k: v.cuda() for k, v in p.items()})
    e = rl.Sim(params, {k: v.cuda() for k, v in p.items()})
    for rep in range(3):
        a.step(64)                      # two graph replays
        for _ in range(64):
            e.step(1)                   # eager launches
        fa = a.fields()                 # eager work between replays
        torch.cuda.synchronize()
        assert same_bits(a.state(), e.state()), rep
        assert torch.equal(fa["theta"], e.fields()["theta"]), rep
    a.close()
    e.close()


def test_batch_graph_replay_matches_eager(rl):
    grids = _grids(precision="fp32")
    mk = lambda: rl.Batch([g[0] for g in grids], [{k: v.cuda() for k, v in g[1].items()} for g in grids])
    a, e = mk(), mk()
    for rep in range(2):
        a.step(96)
        for _ in range(96):
            e.step(1)
        for i in range(len(grids)):
            assert same_bits(a.state(i), e.state(i)), (rep, i)
    a.close()
    e.close()


def test_autotune_keeps_results(rl):
    grids = _grids(precision="fp32")
    mk = lambda: rl.Batch([g[0] for g in grids], [{k: v.cuda() for k, v in g[1].items()} for g in grids])
    a = mk()
    tx, ty = a.autotune(trial_steps=2)
    assert tx * ty == 256
    n_done = a.steps_done
    ref = mk()
    ref.step(n_done)
    for i in range(len(grids)):
        assert same_bits(a.state(i), ref.state(i)), i
    a.close()
    ref.close()


def test_taylor_green_viscosity_on_gpu(rl):
    """nu = (tau - 0.2546)/4 (Sec. 3.2) from a batch of Taylor-Green grids, FP64."""
    from paper_1709_09073_amd import analysis
    Ls, taus = (64, 96), (0.6, 1.0)
    specs = []
    for Lg, tau in zip(Ls, taus):
        p, f = workloads.taylor_green(L=Lg, u0=0.05, tau=tau)
        specs.append((dict(p, stats="MJ", precision="fp64"), f))
    b = rl.Batch([s[0] for s in specs], [{k: v.cuda() for k, v in s[1].items()} for s in specs])
    rate = min(16 * math.pi ** 2 * (t - 0.2546) / 4 / Lg ** 2 for Lg, t in zip(Ls, taus))
    nsteps = int(3 / rate)
    every = nsteps // 30
    ts, sig = [], [[] for _ in specs]
    for t in range(0, nsteps + 1, every):
        if t >= nsteps // 5:
            ts.append(t)
            for i in range(len(specs)):
                sig[i].append(analysis.sigma_u2(b.fields(i, names=("ux", "uy"))))
        b.step(every)
    for i, (Lg, tau) in enumerate(zip(Ls, taus)):
        nu = analysis.viscosity_from_decay(ts, sig[i], Lg)
        paper = (tau - 0.2546) / 4
        print(f"  L={Lg} tau={tau}: nu={nu:.5f} paper {paper:.5f} Grad {tau / 5:.5f}")
        assert abs(nu / paper - 1) < 0.01
        assert abs(nu / (tau / 5) - 1) > 0.05
    b.close()


def test_fourier_conductivity_on_gpu(rl):
    """kappa = 1.5 tau g_3/g_2 (Sec. 3.3; MJ: 1.5 tau) from Fourier-flow grids, FP64."""
    from paper_1709_09073_amd import analysis
    taus = (0.8, 1.5)
    specs = []
    for tau in taus:
        p, f = workloads.fourier(nx=128, ny=2, dT=1e-3, tau=tau)
        specs.append((dict(p, stats="MJ", precision="fp64"), f))
    b = rl.Batch([s[0] for s in specs], [{k: v.cuda() for k, v in s[1].items()} for s in specs])
    b.step(299)
    prev = [b.fields(i) for i in range(2)]
    b.step(1)
    cur = [b.fields(i) for i in range(2)]
    b.step(1)
    nxt = [b.fields(i) for i in range(2)]
    for i, tau in enumerate(taus):
        kappa = analysis.conductivity(prev[i], cur[i], nxt[i])
        print(f"  tau={tau}: kappa={kappa:.6f} paper {1.5 * tau:.6f} Grad {0.375 * tau:.6f}")
        assert abs(kappa / (1.5 * tau) - 1) < 2e-3
    b.close()


TILES = [(32, 8), (64, 4), (128, 2), (256, 1), (16, 16)]


@pytest.mark.parametrize("precision", ["fp64", "fp32", "dev16"])
@pytest.mark.parametrize("nx", [37, 33])
def test_results_do_not_depend_on_the_tile(rl, precision, nx):
    """Every cell's update is the same arithmetic whatever tile covers it: each tile
    shape (ragged in x and y on these nx x 11 grids, walls on x) gives the same bits.
    For 16-bit deviations the tiles with at most 512 halo cells take the staged pull
    and the others the direct one; at nx = 33 a 32-wide tile starts at the hot wall
    cell, whose stencil lies outside its halo and is pulled directly."""
    p, f = workloads.fourier(nx=nx, ny=11, dT=0.04, tau=0.85)
    p = dict(p, stats="FD", precision=precision)
    f = workloads.smooth_random(nx, 11, seed=21, stats="FD", amp_u=0.1)
    print(f"[tiles] FD {nx}x11 walls {precision}: {len(TILES)} tile shapes, 7 steps", flush=True)
    ref = None
    for t in TILES:
        s = rl.Sim(dict(p, tile=t), {k: v.cuda() for k, v in f.items()})
        s.step(7)
        st = s.state().clone()
        assert s.status() == 0
        s.close()
        if ref is None:
            ref = st
        else:
            assert same_bits(st, ref), t


@pytest.mark.parametrize("stats", ["MJ", "FD"])
@pytest.mark.parametrize("precision", ["fp32", "dev16"])
def test_batch_launch_modes_agree(rl, precision, stats):
    """One workgroup per tile and the persistent sweep, for every tile shape, give the
    same bits, and so does a single-grid context: the modes are separate kernels (their
    own register budgets and instruction schedules) over the same arithmetic, and a*b + c
    is fused only within one source expression, so no kernel rounds differently.  (FD:
    the inversion keeps a table row in registers between evaluations in every kernel.)"""
    grids = _grids(stats=stats, precision=precision)
    b = rl.Batch([g[0] for g in grids], [{k: v.cuda() for k, v in g[1].items()} for g in grids])
    b.step(5)
    saved = [b.state(i).clone() for i in range(len(grids))]
    ref = {}
    print(f"[batch] {stats} {precision}: {len(TILES)} tile shapes x 2 launch modes, 4 steps", flush=True)
    for persistent in (0, 96):
        for t in TILES:
            for i in range(len(grids)):
                b.state(i).copy_(saved[i])
            b.configure(t[0], t[1], persistent)
            b.step(4)
            out = [b.state(i).clone() for i in range(len(grids))]
            if persistent not in ref:
                ref[persistent] = out
            else:
                for i in range(len(grids)):
                    assert same_bits(out[i], ref[persistent][i]), (t, persistent, i)
    for i in range(len(grids)):
        assert same_bits(ref[0][i], ref[96][i]), i
    b.close()
    for i, (p, f) in enumerate(grids):
        s = rl.Sim(p, {k: v.cuda() for k, v in f.items()})
        s.step(9)
        assert same_bits(s.state(), ref[96][i]), ("single grid", i)
        s.close()


@pytest.mark.parametrize("precision", ["fp32", "dev16"])
@pytest.mark.parametrize("nx,ny,bc", [(2, 2, "periodic"), (5, 3, "periodic"), (3, 7, "open"), (70, 2, "periodic"),
                                      (2, 19, "open")])
def test_small_grids_every_tile(rl, precision, nx, ny, bc):
    """Grids smaller than a tile, or one tile row or column thin: the halo positions
    wrap (periodic) or clamp (open) past both edges at once, every tile shape gives the
    same bits, and FP32 fields match the oracle to the FP32 bars."""
    f = workloads.smooth_random(nx, ny, seed=nx * 31 + ny, stats="FD", amp_u=0.1)
    params = dict(nx=nx, ny=ny, stats="FD", precision=precision, tau=0.9, bc=(bc,) * 4)
    print(f"[small] FD {nx}x{ny} {bc} {precision}: {len(TILES)} tile shapes, 5 steps", flush=True)
    ref, fields = None, None
    for t in TILES:
        s = rl.Sim(dict(params, tile=t), {k: v.cuda() for k, v in f.items()})
        s.step(5)
        st = s.state().clone()
        assert s.status() == 0
        if ref is None:
            ref, fields = st, {k: v.cpu().numpy() for k, v in s.fields().items()}
        else:
            assert same_bits(st, ref), t
        s.close()
    if precision == "fp32":
        op = L.Params(stats="FD", nx=nx, ny=ny, tau=0.9, bc=dict(xlo=bc, xhi=bc, ylo=bc, yhi=bc))
        fo = L.init_state(op, f["theta"].numpy(), f["ux"].numpy(), f["uy"].numpy(), z=f["z"].numpy())
        for _ in range(5):
            fo, _ = L.step(fo, op)
        want = L.fields(fo, op)
        for key, tol in (("n", 2e-6), ("eps", 2e-6), ("theta", 2e-6), ("z", 5e-6)):
            err = np.abs(fields[key] - want[key]).max() / np.abs(want[key]).max()
            assert err <= tol, (key, err)
