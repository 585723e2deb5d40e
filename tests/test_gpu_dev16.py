"""16-bit deviation storage (RLBM_DEV16): populations stored as SNORM16 deviations
from a per-cell dipole reference with a scale per radial shell.  Checked
against the FP64 oracle (fields after a few steps), against the library's own FP64
path on the hot spot with the paper's error norms (Sec. 3.5: eps_theta, eps_q), and
its storage layout decoded on the host."""
import numpy as np
import pytest
import torch

import workloads
from conftest import same_bits
from dev16 import decode, decode_bound
from oracle import lattice as L
from oracle import quadrature as Q

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rl():
    from paper_1709_09073_amd import rlbm
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return rlbm


WALLS = dict(bc=("wall", "wall", "open", "open"), theta_wall=(0.93, 1.06), tau_mode="theta", tau_a=0.5, tau_b=0.6)


@pytest.mark.parametrize("stats,nsteps,setup", [("MJ", 6, "periodic"), ("FD", 4, "periodic"), ("BE", 4, "periodic"),
                                                ("MJ", 5, "walls"), ("FD", 4, "walls"), ("BE", 4, "walls")])
def test_dev16_against_oracle(rl, stats, nsteps, setup):
    nx, ny = 70, 13
    fields = workloads.smooth_random(nx, ny, seed=31, stats=stats)
    extra = WALLS if setup == "walls" else {}
    print(f"[dev16] {stats} {nx}x{ny} {setup} {nsteps} steps vs oracle", flush=True)
    sim = rl.Sim(dict(nx=nx, ny=ny, stats=stats, precision="dev16", tau=0.9, **extra),
                 {k: v.cuda() for k, v in fields.items()})
    # the initial state decodes to the equilibrium within the coding bound (codes off
    # by 0.6 of a SNORM16 step at most, plus the encoder's conserving correction of
    # rho, alpha, beta; dev16.decode_bound), plus FP32 rounding of f_eq
    f0 = decode(rl, sim.state(), nx, ny, stats)
    if setup == "walls":
        op = L.Params(stats=stats, nx=nx, ny=ny, tau_mode="theta", tau_a=0.5, tau_b=0.6,
                      bc=dict(zip(("xlo", "xhi", "ylo", "yhi"), WALLS["bc"])),
                      theta_wall=dict(xlo=WALLS["theta_wall"][0], xhi=WALLS["theta_wall"][1]))
    else:
        op = L.Params(stats=stats, nx=nx, ny=ny, tau=0.9)
    ref0 = L.init_state(op, fields["theta"].numpy(), fields["ux"].numpy(), fields["uy"].numpy(), z=fields["z"].numpy())
    bound = decode_bound(rl, sim.state(), nx, ny, stats) + 2e-6 * np.abs(ref0)
    worst = (np.abs(f0 - ref0) / bound).max()
    print(f"  {stats}: initial decode error / bound = {worst:.2f}")
    assert worst <= 1.0
    # the encoder keeps each shell's sum over the 12 directions (so N^0 and T^00) and the
    # momentum density T^{0x}, T^{0y}: they agree with the oracle's equilibrium to FP32
    # rounding, far below what the code steps alone would leave
    v = Q.vectors(stats)
    pc = (v["p0"] ** 2 * v["vx"])[:, None, None]
    ps = (v["p0"] ** 2 * v["vy"])[:, None, None]
    shell = lambda a: a.reshape(12, 6, ny, nx).sum(0)
    for name, got0, want0, scale0 in (
            ("shell sums", shell(f0), shell(ref0), shell(np.abs(ref0))),
            ("T^0x", (pc * f0).sum(0), (pc * ref0).sum(0), (np.abs(pc * ref0)).sum(0)),
            ("T^0y", (ps * f0).sum(0), (ps * ref0).sum(0), (np.abs(ps * ref0)).sum(0))):
        rel = (np.abs(got0 - want0) / scale0).max()
        print(f"  {stats}: {name} of the decoded state: {rel:.2e} relative", flush=True)
        assert rel <= 2e-6, (name, rel)
    sim.step(nsteps)
    got = {k: v.cpu().numpy() for k, v in sim.fields().items()}
    sim.close()
    f = ref0
    for _ in range(nsteps):
        f, _ = L.step(f, op)
    ref = L.fields(f, op)
    for key, tol in (("n", 2e-4), ("eps", 2e-4), ("theta", 2e-4), ("ux", 5e-4), ("uy", 5e-4)):
        scale = max(np.abs(ref[key]).max(), 0.01)
        err = np.abs(got[key] - ref[key]).max() / scale
        print(f"  {stats} {key}: {err:.2e}")
        assert err <= tol, (key, err)


def test_dev16_hotspot_error_norms(rl):
    """Fermi-Dirac hot spot (256^2, amp 0.3, sigma 8), 400 steps: DEV16 and FP32
    against the FP64 path of the same library, with the paper's norms
    eps_theta = sum|dtheta| / sum theta and eps_q = sum|dq| / sum|q|."""
    params, fields = workloads.hotspot_fd(L=256, seed=4, sigma=8.0)
    out = {}
    for prec in ("fp64", "fp32", "dev16"):
        sim = rl.Sim(dict(params, precision=prec), {k: v.cuda() for k, v in fields.items()})
        sim.step(400)
        out[prec] = {k: v.cpu().numpy() for k, v in sim.fields().items()}
        sim.close()
    ref = out["fp64"]
    for prec in ("fp32", "dev16"):
        r = out[prec]
        et = np.abs(r["theta"] - ref["theta"]).sum() / ref["theta"].sum()
        eq = (np.abs(r["qx"] - ref["qx"]).sum() + np.abs(r["qy"] - ref["qy"]).sum()) / \
             (np.abs(ref["qx"]).sum() + np.abs(ref["qy"]).sum())
        print(f"  {prec}: eps_theta {et:.2e}  eps_q {eq:.2e}")
        assert et <= 1e-3 and eq <= 1e-3, (prec, et, eq)


def test_dev16_batch_matches_single(rl):
    specs = [(dict(nx=40, ny=9, stats="FD", precision="dev16", tau=0.8), workloads.smooth_random(40, 9, 1, "FD")),
             (dict(nx=33, ny=17, stats="FD", precision="dev16", tau=1.1, bc=("open",) * 4),
              workloads.smooth_random(33, 17, 2, "FD"))]
    b = rl.Batch([s[0] for s in specs], [{k: v.cuda() for k, v in s[1].items()} for s in specs])
    b.step(7)
    for i, (p, f) in enumerate(specs):
        s = rl.Sim(p, {k: v.cuda() for k, v in f.items()})
        s.step(7)
        assert same_bits(b.state(i), s.state()), i
        s.close()
    b.close()
