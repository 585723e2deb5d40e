"""The five workloads at their own sizes and step counts, measured through the C ABI.

* FD hot spot 2048^2, 20000 steps, and BE hot spot 8192^2, 5000 steps: FP32 (fixed
  inversion start) and 16-bit deviations with the network guess against the library's
  FP64 path, which the parity tests tie to the oracle.  Norms of Sec. 3.5:
  eps_theta = sum|theta - theta_64| / sum theta_64 and eps_q = sum|q - q_64| / sum|q_64|
  over both components and the whole grid; n, eps, theta, z as max-norm relative
  errors; u as max|u - u_64| / max|u_64|.  Bar: 1e-3 on eps_theta and eps_q.
* Taylor-Green 512^2, FP32, tau in {0.6, 0.8, 1.0}, 10000 steps: the viscosity from
  the decay of sigma_{u^2} (Eq. sigma-u2) against Eq. nu-ref-eq, and away from Grad's
  tau/5.
* The 64-grid sweep in one launch per step (FP32, graph-replayed), 10000 steps: the
  viscosity of each Taylor-Green grid and the conductivity of each Fourier grid.
* The Fourier-flow set-up of Sec. 3.3 (2048 x 2, 2000 steps, five temperature
  differences, five relaxation times, FP64): the slope a of kappa g_2/g_3 = a tau.

Each run prints its numbers.  The long reference runs are tests of their own (kept in
a module cache for the tests after them), so no single test runs for minutes.
"""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import gfunc as G

pytestmark = pytest.mark.gpu

NU_OFFSET = 0.2546      # Eq. nu-ref-eq: nu = (tau - 0.2546)/4


@pytest.fixture(scope="module")
def rl():
    from paper_1709_09073_amd import rlbm
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return rlbm


def _train_net(rl, make):
    """The guess network as bench.py trains it: pairs from a 512^2 FP32 run of the same
    family (100 steps), 1000 Adam steps."""
    params, fields = make()
    sim = rl.Sim(dict(params, precision="fp32"), fields)
    sim.step(100)
    x, t = sim.inversion_samples()
    sim.close()
    net = rl.GuessNet()
    noise = torch.from_numpy(np.random.default_rng(0).standard_normal(rl.MLP_HIDDEN + 1).astype(np.float32)).cuda()
    net.init(x, t, noise)
    net.train(x, t, iters=1000, lr=3e-3)
    return net


def _run_fields(rl, params, fields, steps, label, chunk=1000):
    sim = rl.Sim(params, fields)
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        sim.step(k)
        sim.sync()
        done += k
        print(f"  [{label}] {done}/{steps} steps", flush=True)
    out = sim.fields()
    status = sim.status()
    sim.close()
    torch.cuda.synchronize()
    return out, status


def _errors(got, ref):
    th, thr = got["theta"], ref["theta"]
    out = {"eps_theta": ((th - thr).abs().sum() / thr.sum()).item(),
           "eps_q": (((got["qx"] - ref["qx"]).abs().sum() + (got["qy"] - ref["qy"]).abs().sum())
                     / (ref["qx"].abs().sum() + ref["qy"].abs().sum())).item()}
    for k in ("n", "eps", "theta", "z"):
        out[f"max_{k}"] = ((got[k] - ref[k]).abs().max() / ref[k].abs().max()).item()
    du = torch.maximum((got["ux"] - ref["ux"]).abs().max(), (got["uy"] - ref["uy"]).abs().max())
    out["max_u"] = (du / torch.maximum(ref["ux"].abs().max(), ref["uy"].abs().max())).item()
    return out


# FP64 reference fields and the trained network of each workload, filled by the
# reference tests and read by the error tests after them
_REF = {}


def _reference(rl, key, make, make_train, steps, label):
    params, fields = make()
    net = _train_net(rl, make_train)
    ref, st = _run_fields(rl, dict(params, precision="fp64"), fields, steps, f"{label} FP64")
    assert st == 0
    _REF[key] = (ref, net)


def _reduced_precision_error(rl, key, make, make_train, prec, steps, label):
    if key not in _REF:          # run alone (-k): take the reference here
        _reference(rl, key, make, make_train, steps, label)
    ref, net = _REF[key]
    params, fields = make()
    guess = "fixed" if prec == "fp32" else "mlp"
    p = dict(params, precision=prec)
    if guess == "mlp":
        p.update(guess="mlp", mlp=net.w)
    got, st = _run_fields(rl, p, fields, steps, f"{label} {prec}")
    assert st == 0
    e = _errors(got, ref)
    del got
    print(f"  {label} {prec} ({guess} guess) vs FP64 after {steps} steps: "
          + ", ".join(f"{k} {v:.2e}" for k, v in e.items()), flush=True)
    assert e["eps_theta"] <= 1e-3 and e["eps_q"] <= 1e-3, (prec, e)
    for k in ("max_n", "max_eps", "max_theta", "max_z", "max_u"):
        assert e[k] <= 1e-2, (prec, k, e[k])
    return e


FD_2048 = lambda: workloads.hotspot_fd(L=2048, device="cuda")
FD_TRAIN = lambda: workloads.hotspot_fd(L=512, seed=11, sigma=16.0, device="cuda")
BE_8192 = lambda: workloads.hotspot_be(L=8192, device="cuda")
BE_TRAIN = lambda: workloads.hotspot_be(L=512, seed=11, device="cuda")


@pytest.mark.slow
def test_fd_hotspot_2048_20k_steps_fp64_reference(rl):
    _reference(rl, "fd", FD_2048, FD_TRAIN, 20000, "FD hot spot 2048^2")


@pytest.mark.slow
@pytest.mark.parametrize("prec", ["fp32", "dev16"])
def test_fd_hotspot_2048_20k_steps_error(rl, prec):
    _reduced_precision_error(rl, "fd", FD_2048, FD_TRAIN, prec, 20000, "FD hot spot 2048^2")


@pytest.mark.slow
def test_be_hotspot_8192_5k_steps_fp64_reference(rl):
    _REF.pop("fd", None)
    torch.cuda.empty_cache()
    _reference(rl, "be", BE_8192, BE_TRAIN, 5000, "BE hot spot 8192^2")


@pytest.mark.slow
@pytest.mark.parametrize("prec", ["fp32", "dev16"])
def test_be_hotspot_8192_5k_steps_error(rl, prec):
    _reduced_precision_error(rl, "be", BE_8192, BE_TRAIN, prec, 5000, "BE hot spot 8192^2")
    if prec == "dev16":
        _REF.pop("be", None)
        torch.cuda.empty_cache()


def _decay_fit(ts, sig, L, t0, t1):
    """nu from the slope of ln sigma_{u^2} over t0 <= t <= t1 (Eq. sigma-u2)."""
    ts, sig = np.asarray(ts, dtype=np.float64), np.asarray(sig, dtype=np.float64)
    m = (ts >= t0) & (ts <= t1)
    assert m.sum() >= 5, (t0, t1)
    slope = np.polyfit(ts[m], np.log(sig[m]), 1)[0]
    return -slope * L * L / (16 * math.pi ** 2)


def _sigma_u2(f):
    u2 = f["ux"] ** 2 + f["uy"] ** 2
    return ((u2 - u2.mean()) ** 2).mean().sqrt().item()


def _tg_nu(rl, L, tau, u0, steps, every, precision, t_fit, efolds=None):
    """nu from sigma_{u^2} sampled every `every` steps, fitted from t_fit on (and, with
    efolds, only while the decay is within that many e-folding times of the Eq.
    nu-ref-eq rate, above the rounding floor)."""
    from paper_1709_09073_amd import analysis
    params, fields = workloads.taylor_green(L=L, u0=u0, tau=tau, device="cuda")
    sim = rl.Sim(dict(params, stats="MJ", precision=precision), fields)
    ts, sig = [], []
    for t in range(0, steps + 1, every):
        ts.append(t)
        sig.append(analysis.sigma_u2(sim.fields(names=("ux", "uy"))))
        if t < steps:
            sim.step(every)
    assert sim.status() == 0
    sim.close()
    t1 = steps
    if efolds is not None:
        te = L * L / (16 * math.pi ** 2 * (tau - NU_OFFSET) / 4)
        t_fit, t1 = min(t_fit, 0.5 * te), min(steps, efolds * te)
    return _decay_fit(ts, sig, L, t_fit, t1)


@pytest.mark.slow
def test_taylor_green_512_fp32_viscosity(rl):
    """Taylor-Green 512^2, FP32 populations, u0 = 0.05, 10000 steps; sigma_{u^2} every
    100 steps, fit from step 1000 on.  Measured: nu = (tau - 0.2554)/4 to 2e-4 at all
    three tau, i.e. 1.0e-3 .. 2.1e-3 below Eq. nu-ref-eq's (tau - 0.2546)/4 (whose
    offset the paper fitted over tau in [0.8, 5] with u0 = 0.1: see the next test);
    the bar is 3e-3, far from Grad's tau/5 (20-40% away)."""
    for tau in (0.6, 0.8, 1.0):
        nu = _tg_nu(rl, 512, tau, 0.05, 10000, 100, "fp32", 1000)
        paper, grad = (tau - NU_OFFSET) / 4, tau / 5
        print(f"  Taylor-Green 512^2 FP32 tau={tau}: nu={nu:.6f}, (tau - 0.2546)/4 = {paper:.6f} "
              f"(rel {nu / paper - 1:+.2e}), offset tau - 4 nu = {tau - 4 * nu:.5f}, Grad tau/5 = {grad:.4f}",
              flush=True)
        assert abs(nu / paper - 1) <= 3e-3
        assert abs(nu / grad - 1) >= 0.05


@pytest.mark.slow
def test_taylor_green_paper_setup(rl):
    """Sec. 3.2's own set-up: 512^2, u0 = 0.1, 45000 steps, relaxation times across
    [0.8, 5], FP64; the offset delta_nu of nu = (tau + delta_nu)/4 from a fit with the
    slope fixed at 1/4.  Paper (MJ): delta_nu = -0.2454 +- 0.0001."""
    taus = (0.8, 1.5, 2.5, 3.5, 5.0)
    nus = []
    for tau in taus:
        nus.append(_tg_nu(rl, 512, tau, 0.1, 45000, 100, "fp64", 5000, efolds=8))
        print(f"  Taylor-Green 512^2 u0=0.1 FP64 tau={tau}: nu={nus[-1]:.6f}, 4 nu - tau = {4 * nus[-1] - tau:.5f}",
              flush=True)
    # Eq. nu-ref-eq: nu = (tau - (1/2 + delta_nu))/4; least squares with the slope 1/4
    delta = float(np.mean(np.array(taus) - 4 * np.array(nus))) - 0.5
    slope = np.polyfit(taus, nus, 1)[0]
    print(f"  delta_nu = {delta:.5f} (paper -0.2454 +- 0.0001), free-slope fit slope {slope:.5f}", flush=True)
    assert abs(delta + 0.2454) <= 1e-3
    assert abs(slope - 0.25) <= 1e-3


def _fourier_kappa(prev, cur, nxt, margin_frac=0.125):
    """kappa = <q^x>/<F> (Eqs. qx-ft-eq, fdt-eq) over the interior of every row, with
    mean n, z and theta there.  Fields are torch (ny, nx) tensors at t - 1, t, t + 1."""
    def gu(d):
        return d["ux"] / torch.sqrt(1 - d["ux"] ** 2 - d["uy"] ** 2)

    T, ux, uy = cur["theta"], cur["ux"], cur["uy"]
    ga = 1 / torch.sqrt(1 - ux ** 2 - uy ** 2)
    dT = torch.gradient(T, dim=1)[0]
    dgu = torch.gradient(gu(cur), dim=1)[0]
    F = -((1 + ux ** 2 * ga ** 2) * dT + T * ga * ((gu(nxt) - gu(prev)) / 2 + ux * dgu))
    nx = T.shape[1]
    m = slice(int(nx * margin_frac), nx - int(nx * margin_frac))
    q, F = cur["qx"][:, m], F[:, m]
    return (q.mean() / F.mean()).item(), q.mean().item(), F.mean().item(), cur["n"][:, m].mean().item(), \
        cur["z"][:, m].mean().item()


def kappa_chapman_enskog(stats, n, z, tau):
    """Conductivity of the Anderson-Witting equation at first order in the gradients
    for the massless 2-D gas, kappa = (3/2) tau n (g_3/g_2)(3 g_1 g_3/g_2^2 - 2); for
    MJ (g_nu = z) it is (3/2) n tau."""
    g = G.g_all(stats, np.array([z]))
    g1, g2, g3 = g[0][0], g[1][0], g[2][0]
    return 1.5 * tau * n * (g3 / g2) * (3 * g1 * g3 / g2 ** 2 - 2)


@pytest.mark.slow
def test_batch_64_transport_10k_steps(rl):
    """The 64-grid sweep, FP32, one launch per step, graph-replayed, 10000 steps: nu of
    every Taylor-Green grid from its own decay window and kappa of every Fourier grid
    at the end against 1.5 n tau (MJ)."""
    import bench
    from paper_1709_09073_amd import analysis
    plist, flist = bench.build_batch("cuda")
    for p in plist:
        p["precision"] = "fp32"
    b = rl.Batch(plist, flist)
    print(f"  [batch 64] status after init 0x{b.status():x}", flush=True)
    tile = b.autotune(trial_steps=3)
    print(f"  [batch 64] tile {tile}, status after autotune 0x{b.status():x}", flush=True)
    b.capture()
    steps = 10000
    tg = [g for g, p in enumerate(plist) if p["bc"][0] == "periodic"]
    fo = [g for g, p in enumerate(plist) if p["bc"][0] == "wall"]
    ts, sig = [], {g: [] for g in tg}
    t = 0
    while True:
        ts.append(t)
        for g in tg:
            sig[g].append(_sigma_u2(b.fields(g, names=("ux", "uy"), check=False)))
        st = b.status()
        if st:
            print(f"  [batch 64] status 0x{st:x} at step {t}", flush=True)
        assert st == 0
        if t >= steps - 1:
            break
        k = 10 if t < 1000 else 100
        k = min(k, steps - 1 - t)
        b.step(k)
        t += k
        if t % 2000 == 0:
            print(f"  [batch 64] {t}/{steps} steps", flush=True)
    prev = {g: b.fields(g) for g in fo}
    b.step(1)
    cur = {g: b.fields(g) for g in fo}
    b.step(1)
    nxt = {g: b.fields(g) for g in fo}
    assert b.status() == 0
    b.close()
    nu_err, ka_err = [], []
    for g in tg:
        L, tau = plist[g]["nx"], plist[g]["tau"]
        paper = (tau - NU_OFFSET) / 4
        te = L * L / (16 * math.pi ** 2 * paper)           # e-folding time of sigma_{u^2}
        nu = _decay_fit(ts, sig[g], L, min(1000, 0.5 * te), min(steps - 1, 4 * te))
        nu_err.append(nu / paper - 1)
        print(f"  grid {g:2d} Taylor-Green L={L} tau={tau:.4f}: nu={nu:.6f} paper {paper:.6f} "
              f"rel {nu / paper - 1:+.2e}", flush=True)
    for g in fo:
        tau = plist[g]["tau"]
        kappa, q, F, n, z = _fourier_kappa(prev[g], cur[g], nxt[g])
        ce = kappa_chapman_enskog("MJ", n, z, tau)
        ka_err.append(kappa / ce - 1)
        print(f"  grid {g:2d} Fourier {plist[g]['nx']}x{plist[g]['ny']} tau={tau:.4f}: kappa={kappa:.6f} "
              f"1.5 n tau = {ce:.6f} rel {kappa / ce - 1:+.2e} (1.5 tau: {1.5 * tau:.6f})", flush=True)
    print(f"  batch 64 (tile {tile}): |nu/paper - 1| max {np.abs(nu_err).max():.2e} over {len(tg)} grids, "
          f"|kappa/(1.5 n tau) - 1| max {np.abs(ka_err).max():.2e} over {len(fo)} grids", flush=True)
    assert np.abs(nu_err).max() <= 1e-2
    assert np.abs(ka_err).max() <= 1e-2


@pytest.mark.parametrize("stats", ["MJ", "FD", "BE"])
def test_fourier_flow_paper_setup(rl, stats):
    """Sec. 3.3: 2048 x 2, n0 = 1, u0 = 0, linear initial theta between walls at
    1 -/+ dT/2, dT in {5, 7.5, 10, 12.5, 15} x 1e-4, 2000 steps, FP64; kappa per tau
    is the slope of <q^x> against <F>; a is the slope of kappa g_2/g_3 against tau
    through the origin.  MJ: a = 1.5 (the paper's 1.4999998 +- 2e-7).  FD, BE: the
    slope follows the Anderson-Witting conductivity at the run's mean n and z (the
    paper prints 1.5 for them too; the method gives 1.416 and 1.596 at n0 = 1).
    The paper does not list its five relaxation times; these span 0.6 .. 1.5.  At
    larger tau the 2000-step value carries an oscillation of the start-up flow: at
    tau = 3 it is +1.7e-5 after 2000 steps and -1.7e-5 after 6000 (printed below)."""
    taus = (0.6, 0.8, 1.0, 1.2, 1.5)
    dTs = (5.0e-4, 7.5e-4, 10.0e-4, 12.5e-4, 15.0e-4)
    specs = []
    for tau in taus:
        for dT in dTs:
            p, f = workloads.fourier(nx=2048, ny=2, dT=dT, tau=tau, device="cuda")
            specs.append((dict(p, stats=stats, precision="fp64"), f))
    b = rl.Batch([s[0] for s in specs], [s[1] for s in specs])
    b.step(1999)
    prev = [b.fields(i) for i in range(len(specs))]
    b.step(1)
    cur = [b.fields(i) for i in range(len(specs))]
    b.step(1)
    nxt = [b.fields(i) for i in range(len(specs))]
    assert b.status() == 0
    b.close()
    ys, predicted = [], []
    for it, tau in enumerate(taus):
        qs, Fs, ns, zs = [], [], [], []
        for jd in range(len(dTs)):
            i = it * len(dTs) + jd
            _, q, F, n, z = _fourier_kappa(prev[i], cur[i], nxt[i])
            qs.append(q)
            Fs.append(F)
            ns.append(n)
            zs.append(z)
        kappa = np.polyfit(Fs, qs, 1)[0]
        n, z = float(np.mean(ns)), float(np.mean(zs))
        g = G.g_all(stats, np.array([z]))
        ys.append(kappa * g[1][0] / g[2][0])
        predicted.append(kappa_chapman_enskog(stats, n, z, tau) * g[1][0] / g[2][0])
        print(f"  {stats} tau={tau}: kappa={kappa:.8f} kappa g2/g3 / tau = {ys[-1] / tau:.8f} "
              f"(Anderson-Witting {predicted[-1] / tau:.8f}), n={n:.6f} z={z:.6f}", flush=True)
    taus_a = np.array(taus)
    a = float(np.dot(taus_a, ys) / np.dot(taus_a, taus_a))
    a_ce = float(np.dot(taus_a, predicted) / np.dot(taus_a, taus_a))
    print(f"  {stats}: a = {a:.8f} (paper {dict(MJ=1.4999998, FD=1.4999998, BE=1.4999997)[stats]}; "
          f"Anderson-Witting at this n, z: {a_ce:.8f})", flush=True)
    if stats == "MJ":
        assert abs(a - 1.5) <= 1e-5
    assert abs(a / a_ce - 1) <= 1e-5
    if stats == "MJ":
        dev = []
        for nsteps in (2000, 6000):
            p, f = workloads.fourier(nx=2048, ny=2, dT=1e-3, tau=3.0, device="cuda")
            s = rl.Sim(dict(p, stats="MJ", precision="fp64"), f)
            s.step(nsteps - 1)
            a0 = s.fields()
            s.step(1)
            a1 = s.fields()
            s.step(1)
            a2 = s.fields()
            s.close()
            kappa = _fourier_kappa(a0, a1, a2)[0]
            dev.append(kappa / 4.5 - 1)
            print(f"  MJ tau=3 after {nsteps} steps: kappa / (1.5 tau) - 1 = {dev[-1]:+.2e}", flush=True)
        assert max(abs(d) for d in dev) < 1e-4
