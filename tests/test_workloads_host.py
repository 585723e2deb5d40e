"""The seeded synthetic inputs have the shapes, ranges and structure their recipes
state (the paper's workloads are formula-defined initial-value problems), and the
same seed gives the same fields."""
import math

import numpy as np
import torch

import workloads


def test_fd_hotspot_recipe():
    p, f = workloads.hotspot_fd(L=256, sigma=8.0)
    assert (p["nx"], p["ny"], p["stats"], p["tau_mode"], p["tau_a"], p["tau_b"]) == (256, 256, "FD", "theta", 2.0, 0.2546)
    assert p["bc"] == ("open",) * 4
    th, z = f["theta"].numpy(), f["z"].numpy()
    assert th.shape == (256, 256) and th.dtype == np.float64
    assert abs(th.max() - 1.3) < 1e-12 and abs(th[128, 128] - 1.3) < 1e-12   # peak at the centre
    assert th.min() >= 1.0 and abs(th[0, 0] - 1.0) < 1e-12
    assert abs(z.min() - 0.5) < 1e-12 and abs(z.max() - 2.0) < 1e-12       # z = 0.5 * 4^s, s in [0, 1]
    assert not f["ux"].any() and not f["uy"].any()


def test_be_hotspot_recipe():
    p, f = workloads.hotspot_be(L=512)
    assert (p["stats"], p["tau_mode"], p["bc"]) == ("BE", "theta", ("open",) * 4)
    z, th = f["z"].numpy(), f["theta"].numpy()
    assert z.min() >= 0.2 and z.max() <= 0.9
    assert th.min() >= 0.5
    assert abs(np.median(z) - 0.55) < 0.05      # the background between the bumps
    assert th.max() > 1.05                      # some bumps are hot


def test_taylor_green_recipe():
    u0 = 0.05
    p, f = workloads.taylor_green(L=64, u0=u0, tau=0.8)
    ux, uy = f["ux"].numpy(), f["uy"].numpy()
    assert abs(np.abs(ux).max() - u0) < 1e-12 and abs(np.abs(uy).max() - u0) < 1e-12
    # divergence-free on the continuum field: d ux/dx + d uy/dy = 0 (spectral derivative)
    k = 2 * np.pi * np.fft.fftfreq(64)
    div = np.fft.ifft2(1j * k[None, :] * np.fft.fft2(ux) + 1j * k[:, None] * np.fft.fft2(uy)).real
    assert np.abs(div).max() < 1e-12
    assert p["bc"] == ("periodic",) * 4 and p["tau"] == 0.8


def test_riemann_recipe():
    p, f = workloads.riemann()
    n = f["n"].numpy()
    assert n.shape == (4, 1024)
    assert (n[:, :512] == 1.0).all() and (n[:, 512:] == 0.139).all()
    assert p["bc"] == ("open", "open", "periodic", "periodic") and p["tau"] == 0.9


def test_batch_specs_recipe():
    specs = workloads.batch_specs(seed=3)
    assert len(specs) == 64
    assert [s["kind"] for s in specs] == ["taylor_green", "fourier"] * 32
    for s in specs:
        assert s["nx"] % 16 == 0 and 64 <= s["nx"] <= 512 and s["ny"] % 16 == 0 and 64 <= s["ny"] <= 512
        assert 0.55 <= s["tau"] <= 1.5
        if s["kind"] == "taylor_green":
            assert s["nx"] == s["ny"]
    cells = sum(s["nx"] * s["ny"] for s in specs)
    assert 5e6 < cells < 8e6                     # about 6.6 M cells


def test_poiseuille_and_shear_recipes():
    p, f = workloads.poiseuille(L=16, nx=4, a=1e-8, tau=3.0)
    assert (p["nx"], p["ny"]) == (4, 17) and p["force"] == (1e-8, 0.0)
    assert p["bc"] == ("periodic", "periodic", "wall_neq", "wall_neq")
    p, f = workloads.shear_wave(L=32, u0=1e-4)
    ux = f["ux"].numpy()[:, 0]
    assert np.allclose(ux, 1e-4 * np.sin(2 * math.pi * np.arange(32) / 32), rtol=0, atol=1e-18)


def test_same_seed_same_fields():
    a = workloads.smooth_random(30, 20, seed=9, stats="BE")
    b = workloads.smooth_random(30, 20, seed=9, stats="BE")
    c = workloads.smooth_random(30, 20, seed=10, stats="BE")
    for k in a:
        assert torch.equal(a[k], b[k])
    assert not torch.equal(a["theta"], c["theta"])
    assert a["z"].min() >= 0.3 and a["z"].max() <= 0.9 + 1e-12
