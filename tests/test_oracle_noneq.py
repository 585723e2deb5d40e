"""The oracle's non-equilibrium tensors pi^{x..x} of ranks 2..5 (Eq. tensors-eq),
pinned by the appendix closed forms: the order-N projection keeps every moment of
degree <= N, so sum_i f^eq_i (p_i^x)^r equals I_2^{0r0}(theta, z, u) for r <= N."""
import numpy as np
import pytest

from oracle import closed_forms as C
from oracle import lattice as L
from oracle import quadrature as Q


def _evolved(stats, order=5, steps=3, seed=5):
    rng = np.random.default_rng(seed)
    nx, ny = 10, 7
    p = L.Params(stats=stats, nx=nx, ny=ny, tau=0.8, order=order)
    th = 1 + 0.2 * rng.random((ny, nx))
    ux = 0.15 * rng.standard_normal((ny, nx))
    uy = 0.15 * rng.standard_normal((ny, nx))
    z = 0.3 + 0.4 * rng.random((ny, nx))
    f = L.run(L.init_state(p, th, ux, uy, z=z), p, steps)
    return p, f


def _closed_form_pi(f, p):
    """sum_i f_i (p^x)^r minus the closed-form equilibrium moment, and a scale."""
    fs = L.stream(f, p)
    mac = L.macroscopic(fs, p)
    I = C.I2_all(mac["theta"], mac["g"], mac["ux"], mac["uy"])
    px = Q.vectors(p.stats)["px"]
    out, scale = {}, {}
    for r in (2, 3, 4, 5):
        out[r] = np.tensordot(px ** r, fs, axes=(0, 0)) - I[(0, r, 0)]
        scale[r] = np.tensordot(np.abs(px) ** r, np.abs(fs), axes=(0, 0))
    return out, scale


@pytest.mark.parametrize("stats", Q.STATS)
def test_fifth_order_against_closed_forms(stats):
    p, f = _evolved(stats)
    pi = L.noneq_tensors(f, p)
    ref, scale = _closed_form_pi(f, p)
    for r in (2, 3, 4, 5):
        err = np.abs(pi[r] - ref[r]) / scale[r]
        assert err.max() <= 1e-13, (r, err.max())
        # the state is far enough from equilibrium for the check to mean something
        assert np.abs(ref[r]).max() > 1e-6 * scale[r].max()


def test_lower_order_keeps_only_degrees_up_to_n():
    p, f = _evolved("MJ", order=3)
    pi = L.noneq_tensors(f, p)
    ref, scale = _closed_form_pi(f, p)
    for r in (2, 3):
        assert (np.abs(pi[r] - ref[r]) / scale[r]).max() <= 1e-13
    for r in (4, 5):
        assert (np.abs(pi[r] - ref[r]) / scale[r]).max() > 1e-6


@pytest.mark.parametrize("stats", Q.STATS)
def test_zero_for_a_uniform_equilibrium(stats):
    p = L.Params(stats=stats, nx=6, ny=5, tau=0.8, order=5)
    one = np.ones((5, 6))
    f = L.init_state(p, 1.1 * one, 0.2 * one, -0.1 * one, z=0.6 * one)
    pi = L.noneq_tensors(f, p)
    fs = L.stream(f, p)
    px = Q.vectors(stats)["px"]
    for r in (2, 3, 4, 5):
        scale = np.tensordot(np.abs(px) ** r, np.abs(fs), axes=(0, 0))
        assert (np.abs(pi[r]) / scale).max() <= 1e-14
