"""The oracle's forced flow and non-equilibrium-extrapolation walls (Sec. 3.4).

Pins: the momentum a forced collision injects has a closed form (below); a rest state
between walls imposing that same state stays at rest; the steady Poiseuille profile is
symmetric and approaches the parabola as L grows.

Closed form of the injection: from a uniform state at rest (T^{0x} = 0, T^{xx} = P),
one step with u' = a tau in the collision gives
  Delta T^{mu x} = (1/tau) U'_nu [T_eq^{nu x}(U') - T^{nu x}]
(the Anderson-Witting weight gamma'(1 - v.u') p^0 equals U'_nu p^nu), and with
T_eq^{nu x} U'_nu = eps U'^x on the lattice (second moments are exact) this is
  Delta T^{0x} = gamma' a (eps + P),   Delta T^{00} = 0,
and likewise Delta N^0 = n (1 - gamma') / tau."""
import math

import numpy as np
import pytest

import workloads
from oracle import lattice as L
from oracle import quadrature as Q


def _params(w, stats="MJ"):
    params, fields = w
    bcs = dict(zip(("xlo", "xhi", "ylo", "yhi"), params["bc"]))
    p = L.Params(stats=stats, nx=params["nx"], ny=params["ny"], tau=params["tau"], bc=bcs,
                 force=params.get("force", (0.0, 0.0)),
                 wall_eq=dict(n=params.get("wall_n", 1.0), theta=params.get("wall_theta", 1.0)))
    f = {k: v.numpy() for k, v in fields.items()}
    return p, L.init_state(p, f["theta"], f["ux"], f["uy"], n=f["n"])


@pytest.mark.parametrize("stats", Q.STATS)
def test_forced_collision_injects_closed_form_momentum(stats):
    a, tau, th, z = 3e-4, 1.7, 1.2, 0.6
    p = L.Params(stats=stats, nx=5, ny=4, tau=tau, force=(a, 0.0))
    one = np.ones((4, 5))
    f0 = L.init_state(p, th * one, 0 * one, 0 * one, z=z * one)
    N0, T0 = L.moments(L.stream(f0, p), stats)
    f1, _ = L.step(f0, p)
    N1, T1 = L.moments(f1, stats)
    eps = T0[0, 0]
    gp = 1.0 / math.sqrt(1.0 - (a * tau) ** 2)
    # Delta T^{0x} ~ 1e-3 eps is a difference of O(eps) sums: compare on the scale of eps
    assert np.abs(T1[0, 1] - gp * a * 1.5 * eps).max() <= 5e-15 * eps.max()
    np.testing.assert_allclose(T1[0, 0], T0[0, 0], rtol=1e-14)
    # and Delta N^0 = (1/tau) U'_nu (n U'^nu - N^nu) = n (1 - gamma') / tau
    np.testing.assert_allclose(N1[0], N0[0] * (1.0 + (1.0 - gp) / tau), rtol=1e-14)
    assert np.abs(T1[0, 2]).max() <= 1e-15 * eps.max()


@pytest.mark.parametrize("stats", Q.STATS)
def test_walls_keep_a_matching_rest_state(stats):
    params, fields = workloads.poiseuille(L=6, a=0.0, tau=1.3)
    p, f = _params((params, fields), stats)
    f0 = f.copy()
    f = L.run(f, p, 20)
    assert np.abs(f - f0).max() <= 1e-13 * np.abs(f0).max()


def _steady(L_, tau=3.0, a=1e-8):
    params, fields = workloads.poiseuille(L=L_, a=a, tau=tau)
    p, f = _params((params, fields))
    nu = (tau - 0.2546) / 4
    f = L.run(f, p, int(math.ceil(30 * L_ * L_ / (math.pi ** 2 * nu))))
    u = L.fields(f, p)["ux"][:, 0]
    y = np.arange(L_ + 1)
    uref = a / (2 * nu) * y * (L_ - y)
    return u, np.sqrt(np.sum((u - uref) ** 2) / np.sum(uref ** 2))


def test_poiseuille_profile_symmetric_and_converging():
    u8, e8 = _steady(8)
    u16, e16 = _steady(16)
    for u in (u8, u16):
        # FP64 floor: u ~ 1e-7 is a difference of O(1) moments
        assert np.abs(u - u[::-1]).max() <= 1e-8 * np.abs(u).max()
    assert u16.max() > 3.5 * u8.max()          # the centre velocity grows like L^2
    assert e16 < e8 / 2.5, (e8, e16)           # and the profile error falls
