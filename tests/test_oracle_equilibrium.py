"""Pins of the expansion (Sec. 2.3, Eqs. expansion-eq, projections-eq)."""
import numpy as np
import pytest

from conftest import read_golden
from oracle import equilibrium as E
from oracle import gfunc as G
from oracle import quadrature as Q


def test_fig1_expansion_errors():
    """MJ at theta = 1, u = (0.6, 0), p = (1, 0): 18.5% at 2nd order, 1.8% at 5th."""
    for order, err, tol in read_golden("fig1_expansion_error.txt"):
        g = G.g_all("MJ", np.array(1.0))
        fN = E.feq_expanded_at("MJ", 1.0, 0.0, 1.0, g, 0.6, 0.0, int(order))
        fx = E.feq_exact("MJ", 1.0, 0.0, 1.0, 1.0, 0.6, 0.0)
        assert abs(abs(fN - fx) / fx - float(err)) <= float(tol), (order, abs(fN - fx) / fx)


def test_basis_dimension():
    for N in range(1, 6):
        assert len(E.basis(N)) == (N + 1) ** 2
        assert len(set(E.basis(N))) == (N + 1) ** 2


@pytest.mark.parametrize("stats,zr", [("MJ", 1.0), ("FD", 1.0), ("BE", 1.0 - 1e-7)])
def test_expansion_exact_at_origin(stats, zr):
    """At theta = 1, u = 0, z = z_r the equilibrium is omega times a constant, which the
    projection keeps exactly: f^eq_i = w_i * c with c = 2 pi z (MJ) or 1 (FD, BE)."""
    _, w = Q.lattice(stats)
    g = G.g_all(stats, np.array(zr))
    feq = E.feq_lattice(stats, np.float64(1.0), g, 0.0, 0.0)
    c = 2 * np.pi * zr if stats == "MJ" else 1.0
    # the outermost shell (weight ~1e-7 of the first) carries ~1e-12 relative rounding
    np.testing.assert_allclose(feq.reshape(12, 6), np.tile(w * c, (12, 1)), rtol=5e-12)


@pytest.mark.parametrize("stats", Q.STATS)
def test_projection_idempotent(stats):
    """The lattice projector maps the sampled basis functions onto themselves:
    M (Phi^T applied to w*phi_b) reproduces w*phi_b (projection of an element of V_5)."""
    M = E.projector(stats)
    v = Q.vectors(stats)
    Phi = np.stack([v["p0"] ** m * v["px"] ** a * v["py"] ** b for (m, a, b) in E.basis()], axis=1)
    for col in (0, 7, 20, 35):
        fvec = v["w"] * Phi[:, col]
        mom = Phi.T @ fvec
        np.testing.assert_allclose(M @ mom, fvec, rtol=1e-9, atol=1e-12 * np.abs(fvec).max())


def test_lower_orders_converge():
    """Errors at p = (1, 0) decrease with the order (Fig. 1 discussion)."""
    g = G.g_all("MJ", np.array(1.0))
    fx = E.feq_exact("MJ", 1.0, 0.0, 1.0, 1.0, 0.6, 0.0)
    errs = [abs(E.feq_expanded_at("MJ", 1.0, 0.0, 1.0, g, 0.6, 0.0, N) - fx) / fx for N in (2, 3, 4, 5)]
    assert errs == sorted(errs, reverse=True)
