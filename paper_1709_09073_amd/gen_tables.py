"""Generate the constant tables compiled into the HIP library (csrc/rlbm_tables.h).

Run:  python -m paper_1709_09073_amd.gen_tables   (needs mpmath; seconds to a minute)

Everything is computed in mpmath at 50 digits and rounded once to FP64.

1. d2v72 radial rules (Sec. 2.4, Eq. quadrature-eq).  The radial moments
   mu_k = int_0^inf omega(p) p^k dp of the weights of Eqs. mj-w-eq, fd-w-eq and
   be-w-eq are integrated numerically; the Gauss rule follows by Golub-Welsch
   (Cholesky factor of the Hankel moment matrix -> Jacobi matrix -> symmetric
   eigen-decomposition).  Per-vector weight w_s = lambda_s * 2 pi / 12.

2. Separable equilibrium projector (Sec. 2.3, Eqs. expansion-eq, projections-eq).
   The span V_5 of the relativistic polynomials is spanned by the harmonic
   functions p^k cos(j phi), p^k sin(j phi), 0 <= j <= k <= 5.  Different
   harmonics are orthogonal under the 12-direction sum, so the projection splits
   into one radial Gram block per harmonic j: G^(j)_{kk'} = c_j sum_s lambda_s
   p_s^{k+k'} (c_0 = 2 pi, c_j = pi).  The moment of p^k T_j(phi) of the
   equilibrium is (general form of Appendix A)
       b_{jk} = k! g_{k+1}(z) theta^{k+1} gamma^k P_{kj}(u^2) * Re/Im (u_x + i u_y)^j,
   where u^j gamma^{2k+1} P_{kj}(u^2) = int cos(j b) (1 - u cos b)^{-(k+1)} db
   (P_{kj} a polynomial of degree (k-j)/2, derived exactly below).  The lattice
   equilibrium is
       f^eq_{s,n} = sum_j r_j(s) A_{j,n},   r_j(s) = sum_k E^(j)_{s,k} G_k P_{kj}(u^2),
       A_{j,n} = Re[(u_x + i u_y)^j e^{-i j phi_n}],  G_k = k! g_{k+1} theta^{k+1} gamma^k,
   with E^(j)_{s,k} = w_s sum_{k'} p_s^{k'} (G^(j))^{-1}_{k'k}.

3. g_nu(z) tables for Fermi-Dirac and Bose-Einstein (Eq. gz-eq) in mu = ln z,
   using d g_nu / d mu = g_{nu-1}: at centres mu_c the values g_m(mu_c) for
   m = 6 down to 6 - NT - 5 give g_nu(mu_c + d) = sum_{t<NT} g_{nu-t}(mu_c) d^t/t!.
   Orders m >= 1 are integrated numerically from the definition; orders m <= 0
   are the exact rational functions (z d/dz)^{-m} [z/(1 + xi z)].
   BE near z = 1 (mu in [-1, 0)) uses the expansion of Li_nu about mu = 0 with
   zeta(nu - t) coefficients and the logarithmic term of order nu - 1.
"""
import os
from fractions import Fraction

import mpmath as mp
import sympy as sp

DPS = 50
STATS = ("MJ", "FD", "BE")
ZC = mp.mpf(1) - mp.mpf(10) ** -7

# g-table layout (shared with the kernels through the generated header)
NT = 14                         # Taylor terms
NG = NT + 5                     # stored orders per centre: m = 6, 5, ..., 6 - NG + 1
FD_MU_MIN, FD_DMU, FD_NC = -12.0, 0.25, 97          # centres -12 .. +12
BE_MU_SPLIT = -1.0                                   # log series on [-1, 0)
BE_MU_MIN, BE_DMU = -12.0, 0.125
BE_NC = int(round((BE_MU_SPLIT - BE_MU_MIN) / BE_DMU)) + 1   # centres -12 .. -1
BE_NZ = 24                                           # terms of the series about mu = 0
# Shorter sums for FP32 / FP16 population storage, where g to 1e-11 relative is far
# below the populations' rounding; check_loose_truncation bounds the omitted tail.
NT_LOOSE = 9
BE_NZ_LOOSE = 15


def _omega(stats, p):
    if stats == "MJ":
        return mp.exp(-p) / (2 * mp.pi)
    if stats == "FD":
        return 1 / (mp.exp(p) + 1)
    return 1 / (mp.exp(p) / ZC - 1)


def radial_moments(stats, kmax=12):
    with mp.workdps(DPS):
        return [mp.quad(lambda p: _omega(stats, p) * p ** k, [0, 1, 4, 12, 30, 80, mp.inf]) for k in range(kmax + 1)]


def golub_welsch(mu, n=6):
    """Nodes and weights of the n-point Gauss rule from moments mu_0..mu_2n."""
    with mp.workdps(DPS):
        H = mp.matrix(n + 1, n + 1)
        for a in range(n + 1):
            for b in range(n + 1):
                H[a, b] = mu[a + b]
        L = mp.cholesky(H)          # H = L L^T, L lower
        R = L.T
        alpha, beta = [], []
        for j in range(n):
            a = R[j, j + 1] / R[j, j]
            if j > 0:
                a -= R[j - 1, j] / R[j - 1, j - 1]
            alpha.append(a)
            if j < n - 1:
                beta.append(R[j + 1, j + 1] / R[j, j])
        J = mp.matrix(n, n)
        for j in range(n):
            J[j, j] = alpha[j]
            if j < n - 1:
                J[j, j + 1] = J[j + 1, j] = beta[j]
        E, Q = mp.eigsy(J)
        order = sorted(range(n), key=lambda i: E[i])
        nodes = [E[i] for i in order]
        weights = [mu[0] * Q[0, i] ** 2 for i in order]
        return nodes, weights


def pkj_polynomials():
    """Exact coefficients (without the 2 pi factor) of P_kj(x), x = u^2:
    int_0^{2pi} cos(j b)(1 - u cos b)^{-(k+1)} db = 2 pi u^j (1 - x)^{-(k + 1/2)} P_kj(x)."""
    out = {}
    for j in range(6):
        for k in range(j, 6):
            # series S(x) = sum_l C(j+2l+k, k) C(j+2l, l) 2^-(j+2l) x^l
            L = 12
            S = [Fraction(sp.binomial(j + 2 * l + k, k) * sp.binomial(j + 2 * l, l), 2 ** (j + 2 * l)) for l in range(L)]
            # (1 - x)^{k + 1/2} as a series
            a = Fraction(2 * k + 1, 2)
            B = [Fraction(1)]
            for m in range(1, L):
                B.append(B[-1] * (a - (m - 1)) / m * -1)
            prod = [sum(S[i] * B[m - i] for i in range(m + 1)) for m in range(L)]
            deg = (k - j) // 2
            assert all(c == 0 for c in prod[deg + 1:]), (k, j, prod)
            out[(j, k)] = prod[:deg + 1] + [Fraction(0)] * (2 - deg)
    return out


def separable_projector(stats, nodes, lam, order=5):
    """E^(j)_{s,k} for j = 0..order, k = j..order, s = 0..5 (mpmath): projection onto V_order."""
    E = {}
    with mp.workdps(DPS):
        for j in range(order + 1):
            cj = 2 * mp.pi if j == 0 else mp.pi
            ks = list(range(j, order + 1))
            G = mp.matrix(len(ks), len(ks))
            for a, k1 in enumerate(ks):
                for b, k2 in enumerate(ks):
                    G[a, b] = cj * mp.fsum(lam[s] * nodes[s] ** (k1 + k2) for s in range(6))
            Gi = G ** -1
            for s in range(6):
                w = lam[s] * 2 * mp.pi / 12
                for b, k in enumerate(ks):
                    E[(j, k, s)] = w * mp.fsum(nodes[s] ** ks[a] * Gi[a, b] for a in range(len(ks)))
    return E


def _neg_order_funcs(xi, mmin):
    """Rational functions g_m(z) for m = 0, -1, ..., mmin: g_0 = z/(1 + xi z),
    g_{m-1} = z d g_m / dz (xi = +1 FD, -1 BE)."""
    z = sp.symbols("z")
    f = z / (1 + xi * z)
    funcs = {0: sp.lambdify(z, f, "mpmath")}
    for m in range(-1, mmin - 1, -1):
        f = sp.simplify(z * sp.diff(f, z))
        funcs[m] = sp.lambdify(z, f, "mpmath")
    return funcs


def _g_pos(xi, nu, mu):
    """g_nu(e^mu), nu >= 1, by numerical integration of Eq. gz-eq."""
    with mp.workdps(30):
        z = mp.exp(mu)
        f = lambda x: x ** (nu - 1) / (mp.exp(x) / z + xi)
        pts = [0, max(mp.mpf(1), mu), max(mp.mpf(2), mu) + 10, max(mp.mpf(2), mu) + 60, mp.inf]
        return mp.quad(f, pts) / mp.gamma(nu)


def g_taylor_table(xi, centres):
    mmin = 6 - NG + 1
    neg = _neg_order_funcs(xi, mmin)
    rows = []
    for mu in centres:
        mu = mp.mpf(mu)
        row = []
        for m in range(6, mmin - 1, -1):
            if m >= 1:
                row.append(_g_pos(xi, m, mu))
            else:
                with mp.workdps(30):
                    row.append(neg[m](mp.exp(mu)))
        rows.append(row)
    return rows


def check_loose_truncation(fd_rows, be_rows, bound=1e-11):
    """Largest relative size of the tail that NT_LOOSE Taylor terms (tables) and
    BE_NZ_LOOSE series terms (about mu = 0) leave out, over each interval a centre
    serves; raises if above bound.  The tail is taken as twice its first term (the
    terms fall by a factor below 1/2 from there on)."""
    worst = 0.0
    for rows, dmu in ((fd_rows, FD_DMU), (be_rows, BE_DMU)):
        h = mp.mpf(dmu) / 2
        for row in rows:
            for m in range(1, 7):
                gm = row[6 - m]
                first = abs(row[6 - m + NT_LOOSE]) * h ** NT_LOOSE / mp.factorial(NT_LOOSE)
                worst = max(worst, float(2 * first / (gm * (1 - 2 * h))))
    with mp.workdps(30):
        mu = -(mp.mpf(-BE_MU_SPLIT) + mp.mpf(BE_DMU) / 2)
        for m in range(1, 7):
            k = BE_NZ_LOOSE
            first = abs(mp.zeta(m - k)) * abs(mu) ** k / mp.factorial(k)
            worst = max(worst, float(2 * first / mp.polylog(m, mp.exp(mu))))
    if worst > bound:
        raise ValueError("shortened g sums leave %.3g relative" % worst)
    return worst


def _fmt(x):
    return repr(float(x))


def emit(path):
    lines = ["// Generated by paper_1709_09073_amd/gen_tables.py -- do not edit.",
             "// Constant tables for the d2v72 relativistic lattice Boltzmann kernels.",
             "#pragma once", "",
             "namespace rlbm_tab {", ""]
    lines.append("constexpr int NT = %d;      // Taylor terms of the g_nu tables" % NT)
    lines.append("constexpr int NG = %d;      // stored orders per centre: m = 6 .. %d" % (NG, 6 - NG + 1))
    lines.append("constexpr double FD_MU_MIN = %r, FD_DMU = %r; constexpr int FD_NC = %d;" % (FD_MU_MIN, FD_DMU, FD_NC))
    lines.append("constexpr double BE_MU_MIN = %r, BE_DMU = %r, BE_MU_SPLIT = %r; constexpr int BE_NC = %d;"
                 % (BE_MU_MIN, BE_DMU, BE_MU_SPLIT, BE_NC))
    lines.append("constexpr int BE_NZ = %d;" % BE_NZ)
    lines.append("constexpr int NT_LOOSE = %d, BE_NZ_LOOSE = %d;   // terms when 1e-11 relative suffices"
                 % (NT_LOOSE, BE_NZ_LOOSE))
    with mp.workdps(DPS):
        lines.append("constexpr double LOG_ZC_BE = %s;" % _fmt(mp.log(ZC)))
        g1c, g2c = mp.polylog(1, ZC), mp.polylog(2, ZC)
        g3c = mp.polylog(3, ZC)
        lines.append("// Bose-Einstein g_1, g_2 and h = g_2^3 / g_3^2 at the condensation fugacity z_c")
        lines.append("constexpr double G1_ZC_BE = %s, G2_ZC_BE = %s, H_ZC_BE = %s;"
                     % (_fmt(g1c), _fmt(g2c), _fmt(g2c ** 3 / g3c ** 2)))
    lines.append("")

    p_all, w_all, E_all = [], [], []
    for st in STATS:
        mu = radial_moments(st)
        nodes, lam = golub_welsch(mu)
        p_all.append(nodes)
        w_all.append([l * 2 * mp.pi / 12 for l in lam])
        E_all.append(separable_projector(st, nodes, lam))
    lines.append("// radial nodes p_s and per-vector weights w_s, [stats][shell]; stats: 0 MJ, 1 FD, 2 BE")
    lines.append("constexpr double P_SHELL[3][6] = {%s};" % ", ".join(
        "{" + ", ".join(_fmt(x) for x in p) + "}" for p in p_all))
    lines.append("constexpr double W_SHELL[3][6] = {%s};" % ", ".join(
        "{" + ", ".join(_fmt(x) for x in w) + "}" for w in w_all))
    pairs = [(j, k) for j in range(6) for k in range(j, 6)]
    lines.append("// separable projector E[stats][pair][shell], pair = (j, k) j-major, k = j..5")
    lines.append("// (constexpr tables are only indexed with compile-time indices: values fold into instructions)")
    body = []
    for E in E_all:
        body.append("{" + ", ".join("{" + ", ".join(_fmt(E[(j, k, s)]) for s in range(6)) + "}" for (j, k) in pairs) + "}")
    lines.append("constexpr double EMAT[3][21][6] = {%s};" % ", ".join(body))
    # lower expansion orders (Maxwell-Juttner): same pair layout, zero where k > order
    lines.append("// projector of order N = 2, 3, 4 for Maxwell-Juttner, EMAT_LO[N - 2][pair][shell]")
    mj_nodes, mj_lam = golub_welsch(radial_moments("MJ"))
    lo = []
    for order in (2, 3, 4):
        El = separable_projector("MJ", mj_nodes, mj_lam, order)
        lo.append("{" + ", ".join("{" + ", ".join(_fmt(El.get((j, k, s_), 0)) for s_ in range(6)) + "}"
                                  for (j, k) in pairs) + "}")
    lines.append("constexpr double EMAT_LO[3][21][6] = {%s};" % ", ".join(lo))
    P = pkj_polynomials()
    lines.append("// P_kj(x) = c0 + c1 x + c2 x^2 including the factor 2 pi, per pair (j, k)")
    with mp.workdps(DPS):
        lines.append("constexpr double PKJ[21][3] = {%s};" % ", ".join(
            "{" + ", ".join(_fmt(2 * mp.pi * mp.mpf(c.numerator) / c.denominator) for c in P[(j, k)]) + "}"
            for (j, k) in pairs))
    # g tables
    fd_c = [FD_MU_MIN + i * FD_DMU for i in range(FD_NC)]
    be_c = [BE_MU_MIN + i * BE_DMU for i in range(BE_NC)]
    fd = g_taylor_table(1, fd_c)
    be = g_taylor_table(-1, be_c)
    print("shortened g sums: tail <= %.2e relative" % check_loose_truncation(fd, be))
    lines.append("// g_m(mu_c) for m = 6, 5, ..., 6-NG+1 at centres mu_c = MU_MIN + i DMU")
    lines.append("__constant__ double FD_TAB[%d][%d] = {%s};" % (FD_NC, NG, ", ".join(
        "{" + ", ".join(_fmt(x) for x in r) + "}" for r in fd)))
    lines.append("__constant__ double BE_TAB[%d][%d] = {%s};" % (BE_NC, NG, ", ".join(
        "{" + ", ".join(_fmt(x) for x in r) + "}" for r in be)))
    with mp.workdps(DPS):
        # zeta(m) for m = 6 .. 6 - BE_NZ - 5 (pole at m = 1 stored as 0)
        zs = [(mp.zeta(m) if m != 1 else mp.mpf(0)) for m in range(6, 6 - BE_NZ - 6, -1)]
        lines.append("// zeta(m) for m = 6 .. %d (m = 1 stored as 0), series of Li about mu = 0" % (6 - BE_NZ - 5))
        lines.append("__constant__ double BE_ZETA[%d] = {%s};" % (len(zs), ", ".join(_fmt(x) for x in zs)))
        lines.append("constexpr double HARMONIC[6] = {%s};" % ", ".join(
            _fmt(mp.fsum(mp.mpf(1) / i for i in range(1, m + 1))) for m in range(6)))
        lines.append("constexpr double INV_FACT[%d] = {%s};" % (BE_NZ + 1, ", ".join(
            _fmt(1 / mp.factorial(i)) for i in range(BE_NZ + 1))))
    lines += ["", "}  // namespace rlbm_tab", ""]
    with open(path, "w") as fh:
        fh.write("\n".join(lines))


if __name__ == "__main__":
    here = os.path.dirname(os.path.abspath(__file__))
    emit(os.path.join(here, "csrc", "rlbm_tables.h"))
    print("wrote", os.path.join(here, "csrc", "rlbm_tables.h"))
