"""Host decoding of RLBM_DEV16 buffers for the tests: f_i = w_k (R_i + s_k q_i / 32767)
with R_{k,n} = rho_k + p_k (alpha cos phi_n + beta sin phi_n) (include/rlbm.h), and the
bound on how far a decoded population may lie from the value that was encoded."""
import numpy as np

from oracle import quadrature as Q

STEP = 1.0 / 32767.0


def parts(rl, buf, nx, ny, stats):
    """(reference R (72, ny, nx), per-population scale s_k (72, ny, nx), q (72, ny, nx)),
    float64 numpy."""
    q, side, scale = rl.dev16_views(buf, nx, ny)
    q = q.double().cpu().numpy()
    sd = side.double().cpu().numpy()
    sc = scale.double().cpu().numpy()
    v = Q.vectors(stats)
    R = sd[v["k"]] + v["p0"][:, None, None] * (sd[6] * v["vx"][:, None, None] + sd[7] * v["vy"][:, None, None])
    return R, sc[v["k"]], q


def decode(rl, buf, nx, ny, stats):
    R, s, q = parts(rl, buf, nx, ny, stats)
    w = Q.vectors(stats)["w"][:, None, None]
    return w * (R + s * q * STEP)


def quantum(rl, buf, nx, ny, stats):
    """Half the SNORM16 step of each population in f units: w_k s_k / (2 * 32767)."""
    _, s, _ = parts(rl, buf, nx, ny, stats)
    w = Q.vectors(stats)["w"][:, None, None]
    return w * s * (0.5 * STEP)


# the hardware's float -> SNORM16 conversion is allowed 0.6 of a step (as graphics APIs
# allow), not the 0.5 of round-to-nearest
CODE_ERR = 0.6 * STEP


def decode_bound(rl, buf, nx, ny, stats):
    """Largest |decoded - encoded| of each population, in f units (72, ny, nx).

    A code is off by at most CODE_ERR s_k.  The encoder then moves rho_k by minus the
    shell's mean code error (at most CODE_ERR s_k) and alpha, beta by minus the codes'
    momentum error over sum_k 6 W_k P_k^3; with sum_n |cos phi_n| = 7.464 over the 12
    directions that shift is at most
        D = 7.464 sum_j W_j P_j^2 CODE_ERR s_j / (6 sum_j W_j P_j^3)
    per coefficient, and p_k (|cos| + |sin|) <= sqrt(2) p_k carries it to a population."""
    _, s, _ = parts(rl, buf, nx, ny, stats)
    v = Q.vectors(stats)
    P, W = Q.lattice(stats)
    P, W = np.asarray(P, dtype=np.float64), np.asarray(W, dtype=np.float64)
    _, side, scale = rl.dev16_views(buf, nx, ny)
    sk = scale.double().cpu().numpy()                                   # (6, ny, nx)
    sum_c = 2 * (1 + 2 * np.cos(np.pi / 6) + 2 * 0.5)
    D = sum_c * np.tensordot(W * P ** 2, sk, axes=1) * CODE_ERR / (6 * (W * P ** 3).sum())
    w = v["w"][:, None, None]
    return w * (2 * CODE_ERR * s + np.sqrt(2) * v["p0"][:, None, None] * D[None])
