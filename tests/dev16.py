"""Host decoding of RLBM_DEV16 buffers for the tests: f_i = w_k (R_i + s_k q_i / 32767)
with R_{k,n} = rho_k + p_k (alpha cos phi_n + beta sin phi_n) (include/rlbm.h)."""
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
