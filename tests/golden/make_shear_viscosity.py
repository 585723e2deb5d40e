"""Writes shear_viscosity.txt: the oracle's kinematic viscosity at tau = 3 from the
decay of a shear wave whose wavevector lies along a lattice axis (the orientation
Poiseuille flow between plates feels, Sec. 3.4), for L = 8 ... 256.

    python tests/golden/make_shear_viscosity.py

Calls only oracle/ (and the seeded input generator); the GPU Poiseuille test
compares its own shear-wave measurement with these values and builds the reference
parabola from them.  The schedule below is the one both sides use.
"""
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TAU = 3.0
SIZES = (8, 16, 32, 64, 128, 256)


def schedule(L_, tau):
    """(total steps, sampling interval, first sampled step exclusive, k^2): two
    e-folding times of the Eq. nu-ref-eq viscosity, 20 samples, the first fifth skipped."""
    nu0 = (tau - 0.2546) / 4
    k2 = (2 * math.pi / L_) ** 2
    total = int(2 / (nu0 * k2))
    return total, max(1, total // 20), total // 5, k2


def fit_nu(ts, amp, k2):
    return -np.polyfit(ts, np.log(amp), 1)[0] / k2


def oracle_shear_nu(L_, tau=TAU):
    import workloads
    from oracle import lattice as L
    params, fields = workloads.shear_wave(L=L_, tau=tau)
    p = L.Params(stats="MJ", nx=params["nx"], ny=params["ny"], tau=tau)
    f = {k: v.numpy() for k, v in fields.items()}
    st = L.init_state(p, f["theta"], f["ux"], f["uy"], n=f["n"])
    total, chunk, skip, k2 = schedule(L_, tau)
    ts, amp = [], []
    t = 0
    while t <= total:
        if t > skip:
            u = L.fields(st, p)["ux"][:, 0]
            ts.append(t)
            amp.append(np.sqrt(np.mean(u * u)))
        st = L.run(st, p, chunk)
        t += chunk
    return fit_nu(ts, amp, k2)


def main():
    rows = []
    for L_ in SIZES:
        nu = oracle_shear_nu(L_)
        print(f"L={L_} nu={nu:.12f}", flush=True)
        rows.append((L_, nu))
    with open(os.path.join(HERE, "shear_viscosity.txt"), "w") as fh:
        fh.write("# Axis-aligned shear-wave viscosity of the FP64 oracle (MJ, n = theta = 1, tau = 3,\n"
                 "# u_x = 1e-4 sin(2 pi y / L) on 4 x L periodic grids), written by make_shear_viscosity.py.\n"
                 "# Eq. nu-ref-eq gives 0.6864 at tau = 3 (Taylor-Green, diagonal wavevectors).\n"
                 "# L nu\n")
        for L_, nu in rows:
            fh.write(f"{L_} {nu:.12f}\n")


if __name__ == "__main__":
    main()
