"""Writes fp64_drift.txt: how far two independent FP64 implementations of the method
drift apart per step, the evidence behind the growth of the FP64 parity bars.

    python tests/golden/make_fp64_drift.py

Runs the oracle (oracle.lattice) and the brute-force checker (oracle.bruteforce:
harmonic-basis equilibrium with numerically integrated moments, dense streaming
matrices, library eigen-solver) side by side on a Maxwell-Juttner shock tube,
64 x 4, n = 1.0 / 0.139, theta = 1, u = 0, tau = 0.9, x open, y periodic, for 500
steps, and records for each field and radial shell the largest err(K)/K over
K = 50, 100, ..., 500 (errors as the parity tests measure them: max-norm relative to
the field's maximum; u against max(|u|_max, 0.01); q against max(|q|_max,
1e-3 eps_max); populations per shell against the shell's maximum).  Calls only
oracle/ and the seeded input generator.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

KEYS = ("n", "eps", "theta", "z", "u", "q") + tuple(f"shell{k}" for k in range(6))


def errors(a, b, fa, fb):
    out = {}
    for k in ("n", "eps", "theta", "z"):
        out[k] = np.abs(fa[k] - fb[k]).max() / np.abs(fb[k]).max()
    out["u"] = max(np.abs(fa["ux"] - fb["ux"]).max(), np.abs(fa["uy"] - fb["uy"]).max()) / \
        max(np.abs(fb["ux"]).max(), np.abs(fb["uy"]).max(), 0.01)
    out["q"] = max(np.abs(fa["qx"] - fb["qx"]).max(), np.abs(fa["qy"] - fb["qy"]).max()) / \
        max(np.abs(fb["qx"]).max(), np.abs(fb["qy"]).max(), 1e-3 * np.abs(fb["eps"]).max())
    for s in range(6):
        out[f"shell{s}"] = np.abs(a[s::6] - b[s::6]).max() / np.abs(b[s::6]).max()
    return out


def drift(nsteps=500, every=50, verbose=True):
    import workloads
    from oracle import bruteforce as B
    from oracle import lattice as L
    params, fields = workloads.riemann(nx=64, ny=4, tau=0.9)
    bcd = dict(zip(("xlo", "xhi", "ylo", "yhi"), params["bc"]))
    p = L.Params(stats="MJ", nx=64, ny=4, tau=0.9, bc=bcd)
    f0 = {k: v.numpy() for k, v in fields.items()}
    a = L.init_state(p, f0["theta"], f0["ux"], f0["uy"], n=f0["n"])
    b = a.copy()
    rate = dict.fromkeys(KEYS, 0.0)
    for k in range(1, nsteps + 1):
        a, _ = L.step(a, p)
        b = B.step(b, "MJ", 0.9, bcd)
        if k % every == 0:
            e = errors(a, b, L.fields(a, p), L.fields(b, p))
            for key in KEYS:
                rate[key] = max(rate[key], e[key] / k)
            if verbose:
                print(k, " ".join(f"{key}={e[key]:.2e}" for key in KEYS), flush=True)
    return rate


def main():
    rate = drift()
    with open(os.path.join(HERE, "fp64_drift.txt"), "w") as fh:
        fh.write("# Drift per step between the FP64 oracle and the FP64 brute-force checker (two independent\n"
                 "# implementations), MJ shock tube 64 x 4, tau = 0.9, 500 steps: max over K of err(K)/K.\n"
                 "# Written by make_fp64_drift.py.\n# key rate_per_step\n")
        for key, v in rate.items():
            fh.write(f"{key} {v:.3e}\n")


if __name__ == "__main__":
    main()
