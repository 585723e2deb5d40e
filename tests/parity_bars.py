"""FP64 parity bars of the HIP path against the oracle, and where they come from.

A bar after K steps is  base + 3 * drift * K  for each field and radial shell:
* drift: how far two independent FP64 implementations of the method (the oracle and
  its brute-force checker) move apart per step, measured on a 500-step shock tube by
  tests/golden/make_fp64_drift.py (tests/golden/fp64_drift.txt);
* base: about three times the largest error the HIP path showed in the short
  parity runs (init, one step, up to 6 steps, walls), rounded up.
Errors are measured as in make_fp64_drift.py: max-norm relative to the field's
maximum (u against max(|u|_max, 0.01), q against max(|q|_max, 1e-3 eps_max));
populations per radial shell against that shell's maximum (the outer shells carry
the rounding of the ill-conditioned radial projection, hence their larger base).
"""
from conftest import read_golden

DRIFT = {k: float(v) for k, v in read_golden("fp64_drift.txt")}

# largest short-run errors seen (init, one step, <= 6 steps with walls, the persistent
# batch kernel): n 1.2e-14, eps 2.1e-14, theta 1.3e-14, z 2.0e-14, u 3.2e-13 (Fourier
# walls, against the 0.01 floor), q 1.6e-12; shells 2.3e-14, 2.2e-14, 2.8e-14, 9.2e-14,
# 4.4e-13, 1.3e-11
FIELD_BASE = dict(n=1e-13, eps=1e-13, theta=1e-13, z=1e-13, u=1e-12, q=5e-12)
SHELL_BASE = (7e-14, 7e-14, 9e-14, 3e-13, 1.5e-12, 4e-11)
FIELD_KEY = dict(n="n", eps="eps", theta="theta", z="z", ux="u", uy="u", qx="q", qy="q")


def field_bar(name, k):
    key = FIELD_KEY[name]
    return FIELD_BASE[key] + 3.0 * DRIFT[key] * k


def shell_bar(s, k):
    return SHELL_BASE[s] + 3.0 * DRIFT[f"shell{s}"] * k
