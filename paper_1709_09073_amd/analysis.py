"""Transport measurements from field snapshots (Sec. 3.2 and Sec. 3.3 of the paper):
host-side reductions over the fields the library returns.

* Taylor-Green: sigma_{u^2}(t) = sqrt(<(u^2 - <u^2>)^2>) decays as exp(-16 pi^2 nu t / L^2)
  (Eq. sigma-u2); nu follows from the slope of ln sigma_{u^2} against t.
* Fourier flow: q^x = kappa F with F(dT) = -{(1 + u_x^2 gamma^2) dT/dx
  + T gamma [d(gamma u_x)/dt + u_x d(gamma u_x)/dx]} (Eqs. qx-ft-eq, fdt-eq); kappa is
  <q^x> / <F> over the interior, with the time derivative from snapshots one step
  before and after.
"""
import math

import numpy as np


def sigma_u2(fields):
    u2 = (fields["ux"] ** 2 + fields["uy"] ** 2).double()
    return float(((u2 - u2.mean()) ** 2).mean().sqrt())


def viscosity_from_decay(times, sigmas, L):
    slope = np.polyfit(np.asarray(times, dtype=np.float64), np.log(np.asarray(sigmas, dtype=np.float64)), 1)[0]
    return -slope * L * L / (16 * math.pi ** 2)


def conductivity(prev, cur, nxt, row=0, margin_frac=0.125):
    """kappa = <q^x>/<F> along one row from fields at t-1, t, t+1 (torch or numpy)."""
    def arr(d, k):
        v = d[k][row]
        return v.cpu().numpy() if hasattr(v, "cpu") else np.asarray(v)

    def gu(d):
        ux, uy = arr(d, "ux"), arr(d, "uy")
        return ux / np.sqrt(1 - ux ** 2 - uy ** 2)

    T, ux, uy = arr(cur, "theta"), arr(cur, "ux"), arr(cur, "uy")
    ga = 1 / np.sqrt(1 - ux ** 2 - uy ** 2)
    F = -((1 + ux ** 2 * ga ** 2) * np.gradient(T)
          + T * ga * ((gu(nxt) - gu(prev)) / 2 + ux * np.gradient(gu(cur))))
    nx = T.size
    m = slice(int(nx * margin_frac), nx - int(nx * margin_frac))
    return float(arr(cur, "qx")[m].mean() / F[m].mean())
