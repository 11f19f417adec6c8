"""FP64 invariants of a state (oracle).  Test infrastructure only.

mass_i      = sum_x C_i                        (exactly summed with math.fsum)
momentum    = sum_x (sum_k e_k f_k + F/2)      (Eq. nmom with rho = 1)
max_abs_c_i = max_x |C_i|, min_c_i = min_x C_i (Fig. 2c tracks max |C_i|)
max_sum_dev = max_x |sum_i C_i - 1|
vcm         = sum_x C_c v / sum_x C_c          (centre-of-mass velocity, Sec. V A)
"""
import math

import numpy as np

from .step import macroscopic


def fsum(a):
    return math.fsum(np.ravel(a).tolist())


def diagnostics(f, g, par, vcm_component=1):
    mac = macroscopic(f, g, par)
    C, v = mac["C"], mac["v"]
    N = par.N
    # solid nodes hold no fluid (all fields 0 there) and are left out
    fl = np.ones(C.shape[1:], dtype=bool) if par.solid is None else ~par.solid
    out = {
        "mass": [fsum(C[i][fl]) for i in range(N)],
        "momentum": [fsum(v[a][fl]) for a in range(3)],
        "max_abs_c": [float(np.abs(C[i][fl]).max()) for i in range(N)],
        "min_c": [float(C[i][fl].min()) for i in range(N)],
        "max_sum_dev": float(np.abs(C.sum(axis=0)[fl] - 1.0).max()),
    }
    c = C[vcm_component]
    den = fsum(c)
    out["vcm"] = [fsum((c * v[a])[fl]) / den if den != 0.0 else 0.0 for a in range(3)]
    out["nan"] = int(not (np.isfinite(f).all() and np.isfinite(g).all()))
    return out
