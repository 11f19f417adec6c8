"""Write quaternary_512_1000.txt: the oracle's state at sampled nodes of the
512 x 512 quaternary phase separation after 1000 time steps.

Workload: D2Q9, N = 4, periodic, C_i = 0.25 + U(-0.02, 0.02) renormalised
(seed 0), every sigma = 0.01, tau = tau_g = 1, m = 0.1, the fourth component
implicit (Sec. II).  The oracle takes about 0.7 s per step at this size, so
the file is written once by this script (python tests/golden/make_quaternary_512.py)
and read by the GPU parity test.  Only oracle/ and the input generator are
called.

Each data line: x y, C_1..C_4, v_x v_y, P, f_1..f_8 (post-streaming), and
g_{i,k} for the three evolved components (i-major, k = 0..8).
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import step as S  # noqa: E402
from oracle.lattice import D2Q9  # noqa: E402

N_SIDE = 512
STEPS = 1000
OUT = os.path.join(HERE, "quaternary_512_1000.txt")


def sample_nodes(n, count=48, seed=2024):
    """Corners, edge midpoints and seeded interior nodes (x, y)."""
    rng = np.random.default_rng(seed)
    fixed = [(0, 0), (n - 1, 0), (0, n - 1), (n - 1, n - 1), (n // 2, 0), (0, n // 2),
             (n - 1, n // 2), (n // 2, n - 1)]
    rest = [tuple(int(v) for v in rng.integers(0, n, size=2)) for _ in range(count - len(fixed))]
    return fixed + rest


def main():
    w = W.quaternary_2d(N_SIDE)
    par = S.Params(D2Q9, w["shape"], w["sigma"], w["tau"], m=w["m"])
    f, g = S.initial_state(par, w["C0"])
    for t in range(STEPS):
        f, g, _ = S.step(f, g, par)
        if (t + 1) % 100 == 0:
            print(f"step {t + 1}", flush=True)
    mac = S.macroscopic(f, g, par)
    C, v, P = mac["C"], mac["v"], mac["P"]
    lines = [
        "# Oracle state after 1000 steps of the 512 x 512 quaternary phase separation",
        "# (D2Q9, N = 4, sigma = 0.01, tau = tau_g = 1, m = 0.1, seed 0; component 4 implicit).",
        "# Written by make_quaternary_512.py from oracle/ only.",
        "# columns: x y C1..C4 vx vy P f1..f8 g[i][k] (i = 1..3, k = 0..8)",
        "# total mass per component: " + " ".join(repr(float(C[i].sum())) for i in range(4)),
    ]
    for (x, y) in sample_nodes(N_SIDE):
        vals = [C[i, 0, y, x] for i in range(4)] + [v[0, 0, y, x], v[1, 0, y, x], P[0, y, x]]
        vals += [f[k, 0, y, x] for k in range(1, 9)]
        vals += [g[i, k, 0, y, x] for i in range(3) for k in range(9)]
        lines.append(f"{x} {y} " + " ".join(repr(float(a)) for a in vals))
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
