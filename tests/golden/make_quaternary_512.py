"""Write quaternary_512_1000.txt: the oracle's state at sampled nodes of the
512 x 512 quaternary phase separation after 1000 time steps.

Workload: D2Q9, N = 4, periodic, C_i = 0.25 + U(-0.02, 0.02) renormalised
(seed 0), every sigma = 0.01, tau = tau_g = 1, m = 0.1, the fourth component
implicit (Sec. II).  The oracle takes about 0.7 s per step at this size, so
the file is written once by this script (python tests/golden/make_quaternary_512.py)
and read by the GPU parity test.  Only oracle/ and the input generator are
called.

The oracle also runs the same case from the input moved by one unit in the
last place at every node (workloads.ulp_perturbed); the relative spread of
each sampled field between the two runs is written to the header.  It is
the conditioning bound of the parity test: two correct implementations that
round differently cannot be expected to agree more closely than the
problem's own response to rounding-sized input differences.

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
FIELDS = ("C", "v", "P", "f", "g")


def sample_nodes(n, count=48, seed=2024):
    """Corners, edge midpoints and seeded interior nodes (x, y)."""
    rng = np.random.default_rng(seed)
    fixed = [(0, 0), (n - 1, 0), (0, n - 1), (n - 1, n - 1), (n // 2, 0), (0, n // 2),
             (n - 1, n // 2), (n // 2, n - 1)]
    rest = [tuple(int(v) for v in rng.integers(0, n, size=2)) for _ in range(count - len(fixed))]
    return fixed + rest


def run(C0, par, label):
    f, g = S.initial_state(par, C0)
    for t in range(STEPS):
        f, g, _ = S.step(f, g, par)
        if (t + 1) % 100 == 0:
            print(f"{label}: step {t + 1}", flush=True)
    mac = S.macroscopic(f, g, par)
    nodes = sample_nodes(N_SIDE)
    xs = np.array([p[0] for p in nodes])
    ys = np.array([p[1] for p in nodes])
    return {"C": mac["C"][:, 0, ys, xs].T, "v": mac["v"][:2, 0, ys, xs].T, "P": mac["P"][0, ys, xs],
            "f": f[1:, 0, ys, xs].T, "g": np.transpose(g[:3, :, 0, ys, xs], (2, 0, 1)),
            "mass": [float(mac["C"][i].sum()) for i in range(4)]}


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def main():
    w = W.quaternary_2d(N_SIDE)
    par = S.Params(D2Q9, w["shape"], w["sigma"], w["tau"], m=w["m"])
    ref = run(w["C0"], par, "reference")
    pert = run(W.ulp_perturbed(w["C0"]), par, "perturbed")
    lines = [
        "# Oracle state after 1000 steps of the 512 x 512 quaternary phase separation",
        "# (D2Q9, N = 4, sigma = 0.01, tau = tau_g = 1, m = 0.1, seed 0; component 4 implicit).",
        "# Written by make_quaternary_512.py from oracle/ only.",
        "# columns: x y C1..C4 vx vy P f1..f8 g[i][k] (i = 1..3, k = 0..8)",
        "# total mass per component: " + " ".join(repr(m) for m in ref["mass"]),
        "# oracle spread under a one-ulp input perturbation (C v P f g): "
        + " ".join(repr(rel(pert[k], ref[k])) for k in FIELDS),
    ]
    for q, (x, y) in enumerate(sample_nodes(N_SIDE)):
        vals = list(ref["C"][q]) + list(ref["v"][q]) + [ref["P"][q]] + list(ref["f"][q])
        vals += list(ref["g"][q].reshape(-1))
        lines.append(f"{x} {y} " + " ".join(repr(float(a)) for a in vals))
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
