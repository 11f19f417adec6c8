"""Metric and tolerances shared by the GPU parity tests.

rel(a, b): max |a - b| over max |b| (the oracle's scale of the field); a
floor replaces a zero or rounding-noise scale.

conditioned(spread): the tolerance of each field, 1e-12 of its scale, or
ten times the spread between two runs of the same implementation whose
inputs differ by one unit in the last place (workloads.ulp_perturbed),
whichever is larger.  Two correct implementations that round differently
cannot agree more closely than the problem's own response to
rounding-sized input differences, so that spread is the conditioning bound
of a comparison; in well-conditioned cases it is far below 1e-12 and the
plain bound applies.
"""
import numpy as np

GATE = 1e-12
FACTOR = 10.0


def rel(a, b, floor=0.0):
    scale = max(float(np.abs(b).max()), floor)
    if scale == 0.0:
        return 0.0 if np.all(a == 0.0) else np.inf
    return float(np.abs(a - b).max() / scale)


def conditioned(spread):
    return {k: max(GATE, FACTOR * v) for k, v in spread.items()}
