"""The reference pressure of nflbm_set_fields (Eq. feq, pressure form).

A uniform pressure P_ref adds 3 w_k P_ref to every f_k and no step of the
method changes that shift, so the library keeps the populations of P - P_ref
and adds P_ref back on read-back.  Without the shift a background pressure
of 1/3 would put f_k near w_k and leave binary16 storage about three decimal
digits for the velocity signal.

* FP16S: a sheared lens run with P = 1/3 everywhere equals the run with
  P = 0 bit for bit in C and v, and its P and f read back shifted by exactly
  1/3 and w_k.
* FP64 against the oracle (which does not shift) with P = 1/3 plus seeded
  noise: every field within the parity gate.
"""
import numpy as np
import pytest

import paper_2605_22214_amd as nf
import workloads as W
from oracle import step as S
from oracle.lattice import D2Q9
from parity_util import GATE, rel

pytestmark = pytest.mark.gpu

W_D2Q9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def _shear(w, u=2e-3):
    ny, nx = w["C0"].shape[2:]
    v = np.zeros((3, 1, ny, nx))
    v[0, 0] = u * np.sin(2 * np.pi * (np.arange(ny)[:, None] + 0.5) / ny)
    return v


def test_fp16s_background_pressure_is_a_pure_shift():
    w = W.lens_2d(32, 24, radius=6.0)
    v0 = _shear(w)
    out = {}
    for p in (0.0, 1.0 / 3.0):
        with nf.Simulation.from_workload(w, precision=nf.FP16S) as sim:
            sim.set_fields(w["C0"], v0, np.full(w["C0"][0].shape, p))
            sim.step(300)
            out[p] = {k: sim.get_field(k) for k in ("C", "V", "P", "F_RAW")}
    a, b = out[1.0 / 3.0], out[0.0]
    assert np.array_equal(a["C"], b["C"])
    assert np.array_equal(a["V"], b["V"])
    assert np.abs((a["P"] - 1.0 / 3.0) - b["P"]).max() <= 1e-15
    shift = (W_D2Q9[1:] * 3.0 * (1.0 / 3.0))[:, None, None, None]
    assert np.abs((a["F_RAW"] - shift) - b["F_RAW"]).max() <= 1e-15
    assert np.abs(b["V"]).max() > 1e-4                  # the flow carries a signal


def test_fp64_background_pressure_matches_oracle():
    w = W.lens_2d(24, 20, radius=5.0)
    v0 = _shear(w)
    rng = np.random.default_rng(7)
    P0 = 1.0 / 3.0 + 1e-4 * rng.uniform(-1.0, 1.0, size=w["C0"][0].shape)
    steps = 40
    par = S.Params(D2Q9, w["shape"], w["sigma"], w["tau"], m=w["m"])
    f, g = S.initial_state(par, w["C0"], v0, P0)
    for _ in range(steps):
        f, g, _ = S.step(f, g, par)
    mac = S.macroscopic(f, g, par)
    with nf.Simulation.from_workload(w, precision=nf.FP64) as sim:
        sim.set_fields(w["C0"], v0, P0)
        sim.step(steps)
        errs = {"C": rel(sim.get_field("C"), mac["C"]), "V": rel(sim.get_field("V"), mac["v"]),
                "P": rel(sim.get_field("P"), mac["P"]), "F_RAW": rel(sim.get_field("F_RAW"), f[1:])}
    for k, e in errs.items():
        assert e <= GATE, (k, errs)
