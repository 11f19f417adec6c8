"""Every component count through the float kernels' record layouts.

The update keeps each LDS position's evolved concentrations as one record of
1, 2 or 4 values (three padded to four) in float and field-major beyond four;
the reconstruction rounds each group of its records up to a multiple of four
values.  D3Q19, periodic and walled, N = 2 to 6 (update records of width 1,
2, 4, 4 and the field-major layout of five evolved components; reconstruction
groups of 4, 4, 4, 4 and 8), 20 steps from a noisy mixture:

* FP64 against the oracle: C and g to 1e-12 of their scale, v and P to 1e-12
  of theirs or ten times their spread under a one-ulp perturbation of the
  input (tests/parity_util.py), whichever is larger;
* FP32 and FP16S against FP64, relative to the field's scale: FP32 within
  5e-6 on C and 1e-4 on v (measured up to 1.3e-6 and 1.2e-5: float
  rounding of C, mu~ and the force over 20 steps), FP16S within 4e-5 on C
  (binary16 records; measured up to 1.6e-5).
Measured errors are written to ncomp.json in the results directory.
"""
import json
import os

import numpy as np
import pytest

import paper_2605_22214_amd as nf
import workloads as W
from oracle import step as S
from oracle.lattice import D3Q19
from parity_util import conditioned, rel

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RESULTS = {}
STEPS = 20


@pytest.fixture(scope="module", autouse=True)
def record():
    yield
    out = os.path.join(ROOT, "gpurun_out")
    os.makedirs(out, exist_ok=True)
    with open(os.path.join(out, "ncomp.json"), "w") as fh:
        json.dump(RESULTS, fh, indent=1, sort_keys=True)


def workload(N, walled):
    w = W.noise("D3Q19", (14, 11, 9), N, amp=0.1, seed=40 + N, sigma=0.006, m=0.05)
    if walled:
        w["walls"] = (True, False, True)
    return w


def gpu(w, precision):
    with nf.Simulation.from_workload(w, precision=precision) as sim:
        sim.set_fields(w["C0"])
        sim.step(STEPS)
        return {k: sim.get_field(k) for k in ("C", "V", "P", "G_RAW")}


@pytest.mark.parametrize("walled", [False, True])
@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_component_counts(N, walled):
    w = workload(N, walled)
    par = S.Params(D3Q19, w["shape"], w["sigma"], w["tau"], D=w["D"], omega_stab=w["omega_stab"],
                   trt_magic=w["trt_magic"], tau_g=w["tau_g"], m=w["m"], body_force=w["body_force"],
                   walls=w["walls"], implicit=N - 1)
    f, g = S.initial_state(par, w["C0"])
    for _ in range(STEPS):
        f, g, _ = S.step(f, g, par)
    mac = S.macroscopic(f, g, par)
    ev = par.evolved
    ref = {"C": mac["C"], "V": mac["v"], "P": mac["P"], "G_RAW": g[ev]}
    g64 = gpu(w, nf.FP64)
    g64p = gpu(dict(w, C0=W.ulp_perturbed(w["C0"])), nf.FP64)
    got = dict(g64, G_RAW=g64["G_RAW"][ev])
    gotp = dict(g64p, G_RAW=g64p["G_RAW"][ev])
    errs = {k: rel(got[k], ref[k]) for k in ref}
    tol = conditioned({k: rel(gotp[k], got[k]) for k in ref})
    g32 = gpu(w, nf.FP32)
    g16 = gpu(w, nf.FP16S)
    e32 = {k: rel(g32[k], g64[k]) for k in ("C", "V")}
    e16 = {"C": rel(g16["C"], g64["C"])}
    RESULTS[f"N{N}_{'walled' if walled else 'periodic'}"] = {
        "fp64_vs_oracle": errs, "tolerance": tol, "fp32_vs_fp64": e32, "fp16s_vs_fp64": e16}
    assert float(np.abs(ref["C"] - w["C0"].reshape(ref["C"].shape)).max()) > 1e-4   # the mixture evolves
    assert errs["C"] <= 1e-12 and errs["G_RAW"] <= 1e-12, errs
    for k in ("V", "P"):
        assert errs[k] <= tol[k], (k, errs, tol)
    assert e32["C"] < 5e-6 and e32["V"] < 1e-4, e32
    assert e16["C"] < 4e-5, e16
