"""Concentration-dependent mobility (Appendix C) through the C ABI.

* FP64 against the oracle run with mobility="c2c2": diffusive-only, with
  hydrodynamics and walls, with tau_g != 1, with Omega != 0, and in 3-D with
  an absent component (which must stay exactly 0).  Per field the metric is
  max |gpu - oracle| / max |oracle|, held to 1e-12 for every field
  (measured at most 6.2e-14).
* FP32 and FP16S storage against FP64 on the diffusive-only case; the
  differences are written to mobility.json in the results directory.
* Fig. 3(d): diffusive coarsening of the N = 4, 400^2 mixture with the
  constant alpha and with alpha = C_i^2 C_j^2 (m* = 10); L(t) of both.
* Batch members with the flag (beside one without it) equal the members
  stepped alone, bit for bit, launching and replaying graphs.
"""
import json
import os

import numpy as np
import pytest

import paper_2605_22214_amd as nf
import workloads as W
from oracle import step as S
from oracle.lattice import D2Q9, D3Q19

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RESULTS = {}
M_STAR = 10.0


@pytest.fixture(scope="module", autouse=True)
def record():
    yield
    out = os.path.join(ROOT, "gpurun_out")
    os.makedirs(out, exist_ok=True)
    with open(os.path.join(out, "mobility.json"), "w") as fh:
        json.dump(RESULTS, fh, indent=1, sort_keys=True)


def rel(a, b):
    scale = np.abs(b).max()
    if scale == 0.0:
        return 0.0 if np.all(a == 0.0) else np.inf
    return float(np.abs(a - b).max() / scale)


def case(name):
    if name == "d2_diffusive":
        w = W.coarsening_2d(40, 4, seed=2)
        return w, dict(hydro=False), 200, -1
    if name == "d2_hydro_walls_tau_g":
        w = W.noise("D2Q9", (32, 32, 1), 3, amp=0.05, seed=5, sigma=0.005)
        w["walls"] = (False, True, False)
        w["tau_g"] = np.array([0.8, 1.0, 1.3])
        w["tau"] = np.array([0.7, 1.0, 1.2])
        w["body_force"] = (1e-6, 0.0, 0.0)
        return w, dict(hydro=True), 120, -1
    if name == "d2_omega":
        w = W.noise("D2Q9", (36, 36, 1), 4, amp=0.05, seed=7, sigma=0.005)
        w["omega_stab"] = 1.0 / 18.0
        return w, dict(hydro=True), 100, -1
    if name == "d3_absent_walls":
        w = W.noise("D3Q19", (14, 12, 10), 4, 5, amp=0.05, seed=9, sigma=0.005)
        w["walls"] = (False, False, True)
        return w, dict(hydro=True), 60, 0
    raise KeyError(name)


def oracle_run(w, okw, steps, implicit):
    lat = D2Q9 if w["lattice"] == "D2Q9" else D3Q19
    N = w["sigma"].shape[0]
    par = S.Params(lat, w["shape"], w["sigma"], w["tau"], D=w["D"], omega_stab=w["omega_stab"],
                   trt_magic=w["trt_magic"], tau_g=w["tau_g"], m=w["m"],
                   body_force=w["body_force"], walls=w["walls"],
                   implicit=(N - 1 if implicit == -1 else implicit),
                   mobility="c2c2", m_star=M_STAR, **okw)
    f, g = S.initial_state(par, w["C0"])
    for _ in range(steps):
        f, g, _ = S.step(f, g, par)
    return f, g, par


def gpu_run(w, okw, steps, implicit, precision):
    w = dict(w)
    w["m"] = M_STAR                 # under the flag, m is m*
    flags = nf.FLAG_C2C2_MOBILITY | (0 if okw.get("hydro", True) else nf.FLAG_NO_HYDRO)
    sim = nf.Simulation.from_workload(w, precision=precision, implicit=implicit, flags=flags)
    sim.set_fields(w["C0"])
    sim.step(steps)
    return sim


@pytest.mark.parametrize("name", ["d2_diffusive", "d2_hydro_walls_tau_g", "d2_omega", "d3_absent_walls"])
def test_fp64_matches_oracle(name):
    w, okw, steps, implicit = case(name)
    f, g, par = oracle_run(w, okw, steps, implicit)
    mac = S.macroscopic(f, g, par)
    with gpu_run(w, okw, steps, implicit, nf.FP64) as sim:
        assert sim.storage_form() == "populations"
        C = sim.get_field("C")
        errs = {"C": rel(C, mac["C"]),
                "G_RAW": rel(sim.get_field("G_RAW")[par.evolved], g[par.evolved]),
                "V": rel(sim.get_field("V"), mac["v"]),
                "P": rel(sim.get_field("P"), mac["P"]),
                "F_RAW": rel(sim.get_field("F_RAW"), f[1:])}
    RESULTS.setdefault("fp64_vs_oracle", {})[name] = errs
    moved = float(np.abs(mac["C"] - w["C0"].reshape(mac["C"].shape)).max())
    assert moved > 1e-4, "the concentrations must evolve"
    assert errs["C"] <= 1e-12 and errs["G_RAW"] <= 1e-12, errs
    for k in ("V", "P", "F_RAW"):
        assert errs[k] <= 1e-12, (k, errs)
    if name == "d3_absent_walls":
        assert np.all(C[4] == 0.0)


def test_storage_precisions_against_fp64():
    w, okw, steps, implicit = case("d2_diffusive")
    with gpu_run(w, okw, steps, implicit, nf.FP64) as s64:
        C64 = s64.get_field("C")
        d64 = s64.diagnostics()
    out = {}
    for name, prec in (("fp32", nf.FP32), ("fp16s", nf.FP16S)):
        with gpu_run(w, okw, steps, implicit, prec) as s:
            C = s.get_field("C")
            d = s.diagnostics()
        out[name] = {"max_abs_dC": float(np.abs(C - C64).max()),
                     "mass_rel_drift": max(abs(a - b) / b for a, b in zip(d["mass"], d64["mass"])),
                     "max_sum_dev": d["max_sum_dev"]}
    RESULTS["precisions_vs_fp64"] = out
    assert out["fp32"]["max_abs_dC"] < 1e-4
    assert out["fp16s"]["max_abs_dC"] < 1e-2
    assert out["fp32"]["mass_rel_drift"] < 1e-6



@pytest.mark.parametrize("mode", ["launch", "graph"])
def test_batch_members_with_c2c2_equal_standalone(mode):
    """Members with the concentration-dependent mobility in a batch, beside
    one without it (which then keeps g as populations too), end bit for bit
    where they end stepped alone: the batch runs their potential and source
    kernels between and after its own two on each member's arguments."""
    ws, flags = [], []
    for k, (shape, walls, c2c2) in enumerate((((32, 24, 1), (False, True, False), True),
                                              ((40, 40, 1), (False, False, False), True),
                                              ((28, 20, 1), (True, False, False), False))):
        w = W.noise("D2Q9", shape, 3, amp=0.05, seed=30 + k, sigma=0.005)
        w["walls"] = walls
        if c2c2:
            w["m"] = M_STAR            # under the flag, m is m*
        ws.append(w)
        flags.append(nf.FLAG_C2C2_MOBILITY if c2c2 else nf.FLAG_G_POPULATIONS)
    steps = 21
    ref = []
    for w, fl in zip(ws, flags):
        with nf.Simulation.from_workload(w, precision=nf.FP64, flags=fl) as s:
            s.set_fields(w["C0"])
            s.step(steps)
            ref.append(s.get_state())
    probs = [nf._Problem.from_workload(w, precision=nf.FP64, flags=fl) for w, fl in zip(ws, flags)]
    with nf.Batch(probs) as b:
        b.set_launch(graph_steps=4)
        for i, w in enumerate(ws):
            b.members[i].set_fields(w["C0"])
        b.step(steps, mode=mode)
        got = [m.get_state() for m in b.members]
    for i in range(len(ws)):
        assert np.array_equal(got[i], ref[i]), i
