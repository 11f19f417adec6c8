"""Convective outflow (Sec. III C, Eq. convect) through the C ABI
(nflbm_set_outflow).

* FP64 against the oracle with the same outflow face: inlet + outflow
  channels of three components on x (walls on y: corner links), on y (x
  periodic: the ghost plane wraps), with tau_g != 1 (the update reads the
  plane buffer of g), an outflow on the x- face fed from x+ with a body force
  (the outward normal points down the axis), the velocity pulse of the oracle's
  test, and D3Q19 with the outflow on x (walls on z) and on z (the ghost
  plane fills a whole LDS plane).  Metric per field as in the parity tests
  (tests/parity_util.py): every field to 1e-12 of its scale, or to ten
  times its spread under a one-ulp perturbation of the input where that is
  larger (F of the pure-phase pulse is rounding noise, scaled by a 1e-12
  floor; its spread sets its bound).
* The outflow state travels with nflbm_get_state / nflbm_set_state, and
  starting it in nflbm_set_outflow after nflbm_set_fields or in
  nflbm_set_fields gives the same bits; in the moment forms as well, where
  plane N's reconstructed values are re-derived after a restore (also the
  autotuner's).
* FP32 and FP16S against the FP64 oracle on the pulse run, within their
  storage error.
* Argument errors: an unwalled or too short axis, the face already open, an
  open face on another axis meeting the outflow plane at a fluid node, solid
  nodes that do not continue through the outflow plane.
"""
import json
import os

import numpy as np
import pytest

import paper_2605_22214_amd as nf
import workloads as W
from oracle import step as S
from oracle.coeffs import equal_sigma
from oracle.lattice import D2Q9, D3Q19
from parity_util import conditioned, rel

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RESULTS = {}


@pytest.fixture(scope="module", autouse=True)
def record():
    yield
    out = os.path.join(ROOT, "gpurun_out")
    os.makedirs(out, exist_ok=True)
    with open(os.path.join(out, "outflow.json"), "w") as fh:
        json.dump(RESULTS, fh, indent=1, sort_keys=True)




def pulse(nx=60, ny=6, u=0.02):
    """The oracle test's pulse: a plug flow u from an inlet on x- carrying a
    Gaussian velocity bump towards the outflow on x+."""
    N = 2
    C0 = np.zeros((N, 1, ny, nx))
    C0[0] = 1.0
    x = np.arange(nx)
    v0 = np.zeros((3, 1, ny, nx))
    v0[0] = u + 0.002 * np.exp(-((x - 20) / 3.0) ** 2)[None, None, :]
    w = W._base("D2Q9", (nx, ny, 1), equal_sigma(N, 0.005), 1.0, 0.05, C0=C0,
                walls=(True, False, False))
    return w, {0: ((u, 0.0, 0.0), (1.0, 0.0))}, 1, v0


def case(name):
    """(workload, open faces, outflow face, initial velocity or None, steps)."""
    if name == "channel_x":
        w = W.noise("D2Q9", (40, 18, 1), 3, amp=0.1, seed=4, sigma=0.006, m=0.05)
        w.update(walls=(True, True, False), trt_magic=3.0 / 16.0, tau=np.array([0.7, 1.0, 1.2]))
        return w, {0: ((2e-3, 0.0, 0.0), (0.8, 0.15, 0.05))}, 1, None, 200
    if name == "channel_y":
        w = W.noise("D2Q9", (16, 30, 1), 3, amp=0.1, seed=5, sigma=0.006, m=0.05)
        w.update(walls=(False, True, False))
        return w, {2: ((3e-4, 2e-3, 0.0), (0.5, 0.3, 0.2))}, 3, None, 150
    if name == "tau_g":
        w = W.noise("D2Q9", (30, 14, 1), 3, amp=0.1, seed=6, sigma=0.006, m=0.05)
        w.update(walls=(True, False, False), tau_g=np.array([0.8, 1.0, 1.3]))
        return w, {0: ((1e-3, 2e-4, 0.0), (0.5, 0.3, 0.2))}, 1, None, 150
    if name == "x_minus":
        w = W.noise("D2Q9", (24, 12, 1), 3, amp=0.1, seed=8, sigma=0.006, m=0.05)
        w.update(walls=(True, True, False), body_force=(-1e-6, 2e-7, 0.0))
        return w, {1: ((-2e-3, 0.0, 0.0), (0.3, 0.3, 0.4))}, 0, None, 200
    if name == "pulse":
        w, faces, out, v0 = pulse()
        return w, faces, out, v0, 120
    if name == "d3_x":
        w = W.noise("D3Q19", (14, 9, 10), 3, amp=0.1, seed=7, sigma=0.006, m=0.05)
        w.update(walls=(True, False, True))
        return w, {0: ((1e-3, 0.0, 0.0), (0.6, 0.3, 0.1))}, 1, None, 60
    if name == "d3_z":
        w = W.noise("D3Q19", (10, 9, 14), 3, amp=0.1, seed=9, sigma=0.006, m=0.05)
        w.update(walls=(False, False, True))
        return w, {4: ((0.0, 2e-4, 1e-3), (0.2, 0.5, 0.3))}, 5, None, 60
    raise KeyError(name)


def oracle_run(w, faces, out, v0, steps):
    lat = D2Q9 if w["lattice"] == "D2Q9" else D3Q19
    N = w["sigma"].shape[0]
    par = S.Params(lat, w["shape"], w["sigma"], w["tau"], D=w["D"], omega_stab=w["omega_stab"],
                   trt_magic=w["trt_magic"], tau_g=w["tau_g"], m=w["m"], body_force=w["body_force"],
                   walls=w["walls"], implicit=N - 1, open_faces=faces, outflow=out)
    f, g = S.initial_state(par, w["C0"], v0)
    for _ in range(steps):
        f, g, _ = S.step(f, g, par)
    return f, g, par


def gpu_sim(w, faces, out, v0, precision):
    sim = nf.Simulation.from_workload(w, precision=precision, flags=nf.FLAG_G_POPULATIONS)
    for face, (vb, Cb) in faces.items():
        sim.set_open_face(face, vb, Cb)
    sim.set_outflow(out)
    sim.set_fields(w["C0"], v0)
    return sim


CASES = ["channel_x", "channel_y", "tau_g", "x_minus", "pulse", "d3_x", "d3_z"]


FLOORS = {"F": 1e-12}   # F of the pure-phase pulse is rounding noise


def gpu_fields(sim, par):
    return {"C": sim.get_field("C"), "G_RAW": sim.get_field("G_RAW")[par.evolved],
            "V": sim.get_field("V"), "P": sim.get_field("P"), "F": sim.get_field("F"),
            "F_RAW": sim.get_field("F_RAW")}


@pytest.mark.parametrize("name", CASES)
def test_fp64_matches_oracle_with_outflow(name):
    w, faces, out, v0, steps = case(name)
    f, g, par = oracle_run(w, faces, out, v0, steps)
    mac = S.macroscopic(f, g, par)
    ref = {"C": mac["C"], "G_RAW": g[par.evolved], "V": mac["v"], "P": mac["P"], "F": mac["F"],
           "F_RAW": f[1:]}
    got = {}
    for key, wk in (("ref", w), ("pert", dict(w, C0=W.ulp_perturbed(w["C0"])))):
        with gpu_sim(wk, faces, out, v0, nf.FP64) as sim:
            sim.step(steps)
            got[key] = gpu_fields(sim, par)
    errs = {k: rel(got["ref"][k], ref[k], FLOORS.get(k, 0.0)) for k in ref}
    tol = conditioned({k: rel(got["pert"][k], got["ref"][k], FLOORS.get(k, 0.0)) for k in ref})
    RESULTS.setdefault("fp64_vs_oracle", {})[name] = dict(errs, U=par.outflow_state["U"])
    RESULTS.setdefault("fp64_tolerance", {})[name] = tol
    assert par.outflow_state["U"] > 0.0          # the outflow convects
    assert errs["C"] <= 1e-12 and errs["G_RAW"] <= 1e-12, errs
    for k in ref:
        assert errs[k] <= tol[k], (k, errs, tol)


def test_outflow_state_round_trip_and_start():
    w, faces, out, v0, _ = case("channel_x")
    with gpu_sim(w, faces, out, v0, nf.FP64) as sim:
        sim.step(15)
        saved = sim.get_state()
        sim.step(20)
        a = sim.get_state()
        sim.set_state(saved)
        sim.step(20)
        b = sim.get_state()
    assert np.array_equal(a, b)
    # the outflow set after set_fields starts from the same state
    with nf.Simulation.from_workload(w, precision=nf.FP64, flags=nf.FLAG_G_POPULATIONS) as sim:
        for face, (vb, Cb) in faces.items():
            sim.set_open_face(face, vb, Cb)
        sim.set_fields(w["C0"], v0)
        sim.set_outflow(out)
        sim.step(35)
        c = sim.get_state()
    assert np.array_equal(a, c)


@pytest.mark.parametrize("name,flags,form", [("channel_x", 0, ("moments", "populations")),
                                             ("pulse", 0, ("moments", "records")),
                                             ("d3_x", 0, ("moments", "records"))])
def test_outflow_state_round_trip_moment_forms(name, flags, form, tmp_path):
    """In the moment form the outflow kernel writes plane N's C, E_B and f
    moments into arrays outside the state; restoring a state re-derives them
    from the restored plane buffers, and so does the autotuner's restore, so
    both continue bit for bit."""
    w, faces, out, v0, _ = case(name)

    def make():
        sim = nf.Simulation.from_workload(w, precision=nf.FP64, flags=flags)
        for face, (vb, Cb) in faces.items():
            sim.set_open_face(face, vb, Cb)
        sim.set_outflow(out)
        sim.set_fields(w["C0"], v0)
        return sim

    with make() as sim:
        assert (sim.storage_form(), sim.f_storage_form()) == form
        sim.step(15)
        saved = sim.get_state()
        sim.step(20)
        a = sim.get_state()
        sim.step(7)                          # plane-N values of a later state
        sim.set_state(saved)
        sim.step(20)
        b = sim.get_state()
    assert np.array_equal(a, b)
    with make() as sim:
        sim.step(15)
        sim.autotune(str(tmp_path / "tune.txt"))   # times steps, then restores
        sim.step(20)
        c = sim.get_state()
    assert np.array_equal(a, c)


@pytest.mark.parametrize("prec,tv,tc", [(nf.FP32, 1e-4, 1e-5), (nf.FP16S, 1e-2, 2e-4)])
def test_reduced_precision_pulse_against_oracle(prec, tv, tc):
    """FP32 and FP16S (binary16 f and g, whose stored numbers carry a
    power-of-two scale that the plane buffer's values must take on) against
    the FP64 oracle.  The FP16S bounds are binary16 storage error: measured
    2.7e-3 of max |v| and 4e-5 on C after 120 steps (a scale slip would be
    off by orders of magnitude)."""
    w, faces, out, v0, steps = case("pulse")
    f, g, par = oracle_run(w, faces, out, v0, steps)
    mac = S.macroscopic(f, g, par)
    with gpu_sim(w, faces, out, v0, prec) as sim:
        sim.step(steps)
        v = sim.get_field("V")
        C = sim.get_field("C")
    errs = {"V": rel(v, mac["v"]), "C": float(np.abs(C - mac["C"]).max())}
    RESULTS[{nf.FP32: "fp32_pulse", nf.FP16S: "fp16s_pulse"}[prec]] = errs
    assert errs["V"] < tv and errs["C"] < tc, errs


def test_outflow_argument_errors():
    w, faces, out, v0, _ = case("channel_x")
    with nf.Simulation.from_workload(w, precision=nf.FP64, flags=nf.FLAG_G_POPULATIONS) as sim:
        with pytest.raises(nf.NflbmError):
            sim.set_outflow(4)                                               # no z in D2Q9
        sim.set_open_face(0, (1e-3, 0, 0), (0.5, 0.3, 0.2))
        with pytest.raises(nf.NflbmError):
            sim.set_outflow(0)                                               # already open
        sim.set_outflow(1)
        with pytest.raises(nf.NflbmError):
            # another axis, meeting the outflow plane at a fluid node
            sim.set_open_face(2, (1e-3, 0, 0), (0.5, 0.3, 0.2))
        bad = np.zeros((1, 18, 40), dtype=bool)
        bad[0, 5, 39] = True                                                 # not through plane N-1
        with pytest.raises(nf.NflbmError):
            sim.set_solid(bad)
        sim.set_outflow(None)
        sim.set_open_face(2, (1e-3, 0, 0), (0.5, 0.3, 0.2))
    w2 = W.noise("D2Q9", (16, 12, 1), 3, seed=1)
    with nf.Simulation.from_workload(w2, precision=nf.FP64, flags=nf.FLAG_G_POPULATIONS) as sim:
        with pytest.raises(nf.NflbmError):
            sim.set_outflow(1)                                               # x is periodic
    w3 = W.noise("D2Q9", (2, 12, 1), 3, seed=1)
    w3["walls"] = (True, False, False)
    with nf.Simulation.from_workload(w3, precision=nf.FP64, flags=nf.FLAG_G_POPULATIONS) as sim:
        with pytest.raises(nf.NflbmError):
            sim.set_outflow(1)                                               # axis too short
