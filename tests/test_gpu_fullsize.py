"""The 256^3 D3Q19 workload that bench.py times (quaternary phase separation
with an absent fifth component, component 1 implicit), at full size and in
the default launch configuration.

* Sampled nodes against the oracle: one time step reads the state within two
  nodes of a node (the stencils reach one neighbour, streaming one more), so
  after s steps C at a node depends only on the initial state within 2 s
  nodes, and v and P (through F and its stencils) within 2 s + 1.  The
  oracle runs s = 3 steps on the periodic 15^3 box cut out of the initial
  field around each sampled node, whose centre then evolves exactly as on
  the full lattice.  The samples sit on tile, z-run and lattice
  boundaries of the launch.  FP64: C, v and P to 1e-12 of their scale
  (measured 2e-13 on v and P, O(1e-7) quantities); FP32 storage: C to
  1e-6 absolute (measured 4.6e-8); FP16S: v to 1e-2 of its scale (measured
  3.6e-4: binary16 f records) and C to 3e-6 absolute.  The FP16S C error
  comes from the binary16 mu~ records (11 significant bits): each step's C
  takes m (1 - w_0) mu~ through them, so a half-ulp of mu~ per step adds up
  over the three steps; measured 7.3e-7, and 1.06e-6 with a build that
  only changed the rounding order of the stencil's constant factors, so the
  bound leaves a factor of three over the larger.
* Properties that hold at any size, FP32, 300 steps: the absent component
  is exactly 0.0 everywhere, sum_i C_i = 1 and the mass of every component
  hold to float rounding.
"""
import json
import os

import numpy as np
import pytest

import paper_2605_22214_amd as nf
import workloads as W
from oracle import step as S
from oracle.lattice import D3Q19

pytestmark = pytest.mark.gpu

SIDE = 256
STEPS = 3
HALF = 2 * STEPS + 1      # dependency radius of v and P after STEPS steps
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RESULTS = {}
SAMPLES = [(0, 0, 0), (63, 3, 7), (64, 4, 8), (255, 255, 255), (127, 128, 64),
           (191, 17, 200), (5, 250, 129), (200, 99, 31)]


@pytest.fixture(scope="module", autouse=True)
def record():
    yield
    out = os.path.join(ROOT, "gpurun_out")
    os.makedirs(out, exist_ok=True)
    with open(os.path.join(out, "fullsize.json"), "w") as fh:
        json.dump(RESULTS, fh, indent=1, sort_keys=True)


@pytest.fixture(scope="module")
def workload():
    return W.quaternary_3d(SIDE)


def oracle_center(w, x, y, z):
    """C, v, P at the centre of the periodic box around (x, y, z) after STEPS."""
    idx = lambda c: np.arange(c - HALF, c + HALF + 1) % SIDE
    sub = w["C0"][:, idx(z)][:, :, idx(y)][:, :, :, idx(x)]
    n = 2 * HALF + 1
    par = S.Params(D3Q19, (n, n, n), w["sigma"], w["tau"], D=w["D"], omega_stab=w["omega_stab"],
                   trt_magic=w["trt_magic"], tau_g=w["tau_g"], m=w["m"], body_force=w["body_force"],
                   implicit=0)
    f, g = S.initial_state(par, sub)
    for _ in range(STEPS):
        f, g, _ = S.step(f, g, par)
    mac = S.macroscopic(f, g, par)
    c = HALF
    return mac["C"][:, c, c, c], mac["v"][:, c, c, c], mac["P"][c, c, c]


@pytest.fixture(scope="module")
def oracle_samples(workload):
    return [oracle_center(workload, *s) for s in SAMPLES]


@pytest.mark.parametrize("prec", [nf.FP64, nf.FP32, nf.FP16S])
def test_full_size_sampled_nodes(workload, oracle_samples, prec):
    w = workload
    with nf.Simulation.from_workload(w, precision=prec, implicit=0) as sim:
        sim.set_fields(w["C0"])
        sim.step(STEPS)
        C = sim.get_field("C")
        V = sim.get_field("V")
        P = sim.get_field("P")
    got_C = np.array([C[:, z, y, x] for (x, y, z) in SAMPLES])
    got_v = np.array([V[:, z, y, x] for (x, y, z) in SAMPLES])
    got_P = np.array([P[z, y, x] for (x, y, z) in SAMPLES])
    ref_C = np.array([o[0] for o in oracle_samples])
    ref_v = np.array([o[1] for o in oracle_samples])
    ref_P = np.array([o[2] for o in oracle_samples])
    assert np.abs(ref_v).max() > 0.0 and np.abs(ref_C[:, 4]).max() == 0.0
    RESULTS[{nf.FP64: "fp64", nf.FP32: "fp32", nf.FP16S: "fp16s"}[prec]] = {
        "C_abs": float(np.abs(got_C - ref_C).max()),
        "v_rel": float(np.abs(got_v - ref_v).max() / np.abs(ref_v).max()),
        "P_rel": float(np.abs(got_P - ref_P).max() / np.abs(ref_P).max())}
    if prec == nf.FP64:
        assert np.abs(got_C - ref_C).max() <= 1e-12 * np.abs(ref_C).max()
        assert np.abs(got_v - ref_v).max() <= 1e-12 * np.abs(ref_v).max()
        assert np.abs(got_P - ref_P).max() <= 1e-12 * np.abs(ref_P).max()
    elif prec == nf.FP32:
        assert np.abs(got_C - ref_C).max() <= 1e-6
    else:
        # binary16 records: v and P carry the rounding of f's, C that of mu~
        assert np.abs(got_C - ref_C).max() <= 3e-6
        assert np.abs(got_v - ref_v).max() <= 1e-2 * np.abs(ref_v).max()
    assert np.all(got_C[:, 4] == 0.0)


def test_full_size_invariants_fp32(workload):
    w = workload
    with nf.Simulation.from_workload(w, precision=nf.FP32, implicit=0) as sim:
        sim.set_fields(w["C0"])
        d0 = sim.diagnostics()
        sim.step(300)
        d1 = sim.diagnostics()
    assert d1["max_abs_c"][4] == 0.0 and d1["min_c"][4] == 0.0
    assert d1["max_sum_dev"] < 1e-6
    for i in range(4):
        assert abs(d1["mass"][i] - d0["mass"][i]) <= 1e-6 * d0["mass"][i], i
