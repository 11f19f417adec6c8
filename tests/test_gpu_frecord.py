"""The record form of f (every node relaxing with omega+ = omega- = 1).

With omega = 1 the post-collision f of a node is fixed by its P, v and F
(Eqs. TRT, FTRT, hydroforce), so the library keeps (fA, F) per node and the
reconstruction forms the moments of the streamed f from the neighbours'
records.  That is the same arithmetic as storing the populations, up to
rounding:

* which configurations take the record form;
* FP64, against the same configuration with NFLBM_FLAG_F_POPULATIONS, every
  field (C, v, P, F, mu~, f, g) within the 1e-12 parity gate: periodic and
  walled lattices, solid nodes, D2Q9 and D3Q19, and initial states with a
  velocity and pressure field (the first step takes each node's f from its
  own record, as the population form stores f^eq(P0, v0) at every node);
  also directly after set_fields, before any step;
* FP32 against FP64 in the record form (storage rounding only);
* checkpoints taken before the first step restore that state bit for bit;
* a batch of members with initial velocities equals the members stepped alone.
"""
import json
import os

import numpy as np
import pytest

import paper_2605_22214_amd as nf
import workloads as W
from parity_util import GATE, rel

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RESULTS = {}
FIELDS = ("C", "V", "P", "F", "MU", "F_RAW", "G_RAW")


@pytest.fixture(scope="module", autouse=True)
def record():
    yield
    out = os.path.join(ROOT, "gpurun_out")
    os.makedirs(out, exist_ok=True)
    with open(os.path.join(out, "frecord.json"), "w") as fh:
        json.dump(RESULTS, fh, indent=1, sort_keys=True)


def _flow(w, u=3e-3, p=2e-4, seed=5):
    """A smooth velocity field and a pressure perturbation on w's lattice."""
    nz, ny, nx = w["C0"].shape[1:]
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    v = np.zeros((3, nz, ny, nx))
    v[0] = u * np.sin(2 * np.pi * (y + 0.5) / ny)
    v[1] = 0.5 * u * np.cos(2 * np.pi * (x + 0.5) / nx)
    if w["lattice"] == "D3Q19":
        v[2] = 0.3 * u * np.sin(2 * np.pi * (x + y + 0.5) / (nx + ny))
    P = p * rng.uniform(-1.0, 1.0, size=(nz, ny, nx))
    return v, P


def cases():
    lens = W.lens_2d(37, 29, radius=7.0)
    d3 = W.noise("D3Q19", (19, 13, 11), 4, 5, amp=0.1, seed=4)
    d2w = W.noise("D2Q9", (41, 23, 1), 3, amp=0.15, seed=9, m=0.05)
    d2w.update(walls=(False, True, False), body_force=(2e-6, 0.0, 0.0))
    d3w = W.noise("D3Q19", (17, 9, 12), 3, amp=0.2, seed=8, m=0.05)
    d3w["walls"] = (True, False, True)
    posts = W.noise("D3Q19", (20, 14, 10), 4, amp=0.1, seed=12, m=0.05)
    posts["walls"] = (False, False, True)
    solid = np.zeros((10, 14, 20), dtype=bool)
    solid[:, 4:8, 6:10] = True
    trt = W.lens_2d(30, 24, radius=6.0)
    trt["trt_magic"] = 0.25          # omega- = 1 at tau = 1: the record form applies
    return [("lens", lens, -1, None), ("d3_absent", d3, 0, None), ("d2_walls_force", d2w, -1, None),
            ("d3_walls_xz", d3w, -1, None), ("d3_posts", posts, -1, solid), ("trt_quarter", trt, -1, None)]


def run(w, prec, implicit, solid, steps, flags=0, flow=True):
    sim = nf.Simulation.from_workload(w, precision=prec, implicit=implicit, flags=flags)
    if solid is not None:
        sim.set_solid(solid)
    v, P = _flow(w) if flow else (None, None)
    sim.set_fields(w["C0"], v, P)
    if steps:
        sim.step(steps)
    out = {k: sim.get_field(k) for k in FIELDS}
    form = sim.f_storage_form()
    sim.close()
    return form, out


def test_which_configurations_take_the_record_form():
    def form(w, prec=nf.FP64, flags=0):
        with nf.Simulation.from_workload(w, precision=prec, flags=flags) as s:
            return s.f_storage_form()
    lens = W.lens_2d(20, 16, radius=4.0)
    assert form(lens) == "records"
    assert form(lens, nf.FP32) == "records"
    assert form(lens, nf.FP16S) == "records"              # binary16 node records
    assert form(lens, flags=nf.FLAG_F_POPULATIONS) == "populations"
    assert form(lens, flags=nf.FLAG_G_POPULATIONS) == "populations"
    assert form(lens, flags=nf.FLAG_NO_HYDRO) == "populations"
    assert form(dict(lens, tau=np.array([1.0, 0.8, 1.0]))) == "populations"
    assert form(dict(lens, trt_magic=3.0 / 16.0)) == "populations"
    assert form(dict(lens, trt_magic=0.25)) == "records"
    assert form(dict(lens, tau_g=np.array([1.0, 0.9, 1.0]))) == "populations"


@pytest.mark.parametrize("steps", [0, 1, 30])
@pytest.mark.parametrize("idx", range(6))
def test_fp64_record_form_equals_populations(idx, steps):
    name, w, implicit, solid = cases()[idx]
    fa, a = run(w, nf.FP64, implicit, solid, steps)
    fb, b = run(w, nf.FP64, implicit, solid, steps, flags=nf.FLAG_F_POPULATIONS)
    assert (fa, fb) == ("records", "populations")
    floors = {"F": 1e-12}
    errs = {k: rel(a[k], b[k], floors.get(k, 0.0)) for k in FIELDS}
    RESULTS.setdefault("fp64_records_vs_populations", {})[f"{name}_{steps}"] = errs
    bad = {k: e for k, e in errs.items() if not e <= GATE}
    assert not bad, (name, steps, errs)
    if name == "d3_absent":
        assert np.all(a["C"][4] == 0.0)
    if solid is not None:
        assert np.all(a["C"][:, solid] == 0.0)


@pytest.mark.parametrize("idx", [0, 1, 4])
def test_fp32_record_form_close_to_fp64(idx):
    name, w, implicit, solid = cases()[idx]
    _, ref = run(w, nf.FP64, implicit, solid, 40)
    form, got = run(w, nf.FP32, implicit, solid, 40)
    assert form == "records"
    errs = {k: rel(got[k], ref[k]) for k in ("C", "V", "P")}
    RESULTS.setdefault("fp32_records_vs_fp64", {})[name] = errs
    assert errs["C"] < 1e-5 and errs["V"] < 1e-3 and errs["P"] < 1e-3, errs


def test_checkpoint_before_the_first_step():
    w = W.noise("D3Q19", (16, 12, 10), 4, seed=3)
    v, P = _flow(w)
    with nf.Simulation.from_workload(w, precision=nf.FP32) as s:
        assert s.f_storage_form() == "records"
        s.set_fields(w["C0"], v, P)
        st = s.get_state()                 # f still the local equilibria
        s.step(6)
        ref = s.get_state()
        s.step(3)
        s.set_state(st)
        s.step(6)
        assert np.array_equal(s.get_state(), ref)


def test_batch_with_initial_velocities_matches_standalone():
    ws = W.batch_members(count=3, seed=21, sides=[40, 33, 48])
    flows = [_flow(w) for w in ws]
    ref = []
    for w, (v, P) in zip(ws, flows):
        with nf.Simulation.from_workload(w, precision=nf.FP32) as s:
            s.set_fields(w["C0"], v, P)
            s.step(9)
            ref.append((s.get_field("C"), s.get_field("V")))
    with nf.Batch.from_workloads(ws, precision=nf.FP32) as b:
        assert b.members[0].f_storage_form() == "records"
        b.set_launch(graph_steps=4)
        for i, (w, (v, P)) in enumerate(zip(ws, flows)):
            b.set_fields(i, w["C0"], v, P)
        b.step(9, "graph")
        for i in range(len(ws)):
            assert np.array_equal(b.members[i].get_field("C"), ref[i][0]), i
            assert np.array_equal(b.members[i].get_field("V"), ref[i][1]), i
