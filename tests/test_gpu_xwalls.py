"""Lattices walled on x alone: the interior tile columns take the periodic kernels.

With walls on x only and no solid nodes, the reconstruction and the update
run the first and last tile columns in the wall variant and the columns
between them in the periodic variant (a node there meets no wall face, and
its arithmetic is the same in both variants).

* FP64 against the oracle, in the moment and population forms of g, on
  lattices wide enough that both kernels split (five or more 16-wide
  columns, three 64-wide ones): D3Q19 with an inlet on x- and the convective
  outflow on x+ (Sec. III C, Eqs. dirvel, dircomp and convect), and D2Q9
  with plain walls on x, TRT and a body force along them.  Every field to
  1e-12 of its scale, or ten times its spread under a one-ulp perturbation
  of the input where that is larger (tests/parity_util.py).
* The same run in FP32 and FP16S gives the same bits with 16-wide tiles
  (split: five columns) as with 64-wide ones (not split: two columns), in
  both forms.
Measured errors are written to xwalls.json in the results directory.
"""
import json
import os

import numpy as np
import pytest

import paper_2605_22214_amd as nf
import workloads as W
from oracle import step as S
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
    with open(os.path.join(out, "xwalls.json"), "w") as fh:
        json.dump(RESULTS, fh, indent=1, sort_keys=True)


def case(name):
    """(workload, open faces, outflow face or None, steps)."""
    if name == "d3_inlet_outflow":
        w = W.noise("D3Q19", (140, 7, 6), 3, amp=0.1, seed=12, sigma=0.006, m=0.05)
        w.update(walls=(True, False, False))
        return w, {0: ((1e-3, 0.0, 0.0), (0.6, 0.3, 0.1))}, 1, 40
    if name == "d2_walls":
        w = W.noise("D2Q9", (150, 20, 1), 4, amp=0.1, seed=13, sigma=0.006, m=0.05)
        w.update(walls=(True, False, False), trt_magic=3.0 / 16.0, body_force=(0.0, 2e-6, 0.0),
                 tau=np.array([0.7, 1.0, 1.2, 0.9]))
        return w, {}, None, 60
    if name == "d3_narrow":
        w = W.noise("D3Q19", (70, 10, 8), 3, amp=0.1, seed=14, sigma=0.006, m=0.05)
        w.update(walls=(True, False, False))
        return w, {0: ((1e-3, 0.0, 0.0), (0.6, 0.3, 0.1))}, 1, 30
    raise KeyError(name)


def make_sim(w, faces, out, precision, flags):
    sim = nf.Simulation.from_workload(w, precision=precision, flags=flags)
    for face, (vb, Cb) in faces.items():
        sim.set_open_face(face, vb, Cb)
    if out is not None:
        sim.set_outflow(out)
    sim.set_fields(w["C0"])
    return sim


def fields(sim, ev):
    return {"C": sim.get_field("C"), "G_RAW": sim.get_field("G_RAW")[ev], "V": sim.get_field("V"),
            "P": sim.get_field("P"), "F": sim.get_field("F"), "F_RAW": sim.get_field("F_RAW")}


FORMS = [0, nf.FLAG_G_POPULATIONS]


@pytest.mark.parametrize("flags", FORMS, ids=["moments", "populations"])
@pytest.mark.parametrize("name", ["d3_inlet_outflow", "d2_walls"])
def test_fp64_matches_oracle(name, flags):
    w, faces, out, steps = case(name)
    lat = D2Q9 if w["lattice"] == "D2Q9" else D3Q19
    N = w["sigma"].shape[0]
    par = S.Params(lat, w["shape"], w["sigma"], w["tau"], D=w["D"], omega_stab=w["omega_stab"],
                   trt_magic=w["trt_magic"], tau_g=w["tau_g"], m=w["m"], body_force=w["body_force"],
                   walls=w["walls"], implicit=N - 1, open_faces=faces, outflow=out)
    f, g = S.initial_state(par, w["C0"])
    for _ in range(steps):
        f, g, _ = S.step(f, g, par)
    mac = S.macroscopic(f, g, par)
    ref = {"C": mac["C"], "G_RAW": g[par.evolved], "V": mac["v"], "P": mac["P"], "F": mac["F"],
           "F_RAW": f[1:]}
    got = {}
    for key, wk in (("ref", w), ("pert", dict(w, C0=W.ulp_perturbed(w["C0"])))):
        with make_sim(wk, faces, out, nf.FP64, flags) as sim:
            ul, _, _ = sim.get_launch()
            cl, _ = sim.get_conc_launch()
            sim.step(steps)
            got[key] = fields(sim, par.evolved)
    columns = [-(-w["shape"][0] // (1 << t)) for t in (ul, cl)]
    errs = {k: rel(got["ref"][k], ref[k]) for k in ref}
    tol = conditioned({k: rel(got["pert"][k], got["ref"][k]) for k in ref})
    RESULTS[f"{name}_{'populations' if flags else 'moments'}"] = {"errors": errs, "tolerance": tol,
                                                                  "tile_columns": columns}
    assert min(columns) >= 3, columns                  # both kernels split
    assert errs["C"] <= 1e-12 and errs["G_RAW"] <= 1e-12, errs
    for k in ref:
        assert errs[k] <= tol[k], (k, errs, tol)


@pytest.mark.parametrize("flags", FORMS, ids=["moments", "populations"])
@pytest.mark.parametrize("prec", [nf.FP32, nf.FP16S], ids=["fp32", "fp16s"])
def test_split_equals_unsplit_bitwise(prec, flags):
    w, faces, out, steps = case("d3_narrow")
    runs = []
    for t in (4, 6):
        with make_sim(w, faces, out, prec, flags) as sim:
            sim.set_launch(t, 4)
            sim.set_conc_launch(t, 4)
            sim.step(steps)
            runs.append(sim.get_state())
    assert np.array_equal(runs[0], runs[1])


def test_default_shape_follows_the_geometry():
    """While the split applies, the reconstruction's z runs leave about 2048
    workgroups over its two launches (runs of 4 planes here) and otherwise
    about 1024 (runs of 8): solid nodes end the split and the default shape
    is chosen again, until a shape is set by hand."""
    w = W.noise("D3Q19", (200, 64, 128), 3, seed=15)
    w["walls"] = (True, False, False)
    post = np.zeros((128, 64, 200), dtype=bool)
    post[:, 4:8, 40:48] = True
    with nf.Simulation.from_workload(w, precision=nf.FP32) as sim:
        assert sim.get_launch()[:2] == (6, 4) and sim.get_conc_launch() == (6, 4)
        sim.set_solid(post)
        assert sim.get_launch()[:2] == (6, 4) and sim.get_conc_launch() == (6, 8)
        sim.set_solid(None)
        assert sim.get_conc_launch() == (6, 4)
        sim.set_launch(4, 2)
        sim.set_solid(post)
        assert sim.get_launch()[:2] == (4, 2) and sim.get_conc_launch() == (6, 4)
