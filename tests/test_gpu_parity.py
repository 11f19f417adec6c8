"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Metric per field: max_x |gpu - oracle| / max_x |oracle|; a field that is zero
everywhere in the oracle must be exactly zero on the GPU.  FP64 storage must
agree to 1e-12 (after 1000 steps for the full-size lens and layered channel).
"""
import numpy as np
import pytest

import paper_2605_22214_amd as nf
import workloads as W
from oracle import analysis as A
from oracle import diag as odiag
from oracle import step as S
from oracle.coeffs import equal_sigma
from oracle.lattice import D2Q9, D3Q19

pytestmark = pytest.mark.gpu


def oracle_params(w, implicit=-1, **kw):
    lat = D2Q9 if w["lattice"] == "D2Q9" else D3Q19
    N = w["sigma"].shape[0]
    return S.Params(lat, w["shape"], w["sigma"], w["tau"], D=w["D"], omega_stab=w["omega_stab"],
                    trt_magic=w["trt_magic"], tau_g=w["tau_g"], m=w["m"],
                    body_force=w["body_force"], walls=w["walls"],
                    implicit=(N - 1 if implicit == -1 else implicit), **kw)


def rel(a, b):
    scale = np.abs(b).max()
    if scale == 0.0:
        return 0.0 if np.all(a == 0.0) else np.inf
    return float(np.abs(a - b).max() / scale)


def compare(sim, f, g, par, tol, label=""):
    mac = S.macroscopic(f, g, par)
    errs = {
        "C": rel(sim.get_field("C"), mac["C"]),
        "V": rel(sim.get_field("V"), mac["v"]),
        "P": rel(sim.get_field("P"), mac["P"]),
        "F": rel(sim.get_field("F"), mac["F"]),
    }
    mu = sim.get_field("MU")
    ev = par.evolved
    errs["MU"] = rel(mu[ev], mac["mu_tilde"][ev])
    errs["F_RAW"] = rel(sim.get_field("F_RAW"), f[1:])
    graw = sim.get_field("G_RAW")
    errs["G_RAW"] = rel(graw[ev], g[ev])
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, f"{label}: {errs}"
    return errs


def run_both(w, steps, precision=nf.FP64, implicit=-1, flags=0, okw=None):
    okw = okw or {}
    par = oracle_params(w, implicit, **okw)
    sim = nf.Simulation.from_workload(w, precision=precision, implicit=implicit, flags=flags)
    sim.set_fields(w["C0"], w.get("v0"))
    f, g = S.initial_state(par, w["C0"], w.get("v0"))
    sim.step(steps)
    for _ in range(steps):
        f, g, _ = S.step(f, g, par)
    return sim, f, g, par


def case_lens_ragged():
    return W.lens_2d(37, 29, radius=7.0)


def case_walls_trt():
    w = W.noise("D2Q9", (45, 21, 1), 4, amp=0.15, seed=11, sigma=0.006, m=0.05)
    w.update(walls=(False, True, False), trt_magic=3.0 / 16.0, body_force=(2e-6, -1e-6, 0.0),
             tau=np.array([0.6, 0.9, 1.3, 1.1]))
    return w


def case_omega_potential():
    sig = equal_sigma(4, 0.005)
    sig[0, 3] = sig[3, 0] = 0.012
    w = W.janus_2d(30, 26, radius=6.0, offset=7.0, sigma=sig)
    w["omega_stab"] = 1.0 / 18.0
    return w


def case_d3_absent():
    return W.noise("D3Q19", (19, 13, 11), 4, 5, amp=0.1, seed=4)


def case_d3_layered_walls():
    w = W.layered_3d(5, 3, 40, nlayers=4, force=1e-5)
    rng = np.random.default_rng(2)
    w["C0"] = w["C0"] + 0.02 * rng.uniform(size=w["C0"].shape)
    w["C0"] /= w["C0"].sum(axis=0)
    return w


def case_d3_thin(nz, walls):
    def mk():
        w = W.noise("D3Q19", (12, 10, nz), 4, amp=0.15, seed=20 + nz, sigma=0.006, m=0.05)
        w["walls"] = walls
        return w
    return mk


@pytest.mark.parametrize("name,mk,steps,implicit,flags", [
    ("lens_ragged", case_lens_ragged, 20, -1, 0),
    # one and two planes: the z march of the reconstruction wraps onto the
    # plane it starts from, or meets the walls at both ends at once
    ("d3_nz1", case_d3_thin(1, (False, False, False)), 8, -1, 0),
    ("d3_nz2", case_d3_thin(2, (False, False, False)), 8, -1, 0),
    ("d3_nz2_walls", case_d3_thin(2, (True, False, True)), 8, -1, 0),
    ("d3_nz3_walls", case_d3_thin(3, (False, True, True)), 8, -1, 0),
    # the largest N: seven evolved components in every per-node array
    ("d3_n8", lambda: W.noise("D3Q19", (13, 9, 11), 8, amp=0.05, seed=31, sigma=0.006, m=0.05), 8, -1, 0),
    ("d2_n8_walls", lambda: dict(W.noise("D2Q9", (33, 21, 1), 8, amp=0.05, seed=32, sigma=0.006, m=0.05),
                                 walls=(True, False, False)), 10, 3, 0),
    ("walls_trt", case_walls_trt, 30, -1, 0),
    ("omega", case_omega_potential, 25, 0, 0),
    ("potential_force", case_omega_potential, 25, 0, nf.FLAG_POTENTIAL_FORCE),
    ("d3_absent", case_d3_absent, 10, 0, 0),
    ("d3_layered_walls", case_d3_layered_walls, 15, -1, 0),
])
@pytest.mark.parametrize("form", ["moments", "populations"])
def test_fp64_parity_small(name, mk, steps, implicit, flags, form):
    w = mk()
    okw = {"force_form": "potential"} if flags & nf.FLAG_POTENTIAL_FORCE else {}
    extra = nf.FLAG_G_POPULATIONS if form == "populations" else 0
    sim, f, g, par = run_both(w, steps, implicit=implicit, flags=flags | extra, okw=okw)
    assert sim.storage_form() == form
    compare(sim, f, g, par, 1e-12, name)


def test_fp64_parity_tau_g_not_one():
    w = W.lens_2d(33, 17, radius=5.0)
    w["tau_g"] = np.array([0.8, 1.2, 1.0])
    sim, f, g, par = run_both(w, 15)
    assert sim.storage_form() == "populations"
    compare(sim, f, g, par, 1e-12, "tau_g")


def test_absent_component_bitwise_zero_all_precisions():
    w = case_d3_absent()
    for prec in (nf.FP64, nf.FP32, nf.FP16S):
        sim = nf.Simulation.from_workload(w, precision=prec, implicit=0)
        sim.set_fields(w["C0"])
        sim.step(30)
        C = sim.get_field("C")
        G = sim.get_field("G_RAW")
        assert np.all(C[4] == 0.0), prec
        assert np.all(G[4] == 0.0), prec
        assert np.all(sim.get_field("MU")[4] == 0.0), prec
        sim.close()


def test_lens_full_size_1000_steps_fp64():
    """64 x 64, N = 3 lens, tau = 1, m = 0.05, after 1000 steps."""
    w = W.lens_2d()
    sim, f, g, par = run_both(w, 1000)
    compare(sim, f, g, par, 1e-12, "lens 1000")


def test_layered_channel_full_size_1000_steps_fp64():
    """16 x 16 x 192, N = 6 between walls, TRT Lambda = 3/16, tau 0.6..1.5,
    F = 1e-7.  The oracle runs one x-y column (the problem is uniform in x and
    y, so every column of the full lattice must equal it)."""
    nz, F = 192, 1e-7
    eta = (np.linspace(0.6, 1.5, 6) - 0.5) / 3.0
    z = np.arange(nz) + 0.5
    prof = A.layered_profile(z, [32.0 * q for q in range(7)], eta, F)
    w = W.layered_3d(16, 16, nz, v0_profile=prof)
    wc = W.layered_3d(1, 1, nz, v0_profile=prof)
    par = oracle_params(wc)
    f, g = S.initial_state(par, wc["C0"], wc["v0"])
    sim = nf.Simulation.from_workload(w)
    sim.set_fields(w["C0"], w["v0"])
    steps = 1000
    sim.step(steps)
    for _ in range(steps):
        f, g, _ = S.step(f, g, par)
    mac = S.macroscopic(f, g, par)
    C = sim.get_field("C")
    V = sim.get_field("V")
    assert rel(C, np.broadcast_to(mac["C"], C.shape)) < 1e-12
    assert rel(V, np.broadcast_to(mac["v"], V.shape)) < 1e-12
    G = sim.get_field("G_RAW")
    assert rel(G[par.evolved], np.broadcast_to(g[par.evolved], G[par.evolved].shape)) < 1e-12


def test_diagnostics_match_oracle():
    w = W.lens_2d(40, 36, radius=8.0)
    w["body_force"] = (1e-6, 0.0, 0.0)
    sim, f, g, par = run_both(w, 40)
    d = sim.diagnostics(vcm_component=2)
    od = odiag.diagnostics(f, g, par, vcm_component=2)
    np.testing.assert_allclose(d["mass"], od["mass"], rtol=1e-13)
    np.testing.assert_allclose(d["momentum"][:2], od["momentum"][:2], rtol=1e-12, atol=1e-16)
    np.testing.assert_allclose(d["max_abs_c"], od["max_abs_c"], rtol=1e-12)
    np.testing.assert_allclose(d["min_c"], od["min_c"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(d["vcm"][:2], od["vcm"][:2], rtol=1e-12, atol=1e-18)
    assert d["nan"] == 0


def test_checkpoint_and_determinism():
    w = W.lens_2d(48, 40, radius=9.0)
    a = nf.Simulation.from_workload(w, precision=nf.FP32)
    a.set_fields(w["C0"])
    a.step(50)
    snap = a.get_state()
    a.step(50)
    ref = a.get_state()
    b = nf.Simulation.from_workload(w, precision=nf.FP32)
    b.set_state(snap)
    b.step(50)
    assert np.array_equal(b.get_state(), ref)
    c = nf.Simulation.from_workload(w, precision=nf.FP32)
    c.set_fields(w["C0"])
    c.step(100)
    assert np.array_equal(c.get_state(), ref)


@pytest.mark.parametrize("prec,tol", [(nf.FP32, 2e-5), (nf.FP16S, 2e-2)])
def test_reduced_precision_close_to_oracle(prec, tol):
    """Storage precision errors after 100 steps of the 64 x 64 lens.  FP32:
    about 1e-6 relative; FP16S (binary16 moving populations, about 2^-11
    relative each): about 1e-3 on C, more on the small fields v and P."""
    w = W.lens_2d()
    sim, f, g, par = run_both(w, 100, precision=prec)
    mac = S.macroscopic(f, g, par)
    e_c = rel(sim.get_field("C"), mac["C"])
    assert e_c < tol
    d = sim.diagnostics()
    od = odiag.diagnostics(f, g, par)
    np.testing.assert_allclose(d["mass"], od["mass"], rtol=1e-6)
