"""nflbm_diagnostics_noalloc through the C ABI: the diagnostics of
nflbm_diagnostics with the reduction's partial records in the library's
fixed device array instead of a buffer it allocates.  Checked against
nflbm_diagnostics on two calls in a row, the second on a smaller lattice
(the array keeps the first call's records; the second must not read them),
then once more on the first lattice."""
import numpy as np
import pytest

import paper_2605_22214_amd as nf
import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("mass", "momentum", "max_abs_c", "min_c", "vcm")


def _close(a, b):
    for k in KEYS:
        x, y = np.asarray(a[k]), np.asarray(b[k])
        scale = max(float(np.abs(y).max()), 1e-300)
        assert float(np.abs(x - y).max()) <= 1e-12 * scale, (k, a[k], b[k])
    assert abs(a["max_sum_dev"] - b["max_sum_dev"]) <= 1e-15
    assert a["nan"] == b["nan"] == 0


def test_noalloc_diagnostics_match_allocating_diagnostics():
    # 48 x 48 x 40 in 16 x 16 tiles: more workgroups than the 2048 records
    big = W.noise("D3Q19", (48, 48, 40), 4, 5, seed=1, amp=0.1)
    small = W.lens_2d(40, 28, radius=6.0)
    sims = []
    for w, implicit, vcm in ((big, 0, 2), (small, -1, 1)):
        sim = nf.Simulation.from_workload(w, precision=nf.FP64, implicit=implicit)
        sim.set_fields(w["C0"])
        sim.step(12)
        a = sim.diagnostics_noalloc(vcm_component=vcm)
        b = sim.diagnostics(vcm_component=vcm)
        _close(a, b)
        assert a["mass"] == b["mass"]           # the same kernels in the same order
        sims.append((sim, vcm))
    sim, vcm = sims[0]
    sim.step(3)
    _close(sim.diagnostics_noalloc(vcm_component=vcm), sim.diagnostics(vcm_component=vcm))
    for s, _ in sims:
        s.close()


def test_noalloc_reports_nan():
    w = W.lens_2d(32, 24, radius=6.0)
    C0 = np.array(w["C0"], copy=True)
    C0[0, 0, 4, 4] = np.nan
    with nf.Simulation.from_workload(w, precision=nf.FP32) as sim:
        sim.set_fields(C0)
        sim.step(3)
        d = sim.diagnostics_noalloc(check=False)
        assert d["nan"] == 1 and d["status"] == -6
