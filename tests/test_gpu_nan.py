"""NaN detection on the stepping path and the diagnostics' in-kernel sums.

* A NaN put into the state through nflbm_set_fields (data, not a fault) is
  found by the first checked step: nflbm_synchronize and nflbm_step_timed
  return ENUMERIC at once, nflbm_step on the call after the flag's copy has
  arrived, and nflbm_diagnostics reports nan = 1.  Steps before the first
  checked one (every 16th by default) report nothing; nflbm_set_fields with
  finite data clears the state.  Both storage forms of g, D2Q9 and D3Q19.
* Batches check every step with one flag for the whole batch.
* nflbm_diagnostics on a lattice with more tiles than the reduction grid
  (grid-stride over tiles) equals the FP64 sums of the fields read back.
"""
import numpy as np
import pytest

import paper_2605_22214_amd as nf
import workloads as W

pytestmark = pytest.mark.gpu

ENUMERIC = -6


def _device_sync():
    import torch
    torch.cuda.synchronize()


def _with_nan(w, node=(3, 5)):
    C0 = np.array(w["C0"], dtype=float, copy=True)
    C0[0, 0, node[1], node[0]] = np.nan
    return C0


@pytest.mark.parametrize("lattice,flags", [("D2Q9", 0), ("D2Q9", nf.FLAG_G_POPULATIONS),
                                           ("D3Q19", 0), ("D3Q19", nf.FLAG_G_POPULATIONS)])
def test_nan_is_reported_by_the_checked_steps(lattice, flags):
    if lattice == "D2Q9":
        w = W.lens_2d(32, 24, radius=6.0)
    else:
        w = W.noise("D3Q19", (12, 10, 8), 3, 4, amp=0.1, seed=3)
    with nf.Simulation.from_workload(w, precision=nf.FP32, flags=flags) as sim:
        sim.set_fields(_with_nan(w))
        sim.step(15)                      # no checked step yet (every 16th)
        sim.synchronize()
        sim.step(1)                       # step 16 is checked
        with pytest.raises(nf.NflbmError) as e:
            sim.synchronize()
        assert e.value.code == ENUMERIC
        d = sim.diagnostics(check=False)
        assert d["nan"] == 1 and d["status"] == ENUMERIC
        # finite data clears it
        sim.set_fields(w["C0"])
        sim.step(40)
        sim.synchronize()
        assert sim.diagnostics()["nan"] == 0


def test_step_reports_nan_on_the_next_call_without_waiting():
    w = W.lens_2d(32, 24, radius=6.0)
    with nf.Simulation.from_workload(w, precision=nf.FP64) as sim:
        sim.set_nan_check(1)
        sim.set_fields(_with_nan(w))
        sim.step(4)                       # queues the steps and the flag's copy
        _device_sync()                    # the copy has now arrived
        with pytest.raises(nf.NflbmError) as e:
            sim.step(1)
        assert e.value.code == ENUMERIC
        with pytest.raises(nf.NflbmError):
            sim.step(1)                   # stays until the state is replaced
        with pytest.raises(nf.NflbmError) as e:
            sim.step_timed(2)
        assert e.value.code == ENUMERIC


def test_nan_check_off_and_set_state_clears():
    w = W.lens_2d(32, 24, radius=6.0)
    with nf.Simulation.from_workload(w, precision=nf.FP32) as sim:
        sim.set_fields(w["C0"])
        clean = sim.get_state()
        sim.set_nan_check(0)
        sim.set_fields(_with_nan(w))
        sim.step(40)
        sim.synchronize()                 # nothing checked
        assert sim.diagnostics(check=False)["nan"] == 1
        sim.set_nan_check(2)
        sim.step(2)
        with pytest.raises(nf.NflbmError):
            sim.synchronize()
        sim.set_state(clean)
        sim.step(4)
        sim.synchronize()
        with pytest.raises(nf.NflbmError):
            sim.set_nan_check(-1)


def test_batch_reports_nan():
    ws = [W.lens_2d(32, 24, radius=6.0), W.lens_2d(40, 32, radius=7.0)]
    with nf.Batch.from_workloads(ws, precision=nf.FP32) as b:
        b.set_fields(0, ws[0]["C0"])
        b.set_fields(1, _with_nan(ws[1]))
        with pytest.raises(nf.NflbmError) as e:
            b.step_timed(4, mode="launch")
        assert e.value.code == ENUMERIC
        b.set_fields(1, ws[1]["C0"])
        b.step_timed(4, mode="graph")     # cleared
        b.step(4, mode="launch")
        _device_sync()
        b.set_fields(0, _with_nan(ws[0]))
        b.step(2, mode="launch")
        _device_sync()
        with pytest.raises(nf.NflbmError):
            b.step(2, mode="launch")


@pytest.mark.parametrize("prec", [nf.FP64, nf.FP32])
def test_diagnostics_grid_stride_match_field_sums(prec):
    """4096 tiles of 16 x 16 on a 1024^2 lattice, more than the 2048
    workgroups of the reduction: every tile is still summed once."""
    w = W.quaternary_2d(1024)
    with nf.Simulation.from_workload(w, precision=prec) as sim:
        sim.set_fields(w["C0"])
        sim.step(30)
        d = sim.diagnostics(vcm_component=1)
        C = sim.get_field("C")
        V = sim.get_field("V")
    tol = 1e-12
    np.testing.assert_allclose(d["mass"], C.sum(axis=(1, 2, 3)), rtol=tol)
    np.testing.assert_allclose(d["momentum"][:2], V[:2].sum(axis=(1, 2, 3)), rtol=1e-9,
                               atol=1e-12 * np.abs(V).sum())
    np.testing.assert_array_equal(d["max_abs_c"], np.abs(C).max(axis=(1, 2, 3)))
    np.testing.assert_array_equal(d["min_c"], C.min(axis=(1, 2, 3)))
    assert d["max_sum_dev"] == pytest.approx(np.abs(C.sum(axis=0) - 1.0).max(), abs=1e-15)
    cm = C[1].sum()
    np.testing.assert_allclose(d["vcm"][:2], (C[1] * V[:2]).sum(axis=(1, 2, 3)) / cm, rtol=1e-9,
                               atol=1e-12 * np.abs(V).max())
    assert d["nan"] == 0
