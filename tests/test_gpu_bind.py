"""Device state in caller memory (nflbm_bind_state) and coefficient read-back.

A torch tensor provides the memory; results must equal those of a simulation
that keeps library memory, bit for bit, across a re-bind to a second tensor,
and closing the simulation must leave the tensor usable."""
import numpy as np
import pytest

import paper_2605_22214_amd as nf
import workloads as W
from oracle.coeffs import Coefficients

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("flags", [0, nf.FLAG_G_POPULATIONS])
def test_bound_state_matches_library_memory(flags):
    import torch
    w = W.noise("D3Q19", (24, 20, 14), 4, 5, amp=0.1, seed=6)
    ref = nf.Simulation.from_workload(w, precision=nf.FP32, implicit=0, flags=flags)
    ref.set_fields(w["C0"])
    ref.step(9)
    want = ref.get_state()
    ref.close()
    nbytes = nf.Simulation.device_bytes(w["lattice"], w["shape"], w["sigma"], w["tau"], implicit=0,
                                        D=w["D"], m=w["m"], precision=nf.FP32, flags=flags)
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    ptr = (buf.data_ptr() + 255) // 256 * 256
    sim = nf.Simulation.from_workload(w, precision=nf.FP32, implicit=0, flags=flags)
    sim.set_fields(w["C0"])
    sim.step(4)
    sim.bind_state(ptr, nbytes)          # state moves into the tensor mid-run
    sim.step(2)
    buf2 = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    ptr2 = (buf2.data_ptr() + 255) // 256 * 256
    sim.bind_state(ptr2, nbytes)         # and again
    sim.step(3)
    assert np.array_equal(sim.get_state(), want)
    with pytest.raises(nf.NflbmError):
        sim.bind_state(ptr2 + 8, nbytes)          # misaligned
    with pytest.raises(nf.NflbmError):
        sim.bind_state(ptr, nbytes - 256)          # too small
    sim.close()
    buf2.fill_(7)                                  # still the caller's memory
    torch.cuda.synchronize()
    assert int(buf2[-1].item()) == 7


def test_get_coeffs_match_oracle():
    sig = np.array([[0, 0.005, 0.003, 0.004], [0.005, 0, 0.006, 0.0045],
                    [0.003, 0.006, 0, 0.0055], [0.004, 0.0045, 0.0055, 0]])
    with nf.Simulation("D2Q9", (16, 16, 1), sig, 1.0, m=0.05) as s:
        a, g = s.get_coeffs()
    o = Coefficients(sig, 4.0)
    assert np.abs(a - o.alpha).max() < 1e-12 * np.abs(o.alpha).max()
    assert np.abs(g - o.gamma).max() < 1e-14
