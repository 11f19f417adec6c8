"""Batches of independent simulations and the launch-shape autotuner.

A batch step runs the same per-node arithmetic as a single simulation's step,
only with the tiles of every member in one launch, so every member must end
bit for bit where it ends when stepped alone -- in every stepping mode
(one launch pair per step, HIP-graph replay, per-member sequences) and
whatever the tile shape.  FP64 members are also checked against the oracle.
"""
import os

import numpy as np
import pytest

import paper_2605_22214_amd as nf
import workloads as W
from oracle import step as S
from oracle.lattice import D2Q9

pytestmark = pytest.mark.gpu


def uneven_members(count, seed, sides):
    ws = W.batch_members(count=count, seed=seed, sides=sides)
    # a member with walls on y and one with a body force, so the batch mixes
    # wall handling and options per member
    ws[1]["walls"] = (False, True, False)
    ws[0]["body_force"] = (2e-6, -1e-6, 0.0)
    return ws


def states(sims):
    return [s.get_state() for s in sims]


def standalone(ws, precision, steps):
    out = []
    for w in ws:
        s = nf.Simulation.from_workload(w, precision=precision)
        s.set_fields(w["C0"])
        s.step(steps)
        out.append(s.get_state())
        s.close()
    return out


@pytest.mark.parametrize("prec", [nf.FP32, nf.FP16S, nf.FP64])
@pytest.mark.parametrize("mode", ["graph", "launch", "per_sim"])
def test_batch_bitwise_equals_standalone(prec, mode):
    sides = [37, 64, 50, 96, 33, 70]
    ws = uneven_members(len(sides), 11, sides)
    steps = 27  # odd: whole graph replays plus a remainder, and a parity flip
    ref = standalone(ws, prec, steps)
    with nf.Batch.from_workloads(ws, precision=prec) as b:
        b.set_launch(graph_steps=8)
        for i, w in enumerate(ws):
            b.members[i].set_fields(w["C0"])
        b.step(steps, mode=mode)
        got = states(b.members)
    for i in range(len(ws)):
        assert np.array_equal(got[i], ref[i]), f"member {i} ({sides[i]}^2)"


@pytest.mark.parametrize("tx_log2", [4, 6])
def test_batch_tile_shapes_agree(tx_log2):
    sides = [40, 96, 17]
    ws = uneven_members(len(sides), 3, sides)
    ref = standalone(ws, nf.FP32, 12)
    with nf.Batch.from_workloads(ws, precision=nf.FP32) as b:
        b.set_launch(tx_log2=tx_log2, graph_steps=4)
        assert b.get_launch()[0] == tx_log2
        for i, w in enumerate(ws):
            b.members[i].set_fields(w["C0"])
        b.step(12, mode="graph")
        got = states(b.members)
    for i in range(len(ws)):
        assert np.array_equal(got[i], ref[i])


def test_graph_replays_match_eager_each_time():
    """Several replays of one captured graph, with host reads and syncs in
    between, each compared with eager launches of the same steps."""
    sides = [48, 64, 35]
    ws = uneven_members(len(sides), 5, sides)
    with nf.Batch.from_workloads(ws, precision=nf.FP32) as bg, \
            nf.Batch.from_workloads(ws, precision=nf.FP32) as be:
        for b in (bg, be):
            b.set_launch(graph_steps=6)
            for i, w in enumerate(ws):
                b.members[i].set_fields(w["C0"])
        for rep in range(4):
            bg.step(6, mode="graph")
            be.step(6, mode="launch")
            for i in range(len(ws)):
                assert np.array_equal(bg.members[i].get_state(), be.members[i].get_state()), (rep, i)
            _ = bg.members[0].diagnostics()   # eager work between replays


def test_member_stepped_alone_then_batch():
    """A member advanced on its own by an odd count leaves the batch's
    argument tables stale; the next batch step must rebuild them."""
    sides = [40, 56]
    ws = uneven_members(len(sides), 7, sides)
    ref = []
    for i, w in enumerate(ws):
        s = nf.Simulation.from_workload(w, precision=nf.FP32)
        s.set_fields(w["C0"])
        s.step(10 + (3 if i == 0 else 0))
        ref.append(s.get_state())
        s.close()
    with nf.Batch.from_workloads(ws, precision=nf.FP32) as b:
        b.set_launch(graph_steps=4)
        for i, w in enumerate(ws):
            b.members[i].set_fields(w["C0"])
        b.step(4, mode="graph")
        b.members[0].step(3)
        b.step(6, mode="graph")
        got = states(b.members)
    for i in range(len(ws)):
        assert np.array_equal(got[i], ref[i])


def test_batch_fp64_matches_oracle():
    sides = [24, 31]
    ws = uneven_members(len(sides), 9, sides)
    steps = 20
    with nf.Batch.from_workloads(ws, precision=nf.FP64) as b:
        b.set_launch(graph_steps=4)
        for i, w in enumerate(ws):
            b.members[i].set_fields(w["C0"])
        b.step(steps, mode="graph")
        got = [m.get_field("C") for m in b.members]
        gotv = [m.get_field("V") for m in b.members]
    for i, w in enumerate(ws):
        par = S.Params(D2Q9, w["shape"], w["sigma"], w["tau"], D=w["D"],
                       omega_stab=w["omega_stab"], m=w["m"], walls=w["walls"],
                       body_force=w["body_force"])
        f, g = S.initial_state(par, w["C0"])
        for _ in range(steps):
            f, g, _ = S.step(f, g, par)
        mac = S.macroscopic(f, g, par)
        Co = mac["C"]
        assert np.abs(got[i] - Co).max() <= 1e-12 * np.abs(Co).max(), i
        vo = mac["v"]
        assert np.abs(gotv[i] - vo).max() <= 1e-12 * max(np.abs(vo).max(), 1e-30) + 1e-18, i


def test_batch_d3q19_with_walls():
    probs = []
    for k, (shape, walls) in enumerate((((20, 12, 9), (False, False, True)),
                                        ((16, 16, 16), (False, False, False)),
                                        ((11, 7, 5), (True, False, False)))):
        w = W.noise("D3Q19", shape, 4, seed=40 + k, sigma=0.006, m=0.05, tau=1.0)
        w["walls"] = walls
        probs.append(w)
    ref = standalone(probs, nf.FP32, 9)
    with nf.Batch.from_workloads(probs, precision=nf.FP32) as b:
        b.set_launch(graph_steps=4)
        for i, w in enumerate(probs):
            b.members[i].set_fields(w["C0"])
        b.step(9, mode="graph")
        got = states(b.members)
    for i in range(len(probs)):
        assert np.array_equal(got[i], ref[i]), i


def test_autotune_keeps_state_and_caches(tmp_path):
    w = W.quaternary_3d(32)
    cache = str(tmp_path / "tune.txt")
    with nf.Simulation.from_workload(w, precision=nf.FP32, implicit=0) as s:
        s.set_fields(w["C0"])
        s.step(3)
        before = s.get_state()
        shape = s.autotune(cache)
        assert shape[0] in (4, 6) and 1 <= shape[1] <= 32
        assert shape[3] in (4, 6) and 1 <= shape[4] <= 32
        assert np.array_equal(s.get_state(), before)
        s.step(5)
        after_tuned = s.get_state()
    with open(cache) as fh:
        lines = fh.read().splitlines()
    assert len(lines) == 1 and lines[0].endswith(f"|{shape[0]} {shape[1]} {shape[3]} {shape[4]}")
    with nf.Simulation.from_workload(w, precision=nf.FP32, implicit=0) as s:
        s.set_fields(w["C0"])
        s.step(3)
        again = s.autotune(cache)                      # from the cache
        assert again[:2] == shape[:2] and again[3:] == shape[3:]
        s.step(5)
        assert np.array_equal(s.get_state(), after_tuned)
    with open(cache) as fh:
        assert len(fh.read().splitlines()) == 1


def test_batch_autotune_keeps_state(tmp_path):
    sides = [64, 96, 40]
    ws = uneven_members(len(sides), 13, sides)
    ref = standalone(ws, nf.FP32, 10)
    cache = str(tmp_path / "btune.txt")
    with nf.Batch.from_workloads(ws, precision=nf.FP32) as b:
        for i, w in enumerate(ws):
            b.members[i].set_fields(w["C0"])
        tx, gs, blocks = b.autotune(cache)
        assert tx in (4, 6) and blocks > 0
        b.step(10, mode="graph")
        got = states(b.members)
    for i in range(len(ws)):
        assert np.array_equal(got[i], ref[i])
    assert os.path.getsize(cache) > 0


def test_reconstruction_launch_shapes_agree():
    """The reconstruction's own launch shape changes no bit of the result."""
    w = W.quaternary_3d(24, nz=19)
    ref = None
    for tx, zc in ((6, 1), (4, 4), (4, 19), (6, 7)):
        with nf.Simulation.from_workload(w, precision=nf.FP32, implicit=0) as s:
            s.set_conc_launch(tx, zc)
            assert s.get_conc_launch() == (tx, zc)
            s.set_fields(w["C0"])
            s.step(11)
            st = s.get_state()
        if ref is None:
            ref = st
        assert np.array_equal(st, ref), (tx, zc)
