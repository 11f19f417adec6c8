"""Throughput of the N-component free-energy LBM update on one MI355X.

Workload: D3Q19 quaternary phase separation with a fifth component that is
exactly zero (the reduction-consistency check), 256^3 periodic nodes,
C_i = 0.25 + U(-0.02, 0.02) renormalised (seed 0), sigma = 0.01 for every
pair, tau = tau_g = 1, m = 0.1.  One "step" is one full time step of the
method over the whole lattice (concentration reconstruction + the fused
stencil / force / collide / stream launch).

Prints ONE JSON line.  value = MLUPS (million lattice-node updates per second)
of the FP32-storage form; the FP16S and FP64 forms are timed the same way and
reported under "forms".  roofline: the update kernel's algorithmic HBM bytes
per launch divided by its mean launch time (HIP events on the stream the
kernel runs on), against the 8 TB/s HBM3E peak.  cpu_baseline: the FP64 NumPy
oracle on a 64^3 sample of the same recipe.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS at N components (FP32/FP16-store vs FP64) and % of HBM roofline"
HBM_PEAK_GBS = 8000.0
Q = 19


def update_bytes_per_node(N, fs, g0s, ts):
    """Algorithmic HBM bytes of one update launch per node: read the Q-1
    moving f populations, the N-1 reconstructed concentrations and E_B, write
    the Q-1 f populations and all Q populations of the N-1 evolved
    components (halo re-reads of C and E_B are not counted)."""
    NE = N - 1
    return (Q - 1) * fs + (NE + 1) * ts + (Q - 1) * fs + NE * ((Q - 1) * fs + g0s)


def conc_bytes_per_node(N, fs, g0s, ts):
    """Read all Q populations of the N-1 evolved components, write C and E_B."""
    NE = N - 1
    return NE * ((Q - 1) * fs + g0s) + (NE + 1) * ts


SIZES = {"fp64": (8, 8, 8), "fp32": (4, 4, 4), "fp16s": (2, 4, 4)}

# HBM bytes per node of one update launch at 256^3, from rocprofv3 FETCH_SIZE
# and WRITE_SIZE (each scaled by what the counter reads for a 1 GiB device copy:
# x2.0 and x1.0), keyed by the SHA-256 of the kernel sources they were taken on.
# The committed summary under profiles/ gives the commands and the raw figures.
TRAFFIC = {
    "sources_sha256": "2d5dbdf1c73613d9f4b2c4958aaf8585c500cdbbc49b6974853ca4ce653e2cb2",
    "n": 256,
    "update_bytes_per_node": {"fp32": 490.7, "fp16s": 257.8, "fp64": 942.7},
}
KERNEL_SOURCES = ("paper_2605_22214_amd/csrc/kernels.hip", "paper_2605_22214_amd/csrc/internal.h")


def kernel_sources_sha256():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def run_form(nf, w, form, steps, warmup, timing_steps):
    import torch
    prec = nf.PRECISIONS[form]
    sim = nf.Simulation.from_workload(w, precision=prec, implicit=0)
    sim.set_fields(w["C0"])
    d0 = sim.diagnostics(vcm_component=0)
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_events = sim.step_timed(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # separate pass: events around every update launch (same stream)
    _, ms_upd = sim.step_timed(timing_steps, per_update=True)
    d1 = sim.diagnostics(vcm_component=0)
    n = w["C0"][0].size
    mlups = n * steps / wall / 1e6
    fs, g0s, ts = SIZES[form]
    N = w["sigma"].shape[0]
    ub = update_bytes_per_node(N, fs, g0s, ts)
    cb = conc_bytes_per_node(N, fs, g0s, ts)
    upd_ms = ms_upd / timing_steps
    out = {
        "mlups": mlups,
        "ms_per_step": wall / steps * 1e3,
        "ms_per_step_events": ms_events / steps,
        "update_ms": upd_ms,
        "update_bytes_per_node": ub,
        "step_bytes_per_node": ub + cb,
        "update_gbs": n * ub / (upd_ms * 1e-3) / 1e9,
        "step_gbs": n * (ub + cb) / (wall / steps) / 1e9,
        "absent_max_abs": d1["max_abs_c"][4],
        "mass_rel_drift": max(abs(a - b) / abs(b) for a, b in zip(d1["mass"][:4], d0["mass"][:4])),
        "momentum_drift": [a - b for a, b in zip(d1["momentum"], d0["momentum"])],
        "nan": d1["nan"],
    }
    out["step_frac_of_peak"] = out["step_gbs"] / HBM_PEAK_GBS
    sim.close()
    return out


def run_batch(nf, count, steps, per_sim_steps, seed=0):
    """Batch of independent D2Q9 N=3 lens / Janus problems (sides 64..512 in
    steps of 32, sigma_13 and sigma_23 drawn from U[0.0025, 0.01]), FP32
    storage: graph replay of whole-batch steps against each member's own
    launch sequence.  MLUPS counts the nodes of all members."""
    import workloads as W
    ws = W.batch_members(count=count, seed=seed)
    b = nf.Batch.from_workloads(ws, precision=nf.FP32)
    for i, w in enumerate(ws):
        b.members[i].set_fields(w["C0"])
    nodes = b.nodes()
    tx, graph_steps, blocks = b.autotune()
    b.step(2 * graph_steps, "graph")
    ms_graph = b.step_timed(steps, "graph")
    ms_launch = b.step_timed(max(2, steps // 10), "launch")
    b.step(2, "per_sim")
    ms_per = b.step_timed(per_sim_steps, "per_sim")
    absent_nan = max(m.diagnostics(check=False)["nan"] for m in b.members[:8])
    b.close()
    graph = nodes * steps / (ms_graph * 1e-3) / 1e6
    per = nodes * per_sim_steps / (ms_per * 1e-3) / 1e6
    return {"workload": f"{count} independent D2Q9 N=3 lens/Janus problems, sides 64..512, FP32",
            "nodes": nodes, "tile_x": 1 << tx, "graph_steps": graph_steps, "workgroups": blocks,
            "graph_mlups": graph, "graph_steps_timed": steps,
            "launch_mlups": nodes * max(2, steps // 10) / (ms_launch * 1e-3) / 1e6,
            "per_sim_mlups": per, "per_sim_steps_timed": per_sim_steps,
            "speedup_graph_vs_per_sim": graph / per, "nan_in_first_8": absent_nan}


def cpu_baseline(sample_n=64, steps=60):
    """The FP64 oracle (not tuned) on a sample_n^3 lattice of the same recipe."""
    import workloads as W
    from oracle import step as S
    from oracle.lattice import D3Q19
    w = W.quaternary_3d(sample_n)
    par = S.Params(D3Q19, w["shape"], w["sigma"], w["tau"], m=w["m"], implicit=0)
    f, g = S.initial_state(par, w["C0"])
    f, g, _ = S.step(f, g, par)
    t0 = time.perf_counter()
    for _ in range(steps):
        f, g, _ = S.step(f, g, par)
    dt = time.perf_counter() - t0
    return {"value": sample_n ** 3 * steps / dt / 1e6, "unit": "MLUPS", "cores": 1,
            "kind": "oracle",
            "sample": f"{sample_n}^3 D3Q19 N=5 (same recipe), {steps} steps, NumPy FP64 on one "
                      f"core ({len(os.sched_getaffinity(0))} visible), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256, help="lattice side")
    ap.add_argument("--forms", default="fp32,fp16s,fp64")
    ap.add_argument("--timing-steps", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batch-count", type=int, default=256,
                    help="members of the batch measurement (0 skips it)")
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 1 GiB, 3 times (for scaling the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 4 * (1 << 28)}))
        return
    if args.gpus != 1:
        print(f"bench.py: this workload runs on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU domain decomposition is not part of this build)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    import paper_2605_22214_amd as nf
    import workloads as W
    nf.lib()
    w = W.quaternary_3d(args.n)
    forms = [f for f in args.forms.split(",") if f]
    results = {}
    for form in forms:
        print(f"bench: timing {form} ({args.n}^3, {args.steps} steps)", file=sys.stderr, flush=True)
        results[form] = run_form(nf, w, form, args.steps, args.warmup, args.timing_steps)
        print(f"bench: {form} {results[form]['mlups']:.1f} MLUPS", file=sys.stderr, flush=True)
    batch = None
    if args.batch_count > 0:
        print(f"bench: batch of {args.batch_count} D2Q9 problems", file=sys.stderr, flush=True)
        batch = run_batch(nf, args.batch_count, args.batch_steps, max(2, args.batch_steps // 10))
        print(f"bench: batch {batch['graph_mlups']:.0f} MLUPS (graph) vs {batch['per_sim_mlups']:.0f} "
              "(per simulation)", file=sys.stderr, flush=True)
    main_form = forms[0]
    r = results[main_form]
    traffic = None
    if (kernel_sources_sha256() == TRAFFIC["sources_sha256"] and args.n == TRAFFIC["n"]
            and main_form in TRAFFIC["update_bytes_per_node"]):
        traffic = TRAFFIC["update_bytes_per_node"][main_form] * args.n ** 3
    roof = {"bound": "hbm", "achieved": r["update_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": r["update_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_unit": "bytes per launch (FETCH_SIZE x2.0 + WRITE_SIZE x1.0)",
            "kernel": "k_update", "bytes_per_node": r["update_bytes_per_node"],
            "mean_launch_ms": r["update_ms"]}
    cpu = None
    if not args.no_cpu:
        print("bench: timing the CPU oracle sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline()
    line = {
        "metric": METRIC,
        "value": r["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16s": "f16-store/f32", "fp64": "f64"}[main_form],
        "data": "synthetic",
        "config": {"workload": f"D3Q19 quaternary phase separation + absent 5th component, "
                               f"{args.n}^3 periodic, {main_form} storage",
                   "lattice": "D3Q19", "shape": [args.n] * 3, "ncomp": 5, "precision": main_form},
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": results,
        "batch": batch,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
