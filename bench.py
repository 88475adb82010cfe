#!/usr/bin/env python3
"""Benchmark: proton histories per second on one MI355X.

Workload: 256x256x200 synthetic CT (2 mm voxels, water with lung, soft
tissue, bone ellipsoids and a titanium rod) irradiated by a 2000-spot
treatment-field stand-in (40 energy layers 70-230 MeV, 5 mm hexagonal grid,
lognormal weights), 1e7 histories per step, FP32 transport state, FP64 dose
and variance tallies.  One step = one full pmc_run_spots_dev call (every
transport generation plus the dose statistics) with the geometry and tables
already resident in HBM.

Prints one JSON line.  The roofline object refers to the transport kernel,
timed with HIP events around each of its launches on the launch stream; the
cpu_baseline object is the FP64 oracle on a bounded sample of the same
workload on this host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU lane-operations of one condensed-history step of the method (counted
# per operation of the step's arithmetic; see the design notes) and the
# chip's peak VALU lane-operation rate: 256 CUs x 64 lanes x 2.4 GHz.
OPS_PER_STEP = 300
PEAK_LANE_OPS = 256 * 64 * 2.4e9


def cpu_baseline(cfg, target_s=10.0):
    from oracle import oracle as O
    from paper_1409_8336_amd import synth
    o = O.Oracle()
    o.load_physics(synth.nuclear_data())
    o.load_geometry(cfg["hu"], cfg["voxel_cm"], synth.material_table())
    probe = 20000
    r = o.run_spots(cfg["spots"], probe, 2)
    rate = probe / max(r["summary"]["wall_s"], 1e-6)
    n = int(min(2_000_000, max(probe, rate * target_s)))
    r = o.run_spots(cfg["spots"], n, 3)
    s = r["summary"]
    o.close()
    return {"value": n / s["wall_s"], "unit": "histories/s", "cores": int(s["threads"]),
            "kind": "oracle",
            "sample": "%d histories of the same 2000-spot field on the same CT (weights-"
                      "proportional allocation), wall %.2f s, %.1f steps/history"
                      % (n, s["wall_s"], s["steps"] / n)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--histories", type=int, default=10_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs on a single MI355X and has no "
              "multi-GPU path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2
    import torch
    from paper_1409_8336_amd import pmc, synth

    cfg = synth.config_field(args.histories)
    eng = pmc.Engine(0)
    eng.load_physics(synth.nuclear_data())
    eng.load_geometry(cfg["hu"], cfg["voxel_cm"], synth.material_table())
    dev = torch.device("cuda:0")
    d_dose = torch.empty(cfg["hu"].shape, dtype=torch.float64, device=dev)
    d_var = torch.empty_like(d_dose)
    stream = torch.cuda.current_stream(dev)
    for _ in range(args.warmup):
        eng.run_spots_dev(cfg["spots"], cfg["n_histories"], cfg["seed"], d_dose, d_var, stream)
    torch.cuda.synchronize()
    sums = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        sums.append(eng.run_spots_dev(cfg["spots"], cfg["n_histories"], cfg["seed"] + i, d_dose,
                                      d_var, stream))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    n_tot = args.steps * cfg["n_histories"]
    steps_tot = sum(s["steps"] for s in sums)
    transport_s = sum(s["transport_ms"] for s in sums) * 1e-3
    launches = sum(s["generations"] for s in sums)
    achieved = OPS_PER_STEP * steps_tot / transport_s
    worst_res = max(abs(s["incident"] - s["deposited"] - s["escaped"] - s["neutral"] - s["overflow"])
                    / s["incident"] for s in sums)
    out = {
        "metric": "proton histories/s (1e7, CT)",
        "value": n_tot / elapsed,
        "unit": "histories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 transport, f64 tallies",
        "data": "synthetic",
        "config": {"workload": "256x256x200 CT (2 mm), 2000-spot 40-layer field 70-230 MeV, "
                               "1e7 histories per step",
                   "histories_per_step": cfg["n_histories"], "spots": int(len(cfg["spots"])),
                   "grid": list(cfg["hu"].shape[::-1]), "k_batches": 10},
        "steps_per_s": steps_tot / elapsed,
        "steps_per_history": steps_tot / n_tot,
        "transport_launches_per_step": launches / args.steps,
        "transport_ms_per_step": 1e3 * transport_s / args.steps,
        "ledger_residual_max": worst_res,
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_LANE_OPS / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_LANE_OPS,
            "traffic": None,
            "kernel": "transport_kernel",
            "avg_launch_ms": 1e3 * transport_s / launches,
            "ops_per_step": OPS_PER_STEP,
        },
    }
    eng.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
