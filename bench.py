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

# Algorithmic memory work of one condensed-history step: one 8-byte voxel
# record gather and one 8-byte FP64 atomic add into the dose tally.
ALG_BYTES_PER_STEP = 16
HBM_PEAK = 8.0e12
# HBM bytes per transport launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs,
# scaled by a plain-copy calibration, valid only for the kernel source whose
# sha256 is recorded (see profiles/); None once the kernel has changed.
TRAFFIC = {"transport_sha256": "83fea2223ea3598eabfc2de9b7639fdb6cd38c25b7a08efeff8416bacad3fcd2",
           "bytes_per_launch": 1.24287e10, "let_bytes_per_launch": 2.59337e10}


def _kernel_sha():
    import hashlib
    with open(os.path.join(ROOT, "paper_1409_8336_amd", "csrc", "transport.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _cpu_model():
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return None


def cpu_baseline(cfg, target_s=15.0, single_s=8.0):
    """The FP64 oracle on this host: all threads (OpenMP over histories) on a
    sample sized for about target_s, then one thread on a sample sized for
    about single_s; the same field, CT and seeds."""
    from oracle import oracle as O
    from paper_1409_8336_amd import synth
    nd, mt = synth.nuclear_data(), synth.material_table()
    o = O.Oracle()
    o.load_physics(nd)
    o.load_geometry(cfg["hu"], cfg["voxel_cm"], mt)
    # a probe long enough that thread start-up does not dominate its rate
    probe = 100_000
    r = o.run_spots(cfg["spots"], probe, 2)
    rate = probe / max(r["summary"]["wall_s"], 1e-6)
    n = int(min(8_000_000, max(probe, rate * target_s)))
    r = o.run_spots(cfg["spots"], n, 3)
    s = r["summary"]
    o.close()
    o1 = O.Oracle(n_threads=1)
    o1.load_physics(nd)
    o1.load_geometry(cfg["hu"], cfg["voxel_cm"], mt)
    rate1 = (n / s["wall_s"]) / max(int(s["threads"]), 1)
    n1 = int(max(2_000, rate1 * single_s))
    r1 = o1.run_spots(cfg["spots"], n1, 4)
    s1 = r1["summary"]
    o1.close()
    # the smaller configurations in full on all threads: the water pencil
    # (1e5 histories) and the CT's three single spots (1e6 histories each)
    configs = {}
    for name, c in (("water pencil 100 MeV, 1e5", synth.config_water_pencil(100_000)),
                    ("CT spot 70 MeV, 1e6", synth.config_ct_spots(70.0, 1_000_000)),
                    ("CT spot 150 MeV, 1e6", synth.config_ct_spots(150.0, 1_000_000)),
                    ("CT spot 230 MeV, 1e6", synth.config_ct_spots(230.0, 1_000_000))):
        oc = O.Oracle()
        oc.load_physics(nd)
        oc.load_geometry(c["hu"], c["voxel_cm"], mt)
        rc = oc.run_spots(c["spots"], c["n_histories"], 1)["summary"]
        oc.close()
        configs[name] = {"histories_per_s": c["n_histories"] / rc["wall_s"], "wall_s": rc["wall_s"],
                         "steps_per_history": rc["steps"] / c["n_histories"]}
    return {"value": n / s["wall_s"], "unit": "histories/s", "cores": int(s["threads"]),
            "kind": "oracle", "configs": configs,
            "sample": "%d histories of the same 2000-spot field on the same CT (weights-"
                      "proportional allocation), wall %.2f s, %.1f steps/history"
                      % (n, s["wall_s"], s["steps"] / n),
            "single_thread": {"value": n1 / s1["wall_s"], "unit": "histories/s", "cores": 1,
                              "sample": "%d histories of the same field, wall %.2f s" % (n1, s1["wall_s"])},
            "cpu_model": _cpu_model()}


def copy_probe():
    """The library's plain read and plain copy kernels on 256 MiB (four
    launches each): the copy, of known size (256 MiB read + 256 MiB written
    per launch), is the reference that scales FETCH_SIZE / WRITE_SIZE
    counter readings."""
    from paper_1409_8336_amd import pmc
    eng = pmc.Engine(0)
    n = 256 * 1024 * 1024
    read_ms, copy_ms = pmc.pmc_stream_probe(eng.ctx, n)
    eng.close()
    print(json.dumps({"copy_probe_bytes": n, "launches": 4, "kernel": "copy_kernel",
                      "read_gbs": n / read_ms / 1e6, "copy_gbs": 2 * n / copy_ms / 1e6}))
    return 0


def bench_plans(args, leg=False):
    """Sixteen plans (grids 96^3..256x256x200, 200-3000 spots, 1e6-1e7
    histories each) in one persistent launch per generation.  leg: return
    the result instead of printing it."""
    import torch
    from paper_1409_8336_amd import pmc, synth
    plans = synth.plan_set(n_plans=16, seed=100)
    eng = pmc.Engine(0, **args.engine_params)
    eng.load_physics(synth.nuclear_data())
    mt = synth.material_table()
    eng.load_geometry(plans[0]["hu"], plans[0]["voxel_cm"], mt)
    ids = [0] + [pmc.pmc_load_geometry_slot(eng.ctx, p["hu"], p["voxel_cm"], mt) for p in plans[1:]]
    spec = []
    for gid, p in zip(ids, plans):
        d = torch.empty(p["hu"].shape, dtype=torch.float64, device="cuda:0")
        spec.append(dict(geometry_id=gid, spots=p["spots"], n_histories=p["n_histories"], d_dose=d,
                         d_var=torch.empty_like(d)))
    for _ in range(args.warmup):
        pmc.pmc_run_plans(eng.ctx, spec, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_sums = []
    for i in range(args.steps):
        all_sums.append(pmc.pmc_run_plans(eng.ctx, spec, 2 + i))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    n_tot = args.steps * sum(p["n_histories"] for p in plans)
    steps_tot = sum(s["steps"] for sums in all_sums for s in sums)
    out = {"metric": "proton histories/s (16-plan batch)", "value": n_tot / elapsed,
           "unit": "histories/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32 transport, f64 tallies",
           "data": "synthetic",
           "config": {"workload": "16 plans, CT 96^3..256x256x200 (2 mm), 200-3000 spots, "
                                  "1e6-1e7 histories each, one persistent launch",
                      "histories_per_step": n_tot // args.steps},
           "steps_per_s": steps_tot / elapsed,
           "launch_shape": {k: all_sums[-1][0][k] for k in ("block_threads", "grid_blocks",
                                                            "cache_slots", "epoch_steps", "refill_lanes",
                                                            "batch_events")},
           "transport_ms_per_step": sum(s[0]["transport_ms"] for s in all_sums) / args.steps,
           "per_plan": _plans_alone(eng, plans, spec, all_sums[-1], elapsed / args.steps),
           "denoiser_per_plan": _plans_denoiser(plans, spec),
           "ledger_residual_max": max(abs(s["incident"] - s["deposited"] - s["escaped"] - s["neutral"]
                                          - s["overflow"]) / s["incident"]
                                      for sums in all_sums for s in sums)}
    eng.close()
    if leg:
        return out
    print(json.dumps(out), flush=True)
    return 0


def _plans_alone(eng, plans, spec, sums, batch_s):
    """Every plan of the batch run on its own (a one-plan launch, after one
    untimed run that also tunes its shape): its wall time and rate, beside
    its share of the batch (the batch wall time split by the plans' steps).
    The sum of the solo times over the batch time is what running the plans
    together saves."""
    import torch
    from paper_1409_8336_amd import pmc
    steps_all = sum(s["steps"] for s in sums)
    rows, solo_total = [], 0.0
    for i, (p, sp) in enumerate(zip(plans, spec)):
        one = [dict(sp)]
        pmc.pmc_run_plans(eng.ctx, one, 50 + i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = pmc.pmc_run_plans(eng.ctx, one, 70 + i)[0]
        torch.cuda.synchronize()
        solo = time.perf_counter() - t0
        solo_total += solo
        rows.append({"grid": list(p["hu"].shape[::-1]), "spots": int(len(p["spots"])),
                     "histories": int(p["n_histories"]), "solo_ms": 1e3 * solo,
                     "solo_histories_per_s": p["n_histories"] / solo,
                     "batch_share_ms": 1e3 * batch_s * sums[i]["steps"] / steps_all,
                     "steps_per_history": r["steps"] / p["n_histories"]})
    return {"plans": rows, "solo_total_ms": 1e3 * solo_total, "batch_ms": 1e3 * batch_s,
            "batch_speedup_vs_one_by_one": solo_total / batch_s}


def _plans_denoiser(plans, spec):
    """Denoiser inference on every plan's dose after the batch: one network
    per plan, its sides rounded up to multiples of 8 (the plan's grid sits at
    the origin, zero outside). Times with the library's initial weights
    (the arithmetic does not depend on them)."""
    import torch
    from paper_1409_8336_amd import unet
    ms = []
    for p, sp in zip(plans, spec):
        d, h, w = (int(v) for v in p["hu"].shape)
        shape = (1,) + tuple(-(-v // 8) * 8 for v in (d, h, w))
        net = unet.UNet(shape, seed=1)
        rho = torch.ones((d, h, w), dtype=torch.float32, device="cuda:0")
        dose = sp["d_dose"].float()
        out = torch.empty_like(dose)
        net.forward_region(dose, rho, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            net.forward_region(dose, rho, out)
        torch.cuda.synchronize()
        ms.append(1e3 * (time.perf_counter() - t0) / 3)
        net.close()
    return {"ms": ms, "total_ms": sum(ms),
            "note": "one inference per plan on its own dose, networks sized to the plan's grid rounded up to 8; initial (untrained) weights: the kernels and their time do not depend on the values"}


def _small_configs(args):
    """The water pencil (1e5 histories) and the CT's single spots at 70, 150
    and 230 MeV (1e6 histories each) on the GPU: device time of a run, after
    one untimed run that also tunes the launch shape; the oracle's rates for
    the same runs are in cpu_baseline.configs."""
    import torch
    from paper_1409_8336_amd import pmc, synth
    res = {}
    for name, c in (("water pencil 100 MeV, 1e5", synth.config_water_pencil(100_000)),
                    ("CT spot 70 MeV, 1e6", synth.config_ct_spots(70.0, 1_000_000)),
                    ("CT spot 150 MeV, 1e6", synth.config_ct_spots(150.0, 1_000_000)),
                    ("CT spot 230 MeV, 1e6", synth.config_ct_spots(230.0, 1_000_000))):
        e = pmc.Engine(0, **args.engine_params)
        e.load_physics(synth.nuclear_data())
        e.load_geometry(c["hu"], c["voxel_cm"], synth.material_table())
        d = torch.empty(c["hu"].shape, dtype=torch.float64, device="cuda:0")
        v = torch.empty_like(d)
        e.run_spots_dev(c["spots"], c["n_histories"], 1, d, v)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 3
        for i in range(reps):
            sm = e.run_spots_dev(c["spots"], c["n_histories"], 2 + i, d, v)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        e.close()
        res[name] = {"histories_per_s": c["n_histories"] / el, "ms_per_run": 1e3 * el,
                     "device_ms": sm["device_ms"], "steps_per_history": sm["steps"] / c["n_histories"]}
    return res


def bench_ct_spots(args):
    """The 128x128x160 CT with titanium rod, one centred spot at 70, 150 and
    230 MeV, 1e6 histories each: histories/s and steps/s per energy."""
    import torch
    from paper_1409_8336_amd import pmc, synth
    per = {}
    total_h, total_s = 0, 0.0
    eng = pmc.Engine(0, **args.engine_params)
    eng.load_physics(synth.nuclear_data())
    cfg0 = synth.config_ct_spots(70.0, 1_000_000)
    eng.load_geometry(cfg0["hu"], cfg0["voxel_cm"], synth.material_table())
    d = torch.empty(cfg0["hu"].shape, dtype=torch.float64, device="cuda:0")
    v = torch.empty_like(d)
    for e_mev in (70.0, 150.0, 230.0):
        cfg = synth.config_ct_spots(e_mev, 1_000_000)
        for _ in range(args.warmup):
            eng.run_spots_dev(cfg["spots"], cfg["n_histories"], 1, d, v)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = 0
        for i in range(args.steps):
            steps += eng.run_spots_dev(cfg["spots"], cfg["n_histories"], 2 + i, d, v)["steps"]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        per["%g MeV" % e_mev] = {"histories_per_s": args.steps * cfg["n_histories"] / el,
                                 "steps_per_s": steps / el,
                                 "steps_per_history": steps / (args.steps * cfg["n_histories"])}
        total_h += args.steps * cfg["n_histories"]
        total_s += el
    eng.close()
    out = {"metric": "proton histories/s (CT single spots)", "value": total_h / total_s,
           "unit": "histories/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * total_s / (3 * args.steps), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32 transport, f64 tallies",
           "data": "synthetic",
           "config": {"workload": "128x128x160 CT (2 mm) with titanium rod, one centred spot "
                                  "(sigma 3 mm) at 70, 150, 230 MeV, 1e6 histories each"},
           "per_energy": per}
    print(json.dumps(out), flush=True)
    return 0


# algorithmic FLOP of one denoiser forward at 160x128x128: 2*27*cin*cout per
# output voxel and convolution (enc1 with its 8 padded input channels)
def unet_forward_flop(d, h, w):
    vox = [d * h * w >> (3 * l) for l in range(4)]
    convs = [(0, 8, 16), (1, 16, 32), (2, 32, 64), (3, 64, 128), (2, 192, 64), (1, 96, 32), (0, 48, 16)]
    return sum(2 * 27 * ci * co * vox[l] for l, ci, co in convs)


def bench_denoiser(args, leg=False):
    """The denoiser at 160x128x128 (one volume): inference and one training
    step (forward, backward, Adam), with the MFMA roofline of the
    convolutions: algorithmic FLOP / time against 2.5 PFLOP/s dense BF16.
    leg: return the result instead of printing it."""
    import torch
    import numpy as np
    from paper_1409_8336_amd import unet
    shape = (1, 160, 128, 128)
    rng = np.random.default_rng(1)
    dose = torch.from_numpy((rng.gamma(2.0, 1.0, shape) * 1e-11).astype(np.float32)).cuda()
    rho = torch.from_numpy(rng.uniform(0.2, 2.0, shape).astype(np.float32)).cuda()
    tgt = dose * 1.05
    out = torch.empty_like(dose)
    net = unet.UNet(shape, seed=1)
    for _ in range(args.warmup + 2):
        net.forward(dose, rho, out)
        net.backward(dose, rho, tgt)
        net.adam_step(1e-4)
    torch.cuda.synchronize()
    reps = max(args.steps, 5)
    t0 = time.perf_counter()
    for _ in range(reps):
        net.forward(dose, rho, out)
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        net.backward(dose, rho, tgt)
        net.adam_step(1e-4)
    torch.cuda.synchronize()
    t_train = (time.perf_counter() - t0) / reps
    net.close()
    fwd = unet_forward_flop(*shape[1:])
    peak = 2.5e15
    # the achievable matrix-core rate on this device: register-only MFMA stream
    p_ms, p_flop = unet.pmc_nn_mfma_probe(20000)
    probe = p_flop / (p_ms * 1e-3)
    out = {"metric": "denoiser inferences/s (160x128x128)", "value": 1.0 / t_inf, "unit": "volumes/s",
           "n_gpus": 1, "steps": reps, "warmup": args.warmup, "ms_per_step": 1e3 * t_inf,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "bf16 (fp32 accumulate)", "data": "synthetic",
           "config": {"workload": "3-D U-Net 16/32/64/128, one 160x128x128 volume, 730,481 parameters"},
           "train_step_ms": 1e3 * t_train,
           "roofline": {"bound": "mfma", "achieved": fwd / t_inf / 1e12, "peak": peak / 1e12,
                        "unit": "TFLOP/s", "frac": fwd / t_inf / peak, "traffic": None,
                        "kernel": "whole forward (7 convolutions and the elementwise kernels)",
                        "flop_per_forward": fwd,
                        "train_achieved": 3 * fwd / t_train / 1e12,
                        "mfma_probe_tflops": probe / 1e12,
                        "frac_of_probe": fwd / t_inf / probe}}
    if leg:
        return out
    print(json.dumps(out), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--histories", type=int, default=10_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=("field", "plans", "ct_spots", "denoiser"), default="field",
                    help="field: the 2000-spot 1e7-history field (default); plans: the "
                         "uneven 16-plan batch in one persistent launch; ct_spots: single "
                         "spots at 70/150/230 MeV in the 128x128x160 CT; denoiser: the U-Net "
                         "at 160x128x128 (inference and training step)")
    ap.add_argument("--let-steps", type=int, default=3,
                    help="field workload: also time this many runs with LET_d scored (0 = skip)")
    ap.add_argument("--inc-steps", type=int, default=2,
                    help="field workload: also time this many runs with non-elastic events by the "
                         "intranuclear cascade (PMC_INC; 0 = skip)")
    ap.add_argument("--option-steps", type=int, default=2,
                    help="field workload: also time this many runs with Vavilov-Gaussian "
                         "straggling and, separately, Moliere scattering (0 = skip)")
    ap.add_argument("--no-legs", dest="legs", action="store_false",
                    help="field workload: skip the 16-plan batch and denoiser legs")
    ap.add_argument("--no-replay", action="store_true",
                    help="field workload: skip the address-trace replay and the probes (counter runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--param", action="append", default=[], metavar="NAME=VALUE",
                    help="engine parameter (pmc_params field), e.g. tally_cache=-1; repeatable")
    args = ap.parse_args()
    args.engine_params = {}
    for kv in args.param:
        k, v = kv.split("=", 1)
        args.engine_params[k] = float(v) if "." in v else int(v)
    if args.copy_probe:
        return copy_probe()
    if args.gpus != 1:
        print("bench.py measures one GPU: the engine runs on a single MI355X and has no "
              "multi-GPU path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2
    import torch
    from paper_1409_8336_amd import pmc, synth

    if args.workload == "plans":
        return bench_plans(args)
    if args.workload == "ct_spots":
        return bench_ct_spots(args)
    if args.workload == "denoiser":
        return bench_denoiser(args)
    cfg = synth.config_field(args.histories)
    eng = pmc.Engine(0, **args.engine_params)
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
    launches = sum(s["launches"] for s in sums)
    achieved = ALG_BYTES_PER_STEP * steps_tot / transport_s
    # the transport's own address stream replayed without the physics, and
    # the plain-read bandwidth of this device
    if args.no_replay:
        # counter runs: the timed transport runs and the legs only
        rep = {"trace_only_ms": 0.0, "gather_ms": 0.0, "atomic_ms": 0.0, "cached_atomic_ms": 0.0,
               "combined_ms": 0.0, "transport_ms": 1e3 * transport_s / launches,
               "steps": steps_tot // args.steps, "steps_traced": 0}
        stream_read_gbs = None
    else:
        rep = pmc.pmc_roofline_replay(eng.ctx, cfg["spots"], cfg["n_histories"], cfg["seed"], stream)
        read_ms, _ = pmc.pmc_stream_probe(eng.ctx, 4 << 30, stream)
        stream_read_gbs = (4 << 30) / read_ms / 1e6
    t_tr = rep["trace_only_ms"]
    t_gather = rep["gather_ms"] - t_tr
    t_atom = min(rep["atomic_ms"], rep["cached_atomic_ms"]) - t_tr
    t_mem = max(t_gather, t_atom) if not args.no_replay else 1e3 * transport_s / launches
    deposits_tot = sum(s["tally_atomics"] for s in sums)
    atomics_tot = sum(s["global_atomics"] for s in sums)
    flush_tot = sum(s["cache_flush_atomics"] for s in sums)
    probe_ms = (pmc.pmc_atomic_probe(eng.ctx, max(1, atomics_tot // args.steps), stream) if not args.no_replay
                else 1e3 * transport_s / args.steps)
    probe_rate = (atomics_tot / args.steps) / (probe_ms * 1e-3)
    atomic_rate = atomics_tot / transport_s
    traffic = None
    if TRAFFIC["transport_sha256"] == _kernel_sha():
        traffic = TRAFFIC["bytes_per_launch"]
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
                   "grid": list(cfg["hu"].shape[::-1]), "k_batches": 10,
                   "engine_params": args.engine_params},
        "steps_per_s": steps_tot / elapsed,
        "secondaries_per_s": sum(s["secondaries"] for s in sums) / elapsed,
        "steps_per_history": steps_tot / n_tot,
        "transport_launches_per_step": launches / args.steps,
        "launch_shape": {k: sums[-1][k] for k in ("block_threads", "grid_blocks", "cache_slots",
                                                   "epoch_steps", "refill_lanes", "batch_events")},
        "transport_ms_per_step": 1e3 * transport_s / args.steps,
        "ledger_residual_max": worst_res,
        # roofline of the transport against the replay of its own address
        # stream -- every step's 8-B voxel gather and 8-B FP64 tally add, in
        # the traced run's order, grid, workgroups, lanes and epochs -- replayed
        # without the physics; the slower of the gather replay and the faster
        # of the direct and LDS-cached atomic replays is the achievable time
        # of the method's memory operations.  frac = that time / the launch.
        "roofline": {
            "bound": "atomic" if t_atom >= t_gather else "gather",
            "achieved": ALG_BYTES_PER_STEP * rep["steps"] / (rep["transport_ms"] * 1e-3) / 1e9,
            "peak": ALG_BYTES_PER_STEP * rep["steps"] / (t_mem * 1e-3) / 1e9,
            "unit": "GB/s",
            "frac": t_mem / rep["transport_ms"],
            "traffic": traffic,
            "kernel": "transport_kernel",
            "basis": "replay of the transport's own gather and FP64-atomic address stream (16 B per step); "
                     "peak = algorithmic bytes / replay time of the binding stream",
            "avg_launch_ms": 1e3 * transport_s / launches,
            "launches_per_step": launches / args.steps,
            "bytes_per_step": ALG_BYTES_PER_STEP,
            "replay": {
                "transport_ms": rep["transport_ms"],
                "gather_ms": t_gather,
                "atomic_ms": rep["atomic_ms"] - t_tr,
                "cached_atomic_ms": rep["cached_atomic_ms"] - t_tr,
                "combined_ms": rep["combined_ms"] - t_tr,
                "combined_frac": (rep["combined_ms"] - t_tr) / rep["transport_ms"],
                "trace_stream_ms": t_tr,
                "steps_traced_frac": rep["steps_traced"] / rep["steps"],
                "note": "replay times net of streaming the 4-byte-per-lane-iteration trace",
            },
            # the same launches against HBM: 16 B per step over the average
            # launch time, against 8 TB/s (HBM does not bind)
            "hbm": {"achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK, "stream_read_gbs": stream_read_gbs,
                    "traffic": traffic},
        },
        "atomic_roofline": {
            "deposits_per_step": deposits_tot / args.steps,
            "tally_atomics_per_step": atomics_tot / args.steps,
            "flush_atomics_per_step": flush_tot / args.steps,
            "achieved_atomics_per_s": atomic_rate,
            "probe_atomics_per_s": probe_rate,
            "frac": atomic_rate / probe_rate,
            "probe": "pmc_atomic_probe: the same number of FP64 atomics into the same tally "
                     "along straight z tracks in the central 40x40 window",
            "note": "deposits go through a per-workgroup LDS cache; tally atomics are the "
                    "FP64 adds that reach device memory (cache misses and flushes)",
        },
    }
    # the same workload with dose-averaged LET scored in the same transport
    # (Sec. III): its rate beside the dose-only one
    if args.let_steps > 0:
        d_let = torch.empty_like(d_dose)
        eng.run_spots_let_dev(cfg["spots"], cfg["n_histories"], cfg["seed"], d_dose, d_let, d_var, stream)
        torch.cuda.synchronize()
        lsums = []
        t0 = time.perf_counter()
        for i in range(args.let_steps):
            lsums.append(eng.run_spots_let_dev(cfg["spots"], cfg["n_histories"], cfg["seed"] + i, d_dose,
                                               d_let, d_var, stream))
        torch.cuda.synchronize()
        let_elapsed = time.perf_counter() - t0
        dose_rate = n_tot / elapsed
        let_rate = args.let_steps * cfg["n_histories"] / let_elapsed
        let_transport_s = sum(s["transport_ms"] for s in lsums) * 1e-3
        let_atomics = sum(s["global_atomics"] for s in lsums)
        out["let_d"] = {
            "histories_per_s": let_rate,
            "achieved_atomics_per_s": let_atomics / let_transport_s,
            "atomic_frac": (let_atomics / let_transport_s) / probe_rate,
            "traffic_bytes_per_launch": (TRAFFIC["let_bytes_per_launch"]
                                         if TRAFFIC["transport_sha256"] == _kernel_sha() else None),
            "ms_per_step": 1e3 * let_elapsed / args.let_steps,
            "transport_ms_per_step": sum(s["transport_ms"] for s in lsums) / args.let_steps,
            "rate_vs_dose_only": let_rate / dose_rate,
            "deposits_per_step": sum(s["tally_atomics"] for s in lsums) / args.let_steps,
            "tally_atomics_per_step": sum(s["global_atomics"] for s in lsums) / args.let_steps,
            "launch_shape": {k: lsums[-1][k] for k in ("block_threads", "grid_blocks", "cache_slots",
                                                        "refill_lanes", "batch_events")},
            "steps": args.let_steps,
        }
        del d_let
    # the same workload with non-elastic events by the intranuclear cascade
    # and evaporation (Sec. II.A.4) instead of the secondary tables
    if args.inc_steps > 0:
        params = dict(args.engine_params)
        params["flags"] = int(params.get("flags", 0)) | pmc.PMC_INC
        ei = pmc.Engine(0, **params)
        ei.load_physics(synth.nuclear_data())
        ei.load_geometry(cfg["hu"], cfg["voxel_cm"], synth.material_table())
        ei.run_spots_dev(cfg["spots"], cfg["n_histories"], cfg["seed"], d_dose, d_var, stream)
        torch.cuda.synchronize()
        isums = []
        t0 = time.perf_counter()
        for i in range(args.inc_steps):
            isums.append(ei.run_spots_dev(cfg["spots"], cfg["n_histories"], cfg["seed"] + i, d_dose, d_var,
                                          stream))
        torch.cuda.synchronize()
        inc_elapsed = time.perf_counter() - t0
        ei.close()
        k = args.inc_steps
        out["inc"] = {
            "histories_per_s": k * cfg["n_histories"] / inc_elapsed,
            "rate_vs_tables": (k * cfg["n_histories"] / inc_elapsed) / (n_tot / elapsed),
            "ms_per_step": 1e3 * inc_elapsed / k,
            "transport_ms_per_step": sum(s["transport_ms"] for s in isums) / k,
            "cascade_ms_per_step": sum(s["inc_ms"] for s in isums) / k,
            "events_per_step": sum(s["inc_events"] for s in isums) / k,
            "cascade_protons_per_step": sum(s["inc_secondaries"] for s in isums) / k,
            "nn_collisions_per_step": sum(s["inc_collisions"] for s in isums) / k,
            "generations": isums[-1]["generations"],
            "launches_per_step": sum(s["launches"] for s in isums) / k,
            "ledger_residual_max": max(abs(s["incident"] - s["deposited"] - s["escaped"] - s["neutral"]
                                           - s["overflow"]) / s["incident"] for s in isums),
            "steps": k,
        }
    # the transport options of Sec. II.A.2 on the same workload: each in an
    # engine of its own (its first run tunes the launch shape)
    if args.option_steps > 0:
        out["options"] = {}
        dose_rate = n_tot / elapsed
        for name, flag in (("vavilov", pmc.PMC_VAVILOV), ("moliere", pmc.PMC_MOLIERE)):
            params = dict(args.engine_params)
            params["flags"] = int(params.get("flags", 0)) | flag
            eo = pmc.Engine(0, **params)
            eo.load_physics(synth.nuclear_data())
            eo.load_geometry(cfg["hu"], cfg["voxel_cm"], synth.material_table())
            eo.run_spots_dev(cfg["spots"], cfg["n_histories"], cfg["seed"], d_dose, d_var, stream)
            torch.cuda.synchronize()
            osums = []
            t0 = time.perf_counter()
            for i in range(args.option_steps):
                osums.append(eo.run_spots_dev(cfg["spots"], cfg["n_histories"], cfg["seed"] + i, d_dose, d_var,
                                              stream))
            torch.cuda.synchronize()
            o_elapsed = time.perf_counter() - t0
            eo.close()
            k = args.option_steps
            out["options"][name] = {
                "histories_per_s": k * cfg["n_histories"] / o_elapsed,
                "rate_vs_default": (k * cfg["n_histories"] / o_elapsed) / dose_rate,
                "ms_per_step": 1e3 * o_elapsed / k,
                "transport_ms_per_step": sum(s["transport_ms"] for s in osums) / k,
                "steps_per_history": sum(s["steps"] for s in osums) / (k * cfg["n_histories"]),
                "launch_shape": {kk: osums[-1][kk] for kk in ("block_threads", "grid_blocks", "cache_slots",
                                                              "refill_lanes", "batch_events")},
                "ledger_residual_max": max(abs(s["incident"] - s["deposited"] - s["escaped"] - s["neutral"]
                                               - s["overflow"]) / s["incident"] for s in osums),
                "steps": k,
            }
    # the other workloads, briefly, so that the same run records them: the
    # uneven 16-plan batch (config 5) and the denoiser (config 4)
    if args.legs:
        import argparse as _ap
        la = _ap.Namespace(**vars(args))
        la.steps, la.warmup = 2, 1
        pb = bench_plans(la, leg=True)
        out["plans_batch"] = {k: pb[k] for k in ("value", "unit", "ms_per_step", "steps", "config",
                                                  "launch_shape", "transport_ms_per_step", "per_plan",
                                                  "denoiser_per_plan", "ledger_residual_max")}
        out["small_configs"] = _small_configs(args)
        la.steps = 5
        dn = bench_denoiser(la, leg=True)
        out["denoiser"] = {k: dn[k] for k in ("value", "unit", "ms_per_step", "train_step_ms", "config",
                                               "roofline")}
    # the same run through host buffers: spots in, dose and variance copied
    # back over PCIe (context only; not the headline value)
    t0 = time.perf_counter()
    eng.run_spots(cfg["spots"], cfg["n_histories"], cfg["seed"])
    out["host_buffers_histories_per_s"] = cfg["n_histories"] / (time.perf_counter() - t0)
    eng.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
