"""Denoiser workflow on one GPU: data set generation with the transport
engine, training of the 3-D U-Net, and the time-to-gamma evaluation.

The learned denoiser has no counterpart in the paper; its evaluation uses
the paper's plan-comparison tool, the 3-D gamma index (Sec. II.D), and the
paper's statistical error estimate (Eq. 5) for the fallback rule.

Data set (inputs are synthetic): case i is a ct_phantom-recipe CT of
128x128x160 voxels of 2 mm with seed 1000 + i and a random field of 1-3
energy layers of 10-60 spots (synth.denoiser_case); the network input is
the dose of n_low histories (Philox key 10000 + i) and the density map, the
target the dose of n_high histories (key 20000 + i).

Time to gamma (per held-out case): the reference is its n_high dose.  Plain
Monte Carlo is swept over SWEEP histories (key 30000 + 16 i + k); T_plain is
the wall time of the smallest N whose gamma pass rate against the reference
reaches 98 % (2 %/2 mm global, 10 % cutoff, 3 mm search at 0.5 mm; the
same at 1 %/1 mm as a stricter second criterion).  The denoised plan costs T_den = T_MC(n_low) +
T_infer when its own pass rate reaches 98 %, else the plain sweep is paid on
top (fallback).  The deployable fallback rule (no reference needed) is also
evaluated: fall back when more than 2 % of the voxels above 10 % of the
maximum differ from the noisy dose by more than 4 of its standard errors.

Run: python -m paper_1409_8336_amd.denoise --cases 400 --held-out 40
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import pmc, synth, unet

SWEEP = (100_000, 200_000, 500_000, 1_000_000, 2_000_000, 5_000_000, 10_000_000, 20_000_000)
# 2 %/2 mm global, 10 % cutoff, 3 mm search at 0.5 mm; and a stricter 1 %/1 mm
CRITERIA = {"2%/2mm": dict(dose_frac=0.02, dta_cm=0.2, cutoff_frac=0.1, search_cm=0.3, step_cm=0.05),
            "1%/1mm": dict(dose_frac=0.01, dta_cm=0.1, cutoff_frac=0.1, search_cm=0.3, step_cm=0.05)}


def _log(msg):
    print("[denoise %s] %s" % (time.strftime("%H:%M:%S"), msg), flush=True)
    sys.stdout.flush()


class Simulator:
    """One transport context with the default physics and material table."""

    def __init__(self, device=0):
        import torch
        self.torch = torch
        self.engine = pmc.Engine(device)
        self.engine.load_physics(synth.nuclear_data())
        self.mt = synth.material_table()
        self.shape = None

    def load(self, case):
        self.engine.load_geometry(case["hu"], case["voxel_cm"], self.mt)
        self.shape = case["hu"].shape

    def density(self):
        rho = self.torch.empty(self.shape, dtype=self.torch.float32, device="cuda")
        pmc.pmc_geometry_density(self.engine.ctx, 0, rho)
        return rho

    def run(self, spots, n, seed, var=True):
        """Dose and variance (float64 device tensors) of n histories and the
        wall time of the call (spots in, results resident on the GPU)."""
        torch = self.torch
        dose = torch.empty(self.shape, dtype=torch.float64, device="cuda")
        v = torch.empty_like(dose) if var else None
        torch.cuda.synchronize()
        t = time.perf_counter()
        self.engine.run_spots_dev(spots, n, seed, dose, v)
        torch.cuda.synchronize()
        return dose, v, time.perf_counter() - t

    def close(self):
        self.engine.close()


def build_dataset(sim, indices, n_low, n_high, log=_log):
    """GPU-resident float32 stacks [len(indices), nz, ny, nx] of low- and
    high-history dose and density, plus the cases' spot lists."""
    torch = sim.torch
    low = high = rho = None
    spots = []
    t0 = time.perf_counter()
    for j, i in enumerate(indices):
        case = synth.denoiser_case(i)
        sim.load(case)
        if low is None:
            shape = (len(indices),) + case["hu"].shape
            low = torch.empty(shape, dtype=torch.float32, device="cuda")
            high = torch.empty_like(low)
            rho = torch.empty_like(low)
        rho[j].copy_(sim.density())
        d, _, _ = sim.run(case["spots"], n_low, 10_000 + i, var=False)
        low[j].copy_(d)
        d, _, _ = sim.run(case["spots"], n_high, 20_000 + i, var=False)
        high[j].copy_(d)
        spots.append(case["spots"])
        if j % 20 == 0 or j == len(indices) - 1:
            log("data %d/%d (case %d, %d spots) %.1f s" % (j + 1, len(indices), i, len(case["spots"]),
                                                         time.perf_counter() - t0))
    return {"low": low, "high": high, "rho": rho, "spots": spots, "indices": list(indices)}


def train(net, data, rows, seconds, lr_max=5e-4, lr_min=1e-5, seed=0, max_steps=None, batch=4,
          clip=3.0, log=_log):
    """Adam on the gradient summed over `batch` full volumes per step (the
    backward call adds into the gradient buffer), cosine learning-rate decay
    over the time budget; a step whose gradient norm exceeds `clip` times the
    running mean of the norms (after 20 steps) is scaled down to that bound.
    Returns [(step, elapsed_s, mean loss of the step)]; net.n_clipped counts
    the clipped steps."""
    import torch
    rng = np.random.default_rng(seed)
    hist = []
    t0 = time.perf_counter()
    step = 0
    last_log = t0
    order = []
    ema, n_clipped = None, 0
    while True:
        el = time.perf_counter() - t0
        if el >= seconds or (max_steps is not None and step >= max_steps):
            break
        frac = min(1.0, el / seconds)
        lr = lr_min + 0.5 * (lr_max - lr_min) * (1 + math.cos(math.pi * frac))
        loss = 0.0
        for _ in range(batch):
            if not order:
                order = list(rng.permutation(rows))
            r = order.pop()
            loss += net.backward(data["low"][r], data["rho"][r], data["high"][r]) / batch
        norm = net.grad_norm()
        scale = 1.0
        if clip and ema is not None and step >= 20 and norm > clip * ema:
            scale = clip * ema / norm
            n_clipped += 1
        ema = norm if ema is None else 0.95 * ema + 0.05 * norm * scale
        net.adam_step(lr, grad_scale=scale)
        step += 1
        hist.append((step, el, loss))
        if time.perf_counter() - last_log > 30:
            recent = np.mean([h[2] for h in hist[-100:]])
            log("train step %d  %.0f s  lr %.2e  loss(avg 100) %.4e  grad norm (mean) %.3e  clipped %d"
                % (step, el, lr, recent, ema, n_clipped))
            last_log = time.perf_counter()
    torch.cuda.synchronize()
    net.n_clipped = n_clipped
    return hist


def _mean_rel_error(a, ref, frac=0.1):
    m = ref >= frac * ref.max()
    return float(np.mean(np.abs(a[m] - ref[m]) / ref[m]))


def evaluate(sim, net, data, rows, log=_log, sweep=SWEEP):
    """Time-to-gamma of plain Monte Carlo against the denoised low-history
    dose for each held-out row."""
    torch = sim.torch
    out = []
    vox = (0.2, 0.2, 0.2)
    # the engine calibrates its launch shape once per problem size: do that
    # outside the timed runs
    case = synth.denoiser_case(data["indices"][rows[0]])
    sim.load(case)
    for n in sweep:
        sim.run(case["spots"], n, 1, var=False)
    for r in rows:
        i = data["indices"][r]
        case = synth.denoiser_case(i)
        sim.load(case)
        ref = data["high"][r].double()
        ref_h = ref.cpu().numpy()
        # noisy input, timed, with its variance (fresh key: a new realisation)
        low, var_low, t_low = sim.run(case["spots"], SWEEP[0], 40_000 + i)
        rho = data["rho"][r]
        low32 = low.float()
        den = torch.empty_like(low32)
        net.forward(low32, rho, den)          # warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        net.forward(low32, rho, den)
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t
        disagree, _ = unet.pmc_denoise_disagreement(den, low, var_low, 0.1, 4.0)
        rule_fallback = disagree > 0.02
        plain = [sim.run(case["spots"], n, 30_000 + 16 * i + k, var=False) for k, n in enumerate(sweep)]
        rec = {"case": i, "t_mc_low_s": t_low, "t_infer_s": t_inf, "disagreement": disagree,
               "rule_fallback": bool(rule_fallback),
               "mre_denoised": _mean_rel_error(den.double().cpu().numpy(), ref_h),
               "mre_low": _mean_rel_error(low.cpu().numpy(), ref_h),
               "plain_wall_s": [p[2] for p in plain], "plain_n": list(sweep)}
        for name, crit in CRITERIA.items():
            g_den, n_eval = unet.pmc_gamma_index(ref, den.double(), vox, **crit)
            g_low, _ = unet.pmc_gamma_index(ref, low, vox, **crit)
            rates = [unet.pmc_gamma_index(ref, p[0], vox, **crit)[0] for p in plain]
            t_plain = n_plain = None
            for n, (_, _, tt), g in zip(sweep, plain, rates):
                if g >= 0.98:
                    t_plain, n_plain = tt, n
                    break
            ok = g_den >= 0.98
            t_den = t_low + t_inf + (0.0 if ok else (t_plain if t_plain is not None else plain[-1][2]))
            rec[name] = {"n_eval": n_eval, "gamma_pass_denoised": g_den, "gamma_pass_low": g_low,
                         "plain_gamma_pass": rates, "t_plain_s": t_plain, "n_plain": n_plain,
                         "t_den_s": t_den, "denoised_ok": bool(ok),
                         "speedup": (t_plain / t_den) if t_plain is not None else None}
            log("eval case %d %s: gamma den %.4f low %.4f  N_plain %s  T_plain %s  T_den %.4f s  speedup %s"
                % (i, name, g_den, g_low, n_plain, "%.4f" % t_plain if t_plain else "-", t_den,
                   "%.2f" % rec[name]["speedup"] if rec[name]["speedup"] else "-"))
        log("eval case %d: T_MC(low) %.2f ms  T_infer %.2f ms  disagreement %.4f  MRE den %.4f low %.4f"
            % (i, 1e3 * t_low, 1e3 * t_inf, disagree, rec["mre_denoised"], rec["mre_low"]))
        out.append(rec)
    return out


def evaluate_plans(sim, params, plans, n_low=100_000, n_ref=100_000_000, log=_log, sweep=SWEEP):
    """Time-to-gamma on the uneven plans of the batch workload: per plan the
    reference is its n_ref-history dose, the denoiser input its n_low-history
    dose (a network of the trained weights sized to the plan's grid rounded
    up to multiples of 8, the plan at the origin, zero outside), and plain
    Monte Carlo is swept over `sweep`; also the pass rate of the plan's own
    history count."""
    torch = sim.torch
    out = []
    for pi, plan in enumerate(plans):
        sim.load(plan)
        d, h, w = (int(v) for v in plan["hu"].shape)
        net = unet.UNet((1,) + tuple(-(-v // 8) * 8 for v in (d, h, w)), seed=0)
        net.set_params(params)
        for n in sweep + (n_low, plan["n_histories"]):   # launch-shape calibration outside the timed runs
            sim.run(plan["spots"], n, 1, var=False)
        ref, _, t_ref = sim.run(plan["spots"], n_ref, 50_000 + pi, var=False)
        low, var_low, t_low = sim.run(plan["spots"], n_low, 60_000 + pi)
        own, _, t_own = sim.run(plan["spots"], plan["n_histories"], 70_000 + pi, var=False)
        rho = sim.density()
        low32 = low.float()
        den = torch.empty_like(low32)
        net.forward_region(low32, rho, den)    # warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        net.forward_region(low32, rho, den)
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t
        net.close()
        disagree, _ = unet.pmc_denoise_disagreement(den, low, var_low, 0.1, 4.0)
        plain = [sim.run(plan["spots"], n, 80_000 + 16 * pi + k, var=False) for k, n in enumerate(sweep)]
        ref_h = ref.cpu().numpy()
        rec = {"plan": pi, "grid": [d, h, w], "spots": int(len(plan["spots"])), "n_plan": plan["n_histories"],
               "t_plan_s": t_own, "t_ref_s": t_ref, "t_mc_low_s": t_low, "t_infer_s": t_inf,
               "disagreement": disagree, "rule_fallback": bool(disagree > 0.02),
               "mre_denoised": _mean_rel_error(den.double().cpu().numpy(), ref_h),
               "mre_low": _mean_rel_error(low.cpu().numpy(), ref_h),
               "plain_wall_s": [p_[2] for p_ in plain], "plain_n": list(sweep)}
        for name, crit in CRITERIA.items():
            g_den, n_eval = unet.pmc_gamma_index(ref, den.double(), vox_of(plan), **crit)
            g_low, _ = unet.pmc_gamma_index(ref, low, vox_of(plan), **crit)
            g_own, _ = unet.pmc_gamma_index(ref, own, vox_of(plan), **crit)
            rates = [unet.pmc_gamma_index(ref, p_[0], vox_of(plan), **crit)[0] for p_ in plain]
            t_plain = n_plain = None
            for n, (_, _, tt), g in zip(sweep, plain, rates):
                if g >= 0.98:
                    t_plain, n_plain = tt, n
                    break
            ok = g_den >= 0.98
            t_den = t_low + t_inf + (0.0 if ok else (t_plain if t_plain is not None else plain[-1][2]))
            rec[name] = {"n_eval": n_eval, "gamma_pass_denoised": g_den, "gamma_pass_low": g_low,
                         "gamma_pass_plan_n": g_own, "plain_gamma_pass": rates, "t_plain_s": t_plain,
                         "n_plain": n_plain, "t_den_s": t_den, "denoised_ok": bool(ok),
                         "speedup": (t_plain / t_den) if t_plain is not None else None}
            log("plan %d %s: gamma den %.4f low %.4f plan-N %.4f  N_plain %s  T_plain %s  T_den %.4f s  speedup %s"
                % (pi, name, g_den, g_low, g_own, n_plain, "%.4f" % t_plain if t_plain else "-", t_den,
                   "%.2f" % rec[name]["speedup"] if rec[name]["speedup"] else "-"))
        log("plan %d %s, %d spots, N %d: T_plan %.2f ms  T_MC(low) %.2f ms  T_infer %.2f ms  MRE den %.4f low %.4f"
            % (pi, "x".join(map(str, (w, h, d))), len(plan["spots"]), plan["n_histories"], 1e3 * t_own,
               1e3 * t_low, 1e3 * t_inf, rec["mre_denoised"], rec["mre_low"]))
        out.append(rec)
    return out


def vox_of(plan):
    return tuple(float(v) for v in plan["voxel_cm"])


def summarize(recs):
    out = {
        "cases": len(recs),
        "median_mre_denoised": float(np.median([r["mre_denoised"] for r in recs])),
        "median_mre_low": float(np.median([r["mre_low"] for r in recs])),
        "median_t_infer_ms": 1e3 * float(np.median([r["t_infer_s"] for r in recs])),
        "median_t_mc_low_ms": 1e3 * float(np.median([r["t_mc_low_s"] for r in recs])),
        "rule_fallbacks": int(sum(r["rule_fallback"] for r in recs)),
    }
    for name in CRITERIA:
        rs = [r[name] for r in recs]
        sp = [x["speedup"] for x in rs if x["speedup"] is not None]
        out[name] = {
            "median_speedup": float(np.median(sp)) if sp else None,
            "cases_with_plain_reaching_98": len(sp),
            "denoised_pass_98": int(sum(x["denoised_ok"] for x in rs)),
            "median_gamma_denoised": float(np.median([x["gamma_pass_denoised"] for x in rs])),
            "median_gamma_low": float(np.median([x["gamma_pass_low"] for x in rs])),
            "median_n_plain": float(np.median([x["n_plain"] for x in rs if x["n_plain"]])) if sp else None,
            "rule_agrees_with_gamma": int(sum(r["rule_fallback"] == (not r[name]["denoised_ok"]) for r in recs)),
        }
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--cases", type=int, default=400)
    ap.add_argument("--held-out", type=int, default=40)
    ap.add_argument("--n-low", type=int, default=100_000)
    ap.add_argument("--n-high", type=int, default=100_000_000)
    ap.add_argument("--train-seconds", type=float, default=300.0)
    ap.add_argument("--lr", type=float, default=5e-4)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None)
    ap.add_argument("--save-params", default=None)
    ap.add_argument("--load-params", default=None,
                    help="trained weights (.npy from --save-params): skip the data set and training")
    ap.add_argument("--plans", type=int, default=0,
                    help="also evaluate time to gamma on this many plans of the uneven batch workload")
    ap.add_argument("--plan-ref", type=int, default=100_000_000, help="reference histories per plan")
    a = ap.parse_args(argv)
    import torch
    sim = Simulator(0)
    if a.load_params:
        params = np.load(a.load_params)
        recs = evaluate_plans(sim, params, synth.plan_set(a.plans or 16, seed=100), a.n_low, a.plan_ref)
        summ = summarize(recs)
        summ.update({"plans": len(recs), "n_low": a.n_low, "n_ref": a.plan_ref, "params": a.load_params})
        _log("plan summary %s" % json.dumps(summ))
        if a.out:
            with open(a.out, "w") as f:
                json.dump({"summary": summ, "plans": recs}, f, indent=1)
        sim.close()
        torch.cuda.synchronize()
        return
    t0 = time.perf_counter()
    data = build_dataset(sim, range(a.cases), a.n_low, a.n_high)
    t_data = time.perf_counter() - t0
    n_train = a.cases - a.held_out
    # one volume [1, d, h, w] per call
    net = unet.UNet((1,) + tuple(data["low"].shape[1:]), seed=a.seed)
    hist = train(net, data, list(range(n_train)), a.train_seconds, lr_max=a.lr, seed=a.seed,
                 batch=a.batch)
    _log("trained %d steps in %.0f s, final loss(avg 100) %.4e"
         % (len(hist), hist[-1][1], np.mean([h[2] for h in hist[-100:]])))
    if a.save_params:
        np.save(a.save_params, net.params())
    recs = evaluate(sim, net, data, list(range(n_train, a.cases)))
    summ = summarize(recs)
    summ.update({"data_s": t_data, "train_steps": len(hist), "train_s": hist[-1][1],
                 "final_loss": float(np.mean([h[2] for h in hist[-100:]])), "n_low": a.n_low,
                 "n_high": a.n_high, "cases_total": a.cases, "train_cases": n_train, "batch": a.batch,
                 "lr_max": a.lr, "clipped_steps": net.n_clipped})
    _log("summary %s" % json.dumps(summ))
    if a.out:
        with open(a.out, "w") as f:
            json.dump({"summary": summ, "cases": recs,
                       "loss_curve": [h for h in hist[:: max(1, len(hist) // 200)]]}, f, indent=1)
    net.close()
    sim.close()
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
