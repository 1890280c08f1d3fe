#!/usr/bin/env python3
"""Throughput benchmark of the superphoton transport on one MI355X.

Workload: the scattering synchrotron sphere -- a uniform sphere of radius
1e14 cm on a 32^3 Cartesian zone grid, Theta_e = 4, B = 1 G, electron density
set by the Thomson depth tau_T in {1e-3, 1e-2, 1e-1} (three instances),
thermal Klein-Nishina Compton scattering with constant bias b = 1/tau_T up to
four scattering generations, N_s = 1e6 superphotons per instance, 128 log
bins over 1e8-1e24 Hz x 6 inclination bins, all in double precision.

One step = for each instance: make superphotons (new seed), track and
scatter all of them to escape/absorption, read the spectrum.  The metric is
superphotons (roots + scattered children) per second of whole-step wall time
with the zone data already resident on the GPU.

Prints one JSON line.  ``--gpus N`` with N > 1 is refused: this build runs
on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

TAUS = (1e-3, 1e-2, 1e-1)
N_S = 1e6
FP64_PEAK_TFLOPS = 78.6

# Algorithmic FP64 operations of the tracking kernel per event (counting
# convention: + - * / sqrt and each elementary function = 1, fused
# multiply-add = 2; comparisons, min/max, floor and integer work not
# counted); the breakdown of each figure is in the comment beside it.  Only
# the tracking kernel's own work is counted: birth and scattering kernels
# are timed apart.
FLOPS_PER = {
    "step": 32,           # flat step: length 4, push 6, zone index 6, optical depths 8, updates 8
    "opacity": 64,        # one opacity evaluation at a point: frame products 17, pitch angle 5,
                          # g(X) and j 11, Kirchhoff nu alpha 9, sigma_h lookup and nu alpha_sc 22
    "split": 20,          # scattering decision that splits: fraction, sub-step, absorption, split
}
STAT_INDEX = {"ROOTS": 0, "CHILDREN": 1, "STEPS": 2, "SCATTER": 4, "NU_TRIALS": 12,
              "DIR_TRIALS": 13, "E_TRIALS": 14, "ANG_TRIALS": 15, "OPACITY_EVALS": 32}


def algorithmic_flops(st) -> float:
    """Work of the tracking launches of a step from the library's counters."""
    return (FLOPS_PER["step"] * st[STAT_INDEX["STEPS"]]
            + FLOPS_PER["opacity"] * st[STAT_INDEX["OPACITY_EVALS"]]
            + FLOPS_PER["split"] * st[STAT_INDEX["SCATTER"]])


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("gm_track.h", "gm_frame.h", "gm_physics.h", "gm_common.h", "gm_emis32.h", "gm_kerr.h",
              "gm_track_ks.h", "gm_api.hip"):
        h.update(open(os.path.join(ROOT, "paper_2602_13198_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def track_variant(waves: int, batch: int) -> str:
    """Name of the compiled FP64 flat tracker a tuning selects."""
    return "track_kernel_flat<%d, false, %s>" % (waves, "true" if batch > 1 else "false")


def measured_traffic(variant):
    """HBM bytes per tracking launch from the committed counter summary, if
    it was taken on the current kernel source and the same variant (else None)."""
    try:
        d = json.load(open(TRAFFIC_JSON))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash() or d.get("kernel") != variant:
        return None
    return d.get("bytes_per_launch")


ISSUE_JSON = os.path.join(ROOT, "profiles", "track_kernel_scattering_sphere_fp64_issue.json")


def measured_issue(variant):
    """Issued FP64 operations per tracking launch from the committed counter
    summary, if it was taken on the current kernel source and the same
    variant (else None)."""
    try:
        d = json.load(open(ISSUE_JSON))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash() or d.get("kernel") != variant:
        return None
    return d.get("issued_fp64_flop_per_launch")


def register_bound(ctx, waves, target_ms=40.0):
    """Attained FP64 FMA rate at the tracker's waves per SIMD for 1, 2, 4 and
    8 independent dependent-FMA chains per lane (library kernel, HIP events)."""
    out = {}
    for chains in (1, 2, 4, 8):
        ms, _, _ = ctx.fma_chain_bound(waves, chains, 20000)
        iters = max(20000, int(20000 * target_ms / max(ms, 1e-3)))
        ms, tf, _ = ctx.fma_chain_bound(waves, chains, iters)
        out[chains] = tf
    return out


def kerr_torus_form(ctx, instance, waves, runs=2):
    """Superphotons/s on the synthetic Kerr torus (a = 0.9375, 256 x 128 MKS
    zones, N_s = 1e7, 200 x 6 bins) in FP64 and in the FP32-emissivity form:
    the refill threshold chosen by one timed round each (Kerr photons live
    ~300 steps, so lanes are refilled earlier than in flat space), then one
    untimed round and `runs` timed make + track + read rounds per form."""
    import torch
    from paper_2602_13198_amd import workloads as W
    wl = W.torus(n_target=1e7)
    ctx.load_zones(wl, instance)
    out = {"workload": "Kerr torus a=0.9375, 256x128 modified Kerr-Schild zones, Fishbone-Moncrief "
                       "torus with 5% log-normal perturbations, R-beta electrons (R_high=40), "
                       "b = 1e3 Theta_e^2, N_s=1e7, 200x6 bins"}
    trial = {}
    for refill in (4, 8, 16):
        ctx.set_tuning(waves, refill)
        ctx.make_superphotons(dict(wl.emit, seed=6999), instance=instance)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.track_scatter(wl.track)
        torch.cuda.synchronize()
        trial[refill] = time.perf_counter() - t0
        ctx.read_spectrum(instance, reset=True)
    best = min(trial, key=trial.get)
    ctx.set_tuning(waves, best)
    out["tuning"] = {"track_waves": waves, "refill_min": best,
                     "trial_track_s": {str(k): round(v, 4) for k, v in trial.items()}}
    for prec, key in ((0, "f64"), (1, "f32_emissivity")):
        def one(seed):
            ctx.make_superphotons(dict(wl.emit, seed=seed), instance=instance)
            st = ctx.track_scatter(dict(wl.track, precision=prec))
            ctx.read_spectrum(instance, reset=True)
            return st
        one(7000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tot = None
        for r in range(runs):
            st = one(7001 + r)
            tot = st if tot is None else tot + st
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        nsp = int(tot[0] + tot[1])
        out[key] = {"value": nsp / dt, "unit": "superphotons/s", "seconds_per_round": dt / runs,
                    "superphotons_per_round": nsp / runs, "steps_per_superphoton": float(tot[2]) / max(nsp, 1),
                    "geodesic_steps_per_s": float(tot[2]) / dt}
    out["f32_speedup"] = out["f32_emissivity"]["value"] / out["f64"]["value"]
    return out


# the variant the committed profiles cover: 2 waves/SIMD, the three
# instances in shared launches (what the autotuner picks on this workload)
TRACK_KERNEL = track_variant(2, 64)
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "track_kernel_scattering_sphere_traffic.json")
TRACE_TXT = os.path.join(ROOT, "profiles", "track_kernel_scattering_sphere_kernel_trace.txt")


def _counter_rows(d):
    import csv
    import glob
    f = sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True))
    if not f:
        raise SystemExit("no counter_collection.csv under %s" % d)
    return list(csv.DictReader(open(f[0])))


def summarize_traffic(fetch_dir, write_dir, commands, copy_mib):
    """Writes the HBM traffic summary of the tracking kernel from two
    rocprofv3 --pmc runs of `bench.py --copy-mib N` (FETCH_SIZE, then
    WRITE_SIZE): KiB per launch, each scaled by what the same counter reads
    for the plain device copy of known size in the same run."""
    out = {"kernel": TRACK_KERNEL,
           "workload": "scattering synchrotron sphere, 3 x N_s=1e6 (tau_T 1e-3/1e-2/1e-1) in shared "
                       "launches, one bench step = 5 tracking launches",
           "kernel_source_hash": kernel_source_hash()}
    factors = {}
    for key, d in (("fetch", fetch_dir), ("write", write_dir)):
        rows = _counter_rows(d)
        mine = [float(r["Counter_Value"]) for r in rows if TRACK_KERNEL in r["Kernel_Name"]]
        copy = max(float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"])
        copy_bytes = copy_mib * 2**20
        # the copy reads and writes copy_bytes once each
        factors[key] = (copy_bytes / 1024.0) / copy
        out["%s_kib_per_launch_raw" % key] = sum(mine) / len(mine)
        out["launches"] = len(mine)
        out.setdefault("copy_calibration", {"bytes": copy_bytes})
        out["copy_calibration"]["%s_kib_raw" % key] = copy
        out["copy_calibration"]["%s_factor" % key] = factors[key]
    out["bytes_per_launch"] = 1024.0 * (out["fetch_kib_per_launch_raw"] * factors["fetch"]
                                        + out["write_kib_per_launch_raw"] * factors["write"])
    out["commands"] = commands
    with open(TRAFFIC_JSON, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out, indent=1))


def summarize_issue(pmc_dir, commands):
    """Writes the issued FP64 operations of the tracking kernel from one
    rocprofv3 --pmc run of the FP64 VALU instruction counters: per wave
    instruction 64 lanes for ADD, MUL and transcendental, 128 for FMA (masked
    lanes and software-function instructions included)."""
    rows = _counter_rows(pmc_dir)
    acc, n = {}, {}
    for r in rows:
        if TRACK_KERNEL not in r["Kernel_Name"]:
            continue
        k = r["Counter_Name"]
        acc[k] = acc.get(k, 0.0) + float(r["Counter_Value"])
        n[k] = n.get(k, 0) + 1
    per = {k: acc[k] / n[k] for k in acc}
    issued = 64.0 * (per["SQ_INSTS_VALU_ADD_F64"] + per["SQ_INSTS_VALU_MUL_F64"]
                     + per["SQ_INSTS_VALU_TRANS_F64"]) + 128.0 * per["SQ_INSTS_VALU_FMA_F64"]
    out = {"kernel": TRACK_KERNEL,
           "workload": "scattering synchrotron sphere, 3 x N_s=1e6 (tau_T 1e-3/1e-2/1e-1)",
           "kernel_source_hash": kernel_source_hash(),
           "launches": max(n.values()),
           "per_launch": per,
           "issued_fp64_flop_per_launch": issued,
           "convention": "64 x (ADD_F64 + MUL_F64 + TRANS_F64) + 128 x FMA_F64 per wave instruction",
           "commands": commands}
    with open(ISSUE_JSON, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out, indent=1))


def summarize_trace(trace_dir, bench_log, command):
    """Writes the kernel-trace summary: rocprofv3 --stats table, one step's
    launches, and the tracker's average launch time as bench.py measured it
    with HIP events in the same run."""
    import csv
    import glob
    stats = sorted(glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True))[0]
    trace = sorted(glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True))[0]
    line = [l for l in open(bench_log) if l.startswith("{")][-1]
    b = json.loads(line)
    rows = list(csv.DictReader(open(stats)))
    mine = [r for r in rows if TRACK_KERNEL in r["Name"]]
    lines = ["# rocprofv3 kernel trace: scattering synchrotron sphere (3 x N_s=1e6, tau_T 1e-3/1e-2/1e-1)",
             "# command: " + command,
             "# bench.py in the same run: %s superphotons/s under the profiler; avg %s launch "
             "%.3f ms over %d timed launches (HIP events); rocprofv3 average over all %s launches: %.3f ms"
             % ("%.4g" % b["value"], TRACK_KERNEL, b["roofline"]["avg_launch_ms"], b["roofline"]["launches"],
                mine[0]["Calls"] if mine else "0", float(mine[0]["AverageNs"]) * 1e-6 if mine else float("nan")),
             "# HBM traffic of the same kernel: track_kernel_scattering_sphere_traffic.json", "",
             "## kernel_stats.csv (top 16)"]
    lines.append(",".join(rows[0].keys()))
    for r in rows[:16]:
        lines.append(",".join(str(v) for v in r.values()))
    tr = list(csv.DictReader(open(trace)))
    tr.sort(key=lambda r: int(r["Start_Timestamp"]))
    lines += ["", "## the last 40 launches of the run: kernel | duration | grid (work-items)"]
    for r in tr[-40:]:
        lines.append("%s | %.3f ms | grid %s" % (
            r["Kernel_Name"][:60], (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6,
            r.get("Grid_Size_X", r.get("Grid_Size", "?"))))
    with open(TRACE_TXT, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines[:8]))


def workloads():
    from paper_2602_13198_amd import workloads as W
    return [W.scattering_sphere(t, n_target=N_S, seed=0, instance=i) for i, t in enumerate(TAUS)]


def cpu_baseline(wls, steps: int):
    """The oracle, as it stands, on `steps` whole bench steps: every root of
    the three instances with all their descendants, seeds 0, 1, ... (the
    GPU's timed steps use the same seeds)."""
    import oracle
    t_total, n_total = 0.0, 0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    o = oracle.Oracle()
    for k, wl in enumerate(wls):
        o.load_zones(wl)
        if k == 0:   # setup outside the timed region: the cross-section table
            o.make_superphotons(wl.emit)
            o.track_scatter(wl.track, 0, 0, n_threads=threads)
            o.read_spectrum(reset=True)
        for s in range(steps):
            t0 = time.perf_counter()
            o.make_superphotons(dict(wl.emit, seed=s))
            o.track_scatter(wl.track, n_threads=threads)
            r = o.read_spectrum(reset=True)
            t_total += time.perf_counter() - t0
            n_total += int(r.stats[0] + r.stats[1])
    o.close()
    return dict(value=n_total / t_total, unit="superphotons/s", cores=threads, kind="oracle",
                sample="%d whole bench steps (seeds 0-%d): every root of the 3 instances (tau_T=%s) "
                       "with all their scattered descendants; make + track; %.1f s, %d superphotons; "
                       "host cores visible: %d" % (steps, steps - 1, list(TAUS), t_total,
                                                   n_total, len(os.sched_getaffinity(0))))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=2,
                    help="whole bench steps timed on the CPU oracle")
    ap.add_argument("--track-waves", type=int, default=0,
                    help="waves/SIMD variant of the tracker (2-4); 0 = autotune")
    ap.add_argument("--refill-min", type=int, default=8)
    ap.add_argument("--batch", type=int, default=64,
                    help="instances per shared launch with --track-waves (1 = one at a time)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--ttx-seeds", type=int, default=3,
                    help="seeds of the time-to-1%% measurement (0 = skip)")
    ap.add_argument("--ttx-anchor", type=float, default=None,
                    help="quantile of the predicted importance at which the learned b equals the plain b")
    ap.add_argument("--ttx-ref-rounds", type=int, default=1024,
                    help="N_s rounds of the plain reference spectrum")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the tracker's HBM traffic summary from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("TRACE_DIR", "BENCH_LOG"),
                    help="write the kernel-trace summary from a rocprofv3 --kernel-trace --stats run and exit")
    ap.add_argument("--summarize-issue", metavar="PMC_DIR",
                    help="write the tracker's issued FP64 operations from a rocprofv3 --pmc run and exit")
    ap.add_argument("--commands", nargs="*", default=[],
                    help="the profiler command lines, recorded in the summaries")
    args = ap.parse_args()
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic, args.commands, args.copy_mib or 1024)
        return
    if args.summarize_issue:
        summarize_issue(args.summarize_issue, args.commands)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace, " && ".join(args.commands))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only (--gpus %d requested): sharding over several "
              "GPUs is not built" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2602_13198_amd import gm

    wls = workloads()
    ctx = gm.Context(0)
    for i, wl in enumerate(wls):
        ctx.load_zones(wl, i)
        ctx.set_instance_bias(i, wl.track)          # b = 1/tau_T per instance
    torch.cuda.synchronize()

    def one_step(seed, precision=0):
        # every instance makes its roots, then one track call runs them all
        # (shared launches up to the batch limit)
        for i, wl in enumerate(wls):
            ctx.make_superphotons(dict(wl.emit, seed=seed), instance=i)
        tot = ctx.track_scatter(dict(wls[0].track, precision=precision))
        for i in range(len(wls)):
            ctx.read_spectrum(i, reset=True)
        return tot

    if args.copy_mib:
        a = torch.empty(args.copy_mib * 2**20, dtype=torch.uint8, device="cuda")
        a.fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    tuning = {"track_waves": args.track_waves, "refill_min": args.refill_min,
              "batch": args.batch, "autotuned": False}
    if args.track_waves:
        ctx.set_tuning(args.track_waves, args.refill_min)
        ctx.set_batch(args.batch)
    else:
        from paper_2602_13198_amd.autotune import autotune
        (w_, r_, b_), table = autotune(ctx, one_step,
                                       log=lambda m: print(m, file=sys.stderr, flush=True))
        tuning = {"track_waves": w_, "refill_min": r_, "batch": b_, "autotuned": True,
                  "candidates": [[a, b, c, round(d, 3), round(e, 3)] for a, b, c, d, e in table]}
    for w in range(args.warmup):
        one_step(1000 + w)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    totals = None
    t0 = time.perf_counter()
    for s in range(args.steps):
        st = one_step(s)
        totals = st if totals is None else totals + st
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    track_ms, launches = ctx.read_timing()
    ctx.set_timing(False)

    # the FP32 precision form on the same workload and tuning, timed the same way
    one_step(2000, precision=1)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    t1 = time.perf_counter()
    tot32 = None
    for s in range(args.steps):
        st = one_step(s, precision=1)
        tot32 = st if tot32 is None else tot32 + st
    torch.cuda.synchronize()
    el32 = time.perf_counter() - t1
    ms32, l32 = ctx.read_timing()
    ctx.set_timing(False)

    n_sp = int(totals[0] + totals[1])
    value = n_sp / elapsed
    flops = algorithmic_flops(totals)
    achieved = flops / launches / (track_ms / launches * 1e-3) / 1e12 if launches else 0.0
    variant = track_variant(tuning["track_waves"], tuning["batch"])
    traffic = measured_traffic(variant)
    issued = measured_issue(variant)
    bound = register_bound(ctx, tuning["track_waves"])
    out = {
        "metric": "superphotons/s",
        "value": value,
        "unit": "superphotons/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "scattering synchrotron sphere: R=1e14 cm, 32^3 Cartesian zones, "
                        "Theta_e=4, B=1 G, tau_T in {1e-3,1e-2,1e-1} (b=1/tau_T, 4 scattering "
                        "generations), N_s=1e6 per tau_T, 128x6 bins, FP64",
            "instances": len(wls),
            "superphotons_per_step": n_sp / args.steps,
            "roots_per_step": int(totals[0]) / args.steps,
            "steps_per_superphoton": float(totals[2]) / max(n_sp, 1),
            "opacity_evals_per_step": float(totals[32]) / max(float(totals[2]), 1.0),
            "tuning": tuning,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": traffic,
            "kernel": variant,
            "launches": launches,
            "avg_launch_ms": track_ms / launches if launches else None,
            "algorithmic_flops_per_launch": flops / launches if launches else None,
            "kernel_time_share": track_ms * 1e-3 / elapsed,
            # issued FP64 rate (counters of the committed profile, per launch,
            # over this run's launch time), and the register-limited bound:
            # FMA chains at the tracker's waves per SIMD
            "issued_fp64_tflops": (issued / (track_ms / launches * 1e-3) / 1e12
                                   if issued and launches else None),
            "register_limited_bound": {
                "waves_per_simd": tuning["track_waves"],
                "tflops_by_chains": {str(k): v for k, v in bound.items()},
                "frac_of_1_chain": achieved / bound[1],
                "frac_of_2_chains": achieved / bound[2],
            },
        },
    }
    # time to 1 % spectral error, plain method, on the tau_T = 0.1 instance
    ttx = None
    if args.ttx_seeds > 0:
        from paper_2602_13198_amd import convergence as CV
        iw = len(wls) - 1
        wl = wls[iw]
        L_ref, cnt_ref, rse_ref, n_ref = CV.reference(ctx, wl, iw, args.ttx_ref_rounds, 100000)
        mask = CV.error_mask(cnt_ref, rse_ref)
        runs = [CV.time_to_error(ctx, wl, iw, L_ref, mask, 200000 + 1000 * k,
                                 wl.emit["n_target"]) for k in range(args.ttx_seeds)]
        secs = [r["seconds"] for r in runs if r["seconds"] is not None]
        # the learned form: records from two plain rounds (disjoint seeds), the
        # network trained on the library's matrix-core kernels, the table built
        # by its inference kernel (counted in the learned time)
        from paper_2602_13198_amd.learned import LearnedBias, collect_records
        torch.cuda.synchronize()
        tt0 = time.perf_counter()
        bin_w = np.where(mask, 1.0 / np.maximum(L_ref, 1e-300), 0.0)
        Xr, Tr = collect_records(ctx, wl, iw, 2, 300000, bin_weight=bin_w)
        lb = LearnedBias(seed=1)
        fit_hist = lb.fit(ctx, Xr, Tr, steps=600, anchor_quantile=args.ttx_anchor)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - tt0
        tt1 = time.perf_counter()
        lb.apply(ctx, wl, iw, b_plain=wl.track["bias_value"], b_max=1e3)
        t_table = time.perf_counter() - tt1
        learned_over = dict(bias_mode=3, bias_max=1e3)
        ctx.set_instance_bias(iw, None)                # the learned table decides
        runs_l = [CV.time_to_error(ctx, wl, iw, L_ref, mask, 400000 + 1000 * k, wl.emit["n_target"],
                                   track_overrides=learned_over) for k in range(args.ttx_seeds)]
        secs_l = [r["seconds"] for r in runs_l if r["seconds"] is not None]
        ctx.set_instance_bias(iw, wl.track)
        med_p = float(np.median(secs)) if len(secs) == len(runs) else None
        med_l = float(np.median(secs_l)) + t_table if len(secs_l) == len(runs_l) else None
        ttx = {
            "workload": "scattering sphere tau_T=0.1 (b=10), plain uniform bias, FP64",
            "target_eps_err": 0.01,
            "plain": {"seconds_median": med_p,
                      "seconds": [r["seconds"] for r in runs],
                      "superphotons": [r["superphotons"] for r in runs],
                      "final_eps": [r["final_eps"] for r in runs]},
            "learned": {"seconds_median": med_l,
                        "seconds": [r["seconds"] for r in runs_l],
                        "superphotons": [r["superphotons"] for r in runs_l],
                        "final_eps": [r["final_eps"] for r in runs_l],
                        "table_build_s": t_table,
                        "training_one_off_s": t_train, "training_records": int(len(Xr)),
                        "training_loss_first_last": [fit_hist[0][1], fit_hist[-1][1]],
                        "bias": "b = exp(learned ln b[zone][ln eps]), clamped to [1, 1e3]"},
            "plain_over_learned": (med_p / med_l) if (med_p and med_l) else None,
            "reference": {"rounds": args.ttx_ref_rounds, "superphotons": n_ref,
                          "masked_bins": int(mask.sum()),
                          "mask": "bins holding >= 1e3 superphotons and a relative standard "
                                  "error <= 10% per N_s=1e6 round",
                          "rounds_of": "N_s = 1e6, seeds disjoint from the reference"},
        }
    n32 = int(tot32[0] + tot32[1])
    out["forms"] = {
        "f32_emissivity": {
            "what": "emissivity, Kirchhoff absorption and hot cross section in FP32 (log space, "
                    "64-byte zone records); geodesics, weights, tallies FP64",
            "value": n32 / el32, "unit": "superphotons/s", "ms_per_step": el32 / args.steps * 1e3,
            "avg_track_launch_ms": ms32 / l32 if l32 else None,
            "speedup_vs_f64": (n32 / el32) / value,
        },
        "kerr_torus": kerr_torus_form(ctx, len(wls), tuning["track_waves"]),
    }
    if ttx is not None:
        out["time_to_1pct"] = ttx
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wls, args.cpu_steps)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
