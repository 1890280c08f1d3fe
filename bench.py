#!/usr/bin/env python3
"""Throughput and time-to-accuracy benchmark of the superphoton transport on
one MI355X.

Headline workload: the Kerr accretion torus under a scattering corona -- a
Fishbone-Moncrief torus (a = 0.9375, R-beta electrons with R_high = 40,
5 % log-normal perturbations in 3-D) on a 192 x 96 x 96 modified
Kerr-Schild grid, with every empty zone between the horizon and 40 r_g
filled by a hot (Theta_e = 1), field-free electron corona whose radial
Thomson depth is 0.1; thermal Klein-Nishina Compton scattering with the
plain constant bias b = 10 up to four generations; N_s = 1e8 per round,
200 log bins over 1e8-1e24 Hz x 6 inclination bins; FP64.

One step = make superphotons (new seed), track and scatter all of them to
escape/capture/absorption, read the spectrum.  value = superphotons (roots
+ scattered children) per second of whole-step wall time, zones resident on
the GPU.  Also measured: the tracking kernel's algorithmic FP64 rate
against the vector peak (HIP events on the library's stream), the time to
1 % spectral error of the plain and the learned and adaptive forms on the
same workload, the FP32 form, the flat scattering sphere and the 64-torus
survey, and the CPU oracle on a sample of the headline workload.

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

FP64_PEAK_TFLOPS = 78.6
N_S = 1e8

# Algorithmic FP64 operations of the Kerr tracking kernel per event
# (convention: + - * / sqrt and each elementary function = 1, fused
# multiply-add = 2; comparisons, min/max, floor, integer and random-number
# work not counted; common subexpressions counted once).  Tracker
# iterations are of three kinds -- a step, a sub-step to a scattering point,
# the first evaluation of a photon taken from the queue -- and each
# corrector pass of the integrator adds its own work.
KS_FLOPS_PER = {
    "point": 363,     # step or sub-step: step size 11, predictor 14, metric + x1/x2 derivatives
                      # (dual numbers) 104, corrector start 8, e_inf 5, zone index 9, opacities 192
                      # (fluid-frame normalisation 95, -k.u 27, pitch angle and j 43, Kirchhoff 7,
                      # sigma_h lookup and nu alpha_sc 20), optical depths and weights 20
    "corrector": 104, # one corrector pass: acceleration 74, wavevector update 16, convergence test 14
    "split": 84,      # sub-step extra: fresh acceleration 74, weight split and new depth 10
    "load": 384,      # photon taken from the queue: metric 104, acceleration 74, e_inf 5, zone 9,
                      # opacities 192
}
# Flat (Cartesian) tracker, for the secondary workload.
FLAT_FLOPS_PER = {
    "step": 32,       # length 4, push 6, zone index 6, optical depths 8, updates 8
    "opacity": 64,    # frame products 17, pitch angle 5, g(X) and j 11, Kirchhoff 9, sigma_h 22
    "split": 20,      # fraction, sub-step, absorption, split
}
S = {"ROOTS": 0, "CHILDREN": 1, "STEPS": 2, "VERLET_IT": 3, "SCATTER": 4, "OPACITY_EVALS": 32}


def ks_flops(st) -> float:
    """Work of the Kerr tracking launches from the library's counters."""
    steps, sub, vit = float(st[S["STEPS"]]), float(st[S["SCATTER"]]), float(st[S["VERLET_IT"]])
    loads = float(st[S["ROOTS"]] + st[S["CHILDREN"]])
    return (KS_FLOPS_PER["point"] * (steps + sub) + KS_FLOPS_PER["corrector"] * vit
            + KS_FLOPS_PER["split"] * sub + KS_FLOPS_PER["load"] * loads)


def flat_flops(st) -> float:
    return (FLAT_FLOPS_PER["step"] * st[S["STEPS"]] + FLAT_FLOPS_PER["opacity"] * st[S["OPACITY_EVALS"]]
            + FLAT_FLOPS_PER["split"] * st[S["SCATTER"]])


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("gm_track.h", "gm_frame.h", "gm_physics.h", "gm_common.h", "gm_emis32.h", "gm_kerr.h",
              "gm_track_ks.h", "gm_api.hip"):
        h.update(open(os.path.join(ROOT, "paper_2602_13198_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def track_variant(waves: int, batch: int, kerr: bool = True, const_bias: bool = True) -> str:
    """Name of the compiled FP64 tracker a tuning selects (the Kerr tracker
    has a form for launches whose instances all have the constant bias)."""
    b = "true" if batch > 1 else "false"
    if kerr:
        return "track_kernel_ks<%d, false, %s, %s>" % (waves, b, "true" if const_bias else "false")
    return "track_kernel_flat<%d, false, %s>" % (waves, b)


# the variant the committed profiles cover: the Kerr tracker at 2 waves/SIMD,
# one instance per launch (the headline workload)
TRACK_KERNEL = track_variant(2, 1)
PROFILE = os.path.join(ROOT, "profiles", "track_kernel_ks_corona_torus")
TRAFFIC_JSON = PROFILE + "_traffic.json"
ISSUE_JSON = PROFILE + "_fp64_issue.json"
TRACE_TXT = PROFILE + "_kernel_trace.txt"
WORKLOAD_TEXT = ("Kerr torus under a scattering corona: a=0.9375, 192x96x96 modified Kerr-Schild zones, "
                 "Fishbone-Moncrief torus (5% log-normal 3-D perturbations, R-beta electrons R_high=40), "
                 "corona n_e ~ 1/r with radial tau_T=0.1, Theta_e=1, B=0 out to 40 r_g; thermal Compton, "
                 "constant bias b=10, 4 generations; N_s=1e8; 200x6 bins; FP64")


FLAT_WORKLOAD_TEXT = ("flat scattering synchrotron sphere: R=1e14 cm, 32^3 Cartesian zones, Theta_e=4, "
                      "B=1 G, tau_T in {1e-3,1e-2,1e-1} (b=1/tau_T), N_s=1e6 each, 128x6 bins, "
                      "three instances in shared launches, FP64")

# kernels whose profiler summaries are kept: the headline's tracker, and the
# flat tracker of the secondary flat sphere field (form: its bench field)
SUMMARY_TARGETS = {
    "corona_torus": dict(kernel=TRACK_KERNEL, prefix=PROFILE, workload=WORKLOAD_TEXT, form=None),
    "scattering_sphere": dict(kernel=track_variant(2, 64, kerr=False),
                              prefix=os.path.join(ROOT, "profiles", "track_kernel_flat_scattering_sphere"),
                              workload=FLAT_WORKLOAD_TEXT, form="flat_scattering_sphere"),
}


def _target_file(target, suffix):
    """Summary file of a target: the headline's module-level names, else
    the target's prefix with the suffix."""
    if target["form"] is None:
        return {"_traffic.json": TRAFFIC_JSON, "_fp64_issue.json": ISSUE_JSON, "_kernel_trace.txt": TRACE_TXT}[suffix]
    return target["prefix"] + suffix


def _summary(path):
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    return d


def measured_traffic(variant):
    """HBM bytes per tracking launch from the committed counter summary, if
    it was taken on the current kernel source and the same variant (else None)."""
    d = _summary(TRAFFIC_JSON)
    if not d or d.get("kernel_source_hash") != kernel_source_hash() or d.get("kernel") != variant:
        return None
    return d.get("bytes_per_launch")


def measured_issue(variant):
    """Issued FP64 operations per tracking launch from the committed counter
    summary, if it was taken on the current kernel source and the same
    variant (else None)."""
    d = _summary(ISSUE_JSON)
    if not d or d.get("kernel_source_hash") != kernel_source_hash() or d.get("kernel") != variant:
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


def _db(d):
    import glob
    f = sorted(glob.glob(os.path.join(d, "**", "*results.db"), recursive=True))
    return f[0] if f else None


def _counter_rows(d):
    """Counter rows (Kernel_Name, Counter_Name, Counter_Value) of a rocprofv3
    --pmc run: its counter_collection.csv, or the counters view of its
    database output."""
    import csv
    import glob
    f = sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True))
    if f:
        return list(csv.DictReader(open(f[0])))
    db = _db(d)
    if not db:
        raise SystemExit("no counter output under %s" % d)
    import sqlite3
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, counter_name, value from counters_collection").fetchall()
    return [{"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v} for k, c, v in rows]


def _trace_rows(d):
    """(per-kernel stats rows, per-launch rows) of a rocprofv3 --kernel-trace
    --stats run, from its CSV files or its database output."""
    import csv
    import glob
    st = sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True))
    tr = sorted(glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True))
    if st and tr:
        return list(csv.DictReader(open(st[0]))), list(csv.DictReader(open(tr[0])))
    import sqlite3
    con = sqlite3.connect(_db(d))
    # the summary view reports microseconds, the per-launch view nanoseconds
    stats = [{"Name": n, "Calls": c, "TotalDurationNs": 1e3 * t, "AverageNs": 1e3 * a, "Percentage": p}
             for n, c, t, a, p in con.execute(
                 "select name, total_calls, total_duration, average, percentage from top_kernels "
                 "order by total_duration desc").fetchall()]
    launches = [{"Kernel_Name": n, "Start_Timestamp": s_, "End_Timestamp": e, "Grid_Size_X": g}
                for n, s_, e, g in con.execute("select name, start, end, grid_x from kernels").fetchall()]
    return stats, launches


def summarize_traffic(fetch_dir, write_dir, commands, copy_mib, target=SUMMARY_TARGETS["corona_torus"]):
    """Writes the HBM traffic summary of a tracking kernel from two
    rocprofv3 --pmc runs of `bench.py --copy-mib N` (FETCH_SIZE, then
    WRITE_SIZE): KiB per launch, each scaled by what the same counter reads
    for the plain device copy of known size in the same run."""
    kernel = target["kernel"]
    out = {"kernel": kernel, "workload": target["workload"], "kernel_source_hash": kernel_source_hash()}
    factors = {}
    for key, d in (("fetch", fetch_dir), ("write", write_dir)):
        rows = _counter_rows(d)
        mine = [float(r["Counter_Value"]) for r in rows if kernel in r["Kernel_Name"]]
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
    with open(_target_file(target, "_traffic.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out, indent=1))


def summarize_issue(pmc_dir, commands, target=SUMMARY_TARGETS["corona_torus"]):
    """Writes the issued FP64 operations of the tracking kernel from one
    rocprofv3 --pmc run of the FP64 VALU instruction counters: per wave
    instruction 64 lanes for ADD, MUL and transcendental, 128 for FMA (masked
    lanes and software-function instructions included)."""
    rows = _counter_rows(pmc_dir)
    acc, n = {}, {}
    for r in rows:
        if target["kernel"] not in r["Kernel_Name"]:
            continue
        k = r["Counter_Name"]
        acc[k] = acc.get(k, 0.0) + float(r["Counter_Value"])
        n[k] = n.get(k, 0) + 1
    per = {k: acc[k] / n[k] for k in acc}
    issued = 64.0 * (per["SQ_INSTS_VALU_ADD_F64"] + per["SQ_INSTS_VALU_MUL_F64"]
                     + per["SQ_INSTS_VALU_TRANS_F64"]) + 128.0 * per["SQ_INSTS_VALU_FMA_F64"]
    out = {"kernel": target["kernel"], "workload": target["workload"], "kernel_source_hash": kernel_source_hash(),
           "launches": max(n.values()), "per_launch": per, "issued_fp64_flop_per_launch": issued,
           "convention": "64 x (ADD_F64 + MUL_F64 + TRANS_F64) + 128 x FMA_F64 per wave instruction",
           "commands": commands}
    with open(_target_file(target, "_fp64_issue.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out, indent=1))


def summarize_trace(trace_dir, bench_log, command, target=SUMMARY_TARGETS["corona_torus"]):
    """Writes the kernel-trace summary: rocprofv3 --stats table, the last
    launches, and the tracker's average launch time as bench.py measured it
    with HIP events in the same run."""
    rows, tr = _trace_rows(trace_dir)
    line = [l for l in open(bench_log) if l.startswith("{")][-1]
    b = json.loads(line)
    kernel = target["kernel"]
    mine = [r for r in rows if kernel in r["Name"]]
    if target["form"] is None:
        value, avg, nl = b["value"], b["roofline"]["avg_launch_ms"], b["roofline"]["launches"]
    else:
        f = b["forms"][target["form"]]
        value, avg, nl = f["value"], f["tracker_avg_launch_ms"], f["tracker_launches"]
    lines = ["# rocprofv3 kernel trace: " + target["workload"],
             "# command: " + command,
             "# bench.py in the same run: %s superphotons/s under the profiler; avg %s launch "
             "%.3f ms over %d timed launches (HIP events); rocprofv3 average over all %s launches: %.3f ms"
             % ("%.4g" % value, kernel, avg, nl,
                mine[0]["Calls"] if mine else "0", float(mine[0]["AverageNs"]) * 1e-6 if mine else float("nan")),
             "# HBM traffic of the same kernel: %s" % os.path.basename(_target_file(target, "_traffic.json")), "",
             "## kernel_stats.csv (top 16)"]
    lines.append(",".join(rows[0].keys()))
    for r in rows[:16]:
        lines.append(",".join(str(v) for v in r.values()))
    tr.sort(key=lambda r: int(r["Start_Timestamp"]))
    lines += ["", "## the last 40 launches of the run: kernel | duration | grid (work-items)"]
    for r in tr[-40:]:
        lines.append("%s | %.3f ms | grid %s" % (
            r["Kernel_Name"][:60], (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6,
            r.get("Grid_Size_X", r.get("Grid_Size", "?"))))
    with open(_target_file(target, "_kernel_trace.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines[:8]))


def headline_workload():
    from paper_2602_13198_amd import workloads as W
    return W.corona_torus(n_target=N_S, seed=0)


def timed_steps(ctx, wl, inst, steps, seed0, precision=0):
    """`steps` make + track + read rounds; returns (wall s, summed counters,
    tracking-kernel event ms, launches)."""
    import torch
    torch.cuda.synchronize()
    ctx.set_timing(True)
    tot = None
    t0 = time.perf_counter()
    for s in range(steps):
        ctx.make_superphotons(dict(wl.emit, seed=seed0 + s), instance=inst)
        st = ctx.track_scatter(dict(wl.track, precision=precision))
        ctx.read_spectrum(inst, reset=True)
        tot = st if tot is None else tot + st
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms, launches = ctx.read_timing()
    ctx.set_timing(False)
    return dt, tot, ms, launches


def graph_form(ctx, wl, inst, rounds=12, div=32, log=lambda m: None):
    """Whole-step time with each root chunk launched directly and as a
    captured HIP graph, on the headline workload at N_s / div per round (the
    rounds of the time-to-1 % measurement, where launches are shortest) and
    at full N_s."""
    import torch
    out = {}
    for name, n_s, reps in (("round_n_s_over_%d" % div, wl.emit["n_target"] / div, rounds),
                            ("full_n_s", wl.emit["n_target"], 2)):
        res = {}
        for mode in (0, 1, 0, 1):           # alternated, the second of each kept
            ctx.set_graph(mode)
            emit = dict(wl.emit, n_target=n_s)
            ctx.make_superphotons(dict(emit, seed=8000), instance=inst)
            ctx.track_scatter(wl.track)
            ctx.read_spectrum(inst, reset=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for r in range(reps):
                ctx.make_superphotons(dict(emit, seed=8001 + r), instance=inst)
                ctx.track_scatter(wl.track)
                ctx.read_spectrum(inst, reset=True)
            torch.cuda.synchronize()
            res["graph" if mode else "direct"] = (time.perf_counter() - t0) / reps * 1e3
            log("graph form: %s %s %.2f ms per step" % (name, "graph" if mode else "direct",
                                                        res["graph" if mode else "direct"]))
        out[name] = {"ms_per_step_direct": res["direct"], "ms_per_step_graph": res["graph"],
                     "graph_speedup": res["direct"] / res["graph"]}
    ctx.set_graph(0)
    return out


def flat_sphere_form(ctx, base_inst, steps=5):
    """The flat scattering synchrotron sphere (32^3 Cartesian zones, Theta_e
    = 4, tau_T in {1e-3, 1e-2, 1e-1} with b = 1/tau_T, N_s = 1e6 each, three
    instances in shared launches, FP64)."""
    import torch
    from paper_2602_13198_amd import workloads as W
    wls = [W.scattering_sphere(t, n_target=1e6, seed=0, instance=base_inst + i)
           for i, t in enumerate((1e-3, 1e-2, 1e-1))]
    for i, wl in enumerate(wls):
        ctx.load_zones(wl, base_inst + i)
        ctx.set_instance_bias(base_inst + i, wl.track)
    ctx.set_tuning(2, 16)

    def step(seed):
        for i, wl in enumerate(wls):
            ctx.make_superphotons(dict(wl.emit, seed=seed), instance=base_inst + i)
        st = ctx.track_scatter(wls[0].track)
        for i in range(len(wls)):
            ctx.read_spectrum(base_inst + i, reset=True)
        return st
    step(9000)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    t0 = time.perf_counter()
    tot = None
    for s in range(steps):
        st = step(9001 + s)
        tot = st if tot is None else tot + st
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms, launches = ctx.read_timing()
    ctx.set_timing(False)
    for i in range(len(wls)):
        ctx.unload(base_inst + i)
    n = int(tot[0] + tot[1])
    fl = flat_flops(tot)
    return {"workload": FLAT_WORKLOAD_TEXT, "tracker_launches": launches,
            "value": n / dt, "unit": "superphotons/s", "ms_per_step": dt / steps * 1e3,
            "tracker": track_variant(2, 64, kerr=False),
            "tracker_avg_launch_ms": ms / launches if launches else None,
            "tracker_algorithmic_tflops": fl / (ms * 1e-3) / 1e12 if ms else None}


def paper_sphere_form(ctx, inst, steps=2, n_s=1e7):
    """The paper's optically thin sphere on its own grid: flat spacetime in
    (t, ln r, theta, phi), 8192 x 128 x 1 zones out to 1e4 cm, R = 1 cm,
    Theta_e = 100, n_e = 1e13, B = 1 G, record at 3000 cm, 2500 bins of 0.01
    in ln nu (tallies in HBM), FP64."""
    import torch
    from paper_2602_13198_amd import workloads as W
    wl = W.paper_thin_sphere(n_target=n_s, seed=0)
    wl.emit["instance"] = inst
    ctx.load_zones(wl, inst)
    ctx.set_instance_bias(inst, wl.track)

    def step(seed, track):
        ctx.make_superphotons(dict(wl.emit, seed=seed), instance=inst)
        st = ctx.track_scatter(track)
        ctx.read_spectrum(inst, reset=True)
        return st

    def timed(track):
        step(9500, track)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tot = None
        for s in range(steps):
            st = step(9501 + s, track)
            tot = st if tot is None else tot + st
        torch.cuda.synchronize()
        return time.perf_counter() - t0, tot
    dt, tot = timed(wl.track)
    # the far-field step rule (x4 beyond the sphere), same seeds
    dtf, totf = timed(wl.with_far_steps(4.0).track)
    ctx.unload(inst)
    n = int(tot[0] + tot[1])
    return {"workload": "the paper's optically thin synchrotron sphere on its log-r grid: R=1 cm, Theta_e=100, "
                        "n_e=1e13, B=1 G, 8192x128x1 (t, ln r, theta, phi) zones to 1e4 cm, record at 3000 cm, "
                        "2500 bins of 0.01 in ln nu, N_s=%g, FP64" % n_s,
            "value": n / dt, "unit": "superphotons/s", "ms_per_step": dt / steps * 1e3,
            "geodesic_steps_per_superphoton": float(tot[2]) / max(n, 1),
            "far_steps_x4": {"value": int(totf[0] + totf[1]) / dtf, "unit": "superphotons/s",
                             "geodesic_steps_per_superphoton": float(totf[2]) / max(int(totf[0] + totf[1]), 1)}}


def power_law_form(ctx, inst, steps=3, n_s=1e6):
    """Compton scattering off power-law electrons: the flat sphere (32^3
    Cartesian zones, R = 1e14 cm, B = 1 G) filled with an isotropic power
    law of index 3 on [10, 1e3], tau_T = 0.05 with b = 1/tau_T, four
    generations, emission 1e9-1e12 Hz, FP64."""
    import torch
    from paper_2602_13198_amd import workloads as W
    wl = W.power_law_sphere(n_target=n_s, seed=0, tau_T=0.05, gamma_max=1e3, nu_min=1e9, nu_max=1e12)
    wl.emit["instance"] = inst
    ctx.load_zones(wl, inst)
    ctx.set_instance_bias(inst, wl.track)

    def step(seed):
        ctx.make_superphotons(dict(wl.emit, seed=seed), instance=inst)
        st = ctx.track_scatter(wl.track)
        ctx.read_spectrum(inst, reset=True)
        return st
    step(9600)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot = None
    for s in range(steps):
        st = step(9601 + s)
        tot = st if tot is None else tot + st
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.unload(inst)
    n = int(tot[0] + tot[1])
    return {"workload": "power-law electrons (p=3 on gamma 10..1e3) in the 32^3 flat sphere, R=1e14 cm, B=1 G, "
                        "tau_T=0.05, b=20, 4 generations, N_s=%g, FP64" % n_s,
            "value": n / dt, "unit": "superphotons/s", "ms_per_step": dt / steps * 1e3,
            "children_per_root": float(tot[1]) / max(float(tot[0]), 1.0)}


def survey_form(ctx, steps=2, n_inst=64, log=lambda m: None):
    """The batched survey: 64 tori (spins -0.5 .. 0.9375, R_high 1 .. 160,
    M_unit log-uniform over two decades, N_s log-uniform on [1e5, 1e7])
    on 192x96x96 grids, FP32 emissivity, tracked in shared launches with
    the tallies in HBM."""
    import torch
    from paper_2602_13198_amd import workloads as W
    t0 = time.perf_counter()
    wls = W.survey()[:n_inst]
    for i, wl in enumerate(wls):
        ctx.load_zones_device(wl.grid, wl.n_e, wl.theta_e, wl.B, wl.ucon, wl.bcon, instance=i)
        ctx.set_instance_bias(i, dict(wl.track))
    torch.cuda.synchronize()
    t_load = time.perf_counter() - t0
    log("survey: %d instances loaded in %.2f s" % (len(wls), t_load))
    ctx.set_batch(64)
    track = dict(wls[0].track, precision=1)

    def step(seed):
        for i, wl in enumerate(wls):
            ctx.make_superphotons(dict(wl.emit, seed=seed + i), instance=i)
        st = ctx.track_scatter(track)
        for i in range(len(wls)):
            ctx.read_spectrum(i, reset=True)
        return st
    tw = time.perf_counter()
    st = step(7000)
    torch.cuda.synchronize()
    log("survey: warm-up step %.2f s, %d superphotons" % (time.perf_counter() - tw, int(st[0] + st[1])))
    t1 = time.perf_counter()
    tot = None
    for s in range(steps):
        st = step(7100 + 100 * s)
        tot = st if tot is None else tot + st
        torch.cuda.synchronize()
        log("survey: step %d done at %.2f s" % (s, time.perf_counter() - t1))
    dt = time.perf_counter() - t1
    for i in range(len(wls)):
        ctx.unload(i)
    n = int(tot[0] + tot[1])
    return {"workload": "survey of %d Kerr tori, 192x96x96 zones each, N_s log-uniform on [1e5,1e7] "
                        "(sum %.3g), FP32 emissivity / FP64 geodesics, shared launches, HBM tallies"
                        % (len(wls), sum(w.emit["n_target"] for w in wls)),
            "value": n / dt, "unit": "superphotons/s", "seconds_per_step": dt / steps,
            "superphotons_per_step": n / steps, "load_s": t_load}


def cpu_baseline(wl, n_roots=2000, target_s=20.0):
    """The oracle, as it stands, on a bounded sample of the headline
    workload: its emission tables for all zones (the whole make, prorated
    per root), then consecutive roots with all their descendants."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    o = oracle.Oracle()
    o.load_zones(wl)
    t0 = time.perf_counter()
    n_all = o.make_superphotons(dict(wl.emit, seed=0))
    t_make = time.perf_counter() - t0
    print("cpu baseline: oracle make %.1f s" % t_make, file=sys.stderr, flush=True)
    # the cross-section table: built once per process, outside the timing
    o.track_scatter(wl.track, 0, 0, n_threads=threads)
    o.read_spectrum(reset=True)
    t_track, n_sp, n_r, start = 0.0, 0, 0, 1000
    while t_track < target_s and n_r < 50 * n_roots:
        t1 = time.perf_counter()
        o.track_scatter(wl.track, start, start + n_roots, n_threads=threads)
        r = o.read_spectrum(reset=True)
        t_track += time.perf_counter() - t1
        n_sp += int(r.stats[0] + r.stats[1])
        n_r += n_roots
        start += n_roots
        print("cpu baseline: %d roots tracked, %.1f s" % (n_r, t_track), file=sys.stderr, flush=True)
    o.close()
    t_prorated = t_track + t_make * n_r / n_all
    return dict(value=n_sp / t_prorated, unit="superphotons/s", cores=threads, kind="oracle",
                sample="headline workload, seed 0: the oracle's make for all %d roots (%.1f s, prorated per "
                       "root) and %d consecutive roots with all their scattered descendants (%d superphotons, "
                       "%.1f s of tracking); host cores visible: %d"
                       % (n_all, t_make, n_r, n_sp, t_track, len(os.sched_getaffinity(0))))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-forms", action="store_true", help="skip the secondary workloads")
    ap.add_argument("--track-waves", type=int, default=2, help="waves/SIMD variant of the tracker (2-4)")
    ap.add_argument("--refill-min", type=int, default=0, help="idle lanes before a refill; 0 = timed trial")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--survey-inst", type=int, default=64, help="tori of the survey form (at most 64)")
    ap.add_argument("--ttx-seeds", type=int, default=3, help="seeds of the time-to-1%% measurement (0 = skip)")
    ap.add_argument("--ttx-ref-rounds", type=int, default=24, help="N_s rounds of the plain reference")
    ap.add_argument("--ttx-round-div", type=int, default=32, help="measured rounds are N_s / this")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the tracker's HBM traffic summary from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("TRACE_DIR", "BENCH_LOG"),
                    help="write the kernel-trace summary from a rocprofv3 --kernel-trace --stats run and exit")
    ap.add_argument("--summarize-issue", metavar="PMC_DIR",
                    help="write the tracker's issued FP64 operations from a rocprofv3 --pmc run and exit")
    ap.add_argument("--commands", nargs="*", default=[], help="the profiler command lines, recorded in the summaries")
    ap.add_argument("--summary-target", default="corona_torus", choices=sorted(SUMMARY_TARGETS),
                    help="the kernel a --summarize-* call writes the summary of")
    args = ap.parse_args()
    target = SUMMARY_TARGETS[args.summary_target]
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic, args.commands, args.copy_mib or 1024, target)
        return
    if args.summarize_issue:
        summarize_issue(args.summarize_issue, args.commands, target)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace, " && ".join(args.commands), target)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only (--gpus %d requested): sharding over several "
              "GPUs is not built" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2602_13198_amd import gm

    def log(m):
        print(m, file=sys.stderr, flush=True)

    wl = headline_workload()
    ctx = gm.Context(0)
    t0 = time.perf_counter()
    ctx.load_zones(wl, 0)
    torch.cuda.synchronize()
    t_load = time.perf_counter() - t0
    log("zones loaded in %.2f s" % t_load)

    if args.copy_mib:
        a = torch.empty(args.copy_mib * 2**20, dtype=torch.uint8, device="cuda")
        a.fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    waves = args.track_waves
    tuning = {"track_waves": waves}
    if args.refill_min:
        refill = args.refill_min
    else:
        trial = {}
        for r in (4, 8, 16):
            ctx.set_tuning(waves, r)
            dt, _, _, _ = timed_steps(ctx, wl, 0, 1, 6900 + r)
            trial[r] = dt
            log("refill %d: %.3f s" % (r, dt))
        refill = min(trial, key=trial.get)
        tuning["trial_step_s"] = {str(k): round(v, 4) for k, v in trial.items()}
    tuning["refill_min"] = refill
    ctx.set_tuning(waves, refill)

    for w in range(args.warmup):
        timed_steps(ctx, wl, 0, 1, 1000 + w)
    elapsed, totals, track_ms, launches = timed_steps(ctx, wl, 0, args.steps, 0)
    log("headline: %d steps in %.3f s" % (args.steps, elapsed))
    n_sp = int(totals[0] + totals[1])
    value = n_sp / elapsed
    flops = ks_flops(totals)
    achieved = flops / (track_ms * 1e-3) / 1e12 if track_ms else 0.0
    variant = track_variant(waves, 1)
    traffic = measured_traffic(variant)
    issued = measured_issue(variant)
    bound = register_bound(ctx, waves)
    evals = float(totals[S["OPACITY_EVALS"]])
    iters = float(totals[S["STEPS"]] + totals[S["SCATTER"]] + totals[S["ROOTS"]] + totals[S["CHILDREN"]])

    # the FP32 precision form, same workload and tuning
    el32, tot32, ms32, l32 = timed_steps(ctx, wl, 0, args.steps, 100, precision=1)
    # the far-field step rule (off in the headline), same workload and seeds
    wlf = wl.with_far_steps(4.0)
    elf, totf, msf, lf = timed_steps(ctx, wlf, 0, args.steps, 100)

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
            "workload": WORKLOAD_TEXT,
            "zones": wl.n_zones,
            "superphotons_per_step": n_sp / args.steps,
            "roots_per_step": int(totals[0]) / args.steps,
            "children_per_step": int(totals[1]) / args.steps,
            "geodesic_steps_per_superphoton": float(totals[S["STEPS"]]) / max(n_sp, 1),
            "corrector_passes_per_step": float(totals[S["VERLET_IT"]]) / max(float(totals[S["STEPS"]] + totals[S["SCATTER"]]), 1.0),
            "load_s": t_load,
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
            "flops_per_event": KS_FLOPS_PER,
            "tracker_iterations_check": [evals, iters],
            "kernel_time_share": track_ms * 1e-3 / elapsed,
            "issued_fp64_tflops": (issued / (track_ms / launches * 1e-3) / 1e12 if issued and launches else None),
            "register_limited_bound": {
                "waves_per_simd": waves,
                "tflops_by_chains": {str(k): v for k, v in bound.items()},
                "frac_of_1_chain": achieved / bound[1],
                "frac_of_2_chains": achieved / bound[2],
            },
        },
        "forms": {
            "f32_emissivity": {
                "what": "emissivity, Kirchhoff absorption and hot cross section in FP32 (log space, 64-byte "
                        "zone records); geodesics, weights, tallies FP64; same workload and tuning",
                "value": int(tot32[0] + tot32[1]) / el32, "unit": "superphotons/s",
                "ms_per_step": el32 / args.steps * 1e3,
                "avg_track_launch_ms": ms32 / l32 if l32 else None,
                "speedup_vs_f64": (int(tot32[0] + tot32[1]) / el32) / value,
            },
            "far_steps": {
                "what": "outgoing photons beyond the plasma (r > %.1f r_g) step 4x further; FP64, same workload "
                        "and tuning; the histories' draws, kinds and weights are those of the default rule"
                        % wlf.track["r_far"],
                "value": int(totf[0] + totf[1]) / elf, "unit": "superphotons/s",
                "ms_per_step": elf / args.steps * 1e3,
                "avg_track_launch_ms": msf / lf if lf else None,
                "geodesic_steps_per_superphoton": float(totf[S["STEPS"]]) / float(totf[0] + totf[1]),
                "speedup_vs_default": (int(totf[0] + totf[1]) / elf) / value,
            },
        },
    }
    print(json.dumps({"partial": True, "value": value, "roofline_frac": achieved / FP64_PEAK_TFLOPS}),
          file=sys.stderr, flush=True)

    if args.ttx_seeds > 0:
        from paper_2602_13198_amd import importance as IM
        out["time_to_1pct"] = IM.compare_forms(ctx, wl, 0, seeds=args.ttx_seeds, ref_rounds=args.ttx_ref_rounds,
                                               round_div=args.ttx_round_div, log=log)
        print(json.dumps({"partial": True, "time_to_1pct": out["time_to_1pct"]}), file=sys.stderr, flush=True)
    if not args.no_forms:
        out["forms"]["hip_graph"] = graph_form(ctx, wl, 0, log=log)
        log("graph form done")
        out["forms"]["flat_scattering_sphere"] = flat_sphere_form(ctx, 1)
        log("flat sphere: %.4g superphotons/s" % out["forms"]["flat_scattering_sphere"]["value"])
        out["forms"]["paper_thin_sphere"] = paper_sphere_form(ctx, 4)
        log("paper thin sphere: %.4g superphotons/s" % out["forms"]["paper_thin_sphere"]["value"])
        out["forms"]["power_law_sphere"] = power_law_form(ctx, 5)
        log("power-law sphere: %.4g superphotons/s" % out["forms"]["power_law_sphere"]["value"])
        ctx.unload(0)
        out["forms"]["survey"] = survey_form(ctx, n_inst=args.survey_inst, log=log)
        log("survey: %.4g superphotons/s" % out["forms"]["survey"]["value"])
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
