#!/usr/bin/env python3
"""Throughput of the messenger-field mapmaking iteration on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large2048] [--forms mixed,fp64]

A step is one messenger iteration (eqn. mcompact of the paper: P m, forward transforms, noise
filter, inverse transforms, binning P^T and the per-pixel 3x3 update) over the whole
time-ordered data set of the workload, already resident in HBM.  The default workload is the
largest single-GPU share: 1024 detectors x 2^22 samples (4.3e9), a 2048x2048 I/Q/U map, FP32
TOD and a uint16 angle-table index, generated on the GPU.  Both forms run, one plan at a time:
the FP32-mixed form gives `value`, the plain FP64 form (the stored TOD promoted) is reported
beside it.  One JSON line is printed; it carries the roofline of the mixed form's dominant pass
(algorithmic bytes per launch over the pass's mean duration from HIP events on the launch
stream), the time to chi^2 targets of the cooled messenger in both forms and of preconditioned
CG, and the CPU oracle timed on a bounded sample on the host (one thread, and all cores).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, GB/s
PASS_NAMES = ["A: residual+column FFT", "B: row FFT+filter+chi2+inverse rows",
              "C: inverse column FFT", "D: binning+3x3 update", "P: map projection"]
KERNEL_SOURCES = ["paper_1705_01893_amd/csrc/kernels.hip", "paper_1705_01893_amd/csrc/fft.h",
                  "paper_1705_01893_amd/csrc/common.h"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def layout_summary(mm, plan) -> list:
    """Distinct transform layouts of the plan's chunks (split, column block, tuner's pick) with counts."""
    seen = {}
    for c in range(plan.nchunk):
        lay = mm.mm_plan_chunk_layout(plan, c)
        key = (lay["M1"], lay["M2"], lay["cb"], lay["pick"], lay["ncand"])
        seen[key] = seen.get(key, 0) + 1
    rows = sorted(seen.items(), key=lambda kv: -kv[1])
    out = [{"M1": k[0], "M2": k[1], "cb": k[2], "pick": k[3], "ncand": k[4], "chunks": n} for k, n in rows[:8]]
    if len(rows) > 8:
        out.append({"other_layouts": len(rows) - 8, "chunks": sum(n for _, n in rows[8:])})
    return out


def load_traffic(workload: str, khash: str):
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_hash") != khash:
        return None
    return t


PASS_KERNELS = ["k_pass_a<", "k_pass_b<", "k_pass_c<", "k_bin<", "k_project<"]


def _is_plan_bin(name: str) -> bool:
    """The plan's precompute binning kernels (k_bin with 2 or 7 accumulated values)."""
    return re.search(r"k_bin<[^,<>]+, (2|7)[,>]", name) is not None


def _counter_rows(run_dir: str):
    import csv
    import glob
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {run_dir}")
    with open(files[0]) as fh:
        return list(csv.DictReader(fh))


def write_traffic(args, form: str, fetch_dir: str, write_dir: str) -> None:
    """HBM bytes per launch of each pass from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (KiB per dispatch).

    Only the workload's dispatches count: those after the plan's precompute binning launch (the
    transform-layout tuner's timing launches come before it) and outside the time-to-chi^2 part
    (not run with --no-chi2).  Counters are scaled by what they read for the plain 1 GiB copy of
    --copy-calibration (the runtime's copy kernel behind torch's 1 GiB device copy)."""
    per = {}
    scale = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _counter_rows(d) if r["Counter_Name"] == counter]
        start = max(int(r["Dispatch_Id"]) for r in rows
                    if _is_plan_bin(r["Kernel_Name"]))
        vals = {}
        for r in rows:
            if int(r["Dispatch_Id"]) <= start:
                continue
            key = (r["Kernel_Name"], r["Dispatch_Id"])
            vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
        # the runtime's copy kernel of torch's 1 GiB device copies (the most common reading among
        # them: other, smaller copies run in the same process)
        copies = [v for (k, _), v in vals.items() if "copybuffer" in k.lower()]
        if not copies:
            raise SystemExit("no copy kernel in the counters: profile a --copy-calibration run")
        big = [v for v in copies if v >= 0.25 * max(copies)]
        mode = max(set(big), key=big.count)
        scale[counter] = (1 << 30) / (mode * 1024.0)
        for i, kname in enumerate(PASS_KERNELS):
            vs = [v for (k, _), v in vals.items() if kname in k]
            if vs:
                per.setdefault(i, {})[counter] = sum(vs) / len(vs) * 1024.0 * scale[counter]
                per[i]["launches_" + counter] = len(vs)
    passes = []
    for i, name in enumerate(PASS_NAMES):
        f = per.get(i, {}).get("FETCH_SIZE")
        w = per.get(i, {}).get("WRITE_SIZE")
        passes.append({"pass": name, "fetch_bytes": f, "write_bytes": w,
                       "bytes_per_launch": (f + w) if f is not None and w is not None else None})
    name = f"{args.workload}_{form}"
    out = {"workload": name, "kernel_hash": kernel_hash(),
           "calibration": {"FETCH_SIZE": scale["FETCH_SIZE"], "WRITE_SIZE": scale["WRITE_SIZE"],
                           "reference": "torch copy of 1 GiB (bench.py --copy-calibration)"},
           "passes": passes,
           "commands": [f"rocprofv3 --pmc {c} --kernel-trace -d <dir> -o run -- python3 bench.py --workload "
                        f"{args.workload} --forms {form} --steps 2 --warmup 1 --no-cpu --no-chi2 "
                        "--copy-calibration" for c in ("FETCH_SIZE", "WRITE_SIZE")]}
    path = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def summarize_counters(run_dirs: list) -> None:
    """Markdown table of per-kernel shader counters (rocprofv3 --pmc runs of SQ_ counters, and of TA_ / TD_ / TCP_ counters for a memory-pipeline table), mean per
    dispatch over the workload's dispatches (those after the plan's precompute binning launch)."""
    per = {}
    for d in run_dirs:
        rows = _counter_rows(d)
        start = max(int(r["Dispatch_Id"]) for r in rows
                    if _is_plan_bin(r["Kernel_Name"]))
        acc, disp = {}, {}
        for r in rows:
            if int(r["Dispatch_Id"]) <= start or "mm::" not in r["Kernel_Name"]:
                continue
            k = r["Kernel_Name"].split("(")[0].replace("void ", "")
            acc.setdefault(k, {}).setdefault(r["Counter_Name"], 0.0)
            acc[k][r["Counter_Name"]] += float(r["Counter_Value"])
            disp.setdefault(k, set()).add(r["Dispatch_Id"])
        for k, cs in acc.items():
            for c, v in cs.items():
                per.setdefault(k, {})[c] = v / len(disp[k])
    print("| kernel | waves | VALU instr / wave | LDS instr / wave | LDS bank-conflict cycles / wave | "
          "waiting (share of wave cycles) | issuing VALU (share) |")
    print("|---|---|---|---|---|---|---|")
    for k, c in sorted(per.items(), key=lambda kv: -kv[1].get("SQ_WAVE_CYCLES", 0.0)):
        w = c.get("SQ_WAVES", 0.0) or 1.0
        cyc = c.get("SQ_WAVE_CYCLES", 0.0) or 1.0
        def f(name, scale=1.0, fmt="{:.0f}"):
            return fmt.format(c[name] * scale) if name in c else "-"
        print(f"| {k} | {w:.0f} | {f('SQ_INSTS_VALU', 1 / w)} | {f('SQ_INSTS_LDS', 1 / w)} | "
              f"{f('SQ_LDS_BANK_CONFLICT', 1 / w)} | {f('SQ_WAIT_ANY', 1 / cyc, '{:.2f}')} | "
              f"{f('SQ_ACTIVE_INST_VALU', 1 / cyc, '{:.2f}')} |")
    mem = {k: c for k, c in per.items() if "TCP_TCC_READ_REQ_sum" in c}
    if mem:
        # memory pipeline: vector L1 -> L2 read requests, their mean latency, and how much of the
        # texture-data unit's busy time is spent stalled on the cache
        print()
        print("| kernel | L1->L2 read requests / dispatch | mean L2 read latency (cycles) | "
              "TD stalled on TC (share of TD busy) | TA address stalled on TC (cycles, sum) |")
        print("|---|---|---|---|---|")
        for k, c in sorted(mem.items(), key=lambda kv: -kv[1]["TCP_TCC_READ_REQ_sum"]):
            req = c["TCP_TCC_READ_REQ_sum"] or 1.0
            lat = c.get("TCP_TCC_READ_REQ_LATENCY_sum", 0.0) / req
            td = c.get("TD_TC_STALL_sum", 0.0) / (c.get("TD_TD_BUSY_sum", 0.0) or 1.0)
            ta = c.get("TA_ADDR_STALLED_BY_TC_CYCLES_sum", 0.0)
            print(f"| {k} | {req:.3g} | {lat:.0f} | {td:.2f} | {ta:.3g} |")


def summarize_trace(trace_dir: str) -> None:
    """Markdown table of the workload's kernels (dispatches after the plan's precompute binning)."""
    import csv
    import glob
    files = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no kernel_trace.csv under {trace_dir}")
    with open(files[0]) as fh:
        rows = list(csv.DictReader(fh))
    start = max(int(r["Dispatch_Id"]) for r in rows
                if _is_plan_bin(r["Kernel_Name"]))
    acc = {}
    for r in rows:
        if int(r["Dispatch_Id"]) <= start or "mm::" not in r["Kernel_Name"]:
            continue
        k = r["Kernel_Name"].split("(")[0].replace("void ", "")
        dt = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
        a = acc.setdefault(k, [0, 0.0])
        a[0] += 1
        a[1] += dt
    total = sum(a[1] for a in acc.values())
    print("| kernel | launches | mean us | share of kernel time |")
    print("|---|---|---|---|")
    for k, (n, t) in sorted(acc.items(), key=lambda kv: -kv[1][1]):
        print(f"| {k} | {n} | {t / n:.1f} | {100 * t / total:.1f}% |")




# ---------------------------------------------------------------------------------------------
# algorithmic bytes: each TOD-sized stream a pass of the four-pass deterministic design must read
# or write once, per sample of the workload (the survey's per-pass table; no plan-side tables)

def pass_bytes_per_sample(tod_bytes: int, psi_bytes: int, nbeam: int = 1) -> list:
    """A: d, pix, psi read + transform buffer written; B: buffer read + written; C: buffer read +
    y written; D: y, pix, psi read.  (The map-sized traffic, ~1% here, is left out.)  Composite
    pointing (nbeam = 2) gathers and bins through two pixel / angle pairs per sample."""
    ptg = nbeam * (4 + psi_bytes)
    return [2 * tod_bytes + ptg, 2 * tod_bytes, 2 * tod_bytes, tod_bytes + ptg]


def host_info() -> dict:
    info = {"nproc": os.cpu_count()}
    try:
        info["cores_available"] = len(os.sched_getaffinity(0))
    except AttributeError:
        info["cores_available"] = os.cpu_count()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal"):
                    info["ram_gib"] = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return info


# ---------------------------------------------------------------------------------------------
# inputs

def make_inputs(cfg, dev, log):
    """The workload in device memory: the large workload is generated on the GPU, the others on the
    host and copied over (both give a synth.device.DeviceProblem)."""
    import numpy as np
    import torch
    from synth.device import DeviceProblem, make_problem_device
    if cfg.name == "large2048":
        return make_problem_device(cfg, dev)
    from synth import make_problem
    prob = make_problem(cfg, workers=16)
    psi = None
    if prob.psi_index is not None:
        psi = torch.from_numpy(prob.psi_index.view(np.int16)).to(dev).view(torch.uint16)
    elif prob.psi is not None:
        psi = torch.from_numpy(prob.psi).to(dev)
    on_dev = lambda a: None if a is None else torch.from_numpy(a).to(dev)  # noqa: E731
    return DeviceProblem(cfg=cfg, chunks=np.arange(cfg.ndet), chunk_off=prob.chunk_off, fsample=prob.fsample,
                         sigma=prob.sigma, fknee=prob.fknee, alpha=prob.alpha, pix=torch.from_numpy(prob.pix).to(dev),
                         psi=psi, psi_table=prob.psi_table, d=torch.from_numpy(prob.d).to(dev), m_true=prob.m_true,
                         pix_b=on_dev(prob.pix_b), psi_b=on_dev(prob.psi_b), weights=prob.weights)


def _form_angles(a, form):
    import torch
    if a is None or a.dtype == torch.uint16:
        return a
    return a.float() if form == "mixed" else a.double()


def form_inputs(P, form):
    """TOD and angles of one form: FP32-mixed takes FP32 TOD and FP32 angles (or the uint16 index),
    FP64 takes the stored values promoted to FP64 (the uint16 index as it is)."""
    import torch
    if form == "mixed":
        d = P.d if P.d.dtype == torch.float32 else P.d.float()
    else:
        d = P.d if P.d.dtype == torch.float64 else P.d.double()
    return d, _form_angles(P.psi, form)


def build_plan(mm, P, form, psi, **over):
    kw = dict(ncomp=P.ncomp, npix=P.npix, nx=P.cfg.nx, chunk_off=P.chunk_off, fsample=P.fsample, sigma=P.sigma,
              fknee=P.fknee, alpha=P.alpha, pix=P.pix, psi=psi, psi_table=P.psi_table,
              precision=mm.MM_MIXED if form == "mixed" else mm.MM_FP64)
    if P.pix_b is not None:  # differential beams: the second pointing component
        kw.update(pix_b=P.pix_b, psi_b=_form_angles(P.psi_b, form), weights=P.weights)
    kw.update(over)
    return mm.mm_plan(**kw)


# ---------------------------------------------------------------------------------------------
# one form: plan, warm-up, the timed K iterations, per-pass durations

def run_form(mm, torch, P, form, args, log):
    import numpy as np
    dev = P.pix.device
    d, psi = form_inputs(P, form)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = build_plan(mm, P, form, psi,
                      map_access={"auto": mm.MM_MAP_AUTO, "gather": mm.MM_MAP_GATHER,
                                  "projected": mm.MM_MAP_PROJECTED}[args.map_access],
                      tune=mm.MM_TUNE_MEASURE if args.tune == "measure" else mm.MM_TUNE_STATIC,
                      binning=mm.MM_BIN_ATOMIC if args.binning == "atomic" else mm.MM_BIN_SORTED,
                      tile_pixels=args.tile_pixels)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    stats = mm.mm_plan_binning_stats(plan)
    log(f"[{form}] plan built in {t_plan:.2f} s ({plan.workspace.numel() / 2**30:.1f} GiB workspace; "
        f"{stats['sub_batches']} sub-batches, {stats['segments']} segments)")
    ns = P.nsamp_total
    m_a = torch.zeros((P.ncomp, P.npix), dtype=torch.float64, device=dev)
    m_b = torch.zeros_like(m_a)
    projected = mm.mm_plan_map_access(plan) == mm.MM_MAP_PROJECTED
    # start from the binned map, as the cooled solve does
    mm.mm_messenger_iter(plan, d, math.inf, m_a, m_a)
    if args.warmup > 0:
        mm.mm_solve(plan, d, [1.0], [args.warmup], m_b, first_inf=False, m0=m_a)
        m_a, m_b = m_b, m_a
    torch.cuda.synchronize()
    # timed region: K chained iterations at lambda = 1 as the solver runs them (one HIP graph; with
    # projected access only the first iteration runs the projection pass).  The graph of this exact
    # call is captured by an untimed call first; the timed call replays it.
    stream = torch.cuda.current_stream()
    mm.mm_solve(plan, d, [1.0], [args.steps], m_b, first_inf=False, m0=m_a)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    mm.mm_solve(plan, d, [1.0], [args.steps], m_b, first_inf=False, m0=m_a)
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    ms_step = total_ms / args.steps
    log(f"[{form}] timed {args.steps} iterations (graph replay): {ms_step:.4f} ms each")
    # per-pass durations: the same K iterations uncaptured, HIP events around every pass on the launch
    # stream (mm_set_timing); not part of the timed region above
    mm.mm_set_timing(plan, True)
    ev2, ev3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev2.record(stream)
    mm.mm_solve(plan, d, [1.0], [args.steps], m_b, first_inf=False, m0=m_a)
    ev3.record(stream)
    torch.cuda.synchronize()
    timed_passes_ms = ev2.elapsed_time(ev3)
    pass_ms, pass_n = mm.mm_get_timing(plan)
    mm.mm_set_timing(plan, False)
    tod_bytes = 4 if form == "mixed" else 8
    psi_bytes = 0 if psi is None else psi.element_size()
    per = pass_bytes_per_sample(tod_bytes, psi_bytes, 2 if P.pix_b is not None else 1)
    avg = [pass_ms[i] / max(pass_n[i], 1) for i in range(5)]
    dom = int(np.argmax(avg[:4]))
    alg = [b * ns for b in per]
    achieved = alg[dom] / (avg[dom] * 1e-3) / 1e9
    khash = kernel_hash()
    traffic = load_traffic(f"{P.cfg.name}_{form}", khash)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": (traffic["passes"][dom]["bytes_per_launch"] if traffic else None),
            "kernel": PASS_NAMES[dom], "bytes_per_sample": per[dom], "samples_per_launch": ns}
    non = int((P.pix >= 0).sum().item()) + (0 if P.pix_b is None else int((P.pix_b >= 0).sum().item()))
    out = {
        "form": form, "value": round(ns / (ms_step * 1e-3), 1), "ms_per_step": round(ms_step, 5),
        "roofline": roof,
        "sweep_roofline_frac": round(sum(per) * ns / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "sweep_bytes_per_sample": sum(per),
        # the bytes no schedule can avoid: d, pix (both beams' for composite pointing) and the
        # on-map angles, each read once per iteration
        "compulsory_frac": round((ns * (tod_bytes + 4 * (2 if P.pix_b is not None else 1)) + non * psi_bytes)
                                 / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "ms_per_step_with_pass_events": round(timed_passes_ms / args.steps, 5),
        "map_access": "projected" if projected else "gather",
        "passes": [{"pass": PASS_NAMES[i], "avg_ms": round(avg[i], 5), "launches": int(pass_n[i]),
                    "alg_bytes": alg[i] if i < 4 else None,
                    "GBs": round(alg[i] / (avg[i] * 1e-3) / 1e9, 1) if (i < 4 and avg[i] > 0) else None}
                   for i in range(5)],
        "plan_s": round(t_plan, 2), "workspace_GiB": round(plan.workspace.numel() / 2 ** 30, 2),
        "binning_lists": stats, "kernel_hash": khash, "layouts": layout_summary(mm, plan),
    }
    plan.close()
    del plan, d
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------------------------
# gap filling (composite noise N = N_0 + N_1): throughput of the four-field iteration

def gapfill_rate(mm, torch, P, form, args, log, eps_frac: float = 0.2, run: int = 200):
    """K gap-filling iterations at lambda = 1 on the workload with a fraction args.gapfill of its
    samples in gaps (runs of `run` samples at seeded random places), after W warm-up iterations.
    The plan moves eps = eps_frac sigma^2 of each chunk's white level into N_1 (tau = sigma^2 - eps)."""
    import numpy as np
    dev = P.pix.device
    d, psi = form_inputs(P, form)
    ns = P.nsamp_total
    rng = np.random.default_rng(1705)
    nrun = max(1, int(args.gapfill * ns / run))
    starts = torch.from_numpy(rng.integers(0, ns - run, size=nrun)).to(dev)
    gaps = torch.zeros(ns, dtype=torch.uint8, device=dev)
    idx = (starts[:, None] + torch.arange(run, device=dev)[None, :]).reshape(-1)
    gaps[idx] = 1
    del idx, starts
    tau = (1.0 - eps_frac) * np.asarray(P.sigma) ** 2
    plan = build_plan(mm, P, form, psi, tau=tau, with_gapfill=True)
    m = torch.zeros((P.ncomp, P.npix), dtype=torch.float64, device=dev)
    mm.mm_solve_gapfill(plan, d, gaps, [1.0], [max(args.warmup, 1)], m, first_inf=True)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    mm.mm_solve_gapfill(plan, d, gaps, [1.0], [args.steps], m, first_inf=False, m0=m)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    frac = float(gaps.float().mean().item())
    log(f"[gapfill {form}] {ms:.3f} ms per iteration ({frac:.3f} of the samples in gaps)")
    plan.close()
    del plan, gaps
    torch.cuda.empty_cache()
    return {"form": form, "value": round(ns / (ms * 1e-3), 1), "unit": "samples/s", "ms_per_step": round(ms, 5),
            "gap_fraction": round(frac, 4), "gap_run": run, "eps_over_sigma2": eps_frac,
            "note": "each iteration: the d_0 filter sweep, the t_0 / map filter sweep, two time-domain field "
                    "updates and the binning pass (eager launches)"}


# ---------------------------------------------------------------------------------------------
# time to a chi^2 target

def _first_at_or_below(hist, target):
    import numpy as np
    idx = np.nonzero(np.asarray(hist) <= target)[0]
    return int(idx[0]) if idx.size else None


def time_to_chi2(mm, torch, P, log, tail: int, cg_max: int, deltas=(1e-5, 1e-4, 1e-3)):
    """Wall time (HIP events around a replayed solve graph, for both solvers) to reach
    chi2_ref (1 + delta).  chi2_ref is the lower of the FP64 messenger run below continued at
    lambda = 1 and FP64 PCG to a relative residual of 1e-10.  Compared: the cooled messenger in
    FP64 and FP32-mixed (the workload's schedule, then `tail` iterations at lambda = 1) and FP64
    PCG from zero.  One plan at a time."""
    dev = P.pix.device
    cfg = P.cfg
    shape = (P.ncomp, P.npix)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    runs, times, its_of = {}, {}, {}
    out = {"nsamp": P.nsamp_total, "targets": {}}
    cg_hist = None
    chi_cg = None
    lams = its = None
    for form in ("fp64", "mixed"):
        d, psi = form_inputs(P, form)
        plan = build_plan(mm, P, form, psi)
        if lams is None:
            levels = mm.mm_cooling_levels(plan, cfg.nlevel, cfg.lambda_max or 0.0)
            lams = levels + [1.0]
            its = [cfg.iters_per_level] * cfg.nlevel + [tail]
        nit = 1 + sum(its)
        m = torch.zeros(shape, dtype=torch.float64, device=dev)
        h = torch.zeros(nit + 1, dtype=torch.float64, device=dev)
        mm.mm_solve(plan, d, lams, its, m, chi2_hist=h)
        torch.cuda.synchronize()
        runs[form] = h.cpu().numpy()
        log(f"[chi2] {form} messenger history: {nit} iterations")
        if form == "fp64":
            mc = torch.zeros(shape, dtype=torch.float64, device=dev)
            hc = torch.zeros(cg_max + 1, dtype=torch.float64, device=dev)
            n_cg = mm.mm_cg_solve(plan, mc, cg_max, d=d, chi2_hist=hc, rtol=1e-10)
            torch.cuda.synchronize()
            cg_hist = hc.cpu().numpy()[: n_cg + 1]
            chi_cg = mm.mm_chi2(plan, d, mc)
            log(f"[chi2] fp64 PCG: {n_cg} iterations")
            ref = min(float(runs["fp64"][-1]), chi_cg)
            out["chi2_ref"] = ref
            out["chi2_ref_source"] = (f"messenger FP64, schedule + {tail} at lambda=1" if runs["fp64"][-1] <= chi_cg
                                      else f"FP64 PCG, {n_cg} iterations (relative residual 1e-10)")
        ref = out["chi2_ref"]

        def timed_solve(niters):
            # schedule prefix of niters iterations (the lambda = inf step first)
            rem = niters - 1
            lam_p, it_p = [], []
            for lam, k in zip(lams, its):
                if rem <= 0:
                    break
                take = min(k, rem)
                lam_p.append(lam)
                it_p.append(take)
                rem -= take
            mm.mm_solve(plan, d, lam_p, it_p, m)  # capture
            torch.cuda.synchronize()
            e0, e1 = ev(), ev()
            e0.record()
            mm.mm_solve(plan, d, lam_p, it_p, m)  # replay
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1)

        for delta in deltas:
            i = _first_at_or_below(runs[form], ref * (1 + delta))  # hist[i]: chi^2 after i iterations
            row = out["targets"].setdefault(f"{delta:g}", {})
            row[f"messenger_{form}"] = ({"iterations": i, "ms": round(timed_solve(i), 3)}
                                        if i is not None and i > 0 else {"iterations": None, "ms": None})
            if form == "fp64":
                j = _first_at_or_below(cg_hist, ref * (1 + delta))
                if j is not None and j > 0:
                    mm.mm_cg_solve(plan, mc, j, d=d)  # capture (a fixed count runs as one graph)
                    torch.cuda.synchronize()
                    e0, e1 = ev(), ev()
                    e0.record()
                    mm.mm_cg_solve(plan, mc, j, d=d)  # replay
                    e1.record()
                    torch.cuda.synchronize()
                    row["cg_fp64"] = {"iterations": j, "ms": round(e0.elapsed_time(e1), 3)}
                else:
                    row["cg_fp64"] = {"iterations": None, "ms": None, "chi2_last": float(cg_hist[-1])}
        plan.close()
        del plan, d
        torch.cuda.empty_cache()
    out["schedule"] = f"1 + {cfg.nlevel}x{cfg.iters_per_level} + {tail} at lambda=1"
    out["chi2_final"] = {k: float(v[-1]) for k, v in runs.items()}
    out["chi2_cg_final"] = chi_cg
    return out


# ---------------------------------------------------------------------------------------------
# the CPU oracle on a bounded sample of the workload

_BARRIER = None


def _oracle_init(barrier):
    global _BARRIER
    _BARRIER = barrier


def _oracle_worker(path, niter, wait):
    """One process: the oracle's plan set-up, then `niter` timed messenger steps (after all the
    processes of a group have set up, when `wait`)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.composite import make_composite_setup
    from oracle.messenger import make_setup, messenger_step
    z = np.load(path)
    with threadpool_limits(limits=1):
        args = (z["chunk_off"], z["fsample"], z["sigma"], z["fknee"], z["alpha"], z["pix"],
                z["psi"] if z["psi"].size else None)
        if "pix_b" in z:
            S = make_composite_setup(*args, z["pix_b"], z["psi_b"] if z["psi_b"].size else None, int(z["npix"]),
                                     int(z["ncomp"]), w_a=float(z["weights"][0]), w_b=float(z["weights"][1]))
        else:
            S = make_setup(*args, int(z["npix"]), int(z["ncomp"]))
        d = z["d"]
        m = np.zeros((S.ncomp, S.npix))
        if wait:
            _BARRIER.wait()
        times = []
        for _ in range(niter):
            t0 = time.perf_counter()
            m = messenger_step(S, d, m, 1.0)
            times.append(time.perf_counter() - t0)
    return int(z["chunk_off"][-1]), times


def cpu_baseline(P, seconds: float, log):
    """The oracle's messenger step (lambda = 1, float64 NumPy) on detector chunks of the workload
    itself, copied from the device: on one host thread over the first 16 chunks, and on all
    available cores as one process per core, each on chunks of its own, timed together."""
    import multiprocessing as mp
    import tempfile
    from concurrent.futures import ProcessPoolExecutor
    import numpy as np
    info = host_info()
    ncores = max(1, min(16, info.get("cores_available") or 1))
    nsub = min(16, P.nchunk)
    tmp = tempfile.mkdtemp(prefix="mm_oracle_")
    ctx = mp.get_context("spawn")

    def dump(name, idx):
        h = P.host_chunks(idx)
        path = os.path.join(tmp, name + ".npz")
        extra = {}
        if "pix_b" in h:
            extra = dict(psi_b=h["psi_b"] if h["psi_b"] is not None else np.zeros(0),
                         weights=np.asarray(P.weights, dtype=np.float64))
        np.savez(path, npix=P.npix, ncomp=P.ncomp, psi=h["psi"] if h["psi"] is not None else np.zeros(0),
                 **extra, **{k: v for k, v in h.items() if k not in ("psi", "psi_b")})
        return path, int(h["chunk_off"][-1])

    try:
        # one thread, 16 chunks
        path, ns1 = dump("single", list(range(nsub)))
        with ProcessPoolExecutor(max_workers=1, mp_context=ctx) as ex:
            n1, times1 = ex.submit(_oracle_worker, path, 3, False).result(timeout=max(600.0, 40 * seconds))
        per1 = float(np.median(times1))
        log(f"[cpu] oracle, one thread, {nsub} chunks: {per1:.2f} s per iteration")
        # all cores: one process per core, chunk groups of their own, timed together
        per_worker = max(1, min(4, P.nchunk // ncores))
        paths = []
        for w in range(ncores):
            idx = [(w * per_worker + k) % P.nchunk for k in range(per_worker)]
            paths.append(dump(f"w{w}", idx)[0])
        bar = ctx.Barrier(ncores)
        with ProcessPoolExecutor(max_workers=ncores, mp_context=ctx, initializer=_oracle_init,
                                 initargs=(bar,)) as ex:
            futs = [ex.submit(_oracle_worker, p_, 2, True) for p_ in paths]
            res = [f.result(timeout=max(900.0, 60 * seconds)) for f in futs]
        rate_all = sum(n / float(np.median(t)) for n, t in res)
        log(f"[cpu] oracle, {ncores} processes: {rate_all:.3e} samples/s together")
    finally:
        import shutil
        shutil.rmtree(tmp, ignore_errors=True)
    return {"value": round(rate_all, 1), "unit": "samples/s", "cores": ncores, "kind": "oracle",
            "sample": (f"float64 NumPy oracle, lambda=1 messenger iterations on chunks of this workload with the "
                       f"full {P.cfg.nx}x{P.cfg.nx} map: {ncores} single-threaded processes at once, each on "
                       f"{per_worker} chunk(s) of its own (median of 2 iterations each), summed; the rate is per "
                       f"sample, so it extrapolates linearly to all {P.nsamp_total} samples"),
            "single_thread": {"value": round(ns1 / per1, 1), "unit": "samples/s", "cores": 1,
                              "sample": f"{nsub} chunks ({ns1} samples), median of 3 iterations, {per1:.2f} s each"},
            "host": info}


# ---------------------------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="large2048")
    ap.add_argument("--forms", default="mixed,fp64",
                    help="comma list of forms to time: mixed (FP32 TOD/transforms), fp64; the first gives value")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-chi2", action="store_true", help="skip the time-to-chi2-target comparison")
    ap.add_argument("--chi2-tail", type=int, default=60, help="lambda = 1 iterations after the schedule")
    ap.add_argument("--cg-max", type=int, default=150)
    ap.add_argument("--tile-pixels", type=int, default=0,
                    help="pixels per binning tile (0: the plan's choice from the map size)")
    ap.add_argument("--map-access", choices=["auto", "gather", "projected"], default="auto",
                    help="how the time-domain sweeps read P m (the plan's rule by default)")
    ap.add_argument("--binning", choices=["sorted", "atomic"], default="sorted",
                    help="deterministic sorted reduction (default) or the FP64-atomic alternative")
    ap.add_argument("--tune", choices=["measure", "static"], default="measure",
                    help="transform layouts: timed at plan time (default) or the fixed rule")
    ap.add_argument("--gapfill", type=float, default=0.0, metavar="FRAC",
                    help="also time gap-filling iterations with this fraction of the samples in gaps")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device-to-device copy (reference for HBM byte counters)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU run: read two rocprofv3 --pmc outputs (FETCH_SIZE, WRITE_SIZE) of a "
                         "--copy-calibration run of one form and write profiles/traffic_<workload>_<form>.json")
    ap.add_argument("--summarize-counters", metavar="PMC_DIR", nargs="+",
                    help="print per-kernel shader-counter ratios from rocprofv3 --pmc runs of SQ_ counters")
    ap.add_argument("--summarize-trace", metavar="TRACE_DIR",
                    help="no GPU run: per-kernel launch count and mean duration of the workload's dispatches "
                         "in a rocprofv3 --kernel-trace output (markdown table)")
    args = ap.parse_args()
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    if any(f not in ("mixed", "fp64") for f in forms) or not forms:
        ap.error("--forms takes mixed and/or fp64")
    if args.write_traffic:
        write_traffic(args, forms[0], *args.write_traffic)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the path shards over detector "
              "chunks with one map all-reduce per iteration, which is not implemented)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from synth import config_by_name
    from paper_1705_01893_amd import mm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    cfg = config_by_name(args.workload)
    log = lambda msg: print(f"[bench] {msg}", file=sys.stderr, flush=True)  # noqa: E731
    log(f"generating {cfg.name}")
    t0 = time.perf_counter()
    P = make_inputs(cfg, dev, log)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    ns = P.nsamp_total
    log(f"generated {ns} samples in {t_gen:.1f} s")
    results = [run_form(mm, torch, P, f, args, log) for f in forms]
    head = results[0]
    gapfill = None
    if args.gapfill > 0:
        if P.pix_b is not None:
            log("gap filling needs single-beam pointing: skipped")
        else:
            gapfill = [gapfill_rate(mm, torch, P, f, args, log) for f in forms]
    # what a plain device-to-device copy reaches on this GPU (read + write bytes per second):
    # the practical ceiling of a streaming pass, beside the published HBM peak
    csrc = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    cdst = torch.empty_like(csrc)
    cdst.copy_(csrc)
    ev4, ev5 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev4.record()
    for _ in range(5):
        cdst.copy_(csrc)
    ev5.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * csrc.numel() * 8 * 5 / (ev4.elapsed_time(ev5) * 1e-3) / 1e9
    del csrc, cdst
    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    chi2_block = None
    if not args.no_chi2:
        log("time to chi^2 target")
        chi2_block = time_to_chi2(mm, torch, P, log, args.chi2_tail, args.cg_max)
    cpu = None
    if not args.no_cpu:
        log("oracle on the host")
        cpu = cpu_baseline(P, args.cpu_seconds, log)
    per_chunk = ns // P.nchunk if len(set(int(x) for x in (P.chunk_off[1:] - P.chunk_off[:-1]))) == 1 else None
    if P.psi is None:
        psi_desc = "temperature only"
    elif P.psi_table is not None:
        psi_desc = "uint16 angle-table index"
    else:
        psi_desc = str(P.psi.dtype).replace("torch.", "") + " angles"
    if P.pix_b is not None:
        psi_desc += f"; differential beams {cfg.diff_sep:g} pixels apart, weights {P.weights[0]:+g} / {P.weights[1]:+g}"
    form_name = {"mixed": "FP32-mixed", "fp64": "FP64"}
    cfg_desc = {"workload": (f"{cfg.name}: {P.nchunk} detectors x {per_chunk if per_chunk else 'uneven'} samples "
                             f"({ns} total), {cfg.nx}x{cfg.nx} map, ncomp={P.ncomp}, {psi_desc}; value: "
                             f"{form_name[head['form']]}"
                             + (f", {', '.join(form_name[r['form']] for r in results[1:])} in detail.forms"
                                if len(results) > 1 else "")),
                "nsamp": ns, "npix": P.npix, "ncomp": P.ncomp, "nchunk": P.nchunk}
    out = {
        "metric": "TOD samples/s per messenger iteration", "value": head["value"], "unit": "samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if head["form"] == "mixed" else "f64", "data": "synthetic", "config": cfg_desc,
        "roofline": head["roofline"], "cpu_baseline": cpu, "time_to_chi2": chi2_block,
        "detail": {"forms": results, "gapfill": gapfill, "copy_GBs": round(copy_gbs, 1),
                   "copy_frac_of_peak": round(copy_gbs / HBM_PEAK_GBS, 4), "generate_s": round(t_gen, 2),
                   "binning": args.binning},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
