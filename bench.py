#!/usr/bin/env python3
"""Benchmark of the sketched plug-and-play fan-beam CT hot path on one MI355X.

Workload (a step): one complete multi-stage sketched PnP-SGD reconstruction at
512 x 512: fan beam with 720 views x 768 bins, b = A x + 0.5% signal-dependent Gaussian
noise, stages 4x4 pooling (128^2 grid), 2x2 (256^2), full resolution, 20 iterations
each, every gradient on 1 of 8 interleaved view subsets, TV-prox denoiser (5 Chambolle
steps, lambda 0.01), FISTA-type momentum (Sec. 2.1 Algorithm 1, Option 2; Sec. 3).
The 60 iterations run as one captured HIP graph; inputs are resident in HBM.

Printed JSON line: PnP iterations/s of the sketched schedule, plus the roofline of the
dominant kernel, the FP64 oracle's rate on host cores, projector GUPS and
time-to-PSNR of the sketched run against full-gradient PnP-FISTA on the same GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published figures used as roofline denominators
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3           # FP32 vector peak, counting packed FP32 (two lanes per operation)
PEAK_FP32_NONPACKED_TFLOPS = 78.6  # the same without packed FP32, which this build leaves out
# algorithmic FP32 operations per unit of work: one Joseph sample (forward or back) is
# 12 operations (position fma, floor, fraction, index, two taps, bounds mask and select,
# interpolation sub + fma, accumulate); a TV-prox step is 30 operations per pixel
# (divergence, gradient, magnitude with sqrt, reciprocal, normalisation)
OPS_PER_SAMPLE = 12
OPS_PER_FP_RAY = 2          # length scaling and residual subtraction
OPS_PER_BP_FINE_PIXEL = 2   # z = y_prev - scale * (U g)
OPS_PER_TV_PIXEL_ITER = 30
OPS_PER_TV_PIXEL_OUT = 8    # final divergence, relaxation, momentum
GATHER_BYTES_PER_SAMPLE = 8  # the two 4-byte interpolation taps of a Joseph sample
KERNEL_DESCRIPTION = {"fp": "Joseph forward projection minus b", "bp": "matched back-projection fused with the "
                      "gradient step", "tv": "TV-prox with relaxation, momentum and pooling epilogue"}
KERNEL_SOURCES = ["paper_2203_07308_amd/csrc/" + f for f in
                  ("device.h", "kernels.hip", "fbpnp_impl.h", "plan.cpp", "tune.cpp")]
TRAFFIC_SUMMARY = "profiles/ms2g512_hbm_traffic.md"
SHIPPED_TUNE_CACHE = "paper_2203_07308_amd/tuned/mi355x_launch_configs.txt"


def tune_cache_path(args) -> str:
    """The autotuner cache file this run uses (see --tune-cache / --retune)."""
    import shutil
    import tempfile

    if args.tune_cache:
        return args.tune_cache
    path = os.path.join(tempfile.mkdtemp(prefix="fbpnp_tune_"), "launch_configs.txt")
    shipped = os.path.join(ROOT, SHIPPED_TUNE_CACHE)
    if not args.retune and os.path.exists(shipped):
        shutil.copyfile(shipped, path)
    return path


def kernel_source_hash() -> str:
    """sha256 over the kernel sources: hardware-counter figures are valid only for this text."""
    import hashlib

    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def launch_kernel(kind: str, cfg: dict, tv_iters: int = 5) -> str:
    """Template name of the kernel that one launch of a fused step runs ("fp", "bp" or
    "tv") under the launch configuration cfg (fb_launch_config fields, as get_config
    returns them), as rocprofv3 names it: the back-projector's gather (bp_px 1, 2, 4) or
    scatter form (bp_px 16, 32), the projector's global or LDS taps."""
    if kind == "fp":
        return ("k_fp_lds" if cfg["fp_lds"] == 2 else "k_fp") + f"<true, {cfg['fp_seg']}>"
    if kind == "bp":
        if cfg["bp_px"] >= 16:
            return f"k_bps<{cfg['bp_px']}, {cfg['bp_vg']}, true>"
        return f"k_bp<{cfg['bp_vg']}, {cfg['bp_px']}, true, false>"
    t = cfg["tv_tile"]
    return f"k_tv<{t}, {6 if tv_iters <= 5 else 9}, {1024 if t == 32 else 256}>"


def bp_form(cfg: dict) -> str:
    return "scatter" if cfg["bp_px"] >= 16 else "gather"


# what limits each launch form on this GPU, read from its counters (SQ_INSTS_VALU, VALU
# busy, SQ_INSTS_LDS, SQ_LDS_BANK_CONFLICT in the committed counter summary); the roofline
# itself stays on the survey's ALU accounting (operations per sample against the FP32 peak)
LIMITER = {
    "bp_scatter": "LDS: one read-add-write of both taps per sample into per-wavefront block copies, "
                  "with bank conflicts (VALU about 0.6 busy)",
    "bp_gather": "VALU issue at full resolution (candidate ranges and per-candidate weights); "
                 "the dependent chain of views per wavefront at the coarse stages",
    "fp": "the scattered tap loads through L1 and L2 at full resolution (their width, lanes per "
          "address and loads in flight each change the time by at most 7 percent); each "
          "wavefront's dependent chain at the coarse stages",
    "tv": "latency of loads, LDS exchanges and barriers between dual steps",
}


def launch_traffic(key: str, path: str | None = None, kernel: str | None = None):
    """HBM bytes per launch of kernel group `key` (e.g. "bp_f1") from the committed
    counter summary, or None when it is missing, was taken from other kernel sources,
    or (with kernel) was measured on another kernel than the one named."""
    import re

    path = path or os.path.join(ROOT, TRAFFIC_SUMMARY)
    if not os.path.exists(path):
        return None, "no counter summary"
    text = open(path).read()
    m = re.search(r"kernel sources sha256: `([0-9a-f]{64})`", text)
    if not m or m.group(1) != kernel_source_hash():
        return None, "counter summary predates the current kernel sources"
    m = re.search(r"^\| " + re.escape(key) + r" \| ([^|\n]*)\|(?:[^|\n]*\|){5}\s*([0-9]+)\s*\|", text, re.M)
    if not m:
        return None, f"no {key} row in the counter summary"
    if kernel is not None and m.group(1).strip() != f"`{kernel}`":
        return None, f"counter summary measured {m.group(1).strip()} for {key}, not `{kernel}`"
    return int(m.group(2)), TRAFFIC_SUMMARY


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the FP64 oracle timing")
    ap.add_argument("--no-ttp", action="store_true", help="skip the time-to-PSNR comparison")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-slice batched workload")
    ap.add_argument("--no-diff", action="store_true",
                    help="skip the differentiation workload (reverse mode through 10 unrolled iterations, 8 slices)")
    ap.add_argument("--no-scenarios", action="store_true",
                    help="skip the paper's three scenarios (sparse-view, low-dose, limited-angle)")
    ap.add_argument("--tune-cache", metavar="PATH",
                    help="autotuner cache to read and extend (default: a temporary copy of the shipped "
                         "MI355X cache, so a run never edits the tree)")
    ap.add_argument("--retune", action="store_true", help="start from an empty autotuner cache")
    ap.add_argument("--tune-only", action="store_true",
                    help="run the autotuner for every launch the bench makes (with --tune-cache), then exit")
    ap.add_argument("--batch-steps", type=int, default=3, help="timed replays of the batched schedule")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--profile", action="store_true",
                    help="short run for hardware-counter passes: two replays of the sketched schedule "
                         "and a 64 MiB device copy (counter calibration); prints no JSON line")
    ap.add_argument("--trace-summary", metavar="DIR",
                    help="print a markdown summary of a rocprofv3 --kernel-trace --stats -f csv output directory "
                         "(no GPU use)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print the HBM traffic summary of two rocprofv3 --pmc runs of --profile "
                         "(FETCH_SIZE, then WRITE_SIZE), calibrated by the 64 MiB copy (no GPU use)")
    ap.add_argument("--counters", nargs="*", default=[], metavar="DIR",
                    help="with --pmc-summary: further rocprofv3 --pmc output directories (any counters), averaged "
                         "per iteration group; with --trace-dir, VALU utilisation and L2 hit rate are derived")
    ap.add_argument("--trace-dir", help="with --pmc-summary: a kernel-trace directory for per-group durations")
    ap.add_argument("--cmd", default="", help="command line quoted in a summary")
    ap.add_argument("--title", default="", help="with --trace-summary: the workload the trace covers")
    ap.add_argument("--forms", action="store_true",
                    help="launch every forward-projector and back-projector form of each stage of the 512^2 "
                         "workload (one 90-view subset) and of the 256^2 sparse-view scenario, ten times each, "
                         "printing a label per form; run under rocprofv3 --kernel-trace and summarise with "
                         "--forms-summary (no JSON line)")
    ap.add_argument("--forms-summary", nargs=2, metavar=("TRACE_DIR", "LOG"),
                    help="kernel durations per form from a rocprofv3 kernel trace of --forms and its log (no GPU use)")
    ap.add_argument("--bench-log", help="log of the profiled command (its JSON line is quoted in a trace summary)")
    ap.add_argument("--section", choices=("differentiation", "batched", "scenarios"),
                    help="run only that workload (as the full run does, with its own set-up) and log its result; "
                         "for kernel traces of one workload (no JSON line)")
    return ap.parse_args()


class Events:
    """Wall time of work enqueued on torch's current stream (the library launches there)."""

    def __init__(self, torch):
        self.torch = torch
        self.a = torch.cuda.Event(enable_timing=True)
        self.b = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.a.record()
        return self

    def __exit__(self, *exc):
        self.b.record()
        self.b.synchronize()
        self.ms = self.a.elapsed_time(self.b)


def _short(name: str) -> str:
    name = name.replace("void ", "").replace("(anonymous namespace)::", "")
    return name[: name.index("(")] if "(" in name else name


def _csv(directory: str, suffix: str):
    import csv
    import glob

    files = sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {directory}")
    with open(files[0]) as fh:
        return list(csv.DictReader(fh))


def label_dispatches(names, grids=None):
    """(group, index) labels of the dispatches that belong to complete replays of the
    sketched schedule, e.g. ("bp_f1", i): a replay is the pooling kernel followed by
    exactly one forward projection, back-projection and denoiser launch per iteration
    (other sequences, such as the autotuner's timing runs, are skipped). With grids
    (each dispatch's grid size), the denoiser launches of a replay must all have the
    grid of the 512^2 image, which excludes runs on other image sizes."""
    from paper_2203_07308_amd import synth

    w = synth.WORKLOADS["ms2g512"]
    stage_f = [f for f, n in w.stages for _ in range(n)]
    T = len(stage_f)
    want = (("k_fp<true", "k_fp_lds<true"), ("k_bp<", "k_bps<"), ("k_tv<",))
    out = []
    i = 0
    while i < len(names):
        if names[i] != "k_prepare":
            i += 1
            continue
        lab, j = [("prepare_f%d" % stage_f[0], i)], i + 1
        for t in range(T):
            if j + 3 > len(names) or not all(names[j + k].startswith(want[k]) for k in range(3)):
                break
            for k, c in enumerate(("fp", "bp", "tv")):
                lab.append((f"{c}_f{stage_f[t]}", j + k))
            j += 3
        else:
            tv_grids = {grids[k] for g, k in lab if g.startswith("tv")} if grids is not None else None
            if tv_grids is None or tv_grids == {TV_GRID_512}:
                out += lab
                i = j
                continue
        i += 1
    return out


def trace_summary(args) -> int:
    stats = _csv(args.trace_summary, "kernel_stats.csv")
    trace = _csv(args.trace_summary, "kernel_trace.csv")
    trace.sort(key=lambda r: int(r["Start_Timestamp"]))
    names = [_short(r["Kernel_Name"]) for r in trace]
    grids = [int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]) for r in trace]
    title = args.title or ("512x512 multi-stage sketched PnP-SGD (720 views x 768 bins, f = 4, 2, 1, "
                           "1 of 8 view subsets)")
    out = [f"# rocprofv3 kernel trace: {title}", "", "Command (repository root, one MI355X, library built):", "",
           "```", args.cmd, "```", "", "Summary: `python bench.py --trace-summary <output dir> --cmd '<command>'"
           + (" --title '<workload>'" if args.title else "")
           + (" --bench-log <log>" if args.bench_log else "") + "`", "",
           "## Kernel statistics over the whole run (rocprofv3 --stats)", "",
           "| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in stats[:30]:
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    groups = {}
    for g, j in label_dispatches(names, grids):
        groups.setdefault(g, []).append(j)
    n_rep = len(groups.get("tv_f1", [])) // 20 if groups else 0
    if groups:
        out += ["", f"## Per iteration group, over {n_rep} complete replays of the schedule (graph and direct calls)",
                "", "| group | kernel | launches | avg us | min us | max us | us per replay |",
                "|---|---|---|---|---|---|---|"]
    for g in sorted(groups, key=lambda k: (k.split("_f")[0], -int(k.split("_f")[1]))):
        d = [(int(trace[j]["End_Timestamp"]) - int(trace[j]["Start_Timestamp"])) / 1e3 for j in groups[g]]
        kn = sorted(set(names[j] for j in groups[g]))
        out.append(f"| {g} | {', '.join('`' + k + '`' for k in kn)} | {len(d)} | {sum(d) / len(d):.2f} | "
                   f"{min(d):.2f} | {max(d):.2f} | {sum(d) / max(n_rep, 1):.1f} |")
    if args.bench_log:
        lines = [ln for ln in open(args.bench_log) if ln.startswith("{")]
        if lines:
            res = json.loads(lines[-1])
            out += ["", "## The profiled command's own result line (HIP-event kernel timing)", "",
                    f"- value: {res['value']} {res['unit']} ({res['ms_per_step']} ms per step)",
                    f"- roofline: `{json.dumps(res['roofline'])}`"]
    print("\n".join(out))
    return 0


def pmc_summary(args) -> int:
    fetch = _csv(args.pmc_summary[0], "counter_collection.csv")
    write = _csv(args.pmc_summary[1], "counter_collection.csv")
    out = ["# HBM traffic per launch: 512x512 multi-stage sketched PnP-SGD (rocprofv3 --pmc)", "",
           "Commands (repository root, one MI355X, library built), one counter per pass:", "", "```", args.cmd, "```",
           "", "Summary: `python bench.py --pmc-summary <FETCH_SIZE dir> <WRITE_SIZE dir> --cmd '<commands>'`", "",
           f"kernel sources sha256: `{kernel_source_hash()}`", ""]
    per = {}
    for rows, cname in ((fetch, "FETCH_SIZE"), (write, "WRITE_SIZE")):
        rows = [r for r in rows if r["Counter_Name"] == cname]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        names = [_short(r["Kernel_Name"]) for r in rows]
        grids = [int(r["Grid_Size"]) for r in rows]
        copies = [r for r, n in zip(rows, names) if n == "__amd_rocclr_copyBuffer"]
        if not copies:
            raise SystemExit("no copy kernel for the calibration")
        copy_kib = float(copies[-1]["Counter_Value"])  # the 64 MiB device copy at the end of --profile
        factor = 65536.0 / copy_kib
        per[cname] = {"copy_kib": copy_kib, "factor": factor, "groups": {}}
        for g, j in label_dispatches(names, grids):
            per[cname]["groups"].setdefault(g, []).append((names[j], float(rows[j]["Counter_Value"])))
    cf, cw = per["FETCH_SIZE"]["factor"], per["WRITE_SIZE"]["factor"]
    dur = trace_durations(args.trace_dir) if args.trace_dir else {}
    out += ["Calibration: a 64 MiB device-to-device copy (`__amd_rocclr_copyBuffer`) reads FETCH_SIZE = "
            f"{per['FETCH_SIZE']['copy_kib']:.0f} KiB and WRITE_SIZE = {per['WRITE_SIZE']['copy_kib']:.0f} KiB, "
            f"so bytes = FETCH_SIZE x 1024 x {cf:.4f} and WRITE_SIZE x 1024 x {cw:.4f}.", "",
            "HBM GB/s = traffic bytes per launch / the group's average duration in the kernel trace; "
            f"its share of the {PEAK_HBM_GBS:.0f} GB/s HBM peak beside it.", "",
            "| group | kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | read bytes | written bytes | "
            "traffic bytes per launch | HBM GB/s | of HBM peak |", "|---|---|---|---|---|---|---|---|---|---|"]
    groups = per["FETCH_SIZE"]["groups"]
    for g in sorted(groups, key=lambda k: (k.split("_f")[0], -int(k.split("_f")[1]))):
        fv = [v for _, v in groups[g]]
        wv = [v for _, v in per["WRITE_SIZE"]["groups"].get(g, [])]
        if not wv:
            continue
        fk, wk = sum(fv) / len(fv), sum(wv) / len(wv)
        rb, wb = fk * 1024 * cf, wk * 1024 * cw
        kn = sorted(set(n for n, _ in groups[g]))
        us = sum(dur[g]) / len(dur[g]) if g in dur else None
        gbs = (rb + wb) / (us * 1e-6) / 1e9 if us else None
        rate = "| |" if gbs is None else f"| {gbs:.0f} | {gbs / PEAK_HBM_GBS:.3f} |"
        out.append(f"| {g} | {', '.join('`' + k + '`' for k in kn)} | {len(fv)} | {fk:.1f} | {wk:.1f} | "
                   f"{rb:.0f} | {wb:.0f} | {rb + wb:.0f} " + rate)
    if args.counters:
        out += counter_tables(args)
    print("\n".join(out))
    return 0


TV_GRID_512 = 512 * 512  # work-items of a denoiser launch on the 512^2 image (one per pixel)


# MI355X: 256 CUs x 4 SIMDs; a wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles
N_SIMD, VALU_CYCLES, CLOCK_GHZ = 1024, 4, 2.4


def trace_durations(trace_dir):
    """Durations (us) of every labelled dispatch in a rocprofv3 kernel trace, per group."""
    trace = _csv(trace_dir, "kernel_trace.csv")
    trace.sort(key=lambda r: int(r["Start_Timestamp"]))
    names = [_short(r["Kernel_Name"]) for r in trace]
    grids = [int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]) for r in trace]
    dur = {}
    for g, j in label_dispatches(names, grids):
        dur.setdefault(g, []).append((int(trace[j]["End_Timestamp"]) - int(trace[j]["Start_Timestamp"])) * 1e-3)
    return dur


def counter_tables(args):
    """Per-group averages of further counter passes, and derived figures: VALU busy
    fraction = SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x cycles of the kernel's duration),
    L2 hit rate = TCC_HIT / (TCC_HIT + TCC_MISS)."""
    per = {}
    for d in args.counters:
        rows = _csv(d, "counter_collection.csv")
        by_counter = {}
        for r in rows:
            by_counter.setdefault(r["Counter_Name"], []).append(r)
        for cname, rs in by_counter.items():
            rs.sort(key=lambda r: int(r["Dispatch_Id"]))
            names = [_short(r["Kernel_Name"]) for r in rs]
            for g, j in label_dispatches(names, [int(r["Grid_Size"]) for r in rs]):
                per.setdefault(g, {}).setdefault(cname, []).append(float(rs[j]["Counter_Value"]))
    dur = trace_durations(args.trace_dir) if args.trace_dir else {}
    cnames = sorted({c for v in per.values() for c in v})
    out = ["", "## Further counters (average per dispatch)", "",
           "| group | " + " | ".join(cnames) + " | avg us (trace) | VALU busy | L2 hit |",
           "|---" * (len(cnames) + 4) + "|"]
    for g in sorted(per, key=lambda k: (k.split("_f")[0], -int(k.split("_f")[1]))):
        m = {c: sum(v) / len(v) for c, v in per[g].items()}
        us = sum(dur[g]) / len(dur[g]) if g in dur else None
        valu = (f"{m['SQ_INSTS_VALU'] * VALU_CYCLES / (N_SIMD * us * 1e-6 * CLOCK_GHZ * 1e9):.2f}"
                if us and "SQ_INSTS_VALU" in m else "")
        hit = (f"{m['TCC_HIT_sum'] / (m['TCC_HIT_sum'] + m['TCC_MISS_sum']):.3f}"
               if "TCC_HIT_sum" in m and "TCC_MISS_sum" in m and m["TCC_HIT_sum"] + m["TCC_MISS_sum"] > 0 else "")
        out.append(f"| {g} | " + " | ".join(f"{m[c]:.0f}" if c in m else "" for c in cnames) +
                   f" | {'' if us is None else f'{us:.2f}'} | {valu} | {hit} |")
    return out


FORM_REPS = 10


def projector_forms(torch, fbpnp, synth) -> int:
    """Every launch form of the projector (lanes per ray; taps from global memory or LDS
    where the stage fits) and of the back-projector (gather with 1, 2, 4 pixels per lane;
    scatter over 16 and 32 pixel blocks; 4, 8, 16 wavefronts per block) at each stage of
    the 512^2 workload (subset 0 of 8: 90 views) and of the 256^2 sparse-view scenario (90
    views), FORM_REPS launches each, after one label line per form."""
    cases = [("ms2g512", synth.WORKLOADS["ms2g512"].geometry, 8),
             ("sparse_view", synth.SCENARIOS["sparse_view"].geometry, 1)]
    for name, gd, n_sub in cases:
        V, nb = gd["n_views"], gd["n_bins"]
        plan = fbpnp.Plan(fbpnp.Geometry(**gd), [4, 2, 1])
        views = torch.from_numpy(synth.subset_views(0, n_sub, V).astype(np.int32)).cuda()
        n_sel = views.numel()
        yb = torch.rand(n_sel * nb, device="cuda")
        for k, f in enumerate((4, 2, 1)):
            ny, nx = plan.coarse_shape(k)
            xs = torch.rand((ny, nx), device="cuda")
            y = torch.empty(n_sel * nb, device="cuda")
            forms = [("fp", dict(fp_seg=seg, fp_lds=lds)) for lds in (1, 2) for seg in (1, 2, 4, 8)]
            forms += [("bp", dict(bp_px=px, bp_vg=vg)) for px in (1, 2, 4, 16, 32) for vg in (4, 8, 16)
                      if not (px == 4 and vg > 4)]
            for kind, cfg in forms:
                try:
                    plan.set_config(k, cfg)
                except fbpnp.FbError:
                    continue
                print(f"form {name} f={f} {kind} " + " ".join(f"{a}={b}" for a, b in cfg.items()), flush=True)
                for _ in range(FORM_REPS):
                    if kind == "fp":
                        fbpnp.fanbeam_fp(plan, k, xs, y, views)
                    else:
                        fbpnp.fanbeam_bp(plan, k, yb, xs, views)
                torch.cuda.synchronize()
            plan.set_config(k, None)
        plan.close()
    # the floor of a dependent kernel: a captured graph of 256 one-element kernels, each
    # depending on the one before, replayed 20 times (HIP events)
    t = torch.zeros(1, device="cuda")
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        t.add_(1.0)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            for _ in range(256):
                t.add_(1.0)
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    with Events(torch) as ev:
        for _ in range(20):
            g.replay()
    print(f"floor {1e3 * ev.ms / (20 * 256):.2f} us per dependent one-element kernel in a graph", flush=True)
    return 0


def forms_summary(args) -> int:
    trace_dir, log_path = args.forms_summary
    trace = _csv(trace_dir, "kernel_trace.csv")
    trace.sort(key=lambda r: int(r["Start_Timestamp"]))
    proj = [r for r in trace if _short(r["Kernel_Name"]).startswith(("k_fp", "k_bp"))]
    labels = [ln.split(None, 1)[1].strip() for ln in open(log_path) if ln.startswith("form ")]
    out = ["# rocprofv3 kernel trace: every projector and back-projector form, per stage", "",
           "Workloads: the 512x512 geometry (720 views x 768 bins) with one 90-view subset, and the 256x256 "
           "sparse-view scenario (90 views x 228 bins); stages f = 4, 2, 1; all-view selections as view lists.", "",
           "Command (repository root, one MI355X, library built):", "", "```", args.cmd, "```", "",
           "Summary: `python bench.py --forms-summary <trace dir> <log> --cmd '<command>'`", "",
           f"Average kernel duration over the last {FORM_REPS - 2} of {FORM_REPS} launches of each form.", "",
           "| workload | stage | kind | form | kernel | avg us |", "|---|---|---|---|---|---|"]
    if len(proj) != FORM_REPS * len(labels):
        raise SystemExit(f"{len(proj)} projector dispatches for {len(labels)} forms")
    for i, lab in enumerate(labels):
        grp = proj[FORM_REPS * i:FORM_REPS * (i + 1)]
        d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in grp[2:]]
        name, stage, kind, *cfg = lab.split()
        out.append(f"| {name} | {stage} | {kind} | {' '.join(cfg)} | `{_short(grp[0]['Kernel_Name'])}` | "
                   f"{sum(d) / len(d):.2f} |")
    floor = [ln.strip() for ln in open(log_path) if ln.startswith("floor ")]
    if floor:
        out += ["", f"Kernel floor measured in the same run: {floor[-1][6:]}."]
    print("\n".join(out))
    return 0


def main() -> int:
    args = parse()
    if args.trace_summary:
        return trace_summary(args)
    if args.forms_summary:
        return forms_summary(args)
    if args.pmc_summary:
        return pmc_summary(args)
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        return 2
    import torch

    from paper_2203_07308_amd import fbpnp, synth

    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    torch.cuda.set_device(0)
    if args.forms:
        return projector_forms(torch, fbpnp, synth)
    if args.section == "differentiation":
        differentiation_section(torch, fbpnp, synth, tune_cache_path(args), reps=max(args.steps, 1))
        return 0
    if args.section == "batched":
        batched_section(torch, fbpnp, synth, args.batch_steps, tune_cache_path(args))
        return 0
    if args.section == "scenarios":
        paper_scenarios(torch, fbpnp, synth, tune_cache_path(args))
        return 0
    w = synth.WORKLOADS["ms2g512"]
    gd = w.geometry
    V, B, N = gd["n_views"], gd["n_bins"], gd["nx"]
    npix = N * N
    factors = [f for f, _ in w.stages]
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), factors)
    stage_of = {f: i for i, f in enumerate(factors)}
    s_full = stage_of[1]

    # ---- inputs (untimed): phantom, b = A x + noise, step sizes, subsets
    t0 = time.time()
    xt = synth.phantom(w)
    xt_d = torch.from_numpy(xt).cuda().reshape(-1)
    ax = torch.empty(V * B, device="cuda")
    fbpnp.fanbeam_fp(plan, s_full, xt_d, ax)
    eps = synth.standard_normal(synth.noise_seed(w), (V, B))
    b_np = synth.add_noise(ax.cpu().numpy().astype(np.float64).reshape(V, B), eps, w.noise_kind,
                           w.noise_level).astype(np.float32)
    b = torch.from_numpy(b_np).cuda().reshape(-1)
    L = {f: fbpnp.power_lipschitz(plan, stage_of[f], 100) for f in factors}
    eta = {f: 1.0 / L[f] for f in factors}
    n_sub = w.n_subsets
    log(f"setup {time.time() - t0:.1f}s  L={L}")

    x = torch.zeros(npix, device="cuda")
    y = torch.zeros(npix, device="cuda")

    def schedule(stages, subset_seed, n_sub_used, momentum=True, t_offset=0):
        T = sum(n for _, n in stages)
        a = synth.momentum_table(T + t_offset, momentum)[t_offset:]
        seq = synth.subset_sequence(subset_seed, T, n_sub_used) if n_sub_used else None
        out = []
        t = 0
        for f, n in stages:
            for _ in range(n):
                out.append((f, None if seq is None else int(seq[t]), float(a[t])))
                t += 1
        return out

    def make_steps(sched, hist=None, events=None, vr=None, snaps=None, stamps=None):
        """pnp_step arguments; vr (optional): per-step variance-reduction mode, with
        snaps[f] = (snapshot projection, snapshot coarse gradient) per stage; stamps
        (optional): int64 device buffer, one end-of-step clock stamp per step."""
        steps = []
        for t, (f, s, a_t) in enumerate(sched):
            mode = 0 if vr is None else vr[t]
            # an interleaved subset goes by (k, n_sub): the kernels compute its view indices
            sub = None if (s is None or mode == 1) else (s, n_sub)
            sigma = 1.0 if sub is None else float(n_sub)
            sp, sg = (None, None) if mode == 0 else snaps[f]
            steps.append(fbpnp.pnp_args(plan, stage_of[f], b, y, x, x, y, eta[f], a_t, None, sigma, w.alpha, w.lam,
                                        w.tau, w.tv_iters, None if hist is None else hist[t],
                                        None if events is None else events[t], mode, sp, sg, subset=sub,
                                        stamp=None if stamps is None else stamps[t:t + 1]))
        return steps

    sk_sched = schedule(w.stages, 3000 * w.seed_base, n_sub)
    T = len(sk_sched)
    # launch configurations for the subset size the iterations use (autotuner, HIP-event timed)
    t0 = time.time()
    tune_cache = tune_cache_path(args)
    if args.tune_only:
        for n_sel in (V, V // n_sub):
            plan.autotune(n_sel=n_sel, cache_path=tune_cache)
        batched_section(torch, fbpnp, synth, 0, tune_cache, tune_only=True)
        differentiation_section(torch, fbpnp, synth, tune_cache, tune_only=True)
        log(f"autotuner cache written to {tune_cache}")
        return 0
    plan.autotune(n_sel=V // n_sub, cache_path=tune_cache)
    configs = {f"f{f}": plan.get_config(stage_of[f], V // n_sub) for f in factors}
    log(f"autotune {time.time() - t0:.1f}s: {configs}")
    graph = fbpnp.Graph(plan, make_steps(sk_sched))

    def run_once(g):
        x.zero_()
        y.zero_()
        g.launch()

    def run_once_direct(steps):
        x.zero_()
        y.zero_()
        for st in steps:
            fbpnp.pnp_step(plan, st)
        torch.cuda.synchronize()

    if args.profile:
        for _ in range(2):
            run_once(graph)
        src = torch.ones(16 << 20, device="cuda")  # 64 MiB read, 64 MiB written
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("profile run done")
        return 0

    # ---- timed region: K complete sketched reconstructions
    for _ in range(args.warmup):
        run_once(graph)
    torch.cuda.synchronize()
    with Events(torch) as ev:
        for _ in range(args.steps):
            run_once(graph)
    torch.cuda.synchronize()
    ms_per_step = ev.ms / args.steps
    iters_per_s = T * args.steps / (ev.ms * 1e-3)
    log(f"sketched schedule: {ms_per_step:.3f} ms per {T}-iteration reconstruction, {iters_per_s:.0f} it/s")

    # ---- per-kernel durations: the same schedule by direct pnp_step calls (with the graph's
    # pooling hand-over), each projector / denoiser kernel started with HIP start/stop events
    # on the launch stream (hipExtLaunchKernelGGL), so an event pair spans exactly one kernel
    reps = args.kernel_reps
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(T)]
    tsteps = make_steps(sk_sched, events=evs)
    fbpnp.chain_steps(tsteps)
    vsamp = {f: plan.view_samples(stage_of[f]) for f in factors}
    sub_views = [synth.subset_views(s, n_sub, V) for s in range(n_sub)]
    acc = {}
    for _ in range(reps):
        run_once_direct(tsteps)
        for t, (f, s, _a) in enumerate(sk_sched):
            smp = sum(vsamp[f][v] for v in sub_views[s])
            n_fine = npix
            flops = {"fp": OPS_PER_SAMPLE * smp + OPS_PER_FP_RAY * len(sub_views[s]) * B,
                     "bp": OPS_PER_SAMPLE * smp + OPS_PER_BP_FINE_PIXEL * n_fine,
                     "tv": n_fine * (w.tv_iters * OPS_PER_TV_PIXEL_ITER + OPS_PER_TV_PIXEL_OUT)}
            for k, name in ((0, "fp"), (2, "bp"), (4, "tv")):
                a_ = acc.setdefault((name, f), {"ms": 0.0, "n": 0, "flop": 0.0, "samples": 0, "pixel_views": 0})
                a_["ms"] += evs[t][k].elapsed_time(evs[t][k + 1])
                a_["n"] += 1
                a_["flop"] += flops[name]
                a_["samples"] += smp if name != "tv" else 0
                a_["pixel_views"] += len(sub_views[s]) * (npix // (f * f)) if name != "tv" else 0
    kernels = {}
    for (name, f), a_ in acc.items():
        sec = a_["ms"] * 1e-3
        kernels[f"{name}_f{f}"] = dict(
            avg_launch_us=1e3 * a_["ms"] / a_["n"], launches_per_step=a_["n"] // reps,
            us_per_step=1e3 * a_["ms"] / reps, flop_per_launch=a_["flop"] / a_["n"],
            tflops=a_["flop"] / sec / 1e12,
            # projectors: exact Joseph samples per second; the conventional views x pixels
            # per second; and the effective gather bandwidth, 8 bytes (two taps) per sample,
            # which is on-chip traffic, not HBM bandwidth
            **({"gsamples_per_s": a_["samples"] / sec / 1e9,
                "conventional_gups": a_["pixel_views"] / sec / 1e9,
                "gather_tb_per_s_effective": GATHER_BYTES_PER_SAMPLE * a_["samples"] / sec / 1e12}
               if name != "tv" else {}))
    # each group's measured HBM rate (committed counter traffic per launch over the live
    # launch time) and its share of the HBM roof; and the same for the timed kernels of a step
    step_bytes, step_us, complete = 0, 0.0, True
    for k, v in kernels.items():
        t_k, _ = launch_traffic(k, kernel=launch_kernel(k[:2], configs[k[3:]], w.tv_iters))
        if t_k:
            rate = t_k / (v["avg_launch_us"] * 1e-6) / 1e9
            v.update(hbm_bytes_per_launch=t_k, hbm_gb_per_s=rate, hbm_frac=rate / PEAK_HBM_GBS)
            step_bytes += t_k * v["launches_per_step"]
            step_us += v["us_per_step"]
        else:
            complete = False
    hbm_step = None
    if complete and step_bytes:
        hbm_step = {"bytes_per_step": step_bytes, "kernel_us_per_step": round(step_us, 2),
                    "gb_per_s": round(step_bytes / (step_us * 1e-6) / 1e9, 1),
                    "frac": round(step_bytes / (step_us * 1e-6) / 1e9 / PEAK_HBM_GBS, 5),
                    "covers": "the projector, back-projector and denoiser launches of a step"}
    for k, v in kernels.items():
        log(f"  {k}: {v}")
    dom_name, dom = max(kernels.items(), key=lambda kv: kv[1]["us_per_step"])
    dom_cfg = configs[dom_name[3:]]
    dom_kernel = launch_kernel(dom_name[:2], dom_cfg, w.tv_iters)
    traffic, traffic_src = launch_traffic(dom_name, kernel=dom_kernel)
    form = f", {bp_form(dom_cfg)} form" if dom_name.startswith("bp") else ""
    limiter = LIMITER["bp_" + bp_form(dom_cfg)] if dom_name.startswith("bp") else LIMITER[dom_name[:2]]
    roofline = {"kernel": f"{dom_name} ({KERNEL_DESCRIPTION[dom_name[:2]]}{form}, pooling factor {dom_name[4:]}): "
                          f"{dom_kernel}",
                "bound": "alu", "achieved": round(dom["tflops"], 4), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(dom["tflops"] / PEAK_FP32_TFLOPS, 5), "traffic": traffic,
                "traffic_source": traffic_src,
                "ops_per_sample": OPS_PER_SAMPLE,
                "peak_nonpacked": PEAK_FP32_NONPACKED_TFLOPS,
                "frac_nonpacked": round(dom["tflops"] / PEAK_FP32_NONPACKED_TFLOPS, 5),
                "avg_launch_us": round(dom["avg_launch_us"], 3),
                "flop_per_launch": round(dom["flop_per_launch"]), "launches_timed": dom["launches_per_step"] * reps,
                "limiter": limiter}
    if traffic:
        # the measured HBM rate of the dominant kernel and its share of the HBM roof
        hbm = traffic / (dom["avg_launch_us"] * 1e-6) / 1e12
        roofline.update(hbm_tb_per_s=round(hbm, 4), hbm_frac=round(hbm * 1e3 / PEAK_HBM_GBS, 5))
    # the HBM bandwidth a plain device copy reaches on this GPU, beside the published figure
    roofline.update(hbm_peak_spec_gb_per_s=PEAK_HBM_GBS, hbm_copy_measured_gb_per_s=round(copy_rate(torch), 1))

    # ---- time-to-PSNR: sketched vs full-gradient PnP-FISTA vs full-resolution PnP-SGD
    ttp = None
    if not args.no_ttp:
        ttp = time_to_psnr(torch, fbpnp, synth, w, plan, stage_of, schedule, make_steps, x, y, xt, T, tune_cache)
        plan.autotune(n_sel=V // n_sub, cache_path=tune_cache)  # back to the subset configuration

    # ---- the 64-slice batched form (its own workload; not part of the value above)
    bat = None
    if not args.no_batch:
        bat = batched_section(torch, fbpnp, synth, args.batch_steps, tune_cache)

    # ---- the differentiation workload: reverse mode through unrolled iterations
    diff = None
    if not args.no_diff:
        diff = differentiation_section(torch, fbpnp, synth, tune_cache)

    # ---- the paper's own experiment shapes: two-stage sketch against PnP-FISTA
    scen = None
    if not args.no_scenarios:
        scen = paper_scenarios(torch, fbpnp, synth, tune_cache)

    # ---- FP64 oracle on host cores (bounded sample of the same schedule), and its
    # projectors and smaller loops beside the GPU's
    cpu = None if args.no_cpu_baseline else cpu_baseline(synth, w, xt, sk_sched, eta, n_sub)
    odet = None
    if not args.no_cpu_baseline:
        odet = oracle_detail(torch, fbpnp, synth, plan, s_full, xt, tune_cache)
        plan.autotune(n_sel=V // n_sub, cache_path=tune_cache)

    result = {
        "metric": "PnP iterations/s, multi-stage sketched PnP-SGD, 512^2 fan-beam",
        "value": round(iters_per_s, 2),
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded 40-ellipse phantom + texture, 0.5% signal-dependent Gaussian noise)",
        "config": {"workload": "ms2g512: 512x512, 720 views x 768 bins, stages f=4,2,1 x 20 iterations, "
                               "1 of 8 view subsets, TV-prox 5 x lambda 0.01, FISTA momentum",
                   "iterations_per_step": T, "image": N, "views": V, "bins": B},
        "roofline": roofline,
        "hbm_per_step": hbm_step,
        "launch_configs": configs,
        "cpu_baseline": cpu,
        "kernels": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kernels.items()},
        "time_to_psnr": ttp,
        "batched": bat,
        "differentiation": diff,
        "paper_scenarios": scen,
        "oracle_detail": odet,
    }
    print(json.dumps(result), flush=True)
    return 0


def differentiation_section(torch, fbpnp, synth, tune_cache, reps=3, tune_only=False):
    """Reverse mode through 10 unrolled two-stage sketched iterations (5 at f = 2, then 5 at
    f = 1, FISTA momentum, all views) on a batch of 8 slices of 512^2 with 360 views x 768
    bins (seeded 20-ellipse phantoms, 1% Gaussian noise): the GPU time of the forward pass
    (which keeps one checkpoint per iteration) and of the backward pass (gradients with
    respect to the 8 initial images and the 10 step sizes), HIP events on the launch
    stream around each pass as the API issues it, median over reps after a warm-up."""
    from paper_2203_07308_amd.autograd import StepSpec, unrolled_pnp

    n, V, nb, S, n2, n1 = 512, 360, 768, 8, 5, 5
    gd = synth.fan_geometry(n, V, nb)
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [2, 1])
    # every iteration takes all views: launch configurations tuned for that view count
    plan.autotune(n_sel=V, cache_path=tune_cache)
    if tune_only:
        plan.close()
        return None
    xts = np.stack([synth.rasterise(synth.random_ellipses(6000 + s, 20, n), n) for s in range(S)]).astype(np.float32)
    xt_d = torch.from_numpy(xts).cuda()
    ax = torch.empty((S, V * nb), device="cuda")
    for s in range(S):
        fbpnp.fanbeam_fp(plan, 1, xt_d[s].reshape(-1), ax[s])
    ax_h = ax.cpu().numpy().astype(np.float64)
    b_h = np.stack([synth.add_noise(ax_h[s], synth.standard_normal(6100 + s, ax_h[s].shape), "gaussian", 0.01)
                    for s in range(S)]).astype(np.float32)
    b = torch.from_numpy(b_h).cuda()
    eta_k = [1.0 / fbpnp.power_lipschitz(plan, k, 100) for k in range(2)]
    a = synth.momentum_table(n2 + n1)
    specs = [StepSpec(0 if t < n2 else 1, a_t=float(a[t])) for t in range(n2 + n1)]
    eta0 = torch.tensor([eta_k[0]] * n2 + [eta_k[1]] * n1, dtype=torch.float32, device="cuda")
    x00 = (0.5 * xt_d + 0.05 * torch.from_numpy(np.random.default_rng(6200).random((S, n, n)).astype(np.float32))
           .cuda()).contiguous()
    fw, bw = [], []
    for r in range(reps + 1):
        x0 = x00.clone().requires_grad_(True)
        eta = eta0.clone().requires_grad_(True)
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        torch.cuda.synchronize()
        e[0].record()
        out = unrolled_pnp(plan, b, specs, x0, eta)
        e[1].record()
        loss = 0.5 * ((out - xt_d) ** 2).sum()
        e[2].record()
        loss.backward()
        e[3].record()
        torch.cuda.synchronize()
        if r:
            fw.append(e[0].elapsed_time(e[1]))
            bw.append(e[2].elapsed_time(e[3]))
    fms, bms = float(np.median(fw)), float(np.median(bw))
    ok = bool(torch.isfinite(x0.grad).all()) and bool(torch.isfinite(eta.grad).all())
    res = {"workload": "8 slices x 512^2, 360 views x 768 bins, 10 unrolled iterations (5 at f = 2, 5 at f = 1), "
                       "all views, FISTA momentum, TV-prox 5 x lambda 0.01; loss 0.5 ||x_10 - x_true||^2",
           "forward_ms": round(fms, 3), "backward_ms": round(bms, 3),
           "backward_over_forward": round(bms / fms, 2),
           "slice_iterations_per_s_forward": round(S * (n2 + n1) / (fms * 1e-3), 1),
           "slice_iterations_per_s_forward_and_backward": round(S * (n2 + n1) / ((fms + bms) * 1e-3), 1),
           "gradients_finite": ok}
    log(f"differentiation: {res}")
    plan.close()
    return res


def time_to_psnr(torch, fbpnp, synth, w, plan, stage_of, schedule, make_steps, x, y, xt, T, tune_cache):
    """Per-iteration PSNR (from an iterate history) against cumulative GPU time, for the
    sketched schedule (minibatch and variance-reduced gradients), full-gradient PnP-FISTA
    and full-resolution PnP-SGD. Each iteration's time comes from its step's clock stamp
    (the device clock when its denoiser kernel finished) against the previous one, over
    five replays of the method's stage graphs from the same start state (median per
    iteration); the first iteration starts at a clock mark written just before them."""
    N = w.n
    npix = N * N
    ref = torch.from_numpy(xt).cuda().reshape(1, -1).double()
    peak = float(xt.max() - xt.min())

    V, B = w.n_views, w.n_bins
    snaps = {f: (torch.zeros(V * B, device="cuda"), torch.zeros((N // f) ** 2, device="cuda"))
             for f, _ in w.stages}

    def run(stages, n_sub_used, seed, t_offset=0, x_init=None, vr=False, vr_epoch=None):
        # each method runs with the launch configurations tuned for its view count
        plan.autotune(n_sel=w.n_views // n_sub_used if n_sub_used else w.n_views, cache_path=tune_cache)
        sched = schedule(stages, seed, n_sub_used, True, t_offset)
        hist = torch.empty((len(sched), npix), device="cuda")
        stage_blocks = []
        t = 0
        for f, n in stages:
            stage_blocks.append((t, t + n))
            t += n
        # variance reduction: an epoch of vr_epoch iterations (default n_sub) opens with a
        # full-view snapshot step; vr_epoch 0: one snapshot at each stage start only
        ep = n_sub_used if vr_epoch is None else vr_epoch
        modes = [1 if (i == a if ep == 0 else (i - a) % ep == 0) else 2
                 for a, bnd in stage_blocks for i in range(a, bnd)] if vr else None
        stamps = torch.zeros(len(sched) + 1, dtype=torch.int64, device="cuda")
        graphs = [fbpnp.Graph(plan, make_steps(sched[a:b], hist[a:b], None, None if modes is None else modes[a:b],
                                               snaps, stamps[a + 1:b + 1])) for a, b in stage_blocks]
        if x_init is None:
            x.zero_()
            y.zero_()
        else:
            x.copy_(x_init[0])
            y.copy_(x_init[1])
        state0 = (x.clone(), y.clone())
        for g in graphs:
            g.launch()
        torch.cuda.synchronize()
        psnr = (10 * torch.log10(peak ** 2 / ((hist.double() - ref) ** 2).mean(dim=1))).cpu().numpy()
        final = (x.clone(), y.clone())
        # timing: the stage graphs replayed back to back 5 times from the same start
        # state; per-iteration times from the step stamps (device clock, khz ticks/ms)
        khz = fbpnp.clock_khz()
        if khz <= 0:
            raise RuntimeError("time-to-PSNR: the device clock rate is unknown")
        reps = []
        for _ in range(5):
            x.copy_(state0[0])
            y.copy_(state0[1])
            stamps.zero_()
            fbpnp.clock_stamp(stamps[0:1])
            for g in graphs:
                g.launch()
            torch.cuda.synchronize()
            reps.append(np.diff(stamps.cpu().numpy().astype(np.float64)) / khz)
        per_iter = np.median(np.stack(reps), axis=0)
        if not (per_iter > 0).all():
            raise RuntimeError("time-to-PSNR: a step stamp is missing or out of order")
        cum = np.cumsum(per_iter)
        for g in graphs:
            g.close()
        return psnr, cum, final

    seed = 3000 * w.seed_base
    ps_full, t_full, _ = run([(1, T)], 0, seed)
    ps_sgd, t_sgd, _ = run([(1, T)], w.n_subsets, seed + 1)
    ps_sk, t_sk, fin = run(w.stages, w.n_subsets, seed)
    ps_vr, t_vr, _ = run(w.stages, w.n_subsets, seed, vr=True)
    ps_vr0, t_vr0, _ = run(w.stages, w.n_subsets, seed, vr=True, vr_epoch=0)
    # extend the sketched run's final stage (same subset stream rule) up to 240 iterations
    ext_p, ext_t = [ps_sk], [t_sk]
    p_star = float(ps_full[-1])
    done = T
    while np.concatenate(ext_p).max() < p_star and done < 240:
        p2, t2, fin = run([(1, 20)], w.n_subsets, seed + done, t_offset=done, x_init=fin)
        ext_p.append(p2)
        ext_t.append(t2 + ext_t[-1][-1])
        done += 20
    ps_sk_all, t_sk_all = np.concatenate(ext_p), np.concatenate(ext_t)

    def first_time(ps, ts, target):
        idx = np.nonzero(ps >= target)[0]
        return None if len(idx) == 0 else round(float(ts[idx[0]]), 4)

    out = {"p_star_db": round(p_star, 3), "definition": "P* = PSNR of full-gradient PnP-FISTA after 60 iterations"}
    for name, ps, ts in (("sketched_ms2g", ps_sk_all, t_sk_all), ("sketched_ms2g_svrg", ps_vr, t_vr),
                         ("sketched_ms2g_svrg_stage_snapshots", ps_vr0, t_vr0),
                         ("full_pnp_fista", ps_full, t_full), ("full_res_pnp_sgd", ps_sgd, t_sgd)):
        out[name] = {
            "iterations": int(len(ps)), "final_psnr_db": round(float(ps[-1]), 3),
            "max_psnr_db": round(float(ps.max()), 3), "total_ms": round(float(ts[-1]), 4),
            "ms_to_p_star": first_time(ps, ts, p_star),
            "ms_to_p_star_minus_0.1": first_time(ps, ts, p_star - 0.1),
            "ms_to_p_star_minus_0.5": first_time(ps, ts, p_star - 0.5),
            "psnr_curve_every_5": [round(float(v), 2) for v in ps[4::5]],
        }
    a, bb = out["sketched_ms2g"]["ms_to_p_star_minus_0.1"], out["full_pnp_fista"]["ms_to_p_star_minus_0.1"]
    out["speedup_to_p_star_minus_0.1"] = None if (a is None or bb is None) else round(bb / a, 3)
    log(f"time-to-PSNR: {out}")
    return out


def batched_section(torch, fbpnp, synth, steps, tune_cache, tune_only=False):
    """The batched form on its own workload: 64 independent slices of uneven sizes and
    view counts, a two-stage sketched schedule (30 iterations at f = 2, 20 at f = 1, all
    views, FISTA momentum), launch configurations from the autotuner, the 50 iterations
    captured as one graph. Compared with the same slices reconstructed one after another
    through per-slice graphs of pnp_step (default configurations)."""
    bw = synth.BATCH_WORKLOADS["batch64"]
    shapes = bw.shapes()
    factors = [f for f, _ in bw.stages]
    t0 = time.time()
    gds = [synth.fan_geometry(n, V) for n, V in shapes]
    batch = fbpnp.Batch([fbpnp.Geometry(**g) for g in gds], factors)
    n = len(gds)
    s_full = factors.index(1)
    b_arena = torch.zeros(batch.sino_size, device="cuda")
    eta = np.zeros((len(factors), n), dtype=np.float32)
    samples = {f: 0 for f in factors}
    for i, g in enumerate(gds):
        sw = bw.slice_workload(i)
        plan = batch.slice_plan(i)
        xt = torch.from_numpy(synth.phantom(sw, i)).cuda().reshape(-1)
        ax = torch.empty(g["n_views"] * g["n_bins"], device="cuda")
        fbpnp.fanbeam_fp(plan, s_full, xt, ax)
        eps = synth.standard_normal(synth.noise_seed(sw, i), (g["n_views"], g["n_bins"]))
        bi = synth.add_noise(ax.cpu().numpy().astype(np.float64).reshape(eps.shape), eps, sw.noise_kind,
                             sw.noise_level).astype(np.float32)
        batch.sinogram(b_arena, i).copy_(torch.from_numpy(bi))
        for k, f in enumerate(factors):
            eta[k, i] = 1.0 / fbpnp.power_lipschitz(plan, k, 50)
            samples[f] += plan.stage_info(k).samples_all_views
    t_setup = time.time() - t0
    t0 = time.time()
    batch.autotune(1, tune_cache)
    t_tune = time.time() - t0
    if tune_only:
        batch.close()
        return None
    cfgs = {f"f{f}": batch.get_config(k, 1) for k, f in enumerate(factors)}
    log(f"batch: setup {t_setup:.1f}s, autotune {t_tune:.1f}s, configs {cfgs}")
    eta_d = [torch.from_numpy(eta[k]).cuda() for k in range(len(factors))]
    T = sum(it for _, it in bw.stages)
    a = synth.momentum_table(T, bw.momentum)
    stage_t = [k for k, (_, it) in enumerate(bw.stages) for _ in range(it)]
    x = torch.zeros(batch.image_size, device="cuda")
    y = torch.zeros(batch.image_size, device="cuda")

    def args_for(events=None):
        return [fbpnp.batch_args(batch, stage_t[t], b_arena, y, x, x, y, eta_d[stage_t[t]], float(a[t]),
                                 alpha=bw.alpha, lam=bw.lam, tau=bw.tau, tv_iters=bw.tv_iters,
                                 events=None if events is None else events[t]) for t in range(T)]

    graph = fbpnp.BatchGraph(batch, args_for())

    def run(g):
        x.zero_()
        y.zero_()
        g.launch()

    run(graph)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        run(graph)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # per-kernel durations (direct calls, start/stop events per kernel)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(T)]
    direct = args_for(evs)
    fbpnp.chain_steps(direct)
    x.zero_()
    y.zero_()
    for st in direct:
        fbpnp.pnp_step_batched(batch, st)
    torch.cuda.synchronize()
    kern = {}
    for t in range(T):
        f = factors[stage_t[t]]
        for k, name in ((0, "fp"), (2, "bp"), (4, "tv")):
            kern.setdefault(f"{name}_f{f}", []).append(evs[t][k].elapsed_time(evs[t][k + 1]))
    kernels = {}
    for key, v in kern.items():
        avg_ms = float(np.mean(v))
        d = {"avg_launch_us": round(avg_ms * 1e3, 3), "launches_per_step": len(v)}
        if not key.startswith("tv"):
            smp = samples[int(key.split("_f")[1])]
            d["gsamples_per_s"] = round(smp / (avg_ms * 1e-3) / 1e9, 2)
        kernels[key] = d
    # the same slices one after another (one graph per slice)
    singles = []
    for i, g in enumerate(gds):
        plan = batch.slice_plan(i)
        xi, yi = batch.image(x, i).reshape(-1), batch.image(y, i).reshape(-1)
        bi = batch.sinogram(b_arena, i).reshape(-1)
        st = [fbpnp.pnp_args(plan, stage_t[t], bi, yi, xi, xi, yi, float(eta[stage_t[t], i]), float(a[t]),
                             alpha=bw.alpha, lam=bw.lam, tau=bw.tau, tv_iters=bw.tv_iters) for t in range(T)]
        singles.append(fbpnp.Graph(plan, st))
    for gi in singles:
        gi.launch()
    torch.cuda.synchronize()
    e0.record()
    for gi in singles:
        gi.launch()
    e1.record()
    e1.synchronize()
    ms_single = e0.elapsed_time(e1)
    for gi in singles:
        gi.close()
    graph.close()
    out = {
        "workload": f"batch64: {n} slices, widths {sorted(set(s for s, _ in shapes))}, views "
                    f"{sorted(set(v for _, v in shapes))}, bins 1.5 x width, stages f=2 x 30 then f=1 x 20, "
                    "all views, TV-prox 5 x lambda 0.01, FISTA momentum",
        "slice_iterations_per_s": round(n * T / (ms * 1e-3), 1),
        "ms_per_batch_reconstruction": round(ms, 3),
        "samples_per_full_res_projection": int(samples[1]),
        "one_slice_at_a_time_ms": round(ms_single, 3),
        "speedup_vs_one_slice_at_a_time": round(ms_single / ms, 3),
        "configs": cfgs,
        "kernels": kernels,
        "autotune_s": round(t_tune, 2),
    }
    log(f"batch: {out}")
    batch.close()
    return out


def psnr_vs_time(torch, fbpnp, plan, stage_of, b, xt, blocks, eta, alpha, lam, tau, tv_iters, reps=5):
    """Runs consecutive stage blocks [(f, iterations)] from x = y = 0 with FISTA momentum
    (t global), one captured graph per block with an iterate history; returns per-iteration
    PSNR against xt and cumulative GPU time (the graphs replayed back to back `reps` times
    from the same start, each iteration's time from its step's clock stamp against the
    previous one, the median per iteration)."""
    from paper_2203_07308_amd import synth

    ny, nx = xt.shape
    npix = nx * ny
    T = sum(n for _, n in blocks)
    a = synth.momentum_table(T)
    x = torch.zeros(npix, device="cuda")
    y = torch.zeros(npix, device="cuda")
    hist = torch.empty((T, npix), device="cuda")
    stamps = torch.zeros(T + 1, dtype=torch.int64, device="cuda")
    graphs, t = [], 0
    for f, n in blocks:
        steps = [fbpnp.pnp_args(plan, stage_of[f], b, y, x, x, y, eta[f], float(a[t + i]), None, 1.0, alpha, lam, tau,
                                tv_iters, hist[t + i], stamp=stamps[t + i + 1:t + i + 2]) for i in range(n)]
        graphs.append(fbpnp.Graph(plan, steps))
        t += n
    for g in graphs:
        g.launch()
    torch.cuda.synchronize()
    ref = torch.from_numpy(xt).cuda().reshape(1, -1).double()
    peak = float(xt.max() - xt.min())
    psnr = (10 * torch.log10(peak ** 2 / ((hist.double() - ref) ** 2).mean(dim=1))).cpu().numpy()
    khz = fbpnp.clock_khz()
    if khz <= 0:
        raise RuntimeError("psnr_vs_time: the device clock rate is unknown")
    runs = []
    for _ in range(reps):
        x.zero_()
        y.zero_()
        stamps.zero_()
        fbpnp.clock_stamp(stamps[0:1])
        for g in graphs:
            g.launch()
        torch.cuda.synchronize()
        runs.append(np.diff(stamps.cpu().numpy().astype(np.float64)) / khz)
    for g in graphs:
        g.close()
    per_iter = np.median(np.stack(runs), axis=0)
    if not (per_iter > 0).all():
        raise RuntimeError("psnr_vs_time: a step stamp is missing or out of order")
    return psnr, np.cumsum(per_iter)


def paper_scenarios(torch, fbpnp, synth, tune_cache):
    """The paper's experiments (Sec. 3) on synthetic disk phantoms: sparse-view, low-dose
    and limited-angle fan-beam CT at 256^2 with 228 bins and Poisson transmission data;
    PnP-MS2G Option 1 with the two-stage sketch (25 iterations at f = 4, 75 at f = 2;
    average pooling and, as in the paper, bicubic resizing) against PnP-FISTA (100
    full-gradient iterations), same TV-prox denoiser, eta = 1/L per
    stage, FISTA momentum. Reports each method's PSNR curve, and the GPU time and the
    projector work (Joseph samples of forward and back-projection) each needs to come
    within 0.1 / 0.5 / 1 dB of PnP-FISTA's final PSNR."""
    out = {}
    for name, sc in synth.SCENARIOS.items():
        g = sc.geometry
        V, B = g["n_views"], g["n_bins"]
        factors = [4, 2, 1]
        stage_of = {f: i for i, f in enumerate(factors)}
        plan = fbpnp.Plan(fbpnp.Geometry(**g), factors)
        plan.autotune(n_sel=V, cache_path=tune_cache)
        xt = sc.phantom()
        ax = torch.empty(V * B, device="cuda")
        fbpnp.fanbeam_fp(plan, stage_of[1], torch.from_numpy(xt).cuda().reshape(-1), ax)
        b_np = sc.data(ax.cpu().numpy().astype(np.float64).reshape(V, B)).astype(np.float32)
        b = torch.from_numpy(b_np).cuda().reshape(-1)
        eta = {f: 1.0 / fbpnp.power_lipschitz(plan, stage_of[f], 100) for f in factors}
        kw = dict(alpha=sc.alpha, lam=sc.lam, tau=sc.tau, tv_iters=sc.tv_iters)
        ps_sk, t_sk = psnr_vs_time(torch, fbpnp, plan, stage_of, b, xt, list(sc.stages), eta, **kw)
        ps_fu, t_fu = psnr_vs_time(torch, fbpnp, plan, stage_of, b, xt, [(1, sc.full_iters)], eta, **kw)
        # the paper's own sketch operator: bicubic S with U = S^T (its own step sizes 1/L)
        plan.set_sketch("bicubic")
        eta_b = {f: 1.0 / fbpnp.power_lipschitz(plan, stage_of[f], 100) for f in factors}
        ps_bi, t_bi = psnr_vs_time(torch, fbpnp, plan, stage_of, b, xt, list(sc.stages), eta_b, **kw)
        plan.set_sketch("pool")
        p_ref = float(ps_fu[-1])

        def first(ps, ts, target):
            idx = np.nonzero(ps >= target)[0]
            return None if len(idx) == 0 else round(float(ts[idx[0]]), 4)

        # projector work per iteration: forward and matched back-projection, every view
        work = {f: 2e-9 * plan.stage_info(stage_of[f]).samples_all_views for f in factors}
        w_sk = np.cumsum([work[f] for f, n in sc.stages for _ in range(n)])
        w_fu = np.cumsum([work[1]] * sc.full_iters)
        res = {"views": V, "bins": B, "angle_range_deg": round(float(np.degrees(sc.angle_range)), 1), "i0": sc.i0,
               "pnp_fista_final_psnr_db": round(p_ref, 3)}
        for key, ps, ts, ws in (("ms2g_two_stage", ps_sk, t_sk, w_sk), ("ms2g_two_stage_bicubic", ps_bi, t_bi, w_sk),
                                ("pnp_fista", ps_fu, t_fu, w_fu)):
            res[key] = {"iterations": int(len(ps)), "final_psnr_db": round(float(ps[-1]), 3),
                        "max_psnr_db": round(float(ps.max()), 3), "total_ms": round(float(ts[-1]), 4),
                        **{f"ms_to_ref_minus_{d}": first(ps, ts, p_ref - d) for d in (0.1, 0.5, 1.0)},
                        **{f"gsamples_to_ref_minus_{d}": first(ps, ws, p_ref - d) for d in (0.1, 0.5, 1.0)},
                        "psnr_curve_every_10": [round(float(v), 2) for v in ps[9::10]]}
        for d in (0.1, 0.5, 1.0):
            for unit, tag in (("ms", "speedup"), ("gsamples", "work_ratio")):
                for key, suffix in (("ms2g_two_stage", ""), ("ms2g_two_stage_bicubic", "_bicubic")):
                    a_ = res[key][f"{unit}_to_ref_minus_{d}"]
                    b_ = res["pnp_fista"][f"{unit}_to_ref_minus_{d}"]
                    res[f"{tag}{suffix}_to_ref_minus_{d}"] = None if (a_ is None or b_ is None) else round(b_ / a_, 3)
        out[name] = res
        log(f"scenario {name}: {res}")
        plan.close()
    return out


def cpu_baseline(synth, w, xt, sk_sched, eta, n_sub, budget_s=10.0):
    """The FP64 oracle (as is) on the host cores, on a bounded sample of the same
    schedule: whole 60-iteration sketched reconstructions from x = 0, repeated until
    about budget_s seconds have passed, on its own b = A x + noise (computed by the
    oracle, untimed)."""
    import oracle

    oracle.build(force=False)
    gd = w.geometry
    og = oracle.Geometry(**gd)
    V = gd["n_views"]
    ax = oracle.fp(og, xt.astype(np.float64))
    b = synth.add_noise(ax, synth.standard_normal(synth.noise_seed(w), ax.shape), w.noise_kind,
                        w.noise_level).astype(np.float32).astype(np.float64)
    sched = [(f, synth.subset_views(s, n_sub, V), float(n_sub)) for f, s, _ in sk_sched]
    et = np.array([eta[f] for f, _, _ in sk_sched])
    a = np.array([a_t for _, _, a_t in sk_sched])
    runs = 0
    t0 = time.time()
    while True:
        oracle.pnp_run(og, b, sched, et, a, w.alpha, w.lam, w.tv_iters, w.tau)
        runs += 1
        dt = time.time() - t0
        if dt >= budget_s or runs >= 50:
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = min(cores, os.cpu_count() or cores)
    iters = runs * len(sched)
    log(f"oracle: {iters} iterations in {dt:.2f}s on {cores} threads")
    return {"value": round(iters / dt, 4), "unit": "iter/s", "cores": cores, "kind": "oracle",
            "sample": f"{runs} complete {len(sched)}-iteration sketched reconstructions of the same workload "
                      f"(FP64 C oracle, OpenMP), {dt:.2f} s"}


def copy_rate(torch, mib=512, reps=10):
    """Device-to-device copy bandwidth (bytes read + bytes written per second, GB/s), median of reps."""
    src = torch.ones(mib << 18, device="cuda")
    dst = torch.empty_like(src)
    ms = _gpu_ms(torch, lambda: dst.copy_(src), reps)
    return 2 * src.numel() * 4 / (ms * 1e-3) / 1e9


def _gpu_ms(torch, fn, reps):
    """Median over reps of one call's duration on the current stream (HIP events), after a warm-up call."""
    fn()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times))


def oracle_detail(torch, fbpnp, synth, plan, s_full, xt, tune_cache):
    """The FP64 oracle beside the GPU, on all host threads and on one: full-view forward
    and back projection of the three workload geometries (64^2, 256^2, 512^2) on their
    f = 1, 2 and 4 grids (one call each; the GPU with its default launch configuration),
    and the complete 64^2 PnP-ISTA and 256^2 two-stage reconstructions (all host threads)."""
    import oracle

    oracle.build(force=False)
    n_all = oracle.set_threads(0)
    out = {"threads_all": n_all, "projectors": {}}
    for name in ("pnp64", "ms2g256", "ms2g512"):
        wl = synth.WORKLOADS[name]
        g2 = wl.geometry
        og2 = oracle.Geometry(**g2)
        V2, B2 = g2["n_views"], g2["n_bins"]
        pl = fbpnp.Plan(fbpnp.Geometry(**g2), [1, 2, 4])
        xt2 = synth.phantom(wl) if name != "ms2g512" else xt
        y64 = np.random.default_rng(17).random((V2, B2))
        yd = torch.from_numpy(y64.astype(np.float32)).cuda().reshape(-1)
        ybuf = torch.empty(V2 * B2, device="cuda")
        entry = {}
        for k, f in enumerate((1, 2, 4)):
            ny, nx = g2["ny"] // f, g2["nx"] // f
            xs = np.asarray(xt2, dtype=np.float64).reshape(ny, f, nx, f).mean(axis=(1, 3))
            xd = torch.from_numpy(xs.astype(np.float32)).cuda().reshape(-1)
            xbuf = torch.empty(nx * ny, device="cuda")
            smp = int(np.sum(pl.view_samples(k)))
            d = {"grid": nx, "samples": smp,
                 "gpu_fp_ms": round(_gpu_ms(torch, lambda: fbpnp.fanbeam_fp(pl, k, xd, ybuf), 20), 4),
                 "gpu_bp_ms": round(_gpu_ms(torch, lambda: fbpnp.fanbeam_bp(pl, k, yd, xbuf), 20), 4)}
            for op, fn in (("fp", lambda: oracle.fp(og2, xs, f)), ("bp", lambda: oracle.bp(og2, y64, f))):
                for th in (n_all, 1):
                    oracle.set_threads(th)
                    t0 = time.time()
                    fn()
                    dt = time.time() - t0
                    d[f"oracle_{op}_s_{th}_threads"] = round(dt, 4)
                    d[f"oracle_{op}_gsamples_per_s_{th}_threads"] = round(smp / dt / 1e9, 4)
                oracle.set_threads(n_all)
            entry[f"f{f}"] = d
        pl.close()
        out["projectors"][name] = entry
    log(f"oracle projectors: {out['projectors']}")
    # whole reconstructions of the two smaller workloads: GPU graph replay against the oracle
    loops = {}
    for name in ("pnp64", "ms2g256"):
        wl = synth.WORKLOADS[name]
        g2 = wl.geometry
        fs = [f for f, _ in wl.stages]
        pl = fbpnp.Plan(fbpnp.Geometry(**g2), fs)
        pl.autotune(n_sel=g2["n_views"], cache_path=tune_cache)
        V2, B2, n2 = g2["n_views"], g2["n_bins"], g2["nx"] * g2["ny"]
        xt2 = synth.phantom(wl)
        ax = torch.empty(V2 * B2, device="cuda")
        fbpnp.fanbeam_fp(pl, fs.index(1), torch.from_numpy(xt2).cuda().reshape(-1), ax)
        eps = synth.standard_normal(synth.noise_seed(wl), (V2, B2))
        b_np = synth.add_noise(ax.cpu().numpy().astype(np.float64).reshape(V2, B2), eps, wl.noise_kind,
                               wl.noise_level).astype(np.float32)
        bd = torch.from_numpy(b_np).cuda().reshape(-1)
        eta2 = {f: 1.0 / fbpnp.power_lipschitz(pl, k, 100) for k, f in enumerate(fs)}
        T2 = wl.n_iters
        a2 = synth.momentum_table(T2, wl.momentum)
        sched = [(k, f) for k, (f, n) in enumerate(wl.stages) for _ in range(n)]
        x2 = torch.zeros(n2, device="cuda")
        y2 = torch.zeros(n2, device="cuda")
        steps = [fbpnp.pnp_args(pl, k, bd, y2, x2, x2, y2, eta2[f], float(a2[t]), None, 1.0, wl.alpha, wl.lam,
                                wl.tau, wl.tv_iters) for t, (k, f) in enumerate(sched)]
        graph = fbpnp.Graph(pl, steps)

        def replay():
            x2.zero_()
            y2.zero_()
            graph.launch()

        gms = _gpu_ms(torch, replay, 5)
        t0 = time.time()
        oracle.pnp_run(oracle.Geometry(**g2), b_np.astype(np.float64), [(f, None, 1.0) for _, f in sched],
                       np.array([eta2[f] for _, f in sched]), np.asarray(a2, dtype=np.float64), wl.alpha, wl.lam,
                       wl.tv_iters, wl.tau)
        ods = time.time() - t0
        loops[name] = {"iterations": T2, "gpu_ms": round(gms, 4), "oracle_s": round(ods, 4),
                       "oracle_threads": n_all, "gpu_over_oracle": round(ods / (gms * 1e-3), 1)}
        graph.close()
    out["loops"] = loops
    log(f"oracle loops: {loops}")
    return out


if __name__ == "__main__":
    sys.exit(main())
