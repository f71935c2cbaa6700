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
PEAK_FP32_TFLOPS = 157.3
# algorithmic FP32 operations per unit of work
FLOP_PER_FP_SAMPLE = 7      # position fma (2), fraction (1), interpolation sub+fma (3), accumulate (1)
FLOP_PER_BP_SAMPLE = 8      # position fma (2), fraction (1), 1-w (1), two weighted fma (4)
FLOP_PER_TV_PIXEL_ITER = 20
FLOP_PER_TV_PIXEL_OUT = 8


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the FP64 oracle timing")
    ap.add_argument("--no-ttp", action="store_true", help="skip the time-to-PSNR comparison")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--profile", action="store_true",
                    help="short run for hardware-counter passes: two replays of the sketched schedule "
                         "and a 64 MiB device copy (counter calibration); prints no JSON line")
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


def main() -> int:
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        return 2
    import torch

    from paper_2203_07308_amd import fbpnp, synth

    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    torch.cuda.set_device(0)
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
    subsets = [torch.from_numpy(synth.subset_views(s, n_sub, V)).cuda() for s in range(n_sub)]
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

    def make_steps(sched, hist=None):
        steps = []
        for t, (f, s, a_t) in enumerate(sched):
            views = None if s is None else subsets[s]
            sigma = 1.0 if s is None else float(n_sub)
            steps.append(fbpnp.pnp_args(plan, stage_of[f], b, y, x, x, y, eta[f], a_t, views, sigma, w.alpha, w.lam,
                                        w.tau, w.tv_iters, None if hist is None else hist[t]))
        return steps

    sk_sched = schedule(w.stages, 3000 * w.seed_base, n_sub)
    T = len(sk_sched)
    graph = fbpnp.Graph(plan, make_steps(sk_sched))

    def run_once(g):
        x.zero_()
        y.zero_()
        g.launch()

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

    # ---- per-kernel timings (standalone entry points, same stream, back-to-back launches)
    kernels = {}
    reps = args.kernel_reps
    sub0 = subsets[0]
    n_sel = sub0.numel()
    samples = {f: plan.stage_info(stage_of[f]).samples_all_views for f in factors}
    sino = torch.empty(V * B, device="cuda")
    for f in factors:
        s = stage_of[f]
        ns = (N // f) ** 2
        v = torch.rand(ns, device="cuda")
        r = torch.rand(n_sel * B, device="cuda")
        out = torch.empty(ns, device="cuda")
        for name, call in (("fp", lambda: fbpnp.fanbeam_fp(plan, s, v, sino[: n_sel * B], sub0)),
                           ("bp", lambda: fbpnp.fanbeam_bp(plan, s, r, out, sub0))):
            call()
            torch.cuda.synchronize()
            with Events(torch) as ev:
                for _ in range(reps):
                    call()
            per = ev.ms / reps
            smp = samples[f] * n_sel / V  # one subset of interleaved views: V/n_sub of the views
            flop = smp * (FLOP_PER_FP_SAMPLE if name == "fp" else FLOP_PER_BP_SAMPLE)
            kernels[f"{name}_f{f}_subset"] = dict(ms=per, samples=smp, gups=smp / (per * 1e-3) / 1e9,
                                                   tflops=flop / (per * 1e-3) / 1e12, launches_per_step=20)
    zz = torch.rand(npix, device="cuda")
    xo = torch.empty(npix, device="cuda")
    fbpnp.tv_prox(zz.reshape(N, N), xo.reshape(N, N), w.lam, w.tv_iters, w.tau)
    torch.cuda.synchronize()
    with Events(torch) as ev:
        for _ in range(reps):
            fbpnp.tv_prox(zz.reshape(N, N), xo.reshape(N, N), w.lam, w.tv_iters, w.tau)
    per = ev.ms / reps
    tv_flop = npix * (w.tv_iters * FLOP_PER_TV_PIXEL_ITER + FLOP_PER_TV_PIXEL_OUT)
    kernels["tv_512"] = dict(ms=per, tflops=tv_flop / (per * 1e-3) / 1e12, launches_per_step=T)
    # full-resolution, all-view projector GUPS (the full-gradient comparator's operator)
    vfull = torch.rand(npix, device="cuda")
    rfull = torch.rand(V * B, device="cuda")
    for name, call in (("fp", lambda: fbpnp.fanbeam_fp(plan, s_full, vfull, sino)),
                       ("bp", lambda: fbpnp.fanbeam_bp(plan, s_full, rfull, xo))):
        call()
        torch.cuda.synchronize()
        with Events(torch) as ev:
            for _ in range(reps):
                call()
        per = ev.ms / reps
        smp = samples[1]
        kernels[f"{name}_f1_allviews"] = dict(ms=per, samples=smp, gups=smp / (per * 1e-3) / 1e9,
                                              conventional_gups=V * npix / (per * 1e-3) / 1e9,
                                              launches_per_step=0)
    for k, v in kernels.items():
        log(f"  {k}: {v}")
    dom_name, dom = max(((k, v) for k, v in kernels.items() if v["launches_per_step"] > 0),
                        key=lambda kv: kv[1]["ms"] * kv[1]["launches_per_step"])
    roofline = {"kernel": dom_name, "bound": "alu", "achieved": round(dom["tflops"], 4),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(dom["tflops"] / PEAK_FP32_TFLOPS, 5),
                "traffic": None, "avg_launch_ms": round(dom["ms"], 5)}

    # ---- time-to-PSNR: sketched vs full-gradient PnP-FISTA vs full-resolution PnP-SGD
    ttp = None
    if not args.no_ttp:
        ttp = time_to_psnr(torch, fbpnp, synth, w, plan, stage_of, schedule, make_steps, x, y, xt, T)

    # ---- FP64 oracle on host cores (bounded sample of the same schedule)
    cpu = None if args.no_cpu_baseline else cpu_baseline(synth, w, xt, sk_sched, eta, n_sub)

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
        "cpu_baseline": cpu,
        "kernels": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kernels.items()},
        "time_to_psnr": ttp,
    }
    print(json.dumps(result), flush=True)
    return 0


def time_to_psnr(torch, fbpnp, synth, w, plan, stage_of, schedule, make_steps, x, y, xt, T):
    """Per-iteration PSNR (from an iterate history) against cumulative GPU time, for the
    sketched schedule, full-gradient PnP-FISTA and full-resolution PnP-SGD."""
    N = w.n
    npix = N * N
    ref = torch.from_numpy(xt).cuda().reshape(1, -1).double()
    peak = float(xt.max() - xt.min())

    def run(stages, n_sub_used, seed, t_offset=0, x_init=None):
        sched = schedule(stages, seed, n_sub_used, True, t_offset)
        hist = torch.empty((len(sched), npix), device="cuda")
        stage_blocks = []
        t = 0
        for f, n in stages:
            stage_blocks.append((t, t + n))
            t += n
        graphs = [fbpnp.Graph(plan, make_steps(sched[a:b], hist[a:b])) for a, b in stage_blocks]
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
        # timing: each stage graph replayed 5 times from the same start state (work is data-independent)
        per_iter = []
        for (a, bnd), g in zip(stage_blocks, graphs):
            times = []
            for _ in range(5):
                x.copy_(state0[0])
                y.copy_(state0[1])
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                g.launch()
                e1.record()
                e1.synchronize()
                times.append(e0.elapsed_time(e1))
            per_iter += [float(np.median(times)) / (bnd - a)] * (bnd - a)
        cum = np.cumsum(per_iter)
        for g in graphs:
            g.close()
        return psnr, cum, final

    seed = 3000 * w.seed_base
    ps_full, t_full, _ = run([(1, T)], 0, seed)
    ps_sgd, t_sgd, _ = run([(1, T)], w.n_subsets, seed + 1)
    ps_sk, t_sk, fin = run(w.stages, w.n_subsets, seed)
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
    for name, ps, ts in (("sketched_ms2g", ps_sk_all, t_sk_all), ("full_pnp_fista", ps_full, t_full),
                         ("full_res_pnp_sgd", ps_sgd, t_sgd)):
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


if __name__ == "__main__":
    sys.exit(main())
