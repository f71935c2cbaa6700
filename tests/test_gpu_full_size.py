"""GPU parity at the workloads' own sizes and schedules, in the launch shapes the benchmark
runs (the shipped autotuner cache), against the FP64 oracle:

  * the 512^2 multi-stage sketched PnP-SGD schedule (Algorithm 1, Option 2): 720 views x
    768 bins, 20 iterations each at f = 4, 2, 1, 1 of 8 interleaved view subsets drawn from
    the benchmark's seeded stream, per-stage steps 1 / L, FISTA momentum, all 60 iterations
    as one captured graph; and the same problem with every view per gradient, in the launch
    shapes tuned for all 720 views (f = 4, then f = 1);
  * the 64-slice batched workload (widths 128 to 512, 180 / 360 / 720 views, 1.5 x width
    bins, two-stage sketch) with its tuned batch configuration: every slice bitwise equal to
    the same slice run alone, and two slices (384^2 x 720 views, 512^2 x 360 views) against
    the oracle over 5 iterations per stage;
  * the paper's three 256^2 scan scenarios (Sec. 3) over their whole 25 + 75 two-stage
    schedule;
  * a 4096^2 grid, and the refusal of a grid past the 32-bit line-image offsets.

Reconstruction bar: relative L2 <= 1e-4 (the reconstruction tolerance of the path). The
oracle's step sizes for the two larger problems come from tests/golden/oracle_step_sizes.txt
(written by the oracle alone; 100 power iterations at 512^2 take minutes of host time).
"""
import math
import os
import shutil
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2203_07308_amd import fbpnp, synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SHIPPED_CACHE = os.path.join(ROOT, "paper_2203_07308_amd", "tuned", "mi355x_launch_configs.txt")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fbpnp.load()


def dev(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def oracle_lipschitz():
    """{(workload, factor): L} from the committed oracle step-size file."""
    out = {}
    with open(os.path.join(ROOT, "tests", "golden", "oracle_step_sizes.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].split()
            if line:
                out[(line[0], int(line[1]))] = float(line[2])
    return out


def tuned_cache(tmp_path):
    path = tmp_path / "launch_configs.txt"
    shutil.copyfile(SHIPPED_CACHE, path)
    return str(path)


def test_ms2g512_whole_schedule_as_benchmarked(tmp_path):
    w = synth.WORKLOADS["ms2g512"]
    gd = w.geometry
    og = oracle.Geometry(**gd)
    V, n_sub = gd["n_views"], w.n_subsets
    xt = synth.phantom(w)
    ax = oracle.fp(og, xt.astype(np.float64))
    b = synth.add_noise(ax, synth.standard_normal(synth.noise_seed(w), ax.shape), w.noise_kind,
                        w.noise_level).astype(np.float32)
    L = oracle_lipschitz()
    factors = [f for f, _ in w.stages]
    fs = [f for f, n in w.stages for _ in range(n)]
    T = len(fs)
    seq = synth.subset_sequence(3000 * w.seed_base, T, n_sub)  # the benchmark's subset stream
    eta = np.array([1.0 / L[("ms2g512", f)] for f in fs])
    a = synth.momentum_table(T, w.momentum)
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), factors)
    plan.autotune(n_sel=V // n_sub, cache_path=tuned_cache(tmp_path))
    say("ms2g512 whole schedule", [plan.get_config(k, V // n_sub) for k in range(len(factors))])
    npix = gd["nx"] * gd["ny"]
    bd = dev(b).reshape(-1)
    x = torch.zeros(npix, device="cuda")
    y = torch.zeros(npix, device="cuda")
    hist = torch.zeros((T, npix), device="cuda")
    steps = [fbpnp.pnp_args(plan, factors.index(fs[t]), bd, y, x, x, y, float(eta[t]), float(a[t]), None,
                            float(n_sub), w.alpha, w.lam, w.tau, w.tv_iters, hist[t],
                            subset=(int(seq[t]), n_sub)) for t in range(T)]
    g = fbpnp.Graph(plan, steps)
    g.launch()
    got, got_hist = host(x).reshape(gd["ny"], gd["nx"]), host(hist)
    g.close()
    sched_o = [(fs[t], synth.subset_views(int(seq[t]), n_sub, V), float(n_sub)) for t in range(T)]
    ref, ref_hist = oracle.pnp_run(og, b.astype(np.float64), sched_o, eta, a, w.alpha, w.lam, w.tv_iters, w.tau,
                                   history=True)
    errs = [rel(got_hist[t].reshape(ref.shape), ref_hist[t]) for t in range(T)]
    say("ms2g512 worst iterate error", max(errs), "final", rel(got, ref))
    assert rel(got, ref) <= 1e-4, rel(got, ref)
    assert max(errs) <= 1e-4, (int(np.argmax(errs)), max(errs))
    # the reconstruction improves on the data: the schedule does what it is for
    assert oracle.psnr(ref, xt) > 30.0


def test_ms2g512_all_views_in_the_tuned_launch_shapes(tmp_path):
    """The 512^2 problem with every view in each gradient (the full-gradient PnP-FISTA run of the
    time-to-PSNR comparison), in the launch shapes the shipped cache holds for 720 selected
    views: 3 iterations at f = 4, then 4 at f = 1, steps 1 / L, FISTA momentum, by direct
    pnp_step calls, each iterate against the oracle's."""
    w = synth.WORKLOADS["ms2g512"]
    gd = w.geometry
    og = oracle.Geometry(**gd)
    V = gd["n_views"]
    xt = synth.phantom(w)
    ax = oracle.fp(og, xt.astype(np.float64))
    b = synth.add_noise(ax, synth.standard_normal(synth.noise_seed(w), ax.shape), w.noise_kind,
                        w.noise_level).astype(np.float32)
    L = oracle_lipschitz()
    factors = [4, 1]
    fs = [4] * 3 + [1] * 4
    T = len(fs)
    eta = np.array([1.0 / L[("ms2g512", f)] for f in fs])
    a = synth.momentum_table(T, True)
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), factors)
    plan.autotune(n_sel=V, cache_path=tuned_cache(tmp_path))
    say("ms2g512 all views", [plan.get_config(k, V) for k in range(len(factors))])
    npix = gd["nx"] * gd["ny"]
    bd = dev(b).reshape(-1)
    x = torch.zeros(npix, device="cuda")
    y = torch.zeros(npix, device="cuda")
    hist = torch.zeros((T, npix), device="cuda")
    for t in range(T):
        fbpnp.pnp_step(plan, fbpnp.pnp_args(plan, factors.index(fs[t]), bd, y, x, x, y, float(eta[t]), float(a[t]),
                                            None, 1.0, w.alpha, w.lam, w.tau, w.tv_iters, hist[t]))
    got_hist = host(hist)
    sched_o = [(f, None, 1.0) for f in fs]
    ref, ref_hist = oracle.pnp_run(og, b.astype(np.float64), sched_o, eta, a, w.alpha, w.lam, w.tv_iters, w.tau,
                                   history=True)
    errs = [rel(got_hist[t].reshape(ref.shape), ref_hist[t]) for t in range(T)]
    say("ms2g512 all views, error per iterate", errs)
    assert max(errs) <= 1e-4, (int(np.argmax(errs)), max(errs))


def test_largest_grids():
    """A 4096^2 grid (6 views x 6144 bins, stages f = 8 and 1): each view's projection at both
    stages, the back-projection in the gather and scatter forms, and two fused steps (f = 8,
    then f = 1) against the oracle; and a grid whose two line images would need byte offsets
    beyond 32 bits is refused when the plan is created, before anything is launched."""
    n = 4096
    gd = synth.fan_geometry(n, 6, 6144)
    og = oracle.Geometry(**gd)
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [8, 1])
    c = (np.arange(n) - (n - 1) / 2) / n
    xt = ((c[None, :] ** 2 + c[:, None] ** 2 < 0.16) * (1.0 + 0.5 * c[None, :] - 0.3 * c[:, None])).astype(np.float32)
    rng = np.random.default_rng(17)
    for k, f in enumerate((8, 1)):
        xs = oracle.down(xt, f)
        ref = oracle.fp(og, xs, f)
        y = torch.empty(6 * gd["n_bins"], device="cuda")
        say("largest fp", f)
        fbpnp.fanbeam_fp(plan, k, dev(xs).reshape(-1), y)
        got = host(y).reshape(ref.shape)
        per_view = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
        assert per_view.max() <= 1e-5, (f, per_view.max())
        r = (rng.random(ref.shape) - 0.3).astype(np.float32)
        refb = oracle.bp(og, r.astype(np.float64), f, None, 1.0)
        # A sample's position p (|p| < n / 2f in centred pixels) is rounded to float once, so
        # its two weights carry an error of rms ulp(p) / sqrt(12), which a back-projected
        # pixel (a sum of a few samples) keeps, while a projection (a sum of thousands)
        # averages it down; the bar is three times that rms at the largest |p|, and 1e-5
        # below it (up to 512^2).
        tol_bp = max(1e-5, 3.0 * 2.0 ** (math.ceil(math.log2(n / (2 * f))) - 24) / math.sqrt(12.0))
        for form in (None, dict(fp_seg=0, bp_px=2, bp_vg=16, tv_tile=0), dict(fp_seg=0, bp_px=32, bp_vg=16, tv_tile=0)):
            plan.set_config(k, form)
            xb = torch.empty((n // f) * (n // f), device="cuda")
            say("largest bp", f, form)
            fbpnp.fanbeam_bp(plan, k, dev(r).reshape(-1), xb)
            err = rel(host(xb).reshape(refb.shape), refb)
            say("largest bp error", f, form, err, "bar", tol_bp)
            assert err <= tol_bp, (f, form, err, tol_bp)
        plan.set_config(k, None)
    b = oracle.fp(og, xt.astype(np.float64)).astype(np.float32)
    L = oracle.power_lipschitz(og, 8, 10)
    eta, a = np.array([1.0 / L, 1.0 / L]), synth.momentum_table(2, True)
    bd = dev(b).reshape(-1)
    x = torch.zeros(n * n, device="cuda")
    yv = torch.zeros(n * n, device="cuda")
    hist = torch.zeros((2, n * n), device="cuda")
    for t, k in enumerate((0, 1)):
        say("largest step", t)
        fbpnp.pnp_step(plan, fbpnp.pnp_args(plan, k, bd, yv, x, x, yv, float(eta[t]), float(a[t]), None, 1.0,
                                            1.0, 0.01, 0.125, 5, hist[t]))
    got = host(hist)
    _, ref_hist = oracle.pnp_run(og, b.astype(np.float64), [(8, None, 1.0), (1, None, 1.0)], eta, a, history=True)
    errs = [rel(got[t].reshape(n, n), ref_hist[t]) for t in range(2)]
    say("largest steps, error per iterate", errs)
    assert max(errs) <= 1e-4, errs
    # 2 x 23200 x 23204 floats of line images: byte offsets past 2^31
    too_big = synth.fan_geometry(23200, 1, 8)
    with pytest.raises(fbpnp.FbError) as e:
        fbpnp.Plan(fbpnp.Geometry(**too_big), [1])
    assert e.value.status == -1 and "32-bit" in str(e.value)


BATCH_ORACLE_SLICES = (3, 24)  # 384^2 x 720 views and 512^2 x 360 views


def test_batch64_real_shapes_tuned(tmp_path):
    bw = synth.BATCH_WORKLOADS["batch64"]
    shapes = bw.shapes()
    factors = [f for f, _ in bw.stages]
    gds = [synth.fan_geometry(n, V) for n, V in shapes]
    batch = fbpnp.Batch([fbpnp.Geometry(**g) for g in gds], factors)
    batch.autotune(1, tuned_cache(tmp_path))
    cfgs = [batch.get_config(k, 1) for k in range(len(factors))]
    say("batch64 configs", cfgs)
    L = oracle_lipschitz()
    b_arena = torch.zeros(batch.sino_size, device="cuda")
    eta = np.zeros((len(factors), len(gds)), dtype=np.float32)
    bs = {}
    for i, g in enumerate(gds):
        sw = bw.slice_workload(i)
        xt = synth.phantom(sw, i)
        eps = synth.standard_normal(synth.noise_seed(sw, i), (g["n_views"], g["n_bins"]))
        if i in BATCH_ORACLE_SLICES:
            ax = oracle.fp(oracle.Geometry(**g), xt.astype(np.float64))
            for k, f in enumerate(factors):
                eta[k, i] = 1.0 / L[(f"batch64[{i}]", f)]
        else:
            # slices compared only with their own single-slice runs: data and steps from the GPU
            plan = batch.slice_plan(i)
            axd = torch.empty(g["n_views"] * g["n_bins"], device="cuda")
            fbpnp.fanbeam_fp(plan, factors.index(1), dev(xt).reshape(-1), axd)
            ax = host(axd).reshape(eps.shape)
            for k in range(len(factors)):
                eta[k, i] = 1.0 / fbpnp.power_lipschitz(plan, k, 30)
        bs[i] = synth.add_noise(ax, eps, sw.noise_kind, sw.noise_level).astype(np.float32)
        batch.sinogram(b_arena, i).copy_(dev(bs[i]))
    n_it = 5
    stage_t = [0] * n_it + [1] * n_it
    T = len(stage_t)
    a = synth.momentum_table(T, bw.momentum)
    eta_d = [dev(eta[k]) for k in range(len(factors))]
    x = torch.zeros(batch.image_size, device="cuda")
    y = torch.zeros(batch.image_size, device="cuda")
    steps = [fbpnp.batch_args(batch, stage_t[t], b_arena, y, x, x, y, eta_d[stage_t[t]], float(a[t]),
                              alpha=bw.alpha, lam=bw.lam, tau=bw.tau, tv_iters=bw.tv_iters) for t in range(T)]
    say("batch64 graph", len(gds), "slices")
    g = fbpnp.BatchGraph(batch, steps)
    g.launch()
    torch.cuda.synchronize()
    g.close()
    # every slice alone, same launch configuration, direct chained calls
    for i, gd in enumerate(gds):
        plan = fbpnp.Plan(fbpnp.Geometry(**gd), factors)
        for k, c in enumerate(cfgs):
            plan.set_config(k, c)
        npix = gd["nx"] * gd["ny"]
        xs = torch.zeros(npix, device="cuda")
        ys = torch.zeros(npix, device="cuda")
        bd = dev(bs[i]).reshape(-1)
        st = [fbpnp.pnp_args(plan, stage_t[t], bd, ys, xs, xs, ys, float(eta[stage_t[t], i]), float(a[t]),
                             None, 1.0, bw.alpha, bw.lam, bw.tau, bw.tv_iters) for t in range(T)]
        fbpnp.chain_steps(st)
        for s in st:
            fbpnp.pnp_step(plan, s)
        single = host(xs)
        batched = host(batch.image(x, i)).reshape(-1)
        if not np.array_equal(single, batched):
            raise AssertionError(f"slice {i} {shapes[i]}: batched differs from single-slice, "
                                 f"max |diff| {np.max(np.abs(single - batched))}")
        plan.close()
    for i in BATCH_ORACLE_SLICES:
        gd = gds[i]
        sched_o = [(factors[k], None, 1.0) for k in stage_t]
        et = np.array([eta[k, i] for k in stage_t], dtype=np.float64)
        ref = oracle.pnp_run(oracle.Geometry(**gd), bs[i].astype(np.float64), sched_o, et, a, bw.alpha, bw.lam,
                             bw.tv_iters, bw.tau)
        got = host(batch.image(x, i)).reshape(ref.shape)
        say("batch64 slice vs oracle", i, shapes[i], rel(got, ref))
        assert rel(got, ref) <= 1e-4, (i, rel(got, ref))
    batch.close()


@pytest.mark.parametrize("name", sorted(synth.SCENARIOS))
def test_scenario_whole_schedule(name):
    """25 iterations at f = 4, then 75 at f = 2 (m1 = d/16, m2 = d/4), all views, Poisson log data,
    FISTA momentum, one captured graph, against the oracle's loop."""
    sc = synth.SCENARIOS[name]
    g = sc.geometry
    og = oracle.Geometry(**g)
    x = sc.phantom()
    b = sc.data(oracle.fp(og, x.astype(np.float64))).astype(np.float32)
    plan = fbpnp.Plan(fbpnp.Geometry(**g), [4, 2])
    L4, L2 = oracle.power_lipschitz(og, 4, 100), oracle.power_lipschitz(og, 2, 100)
    fs = [4] * 25 + [2] * 75
    T = len(fs)
    eta = np.array([1 / L4 if f == 4 else 1 / L2 for f in fs])
    a = synth.momentum_table(T)
    say("scenario whole schedule", name)
    npix = g["nx"] * g["ny"]
    xb = torch.zeros(npix, device="cuda")
    yb = torch.zeros(npix, device="cuda")
    bd = dev(b).reshape(-1)
    steps = [fbpnp.pnp_args(plan, 0 if fs[t] == 4 else 1, bd, yb, xb, xb, yb, float(eta[t]), float(a[t]), None,
                            1.0, sc.alpha, sc.lam, sc.tau, sc.tv_iters) for t in range(T)]
    gr = fbpnp.Graph(plan, steps)
    gr.launch()
    got = host(xb).reshape(g["ny"], g["nx"])
    gr.close()
    ref = oracle.pnp_run(og, b.astype(np.float64), [(f, None, 1.0) for f in fs], eta, a, sc.alpha, sc.lam,
                         sc.tv_iters, sc.tau)
    say("scenario", name, rel(got, ref))
    assert rel(got, ref) <= 1e-4, (name, rel(got, ref))
