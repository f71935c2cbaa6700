"""GPU tests of the batched form: every slice of a batched run equals the same slice
run alone through pnp_step with the same launch configuration (bitwise), a slice
matches the FP64 oracle's loop, the captured batch graph equals direct calls, and
every autotuner candidate agrees with the default configuration."""
import sys

import numpy as np
import pytest
import torch

import oracle
from random_geometry import random_geometry
from paper_2203_07308_amd import fbpnp, synth

pytestmark = pytest.mark.gpu


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


# uneven slices: sizes, view counts (47: ragged subsets), detectors
SLICES = [(96, 90), (64, 47), (128, 120), (48, 60), (80, 90)]
FACTORS = [2, 1]


def make_batch(slices=SLICES, seed=40, factors=FACTORS, heights=None):
    """slices: (width, views); heights: optional image heights (default square)."""
    gds = [synth.fan_geometry(n, V) for n, V in slices]
    for g, h in zip(gds, heights or []):
        g["ny"] = h
    batch = fbpnp.Batch([fbpnp.Geometry(**g) for g in gds], factors)
    xts, bs = [], []
    for i, g in enumerate(gds):
        n = g["nx"]
        m = max(n, g["ny"])
        xt = synth.rasterise(synth.random_ellipses(seed + i, 10, m), m)[:g["ny"], :n].copy()
        ax = oracle.fp(oracle.Geometry(**g), xt.astype(np.float64))
        bs.append(synth.add_noise(ax, synth.standard_normal(seed + 50 + i, ax.shape), "gaussian",
                                  0.01).astype(np.float32))
        xts.append(xt)
    b_arena = torch.zeros(batch.sino_size, device="cuda")
    for i, b in enumerate(bs):
        batch.sinogram(b_arena, i).copy_(dev(b))
    return gds, batch, xts, bs, b_arena


def schedule(n_f2=3, n_f1=3, n_sub=3):
    """(stage, n_sub, subset, sigma, a_t): subsets at the coarse stage, all views at f = 1."""
    T = n_f2 + n_f1
    a = synth.momentum_table(T)
    seq = synth.subset_sequence(91, T, n_sub)
    out = []
    for t in range(T):
        if t < n_f2:
            out.append((0, n_sub, int(seq[t]), float(n_sub), float(a[t])))
        else:
            out.append((1, 1, 0, 1.0, float(a[t])))
    return out


def etas(batch, gds, factors=FACTORS):
    """Per (stage, slice) step sizes 1/L from the slices' own plans."""
    e = np.zeros((len(factors), len(gds)), dtype=np.float32)
    for i in range(len(gds)):
        p = batch.slice_plan(i)
        for k in range(len(factors)):
            e[k, i] = 1.0 / fbpnp.power_lipschitz(p, k, 30)
    return e


def run_batched(batch, b_arena, sched, eta, graph=False, alpha=1.0):
    x = torch.zeros(batch.image_size, device="cuda")
    y = torch.zeros(batch.image_size, device="cuda")
    eta_d = [dev(eta[k]) for k in range(eta.shape[0])]
    steps = [fbpnp.batch_args(batch, k, b_arena, y, x, x, y, eta_d[k], a_t, n_sub, sub, sigma, alpha)
             for k, n_sub, sub, sigma, a_t in sched]
    if graph:
        g = fbpnp.BatchGraph(batch, steps)
        g.launch()
        torch.cuda.synchronize()
        out1 = x.clone()
        x.zero_()
        y.zero_()
        g.launch()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(out1), host(x))  # replays are identical
        g.close()
    else:
        for n_sub in sorted({s[1] for s in sched}):
            batch.prepare(n_sub)  # set-up: the work lists of steps with these subset counts
        fbpnp.chain_steps(steps)
        for st in steps:
            fbpnp.pnp_step_batched(batch, st)
    torch.cuda.synchronize()
    return x


def run_single(g, b, sched, eta_i, cfgs, alpha=1.0, factors=FACTORS):
    plan = fbpnp.Plan(fbpnp.Geometry(**g), factors)
    for k, c in enumerate(cfgs):
        plan.set_config(k, c)
    npix = g["nx"] * g["ny"]
    x = torch.zeros(npix, device="cuda")
    y = torch.zeros(npix, device="cuda")
    bd = dev(b).reshape(-1)
    keep, steps = [], []
    for k, n_sub, sub, sigma, a_t in sched:
        views = None if n_sub <= 1 else dev(synth.subset_views(sub, n_sub, g["n_views"]), np.int32)
        keep.append(views)
        steps.append(fbpnp.pnp_args(plan, k, bd, y, x, x, y, float(eta_i[k]), a_t, views, sigma, alpha))
    fbpnp.chain_steps(steps)
    for st in steps:
        fbpnp.pnp_step(plan, st)
    return host(x).reshape(g["ny"], g["nx"])


def test_batched_slices_equal_single_slice_runs():
    gds, batch, xts, bs, b_arena = make_batch()
    sched = schedule()
    eta = etas(batch, gds)
    say("batched eager", [(g["nx"], g["n_views"]) for g in gds])
    x = run_batched(batch, b_arena, sched, eta)
    cfgs = [batch.get_config(k, 3 if k == 0 else 1) for k in range(len(FACTORS))]
    for i, g in enumerate(gds):
        say("single slice", i)
        ref = run_single(g, bs[i], sched, eta[:, i], cfgs)
        np.testing.assert_array_equal(host(batch.image(x, i)), ref)


def test_batched_scatter_form_equals_single_slice_runs():
    """The scatter back-projector in a batched launch, bit for bit the same slice run alone."""
    gds, batch, xts, bs, b_arena = make_batch(seed=70)
    sched = schedule()
    eta = etas(batch, gds)
    forms = [dict(fp_seg=0, bp_px=16, bp_vg=4, tv_tile=0), dict(fp_seg=0, bp_px=32, bp_vg=8, tv_tile=0)]
    for k in range(len(FACTORS)):
        batch.set_config(k, forms[k % len(forms)])
    say("batched scatter", [(g["nx"], g["n_views"]) for g in gds])
    x = run_batched(batch, b_arena, sched, eta)
    xg = run_batched(batch, b_arena, sched, eta, graph=True)
    np.testing.assert_array_equal(host(x), host(xg))
    cfgs = [batch.get_config(k, 3 if k == 0 else 1) for k in range(len(FACTORS))]
    assert all(c["bp_px"] in (16, 32) for c in cfgs)
    for i, g in enumerate(gds):
        say("single slice, scatter", i)
        ref = run_single(g, bs[i], sched, eta[:, i], cfgs)
        np.testing.assert_array_equal(host(batch.image(x, i)), ref)


def test_batched_graph_equals_direct_calls():
    gds, batch, xts, bs, b_arena = make_batch(seed=60)
    sched = schedule(4, 2, 4)
    eta = etas(batch, gds)
    say("batched graph")
    xe = host(run_batched(batch, b_arena, sched, eta))
    xg = host(run_batched(batch, b_arena, sched, eta, graph=True))
    np.testing.assert_array_equal(xe, xg)


def test_batched_rectangular_slices():
    """Slices wider than tall and taller than wide (64 x 40, 48 x 96, 80 x 18) in one batch: equal to
    single-slice runs bitwise, and one slice against the oracle's loop."""
    gds, batch, xts, bs, b_arena = make_batch(slices=[(64, 30), (48, 20), (80, 16)], seed=97,
                                              heights=[40, 96, 18])
    sched = schedule(3, 3, 3)
    eta = etas(batch, gds)
    say("batched rectangular")
    xd = run_batched(batch, b_arena, sched, eta)
    cfgs = [batch.get_config(k, 3 if k == 0 else 1) for k in range(len(FACTORS))]
    for i, g in enumerate(gds):
        ref = run_single(g, bs[i], sched, eta[:, i], cfgs)
        np.testing.assert_array_equal(host(batch.image(xd, i)), ref)
    og = oracle.Geometry(**gds[1])
    so = [(FACTORS[k], None if n_sub <= 1 else synth.subset_views(sub, n_sub, gds[1]["n_views"]), sigma)
          for k, n_sub, sub, sigma, _ in sched]
    et = np.array([eta[k, 1] for k, *_ in sched], dtype=np.float64)
    a = np.array([s[4] for s in sched])
    ref = oracle.pnp_run(og, bs[1].astype(np.float64), so, et, a)
    assert rel(host(batch.image(xd, 1)), ref) <= 1e-4, rel(host(batch.image(xd, 1)), ref)


def test_batched_factor_not_dividing_the_tv_tile():
    """Stage factors 3 and 1: 3 divides neither TV tile, so a step followed by a step at f = 3 pools
    y_t in a launch of its own after the denoiser instead of in its epilogue. Graph replays equal
    direct chained calls and single-slice runs, and a slice matches the oracle's loop."""
    factors = [3, 1]
    gds, batch, xts, bs, b_arena = make_batch(slices=[(48, 30), (96, 47)], seed=95, factors=factors)
    sched = schedule(4, 3, 3)
    eta = etas(batch, gds, factors)
    say("batched factor 3")
    xd = run_batched(batch, b_arena, sched, eta)
    xg = host(run_batched(batch, b_arena, sched, eta, graph=True))
    np.testing.assert_array_equal(host(xd), xg)
    cfgs = [batch.get_config(k, 3 if k == 0 else 1) for k in range(len(factors))]
    for i, g in enumerate(gds):
        ref = run_single(g, bs[i], sched, eta[:, i], cfgs, factors=factors)
        np.testing.assert_array_equal(host(batch.image(xd, i)), ref)
    og = oracle.Geometry(**gds[0])
    so = [(factors[k], None if n_sub <= 1 else synth.subset_views(sub, n_sub, gds[0]["n_views"]), sigma)
          for k, n_sub, sub, sigma, _ in sched]
    et = np.array([eta[k, 0] for k, *_ in sched], dtype=np.float64)
    a = np.array([s[4] for s in sched])
    ref = oracle.pnp_run(og, bs[0].astype(np.float64), so, et, a)
    got = host(batch.image(xd, 0))
    assert rel(got, ref) <= 1e-4, rel(got, ref)


def test_batched_blocks_reaching_the_source():
    """A slice with a coarse stage (f = 8, 9 x 4 stage pixels of 7.4 mm) and the source at 3 image
    circumradii beside an ordinary slice: with 2 x 2 pixels per lane its back-projection blocks reach
    the source circle, so the batch's back-projection at that stage takes every bin as a candidate.
    Direct chained calls equal the graph; the close slice equals its single-slice run bit for bit (the
    same every-bin variant), the other one to rounding (the batch ran it in that variant too); both
    slices match the oracle."""
    close = dict(nx=72, ny=32, pixel_mm=0.921235, n_views=28, n_bins=68, sod_mm=108.3165, sdd_mm=319.056,
                 det_pitch_mm=5.43828, det_offset_mm=17.0564, angle0_rad=0.769074, angle_step_rad=0.224399)
    gds = [close, synth.fan_geometry(64, 30)]
    factors = [8, 1]
    batch = fbpnp.Batch([fbpnp.Geometry(**g) for g in gds], factors)
    batch.set_config(0, dict(fp_seg=0, bp_px=2, bp_vg=4, tv_tile=0))
    bs = []
    b_arena = torch.zeros(batch.sino_size, device="cuda")
    for i, g in enumerate(gds):
        xt = synth.rasterise(synth.random_ellipses(120 + i, 10, max(g["nx"], g["ny"])),
                             max(g["nx"], g["ny"]))[:g["ny"], :g["nx"]].copy()
        bs.append(oracle.fp(oracle.Geometry(**g), xt.astype(np.float64)).astype(np.float32))
        batch.sinogram(b_arena, i).copy_(dev(bs[i]))
    sched = schedule(3, 2, 2)
    eta = etas(batch, gds, factors)
    say("batched blocks reaching the source")
    xd = run_batched(batch, b_arena, sched, eta)
    np.testing.assert_array_equal(host(xd), host(run_batched(batch, b_arena, sched, eta, graph=True)))
    cfgs = [batch.get_config(k, 2 if k == 0 else 1) for k in range(len(factors))]
    for i, g in enumerate(gds):
        single = run_single(g, bs[i], sched, eta[:, i], cfgs, factors=factors)
        if i == 0:
            np.testing.assert_array_equal(host(batch.image(xd, i)), single)
        else:
            assert rel(host(batch.image(xd, i)), single) <= 1e-6
        so = [(factors[k], None if n_sub <= 1 else synth.subset_views(sub, n_sub, g["n_views"]), sigma)
              for k, n_sub, sub, sigma, _ in sched]
        et = np.array([eta[k, i] for k, *_ in sched], dtype=np.float64)
        a = np.array([q[4] for q in sched])
        ref = oracle.pnp_run(oracle.Geometry(**g), bs[i].astype(np.float64), so, et, a)
        assert rel(host(batch.image(xd, i)), ref) <= 1e-4, (i, rel(host(batch.image(xd, i)), ref))


@pytest.mark.parametrize("seed", range(6))
def test_batched_random_slices(seed):
    """Three seeded random slices (sizes rounded down to a shared factor of 1 to 4, their own views,
    bins, detectors and source distances) in one batch: the graph equals direct chained calls and
    single-slice runs, and each slice matches the oracle's loop."""
    rng = np.random.default_rng(700 + seed)
    fc = int(rng.integers(1, 5))
    gds = []
    for k in range(3):
        g, _ = random_geometry(1000 + 10 * seed + k)
        g["nx"], g["ny"] = fc * max(1, g["nx"] // fc), fc * max(1, g["ny"] // fc)
        gds.append(g)
    factors = [fc, 1] if fc > 1 else [1]
    batch = fbpnp.Batch([fbpnp.Geometry(**g) for g in gds], factors)
    bs = []
    b_arena = torch.zeros(batch.sino_size, device="cuda")
    for i, g in enumerate(gds):
        xt = rng.random((g["ny"], g["nx"]))
        bs.append(oracle.fp(oracle.Geometry(**g), xt).astype(np.float32))
        batch.sinogram(b_arena, i).copy_(dev(bs[i]))
    T = 4
    a_t = synth.momentum_table(T)
    sched = [(0 if (len(factors) > 1 and t < 2) else len(factors) - 1, 1, 0, 1.0, float(a_t[t])) for t in range(T)]
    eta = etas(batch, gds, factors)
    say("batched random", seed, fc, [(g["nx"], g["ny"], g["n_views"], g["n_bins"]) for g in gds])
    xd = run_batched(batch, b_arena, sched, eta)
    np.testing.assert_array_equal(host(xd), host(run_batched(batch, b_arena, sched, eta, graph=True)))
    cfgs = [batch.get_config(k, 1) for k in range(len(factors))]
    for i, g in enumerate(gds):
        got = host(batch.image(xd, i))
        single = run_single(g, bs[i], sched, eta[:, i], cfgs, factors=factors)
        assert rel(got, single) <= 1e-6, (i, rel(got, single))
        so = [(factors[k], None, 1.0) for k, *_ in sched]
        et = np.array([eta[k, i] for k, *_ in sched], dtype=np.float64)
        ref = oracle.pnp_run(oracle.Geometry(**g), bs[i].astype(np.float64), so, et, np.asarray(a_t))
        assert rel(got, ref) <= 1e-4, (i, rel(got, ref))


def test_batched_slice_matches_oracle_loop():
    """Two slices of a batch against the FP64 oracle's sketched loop (relative L2 1e-4)."""
    gds, batch, xts, bs, b_arena = make_batch(slices=[(64, 90), (96, 47)], seed=70)
    sched = schedule(6, 6, 3)
    eta = etas(batch, gds)
    say("batched vs oracle")
    x = run_batched(batch, b_arena, sched, eta, alpha=0.9)
    for i, g in enumerate(gds):
        og = oracle.Geometry(**g)
        so = [(FACTORS[k], None if n_sub <= 1 else synth.subset_views(sub, n_sub, g["n_views"]), sigma)
              for k, n_sub, sub, sigma, _ in sched]
        et = np.array([eta[k, i] for k, *_ in sched], dtype=np.float64)
        a = np.array([s[4] for s in sched])
        ref = oracle.pnp_run(og, bs[i].astype(np.float64), so, et, a, alpha=0.9)
        got = host(batch.image(x, i))
        assert rel(got, ref) <= 1e-4, (i, rel(got, ref))


def candidate_configs():
    out = []
    for seg in (1, 2, 4, 8):
        for px, vg in ((1, 1), (1, 4), (2, 2), (2, 16), (4, 1), (4, 4), (16, 4), (32, 16)):
            for tile in (16, 32):
                out.append(dict(fp_seg=seg, bp_px=px, bp_vg=vg, tv_tile=tile))
    return out


def test_batched_autotuner_candidates_agree_and_cache(tmp_path):
    gds, batch, xts, bs, b_arena = make_batch(seed=80)
    sched = schedule(2, 2, 3)
    eta = etas(batch, gds)
    base = host(run_batched(batch, b_arena, sched, eta))
    say("batched candidates", len(candidate_configs()))
    for c in candidate_configs():
        for k in range(len(FACTORS)):
            batch.set_config(k, c)
        got = host(run_batched(batch, b_arena, sched, eta))
        for i in range(len(gds)):
            o = slice(batch.image_offsets[i], batch.image_offsets[i] + gds[i]["nx"] * gds[i]["ny"])
            assert rel(got[o], base[o]) <= 1e-5, (c, i, rel(got[o], base[o]))
    for k in range(len(FACTORS)):
        batch.set_config(k, None)
    cache = tmp_path / "tune.txt"
    say("batched autotune")
    batch.autotune(3, str(cache))
    tuned = [batch.get_config(k, 3) for k in range(len(FACTORS))]
    lines = cache.read_text().splitlines()
    assert len(lines) == len(FACTORS)
    for c in tuned:
        assert c["fp_seg"] in (1, 2, 4, 8) and c["bp_px"] in (1, 2, 4, 16, 32) and c["tv_tile"] in (16, 32)
    got = host(run_batched(batch, b_arena, sched, eta))
    assert rel(got, base) <= 1e-5
    # a second batch of the same slices takes the cached choice (no new cache lines)
    batch2 = fbpnp.Batch(batch.geoms, FACTORS)
    batch2.autotune(3, str(cache))
    assert [batch2.get_config(k, 3) for k in range(len(FACTORS))] == tuned
    assert len(cache.read_text().splitlines()) == len(FACTORS)


def test_plan_configs_match_oracle_and_autotune(tmp_path):
    g = synth.fan_geometry(96, 60)
    og = oracle.Geometry(**g)
    plan = fbpnp.Plan(fbpnp.Geometry(**g), [2, 1])
    img = synth.rasterise(synth.random_ellipses(5, 8, 96), 96)
    sino = np.random.default_rng(4).random((60, g["n_bins"]))
    views = synth.subset_views(1, 4, 60)
    vd = dev(views, np.int32)
    for k, f in enumerate((2, 1)):
        v = oracle.down(img, f)
        ref_fp = oracle.fp(og, v, f=f, views=views)
        ref_bp = oracle.bp(og, sino[views], f=f, views=views)
        for c in candidate_configs()[::5]:
            plan.set_config(k, c)
            y = torch.empty(len(views) * g["n_bins"], device="cuda")
            fbpnp.fanbeam_fp(plan, k, dev(v).reshape(-1), y, vd)
            assert rel(host(y).reshape(ref_fp.shape), ref_fp) <= 1e-5, (c, k)
            xo = torch.empty(v.size, device="cuda")
            fbpnp.fanbeam_bp(plan, k, dev(sino[views]).reshape(-1), xo, vd)
            assert rel(host(xo).reshape(ref_bp.shape), ref_bp) <= 2e-5, (c, k)
        plan.set_config(k, None)
    say("plan autotune")
    plan.autotune(len(views), str(tmp_path / "t.txt"))
    for k in range(2):
        c = plan.get_config(k, len(views))
        assert c["fp_seg"] in (1, 2, 4, 8) and c["bp_vg"] >= 1


def test_plan_autotune_all_views_sinogram_larger_than_image(tmp_path):
    """Autotuning with every view selected, where a projection (90 x 96) holds more
    values than the image (64 x 64): the tuner's projection buffer is sized for it."""
    g = synth.fan_geometry(64, 90)
    og = oracle.Geometry(**g)
    plan = fbpnp.Plan(fbpnp.Geometry(**g), [2, 1])
    say("plan autotune all views")
    plan.autotune(90, str(tmp_path / "t.txt"))
    img = synth.rasterise(synth.random_ellipses(6, 8, 64), 64)
    for k, f in enumerate((2, 1)):
        v = oracle.down(img, f)
        y = torch.empty(90 * g["n_bins"], device="cuda")
        fbpnp.fanbeam_fp(plan, k, dev(v).reshape(-1), y)
        ref = oracle.fp(og, v, f=f)
        assert rel(host(y).reshape(ref.shape), ref) <= 1e-5, (k, plan.get_config(k, 90))


def test_batch_rejects_bad_arguments():
    gds = [synth.fan_geometry(64, 30), synth.fan_geometry(48, 20)]
    batch = fbpnp.Batch([fbpnp.Geometry(**g) for g in gds], [2, 1])
    x = torch.zeros(batch.image_size, device="cuda")
    b = torch.zeros(batch.sino_size, device="cuda")
    eta = torch.ones(2, device="cuda")
    with pytest.raises(fbpnp.FbError):
        fbpnp.pnp_step_batched(batch, fbpnp.batch_args(batch, 0, b, x, x, x, x, eta, 0.0, n_sub=3, subset=3))
    with pytest.raises(fbpnp.FbError):
        fbpnp.pnp_step_batched(batch, fbpnp.batch_args(batch, 2, b, x, x, x, x, eta, 0.0))
    with pytest.raises(fbpnp.FbError):
        batch.set_config(0, dict(fp_seg=3, bp_px=0, bp_vg=0, tv_tile=0))
    with pytest.raises(fbpnp.FbError):
        batch.set_config(0, dict(fp_seg=0, bp_px=4, bp_vg=8, tv_tile=0))
    with pytest.raises(fbpnp.FbError):
        fbpnp.Batch([fbpnp.Geometry(**synth.fan_geometry(63, 30))], [2])  # 2 does not divide 63
    # a step never builds work lists itself: steps with subsets need a set-up call first
    y = torch.zeros_like(x)
    with pytest.raises(fbpnp.FbError, match="fb_batch_prepare"):
        fbpnp.pnp_step_batched(batch, fbpnp.batch_args(batch, 0, b, y, x, x, y, eta, 0.0, n_sub=3, subset=1,
                                                       sigma=3.0))
    batch.prepare(3)
    fbpnp.pnp_step_batched(batch, fbpnp.batch_args(batch, 0, b, y, x, x, y, eta, 0.0, n_sub=3, subset=1, sigma=3.0))
    # a configuration change keeps the prepared subset counts runnable
    batch.set_config(0, dict(fp_seg=1, bp_px=1, bp_vg=2, tv_tile=16))
    fbpnp.pnp_step_batched(batch, fbpnp.batch_args(batch, 0, b, y, x, x, y, eta, 0.0, n_sub=3, subset=2, sigma=3.0))
    torch.cuda.synchronize()
    with pytest.raises(ValueError):
        fbpnp.batch_args(batch, 0, b[:10], x, x, x, x, eta, 0.0)
