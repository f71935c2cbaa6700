"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances (FP32 GPU against FP64 oracle):
  * projections: relative L2 per view <= 1e-5;
  * backprojection of a projection-like (non-negative) sinogram: relative L2 <= 1e-5;
    of a zero-mean random sinogram, whose sum cancels, <= 2e-5 (every term carries a
    weight error of about one float ulp of a pixel position, which the cancelling
    sum does not shrink);
  * pooling, upsampling: <= 1e-6; TV-prox: <= 1e-6 relative L2;
  * reconstructions (whole PnP loops): relative L2 <= 1e-4.
"""
import math
import os
import shutil
import sys

import numpy as np
import pytest
import torch

import oracle
from random_geometry import coarse_random_geometry, random_geometry
from paper_2203_07308_amd import fbpnp, synth

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fbpnp.load()
    yield
    torch.cuda.synchronize()


def dev(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def make_geom(n, V, nb=None, ny=None, wide=None, **kw):
    g = synth.fan_geometry(n, V, nb, sod_over_radius=wide)
    if ny is not None:
        g["ny"] = ny
    g.update(kw)
    return g


def ellipse_image(ny, nx, seed):
    n = max(nx, ny)
    img = synth.rasterise(synth.random_ellipses(seed, 12, n), n)
    return img[:ny, :nx].copy()


GEOMS = {
    "64": dict(n=64, V=90),
    "256": dict(n=256, V=360),
    "512": dict(n=512, V=720),
    "1024": dict(n=1024, V=16),
    "ragged": dict(n=70, V=37, nb=101, ny=52, det_offset_mm=1.3, angle0_rad=0.2),
    "diag": dict(n=40, V=8, angle0_rad=math.pi / 4),
    "tiny": dict(n=8, V=4, nb=12),
    # source at 1.5 image circumradii: a fan of about 85 degrees (the plan's limit is 90)
    "widefan": dict(n=128, V=90, nb=256, wide=1.5),
    # 0.15 pixel per bin at the isocentre: a 32-pixel block's footprint spans about 200 bins,
    # more than the back-projector stages per view at once (several chunks per view)
    "finepitch": dict(n=96, V=12, nb=640, det_pitch_mm=0.3),
    # detector shifted by about half its width: many bins see no pixel (rays without samples
    # next to the image edge, in every view)
    "offset": dict(n=64, V=30, nb=64, det_offset_mm=60.0),
}

FP_CASES = [
    ("64", 1, None), ("64", 2, None), ("64", 4, None),
    ("256", 1, None), ("256", 2, None), ("256", 2, ("sub", 5, 8)),
    ("512", 1, None), ("512", 2, None), ("512", 4, None), ("512", 1, ("sub", 3, 8)), ("512", 1, ("sub", 1, 2)),
    ("1024", 1, None),
    ("ragged", 1, None), ("ragged", 2, ("list", [36, 0, 17, 17, 5])),
    ("diag", 1, None), ("diag", 2, None), ("tiny", 1, None), ("tiny", 2, ("list", [2])),
    ("widefan", 1, None), ("widefan", 2, None), ("widefan", 4, ("sub", 1, 4)),
    ("finepitch", 1, None), ("finepitch", 2, ("sub", 1, 3)),
    ("offset", 1, None), ("offset", 2, None), ("offset", 4, ("sub", 2, 3)),
]


def setup_case(name, f, sel):
    gd = make_geom(**GEOMS[name])
    og = oracle.Geometry(**gd)
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [f])
    if sel is None:
        views = None
    elif sel[0] == "sub":
        views = synth.subset_views(sel[1], sel[2], gd["n_views"])
    else:
        views = np.array(sel[1], dtype=np.int32)
    return gd, og, plan, views


def fp_forms(plan, stage):
    """Forward-projector launch shapes: the built-in one, and where the stage's line images
    fit in LDS, the LDS-staged form with one and eight lanes per ray."""
    forms = [None]
    try:
        plan.set_config(stage, dict(fp_seg=1, fp_lds=2))
        forms += [dict(fp_seg=1, fp_lds=2), dict(fp_seg=8, fp_lds=2)]
    except fbpnp.FbError:
        pass
    plan.set_config(stage, None)
    return forms


@pytest.mark.parametrize("name,f,sel", FP_CASES)
def test_fanbeam_fp_matches_oracle(name, f, sel):
    gd, og, plan, views = setup_case(name, f, sel)
    nys, nxs = gd["ny"] // f, gd["nx"] // f
    x = ellipse_image(nys, nxs, 11).astype(np.float32)
    n_sel = gd["n_views"] if views is None else len(views)
    ref = oracle.fp(og, x.astype(np.float64), f, views)
    outs = []
    for form in fp_forms(plan, 0):
        say("fp", name, f, sel, form)
        plan.set_config(0, form)
        y = torch.empty(n_sel * gd["n_bins"], device="cuda")
        fbpnp.fanbeam_fp(plan, 0, dev(x), y, None if views is None else dev(views, np.int32))
        got = host(y).reshape(n_sel, gd["n_bins"])
        outs.append(got)
        for i in range(n_sel):
            if np.linalg.norm(ref[i]) > 0:
                assert rel(got[i], ref[i]) <= 1e-5, (form, i, rel(got[i], ref[i]))
            else:
                assert np.all(got[i] == 0)
    # the taps are the same floats wherever they are read from: the LDS form with the
    # built-in lanes per ray equals the global one bit for bit
    if len(outs) > 1:
        plan.set_config(0, None)
        seg = plan.get_config(0, n_sel)["fp_seg"]
        plan.set_config(0, dict(fp_seg=seg, fp_lds=2))
        y = torch.empty(n_sel * gd["n_bins"], device="cuda")
        fbpnp.fanbeam_fp(plan, 0, dev(x), y, None if views is None else dev(views, np.int32))
        np.testing.assert_array_equal(host(y).reshape(n_sel, gd["n_bins"]), outs[0])
        plan.set_config(0, None)


def test_fp_lds_refused_where_the_stage_does_not_fit():
    gd = make_geom(**GEOMS["512"])
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [1, 4])
    with pytest.raises(fbpnp.FbError):
        plan.set_config(0, dict(fp_lds=2))
    plan.set_config(1, dict(fp_lds=2))
    assert plan.get_config(1)["fp_lds"] == 2
    with pytest.raises(fbpnp.FbError):
        plan.set_config(1, dict(fp_lds=3))


# backprojector launch shapes: the built-in choice, each pixel block size of the gather form
# and each block side of the scatter form
BP_FORMS = [dict(), dict(bp_px=1, bp_vg=16), dict(bp_px=2, bp_vg=4), dict(bp_px=4, bp_vg=1),
            dict(bp_px=16, bp_vg=4), dict(bp_px=32, bp_vg=16), dict(bp_px=32, bp_vg=1)]


@pytest.mark.parametrize("name,f,sel", FP_CASES)
def test_fanbeam_bp_matches_oracle(name, f, sel):
    gd, og, plan, views = setup_case(name, f, sel)
    nys, nxs = gd["ny"] // f, gd["nx"] // f
    n_sel = gd["n_views"] if views is None else len(views)
    dv = None if views is None else dev(views, np.int32)
    # a projection-like sinogram and a zero-mean random one
    ysin = oracle.fp(og, ellipse_image(nys, nxs, 5), f, views).astype(np.float32)
    yrnd = (np.random.default_rng(7).random((n_sel, gd["n_bins"])) - 0.5).astype(np.float32)
    for y, tol in ((ysin, 1e-5), (yrnd, 2e-5)):
        ref = oracle.bp(og, y.astype(np.float64), f, views, 0.75)
        for form in BP_FORMS:
            say("bp", name, f, sel, form)
            plan.set_config(0, form)
            x = torch.empty(nys * nxs, device="cuda")
            fbpnp.fanbeam_bp(plan, 0, dev(y), x, dv, scale=0.75)
            got = host(x).reshape(nys, nxs)
            assert rel(got, ref) <= tol, (form, rel(got, ref))


@pytest.mark.parametrize("form", [dict(fp_seg=0, bp_px=32, bp_vg=16, tv_tile=0),
                                  dict(fp_seg=0, bp_px=16, bp_vg=16, tv_tile=0)])
def test_scatter_bp_repeats_bit_for_bit_at_512(form):
    """The scatter back-projector at 512^2, f = 1, on a 90-view subset (the benchmarked
    full-resolution shape): five launches give the same bits, as a lost update between
    lanes of one wavefront would not, and match the oracle. Also fused, inside pnp_step:
    repeated steps from the same inputs give the same bits."""
    gd, og, plan, views = setup_case("512", 1, ("sub", 5, 8))
    plan.set_config(0, form)
    rng = np.random.default_rng(23)
    y = (rng.random((len(views), gd["n_bins"])) - 0.4).astype(np.float32)
    ref = oracle.bp(og, y.astype(np.float64), 1, views, 1.0)
    dv, dy = dev(views, np.int32), dev(y)
    outs = []
    for _ in range(5):
        x = torch.empty(gd["nx"] * gd["ny"], device="cuda")
        fbpnp.fanbeam_bp(plan, 0, dy, x, dv)
        outs.append(host(x))
    say("scatter repeat", form, rel(outs[0].reshape(ref.shape), ref))
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])
    assert rel(outs[0].reshape(ref.shape), ref) <= 2e-5
    b = dev(rng.random((gd["n_views"], gd["n_bins"])).astype(np.float32))
    yp = dev(ellipse_image(gd["ny"], gd["nx"], 5).astype(np.float32))
    xp = yp.clone()
    zs = []
    for _ in range(3):
        xo, yo = torch.empty_like(yp), torch.empty_like(yp)
        fbpnp.pnp_step(plan, fbpnp.pnp_args(plan, 0, b, yp, xp, xo, yo, 1e-6, 0.5, dv, 8.0))
        zs.append(host(xo))
    for z in zs[1:]:
        np.testing.assert_array_equal(z, zs[0])


def test_fanbeam_bp_skips_invalid_views():
    """View indices outside [0, n_views) add nothing and repeats add twice, in every launch shape."""
    gd, og, plan, _ = setup_case("ragged", 1, None)
    views = np.array([36, -1, 17, 37, 17, 1 << 20, 2], dtype=np.int32)
    ok = (views >= 0) & (views < gd["n_views"])
    y = (np.random.default_rng(3).random((len(views), gd["n_bins"])) + 0.5).astype(np.float32)
    ref = oracle.bp(og, y[ok].astype(np.float64), 1, views[ok], 1.0)
    for form in BP_FORMS:
        say("bp invalid views", form)
        plan.set_config(0, form)
        x = torch.empty(gd["nx"] * gd["ny"], device="cuda")
        fbpnp.fanbeam_bp(plan, 0, dev(y), x, dev(views, np.int32))
        assert rel(host(x).reshape(ref.shape), ref) <= 1e-5, form


def test_check_views_reports_the_first_index_outside_the_views():
    """fb_check_views: FB_ESUBSET naming the first bad position and its value, for indices
    below 0 and at or above n_views, and for a list longer than the views; valid lists
    (repeats included) pass. A 720-view plan checks a list spread over several blocks."""
    gd, og, plan, _ = setup_case("ragged", 1, None)
    V = gd["n_views"]
    fbpnp.check_views(plan, dev(np.array([0, V - 1, 3, 3], dtype=np.int32), np.int32))
    fbpnp.check_views(plan, dev(np.arange(V, dtype=np.int32)[::-1].copy(), np.int32))
    for lst, pos, val in (([36, -1, 17, 37, 1 << 20], 1, -1), ([2, 5, V], 2, V)):
        with pytest.raises(fbpnp.FbError) as e:
            fbpnp.check_views(plan, dev(np.array(lst, dtype=np.int32), np.int32))
        assert e.value.status == -4 and f"views[{pos}] = {val} " in str(e.value), str(e.value)
    with pytest.raises(fbpnp.FbError) as e:
        fbpnp.check_views(plan, dev(np.zeros(V + 1, dtype=np.int32), np.int32))
    assert e.value.status == -4
    big = fbpnp.Plan(fbpnp.Geometry(**synth.WORKLOADS["ms2g512"].geometry), [4])
    W = big.geom.n_views
    lst = np.arange(W, dtype=np.int32) % 97
    fbpnp.check_views(big, dev(lst, np.int32))
    lst[650], lst[300], lst[601] = -7, W + 3, W
    with pytest.raises(fbpnp.FbError) as e:
        fbpnp.check_views(big, dev(lst, np.int32))
    assert e.value.status == -4 and f"views[300] = {W + 3} " in str(e.value), str(e.value)


@pytest.mark.parametrize("name,f", [("256", 1), ("512", 4), ("ragged", 2), ("512", 1), ("widefan", 1),
                                    ("finepitch", 1)])
def test_fp32_adjoint_identity(name, f):
    """<A x, y> = <x, A^T y> between the GPU projector and the GPU backprojector (each launch shape)."""
    gd, og, plan, _ = setup_case(name, f, None)
    nys, nxs = gd["ny"] // f, gd["nx"] // f
    rng = np.random.default_rng(1)
    x = rng.random((nys, nxs)).astype(np.float32)
    y = rng.random((gd["n_views"], gd["n_bins"])).astype(np.float32)
    ax = torch.empty(y.size, device="cuda")
    fbpnp.fanbeam_fp(plan, 0, dev(x), ax)
    lhs = np.vdot(host(ax), y.ravel().astype(np.float64))
    for form in BP_FORMS:
        say("adjoint", name, f, form)
        plan.set_config(0, form)
        aty = torch.empty(x.size, device="cuda")
        fbpnp.fanbeam_bp(plan, 0, dev(y), aty)
        rhs = np.vdot(x.ravel().astype(np.float64), host(aty))
        assert abs(lhs - rhs) <= 1e-5 * abs(lhs), form


def degenerate_geom(nx, ny, V, B, pitch=2.0, off=0.0, factors=(1,)):
    return dict(nx=nx, ny=ny, pixel_mm=1.0, n_views=V, n_bins=B, sod_mm=50.0, sdd_mm=100.0, det_pitch_mm=pitch,
                det_offset_mm=off, angle0_rad=0.1, angle_step_rad=2 * math.pi / V), list(factors)


DEGENERATE = {
    "1x1": degenerate_geom(1, 1, 3, 1),
    "1x7": degenerate_geom(1, 7, 5, 4),
    "9x1": degenerate_geom(9, 1, 2, 3, off=0.7),
    "one_view_one_bin": degenerate_geom(16, 16, 1, 1, pitch=1.0, factors=(1, 2, 16)),
    "2x2": degenerate_geom(2, 2, 4, 2, pitch=0.5, factors=(1, 2)),
}


@pytest.mark.parametrize("name", list(DEGENERATE))
def test_degenerate_geometries_match_oracle(name):
    """One-pixel and one-line grids, a single view or bin, stages of a single pixel: projection,
    back-projection in every launch shape, the adjoint identity and a fused step, against the oracle."""
    gd, factors = DEGENERATE[name]
    og = oracle.Geometry(**gd)
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), factors)
    rng = np.random.default_rng(5)
    for k, f in enumerate(factors):
        nys, nxs = gd["ny"] // f, gd["nx"] // f
        x = rng.random((nys, nxs)).astype(np.float32)
        y = rng.random((gd["n_views"], gd["n_bins"])).astype(np.float32)
        say("degenerate", name, f)
        ax = torch.empty(y.size, device="cuda")
        fbpnp.fanbeam_fp(plan, k, dev(x), ax)
        ref = oracle.fp(og, x.astype(np.float64), f)
        assert rel(host(ax).reshape(ref.shape), ref) <= 1e-5
        lhs = np.vdot(host(ax), y.ravel().astype(np.float64))
        refb = oracle.bp(og, y.astype(np.float64), f)
        for form in BP_FORMS:
            plan.set_config(k, form)
            aty = torch.empty(x.size, device="cuda")
            fbpnp.fanbeam_bp(plan, k, dev(y), aty)
            got = host(aty)
            assert rel(got.reshape(refb.shape), refb) <= 1e-5, form
            rhs = np.vdot(x.ravel().astype(np.float64), got)
            assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), 1e-30), form
        plan.set_config(k, None)
    xt = rng.random((gd["ny"], gd["nx"]))
    b = oracle.fp(og, xt).astype(np.float32)
    sched_g = [(k, None, 1.0) for k in range(len(factors))] + [(0, None, 1.0)]
    sched_o = [(f, None, 1.0) for f in factors] + [(factors[0], None, 1.0)]
    eta = np.full(len(sched_g), 0.01)
    a = synth.momentum_table(len(sched_g))
    x_g = run_gpu(plan, gd, b, sched_g, eta, a, graph=True)
    x_o = oracle.pnp_run(og, b.astype(np.float64), sched_o, eta, a)
    assert rel(x_g, x_o) <= 1e-5, rel(x_g, x_o)


@pytest.mark.parametrize("seed", range(40))
def test_random_geometries_match_oracle(seed):
    """Projection, back-projection in every launch shape, the adjoint identity, and three fused steps
    captured as a graph, on a seeded random geometry (seeds 24 and up: a coarse stage), against the
    oracle."""
    gd, f = random_geometry(seed) if seed < 24 else coarse_random_geometry(seed)
    og = oracle.Geometry(**gd)
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [f])
    rng = np.random.default_rng(100 + seed)
    nys, nxs = gd["ny"] // f, gd["nx"] // f
    x = rng.random((nys, nxs)).astype(np.float32)
    y = (0.5 + rng.random((gd["n_views"], gd["n_bins"]))).astype(np.float32)
    say("random geometry", seed, gd["nx"], gd["ny"], gd["n_views"], gd["n_bins"], f)
    ax = torch.empty(y.size, device="cuda")
    fbpnp.fanbeam_fp(plan, 0, dev(x), ax)
    got = host(ax).reshape(y.shape)
    ref = oracle.fp(og, x.astype(np.float64), f)
    for i in range(y.shape[0]):
        if np.linalg.norm(ref[i]) > 0:
            assert rel(got[i], ref[i]) <= 1e-5, (i, rel(got[i], ref[i]))
        else:
            assert np.all(got[i] == 0)
    lhs = np.vdot(got.ravel().astype(np.float64), y.ravel().astype(np.float64))
    refb = oracle.bp(og, y.astype(np.float64), f)
    for form in BP_FORMS:
        plan.set_config(0, form)
        aty = torch.empty(x.size, device="cuda")
        fbpnp.fanbeam_bp(plan, 0, dev(y), aty)
        gb = host(aty)
        assert rel(gb.reshape(refb.shape), refb) <= 1e-5, (form, rel(gb.reshape(refb.shape), refb))
        rhs = np.vdot(x.ravel().astype(np.float64), gb.astype(np.float64))
        assert abs(lhs - rhs) <= 1e-5 * abs(lhs), form
    plan.set_config(0, None)
    xt = rng.random((gd["ny"], gd["nx"]))
    b = oracle.fp(og, xt).astype(np.float32)
    eta = np.full(3, 1.0 / oracle.power_lipschitz(og, f, 30))
    a = synth.momentum_table(3)
    xg = run_gpu(plan, gd, b, [(0, None, 1.0)] * 3, eta, a, graph=True)
    xo = oracle.pnp_run(og, b.astype(np.float64), [(f, None, 1.0)] * 3, eta, a)
    assert rel(xg, xo) <= 2e-5, rel(xg, xo)
    # the step size's power iteration (all views), and pooling and its adjoint at this factor
    L = fbpnp.power_lipschitz(plan, 0, 30)
    assert abs(L - 1.0 / eta[0]) <= 1e-4 * L, (L, 1.0 / eta[0])
    xs = rng.random((gd["ny"], gd["nx"])).astype(np.float32)
    v = torch.empty((nys, nxs), device="cuda")
    fbpnp.sketch_down(dev(xs), f, v)
    np.testing.assert_allclose(host(v), oracle.down(xs, f), rtol=1e-6, atol=1e-7)
    up = torch.empty((gd["ny"], gd["nx"]), device="cuda")
    fbpnp.sketch_up(dev(x), f, up)
    np.testing.assert_allclose(host(up), oracle.up(x, f), rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("name", ["256", "widefan"])
def test_stage_sample_counts_match_oracle(name):
    gd = make_geom(**GEOMS[name])
    n = gd["nx"]
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [1, 2, 4])
    og = oracle.Geometry(**gd)
    for s, f in enumerate([1, 2, 4]):
        info = plan.stage_info(s)
        assert (info.factor, info.nxs, info.nys) == (f, n // f, n // f)
        ref = oracle.count_samples(og, f)
        # the plan decides validity in the kernels' FP32 evaluation of the position:
        # a few samples within one rounding of the grid edge (weight ~0) may differ
        assert abs(info.samples_all_views - ref) <= 4 + 1e-6 * ref, (f, info.samples_all_views, ref)
        per_view = plan.view_samples(s)
        assert sum(per_view) == info.samples_all_views
        for k in (0, 17, gd["n_views"] // 2 + 1, gd["n_views"] - 1):
            rk = oracle.count_samples(og, f, np.array([k], dtype=np.int32))
            assert abs(per_view[k] - rk) <= 2 + 1e-5 * rk, (f, k, per_view[k], rk)


@pytest.mark.parametrize("shape,f", [((64, 64), 1), ((64, 64), 2), ((512, 512), 4), ((48, 80), 4), ((30, 42), 3)])
def test_sketch_down_up_match_oracle(shape, f):
    say("sketch", shape, f)
    x = np.random.default_rng(2).random(shape).astype(np.float32)
    v = torch.empty((shape[0] // f, shape[1] // f), device="cuda")
    fbpnp.sketch_down(dev(x), f, v)
    np.testing.assert_allclose(host(v), oracle.down(x, f), rtol=1e-6, atol=1e-7)
    vv = np.random.default_rng(3).random((shape[0] // f, shape[1] // f)).astype(np.float32)
    up = torch.empty(shape, device="cuda")
    fbpnp.sketch_up(dev(vv), f, up)
    np.testing.assert_allclose(host(up), oracle.up(vv, f), rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("shape,lam,iters", [((64, 64), 0.01, 5), ((256, 256), 0.01, 5), ((512, 512), 0.01, 5),
                                             ((37, 70), 0.05, 3), ((96, 64), 0.02, 8), ((64, 80), 0.02, 21),
                                             ((512, 512), 0.02, 8), ((520, 600), 0.01, 12),
                                             ((16, 16), 0.0, 5)])
def test_tv_prox_matches_oracle(shape, lam, iters):
    say("tv", shape, lam, iters)
    z = (ellipse_image(*shape, 9) + 0.05 * np.random.default_rng(4).standard_normal(shape)).astype(np.float32)
    x = torch.empty(shape, device="cuda")
    fbpnp.tv_prox(dev(z), x, lam, iters)
    ref = oracle.tv_prox(z.astype(np.float64), lam, iters)
    assert rel(host(x), ref) <= 1e-6, rel(host(x), ref)


def problem(name, seed=0):
    w = synth.WORKLOADS[name]
    gd = w.geometry
    og = oracle.Geometry(**gd)
    xt = synth.phantom(w)
    ax = oracle.fp(og, xt.astype(np.float64))
    b = synth.add_noise(ax, synth.standard_normal(synth.noise_seed(w), ax.shape), w.noise_kind,
                        w.noise_level).astype(np.float32)
    return w, gd, og, xt, b


def run_gpu(plan, gd, b, sched, eta, a, alpha=1.0, lam=0.01, history=False, graph=False, chained=False,
            events=None, tv_iters=5, stamps=None):
    """Runs the schedule with pnp_step (or as one captured graph). sched: (stage_index, views, sigma).
    chained: direct calls with the graph's pooling hand-over; events: list that receives six
    timing events per step; stamps: zeroed int64 device buffer of len(sched) + 1 (a clock
    mark, then one end-of-step stamp per step)."""
    npix = gd["nx"] * gd["ny"]
    bd = dev(b)
    xb = torch.zeros(npix, device="cuda")
    yb = torch.zeros(npix, device="cuda")
    hist = torch.zeros((len(sched), npix), device="cuda") if history else None
    keep = []
    steps = []
    for t, (s, views, sigma) in enumerate(sched):
        dv = None if views is None else dev(views, np.int32)
        keep.append(dv)
        ev = None
        if events is not None:
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
            events.append(ev)
        steps.append(fbpnp.pnp_args(plan, s, bd, yb, xb, xb, yb, float(eta[t]), float(a[t]), dv, sigma,
                                    alpha, lam, 0.125, tv_iters, None if hist is None else hist[t], ev,
                                    stamp=None if stamps is None else stamps[t + 1:t + 2]))
    if chained:
        fbpnp.chain_steps(steps)
    if stamps is not None:
        fbpnp.clock_stamp(stamps[0:1])
    if graph:
        g = fbpnp.Graph(plan, steps)
        g.launch()
        torch.cuda.synchronize()
        g.close()
    else:
        for st in steps:
            fbpnp.pnp_step(plan, st)
    out = host(xb).reshape(gd["ny"], gd["nx"])
    return (out, host(hist)) if history else out


def test_pnp_step_matches_oracle_iterations():
    """Three mixed iterations: f = 2 then f = 1, view subsets, momentum, alpha < 1."""
    w, gd, og, xt, b = problem("pnp64")
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [1, 2])
    sub = synth.subset_views(1, 3, gd["n_views"])
    sched_g = [(1, None, 1.0), (1, sub, 3.0), (0, sub, 3.0), (0, None, 1.0)]
    sched_o = [(2, None, 1.0), (2, sub, 3.0), (1, sub, 3.0), (1, None, 1.0)]
    eta = np.array([2e-4, 1.5e-4, 1e-4, 1e-4])
    a = synth.momentum_table(4)
    say("pnp_step 64")
    x, hist = run_gpu(plan, gd, b, sched_g, eta, a, alpha=0.8, history=True)
    ref, rhist = oracle.pnp_run(og, b.astype(np.float64), sched_o, eta, a, alpha=0.8, history=True)
    for t in range(4):
        assert rel(hist[t].reshape(ref.shape), rhist[t]) <= 2e-5, (t, rel(hist[t].reshape(ref.shape), rhist[t]))
    assert rel(x, ref) <= 2e-5


@pytest.mark.parametrize("form", BP_FORMS)
def test_pnp_step_large_odd_pooling_factors(form):
    """Fused steps at f = 30, 24 and 5 on a 240 x 120 grid (stage grids 8 x 4, 10 x 5 and 48 x 24,
    ragged pixel blocks): the back-projector epilogue takes exact quotients by f and by the block
    width in fine pixels for factors that are not powers of two, up to blocks of 32 x 30 fine
    pixels."""
    gd = make_geom(n=240, V=24, ny=120)
    og = oracle.Geometry(**gd)
    xt = ellipse_image(gd["ny"], gd["nx"], 9)
    b = oracle.fp(og, xt.astype(np.float64)).astype(np.float32)
    factors = [30, 24, 5]
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), factors)
    for k in range(3):
        plan.set_config(k, form)
    order = [0, 1, 2, 0, 2]
    sched_g = [(k, None, 1.0) for k in order]
    sched_o = [(factors[k], None, 1.0) for k in order]
    eta = np.array([1.0 / oracle.power_lipschitz(og, factors[k], 40) for k in order])
    a = synth.momentum_table(len(order))
    say("pnp_step large factors", form)
    x, hist = run_gpu(plan, gd, b, sched_g, eta, a, history=True)
    ref, rhist = oracle.pnp_run(og, b.astype(np.float64), sched_o, eta, a, history=True)
    for t in range(len(order)):
        got = hist[t].reshape(ref.shape)
        assert rel(got, rhist[t]) <= 2e-5, (t, rel(got, rhist[t]))
    # chained steps pool y_t for the next stage after the denoiser: in its epilogue when the
    # factor divides the TV tile, else by a pooling launch of their own (30 and 24 divide neither)
    say("pnp_step large factors, chained and graph", form)
    np.testing.assert_array_equal(run_gpu(plan, gd, b, sched_g, eta, a, chained=True), x)
    np.testing.assert_array_equal(run_gpu(plan, gd, b, sched_g, eta, a, graph=True), x)


@pytest.mark.parametrize("lam,tv_iters,alpha", [(0.02, 8, 1.0), (0.01, 6, 0.7), (0.0, 5, 1.0), (0.01, 0, 0.8)])
def test_pnp_step_denoiser_settings(lam, tv_iters, alpha):
    """Fused steps with 6 to 8 TV steps (the deeper-halo denoiser), with lambda = 0 and with no TV
    step (the denoiser kernel then only relaxes and applies the momentum), as direct calls and as
    a graph (whose steps pool in the denoiser's epilogue)."""
    w, gd, og, xt, b = problem("pnp64")
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [2, 1])
    sched_g = [(0, None, 1.0)] * 3 + [(1, None, 1.0)] * 3
    sched_o = [(2, None, 1.0)] * 3 + [(1, None, 1.0)] * 3
    eta = np.full(6, 1.0 / oracle.power_lipschitz(og, 1, 40))
    a = synth.momentum_table(6)
    say("pnp_step denoiser", lam, tv_iters, alpha)
    x = run_gpu(plan, gd, b, sched_g, eta, a, alpha=alpha, lam=lam, tv_iters=tv_iters)
    ref = oracle.pnp_run(og, b.astype(np.float64), sched_o, eta, a, alpha=alpha, lam=lam, tv_iters=tv_iters)
    assert rel(x, ref) <= 2e-5, rel(x, ref)
    g = run_gpu(plan, gd, b, sched_g, eta, a, alpha=alpha, lam=lam, tv_iters=tv_iters, graph=True)
    np.testing.assert_array_equal(g, x)


def oracle_step(og, f):
    return 1.0 / oracle.power_lipschitz(og, f, 100)


def test_loop_pnp64_full_gradient_50_iterations():
    """Plain full-gradient PnP-ISTA at 64^2, 50 iterations: reconstruction within 1e-4."""
    w, gd, og, xt, b = problem("pnp64")
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [1])
    eta = np.full(50, oracle_step(og, 1))
    a = np.zeros(50)
    say("loop pnp64")
    x = run_gpu(plan, gd, b, [(0, None, 1.0)] * 50, eta, a)
    ref = oracle.pnp_run(og, b.astype(np.float64), [(1, None, 1.0)] * 50, eta, a)
    assert rel(x, ref) <= 1e-4, rel(x, ref)
    assert oracle.psnr(ref, xt) > 15.0


def test_loop_ms2g256_two_stage():
    """Two-stage sketched PnP at 256^2 (30 at f = 2, then 20 at f = 1), FISTA momentum."""
    w, gd, og, xt, b = problem("ms2g256")
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [2, 1])
    L2, L1 = oracle.power_lipschitz(og, 2, 60), oracle.power_lipschitz(og, 1, 60)
    T = 50
    eta = np.array([1 / L2] * 30 + [1 / L1] * 20)
    a = synth.momentum_table(T)
    say("loop ms2g256")
    x = run_gpu(plan, gd, b, [(0, None, 1.0)] * 30 + [(1, None, 1.0)] * 20, eta, a)
    ref = oracle.pnp_run(og, b.astype(np.float64), [(2, None, 1.0)] * 30 + [(1, None, 1.0)] * 20, eta, a)
    assert rel(x, ref) <= 1e-4, rel(x, ref)


def test_loop_ms2g512_subsets_multistage(tmp_path):
    """Multi-stage sketched PnP-SGD at 512^2, 1 of 8 view subsets, f = 4, 2, 1 (4 each), with the
    built-in launch shapes and with those the benchmark runs (the shipped autotuner cache)."""
    w, gd, og, xt, b = problem("ms2g512")
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [4, 2, 1])
    seq = synth.subset_sequence(3000 * 3, 12, 8)
    eta_k = {4: 1 / oracle.power_lipschitz(og, 4, 30), 2: 1 / oracle.power_lipschitz(og, 2, 30)}
    eta_k[1] = eta_k[2]
    fs = [4] * 4 + [2] * 4 + [1] * 4
    sched_o = [(fs[t], synth.subset_views(seq[t], 8, gd["n_views"]), 8.0) for t in range(12)]
    sched_g = [({4: 0, 2: 1, 1: 2}[fs[t]], sched_o[t][1], 8.0) for t in range(12)]
    eta = np.array([eta_k[f] for f in fs])
    a = synth.momentum_table(12)
    say("loop ms2g512")
    x = run_gpu(plan, gd, b, sched_g, eta, a)
    ref = oracle.pnp_run(og, b.astype(np.float64), sched_o, eta, a)
    assert rel(x, ref) <= 1e-4, rel(x, ref)
    cache = tmp_path / "launch_configs.txt"
    shutil.copyfile(os.path.join(ROOT, "paper_2203_07308_amd", "tuned", "mi355x_launch_configs.txt"), cache)
    plan.autotune(n_sel=gd["n_views"] // 8, cache_path=str(cache))
    say("loop ms2g512 tuned", [plan.get_config(k, gd["n_views"] // 8) for k in range(3)])
    x = run_gpu(plan, gd, b, sched_g, eta, a)
    assert rel(x, ref) <= 1e-4, rel(x, ref)


def test_loop_ms2g256_two_stage_scatter_backprojection():
    """The 256^2 two-stage loop with the scatter back-projector at both stages (block sides 16
    and 32) and the LDS-staged projector at the 128^2 stage, direct and as a graph, against the
    oracle's loop."""
    w, gd, og, xt, b = problem("ms2g256")
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [2, 1])
    plan.set_config(0, dict(fp_seg=0, bp_px=16, bp_vg=16, tv_tile=0, fp_lds=2))
    plan.set_config(1, dict(fp_seg=0, bp_px=32, bp_vg=16, tv_tile=0))
    L2, L1 = oracle.power_lipschitz(og, 2, 60), oracle.power_lipschitz(og, 1, 60)
    eta = np.array([1 / L2] * 30 + [1 / L1] * 20)
    a = synth.momentum_table(50)
    sched_g = [(0, None, 1.0)] * 30 + [(1, None, 1.0)] * 20
    say("loop ms2g256 scatter")
    x = run_gpu(plan, gd, b, sched_g, eta, a)
    ref = oracle.pnp_run(og, b.astype(np.float64), [(2, None, 1.0)] * 30 + [(1, None, 1.0)] * 20, eta, a)
    assert rel(x, ref) <= 1e-4, rel(x, ref)
    np.testing.assert_array_equal(run_gpu(plan, gd, b, sched_g, eta, a, graph=True), x)


def test_loop_widefan_two_stage_subsets():
    """Sketched PnP-SGD on the 85-degree fan: 8 iterations at f = 2, then 8 at f = 1, 1 of 3 view
    subsets (sigma = 3), FISTA momentum, against the oracle's loop."""
    gd = make_geom(**GEOMS["widefan"])
    og = oracle.Geometry(**gd)
    xt = ellipse_image(gd["ny"], gd["nx"], 21)
    ax = oracle.fp(og, xt.astype(np.float64))
    b = (ax + 0.01 * ax.max() * synth.standard_normal(77, ax.shape)).astype(np.float32)
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [2, 1])
    L2, L1 = oracle.power_lipschitz(og, 2, 40), oracle.power_lipschitz(og, 1, 40)
    T = 16
    seq = synth.subset_sequence(91, T, 3)
    fs = [2] * 8 + [1] * 8
    sched_o = [(fs[t], synth.subset_views(seq[t], 3, gd["n_views"]), 3.0) for t in range(T)]
    sched_g = [({2: 0, 1: 1}[fs[t]], sched_o[t][1], 3.0) for t in range(T)]
    eta = np.array([1 / L2 if f == 2 else 1 / L1 for f in fs])
    a = synth.momentum_table(T)
    say("loop widefan")
    x = run_gpu(plan, gd, b, sched_g, eta, a)
    ref = oracle.pnp_run(og, b.astype(np.float64), sched_o, eta, a)
    assert rel(x, ref) <= 1e-4, rel(x, ref)


def test_graph_replay_equals_eager_and_is_deterministic():
    w, gd, og, xt, b = problem("pnp64")
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [2, 1])
    sub = synth.subset_views(2, 4, gd["n_views"])
    sched = [(0, sub, 4.0)] * 3 + [(1, None, 1.0)] * 3
    eta = np.full(6, 1e-4)
    a = synth.momentum_table(6)
    say("graph vs eager")
    e1 = run_gpu(plan, gd, b, sched, eta, a)
    e2 = run_gpu(plan, gd, b, sched, eta, a)
    g1 = run_gpu(plan, gd, b, sched, eta, a, graph=True)
    np.testing.assert_array_equal(e1, e2)
    np.testing.assert_array_equal(e1, g1)
    # direct calls with the graph's pooling hand-over and kernel timing events: same bits
    evs = []
    c1 = run_gpu(plan, gd, b, sched, eta, a, chained=True, events=evs)
    np.testing.assert_array_equal(e1, c1)
    torch.cuda.synchronize()
    for ev in evs:
        for k in (0, 2, 4):
            ms = ev[k].elapsed_time(ev[k + 1])
            assert 0.0 < ms < 50.0, ms


def test_step_stamps_mark_each_step_end_and_change_nothing():
    """With stamps, each step records the device clock when its denoiser kernel finished: after the
    start mark, strictly increasing, spanning no more than the events around the run; the iterates are
    bitwise those of the unstamped run (direct calls and graph)."""
    w, gd, og, xt, b = problem("pnp64")
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [2, 1])
    sub = synth.subset_views(0, 4, gd["n_views"])
    sched = [(0, sub, 4.0)] * 3 + [(1, None, 1.0)] * 3
    eta = np.full(6, 1e-4)
    a = synth.momentum_table(6)
    khz = fbpnp.clock_khz()
    assert khz > 0
    say("step stamps")
    ref = run_gpu(plan, gd, b, sched, eta, a, graph=True)
    for graph in (False, True):
        stamps = torch.zeros(7, dtype=torch.int64, device="cuda")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        out = run_gpu(plan, gd, b, sched, eta, a, graph=graph, stamps=stamps)
        e1.record()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out, ref)
        st = host(stamps).astype(np.int64)
        assert st[0] > 0 and (np.diff(st) > 0).all(), st
        span_ms = (st[-1] - st[0]) / khz
        assert 0.0 < span_ms <= e0.elapsed_time(e1) * 1.05 + 0.01, (span_ms, e0.elapsed_time(e1))


def test_side_stream_equals_default_stream():
    """The same schedule issued on a non-default stream, as direct calls and as a graph, gives the same
    bits as on the default stream: every launch and copy of a step goes to the caller's stream."""
    w, gd, og, xt, b = problem("pnp64")
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [2, 1])
    sub = synth.subset_views(1, 4, gd["n_views"])
    sched = [(0, sub, 4.0)] * 3 + [(1, None, 1.0)] * 3
    eta = np.full(6, 1e-4)
    a = synth.momentum_table(6)
    say("side stream")
    ref = run_gpu(plan, gd, b, sched, eta, a)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        direct = run_gpu(plan, gd, b, sched, eta, a, chained=True)
        graph = run_gpu(plan, gd, b, sched, eta, a, graph=True)
    side.synchronize()
    np.testing.assert_array_equal(direct, ref)
    np.testing.assert_array_equal(graph, ref)


def test_power_lipschitz_matches_oracle():
    gd = make_geom(**GEOMS["64"])
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [1, 2])
    og = oracle.Geometry(**gd)
    for s, f in enumerate([1, 2]):
        say("power", f)
        L = fbpnp.power_lipschitz(plan, s, 30)
        ref = oracle.power_lipschitz(og, f, 30)
        assert abs(L - ref) <= 1e-4 * ref, (L, ref)


def test_invalid_calls_raise_before_launch():
    gd = make_geom(**GEOMS["64"])
    with pytest.raises(fbpnp.FbError):
        fbpnp.Plan(fbpnp.Geometry(**gd), [64])  # factors above 32 are refused
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [1])
    x = torch.zeros(64 * 64, device="cuda")
    y = torch.zeros(90 * 96, device="cuda")
    with pytest.raises(fbpnp.FbError):
        fbpnp._check(fbpnp.load().fanbeam_fp(plan.handle, 3, fbpnp._ptr(x), fbpnp._ptr(y), None, 90, None))
    with pytest.raises(fbpnp.FbError):
        fbpnp._check(fbpnp.load().fanbeam_fp(plan.handle, 0, fbpnp._ptr(x), fbpnp._ptr(y), None, 91, None))
    with pytest.raises(fbpnp.FbError):  # an empty view selection is refused, not launched
        fbpnp._check(fbpnp.load().fanbeam_bp(plan.handle, 0, fbpnp._ptr(y), fbpnp._ptr(x), None, 0, 1.0, None))
    with pytest.raises(ValueError):
        fbpnp.fanbeam_fp(plan, 0, x[:10], y)
