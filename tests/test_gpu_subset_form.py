"""pnp_step with an interleaved view subset given as (subset, n_sub), whose view
indices the kernels compute (Algorithm 1, Option 2), against the same subsets
given as device view lists: the results must be bitwise equal, directly, as a
graph, in the variance-reduced modes and in reverse mode."""
import numpy as np
import pytest
import torch

from random_geometry import random_geometry
from paper_2203_07308_amd import fbpnp, synth

pytestmark = pytest.mark.gpu

FIXED = dict(nx=70, ny=52, pixel_mm=1.0, n_views=90, n_bins=96, sod_mm=200.0, sdd_mm=400.0,
             det_pitch_mm=1.6, det_offset_mm=0.0, angle0_rad=0.0, angle_step_rad=None)


def _setup(gd, factors, seed):
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), factors)
    rng = np.random.default_rng(seed)
    V, nb = gd["n_views"], gd["n_bins"]
    b = torch.from_numpy(rng.random(V * nb).astype(np.float32)).cuda()
    eta = 0.5 / max(fbpnp.power_lipschitz(plan, 0, 20), 1e-12)
    return plan, b, eta


def _steps(plan, b, x, y, eta, sched, n_sub, form, keep, **kw):
    V = plan.geom.n_views
    steps = []
    for t, (k, s) in enumerate(sched):
        if form == "list":
            v = torch.from_numpy(synth.subset_views(s, n_sub, V)).cuda()
            keep.append(v)
            sel = dict(views=v)
        else:
            sel = dict(subset=(s, n_sub))
        steps.append(fbpnp.pnp_args(plan, k, b, y, x, x, y, eta, 0.3 + 0.1 * t, sigma=float(n_sub), **sel, **kw))
    return steps


def _run(plan, b, eta, sched, n_sub, form, graph):
    npix = plan.geom.nx * plan.geom.ny
    x = torch.zeros(npix, device="cuda")
    y = torch.zeros(npix, device="cuda")
    keep = []
    steps = _steps(plan, b, x, y, eta, sched, n_sub, form, keep)
    if graph:
        g = fbpnp.Graph(plan, steps)
        g.launch()
        torch.cuda.synchronize()
        g.close()
    else:
        for a in steps:
            fbpnp.pnp_step(plan, a)
        torch.cuda.synchronize()
    return x.cpu(), y.cpu()


def _cases():
    out = [("fixed", FIXED, [2, 1], 4), ("fixed8", FIXED, [1], 8), ("fixed3", dict(FIXED, nx=72, ny=54), [3, 1], 3)]
    for seed in range(6):
        gd, f = random_geometry(7100 + seed)
        n_sub = 2 + seed % 3
        if gd["n_views"] >= n_sub:
            out.append((f"random{seed}", gd, [f, 1] if f > 1 else [1], n_sub))
    return out


@pytest.mark.parametrize("graph", [False, True], ids=["direct", "graph"])
@pytest.mark.parametrize("name,gd,factors,n_sub", _cases(), ids=[c[0] for c in _cases()])
def test_subset_form_matches_view_lists(name, gd, factors, n_sub, graph):
    plan, b, eta = _setup(gd, factors, 11)
    last = len(factors) - 1
    # every subset once, including the shorter ones when n_sub does not divide n_views
    sched = [(0 if t < n_sub // 2 + 1 else last, t % n_sub) for t in range(n_sub + 1)]
    xl, yl = _run(plan, b, eta, sched, n_sub, "list", graph)
    xc, yc = _run(plan, b, eta, sched, n_sub, "subset", graph)
    assert torch.isfinite(xl).all() and xl.abs().max() > 0
    assert torch.equal(xl, xc) and torch.equal(yl, yc)


def test_subset_of_one_is_every_view():
    plan, b, eta = _setup(FIXED, [2], 5)
    npix = plan.geom.nx * plan.geom.ny
    res = []
    for kw in (dict(), dict(subset=(0, 1))):
        x = torch.zeros(npix, device="cuda")
        y = torch.zeros(npix, device="cuda")
        for t in range(3):
            fbpnp.pnp_step(plan, fbpnp.pnp_args(plan, 0, b, y, x, x, y, eta, 0.2, **kw))
        torch.cuda.synchronize()
        res.append(x.cpu())
    assert torch.equal(res[0], res[1])


def test_subset_form_variance_reduced():
    """SVRG (snapshot with every view, then corrected subset steps) in both forms."""
    plan, b, eta = _setup(FIXED, [2], 9)
    n_sub = 4
    V, nb = FIXED["n_views"], FIXED["n_bins"]
    nys, nxs = plan.coarse_shape(0)
    out = []
    for form in ("list", "subset"):
        npix = plan.geom.nx * plan.geom.ny
        x = torch.zeros(npix, device="cuda")
        y = torch.zeros(npix, device="cuda")
        sp = torch.zeros(V * nb, device="cuda")
        sg = torch.zeros(nxs * nys, device="cuda")
        snap = fbpnp.pnp_args(plan, 0, b, y, x, x, y, eta, 0.0, vr_mode=1, snap_proj=sp, snap_grad=sg)
        fbpnp.pnp_step(plan, snap)
        keep = []
        for a in _steps(plan, b, x, y, eta, [(0, s) for s in (2, 0, 3)], n_sub, form, keep, vr_mode=2,
                        snap_proj=sp, snap_grad=sg):
            fbpnp.pnp_step(plan, a)
        torch.cuda.synchronize()
        out.append(x.cpu())
    assert torch.equal(out[0], out[1])


def test_subset_form_reverse_mode():
    plan, b, eta = _setup(FIXED, [2, 1], 13)
    npix = plan.geom.nx * plan.geom.ny
    rng = np.random.default_rng(3)
    x0 = torch.from_numpy(rng.random(npix).astype(np.float32)).cuda()
    y0 = torch.from_numpy(rng.random(npix).astype(np.float32)).cuda()
    xbar = torch.from_numpy(rng.standard_normal(npix).astype(np.float32)).cuda()
    ybar = torch.from_numpy(rng.standard_normal(npix).astype(np.float32)).cuda()
    ws = fbpnp.pnp_vjp_workspace(plan)
    res = []
    for form in ("list", "subset"):
        x1 = torch.empty(npix, device="cuda")
        y1 = torch.empty(npix, device="cuda")
        keep = []
        a = _steps(plan, b, x0, y0, eta, [(1, 2)], 3, form, keep)[0]
        a.x_out, a.y_out = x1.data_ptr(), y1.data_ptr()
        xbp = torch.zeros(npix, device="cuda")
        ybp = torch.zeros(npix, device="cuda")
        eb = torch.zeros(1, device="cuda")
        fbpnp.pnp_step_vjp(plan, a, xbar, ybar, xbp, ybp, eb, ws)
        torch.cuda.synchronize()
        res.append((xbp.cpu(), ybp.cpu(), eb.cpu()))
    for u, v in zip(*res):
        assert torch.equal(u, v)
    assert res[0][1].abs().max() > 0


def test_subset_form_rejects_bad_selections():
    plan, b, eta = _setup(FIXED, [1], 1)
    npix = plan.geom.nx * plan.geom.ny
    x = torch.zeros(npix, device="cuda")
    y = torch.zeros(npix, device="cuda")
    v = torch.arange(0, 90, 4, dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError):
        fbpnp.pnp_args(plan, 0, b, y, x, x, y, eta, 0.0, views=v, subset=(0, 4))

    def bad(**fields):
        a = fbpnp.pnp_args(plan, 0, b, y, x, x, y, eta, 0.0, subset=(1, 4))
        for k, val in fields.items():
            setattr(a, k, val)
        with pytest.raises(fbpnp.FbError):
            fbpnp.pnp_step(plan, a)

    bad(views=v.data_ptr())          # a list and a subset together
    bad(subset=4)                    # subset outside [0, n_sub)
    bad(subset=-1)
    bad(n_sel=22)                    # subset 1 of 4 holds 23 of the 90 views
    bad(n_sub=-2, subset=0)          # negative n_sub
    bad(n_sub=0, subset=1)           # a subset index without n_sub
    bad(n_sub=200, subset=150)       # a subset with no view
    torch.cuda.synchronize()
