"""GPU parity of the reverse mode: tv_prox_vjp, pnp_step_vjp and the UnrolledPnP autograd
function against the FP64 oracle's adjoint (orc_pnp_vjp, itself pinned by central
differences) and against central finite differences of the oracle's forward loop.

Tolerances: TV-prox VJP 1e-4 relative L2 (FP32 recomputation of the dual iterates,
whose normalisation derivative amplifies rounding where |grad| is small); unrolled
gradients 1e-3 relative, the differentiation workload's stated bound.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from random_geometry import random_geometry
from paper_2203_07308_amd import fbpnp, synth
from paper_2203_07308_amd.autograd import StepSpec, unrolled_pnp

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


@pytest.mark.parametrize("shape,lam,iters,alpha", [((64, 64), 0.01, 5, 1.0), ((37, 70), 0.05, 3, 0.6),
                                                   ((128, 96), 0.02, 5, 1.0),
                                                   # several 32 x 32 tiles of the one-launch sweep, ragged edges
                                                   ((100, 70), 0.02, 5, 1.0), ((65, 129), 0.03, 4, 0.8),
                                                   ((33, 33), 0.05, 1, 1.0), ((1, 40), 0.02, 5, 1.0),
                                                   ((40, 1), 0.02, 2, 1.0), ((2, 3), 0.1, 5, 0.5),
                                                   ((256, 256), 0.01, 5, 1.0),
                                                   # more steps than one launch holds: the launch chain
                                                   ((70, 52), 0.02, 7, 1.0)])
def test_tv_prox_vjp_matches_oracle(shape, lam, iters, alpha):
    say("tv vjp", shape, lam, iters, alpha)
    rng = np.random.default_rng(3)
    n = max(shape)
    z = (synth.rasterise(synth.random_ellipses(4, 8, n), n)[: shape[0], : shape[1]]
         + 0.05 * rng.standard_normal(shape)).astype(np.float32)
    xb = rng.standard_normal(shape).astype(np.float32)
    zb = torch.empty(shape, device="cuda")
    fbpnp.tv_prox_vjp(dev(z), dev(xb), zb, lam, iters, 0.125, alpha)
    ref = oracle.tv_relax_vjp(z.astype(np.float64), xb.astype(np.float64), lam, iters, 0.125, alpha)
    got = host(zb)
    assert rel(got, ref) <= 1e-4, rel(got, ref)
    # no cell (tile edges included) is far off
    assert np.max(np.abs(got - ref)) <= 1e-4 * np.max(np.abs(ref)), np.max(np.abs(got - ref))


def make_problem(n, V, nb, seed, nslices=1):
    gd = synth.fan_geometry(n, V, nb)
    og = oracle.Geometry(**gd)
    xts, bs = [], []
    for s in range(nslices):
        xt = synth.rasterise(synth.random_ellipses(seed + s, 12, n), n)
        ax = oracle.fp(og, xt)
        eps = synth.standard_normal(seed + 100 + s, ax.shape)
        bs.append(synth.add_noise(ax, eps, "gaussian", 0.01).astype(np.float32))
        xts.append(xt)
    return gd, og, xts, bs


def schedule(gd, n_f2, n_f1, subsets, fc=2):
    """Two-stage schedule (f = fc, default 2, then f = 1) with FISTA momentum and optional subsets."""
    T = n_f2 + n_f1
    a = synth.momentum_table(T)
    seq = synth.subset_sequence(77, T, subsets) if subsets else None
    sched_o, specs = [], []
    for t in range(T):
        f, stage = (fc, 0) if t < n_f2 else (1, 1)
        views = None if seq is None else synth.subset_views(int(seq[t]), subsets, gd["n_views"])
        sigma = float(subsets) if subsets else 1.0
        sched_o.append((f, views, sigma))
        specs.append(StepSpec(stage, None if views is None else dev(views, np.int32), sigma, float(a[t])))
    return sched_o, specs, a


def run_case(gd, og, xt, b, n_f2, n_f1, subsets, x0, eta, fc=2, tv_iters=5, alpha=1.0):
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [fc, 1])
    sched_o, specs, a = schedule(gd, n_f2, n_f1, subsets, fc)
    for st in specs:
        st.tv_iters, st.alpha = tv_iters, alpha
    x0_t = dev(x0).requires_grad_(True)
    eta_t = torch.tensor(eta, dtype=torch.float32, device="cuda", requires_grad=True)
    xT = unrolled_pnp(plan, dev(b).reshape(-1), specs, x0_t, eta_t)
    loss = 0.5 * ((xT - dev(xt)) ** 2).sum()
    loss.backward()
    g_x0, g_eta = host(x0_t.grad), host(eta_t.grad)
    kw = dict(tv_iters=tv_iters, alpha=alpha)
    r_x0, r_eta = oracle.pnp_vjp(og, b.astype(np.float64), sched_o, eta, a,
                                 oracle.pnp_run(og, b.astype(np.float64), sched_o, eta, a, x0=x0, **kw) - xt, x0=x0,
                                 **kw)
    return g_x0, g_eta, r_x0, r_eta, sched_o, a


def test_unrolled_gradients_match_oracle_small():
    """10 unrolled two-stage iterations at 64^2 with view subsets and momentum."""
    gd, og, xts, bs = make_problem(64, 90, 96, 5)
    L = oracle.power_lipschitz(og, 1, 50)
    eta = np.full(10, 1.0 / L) * np.linspace(1.0, 0.8, 10)
    x0 = (0.5 * xts[0] + 0.05 * np.random.default_rng(9).random((64, 64))).astype(np.float32).astype(np.float64)
    say("unrolled 64")
    g_x0, g_eta, r_x0, r_eta, sched_o, a = run_case(gd, og, xts[0], bs[0], 5, 5, 3, x0, eta)
    assert rel(g_x0, r_x0) <= 1e-3, rel(g_x0, r_x0)
    assert rel(g_eta, r_eta) <= 1e-3, (g_eta, r_eta)
    # and central differences of the FP64 forward loop, h = 1e-3 (relative on eta)
    b64 = bs[0].astype(np.float64)
    loss = lambda x0_, eta_: 0.5 * np.sum((oracle.pnp_run(og, b64, sched_o, eta_, a, x0=x0_) - xts[0]) ** 2)  # noqa
    d = np.random.default_rng(11).standard_normal((64, 64))
    h = 1e-3
    fd = (loss(x0 + h * d, eta) - loss(x0 - h * d, eta)) / (2 * h)
    assert abs(fd - np.vdot(d, g_x0)) <= 1e-3 * abs(fd), (fd, np.vdot(d, g_x0))
    for t in (0, 4, 9):
        e = np.zeros(10)
        e[t] = h * eta[t]
        fd = (loss(x0, eta + e) - loss(x0, eta - e)) / (2 * e[t])
        assert abs(fd - g_eta[t]) <= 1e-3 * max(abs(fd), 1e-6 * np.abs(r_eta).max()), (t, fd, g_eta[t])


@pytest.mark.parametrize("tv_iters,alpha", [(7, 1.0), (3, 0.7)])
def test_unrolled_gradients_other_denoiser_step_counts(tv_iters, alpha):
    """6 unrolled iterations at 48^2 (3 at f = 2, 3 at f = 1, 1 of 3 view subsets) with 7 denoiser
    steps, whose reverse sweep is the launch chain with its workspace inside the step's own
    workspace, and with 3 steps and relaxation alpha < 1 (the one-launch sweep)."""
    gd, og, xts, bs = make_problem(48, 60, 72, 17)
    L = oracle.power_lipschitz(og, 1, 50)
    eta = np.full(6, 1.0 / L)
    x0 = (0.5 * xts[0]).astype(np.float32).astype(np.float64)
    say(f"unrolled 48, tv_iters {tv_iters}, alpha {alpha}")
    g_x0, g_eta, r_x0, r_eta, *_ = run_case(gd, og, xts[0], bs[0], 3, 3, 3, x0, eta, tv_iters=tv_iters, alpha=alpha)
    assert rel(g_x0, r_x0) <= 1e-3, rel(g_x0, r_x0)
    assert rel(g_eta, r_eta) <= 1e-3, (g_eta, r_eta)


@pytest.mark.parametrize("fc,subsets", [(2, 3), (1, 0), (3, 5)])
def test_step_vjp_with_stored_gradient_equals_recomputation(fc, subsets):
    """pnp_step stores the coarse gradient g (G = sigma U g) when grad is set; it matches the oracle's
    gradient, and pnp_step_vjp fed with it gives bitwise the results of the reverse step that
    recomputes g (same kernels and launch configuration)."""
    n, V, nb = 60, 45, 90
    gd, og, xts, bs = make_problem(n, V, nb, 23)
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [fc, 1])
    rng = np.random.default_rng(29)
    y_prev = (0.5 * xts[0] + 0.05 * rng.random((n, n))).astype(np.float32)
    x_prev = (0.4 * xts[0]).astype(np.float32)
    views = synth.subset_views(1, subsets, V) if subsets else None
    sigma = float(subsets) if subsets else 1.0
    eta = 1.0 / oracle.power_lipschitz(og, fc, 50)
    nys, nxs = plan.coarse_shape(0)
    g = torch.full((nys * nxs,), float("nan"), device="cuda")
    vd = None if views is None else dev(views, np.int32)
    b, yp, xp = dev(bs[0]).reshape(-1), dev(y_prev).reshape(-1), dev(x_prev).reshape(-1)
    xo, yo = torch.empty(n * n, device="cuda"), torch.empty(n * n, device="cuda")
    say(f"stored gradient, f = {fc}, subsets {subsets}")
    fbpnp.pnp_step(plan, fbpnp.pnp_args(plan, 0, b, yp, xp, xo, yo, eta, 0.3, vd, sigma, 0.9, grad=g))
    ref = oracle.grad(og, y_prev, bs[0], fc, views, sigma)[::fc, ::fc] * (fc * fc) / sigma
    assert rel(host(g).reshape(nys, nxs), ref) <= 1e-5, rel(host(g).reshape(nys, nxs), ref)
    xbar = dev(rng.standard_normal((n, n)).astype(np.float32)).reshape(-1)
    ybar = dev(rng.standard_normal((n, n)).astype(np.float32)).reshape(-1)
    ws = fbpnp.pnp_vjp_workspace(plan)
    out = []
    for grad in (g, None):
        args = fbpnp.pnp_args(plan, 0, b, yp, xp, xp, yp, eta, 0.3, vd, sigma, 0.9, grad=grad)
        r = (torch.empty(n * n, device="cuda"), torch.empty(n * n, device="cuda"), torch.zeros(1, device="cuda"))
        fbpnp.pnp_step_vjp(plan, args, xbar, ybar, r[0], r[1], r[2], ws)
        out.append([host(t) for t in r])
    for a_, b_ in zip(*out):
        assert np.array_equal(a_, b_)


def test_step_grad_checkpoint_is_refused_where_it_does_not_apply():
    """grad is stored for minibatch steps with the pooling sketch only."""
    gd, og, xts, bs = make_problem(32, 16, 48, 31)
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [2, 1])
    b = dev(bs[0]).reshape(-1)
    y = torch.zeros(32 * 32, device="cuda")
    x, xo, yo = y.clone(), y.clone(), y.clone()
    g = torch.zeros(16 * 16, device="cuda")
    snap_p = torch.zeros(16 * 48, device="cuda")
    args = fbpnp.pnp_args(plan, 0, b, y, x, xo, yo, 1e-3, 0.0, vr_mode=1, snap_proj=snap_p, snap_grad=g.clone(),
                          grad=g)
    with pytest.raises(fbpnp.FbError):
        fbpnp.pnp_step(plan, args)
    plan.set_sketch("bicubic")
    with pytest.raises(fbpnp.FbError):
        fbpnp.pnp_step(plan, fbpnp.pnp_args(plan, 0, b, y, x, xo, yo, 1e-3, 0.0, grad=g))


def test_unrolled_gradients_coarse_factor_three():
    """8 unrolled iterations at 60^2, 4 at f = 3 then 4 at f = 1, 1 of 5 view subsets: the reverse
    pass pools and back-projects with a factor that divides neither TV tile."""
    gd, og, xts, bs = make_problem(60, 45, 90, 13)
    L = oracle.power_lipschitz(og, 1, 50)
    eta = np.full(8, 1.0 / L)
    x0 = np.zeros((60, 60))
    say("unrolled 60, f = 3")
    g_x0, g_eta, r_x0, r_eta, *_ = run_case(gd, og, xts[0], bs[0], 4, 4, 5, x0, eta, fc=3)
    assert rel(g_x0, r_x0) <= 1e-3, rel(g_x0, r_x0)
    assert rel(g_eta, r_eta) <= 1e-3, (g_eta, r_eta)


@pytest.mark.parametrize("seed", range(6))
def test_unrolled_gradients_on_random_geometries(seed):
    """Gradients of 4 unrolled iterations (2 at the geometry's pooling factor, then 2 at f = 1, all
    views) with respect to x0 and every step size, on seeded random geometries, against the oracle's
    reverse pass."""
    gd, f = random_geometry(80 + seed)
    og = oracle.Geometry(**gd)
    factors = [f, 1] if f > 1 else [1]
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), factors)
    rng = np.random.default_rng(seed)
    xt = rng.random((gd["ny"], gd["nx"]))
    b = oracle.fp(og, xt).astype(np.float32)
    T = 4
    a = synth.momentum_table(T)
    stages = [0, 0, len(factors) - 1, len(factors) - 1]
    sched_o = [(factors[k], None, 1.0) for k in stages]
    specs = [StepSpec(k, None, 1.0, float(a[t])) for t, k in enumerate(stages)]
    eta = np.full(T, 0.5 / oracle.power_lipschitz(og, 1, 30))
    x0 = 0.3 * xt
    say("unrolled random", seed, gd["nx"], gd["ny"], f)
    x0_t = dev(x0).requires_grad_(True)
    eta_t = torch.tensor(eta, dtype=torch.float32, device="cuda", requires_grad=True)
    xT = unrolled_pnp(plan, dev(b).reshape(-1), specs, x0_t, eta_t)
    loss = 0.5 * ((xT - dev(xt)) ** 2).sum()
    loss.backward()
    r_x0, r_eta = oracle.pnp_vjp(og, b.astype(np.float64), sched_o, eta, a,
                                 oracle.pnp_run(og, b.astype(np.float64), sched_o, eta, a, x0=x0) - xt, x0=x0)
    assert rel(host(x0_t.grad), r_x0) <= 1e-3, rel(host(x0_t.grad), r_x0)
    assert rel(host(eta_t.grad), r_eta) <= 1e-3, (host(eta_t.grad), r_eta)


def test_unrolled_gradients_odd_sized_image():
    """A 65 x 63 image (an odd pixel count) with 5 TV steps: the reverse pass's double-precision
    partial sums follow an odd number of floats in its workspace, which must stay aligned."""
    gd = synth.fan_geometry(65, 40, 100)
    gd["ny"] = 63
    og = oracle.Geometry(**gd)
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [1])
    rng = np.random.default_rng(5)
    xt = rng.random((63, 65))
    b = oracle.fp(og, xt).astype(np.float32)
    T = 3
    a = synth.momentum_table(T)
    sched_o = [(1, None, 1.0)] * T
    specs = [StepSpec(0, None, 1.0, float(a[t])) for t in range(T)]
    eta = np.full(T, 0.5 / oracle.power_lipschitz(og, 1, 30))
    x0 = 0.3 * xt
    say("unrolled odd size 65 x 63")
    x0_t = dev(x0).requires_grad_(True)
    eta_t = torch.tensor(eta, dtype=torch.float32, device="cuda", requires_grad=True)
    xT = unrolled_pnp(plan, dev(b).reshape(-1), specs, x0_t, eta_t)
    (0.5 * ((xT - dev(xt)) ** 2).sum()).backward()
    r_x0, r_eta = oracle.pnp_vjp(og, b.astype(np.float64), sched_o, eta, a,
                                 oracle.pnp_run(og, b.astype(np.float64), sched_o, eta, a, x0=x0) - xt, x0=x0)
    assert rel(host(x0_t.grad), r_x0) <= 1e-3, rel(host(x0_t.grad), r_x0)
    assert rel(host(eta_t.grad), r_eta) <= 1e-3, (host(eta_t.grad), r_eta)


@pytest.mark.slow
def test_unrolled_gradients_differentiation_workload():
    """The differentiation workload's shape: 10 unrolled two-stage iterations (5 at f = 2,
    5 at f = 1) at 512^2, 360 views x 768 bins, all views; one slice checked against the
    oracle adjoint and central differences (h = 1e-3), and a batch of 8 slices against
    the sum of single-slice runs."""
    gd, og, xts, bs = make_problem(512, 360, 768, 21, nslices=8)
    eta = np.full(10, 1.0 / 356000.0)
    rng = np.random.default_rng(13)
    x0 = (0.5 * xts[0] + 0.05 * rng.random((512, 512))).astype(np.float32).astype(np.float64)
    say("unrolled 512 single slice")
    g_x0, g_eta, r_x0, r_eta, sched_o, a = run_case(gd, og, xts[0], bs[0], 5, 5, 0, x0, eta)
    assert rel(g_x0, r_x0) <= 1e-3, rel(g_x0, r_x0)
    assert rel(g_eta, r_eta) <= 1e-3, (g_eta, r_eta)
    b64 = bs[0].astype(np.float64)
    loss = lambda x0_, eta_: 0.5 * np.sum((oracle.pnp_run(og, b64, sched_o, eta_, a, x0=x0_) - xts[0]) ** 2)  # noqa
    d = rng.standard_normal((512, 512))
    h = 1e-3
    fd = (loss(x0 + h * d, eta) - loss(x0 - h * d, eta)) / (2 * h)
    assert abs(fd - np.vdot(d, g_x0)) <= 1e-3 * abs(fd), (fd, np.vdot(d, g_x0))
    e = np.zeros(10)
    e[9] = h * eta[9]
    fd = (loss(x0, eta + e) - loss(x0, eta - e)) / (2 * e[9])
    assert abs(fd - g_eta[9]) <= 1e-3 * abs(fd), (fd, g_eta[9])
    # batch of 8 slices: x0 gradients per slice, eta gradients summed over slices
    say("unrolled 512 batch of 8")
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [2, 1])
    _, specs, _ = schedule(gd, 5, 5, 0)
    x0s = np.stack([(0.5 * xt + 0.05 * rng.random((512, 512))) for xt in xts]).astype(np.float32)
    xb = dev(x0s).requires_grad_(True)
    et = torch.tensor(eta, dtype=torch.float32, device="cuda", requires_grad=True)
    bb = dev(np.stack([b.reshape(-1) for b in bs]))
    xT = unrolled_pnp(plan, bb, specs, xb, et)
    (0.5 * ((xT - dev(np.stack(xts))) ** 2).sum()).backward()
    gb, ge = host(xb.grad), host(et.grad)
    acc_eta = np.zeros(10)
    for s in (0, 7):
        x1 = dev(x0s[s]).requires_grad_(True)
        e1 = torch.tensor(eta, dtype=torch.float32, device="cuda", requires_grad=True)
        out = unrolled_pnp(plan, bb[s], specs, x1, e1)
        (0.5 * ((out - dev(xts[s])) ** 2).sum()).backward()
        np.testing.assert_array_equal(gb[s], host(x1.grad))
    for s in range(8):
        e1 = torch.tensor(eta, dtype=torch.float32, device="cuda", requires_grad=True)
        out = unrolled_pnp(plan, bb[s], specs, dev(x0s[s]), e1)
        (0.5 * ((out - dev(xts[s])) ** 2).sum()).backward()
        acc_eta += host(e1.grad)
    np.testing.assert_allclose(ge, acc_eta, rtol=1e-5)
