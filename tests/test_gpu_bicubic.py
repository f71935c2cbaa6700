"""GPU parity of the bicubic sketch (the paper's resizing choice, Sec. 3) and of PnP
iterations that use it, against the FP64 oracle: S and U = S^T on several grids, the
two-stage sketched loop, graph capture, the power iteration, and argument checks."""
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


# the last three have stage axes of 1 to 4 pixels, shorter than the kernel's window of 4 f inputs,
# so the half-sample reflection folds more than once
@pytest.mark.parametrize("n,ny,factors", [(64, None, [2, 4]), (512, None, [4, 2]), (96, 60, [3, 2]), (16, None, [8]),
                                          (9, 3, [3]), (12, 6, [6, 3]), (10, None, [5])])
def test_bicubic_sketch_and_adjoint_match_oracle(n, ny, factors):
    g = synth.fan_geometry(n, 8)
    if ny is not None:
        g["ny"] = ny
    plan = fbpnp.Plan(fbpnp.Geometry(**g), factors)
    plan.set_sketch("bicubic")
    rng = np.random.default_rng(n)
    nyy = g["ny"]
    x = rng.random((nyy, n)).astype(np.float32)
    for k, f in enumerate(factors):
        say("bicubic sketch", n, nyy, f)
        v = torch.empty((nyy // f) * (n // f), device="cuda")
        plan.sketch_down(k, dev(x).reshape(-1), v)
        ref = oracle.sketch_down(x, f, "bicubic")
        assert rel(host(v).reshape(ref.shape), ref) <= 1e-6
        w = rng.standard_normal(ref.shape).astype(np.float32)
        up = torch.empty(nyy * n, device="cuda")
        plan.sketch_up(k, dev(w).reshape(-1), up)
        refu = oracle.sketch_up(w, f, "bicubic")
        assert rel(host(up).reshape(refu.shape), refu) <= 1e-6


def scenario_problem():
    sc = synth.SCENARIOS["sparse_view"]
    g = sc.geometry
    og = oracle.Geometry(**g)
    x = sc.phantom()
    b = sc.data(oracle.fp(og, x.astype(np.float64))).astype(np.float32)
    return sc, g, og, x, b


def run_bicubic(plan, g, b, sched, eta, a, sc, graph=False):
    npix = g["nx"] * g["ny"]
    xb = torch.zeros(npix, device="cuda")
    yb = torch.zeros(npix, device="cuda")
    bd = dev(b).reshape(-1)
    steps = [fbpnp.pnp_args(plan, k, bd, yb, xb, xb, yb, float(eta[t]), float(a[t]), None, 1.0, sc.alpha, sc.lam,
                            sc.tau, sc.tv_iters) for t, k in enumerate(sched)]
    if graph:
        gr = fbpnp.Graph(plan, steps)
        gr.launch()
    else:
        fbpnp.chain_steps(steps)
        for st in steps:
            fbpnp.pnp_step(plan, st)
    return host(xb).reshape(g["ny"], g["nx"])


def test_bicubic_two_stage_loop_matches_oracle_and_graph():
    """The paper's two-stage schedule with its bicubic sketch: 5 iterations at f = 4,
    5 at f = 2, then 2 full iterations (stage hand-over into f = 1 included)."""
    sc, g, og, x, b = scenario_problem()
    plan = fbpnp.Plan(fbpnp.Geometry(**g), [4, 2, 1])
    plan.set_sketch("bicubic")
    L = {f: oracle.power_lipschitz(og, f, 40, sketch="bicubic") for f in (4, 2, 1)}
    fs = [4] * 5 + [2] * 5 + [1] * 2
    sched = [{4: 0, 2: 1, 1: 2}[f] for f in fs]
    eta = np.array([1.0 / L[f] for f in fs])
    a = synth.momentum_table(len(fs))
    say("bicubic loop")
    got = run_bicubic(plan, g, b, sched, eta, a, sc)
    ref = oracle.pnp_run(og, b.astype(np.float64), [(f, None, 1.0) for f in fs], eta, a, sc.alpha, sc.lam,
                         sc.tv_iters, sc.tau, sketch="bicubic")
    assert rel(got, ref) <= 1e-4, rel(got, ref)
    pool = oracle.pnp_run(og, b.astype(np.float64), [(f, None, 1.0) for f in fs], eta, a, sc.alpha, sc.lam,
                          sc.tv_iters, sc.tau)
    assert rel(pool, ref) > 1e-3  # the bicubic sketch is what was compared
    say("bicubic graph")
    np.testing.assert_array_equal(got, run_bicubic(plan, g, b, sched, eta, a, sc, graph=True))


def test_bicubic_power_iteration_matches_oracle():
    sc, g, og, x, b = scenario_problem()
    plan = fbpnp.Plan(fbpnp.Geometry(**g), [4, 2])
    plan.set_sketch("bicubic")
    for k, f in enumerate((4, 2)):
        say("bicubic power", f)
        L = fbpnp.power_lipschitz(plan, k, 30)
        ref = oracle.power_lipschitz(og, f, 30, sketch="bicubic")
        assert abs(L - ref) <= 1e-4 * ref, (L, ref)


def test_bicubic_argument_checks():
    g = synth.fan_geometry(64, 30)
    plan = fbpnp.Plan(fbpnp.Geometry(**g), [2])
    plan.set_sketch("bicubic")
    npix = 64 * 64
    x = torch.zeros(npix, device="cuda")
    b = torch.zeros(30 * 96, device="cuda")
    sp, sg = torch.zeros(30 * 96, device="cuda"), torch.zeros(32 * 32, device="cuda")
    with pytest.raises(fbpnp.FbError):
        fbpnp.pnp_step(plan, fbpnp.pnp_args(plan, 0, b, x, x, x, x, 1e-4, 0.0, vr_mode=1, snap_proj=sp,
                                            snap_grad=sg))
    with pytest.raises(fbpnp.FbError):
        fbpnp.pnp_step_vjp(plan, fbpnp.pnp_args(plan, 0, b, x, x, x, x, 1e-4, 0.0), x, x, torch.empty_like(x),
                           torch.empty_like(x), torch.zeros(1, device="cuda"), fbpnp.pnp_vjp_workspace(plan))
    with pytest.raises(KeyError):
        plan.set_sketch("lanczos")
    plan.set_sketch("pool")  # back to pooling: the step runs
    fbpnp.pnp_step(plan, fbpnp.pnp_args(plan, 0, b, x, x, x, torch.zeros_like(x), 1e-4, 0.0))


@pytest.mark.parametrize("seed", range(12))
def test_bicubic_steps_on_random_geometries(seed):
    """Three fused steps with the bicubic sketch, as a graph, on seeded random geometries with a
    pooling factor (grids from a few to 80 pixels a side, close and far sources), against the oracle."""
    g, f = random_geometry(40 + seed)
    if f == 1:
        f = 1 if g["nx"] % 2 or g["ny"] % 2 else 2
    og = oracle.Geometry(**g)
    plan = fbpnp.Plan(fbpnp.Geometry(**g), [f, 1] if f > 1 else [1])
    plan.set_sketch("bicubic")
    xt = np.random.default_rng(seed).random((g["ny"], g["nx"]))
    b = oracle.fp(og, xt).astype(np.float32)
    eta = np.full(3, 1.0 / oracle.power_lipschitz(og, f, 30, sketch="bicubic"))
    a = synth.momentum_table(3)
    say("bicubic random", seed, g["nx"], g["ny"], f)
    npix = g["nx"] * g["ny"]
    xb = torch.zeros(npix, device="cuda")
    yb = torch.zeros(npix, device="cuda")
    bd = dev(b).reshape(-1)
    steps = [fbpnp.pnp_args(plan, 0, bd, yb, xb, xb, yb, float(eta[t]), float(a[t])) for t in range(3)]
    gr = fbpnp.Graph(plan, steps)
    gr.launch()
    torch.cuda.synchronize()
    gr.close()
    got = host(xb).reshape(g["ny"], g["nx"])
    ref = oracle.pnp_run(og, b.astype(np.float64), [(f, None, 1.0)] * 3, eta, a, sketch="bicubic")
    assert rel(got, ref) <= 2e-5, rel(got, ref)
