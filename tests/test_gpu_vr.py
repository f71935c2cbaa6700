"""GPU parity of the variance-reduced (SVRG) minibatch gradient over view subsets
against the FP64 oracle: snapshot outputs, loops at 64^2 and two-stage 256^2, graph
capture, and argument checks."""
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


def problem(name):
    w = synth.WORKLOADS[name]
    gd = w.geometry
    og = oracle.Geometry(**gd)
    xt = synth.phantom(w)
    ax = oracle.fp(og, xt.astype(np.float64))
    b = synth.add_noise(ax, synth.standard_normal(synth.noise_seed(w), ax.shape), w.noise_kind,
                        w.noise_level).astype(np.float32)
    return gd, og, xt, b


def vr_schedule(stages, n_sub, seed):
    """[(stage index, f, mode, subset)]: an epoch of n_sub iterations starts with a snapshot."""
    out, t = [], 0
    seq = synth.subset_sequence(seed, sum(n for _, n in stages), n_sub)
    for k, (f, n) in enumerate(stages):
        for i in range(n):
            out.append((k, f, 1 if i % n_sub == 0 else 2, int(seq[t])))
            t += 1
    return out


def run(gd, b, stages, sched, eta, a, n_sub, graph=False):
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [f for f, _ in stages])
    V, B = gd["n_views"], gd["n_bins"]
    npix = gd["nx"] * gd["ny"]
    bd = dev(b).reshape(-1)
    x = torch.zeros(npix, device="cuda")
    y = torch.zeros(npix, device="cuda")
    snaps = [(torch.zeros(V * B, device="cuda"), torch.zeros((gd["ny"] // f) * (gd["nx"] // f), device="cuda"))
             for f, _ in stages]
    keep, steps = [], []
    for t, (k, f, mode, s) in enumerate(sched):
        views = None if mode == 1 else dev(synth.subset_views(s, n_sub, V), np.int32)
        keep.append(views)
        sigma = 1.0 if mode == 1 else float(n_sub)
        steps.append(fbpnp.pnp_args(plan, k, bd, y, x, x, y, float(eta[t]), float(a[t]), views, sigma,
                                    vr_mode=mode, snap_proj=snaps[k][0], snap_grad=snaps[k][1]))
    if graph:
        g = fbpnp.Graph(plan, steps)
        g.launch()
    else:
        fbpnp.chain_steps(steps)
        for st in steps:
            fbpnp.pnp_step(plan, st)
    return host(x).reshape(gd["ny"], gd["nx"]), snaps, plan


def oracle_run(og, b, sched, eta, a, n_sub, V):
    so = [(f, None if mode == 1 else synth.subset_views(s, n_sub, V), 1.0 if mode == 1 else float(n_sub))
          for _, f, mode, s in sched]
    return oracle.pnp_run(og, b.astype(np.float64), so, eta, a, vr=[m for _, _, m, _ in sched])


def test_snapshot_records_projection_and_coarse_gradient():
    gd, og, xt, b = problem("ms2g256")
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [2])
    V, B = gd["n_views"], gd["n_bins"]
    y0 = (0.5 * xt).astype(np.float32)
    yd = dev(y0).reshape(-1)
    x = yd.clone()
    sp = torch.zeros(V * B, device="cuda")
    sg = torch.zeros(128 * 128, device="cuda")
    say("svrg snapshot")
    fbpnp.pnp_step(plan, fbpnp.pnp_args(plan, 0, dev(b).reshape(-1), yd, x, x.clone(), yd.clone(), 1e-6, 0.0,
                                        vr_mode=1, snap_proj=sp, snap_grad=sg))
    v = oracle.down(y0.astype(np.float64), 2)
    ref_p = oracle.fp(og, v, f=2)
    got_p = host(sp).reshape(ref_p.shape)
    per_view = np.linalg.norm(got_p - ref_p, axis=1) / np.linalg.norm(ref_p, axis=1)
    assert per_view.max() <= 1e-5
    ref_g = oracle.bp(og, ref_p - b.astype(np.float64), f=2)
    assert rel(host(sg).reshape(ref_g.shape), ref_g) <= 2e-5


def test_svrg_loop_matches_oracle_64():
    gd, og, xt, b = problem("pnp64")
    stages = [(1, 12)]
    sched = vr_schedule(stages, 3, 31)
    L = oracle.power_lipschitz(og, 1, 60)
    eta = np.full(12, 1.0 / L)
    a = synth.momentum_table(12)
    say("svrg loop 64")
    got, _, _ = run(gd, b, stages, sched, eta, a, 3)
    ref = oracle_run(og, b, sched, eta, a, 3, gd["n_views"])
    assert rel(got, ref) <= 1e-4, rel(got, ref)


def test_svrg_two_stage_256_matches_oracle_and_graph():
    gd, og, xt, b = problem("ms2g256")
    stages = [(2, 8), (1, 8)]
    sched = vr_schedule(stages, 4, 41)
    L2, L1 = oracle.power_lipschitz(og, 2, 60), oracle.power_lipschitz(og, 1, 60)
    eta = np.array([1 / L2] * 8 + [1 / L1] * 8)
    a = synth.momentum_table(16)
    say("svrg two-stage 256")
    got, _, _ = run(gd, b, stages, sched, eta, a, 4)
    ref = oracle_run(og, b, sched, eta, a, 4, gd["n_views"])
    assert rel(got, ref) <= 1e-4, rel(got, ref)
    say("svrg graph")
    gg, _, _ = run(gd, b, stages, sched, eta, a, 4, graph=True)
    np.testing.assert_array_equal(got, gg)


@pytest.mark.parametrize("seed", range(6))
def test_svrg_on_random_geometries(seed):
    """SVRG over 3 view subsets on seeded random geometries (a coarse stage when the grid allows one,
    then f = 1; 6 iterations each), direct and as a graph, against the oracle."""
    gd, f = random_geometry(200 + seed)
    og = oracle.Geometry(**gd)
    stages = [(f, 6), (1, 6)] if f > 1 else [(1, 6)]
    n_sub = 3
    sched = vr_schedule(stages, n_sub, 51 + seed)
    L = {ff: oracle.power_lipschitz(og, ff, 30) for ff, _ in stages}
    eta = np.array([0.5 / L[ff] for _, ff, _, _ in sched])
    a = synth.momentum_table(len(sched))
    b = oracle.fp(og, np.random.default_rng(seed).random((gd["ny"], gd["nx"]))).astype(np.float32)
    say("svrg random", seed, gd["nx"], gd["ny"], gd["n_views"], f)
    got, _, _ = run(gd, b, stages, sched, eta, a, n_sub)
    ref = oracle_run(og, b, sched, eta, a, n_sub, gd["n_views"])
    assert rel(got, ref) <= 1e-4, rel(got, ref)
    gg, _, _ = run(gd, b, stages, sched, eta, a, n_sub, graph=True)
    np.testing.assert_array_equal(got, gg)


def test_svrg_argument_checks():
    gd, og, xt, b = problem("pnp64")
    plan = fbpnp.Plan(fbpnp.Geometry(**gd), [1])
    npix = 64 * 64
    x = torch.zeros(npix, device="cuda")
    bd = dev(b).reshape(-1)
    sp = torch.zeros(90 * 96, device="cuda")
    sg = torch.zeros(npix, device="cuda")
    sub = dev(synth.subset_views(0, 3, 90), np.int32)
    with pytest.raises(fbpnp.FbError):  # a snapshot needs every view
        fbpnp.pnp_step(plan, fbpnp.pnp_args(plan, 0, bd, x, x, x, x, 1e-4, 0.0, sub, 3.0, vr_mode=1,
                                            snap_proj=sp, snap_grad=sg))
    # ... each once: a list of n_views entries with repeats would leave rows of snap_proj stale
    rep = dev(np.repeat(np.arange(45, dtype=np.int32), 2), np.int32)
    with pytest.raises(fbpnp.FbError):
        fbpnp.pnp_step(plan, fbpnp.pnp_args(plan, 0, bd, x, x, x, x, 1e-4, 0.0, rep, 1.0, vr_mode=1,
                                            snap_proj=sp, snap_grad=sg))
    a = fbpnp.pnp_args(plan, 0, bd, x, x, x, x, 1e-4, 0.0, vr_mode=2, snap_proj=sp, snap_grad=sg)
    a.snap_grad = None
    with pytest.raises(fbpnp.FbError):
        fbpnp.pnp_step(plan, a)
    ws = fbpnp.pnp_vjp_workspace(plan)
    a = fbpnp.pnp_args(plan, 0, bd, x, x, x, x, 1e-4, 0.0, vr_mode=2, snap_proj=sp, snap_grad=sg)
    with pytest.raises(fbpnp.FbError):
        fbpnp.pnp_step_vjp(plan, a, x, x, torch.empty_like(x), torch.empty_like(x),
                           torch.zeros(1, device="cuda"), ws)
