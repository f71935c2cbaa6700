"""Pins of the oracle's reverse mode (differentiation of unrolled PnP-MS2G iterations).

The forward maps are pinned elsewhere; here their vector-Jacobian products are checked
against central finite differences of those forward maps (error O(h^2)), and the
linear part against the adjoint identity.
"""
import numpy as np
import pytest

import oracle
from paper_2203_07308_amd import synth


@pytest.mark.parametrize("shape,lam,iters,alpha", [((9, 11), 0.05, 5, 1.0), ((12, 12), 0.01, 5, 1.0),
                                                    ((8, 10), 0.1, 3, 0.6), ((1, 7), 0.2, 4, 1.0)])
def test_tv_relax_vjp_matches_central_differences(shape, lam, iters, alpha):
    rng = np.random.default_rng(1)
    z = rng.random(shape) + np.linspace(0, 1, shape[1])[None, :]
    xbar = rng.standard_normal(shape)
    R = lambda u: (1 - alpha) * u + alpha * oracle.tv_prox(u, lam, iters)  # noqa: E731
    zbar = oracle.tv_relax_vjp(z, xbar, lam, iters, 0.125, alpha)
    for k in range(3):
        d = rng.standard_normal(shape)
        h = 1e-5
        fd = np.vdot(R(z + h * d) - R(z - h * d), xbar) / (2 * h)
        assert abs(fd - np.vdot(d, zbar)) <= 1e-7 * max(1.0, abs(fd)), (k, fd, np.vdot(d, zbar))


def test_tv_relax_vjp_identity_cases():
    rng = np.random.default_rng(2)
    z, xb = rng.random((6, 6)), rng.standard_normal((6, 6))
    np.testing.assert_array_equal(oracle.tv_relax_vjp(z, xb, 0.0, 5), xb)
    np.testing.assert_allclose(oracle.tv_relax_vjp(z, xb, 0.1, 5, alpha=0.0), xb, rtol=0, atol=0)


def tiny_problem(seed=0):
    n, V = 16, 8
    geo = synth.fan_geometry(n, V)
    g = oracle.Geometry(**geo)
    rng = np.random.default_rng(seed)
    xt = synth.rasterise(synth.random_ellipses(seed, 3, n), n)
    b = oracle.fp(g, xt) + 0.01 * rng.standard_normal((V, geo["n_bins"]))
    return geo, g, xt, b


@pytest.mark.parametrize("alpha,momentum", [(1.0, True), (0.7, True), (1.0, False)])
def test_pnp_vjp_matches_central_differences(alpha, momentum):
    """L = 1/2 ||x_T - x_ref||^2 through two-stage sketched iterations with a view subset."""
    geo, g, xt, b = tiny_problem()
    T = 5
    sub = synth.subset_views(1, 2, geo["n_views"])
    sched = [(2, None, 1.0), (2, sub, 2.0), (1, None, 1.0), (1, sub, 2.0), (1, None, 1.0)]
    eta = np.array([2e-3, 1.5e-3, 1e-3, 1e-3, 8e-4])
    a = synth.momentum_table(T, momentum)
    x0 = 0.3 * np.random.default_rng(5).random((16, 16))
    lam = 0.02

    def loss(x0_, eta_):
        xT = oracle.pnp_run(g, b, sched, eta_, a, alpha=alpha, lam=lam, x0=x0_)
        return 0.5 * np.sum((xT - xt) ** 2), xT

    L0, xT = loss(x0, eta)
    x0_bar, eta_bar = oracle.pnp_vjp(g, b, sched, eta, a, xT - xt, alpha=alpha, lam=lam, x0=x0)
    rng = np.random.default_rng(7)
    for _ in range(3):
        d = rng.standard_normal(x0.shape)
        h = 1e-5
        fd = (loss(x0 + h * d, eta)[0] - loss(x0 - h * d, eta)[0]) / (2 * h)
        assert abs(fd - np.vdot(d, x0_bar)) <= 1e-6 * max(abs(fd), 1e-3), (fd, np.vdot(d, x0_bar))
    for t in range(T):
        e = np.zeros(T)
        e[t] = eta[t] * 1e-4
        fd = (loss(x0, eta + e)[0] - loss(x0, eta - e)[0]) / (2 * e[t])
        assert abs(fd - eta_bar[t]) <= 1e-5 * max(abs(fd), 1e-3), (t, fd, eta_bar[t])


def test_linear_part_of_iteration_is_symmetric():
    """With TV = identity and a = 0 one step is y -> y - eta H y + eta c with H symmetric, so
    the reverse mode is the same linear map: <J d1, d2> = <d1, J d2> (adjoint identity)."""
    geo, g, xt, b = tiny_problem(1)
    sched = [(2, None, 1.0)]
    eta = np.array([3e-3])
    a = np.zeros(1)
    rng = np.random.default_rng(3)
    d1, d2 = rng.standard_normal((16, 16)), rng.standard_normal((16, 16))
    zero_b = np.zeros_like(b)
    J = lambda d: oracle.pnp_run(g, zero_b, sched, eta, a, lam=0.0, x0=d)  # noqa: E731
    Jt = lambda d: oracle.pnp_vjp(g, zero_b, sched, eta, a, d, lam=0.0, x0=np.zeros((16, 16)))[0]  # noqa: E731
    assert abs(np.vdot(J(d1), d2) - np.vdot(d1, Jt(d2))) <= 1e-12 * np.linalg.norm(d1) * np.linalg.norm(d2)
