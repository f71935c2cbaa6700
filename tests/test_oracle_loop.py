"""Pins of the oracle's sketch, sketched gradient, step size and PnP-MS2G loop.

Paper: sketched objective f(b, A_s S(x)) (Sec. 2.1, Eq. (4)); sketched gradient
U(A_s^T A_s S(x) - A_s^T b) (Eq. (6)); minibatch form (Eq. (7)); Algorithm 1;
eta = O(1/L), a_i = (i-1)/(i+3), alpha = 1 (Sec. 3).

Independent facts used: reshape-mean definition of pooling, adjoint identities,
the quadratic objective's exact central differences, closed-form Landweber and
momentum recurrences through LAPACK's eigh on dense matrices, and the largest
eigenvalue from eigh for the power iteration.
"""
import numpy as np
import pytest

import oracle
from paper_2203_07308_amd import synth


def pool_matrix(n, f):
    """Dense D_f for an n x n image (rows of averaging weights)."""
    ns = n // f
    D = np.zeros((ns * ns, n * n))
    for R in range(ns):
        for C in range(ns):
            for a in range(f):
                for b in range(f):
                    D[R * ns + C, (f * R + a) * n + f * C + b] = 1.0 / f ** 2
    return D


@pytest.mark.parametrize("f", [1, 2, 4])
def test_pooling_identities(f):
    n = 16
    rng = np.random.default_rng(f)
    x = rng.random((n, n))
    v = rng.random((n // f, n // f))
    Dx = oracle.down(x, f)
    np.testing.assert_allclose(Dx, x.reshape(n // f, f, n // f, f).mean(axis=(1, 3)), rtol=1e-14)
    np.testing.assert_allclose(oracle.up(v, f), np.kron(v, np.ones((f, f))) / f ** 2, rtol=1e-15)
    assert abs(np.vdot(Dx, v) - np.vdot(x, oracle.up(v, f))) < 1e-13
    np.testing.assert_allclose(oracle.down(oracle.up(v, f), f), v / f ** 2, rtol=1e-14)
    np.testing.assert_allclose(oracle.down(np.ones((n, n)), f), np.ones((n // f, n // f)), rtol=1e-15)
    if f == 1:
        np.testing.assert_array_equal(Dx, x)


def small_problem(n=16, V=12, seed=0):
    geo = synth.fan_geometry(n, V)
    g = oracle.Geometry(**geo)
    rng = np.random.default_rng(seed)
    b = rng.random((V, geo["n_bins"])) * 5
    y = rng.random((n, n))
    return geo, g, b, y


def test_factor_one_gradient_is_full_gradient():
    """With f = 1 the sketched gradient is A^T(Ay - b) (Sec. 2.1, Eq. (5) vs Eq. (6))."""
    geo, g, b, y = small_problem()
    A = oracle.dense_matrix(g, 1)
    full = (A.T @ (A @ y.ravel() - b.ravel())).reshape(y.shape)
    np.testing.assert_allclose(oracle.grad(g, y, b, 1), full, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("f", [1, 2, 4])
def test_gradient_is_exact_gradient_of_sketched_objective(f):
    """F(x) = 1/2 ||A_s D x - b||^2 is quadratic, so its central difference along any
    direction equals <G, delta> up to rounding, for any step h."""
    geo, g, b, y = small_problem(seed=f)
    F = lambda x: 0.5 * np.sum((oracle.fp(g, oracle.down(x, f), f) - b) ** 2)  # noqa: E731
    G = oracle.grad(g, y, b, f)
    rng = np.random.default_rng(10 + f)
    for h in (1e-2, 1.0):
        d = rng.standard_normal(y.shape)
        fd = (F(y + h * d) - F(y - h * d)) / (2 * h)
        assert abs(fd - np.vdot(G, d)) <= 1e-9 * abs(fd) + 1e-9


def test_sketched_gradient_matches_dense_product():
    geo, g, b, y = small_problem(n=16, V=8)
    f = 2
    As = oracle.dense_matrix(g, f)
    D = pool_matrix(16, f)
    B = As @ D
    np.testing.assert_allclose(oracle.grad(g, y, b, f).ravel(), B.T @ (B @ y.ravel() - b.ravel()),
                               rtol=1e-11, atol=1e-11)


def test_subset_gradients_partition_the_full_gradient():
    """Sum over the interleaved subsets of the (unscaled) minibatch gradients = full gradient,
    and with sigma = n_sub each minibatch gradient is unbiased (Sec. 2.1, Eq. (7))."""
    geo, g, b, y = small_problem(V=16)
    for f in (1, 2):
        full = oracle.grad(g, y, b, f)
        parts = [oracle.grad(g, y, b, f, synth.subset_views(s, 4, 16), 1.0) for s in range(4)]
        np.testing.assert_allclose(sum(parts), full, rtol=1e-11, atol=1e-11)
        scaled = [oracle.grad(g, y, b, f, synth.subset_views(s, 4, 16), 4.0) for s in range(4)]
        np.testing.assert_allclose(np.mean(scaled, axis=0), full, rtol=1e-11, atol=1e-11)


def test_landweber_closed_form():
    """TV = identity (lambda = 0), alpha = 1, a = 0: x_T = sum_{t<T} (I - eta A^T A)^t eta A^T b,
    evaluated in the eigenbasis of A^T A."""
    n, V, T = 12, 8, 25
    geo = synth.fan_geometry(n, V)
    g = oracle.Geometry(**geo)
    A = oracle.dense_matrix(g, 1)
    b = np.random.default_rng(1).random((V, geo["n_bins"]))
    lam_, Q = np.linalg.eigh(A.T @ A)
    eta = 1.0 / lam_[-1]
    c = Q.T @ (A.T @ b.ravel())
    mult = 1 - eta * lam_
    s = np.where(np.abs(eta * lam_) > 1e-14, (1 - mult ** T) / np.where(eta * lam_ == 0, 1, eta * lam_),
                 float(T))
    expect = Q @ (eta * s * c)
    sched = [(1, None, 1.0)] * T
    x = oracle.pnp_run(g, b, sched, np.full(T, eta), np.zeros(T), lam=0.0)
    np.testing.assert_allclose(x.ravel(), expect, rtol=1e-9, atol=1e-9 * np.abs(expect).max())


def test_momentum_recurrence_in_eigenbasis():
    """With a_t = (t-1)/(t+3) and TV = identity, every eigencomponent follows the scalar
    two-term recurrence of Algorithm 1 (Sec. 3 momentum)."""
    n, V, T = 10, 6, 30
    geo = synth.fan_geometry(n, V)
    g = oracle.Geometry(**geo)
    f = 2
    B = oracle.dense_matrix(g, f) @ pool_matrix(n, f)
    b = np.random.default_rng(2).random((V, geo["n_bins"]))
    lam_, Q = np.linalg.eigh(B.T @ B)
    eta = 0.9 / lam_[-1]
    c = Q.T @ (B.T @ b.ravel())
    a = synth.momentum_table(T)
    xs, ys = np.zeros_like(c), np.zeros_like(c)
    for t in range(T):
        xn = ys - eta * (lam_ * ys - c)
        ys = xn + a[t] * (xn - xs)
        xs = xn
    x = oracle.pnp_run(g, b, [(f, None, 1.0)] * T, np.full(T, eta), a, lam=0.0)
    np.testing.assert_allclose(x.ravel(), Q @ xs, rtol=1e-9, atol=1e-9 * np.abs(xs).max())


def test_minibatch_loop_matches_dense_recurrence():
    """Option 2 (Algorithm 1) with a drawn subset sequence; TV = identity, so any alpha
    leaves z unchanged."""
    n, V, T = 10, 8, 12
    geo = synth.fan_geometry(n, V)
    g = oracle.Geometry(**geo)
    A = oracle.dense_matrix(g, 1)
    nb = geo["n_bins"]
    b = np.random.default_rng(3).random((V, nb))
    seq = synth.subset_sequence(9, T, 4)
    eta = 0.5 / np.linalg.eigvalsh(A.T @ A)[-1]
    x = np.zeros(n * n)
    xp, y = x.copy(), x.copy()
    a = synth.momentum_table(T)
    for t in range(T):
        rows = np.concatenate([np.arange(k * nb, (k + 1) * nb) for k in synth.subset_views(seq[t], 4, V)])
        Ms = A[rows]
        z = y - eta * 4.0 * (Ms.T @ (Ms @ y - b.ravel()[rows]))
        x = z
        y = x + a[t] * (x - xp)
        xp = x
    sched = [(1, synth.subset_views(s, 4, V), 4.0) for s in seq]
    xo = oracle.pnp_run(g, b, sched, np.full(T, eta), a, alpha=0.6, lam=0.0)
    np.testing.assert_allclose(xo.ravel(), x, rtol=1e-10, atol=1e-12)


def test_history_and_relaxation():
    geo, g, b, y = small_problem(n=16, V=8)
    T = 4
    sched = [(2, None, 1.0)] * 2 + [(1, None, 1.0)] * 2
    eta = np.full(T, 1e-3)
    a = synth.momentum_table(T)
    alpha = 0.7
    x, hist = oracle.pnp_run(g, b, sched, eta, a, alpha=alpha, history=True)
    np.testing.assert_array_equal(hist[-1], x)
    # step by step with the oracle's own blocks: relaxation alpha between z and TV(z)
    xp = np.zeros((16, 16))
    yy = xp.copy()
    for t in range(T):
        z = yy - eta[t] * oracle.grad(g, yy, b, sched[t][0])
        xt = (1 - alpha) * z + alpha * oracle.tv_prox(z, 0.01, 5)
        np.testing.assert_allclose(hist[t], xt, rtol=1e-12, atol=1e-14)
        yy = xt + a[t] * (xt - xp)
        xp = xt


@pytest.mark.parametrize("f", [1, 2])
def test_power_iteration_reaches_largest_eigenvalue(f):
    n, V = 12, 10
    geo = synth.fan_geometry(n, V)
    g = oracle.Geometry(**geo)
    B = oracle.dense_matrix(g, f) @ pool_matrix(n, f)
    lmax = np.linalg.eigvalsh(B.T @ B)[-1]
    L = oracle.power_lipschitz(g, f, 100)
    assert abs(L - lmax) <= 1e-8 * lmax


def test_psnr_closed_form():
    ref = np.linspace(-1.0, 3.0, 100).reshape(10, 10)
    x = ref + 0.01
    assert abs(oracle.psnr(x, ref) - 10 * np.log10(16.0 / 1e-4)) < 1e-9
