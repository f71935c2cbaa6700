"""Pins of the oracle's variance-reduced minibatch gradient (SVRG over view subsets; the
paper names such estimators as replacements of the vanilla minibatch one, Sec. 2.1
after Eq. (7)).

Independent facts used: the estimator is exact at its own snapshot; averaged over the
partition of views into subsets it is the full gradient (unbiasedness); its error is
linear in y - y_snap and free of b; and the loop equals a dense-matrix recurrence."""
import numpy as np
import pytest

import oracle
from paper_2203_07308_amd import synth


@pytest.fixture(scope="module")
def small():
    geo = synth.fan_geometry(16, 12)
    g = oracle.Geometry(**geo)
    rng = np.random.default_rng(21)
    b = rng.random((12, geo["n_bins"]))
    y = synth.rasterise(synth.random_ellipses(5, 4, 16), 16)
    ys = y + 0.1 * rng.standard_normal(y.shape)
    return g, b, y, ys


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("f", [1, 2])
def test_exact_at_snapshot(small, f):
    g, b, y, _ = small
    full = oracle.grad(g, y, b, f)
    for s in range(3):
        vr = oracle.grad_vr(g, y, b, y, f, synth.subset_views(s, 3, 12), 3.0)
        assert rel(vr, full) <= 1e-13


@pytest.mark.parametrize("f", [1, 2])
def test_unbiased_over_the_subset_partition(small, f):
    g, b, y, ys = small
    full = oracle.grad(g, y, b, f)
    mean = sum(oracle.grad_vr(g, y, b, ys, f, synth.subset_views(s, 4, 12), 4.0) for s in range(4)) / 4
    assert rel(mean, full) <= 1e-12
    # a single subset is not the full gradient (the test above is not vacuous)
    assert rel(oracle.grad_vr(g, y, b, ys, f, synth.subset_views(0, 4, 12), 4.0), full) > 1e-6


def test_error_is_linear_in_the_snapshot_offset_and_free_of_b(small):
    g, b, y, ys = small
    d = ys - y
    sub = synth.subset_views(1, 4, 12)
    err = lambda yy, bb: oracle.grad_vr(g, y, bb, yy, 1, sub, 4.0) - oracle.grad(g, y, bb, 1)  # noqa: E731
    e1, e2 = err(y + d, b), err(y + 2 * d, b)
    np.testing.assert_allclose(e2, 2 * e1, rtol=1e-9, atol=1e-12 * np.abs(e1).max())
    np.testing.assert_allclose(err(y + d, 5 * b), e1, rtol=1e-9, atol=1e-12 * np.abs(e1).max())


def test_loop_matches_dense_recurrence():
    """Epochs of 4 iterations (a full-gradient snapshot step, then 3 variance-reduced
    subset steps); TV = identity, FISTA momentum."""
    n, V, T, m = 10, 8, 12, 4
    geo = synth.fan_geometry(n, V)
    g = oracle.Geometry(**geo)
    A = oracle.dense_matrix(g, 1)
    nb = geo["n_bins"]
    b = np.random.default_rng(3).random((V, nb)).ravel()
    seq = synth.subset_sequence(19, T, m)
    eta = 0.5 / np.linalg.eigvalsh(A.T @ A)[-1]
    a = synth.momentum_table(T)
    x = np.zeros(n * n)
    xp, y = x.copy(), x.copy()
    modes, sched = [], []
    for t in range(T):
        rows = np.concatenate([np.arange(k * nb, (k + 1) * nb) for k in synth.subset_views(seq[t], m, V)])
        if t % m == 0:
            ysnap = y.copy()
            gr = A.T @ (A @ y - b)
            modes.append(1)
        else:
            Ms = A[rows]
            gr = m * (Ms.T @ (Ms @ (y - ysnap))) + A.T @ (A @ ysnap - b)
            modes.append(2)
        sched.append((1, synth.subset_views(seq[t], m, V), float(m)))
        x = y - eta * gr
        y = x + a[t] * (x - xp)
        xp = x
    xo = oracle.pnp_run(g, b.reshape(V, nb), sched, np.full(T, eta), a, alpha=1.0, lam=0.0, vr=modes)
    np.testing.assert_allclose(xo.ravel(), x, rtol=1e-10, atol=1e-12)


def test_snapshot_must_precede_variance_reduced_steps():
    geo = synth.fan_geometry(8, 4, 12)
    g = oracle.Geometry(**geo)
    b = np.zeros((4, 12))
    with pytest.raises(ValueError):
        oracle.pnp_run(g, b, [(1, None, 1.0), (2, None, 1.0)], np.ones(2), np.zeros(2), vr=[1, 2])
