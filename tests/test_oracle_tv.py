"""Pins of the oracle's TV-prox denoiser (Chambolle's dual projection).

The paper allows a TV proximal operator as the denoiser D (Sec. 2.1, list after
Eq. (5)); the workloads fix 5 iterations with lambda = 0.01. The oracle is checked
against: the exact two-pixel prox, an independent projected-gradient solver of the ROF
dual built on a sparse difference matrix, and invariants (identity cases, mean).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle


def grad_matrix(ny, nx):
    """Forward differences, zero on the last row (row part) and last column (column part)."""
    def d1(n):
        m = sp.lil_matrix((n, n))
        for i in range(n - 1):
            m[i, i], m[i, i + 1] = -1.0, 1.0
        return m.tocsr()
    Gr = sp.kron(d1(ny), sp.identity(nx))
    Gc = sp.kron(sp.identity(ny), d1(nx))
    return sp.vstack([Gr, Gc]).tocsr()


def rof_projected_gradient(z, lam, iters=20000):
    """argmin_x 1/2||x - z||^2 + lam sum_i |(G x)_i|_2 by accelerated projected gradient
    on the dual min_{|p_i|<=1} 1/2 ||z - lam G^T p||^2, x = z - lam G^T p."""
    ny, nx = z.shape
    G = grad_matrix(ny, nx)
    zf = z.ravel()
    n = zf.size
    p = np.zeros(2 * n)
    q = p.copy()
    tk = 1.0
    step = 1.0 / (8.0 * lam * lam)

    def proj(v):
        a, b = v[:n], v[n:]
        m = np.maximum(1.0, np.sqrt(a * a + b * b))
        return np.concatenate([a / m, b / m])

    for _ in range(iters):
        gq = -lam * (G @ (zf - lam * (G.T @ q)))
        pn = proj(q - step * gq)
        tn = 0.5 * (1 + np.sqrt(1 + 4 * tk * tk))
        q = pn + (tk - 1) / tn * (pn - p)
        p, tk = pn, tn
    return (zf - lam * (G.T @ p)).reshape(z.shape)


def tv_iso(x):
    G = grad_matrix(*x.shape)
    g = G @ x.ravel()
    n = x.size
    return np.sum(np.sqrt(g[:n] ** 2 + g[n:] ** 2))


def test_lambda_zero_is_identity():
    z = np.random.default_rng(0).random((9, 7))
    np.testing.assert_array_equal(oracle.tv_prox(z, 0.0, 5), z)


def test_constant_image_is_fixed():
    z = np.full((8, 11), 0.37)
    np.testing.assert_allclose(oracle.tv_prox(z, 0.01, 5), z, rtol=0, atol=1e-15)


@pytest.mark.parametrize("shape", [(16, 16), (7, 13), (1, 9)])
def test_mean_is_preserved(shape):
    z = np.random.default_rng(1).random(shape)
    x = oracle.tv_prox(z, 0.05, 5)
    assert abs(x.mean() - z.mean()) < 1e-14
    assert not np.allclose(x, z)


@pytest.mark.parametrize("a,b,lam", [(0.2, 0.9, 0.1), (0.9, 0.2, 0.1), (0.5, 0.55, 0.1), (1.0, 0.0, 0.3)])
def test_two_pixel_closed_form(a, b, lam):
    """Exact prox of lam |x2 - x1| on [a, b]: shrink the jump by 2 lam or merge to the mean."""
    z = np.array([[a, b]])
    x = oracle.tv_prox(z, lam, 20000)
    if abs(b - a) > 2 * lam:
        s = np.sign(b - a)
        expect = np.array([[a + lam * s, b - lam * s]])
    else:
        expect = np.full((1, 2), 0.5 * (a + b))
    np.testing.assert_allclose(x, expect, atol=1e-10)


@pytest.mark.parametrize("shape,lam", [((1, 12), 0.05), ((6, 6), 0.04), ((5, 8), 0.1)])
def test_converges_to_rof_minimiser(shape, lam):
    """Many Chambolle steps reach the ROF minimiser found by an independent dual solver."""
    rng = np.random.default_rng(2)
    z = rng.random(shape)
    z[:, : shape[1] // 2] += 0.5
    ref = rof_projected_gradient(z, lam)
    x = oracle.tv_prox(z, lam, 40000)
    np.testing.assert_allclose(x, ref, atol=2e-7)
    # and it is the minimiser of the primal objective written independently
    P = lambda u: 0.5 * np.sum((u - z) ** 2) + lam * tv_iso(u)  # noqa: E731
    assert P(x) <= P(ref) + 1e-10
    for _ in range(5):
        assert P(x) <= P(x + 1e-3 * rng.standard_normal(shape))


def test_five_steps_reduce_the_rof_objective():
    """The 5-step denoiser used in every workload moves toward the ROF minimiser."""
    rng = np.random.default_rng(4)
    z = rng.random((12, 12)) * 0.1
    z[3:9, 3:9] += 1.0
    lam = 0.01
    P = lambda u: 0.5 * np.sum((u - z) ** 2) + lam * tv_iso(u)  # noqa: E731
    x5 = oracle.tv_prox(z, lam, 5)
    ref = rof_projected_gradient(z, lam)
    assert P(ref) < P(x5) < P(z)
    assert np.linalg.norm(x5 - ref) < np.linalg.norm(z - ref)


def _golden_tv_cases():
    """Rows of tests/golden/tv_prox_chambolle_small.txt: (name, z, n_iter, x) with x exact."""
    import os
    import re
    from fractions import Fraction

    def value(s):
        return sum(Fraction(t) for t in re.findall(r"[+-]?\d+(?:/\d+)?", s))

    path = os.path.join(os.path.dirname(__file__), "golden", "tv_prox_chambolle_small.txt")
    cases = []
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        head, xs = line.split("|")
        f = head.split()
        name, ny, nx, n_iter = f[0], int(f[1]), int(f[2]), int(f[3])
        z = np.array([float(value(v)) for v in f[4:]]).reshape(ny, nx)
        x = np.array([float(value(v)) for v in xs.split()]).reshape(ny, nx)
        cases.append((f"{name}-n{n_iter}", z, n_iter, x))
    return cases


@pytest.mark.parametrize("name,z,n_iter,expect", _golden_tv_cases(), ids=[c[0] for c in _golden_tv_cases()])
def test_finite_step_map_matches_hand_derivation(name, z, n_iter, expect):
    """The n-step map itself (not only its limit) against values worked out by hand in exact
    fractions: the 1 x 2 recurrence for n = 1..6, its upright twin, two coupled duals of a
    1 x 3 image for two steps, and one isotropic step on a 2 x 2 image."""
    x = oracle.tv_prox(z, 1.0 / 64.0, n_iter, 0.125)
    np.testing.assert_allclose(x, expect, rtol=0, atol=1e-15)
    # a step more or less gives a different image (the count is pinned, not just the limit)
    for m in (n_iter - 1, n_iter + 1):
        if m >= 0:
            assert np.max(np.abs(oracle.tv_prox(z, 1.0 / 64.0, m, 0.125) - expect)) > 1e-6


def _chambolle_dense(z, lam, n_iter, tau):
    """The same dual steps written on the sparse difference matrix G (div = -G^T), vectorised
    over pixels: an independent formulation for brute-force comparison on small images."""
    ny, nx = z.shape
    G = grad_matrix(ny, nx)
    n = z.size
    zf = z.ravel()
    p = np.zeros(2 * n)
    for _ in range(n_iter):
        q = G @ (-(G.T @ p) - zf / lam)
        mag = np.sqrt(q[:n] ** 2 + q[n:] ** 2)
        p = (p + tau * q) / np.concatenate([1 + tau * mag, 1 + tau * mag])
    return (zf + lam * (G.T @ p)).reshape(ny, nx)


@pytest.mark.parametrize("shape", [(5, 7), (8, 3), (1, 6), (6, 1)])
@pytest.mark.parametrize("n_iter", [1, 2, 5, 8])
def test_finite_step_map_matches_matrix_form(shape, n_iter):
    rng = np.random.default_rng(10 + n_iter)
    z = rng.random(shape)
    x = oracle.tv_prox(z, 0.01, n_iter, 0.125)
    np.testing.assert_allclose(x, _chambolle_dense(z, 0.01, n_iter, 0.125), rtol=0, atol=1e-12)
