"""Pins of the oracle's bicubic sketch S and its adjoint U = S^T (the paper's bicubic
resizing choice, Sec. 3, with U read as the adjoint so that the sketched gradient stays
exact, Sec. 2.1 Eq. (6)).

Independent facts used: the hand-derived weights of tests/golden/bicubic_f2_weights.txt;
the identity at f = 1; exact reproduction of linear ramps away from the ends (which pins
the output centres); adjointness between the two separately written 2-D passes and the
Kronecker product of the 1-D matrices; exact central differences of the quadratic
sketched objective; the largest eigenvalue of the dense sketched operator."""
import os

import numpy as np
import pytest

import oracle
from paper_2203_07308_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "bicubic_f2_weights.txt")


def golden():
    rows = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        key, *vals = line.split()
        rows[key] = np.array([float(v) for v in vals])
    return rows


def test_factor_two_weights_match_hand_derivation():
    g = golden()
    S = oracle.bicubic_matrix(32, 2)
    o = 7  # interior row: u = 14.5, inputs 11..18
    np.testing.assert_array_equal(S[o, 11:19], g["interior"])
    assert np.count_nonzero(S[o]) == 8
    np.testing.assert_array_equal(S[0, :5], g["first"])
    assert np.count_nonzero(S[0]) == 5
    # the last row mirrors the first
    np.testing.assert_array_equal(S[-1, -5:], g["first"][::-1])


def test_factor_one_is_identity():
    np.testing.assert_array_equal(oracle.bicubic_matrix(17, 1), np.eye(17))
    x = np.random.default_rng(1).random((12, 20))
    np.testing.assert_array_equal(oracle.sketch_down(x, 1, "bicubic"), x)


@pytest.mark.parametrize("n,f", [(64, 2), (64, 4), (60, 3)])
def test_linear_ramps_are_reproduced_away_from_the_ends(n, f):
    S = oracle.bicubic_matrix(n, f)
    ramp = np.arange(n, dtype=np.float64)
    u = (np.arange(n // f) + 0.5) * f - 0.5
    inner = slice(2, n // f - 2)
    np.testing.assert_allclose((S @ ramp)[inner], u[inner], rtol=0, atol=1e-12)
    np.testing.assert_allclose(S.sum(axis=1), 1.0, atol=1e-14)


@pytest.mark.parametrize("shape,f", [((48, 64), 2), ((64, 64), 4), ((36, 24), 3)])
def test_two_dimensional_passes_are_the_kronecker_product_and_adjoint(shape, f):
    ny, nx = shape
    rng = np.random.default_rng(2)
    x = rng.random(shape)
    v = rng.random((ny // f, nx // f))
    K = np.kron(oracle.bicubic_matrix(ny, f), oracle.bicubic_matrix(nx, f))
    np.testing.assert_allclose(oracle.sketch_down(x, f, "bicubic").ravel(), K @ x.ravel(), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(oracle.sketch_up(v, f, "bicubic").ravel(), K.T @ v.ravel(), rtol=1e-13, atol=1e-14)
    lhs = np.vdot(oracle.sketch_down(x, f, "bicubic"), v)
    rhs = np.vdot(x, oracle.sketch_up(v, f, "bicubic"))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("f", [2, 4])
def test_bicubic_gradient_is_exact_gradient(f):
    geo = synth.fan_geometry(16, 10)
    g = oracle.Geometry(**geo)
    rng = np.random.default_rng(3)
    b = rng.random((10, geo["n_bins"]))
    y = rng.random((16, 16))
    d = rng.standard_normal((16, 16))
    grad = oracle.grad(g, y, b, f, sketch="bicubic")

    def obj(x):
        r = oracle.fp(g, oracle.sketch_down(x, f, "bicubic"), f=f) - b
        return 0.5 * np.sum(r * r)

    h = 1e-3
    fd = (obj(y + h * d) - obj(y - h * d)) / (2 * h)
    assert abs(fd - np.vdot(grad, d)) <= 1e-9 * abs(fd)
    # and it differs from the pooling sketch's gradient (the kind is honoured)
    assert np.linalg.norm(grad - oracle.grad(g, y, b, f)) > 1e-3 * np.linalg.norm(grad)


def test_bicubic_at_factor_one_equals_pooling_path():
    geo = synth.fan_geometry(16, 10)
    g = oracle.Geometry(**geo)
    rng = np.random.default_rng(4)
    b = rng.random((10, geo["n_bins"]))
    y = rng.random((16, 16))
    np.testing.assert_array_equal(oracle.grad(g, y, b, 1, sketch="bicubic"), oracle.grad(g, y, b, 1))


def test_power_iteration_bicubic():
    n, f = 12, 2
    geo = synth.fan_geometry(n, 10)
    g = oracle.Geometry(**geo)
    K = np.kron(oracle.bicubic_matrix(n, f), oracle.bicubic_matrix(n, f))
    B = oracle.dense_matrix(g, f) @ K
    lam = np.linalg.eigvalsh(B.T @ B)[-1]
    L = oracle.power_lipschitz(g, f, 500, sketch="bicubic")
    assert abs(L - lam) <= 1e-8 * lam
