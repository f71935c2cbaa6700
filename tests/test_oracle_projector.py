"""Pins of the oracle's fan-beam Joseph projector and its transpose.

The paper names no projector (Sec. 3 only states fan-beam CT of 256^2 images); the
oracle's reading is Joseph's ray-driven method. These tests tie it to facts that do
not come from its own code:
  * analytic line integrals of ellipses (chord length x density), with the rays
    described independently by source angle and fan angle;
  * exactness of Joseph's rule for affine images on interior rays;
  * the 90-degree rotation symmetry of the geometry;
  * the transpose identity <Ax, y> = <x, A^T y> and the dense matrix.
"""
import numpy as np
import pytest

import oracle
from paper_2203_07308_amd import synth


def rays(geo, views):
    """Independent description: source at angle beta, ray at angle beta + pi - gamma,
    gamma = atan(u / sdd) the fan angle of the bin centre u."""
    B = geo["n_bins"]
    out = []
    for k in views:
        beta = geo["angle0_rad"] + k * geo["angle_step_rad"]
        u = (np.arange(B) - (B - 1) / 2) * geo["det_pitch_mm"] + geo["det_offset_mm"]
        th = beta + np.pi - np.arctan2(u, geo["sdd_mm"])
        S = geo["sod_mm"] * np.array([np.cos(beta), np.sin(beta)])
        out.append((np.broadcast_to(S, (B, 2)), np.stack([np.cos(th), np.sin(th)], 1)))
    return out


def ellipse_integrals(e, geo, views):
    """Line integral = sum of density x chord length, chord from the ray/ellipse quadratic."""
    res = []
    for S, D in rays(geo, views):
        tot = np.zeros(len(D))
        for i in range(len(e.cx)):
            c, s = np.cos(e.phi[i]), np.sin(e.phi[i])
            px, py = S[:, 0] - e.cx[i], S[:, 1] - e.cy[i]
            qx, qy = px * c + py * s, -px * s + py * c
            dx, dy = D[:, 0] * c + D[:, 1] * s, -D[:, 0] * s + D[:, 1] * c
            A = dx ** 2 / e.a[i] ** 2 + dy ** 2 / e.b[i] ** 2
            Bq = 2 * (qx * dx / e.a[i] ** 2 + qy * dy / e.b[i] ** 2)
            C = qx ** 2 / e.a[i] ** 2 + qy ** 2 / e.b[i] ** 2 - 1
            disc = Bq ** 2 - 4 * A * C
            tot += e.rho[i] * np.where(disc > 0, np.sqrt(np.maximum(disc, 0)) / A, 0)
        res.append(tot)
    return np.array(res)


# source at 1.5 image circumradii: a fan of about 85 degrees (the plan's limit is 90)
WIDE = 1.5


@pytest.mark.parametrize("wide", [None, WIDE])
def test_disk_chord_closed_form(wide):
    """A centred disk of radius R and density 1: integral 2 sqrt(R^2 - s^2) at distance s."""
    n = 128
    geo = synth.fan_geometry(n, 8, None if wide is None else 256, sod_over_radius=wide)
    R = 40.0
    e = synth.Ellipses(np.zeros(1), np.zeros(1), np.full(1, R), np.full(1, R), np.zeros(1), np.ones(1))
    an = ellipse_integrals(e, geo, range(8))
    S, D = rays(geo, [0])[0]
    s = np.abs(S[:, 0] * D[:, 1] - S[:, 1] * D[:, 0])
    expect = 2 * np.sqrt(np.maximum(R ** 2 - s ** 2, 0))
    np.testing.assert_allclose(an[0], expect, atol=1e-9)
    np.testing.assert_allclose(an, np.broadcast_to(expect, an.shape), atol=1e-9)
    p = oracle.fp(oracle.Geometry(**geo), synth.rasterise(e, n))
    assert np.linalg.norm(p - an) / np.linalg.norm(an) < 0.01


def test_ellipse_integrals_converge_first_order():
    """Joseph on the rasterised phantom converges to the analytic sinogram as h -> 0."""
    e0 = synth.random_ellipses(7, 5, 64)
    errs = []
    for n in (32, 64, 128, 256):
        sc = n / 64
        e = synth.Ellipses(e0.cx * sc, e0.cy * sc, e0.a * sc, e0.b * sc, e0.phi, e0.rho)
        geo = synth.fan_geometry(n, 36)
        p = oracle.fp(oracle.Geometry(**geo), synth.rasterise(e, n))
        an = ellipse_integrals(e, geo, range(36))
        errs.append(np.linalg.norm(p - an) / np.linalg.norm(an))
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(ratios > 1.8), (errs, ratios)
    assert errs[-1] < 0.01, errs


@pytest.mark.parametrize("n,f,wide", [(32, 1, None), (48, 1, None), (64, 2, None), (64, 4, None),
                                      (48, 1, WIDE), (64, 2, WIDE)])
def test_affine_image_exact_on_interior_rays(n, f, wide):
    """For X = a + b x + c y at pixel centres, Joseph's sum equals the exact integral of
    the affine function over the chord between the outer pixel edges of the sampled axis,
    on every ray whose interpolation never leaves the grid (midpoint rule and linear
    interpolation are both exact for affine functions)."""
    V = 16
    geo = synth.fan_geometry(n, V, None if wide is None else 2 * n, sod_over_radius=wide)
    g = oracle.Geometry(**geo)
    ns, hs = n // f, f * geo["pixel_mm"]
    a0, bx, cy = 0.7, 0.013, -0.021
    ctr = (np.arange(ns) - 0.5 * (ns - 1)) * hs
    X = a0 + bx * ctr[None, :] + cy * ctr[:, None]
    p = oracle.fp(g, X, f=f)
    half = 0.5 * ns * hs
    checked = {"x": 0, "y": 0}
    for k, (S, D) in enumerate(rays(geo, range(V))):
        for j in range(geo["n_bins"]):
            sx, sy = S[j]
            dx, dy = D[j]
            if abs(dx) >= abs(dy):
                t = (ctr - sx) / dx
                other = (sy + t * dy) / hs + 0.5 * (ns - 1)
                t1, t2 = (-half - sx) / dx, (half - sx) / dx
                key = "x"
            else:
                t = (ctr - sy) / dy
                other = (sx + t * dx) / hs + 0.5 * (ns - 1)
                t1, t2 = (-half - sy) / dy, (half - sy) / dy
                key = "y"
            if other.min() < 1e-9 or other.max() > ns - 1 - 1e-9:
                continue
            tm = 0.5 * (t1 + t2)
            exact = abs(t2 - t1) * (a0 + bx * (sx + tm * dx) + cy * (sy + tm * dy))
            assert abs(p[k, j] - exact) <= 1e-12 * abs(exact), (k, j, p[k, j], exact)
            checked[key] += 1
    assert checked["x"] > 20 and checked["y"] > 20, checked


def test_rotation_by_quarter_turn():
    """Rotating the image by +90 degrees about the isocentre equals advancing the view
    angle by a quarter turn: fp(rot X)[k + V/4] = fp(X)[k]."""
    n, V = 40, 24
    geo = synth.fan_geometry(n, V)
    g = oracle.Geometry(**geo)
    X = np.random.default_rng(3).random((n, n))
    # pixel (r, c) at (x_c, y_r) moves to (-y_r, x_c): new column n-1-r, new row c
    Xr = np.empty_like(X)
    r, c = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    Xr[c, n - 1 - r] = X[r, c]
    p, pr = oracle.fp(g, X), oracle.fp(g, Xr)
    q = V // 4
    # skip rays that sit within rounding of the 45-degree dominance tie
    mask = np.ones_like(p, dtype=bool)
    for k, (S, D) in enumerate(rays(geo, range(V))):
        mask[k] = np.abs(np.abs(D[:, 0]) - np.abs(D[:, 1])) > 1e-9
    np.testing.assert_allclose(pr[q:][mask[:-q]], p[:-q][mask[:-q]], rtol=1e-12, atol=1e-12)


def test_linearity_and_zero():
    geo = synth.fan_geometry(32, 12)
    g = oracle.Geometry(**geo)
    rng = np.random.default_rng(5)
    x1, x2 = rng.random((32, 32)), rng.random((32, 32))
    assert np.all(oracle.fp(g, np.zeros((32, 32))) == 0)
    np.testing.assert_allclose(oracle.fp(g, 2.5 * x1 - x2), 2.5 * oracle.fp(g, x1) - oracle.fp(g, x2),
                               rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n,V,f,sub,wide", [(64, 90, 1, None, None), (64, 90, 2, None, None),
                                            (64, 90, 4, None, None), (48, 30, 2, [1, 4, 7, 29], None),
                                            (40, 36, 1, [35, 0, 17], None), (48, 30, 1, None, WIDE),
                                            (48, 30, 4, [2, 9, 0], WIDE)])
def test_transpose_identity(n, V, f, sub, wide):
    """<M A_s x, y> = <x, (M A_s)^T y> to 1e-12 relative."""
    geo = synth.fan_geometry(n, V, None if wide is None else 2 * n, sod_over_radius=wide)
    g = oracle.Geometry(**geo)
    rng = np.random.default_rng(11)
    x = rng.standard_normal((n // f, n // f))
    ns = V if sub is None else len(sub)
    y = rng.standard_normal((ns, geo["n_bins"]))
    lhs = np.vdot(oracle.fp(g, x, f, sub), y)
    rhs = np.vdot(x, oracle.bp(g, y, f, sub))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), np.linalg.norm(x) * np.linalg.norm(y) * 1e-3)


def test_dense_matrix_matches_ray_march_and_transpose():
    geo = synth.fan_geometry(12, 8)
    g = oracle.Geometry(**geo)
    sub = [0, 3, 5]
    for f in (1, 2):
        A = oracle.dense_matrix(g, f, sub)
        ns = 12 // f
        rng = np.random.default_rng(f)
        x = rng.random((ns, ns))
        y = rng.random((3, geo["n_bins"]))
        np.testing.assert_allclose(A @ x.ravel(), oracle.fp(g, x, f, sub).ravel(), rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(A.T @ y.ravel(), oracle.bp(g, y, f, sub).ravel(), rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(oracle.bp(g, y, f, sub, scale=-3.0), -3.0 * oracle.bp(g, y, f, sub),
                                   rtol=1e-15, atol=0)


def test_subset_rows_are_rows_of_full_projection():
    geo = synth.fan_geometry(32, 16)
    g = oracle.Geometry(**geo)
    x = np.random.default_rng(2).random((32, 32))
    full = oracle.fp(g, x)
    sub = synth.subset_views(3, 8, 16)
    np.testing.assert_array_equal(oracle.fp(g, x, 1, sub), full[sub])


@pytest.mark.parametrize("wide", [None, WIDE])
def test_sample_count_brute_force(wide):
    """Count of in-grid samples against a direct enumeration with the independent rays."""
    n, V = 24, 8
    geo = synth.fan_geometry(n, V, None if wide is None else 48, sod_over_radius=wide)
    g = oracle.Geometry(**geo)
    ctr = (np.arange(n) - 0.5 * (n - 1))
    total = 0
    for S, D in rays(geo, range(V)):
        for (sx, sy), (dx, dy) in zip(S, D):
            if abs(dx) >= abs(dy):
                pos = (sy + (ctr - sx) / dx * dy) + 0.5 * (n - 1)
            else:
                pos = (sx + (ctr - sy) / dy * dx) + 0.5 * (n - 1)
            total += int(np.sum((pos > -1) & (pos < n)))
    assert oracle.count_samples(g) == total
