"""Seeded synthetic inputs for fan-beam CT experiments.

This module only draws and describes inputs: phantoms, Gaussian draws, view-subset
sequences, geometry and schedule descriptions. It holds none of the reconstruction
arithmetic (no projector, no sketch, no denoiser); the GPU library and the FP64
oracle both consume what it produces.

Stand-ins: the paper's test images (a disk phantom, a head and a chest slice, Sec. 3)
are not available, so every image is a seeded random-ellipse phantom of the same
shape class, optionally with a low-amplitude smooth texture.

Readings (where neither the paper nor the workload descriptions fix a choice):
  * geometry scales with the width n: pixel 1 mm, source-to-isocentre 7.8125 n mm,
    source-to-detector twice that, 1.5 n bins whose pitch is 2 mm (1 pixel referred
    to the isocentre), bins centred, views equally spaced over [0, 2 pi) from 0;
  * ellipses: centre uniform in the disc of radius 0.6 R (R = n h / 2), semi-axes
    uniform in [0.05 R, 0.35 R], orientation uniform in [0, pi), density uniform in
    [0, 1], ellipses add; pixel value = density x covered fraction by 4 x 4 point
    sampling;
  * texture: white N(0,1) noise, Gaussian-smoothed (sigma 2 px), rescaled to standard
    deviation 0.02 and masked to the field-of-view disc;
  * noise: additive Gaussian with sigma = level * max(Ax), or "poisson-like" with
    sigma_i = level * sqrt(max(Ax) * (Ax)_i);
  * view subsets: subset s of n_sub holds the views k = s (mod n_sub); the subset of
    each iteration is drawn i.i.d. uniform.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# ----------------------------------------------------------------------------------
# geometry and workloads (plain descriptions)
# ----------------------------------------------------------------------------------

def fan_geometry(n: int, n_views: int, n_bins: int | None = None, angle_range: float = 2 * math.pi,
                 iso_pitch_px: float = 1.0, sod_over_radius: float | None = None) -> dict:
    """Geometry parameters for an n x n grid of 1 mm pixels; a detector bin spans
    iso_pitch_px pixels at the isocentre.
    sod_over_radius: a wide fan instead, with the source at that multiple of the
    image's circumradius and the bins spread over the fan that covers the image."""
    h = 1.0
    nb = int(round(1.5 * n)) if n_bins is None else n_bins
    sod = 7.8125 * n * h
    sdd = 2.0 * sod
    pitch = iso_pitch_px * h * sdd / sod
    if sod_over_radius is not None:
        radius = n * h / math.sqrt(2.0)
        sod = sod_over_radius * radius
        sdd = 2.0 * sod
        half_fan = math.asin(radius / sod)
        pitch = 1.02 * 2.0 * sdd * math.tan(half_fan) / nb
    return dict(
        nx=n, ny=n, pixel_mm=h, n_views=n_views, n_bins=nb,
        sod_mm=sod, sdd_mm=sdd, det_pitch_mm=pitch, det_offset_mm=0.0,
        angle0_rad=0.0, angle_step_rad=angle_range / n_views,
    )


@dataclass
class Workload:
    """A reconstruction workload: image, geometry, data model and stage schedule."""
    name: str
    n: int
    n_views: int
    n_bins: int
    n_ellipses: int
    texture: bool
    noise_kind: str          # "gaussian" or "poisson-like"
    noise_level: float
    stages: list             # [(pooling factor f, iterations)]
    n_subsets: int           # 0: every gradient uses all views
    momentum: bool           # FISTA-type a_t = (t-1)/(t+3); False: a_t = 0 (PnP-ISTA)
    lam: float = 0.01
    tv_iters: int = 5
    tau: float = 0.125
    alpha: float = 1.0
    seed_base: int = 0

    @property
    def geometry(self) -> dict:
        return fan_geometry(self.n, self.n_views, self.n_bins)

    @property
    def n_iters(self) -> int:
        return sum(it for _, it in self.stages)


WORKLOADS = {
    # plain full-gradient PnP-ISTA, 64^2, 90 views x 96 bins
    "pnp64": Workload("pnp64", 64, 90, 96, 10, False, "gaussian", 0.01, [(1, 50)], 0, False, seed_base=1),
    # two-stage sketched PnP, 256^2, 360 views x 384 bins
    "ms2g256": Workload("ms2g256", 256, 360, 384, 20, False, "gaussian", 0.01, [(2, 30), (1, 20)], 0, True,
                        seed_base=2),
    # multi-stage sketched PnP-SGD, 512^2, 720 views x 768 bins, 1 of 8 view subsets
    "ms2g512": Workload("ms2g512", 512, 720, 768, 40, True, "poisson-like", 0.005, [(4, 20), (2, 20), (1, 20)],
                        8, True, seed_base=3),
}


@dataclass
class BatchWorkload:
    """Many independent slices of uneven sizes and view counts, one shared stage schedule.
    Slice i draws its width from `sizes` and its view count from `view_counts` (uniform,
    seeded), has 1.5 n bins, and its phantom and noise seeds follow `slice_workload(i)`."""
    name: str
    n_slices: int
    sizes: tuple
    view_counts: tuple
    n_ellipses: int
    noise_kind: str
    noise_level: float
    stages: list
    n_subsets: int
    momentum: bool
    lam: float = 0.01
    tv_iters: int = 5
    tau: float = 0.125
    alpha: float = 1.0
    seed_base: int = 0

    def shapes(self) -> list:
        """[(n, n_views)] per slice."""
        rng = np.random.default_rng(4000 * self.seed_base)
        n = rng.choice(np.asarray(self.sizes), self.n_slices)
        v = rng.choice(np.asarray(self.view_counts), self.n_slices)
        return [(int(a), int(b)) for a, b in zip(n, v)]

    def slice_workload(self, i: int) -> Workload:
        n, V = self.shapes()[i]
        return Workload(f"{self.name}[{i}]", n, V, int(round(1.5 * n)), self.n_ellipses, False, self.noise_kind,
                        self.noise_level, self.stages, self.n_subsets, self.momentum, self.lam, self.tv_iters,
                        self.tau, self.alpha, self.seed_base)


BATCH_WORKLOADS = {
    # 64 slices, widths from {128, ..., 512}, 180 / 360 / 720 views, two-stage sketch (30 at f = 2, 20 at f = 1)
    "batch64": BatchWorkload("batch64", 64, (128, 192, 256, 384, 512), (180, 360, 720), 20, "gaussian", 0.01,
                             [(2, 30), (1, 20)], 0, True, seed_base=4),
}


@dataclass
class Scenario:
    """One of the paper's experiments (Sec. 3): a 256 x 256 disk phantom, fan beam with 228
    bins covering the field of view, Poisson transmission data at incident count i0, and the
    two-stage sketch schedule (f = 4, then f = 2) against full-gradient PnP-FISTA."""
    name: str
    n_views: int
    angle_range: float
    i0: float
    n: int = 256
    n_bins: int = 228
    n_disks: int = 10
    mu0: float = 0.02           # 1/mm per unit density (about water)
    stages: tuple = ((4, 25), (2, 75))
    full_iters: int = 100
    lam: float = 0.01
    tv_iters: int = 5
    tau: float = 0.125
    alpha: float = 1.0
    seed_base: int = 5

    @property
    def geometry(self) -> dict:
        return fan_geometry(self.n, self.n_views, self.n_bins, self.angle_range, self.n / self.n_bins)

    def phantom(self) -> np.ndarray:
        return rasterise(random_disks(1000 * self.seed_base, self.n_disks, self.n), self.n).astype(np.float32)

    def data(self, ax: np.ndarray) -> np.ndarray:
        """Log transmission data (density units) for line integrals ax of the phantom."""
        return transmission_data(ax, self.i0, self.mu0, 2000 * self.seed_base + self.n_views)


SCENARIOS = {
    "sparse_view": Scenario("sparse_view", 90, 2 * math.pi, 10 ** 5.5),
    "low_dose": Scenario("low_dose", 360, 2 * math.pi, 10 ** 3.5),
    "limited_angle": Scenario("limited_angle", 90, math.pi, 10 ** 5.5),
}


def momentum_table(T: int, fista: bool = True) -> np.ndarray:
    """a_t for t = 1..T: (t-1)/(t+3) for the FISTA-type sequence of Sec. 3, else 0."""
    t = np.arange(1, T + 1, dtype=np.float64)
    return (t - 1.0) / (t + 3.0) if fista else np.zeros(T)


# ----------------------------------------------------------------------------------
# phantoms
# ----------------------------------------------------------------------------------

@dataclass
class Ellipses:
    cx: np.ndarray
    cy: np.ndarray
    a: np.ndarray
    b: np.ndarray
    phi: np.ndarray
    rho: np.ndarray
    extra: dict = field(default_factory=dict)


def random_ellipses(seed: int, count: int, n: int, pixel_mm: float = 1.0) -> Ellipses:
    rng = np.random.default_rng(seed)
    R = 0.5 * n * pixel_mm
    rad = 0.6 * R * np.sqrt(rng.random(count))
    ang = 2 * np.pi * rng.random(count)
    a = rng.uniform(0.05 * R, 0.35 * R, count)
    b = rng.uniform(0.05 * R, 0.35 * R, count)
    phi = rng.uniform(0.0, np.pi, count)
    rho = rng.random(count)
    return Ellipses(rad * np.cos(ang), rad * np.sin(ang), a, b, phi, rho)


def rasterise(e: Ellipses, n: int, pixel_mm: float = 1.0, sub: int = 4) -> np.ndarray:
    """Covered-area rasterisation by sub x sub point sampling; row r is y, column c is x."""
    img = np.zeros((n, n))
    h = pixel_mm
    offs = ((np.arange(sub) + 0.5) / sub - 0.5) * h
    centre = (np.arange(n) - 0.5 * (n - 1)) * h
    for i in range(len(e.cx)):
        ext = max(e.a[i], e.b[i]) + h
        c_lo = max(0, int(math.floor((e.cx[i] - ext) / h + 0.5 * (n - 1))))
        c_hi = min(n - 1, int(math.ceil((e.cx[i] + ext) / h + 0.5 * (n - 1))))
        r_lo = max(0, int(math.floor((e.cy[i] - ext) / h + 0.5 * (n - 1))))
        r_hi = min(n - 1, int(math.ceil((e.cy[i] + ext) / h + 0.5 * (n - 1))))
        if c_lo > c_hi or r_lo > r_hi:
            continue
        xs = (centre[c_lo:c_hi + 1][None, :, None, None] + offs[None, None, None, :]) - e.cx[i]
        ys = (centre[r_lo:r_hi + 1][:, None, None, None] + offs[None, None, :, None]) - e.cy[i]
        cp, sp = math.cos(e.phi[i]), math.sin(e.phi[i])
        u = xs * cp + ys * sp
        v = -xs * sp + ys * cp
        inside = (u / e.a[i]) ** 2 + (v / e.b[i]) ** 2 <= 1.0
        img[r_lo:r_hi + 1, c_lo:c_hi + 1] += e.rho[i] * inside.mean(axis=(2, 3))
    return img


def random_disks(seed: int, count: int, n: int, pixel_mm: float = 1.0) -> Ellipses:
    """A disk phantom: a background disk of radius 0.85 R and density 0.4, and `count`
    disks of various sizes inside it (radius uniform in [0.03 R, 0.2 R], centre uniform in
    the disc of radius 0.55 R, density uniform in [0.1, 0.6]); densities add."""
    rng = np.random.default_rng(seed)
    R = 0.5 * n * pixel_mm
    rad = 0.55 * R * np.sqrt(rng.random(count))
    ang = 2 * np.pi * rng.random(count)
    r = rng.uniform(0.03 * R, 0.2 * R, count)
    rho = rng.uniform(0.1, 0.6, count)
    cx = np.concatenate([[0.0], rad * np.cos(ang)])
    cy = np.concatenate([[0.0], rad * np.sin(ang)])
    rr = np.concatenate([[0.85 * R], r])
    return Ellipses(cx, cy, rr, rr.copy(), np.zeros(count + 1), np.concatenate([[0.4], rho]))


def transmission_data(ax: np.ndarray, i0: float, mu0: float, seed: int) -> np.ndarray:
    """Poisson transmission measurement and its log, in the phantom's density units:
    counts ~ Poisson(I0 exp(-mu0 Ax)), b = -log(max(counts, 0.5) / I0) / mu0
    (ax: line integrals of the density image, mm; mu0: attenuation per unit density, 1/mm;
    a zero count is read as half a count)."""
    ax = np.asarray(ax, dtype=np.float64)
    counts = np.random.default_rng(seed).poisson(i0 * np.exp(-mu0 * ax)).astype(np.float64)
    return -np.log(np.maximum(counts, 0.5) / i0) / mu0


def texture(seed: int, n: int, std: float = 0.02, smooth_px: float = 2.0) -> np.ndarray:
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    t = gaussian_filter(rng.standard_normal((n, n)), smooth_px)
    t *= std / t.std()
    centre = np.arange(n) - 0.5 * (n - 1)
    disc = (centre[None, :] ** 2 + centre[:, None] ** 2) <= (0.5 * n) ** 2
    return t * disc


def phantom(w: Workload, slice_index: int = 0) -> np.ndarray:
    """Ground truth x for a workload: float32 array, shape (n, n)."""
    seed = 1000 * w.seed_base + slice_index
    img = rasterise(random_ellipses(seed, w.n_ellipses, w.n), w.n)
    if w.texture:
        img = img + texture(seed + 500, w.n)
    return img.astype(np.float32)


# ----------------------------------------------------------------------------------
# noise and minibatches
# ----------------------------------------------------------------------------------

def standard_normal(seed: int, shape) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(shape)


def add_noise(ax: np.ndarray, eps: np.ndarray, kind: str, level: float) -> np.ndarray:
    """b = Ax + w with the configured noise model (data model of Sec. 1, Eq. (1))."""
    ax = np.asarray(ax, dtype=np.float64)
    peak = float(ax.max())
    if kind == "gaussian":
        return ax + level * peak * eps
    if kind == "poisson-like":
        return ax + level * np.sqrt(peak * np.clip(ax, 0.0, None)) * eps
    raise ValueError(kind)


def noise_seed(w: Workload, slice_index: int = 0) -> int:
    return 2000 * w.seed_base + slice_index


def subset_sequence(seed: int, T: int, n_sub: int) -> np.ndarray:
    return np.random.default_rng(seed).integers(0, n_sub, T).astype(np.int32)


def subset_views(s: int, n_sub: int, n_views: int) -> np.ndarray:
    """Views of subset s: k = s (mod n_sub), ascending."""
    return np.arange(s, n_views, n_sub, dtype=np.int32)
