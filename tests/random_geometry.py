"""Seeded random valid fan-beam geometries for the parity tests (inputs only: sizes, distances,
detector and angles; no part of the method's arithmetic)."""
import math

import numpy as np


def random_geometry(seed):
    """A seeded random valid geometry: grid up to 80 x 80 (often with a common factor), pixel 0.5 to
    2 mm, source at 1.45 to 20 image circumradii, detector pitch and offset drawn with the fan kept
    under 90 degrees, a random start angle, sometimes a limited angular range; and a pooling factor."""
    rng = np.random.default_rng(seed)
    nx, ny = int(rng.integers(1, 81)), int(rng.integers(1, 81))
    if rng.random() < 0.5:
        k = int(rng.choice([2, 3, 4, 8]))
        nx, ny = max(k, nx - nx % k), max(k, ny - ny % k)
    h = float(rng.uniform(0.5, 2.0))
    radius = 0.5 * h * math.hypot(nx, ny)
    sod = radius * float(rng.uniform(1.45, 20.0))
    sdd = sod * float(rng.uniform(1.2, 3.0))
    V, B = int(rng.integers(1, 41)), int(rng.integers(1, 121))
    pitch = float(rng.uniform(0.2, 3.0)) * h * sdd / sod
    off = float(rng.uniform(-0.3, 0.3)) * B * pitch
    umax = 0.5 * (B - 1) * pitch + abs(off)
    if umax >= 0.95 * sdd:
        scale = 0.9 * sdd / umax
        pitch, off = pitch * scale, off * scale
    span = 2 * math.pi * (1.0 if rng.random() < 0.7 else float(rng.uniform(0.3, 1.0)))
    gd = dict(nx=nx, ny=ny, pixel_mm=h, n_views=V, n_bins=B, sod_mm=sod, sdd_mm=sdd, det_pitch_mm=pitch,
              det_offset_mm=off, angle0_rad=float(rng.uniform(0, 2 * math.pi)), angle_step_rad=span / V)
    divs = [f for f in range(2, 9) if nx % f == 0 and ny % f == 0]
    return gd, (int(rng.choice(divs)) if divs else 1)


def coarse_random_geometry(seed):
    """A random geometry as above with a coarse stage: factor 8, 16 or 32 on a grid of 1 to 3 stage
    pixels a side, the source at 1.45 to 4 image circumradii (back-projection blocks that often reach
    the source circle)."""
    gd, _ = random_geometry(seed)
    rng = np.random.default_rng(10_000 + seed)
    f = int(rng.choice([8, 16, 32]))
    gd["nx"], gd["ny"] = f * int(rng.integers(1, 4)), f * int(rng.integers(1, 4))
    radius = 0.5 * gd["pixel_mm"] * math.hypot(gd["nx"], gd["ny"])
    gd["sod_mm"] = radius * float(rng.uniform(1.45, 4.0))
    gd["sdd_mm"] = 2.0 * gd["sod_mm"]
    umax = 0.5 * (gd["n_bins"] - 1) * gd["det_pitch_mm"] + abs(gd["det_offset_mm"])
    if umax >= 0.95 * gd["sdd_mm"]:
        scale = 0.9 * gd["sdd_mm"] / umax
        gd["det_pitch_mm"] *= scale
        gd["det_offset_mm"] *= scale
    return gd, f
