"""The random geometries of the parity tests are valid plan inputs: the image circle lies inside the
source circle, the fan is narrower than 90 degrees, and the pooling factor divides the grid."""
import math

import pytest

from random_geometry import coarse_random_geometry, random_geometry


@pytest.mark.parametrize("make", [random_geometry, coarse_random_geometry])
def test_random_geometries_are_valid(make):
    for seed in range(64):
        g, f = make(seed)
        radius = 0.5 * g["pixel_mm"] * math.hypot(g["nx"], g["ny"])
        assert radius < g["sod_mm"], seed
        assert 0.5 * (g["n_bins"] - 1) * g["det_pitch_mm"] + abs(g["det_offset_mm"]) < g["sdd_mm"], seed
        assert g["nx"] % f == 0 and g["ny"] % f == 0, seed
        assert 1 <= g["n_views"] and 1 <= g["n_bins"] and g["angle_step_rad"] > 0, seed
