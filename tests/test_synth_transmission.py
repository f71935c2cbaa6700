"""Input generation for the paper's experiments (Sec. 3): Poisson transmission data and
its log, in density units, and the scenario geometries (no GPU)."""
import math

import numpy as np

from paper_2203_07308_amd import synth


def test_log_data_tends_to_line_integrals_at_high_count():
    ax = np.linspace(0.0, 150.0, 4001).reshape(1, -1)
    b = synth.transmission_data(ax, 1e15, 0.02, 3)
    # Poisson relative deviation ~ (I0 e^{-3})^{-1/2} ~ 1.4e-7, divided by mu0 = 0.02
    assert np.max(np.abs(b - ax)) < 1e-4


def test_zero_counts_are_read_as_half_a_count():
    ax = np.full((3, 50), 400.0)  # I0 e^{-8} ~ 0.03 counts: almost all zero
    b = synth.transmission_data(ax, 100.0, 0.02, 4)
    counts0 = np.isclose(b, -math.log(0.5 / 100.0) / 0.02)
    assert counts0.mean() > 0.9
    assert np.all(b[~counts0] <= -math.log(1.0 / 100.0) / 0.02 + 1e-9)


def test_mean_count_follows_beer_lambert():
    ax = np.full((200, 200), 50.0)
    b = synth.transmission_data(ax, 1e4, 0.02, 5)
    counts = 1e4 * np.exp(-0.02 * b)  # invert the log: the drawn counts
    assert abs(counts.mean() - 1e4 * math.exp(-1.0)) < 5 * math.sqrt(1e4 * math.exp(-1.0) / counts.size)
    np.testing.assert_allclose(counts, np.round(counts), atol=1e-6)


def test_scenarios_match_the_paper_shapes():
    sv, ld, la = (synth.SCENARIOS[k] for k in ("sparse_view", "low_dose", "limited_angle"))
    for sc, V, span, i0 in ((sv, 90, 360, 10 ** 5.5), (ld, 360, 360, 10 ** 3.5), (la, 90, 180, 10 ** 5.5)):
        g = sc.geometry
        assert (g["nx"], g["ny"], g["n_bins"], g["n_views"]) == (256, 256, 228, V)
        assert g["n_views"] * g["n_bins"] in (20520, 82080)
        assert math.isclose(math.degrees(g["angle_step_rad"] * V), span)
        assert sc.i0 == i0
        # the 228 bins span the 256 mm field of view at the isocentre
        assert math.isclose(g["n_bins"] * g["det_pitch_mm"] * g["sod_mm"] / g["sdd_mm"], 256.0)
        assert [f for f, _ in sc.stages] == [4, 2]  # m1 = d / 16, m2 = d / 4
    x = sv.phantom()
    assert x.shape == (256, 256) and x.min() >= 0.0 and 0.4 <= x.max() <= 0.4 + 0.6 * 10
