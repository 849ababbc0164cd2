"""Pins of the normalised Hausdorff evaluation harness (Section 2.3, Eqs. 4-6)."""
import math

import numpy as np
from scipy.spatial.distance import directed_hausdorff

from paper_2210_14771_amd import evaluate as ev


def test_two_full_circles_closed_form():
    # for two circles fully inside the frame, H = |dc| + |dr|
    w, h = 1920, 1080
    for (c1, c2) in [((960, 540, 400), (963, 544, 410)), ((900, 500, 300), (900, 500, 305)),
                     ((1000, 600, 350), (990, 590, 350))]:
        d = math.hypot(c1[0] - c2[0], c1[1] - c2[1]) + abs(c1[2] - c2[2])
        got = ev.normalised_hausdorff(w, h, c1, c2)
        assert abs(got - d) < 0.06


def test_identical_and_rectangles():
    assert ev.normalised_hausdorff(640, 480, None, None) == 0.0
    assert ev.normalised_hausdorff(640, 480, (320, 240, 250), (320, 240, 250)) == 0.0


def test_matches_scipy_directed_hausdorff():
    a = ev.edge_points(640, 480, (300, 250, 280))
    b = ev.edge_points(640, 480, (330, 230, 300))
    ref = max(directed_hausdorff(a, b)[0], directed_hausdorff(b, a)[0])
    assert abs(ev.hausdorff(a, b) - ref) < 1e-9


def test_directed_distance_equals_brute_force():
    # the subset bound only prunes points that cannot attain the maximum:
    # scattered clouds, clustered clouds and curves, several subset steps
    rng = np.random.default_rng(3)
    for trial in range(24):
        na, nb = rng.integers(1, 900, 2)
        a = rng.normal(0, rng.uniform(1, 50), (na, 2)) + rng.uniform(-80, 80, 2)
        if trial % 3 == 0:
            t = rng.uniform(0, 2 * np.pi, nb)
            b = np.stack([np.cos(t), np.sin(t)], 1) * rng.uniform(5, 60)
        else:
            b = rng.normal(0, rng.uniform(1, 50), (nb, 2))
        brute = np.sqrt(((a[:, None, :] - b[None, :, :]) ** 2).sum(-1)).min(1).max()
        for step in (1, 2, 7, 16, 64):
            assert abs(ev.directed_hausdorff(a, b, step) - brute) < 1e-9, (trial, step)


def test_far_concentric_and_missing_estimates_match_scipy():
    # the cases the bound is for: estimates far from the truth, a missing
    # estimate (the rectangle), concentric circles a few pixels apart
    w, h = 160, 90
    gt = (83.0, 43.0, 49.5)
    for est in (gt, (83.2, 42.9, 49.8), (83.0, 43.0, 54.0), (83.0, 43.0, 69.5),
                (30.0, 60.0, 12.0), (150.0, -20.0, 40.0), None):
        a, b = ev.edge_points(w, h, gt), ev.edge_points(w, h, est)
        ref = max(directed_hausdorff(a, b)[0], directed_hausdorff(b, a)[0])
        assert abs(ev.hausdorff(a, b) - ref) < 1e-9, est


def test_normalisation_eq6():
    # 640x480 frame: 1 native px counts as 2202.9 / 800 normalised px
    got = ev.normalised_hausdorff(640, 480, (320, 240, 100), (320, 240, 101))
    assert abs(got - 2202.907 / 800.0) < 0.2


def test_clipped_circle_edges():
    # a partial circle: its edge includes the rectangle sides inside the disc
    pts = ev.edge_points(1920, 1080, (960, 540, 1000))
    assert np.any(np.isclose(pts[:, 1], -0.5)) and np.any(np.isclose(pts[:, 0], -0.5))
    # disc covering the whole frame equals the rectangle
    big = ev.normalised_hausdorff(1920, 1080, (960, 540, 5000), None)
    assert big == 0.0


def test_summary():
    s = ev.summarise([1.0, 3.0, 20.0, 30.0])
    assert s["frac_le_2px"] == 0.25 and s["miss_pct"] == 50.0 and s["bad_miss_pct"] == 25.0


def test_breakdown_by_kind_and_border_sigma():
    from paper_2210_14771_amd import synth
    specs = [synth.FrameSpec(1920, 1080, k, 960.0, 540.0, 500.0, s, 1.0, 0.0, 100.0)
             for k, s in [(0, 3.0), (1, 5.0), (2, 7.0), (0, 9.0), (1, 4.0)]]
    b = ev.breakdown(specs, [1.0, 3.0, 0.0, 1.5, 2.0], [1, 1, 0, 1, 1])
    assert b["by_kind"]["partial"] == {"n": 2, "frac_le_2px": 1.0, "median_px": 1.25,
                                       "valid_frac": 1.0}
    assert b["by_kind"]["full"]["n"] == 2 and b["by_kind"]["full"]["frac_le_2px"] == 0.5
    assert b["by_kind"]["noborder"]["valid_frac"] == 0.0
    # border-free frames have no border noise: left out of the sigma buckets
    sig = b["by_border_sigma"]
    assert sig["0-4"]["n"] == 1 and sig["4-6"]["n"] == 2 and sig["6-8"] == {"n": 0}
    assert sig[">=8"]["frac_le_2px"] == 1.0
