"""Pins of the oracle's last steps (Section 2.2.5 and Appendix A, Table A1):
the radius and centre limits of an attempt, the choice of the best attempt
with its tie-break, the circle-score threshold t_cs, and the integer luma.

Each case is built so that a plausible slip fails it: the width swapped for
the height in a limit, the radius compared squared, an inclusive bound made
strict, the frame centre taken at (W/2, H/2), the best attempt taken last
among equals or from outside the limits, the threshold not divided by P, and
the luma truncated instead of rounded.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2210_14771_amd import synth

Q24 = 1 << 24


# --------------------------------------------- radius and centre limits ---

# A tall frame (W < H), so a limit scaled by the height instead of the width
# gives a different outcome.  Three integer points span a rectangle's corner;
# the circle through them has the rectangle's centre and half its diagonal,
# both exact in float64.  refine_iters = 0 keeps that circle as the attempt's.
TALL_W, TALL_H = 200, 400


def _corner_attempt(x0, x1, y0, y1, **kw):
    p = oracle.params(sampler=1, attempts=1, refine_iters=0, **kw)
    xs = [x0, x1, x0]
    ys = [y0, y0, y1]
    att = oracle.ransac_attempts(xs, ys, [Q24 // 2] * 3, TALL_W, TALL_H, 0, p)[0]
    cx, cy = (x0 + x1) / 2, (y0 + y1) / 2
    r2 = ((x1 - x0) ** 2 + (y1 - y0) ** 2) / 4
    assert (att["cx"], att["cy"], att["r2"]) == (cx, cy, r2)   # the exact circle
    assert att["inliers"] == 3
    return att


# (case, corners, expected status): limits 0.1 W = 20, 0.8 W = 160 and
# 0.2 W = 40 are exact in float64 for W = 200
LIMIT_CASES = [
    # radius exactly r_max W (96^2 + 128^2 = 160^2): inclusive, kept
    ("r_max_on", (4, 196, 72, 328), 2),
    # radius sqrt(192^2 + 257^2) / 2 = 160.40 > r_max W (but < r_max H)
    ("r_max_over", (4, 196, 72, 329), 1),
    # radius exactly r_min W (12^2 + 16^2 = 20^2): inclusive, kept
    ("r_min_on", (88, 112, 184, 216), 2),
    # radius sqrt(24^2 + 31^2) / 2 = 19.60 < r_min W
    ("r_min_under", (88, 112, 184, 215), 1),
    # centre (123.5, 231.5): offset (24, 32) from (99.5, 199.5), exactly d_max W
    ("d_max_on", (93, 154, 201, 262), 2),
    # centre (124.5, 231.5): offset (25, 32), 41 > d_max W (but < d_max H,
    # and within d_max W of (W/2, H/2))
    ("d_max_over", (94, 155, 201, 262), 1),
    # centre offset (0, 41) straight down the tall axis: beyond d_max W
    ("d_max_over_y", (70, 129, 212, 269), 1),
]


@pytest.mark.parametrize("case,corners,status", LIMIT_CASES, ids=[c[0] for c in LIMIT_CASES])
def test_attempt_limits_on_tall_frame(case, corners, status):
    att = _corner_attempt(*corners)
    assert att["status"] == status
    # the same facts stated with Euclidean distances and exact rationals
    x0, x1, y0, y1 = corners
    cx, cy = Fraction(x0 + x1, 2), Fraction(y0 + y1, 2)
    r2 = (Fraction(x1 - x0) ** 2 + Fraction(y1 - y0) ** 2) / 4
    d2 = (cx - Fraction(TALL_W - 1, 2)) ** 2 + (cy - Fraction(TALL_H - 1, 2)) ** 2
    keep = (Fraction(20) ** 2 <= r2 <= Fraction(160) ** 2) and d2 <= Fraction(40) ** 2
    assert status == (2 if keep else 1)


def test_cases_tell_width_from_height():
    # the same cases with the limits scaled by the height: the outcome of each
    # bound's discriminating case changes, so a W/H slip fails above
    def status(corners, ext):
        x0, x1, y0, y1 = corners
        r = math.hypot(x1 - x0, y1 - y0) / 2
        d = math.hypot((x0 + x1) / 2 - (TALL_W - 1) / 2, (y0 + y1) / 2 - (TALL_H - 1) / 2)
        return 2 if 0.1 * ext <= r <= 0.8 * ext and d <= 0.2 * ext else 1

    assert all(status(c, TALL_W) == st for _, c, st in LIMIT_CASES)
    differ = {name for name, c, st in LIMIT_CASES if status(c, TALL_H) != st}
    assert {"r_min_on", "r_max_over", "d_max_over", "d_max_over_y"} <= differ


def test_limit_parameters_move_the_bounds():
    # raising r_max by one part in 10^9 keeps nothing new; by 1 % keeps r = 160.40
    assert _corner_attempt(4, 196, 72, 329, r_max=0.8 * (1 + 1e-9))["status"] == 1
    assert _corner_attempt(4, 196, 72, 329, r_max=0.81)["status"] == 2
    assert _corner_attempt(94, 155, 201, 262, d_max=0.21)["status"] == 2
    assert _corner_attempt(88, 112, 184, 215, r_min=0.09)["status"] == 2


# ------------------------------------ best attempt and circle threshold ---

def _disc_frame(W=160, H=120, cx=70.0, cy=64.0, r=50.0):
    """A bright disc on black: every strip crossing the disc yields an exact
    edge point, a strip that misses it yields only zero scores (dropped by
    t_ps), so fewer points are kept than there are candidates."""
    yy, xx = np.mgrid[0:H, 0:W]
    disc = (xx - cx) ** 2 + (yy - cy) ** 2 <= r * r
    return np.repeat(np.where(disc, 160, 0).astype(np.uint8)[..., None], 3, axis=2)


def _py_select(att, P, t_cs):
    """Section 2.2.5's choice: the kept attempt of largest summed score,
    the smallest index among equals; valid when that sum over P reaches t_cs
    (compared as exact rationals)."""
    kept = np.flatnonzero(att["status"] == 2)
    if len(kept) == 0:
        return -1, 0, 2
    q = att["qsum"][kept]
    best = int(kept[np.flatnonzero(q == q.max())[0]])
    valid = Fraction(int(att["qsum"][best]), Q24 * P) >= Fraction(t_cs)
    return best, int(valid), 0 if valid else 3


def test_threshold_is_inclusive_and_divided_by_p():
    frame = _disc_frame()
    p = oracle.params(n_hstrips=2, n_vstrips=2, attempts=64)
    P = 8                               # a power of two: q / (2^24 P) is exact
    res, pts, att = oracle.estimate(frame, p, uid=5, with_points=True, with_attempts=True)
    assert res["valid"] == 1 and 3 <= res["n_points"] < P
    q = int(res["qsum"])
    assert q > 1
    assert res["score"] == np.float32(q / (Q24 * P))
    cases = [(Fraction(q, Q24 * P), 1, 0), (Fraction(q + 1, Q24 * P), 0, 3),
             (Fraction(q - 1, Q24 * P), 1, 0)]
    for t, valid, reason in cases:
        t_cs = float(t)
        assert Fraction(t_cs) == t          # exact: the bound sits on the sum
        r = oracle.estimate(frame, oracle.params(n_hstrips=2, n_vstrips=2, attempts=64,
                                                 t_cs=t_cs), uid=5)
        assert (r["valid"], r["reason"]) == (valid, reason), t
        # the threshold changes the verdict only, never the circle
        assert (r["qsum"], r["best_attempt"], r["cxd"], r["r2d"]) == \
            (res["qsum"], res["best_attempt"], res["cxd"], res["r2d"])
    # dividing by the kept points n instead of P would have moved the bound
    n = int(res["n_points"])
    assert Fraction(q, Q24 * n) != Fraction(q, Q24 * P)


def test_best_attempt_tie_goes_to_smallest_index():
    # every triple of points on one exact disc edge refits to the same circle:
    # all kept attempts tie on the summed score
    frame = _disc_frame()
    p = oracle.params(n_hstrips=2, n_vstrips=2, attempts=64)
    res, att = oracle.estimate(frame, p, uid=5, with_attempts=True)
    kept = np.flatnonzero(att["status"] == 2)
    top = kept[att["qsum"][kept] == att["qsum"][kept].max()]
    assert len(top) >= 2
    assert res["best_attempt"] == top[0]
    best, valid, reason = _py_select(att, 8, p.t_cs)
    assert res["best_attempt"] == best == top.min()


def _tiny_frame(seed):
    fr, specs = synth.make_batch(synth.SMALL_640x480, 1, start=seed)
    return fr[0][::5, ::5].copy()       # 128 x 96


@pytest.mark.parametrize("seed", [1, 4, 5, 6])
@pytest.mark.parametrize("r_max", [0.8, 0.3])
def test_selection_matches_independent_statement(seed, r_max):
    frame = _tiny_frame(seed)
    p = oracle.params(n_hstrips=4, n_vstrips=3, attempts=512, r_max=r_max)
    P = 14
    res, att = oracle.estimate(frame, p, uid=seed, with_attempts=True)
    best, valid, reason = _py_select(att, P, p.t_cs)
    assert res["best_attempt"] == best
    assert (res["valid"], res["reason"]) == (valid, reason)
    if best >= 0:
        a = att[best]
        assert (res["qsum"], res["inliers"], res["cxd"], res["cyd"], res["r2d"]) == \
            (a["qsum"], a["inliers"], a["cx"], a["cy"], a["r2"])


def test_selection_skips_higher_scoring_rejected_attempts():
    # with a tight r_max the circles with the most inliers are rejected, and
    # the chosen attempt is a kept one of lower score
    seen = 0
    for seed in (1, 4, 5, 6):
        frame = _tiny_frame(seed)
        p = oracle.params(n_hstrips=4, n_vstrips=3, attempts=512, r_max=0.3)
        res, att = oracle.estimate(frame, p, uid=seed, with_attempts=True)
        if res["best_attempt"] >= 0 and att["qsum"][att["status"] == 1].max(initial=0) > res["qsum"]:
            seen += 1
    assert seen >= 1


def test_frames_without_kept_attempts_report_reason_2():
    frame = _tiny_frame(1)
    p = oracle.params(n_hstrips=4, n_vstrips=3, attempts=256, r_max=0.01)
    res, att = oracle.estimate(frame, p, uid=1, with_attempts=True)
    assert res["n_points"] >= 3 and not np.any(att["status"] == 2)
    assert (res["valid"], res["reason"], res["best_attempt"]) == (0, 2, -1)


# ------------------------------------------------------------- luma -----

def test_luma_rounds_half_up():
    """Y is the integer nearest to (77 R + 150 G + 29 B) / 256, halves
    rounded up: exact rationals over every (R, G) and three B values."""
    half = Fraction(1, 2)
    for b in (0, 101, 255):
        for r in range(256):
            for g in range(256):
                s = 77 * r + 150 * g + 29 * b
                y = oracle.luma(r, g, b)
                assert y == math.floor(Fraction(s, 256) + half)
                assert abs(Fraction(y) - Fraction(s, 256)) <= half
    # a grey pixel keeps its value (the weights sum to 256)
    assert all(oracle.luma(v, v, v) == v for v in range(256))
