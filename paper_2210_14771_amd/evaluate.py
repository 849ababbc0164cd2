"""Normalised Hausdorff error of a content-area estimate (Section 2.3).

Evaluation harness, not part of the estimator: it compares an estimated
content area with the ground truth of a synthetic frame.

The content area is the disc intersected with the sensor rectangle
[-0.5, W-0.5] x [-0.5, H-0.5] in pixel-index coordinates, or the whole
rectangle when there is no valid circle (Section 2.2.1).  Its edge is
sampled every <= 0.1 px: the arcs of the circle inside the rectangle plus
the rectangle's sides inside the disc.  H(A, B) = max(h(A, B), h(B, A)) with
Euclidean distances (Eqs. 4-5), scaled by the ratio of the 1920x1080
diagonal to the frame's diagonal (Eq. 6).  Misses and bad misses are errors
above 15 px and 25 px.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial import cKDTree

D_REF = math.hypot(1920.0, 1080.0)
MISS_PX = 15.0
BAD_MISS_PX = 25.0


def edge_points(w: int, h: int, circle: tuple[float, float, float] | None,
                spacing: float = 0.1) -> np.ndarray:
    """Points along the edge of disc(circle) intersected with the frame rectangle."""
    x0, x1, y0, y1 = -0.5, w - 0.5, -0.5, h - 0.5
    sides = []
    for (ax, ay, bx, by) in ((x0, y0, x1, y0), (x1, y0, x1, y1), (x1, y1, x0, y1),
                             (x0, y1, x0, y0)):
        n = int(math.ceil(math.hypot(bx - ax, by - ay) / spacing)) + 1
        t = np.linspace(0.0, 1.0, n)
        sides.append(np.stack([ax + t * (bx - ax), ay + t * (by - ay)], 1))
    rect = np.concatenate(sides)
    if circle is None:
        return rect
    cx, cy, r = circle
    inside = np.hypot(rect[:, 0] - cx, rect[:, 1] - cy) <= r
    n = int(math.ceil(2 * math.pi * r / spacing)) + 1
    a = np.linspace(0.0, 2 * math.pi, n, endpoint=False)
    arc = np.stack([cx + r * np.cos(a), cy + r * np.sin(a)], 1)
    tol = 1e-9
    keep = ((arc[:, 0] >= x0 - tol) & (arc[:, 0] <= x1 + tol) & (arc[:, 1] >= y0 - tol)
            & (arc[:, 1] <= y1 + tol))
    if not keep.any():
        # disc covers the rectangle, or misses it entirely
        return rect if inside.all() else arc
    return np.concatenate([arc[keep], rect[inside]])


def directed_hausdorff(a: np.ndarray, b: np.ndarray, step: int = 16) -> float:
    """h(A, B) = max over a of the distance to its nearest point of b, exact.

    Nearest-neighbour queries against every point of b are slow for points
    far from b, so every a is first measured against the subset b[::step]:
    that distance u(a) is an upper bound, and u(a) - delta a lower bound,
    where delta is the largest distance from a point of b to the subset.  So
    h >= max u - delta, and only the points with u(a) >= max u - delta can
    attain the maximum; those alone are measured against all of b."""
    sub = cKDTree(b[::step])
    delta = sub.query(b, workers=-1)[0].max()
    u = sub.query(a, workers=-1)[0]
    cand = u >= u.max() - delta
    return float(cKDTree(b).query(a[cand], workers=-1)[0].max())


def hausdorff(a: np.ndarray, b: np.ndarray) -> float:
    """H(A, B) = max(h(A, B), h(B, A)) over the two point sets (Eq. 4)."""
    return max(directed_hausdorff(a, b), directed_hausdorff(b, a))


def normalised_hausdorff(w: int, h: int, gt: tuple[float, float, float] | None,
                         est: tuple[float, float, float] | None) -> float:
    """NH(A, B) = (d / d_I) H(A, B), d = 1920x1080 diagonal, d_I = frame diagonal."""
    return hausdorff(edge_points(w, h, gt), edge_points(w, h, est)) * D_REF / math.hypot(w, h)


def summarise(errors) -> dict:
    e = np.asarray(errors, dtype=np.float64)
    if e.size == 0:
        return {}
    return {
        "mean_px": float(e.mean()),
        "median_px": float(np.median(e)),
        "p95_px": float(np.percentile(e, 95)),
        "frac_le_2px": float((e <= 2.0).mean()),
        "miss_pct": float(100.0 * (e > MISS_PX).mean()),
        "bad_miss_pct": float(100.0 * (e > BAD_MISS_PX).mean()),
        "n": int(e.size),
    }


def frame_errors(specs, cx, cy, r, valid) -> np.ndarray:
    """Normalised Hausdorff error of each estimate against its FrameSpec."""
    out = []
    for i, s in enumerate(specs):
        gt = (s.cx, s.cy, s.r) if s.has_border else None
        est = (float(cx[i]), float(cy[i]), float(r[i])) if bool(valid[i]) else None
        out.append(normalised_hausdorff(s.width, s.height, gt, est))
    return np.asarray(out)


# border noise sigma buckets of the breakdown (the 1080p workloads draw
# sigma in 2-8, the hard frames in 2-12)
SIGMA_BUCKETS = ((0.0, 4.0), (4.0, 6.0), (6.0, 8.0), (8.0, 100.0))


def breakdown(specs, errors, valid) -> dict:
    """Share of frames within 2 px, median error, valid share and count per
    frame kind and per border noise sigma bucket."""
    from .synth import KIND_NAMES
    e = np.asarray(errors, dtype=np.float64)
    v = np.asarray(valid, dtype=bool)

    def cell(sel):
        sel = np.asarray(sel, dtype=bool)
        if not sel.any():
            return {"n": 0}
        return {"n": int(sel.sum()), "frac_le_2px": float((e[sel] <= 2.0).mean()),
                "median_px": float(np.median(e[sel])), "valid_frac": float(v[sel].mean())}

    kinds = np.array([s.kind for s in specs])
    sig = np.array([s.border_sigma for s in specs])
    by_kind = {name: cell(kinds == k) for k, name in KIND_NAMES.items()}
    by_sigma = {f"{lo:g}-{hi:g}" if hi < 100 else f">={lo:g}": cell((sig >= lo) & (sig < hi)
                                                                    & (kinds != 2))
                for lo, hi in SIGMA_BUCKETS}
    return {"by_kind": by_kind, "by_border_sigma": by_sigma}


def accuracy(est, frames_dev, specs, params, uids=None, by: bool = False) -> dict:
    """Run the estimator once on device frames and summarise its error
    against the ground truth (plus the valid and fallback shares; with
    `by`, the breakdown by frame kind and border noise)."""
    import torch
    B = len(specs)
    res = est.estimate_area(frames_dev, params, list(range(B)) if uids is None else uids)
    torch.cuda.synchronize()
    raw = res.raw.cpu().numpy()
    cx, cy, r = (raw[:, k].view(np.float32) for k in range(3))
    valid = raw[:, 6] != 0
    errs = frame_errors(specs, cx, cy, r, valid)
    out = summarise(errs)
    out["valid_frac"] = float(valid.mean())
    out["fallback_frac"] = float((raw[:, 7] >= 256).mean())
    if by:
        out.update(breakdown(specs, errs, valid))
    return out

