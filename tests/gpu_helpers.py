"""Shared plumbing of the GPU parity tests: run the HIP path through the C ABI
and the CPU oracle on the same seeded inputs, and compare element by element."""
from __future__ import annotations

import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle
from paper_2210_14771_amd import api, synth

# Tolerance on circle parameters: the numeric contract makes both sides
# compute the same IEEE operations in the same order, so the values are
# expected to be bit-identical; 1e-3 px is the stated acceptance bound.
CIRCLE_TOL_PX = 1e-3


def say(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_params(**kw) -> oracle.Params:
    kw = dict(kw)
    if "ransac_attempts" in kw:
        kw["attempts"] = kw.pop("ransac_attempts")
    return oracle.params(**kw)


def gen_batch(wl, n, start=0, width=None, height=None, threads=8):
    with ThreadPoolExecutor(threads) as ex:
        out = list(ex.map(lambda i: synth.make_frame(wl, i, width, height), range(start, start + n)))
    return np.stack([o[0] for o in out]), [o[1] for o in out]


def run_gpu(est, frames_dev, params_kw, uids, what=("res",)):
    import torch
    p = api.default_params(**params_kw)
    out = {}
    if "pts" in what:
        r, pts = est.debug_candidates(frames_dev, p, uids)
        torch.cuda.synchronize()
        out["pts"] = api.points_numpy(pts)
        out["res"] = r.numpy()
    if "att" in what:
        r, att = est.debug_attempts(frames_dev, p, uids)
        torch.cuda.synchronize()
        out["att"] = api.attempts_numpy(att)
        out["res_att"] = r.numpy()
    if "res" in what:
        r = est.estimate_area(frames_dev, p, uids)
        torch.cuda.synchronize()
        out["res"] = r.numpy()
    return out


def run_oracle(frames, params_kw, uids, threads=8, attempts=False):
    p = oracle_params(**params_kw)
    B = len(frames)
    res, pts, att = [None] * B, [None] * B, [None] * B

    def one(i):
        if attempts:
            res[i], pts[i], att[i] = oracle.estimate(frames[i], p, int(uids[i]), True, True)
        else:
            res[i], pts[i] = oracle.estimate(frames[i], p, int(uids[i]), True)

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(one, range(B)))
    return res, pts, att


def assert_points_equal(gpu_pts, ora_pts):
    """Candidates: coordinates and score bits identical."""
    B = len(ora_pts)
    for f in range(B):
        g, o = gpu_pts[f], ora_pts[f]
        bad = np.flatnonzero((g["x"] != o["x"]) | (g["y"] != o["y"])
                             | (g["score"].view(np.uint32) != o["score"].view(np.uint32)))
        assert bad.size == 0, (
            f"frame {f}: {bad.size} candidates differ, first #{bad[0]}: gpu "
            f"({g['x'][bad[0]]},{g['y'][bad[0]]},{g['score'][bad[0]]!r}) oracle "
            f"({o['x'][bad[0]]},{o['y'][bad[0]]},{o['score'][bad[0]]!r})")


def assert_attempts_equal(gpu_att, ora_att):
    """Per-attempt triple, status, inlier count and score sum identical;
    circle within CIRCLE_TOL_PX (and counted bitwise)."""
    B = len(ora_att)
    n_bits_equal = 0
    n_total = 0
    for f in range(B):
        g, o = gpu_att[f], ora_att[f]
        for k in ("status", "fail_stage", "i0", "i1", "i2", "inliers", "qsum"):
            bad = np.flatnonzero(g[k] != o[k])
            assert bad.size == 0, (f"frame {f} field {k}: {bad.size} attempts differ, first "
                                   f"#{bad[0]}: gpu {g[k][bad[0]]} oracle {o[k][bad[0]]}")
        for k in ("cx", "cy", "r2"):
            d = np.abs(g[k] - o[k])
            tol = CIRCLE_TOL_PX if k != "r2" else CIRCLE_TOL_PX * (2 * np.sqrt(np.abs(o[k])) + 1)
            assert np.all(d <= tol), f"frame {f} field {k}: max diff {d.max()}"
            n_bits_equal += int(np.sum(g[k].view(np.uint64) == o[k].view(np.uint64)))
            n_total += d.size
    return n_bits_equal, n_total


def assert_results_equal(gpu_res, ora_res):
    B = len(ora_res)
    for f in range(B):
        g, o = gpu_res[f], ora_res[f]
        for k in ("valid", "reason", "n_points", "inliers"):
            assert g[k] == o[k], f"frame {f} field {k}: gpu {g[k]} oracle {o[k]}"
        for k in ("cx", "cy", "r"):
            assert abs(float(g[k]) - float(o[k])) <= CIRCLE_TOL_PX, (
                f"frame {f} field {k}: gpu {g[k]!r} oracle {o[k]!r}")
        assert abs(float(g["score"]) - float(o["score"])) <= 1e-6
