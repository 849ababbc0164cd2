"""Serving benchmark: 48 simulated video streams of mixed resolution with
Poisson arrivals at 30-60 fps, served by the native continuous-batching loop
with the handcrafted and the learned scorer side by side.  Prints one JSON
line: per scorer the frames served, frames/s, p50/p99 latency from
submission to the result being seen on the host, mean batch size, and the
accuracy of the frames' own estimates and of the streams' filtered circles.

Each scorer's server is fed in real time from its creation.  The accuracy
is evaluated on the host after the serving run, on an evenly spaced sample
of the served frames (the normalised Hausdorff error of a 4K frame takes up
to a few tenths of a second), with a progress line per block of frames.

    python -m paper_2210_14771_amd.serve_bench [--streams 48] [--seconds 0.4]
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np

from . import api, evaluate, serve, train_scorer


def accuracy_sample(served, n: int) -> list:
    """At most n served records, evenly spaced in (stream, seq) order."""
    recs = sorted(served, key=lambda r: (r["stream"], r["seq"]))
    if len(recs) <= n:
        return recs
    idx = np.linspace(0, len(recs) - 1, n).round().astype(np.int64)
    return [recs[i] for i in np.unique(idx)]


def accuracy(served, streams, log=None, block: int = 16) -> dict:
    """Error of each record's own estimate and of its stream's filtered
    circle against the frame's ground truth."""
    by = {st.stream_id: st for st in streams}
    own, filt = [], []
    specs = []
    for r in served:
        st = by[r["stream"]]
        spec = st.specs[r["seq"] % len(st.specs)]
        specs.append(spec)
        cx, cy, rad, _, _, _, valid, _ = r["result"]
        own.append((cx, cy, rad, valid))
        fv, fx, fy, fr, _ = r["filtered"]
        filt.append((fx, fy, fr, fv))
    out = {}
    for name, rows in (("frame", own), ("filtered", filt)):
        a = np.array(rows, dtype=np.float64)
        errs = []
        for k in range(0, len(specs), block):
            sl = slice(k, k + block)
            errs.append(evaluate.frame_errors(specs[sl], a[sl, 0], a[sl, 1], a[sl, 2],
                                              a[sl, 3] != 0))
            if log:
                log(f"accuracy ({name}): {min(k + block, len(specs))} of {len(specs)} frames")
        out[name] = evaluate.summarise(np.concatenate(errs) if errs else np.zeros(0))
    return out


def run_benchmark(n_streams: int = 48, seconds: float = 0.4, frames_per_stream: int = 6,
                  max_batch: int = 64, budget_gib: float = 4.0, log=None,
                  accuracy_frames: int = 96) -> dict:
    """Per scorer one server, fed in real time from its creation: each
    frame submitted at its arrival time, the server stepped until every
    frame is served.  Then a second server takes the same frames as one
    backlog (every frame submitted at once, each stream's ring admitting two
    at a time): the throughput of continuous batching under full load; and
    a third the backlog with every frame lent (read in place, no ring
    copies, batches limited by max_batch only)."""
    import torch

    if log:
        log(f"rendering {n_streams} streams")
    streams = serve.make_streams(n_streams, frames_per_stream, seconds, seed=1)
    est = api.Estimator(0)
    kw = dict(n_hstrips=32, n_vstrips=32, ransac_attempts=1024)
    n_frames = sum(len(s.arrivals) for s in streams)
    line = {"metric": f"serving latency, {n_streams} mixed-resolution streams",
            "streams": n_streams, "seconds": seconds, "frames": n_frames,
            "arrival_fps": n_frames / seconds,
            "shapes": [f"{w}x{h}" for w, h in serve.SERVE_SHAPES],
            "latency": "submission to the result seen on the host"}
    runs = [("plain", dict(kw))]
    model = os.path.join(train_scorer.MODEL_DIR, train_scorer.MODEL_FILE)
    if os.path.exists(model):
        est.set_model(train_scorer.load_model(model))
        runs.append(("learned", dict(kw, scorer=1, fallback_inlier_frac=0.5)))
    model2d = os.path.join(train_scorer.MODEL_DIR, train_scorer.MODEL_FILE_2D)
    if os.path.exists(model2d):
        est.set_model_2d(train_scorer.load_model_2d(model2d))
        runs.append(("learned_2d", dict(kw, scorer=2, fallback_inlier_frac=0.5)))
    for name, params in runs:
        cfg = serve.server_config(max_batch=max_batch, hbm_budget=int(budget_gib * (1 << 30)),
                                  **params)
        srv = serve.Server(est, cfg)
        if log:
            log(f"serving ({name})")
        served, wall = serve.run(srv, streams, realtime=True, timeout_s=60, progress=log)
        stats = srv.stats()
        srv.close()
        rec = serve.latency_summary(served, wall)
        if log:
            log(f"served {len(served)} frames in {wall:.2f} s ({name})")
        rec["batches"] = stats["batches"]
        sample = accuracy_sample(served, accuracy_frames)
        rec["accuracy"] = accuracy(sample, streams, log)
        rec["accuracy"]["frames_evaluated"] = len(sample)
        srv = serve.Server(est, cfg)
        if log:
            log(f"serving ({name}, backlog)")
        served_b, wall_b = serve.run(srv, streams, realtime=False, timeout_s=60, progress=log)
        stats_b = srv.stats()
        srv.close()
        rec["backlog"] = dict(serve.latency_summary(served_b, wall_b),
                              batches=stats_b["batches"])
        # the same backlog with the frames lent to the server: read in
        # place, no ring copies
        srv = serve.Server(est, cfg)
        if log:
            log(f"serving ({name}, backlog, lent frames)")
        served_l, wall_l = serve.run(srv, streams, realtime=False, timeout_s=60, progress=log,
                                     lend=True)
        stats_l = srv.stats()
        srv.close()
        rec["backlog_lent"] = dict(serve.latency_summary(served_l, wall_l),
                                   batches=stats_l["batches"])
        line[name] = rec
    torch.cuda.synchronize()
    est.close()
    return line


def main():
    """The benchmark's command line."""
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--streams", type=int, default=48)
    ap.add_argument("--seconds", type=float, default=0.4)
    ap.add_argument("--frames-per-stream", type=int, default=6)
    ap.add_argument("--max-batch", type=int, default=64)
    ap.add_argument("--budget-gib", type=float, default=4.0)
    ap.add_argument("--accuracy-frames", type=int, default=96,
                    help="served frames per scorer whose accuracy is evaluated")
    a = ap.parse_args()
    import sys

    def log(msg):
        print("# " + msg, file=sys.stderr, flush=True)

    line = run_benchmark(a.streams, a.seconds, a.frames_per_stream, a.max_batch, a.budget_gib,
                         log, a.accuracy_frames)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
