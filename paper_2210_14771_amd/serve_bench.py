"""Serving benchmark: 48 simulated video streams of mixed resolution with
Poisson arrivals at 30-60 fps, served by the native continuous-batching loop
with the handcrafted and the learned scorer side by side.  Prints one JSON
line: per scorer the frames served, frames/s, p50/p99 latency from
submission to the result being seen on the host, mean batch size, and the
accuracy of the frames' own estimates and of the streams' filtered circles.

    python -m paper_2210_14771_amd.serve_bench [--streams 48] [--seconds 0.3]
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np

from . import api, evaluate, serve, train_scorer


def accuracy(served, streams) -> dict:
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
        e = evaluate.frame_errors(specs, a[:, 0], a[:, 1], a[:, 2], a[:, 3] != 0)
        out[name] = evaluate.summarise(e)
    return out


OPEN_ISSUE = ("serve_bench is switched off: its realtime run (after a warm-up server in the "
              "same process) stopped making progress on the GPU three times; the cause is not "
              "found yet, so this case is not run until it is")


def main():
    raise SystemExit(OPEN_ISSUE)


def run_benchmark():
    """The benchmark proper (not run while OPEN_ISSUE stands)."""
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--streams", type=int, default=48)
    # a server has so far only been run to about 900 batches (0.4 s of the
    # 48 streams); a 2 s run stopped making progress after 2178 batches, cause
    # not found, so the default window stays well inside the tested range
    ap.add_argument("--seconds", type=float, default=0.3)
    ap.add_argument("--frames-per-stream", type=int, default=16)
    ap.add_argument("--max-batch", type=int, default=64)
    ap.add_argument("--budget-gib", type=float, default=4.0)
    a = ap.parse_args()
    import sys
    import torch

    def log(msg):
        print("# " + msg, file=sys.stderr, flush=True)

    print(f"# rendering {a.streams} streams", flush=True)
    streams = serve.make_streams(a.streams, a.frames_per_stream, a.seconds)
    est = api.Estimator(0)
    kw = dict(n_hstrips=32, n_vstrips=32, ransac_attempts=1024)
    line = {"metric": "serving latency, 48 mixed-resolution streams", "streams": a.streams,
            "seconds": a.seconds,
            "arrival_fps": float(sum(len(s.arrivals) for s in streams) / a.seconds)}
    runs = [("plain", dict(kw))]
    model = os.path.join(train_scorer.MODEL_DIR, train_scorer.MODEL_FILE)
    if os.path.exists(model):
        est.set_model(train_scorer.load_model(model))
        runs.append(("learned", dict(kw, scorer=1, fallback_inlier_frac=0.5)))
    for name, params in runs:
        cfg = serve.server_config(max_batch=a.max_batch, hbm_budget=int(a.budget_gib * (1 << 30)),
                                  **params)
        srv = serve.Server(est, cfg)
        serve.run(srv, streams, realtime=False, timeout_s=60, progress=log)   # warm-up
        srv.close()
        srv = serve.Server(est, cfg)
        print(f"# serving ({name})", flush=True)
        served, wall = serve.run(srv, streams, realtime=True, timeout_s=60, progress=log)
        stats = srv.stats()
        srv.close()
        rec = serve.latency_summary(served, wall)
        rec["batches"] = stats["batches"]
        rec["accuracy"] = accuracy(served, streams)
        line[name] = rec
    torch.cuda.synchronize()
    est.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
