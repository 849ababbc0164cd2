"""Issue a fixed number of calls of one configuration, for profiler runs
(rocprofv3 --kernel-trace / --pmc): device-rendered synthetic frames, the
committed models for the learned scorers, nothing timed here.

    python -m paper_2210_14771_amd.prof_calls --scorer 2d --calls 10
"""
from __future__ import annotations

import argparse
import sys


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--scorer", choices=["plain", "1d", "2d"], action="append",
                    help="scorer(s) to call, in turn (default: all three)")
    ap.add_argument("--calls", type=int, default=5, help="calls per scorer")
    ap.add_argument("--frames", type=int, default=64)
    ap.add_argument("--size", default="1920x1080", help="WIDTHxHEIGHT")
    ap.add_argument("--strips", type=int, default=32, help="horizontal and vertical strips")
    ap.add_argument("--attempts", type=int, default=1024)
    a = ap.parse_args(argv)
    import torch
    from . import api, synth, synth_gpu, train_scorer
    W, H = (int(v) for v in a.size.split("x"))
    wl = synth.HD_1080p
    recs = [synth_gpu.draw_recipe(wl, 120, i, False, W, H) for i in range(a.frames)] \
        if (W, H) != (wl.width, wl.height) else None
    if recs is None:
        frames, _ = synth_gpu.render_set(wl, 120, a.frames, False)
    else:
        frames = synth_gpu.DeviceRecipes(recs).render_frames()
    est = api.Estimator(0)
    scorers = a.scorer or ["plain", "1d", "2d"]
    if "1d" in scorers:
        est.set_model(train_scorer.load_model())
    if "2d" in scorers:
        est.set_model_2d(train_scorer.load_model_2d())
    uids = list(range(a.frames))
    out = torch.empty((a.frames, 8), dtype=torch.int32, device="cuda")
    code = {"plain": 0, "1d": 1, "2d": 2}
    for sc in scorers:
        p = api.default_params(n_hstrips=a.strips, n_vstrips=a.strips,
                               ransac_attempts=a.attempts, scorer=code[sc])
        for _ in range(a.calls):
            est.estimate_area(frames, p, uids, out=out)
        torch.cuda.synchronize()
        print(f"{sc}: {a.calls} calls of {a.frames} x {W}x{H}", flush=True)
    est.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
