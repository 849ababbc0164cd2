"""Serving loop binding (ca_server_*) and a simulated multi-stream workload.

The native server (csrc/ca_server.cpp) does admission, copies, continuous
batching and the per-stream temporal filter; this module marshals its calls
and drives it with simulated video streams: Poisson frame arrivals at 30-60
fps per stream, mixed resolutions, the circle drifting slowly per stream
(centre random walk, occasional zoom jumps).  Frames are device-rendered
ahead of time into a frame store in HBM that stands for the capture source.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import time

import numpy as np

from . import _native as N
from . import synth, synth_gpu


def server_config(max_streams=64, ring_slots=2, max_batch=256, max_inflight=2,
                  hbm_budget=4 << 30, smooth=0.8, **params) -> N.ServerConfig:
    from .api import default_params
    c = N.ServerConfig()
    c.max_streams, c.ring_slots, c.max_batch = max_streams, ring_slots, max_batch
    c.max_inflight, c.hbm_budget, c.smooth = max_inflight, hbm_budget, smooth
    c.params = default_params(**params)
    return c


class Server:
    """Thin wrapper over a native ca_server (one per estimator context)."""

    def __init__(self, est, cfg: N.ServerConfig):
        self._est = est
        self._s = C.c_void_p()
        N.check(N.lib().ca_server_create(est._ctx, C.byref(cfg), C.byref(self._s)),
                "ca_server_create")
        self._buf = (N.Served * 4096)()

    def close(self):
        if self._s:
            N.lib().ca_server_destroy(self._s)
            self._s = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def open(self, stream_id: int, width: int, height: int) -> bool:
        adm = C.c_int32()
        N.check(N.lib().ca_server_open(self._s, stream_id, width, height, C.byref(adm)),
                "ca_server_open")
        return bool(adm.value)

    def close_stream(self, stream_id: int) -> None:
        N.check(N.lib().ca_server_close(self._s, stream_id), "ca_server_close")

    def submit(self, stream_id: int, seq: int, frame, lend: bool = False) -> None:
        """`frame`: a device uint8 [H, W, 3] tensor (kept alive and unchanged
        by the caller until served).  With `lend` the server reads it in
        place instead of copying it into the stream's ring."""
        N.check(N.lib().ca_server_submit(self._s, stream_id, seq, C.c_void_p(frame.data_ptr()),
                                         frame.stride(0), 2 if lend else 1), "ca_server_submit")

    def step(self) -> list:
        n = C.c_int32()
        N.check(N.lib().ca_server_step(self._s, self._buf, len(self._buf), C.byref(n)),
                "ca_server_step")
        return [self._buf[i] for i in range(n.value)]

    def stats(self) -> dict:
        a = (C.c_int64 * 8)()
        N.check(N.lib().ca_server_stats(self._s, a), "ca_server_stats")
        keys = ("submitted", "served", "queued", "in_flight", "streams_admitted",
                "streams_waiting", "batches", "budget_used")
        return dict(zip(keys, list(a)))


def served_record(s) -> dict:
    r = s.result
    return {"stream": s.stream_id, "seq": int(s.seq),
            "result": (r.cx, r.cy, r.r, r.score, r.inliers, r.n_points, r.valid, r.reason),
            "filtered": (s.filtered_valid, s.fcx, s.fcy, s.fr, s.fweight),
            "latency_ms": (s.t_done_ns - s.t_submit_ns) * 1e-6,
            "queue_ms": (s.t_launch_ns - s.t_submit_ns) * 1e-6,
            "batch": s.batch_size}


# ------------------------------------------------------------ simulation --

SERVE_SHAPES = ((1280, 720), (1920, 1080), (3840, 2160))
SERVE_STREAM = 130          # seed stream of the serving frames


@dataclasses.dataclass
class SimStream:
    stream_id: int
    width: int
    height: int
    fps: float
    frames: list            # device tensors [H, W, 3], cycled
    specs: list
    arrivals: np.ndarray    # seconds from the start


def drifting_recipes(stream_id: int, width: int, height: int, n: int,
                     rng: np.random.Generator):
    """n frames of one stream: the circle's centre takes a random walk of
    0.5 px per frame, its radius jumps by +-10 % now and then (zoom)."""
    first = synth_gpu.draw_recipe(synth.HD_1080p, SERVE_STREAM, stream_id, False, width, height)
    base = first.spec
    recs = []
    cx, cy, r = base.cx, base.cy, base.r
    for k in range(n):
        # the same tissue, fresh pixel noise every frame
        key = tuple(int(v) for v in rng.integers(0, 2 ** 32, 2, dtype=np.uint64))
        if k:
            cx += float(rng.normal(0, 0.5))
            cy += float(rng.normal(0, 0.5))
            if rng.uniform() < 0.02:
                r *= 1.0 + float(rng.choice([-0.1, 0.1]))
        spec = dataclasses.replace(base, cx=cx, cy=cy, r=r)
        recs.append(synth_gpu.Recipe(spec, None, first.grids, key))
    return recs


def make_streams(n_streams: int = 48, frames_per_stream: int = 16, duration_s: float = 2.0,
                 seed: int = 0, shapes=SERVE_SHAPES):
    """Simulated streams with device-rendered frames and Poisson arrivals."""
    rng = np.random.default_rng(seed)
    out = []
    for sid in range(n_streams):
        w, h = shapes[sid % len(shapes)]
        fps = float(rng.uniform(30.0, 60.0))
        recs = drifting_recipes(sid, w, h, frames_per_stream, rng)
        frames = synth_gpu.DeviceRecipes(recs).render_frames()
        t, arr = 0.0, []
        while True:
            t += float(rng.exponential(1.0 / fps))
            if t >= duration_s:
                break
            arr.append(t)
        out.append(SimStream(sid, w, h, fps, [frames[i] for i in range(frames.shape[0])],
                             [r.spec for r in recs], np.array(arr)))
    return out


def run(server: Server, streams, realtime: bool = True, only=None, timeout_s: float = 120.0,
        progress=None, lend: bool = False):
    """Submit every stream's frames at their arrival times (or as fast as
    possible), step the server until all are served; returns the served
    records and the wall time.  Raises if the frames are not all served
    within timeout_s."""
    import torch
    torch.cuda.synchronize()
    events = []
    for st in streams:
        if only is not None and st.stream_id not in only:
            continue
        for k, t in enumerate(st.arrivals):
            events.append((float(t), st.stream_id, k))
    events.sort()
    by_id = {st.stream_id: st for st in streams}
    for sid in sorted({e[1] for e in events}):
        st = by_id[sid]
        server.open(sid, st.width, st.height)
    served = []
    t0 = time.perf_counter()
    i = 0
    next_report = 1.0
    while i < len(events) or len(served) < len(events):
        now = time.perf_counter() - t0
        if progress is not None and now >= next_report:
            progress(f"t={now:.1f}s submitted {i} served {len(served)} {server.stats()}")
            next_report += 1.0
        while i < len(events) and (not realtime or events[i][0] <= now):
            _, sid, k = events[i]
            st = by_id[sid]
            server.submit(sid, k, st.frames[k % len(st.frames)], lend)
            i += 1
        served += [served_record(s) for s in server.step()]
        if now > timeout_s:
            raise RuntimeError(f"serving stalled: {len(served)} of {len(events)} served, "
                               f"{server.stats()}")
    wall = time.perf_counter() - t0
    for sid in sorted({e[1] for e in events}):
        server.close_stream(sid)
    server.step()
    return served, wall


def latency_summary(served, wall: float) -> dict:
    lat = np.array([s["latency_ms"] for s in served])
    q = np.array([s["queue_ms"] for s in served])
    return {"frames": len(served), "wall_s": wall, "frames_per_s": len(served) / wall,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max()), "queue_p50_ms": float(np.percentile(q, 50)),
            "mean_batch": float(np.mean([s["batch"] for s in served]))}
