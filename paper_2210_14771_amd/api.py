"""Python binding of the content-area estimator (argument marshalling only).

PyTorch supplies device memory and the current HIP stream; every step of the
estimate runs in the library's gfx950 kernels behind the C ABI.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Sequence

import torch

from . import _native as N


def default_params(**overrides) -> N.Params:
    """Table A1 defaults (ca_default_params) with keyword overrides."""
    p = N.Params()
    N.lib().ca_default_params(C.byref(p))
    for k, v in overrides.items():
        if k == "attempts":
            k = "ransac_attempts"
        if not any(k == f for f, _ in N.Params._fields_):
            raise KeyError(f"unknown parameter {k!r}")
        setattr(p, k, v)
    return p


def _as_params(params) -> N.Params:
    if params is None:
        return default_params()
    if isinstance(params, N.Params):
        return params
    if isinstance(params, dict):
        return default_params(**params)
    raise TypeError("params must be None, a dict or a Params")


# one ca_result (32 bytes) as a numpy structured type
RESULT_DTYPE = [("cx", "<f4"), ("cy", "<f4"), ("r", "<f4"), ("score", "<f4"),
                ("inliers", "<i4"), ("n_points", "<i4"), ("valid", "<i4"), ("reason", "<i4")]


@dataclasses.dataclass
class Result:
    """Per-frame estimates (device tensors of length B)."""
    raw: torch.Tensor  # int32 [B, 8], one ca_result per row

    @property
    def cx(self) -> torch.Tensor:
        return self.raw[:, 0].view(torch.float32)

    @property
    def cy(self) -> torch.Tensor:
        return self.raw[:, 1].view(torch.float32)

    @property
    def r(self) -> torch.Tensor:
        return self.raw[:, 2].view(torch.float32)

    @property
    def score(self) -> torch.Tensor:
        return self.raw[:, 3].view(torch.float32)

    @property
    def inliers(self) -> torch.Tensor:
        return self.raw[:, 4]

    @property
    def n_points(self) -> torch.Tensor:
        return self.raw[:, 5]

    @property
    def valid(self) -> torch.Tensor:
        return self.raw[:, 6] != 0

    @property
    def reason(self) -> torch.Tensor:
        return self.raw[:, 7]

    def numpy(self):
        return self.raw.cpu().numpy().view(RESULT_DTYPE).reshape(-1)


_layout_cache: dict = {}


def _batch_layout(frames: torch.Tensor, frame_uids):
    """Descriptors of a [B, H, W, 3] tensor computed from its strides (cached)."""
    if frames.dtype != torch.uint8:
        raise ValueError("frames must be uint8 [B, H, W, 3]")
    if frames.device.type != "cuda":
        raise ValueError("frames must be on a GPU")
    if frames.stride(2) != 3 or frames.stride(3) != 1:
        raise ValueError("pixels must be packed RGB (stride 3 along W, 1 along channels)")
    B, H, W, _ = frames.shape
    uids = tuple(range(B)) if frame_uids is None else tuple(int(u) for u in frame_uids)
    if len(uids) != B:
        raise ValueError("frame_uids must have one entry per frame")
    key = (tuple(frames.shape), tuple(frames.stride()), uids)
    descs = _layout_cache.get(key)
    if descs is None:
        descs = (N.FrameDesc * B)()
        for i in range(B):
            d = descs[i]
            d.width, d.height = W, H
            d.row_stride = frames.stride(1)
            d.pixel_stride = 3
            d.byte_offset = i * frames.stride(0)
            d.frame_uid = uids[i] & 0xFFFFFFFFFFFFFFFF
        if len(_layout_cache) > 64:
            _layout_cache.clear()
        _layout_cache[key] = descs
    return frames.data_ptr(), descs, B, frames.device


def _frames_layout(frames, frame_uids):
    """(base pointer, FrameDesc array, n, device) for a [B,H,W,3] tensor or a
    list of [H,W,3] tensors (mixed resolutions) on one device."""
    if isinstance(frames, torch.Tensor):
        if frames.dim() == 3:
            frames = frames.unsqueeze(0)
        if frames.dim() != 4 or frames.shape[-1] != 3:
            raise ValueError("frames must be uint8 [B, H, W, 3]")
        if frames.stride(0) >= 0 and frames.shape[0] > 0:
            return _batch_layout(frames, frame_uids)
        items = [frames[i] for i in range(frames.shape[0])]
        dev = frames.device
    else:
        items = list(frames)
        if not items:
            raise ValueError("empty frame list")
        dev = items[0].device
    for t in items:
        if t.dtype != torch.uint8 or t.dim() != 3 or t.shape[-1] != 3:
            raise ValueError("each frame must be uint8 [H, W, 3]")
        if t.device != dev or dev.type != "cuda":
            raise ValueError("frames must all be on one GPU")
        if t.stride(2) != 1 or t.stride(1) != 3:
            raise ValueError("pixels must be packed RGB (stride 3 along W, 1 along channels)")
    n = len(items)
    if frame_uids is None:
        uids = list(range(n))
    else:
        uids = [int(u) for u in frame_uids]
        if len(uids) != n:
            raise ValueError("frame_uids must have one entry per frame")
    base = min(t.data_ptr() for t in items)
    descs = (N.FrameDesc * n)()
    for i, t in enumerate(items):
        d = descs[i]
        d.width, d.height = t.shape[1], t.shape[0]
        d.row_stride = t.stride(0)
        d.pixel_stride = 3
        d.byte_offset = t.data_ptr() - base
        d.frame_uid = uids[i] & 0xFFFFFFFFFFFFFFFF
    return base, descs, n, dev


class Estimator:
    """One library context on one GPU (not thread-safe: one per host thread)."""

    def __init__(self, device=None, workspace_budget: int = 1 << 30):
        if not torch.cuda.is_available():
            raise RuntimeError("the content-area estimator needs a HIP GPU")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        ctx = C.c_void_p()
        N.check(N.lib().ca_create(C.byref(ctx), self.device.index, workspace_budget),
                "ca_create")
        self._ctx = ctx

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            N.lib().ca_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    OPTIONS = {"schedule": N.CA_OPT_SCHEDULE, "lag": N.CA_OPT_LAG, "queues": N.CA_OPT_QUEUES,
               "grid": N.CA_OPT_GRID, "spin_limit": N.CA_OPT_SPIN_LIMIT,
               "pipeline": N.CA_OPT_PIPELINE, "strips_per_group": N.CA_OPT_STRIPS_PER_GROUP,
               "ransac_lanes": N.CA_OPT_RANSAC_LANES}

    def set_option(self, name: str, value: int) -> None:
        """Options: schedule ("split"/"fused"/"auto" or 0/1/2), pipeline (sub-batches of a split
        call), lag, queues, grid, spin_limit (fused schedule)."""
        if name == "schedule" and isinstance(value, str):
            value = {"fused": N.CA_SCHEDULE_FUSED, "split": N.CA_SCHEDULE_SPLIT,
                     "auto": N.CA_SCHEDULE_AUTO}[value]
        N.check(N.lib().ca_set_option(self._ctx, self.OPTIONS[name], int(value)), "ca_set_option")

    def get_option(self, name: str) -> int:
        v = C.c_int64()
        N.check(N.lib().ca_get_option(self._ctx, self.OPTIONS[name], C.byref(v)), "ca_get_option")
        return v.value

    def device_status(self) -> None:
        """Raise if a fused call's wait gave up at its spin limit (synchronises)."""
        N.check(N.lib().ca_device_status(self._ctx), "ca_device_status")

    def set_model(self, params) -> None:
        """Load the learned scorer (CA_CNN_PARAMS float32 values, model-file order)."""
        import numpy as np
        a = np.ascontiguousarray(params, dtype=np.float32).ravel()
        N.check(N.lib().ca_set_model(self._ctx, a.ctypes.data_as(C.POINTER(C.c_float)), a.size),
                "ca_set_model")

    def cnn_window_logits(self, windows: torch.Tensor, ranges: torch.Tensor,
                          stream=None) -> torch.Tensor:
        """Logits [n, 112] of uint8 windows [n, 8, 128, 3] with int32 ranges [n, 2]."""
        if windows.dtype != torch.uint8 or tuple(windows.shape[1:]) != (8, N.CA_CNN_WINDOW, 3):
            raise ValueError("windows must be uint8 [n, 8, 128, 3]")
        windows = windows.contiguous()
        ranges = ranges.to(torch.int32).contiguous()
        n = windows.shape[0]
        z = torch.empty((n, N.CA_CNN_OUTPUTS), dtype=torch.float32, device=self.device)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        N.check(N.lib().ca_cnn_window_logits(self._ctx, C.c_void_p(windows.data_ptr()),
                                             C.c_void_p(ranges.data_ptr()), n,
                                             C.c_void_p(z.data_ptr()), C.c_void_p(s.cuda_stream)),
                "ca_cnn_window_logits")
        return z

    def get_model(self, with_momentum: bool = False):
        """Master weights (and the SGD momentum) as float32 numpy arrays."""
        import numpy as np
        prm = np.empty(N.CA_CNN_PARAMS, dtype=np.float32)
        mom = np.empty(N.CA_CNN_PARAMS, dtype=np.float32) if with_momentum else None
        fp = C.POINTER(C.c_float)
        N.check(N.lib().ca_get_model(self._ctx, prm.ctypes.data_as(fp),
                                     mom.ctypes.data_as(fp) if mom is not None else None,
                                     prm.size), "ca_get_model")
        return (prm, mom) if with_momentum else prm

    def set_momentum(self, momentum) -> None:
        import numpy as np
        a = np.ascontiguousarray(momentum, dtype=np.float32).ravel()
        N.check(N.lib().ca_set_momentum(self._ctx, a.ctypes.data_as(C.POINTER(C.c_float)), a.size),
                "ca_set_momentum")

    def cnn_gradients(self, windows: torch.Tensor, ranges: torch.Tensor, targets: torch.Tensor,
                      weights: torch.Tensor, scale: float, stream=None):
        """(grad [CA_CNN_PARAMS], loss [1]) device tensors of the weighted soft BCE."""
        if windows.dtype != torch.uint8 or tuple(windows.shape[1:]) != (8, N.CA_CNN_WINDOW, 3):
            raise ValueError("windows must be uint8 [n, 8, 128, 3]")
        n = windows.shape[0]
        for t, name in ((targets, "targets"), (weights, "weights")):
            if t.dtype != torch.float32 or tuple(t.shape) != (n, N.CA_CNN_OUTPUTS):
                raise ValueError(f"{name} must be float32 [n, {N.CA_CNN_OUTPUTS}]")
        if tuple(ranges.shape) != (n, 2):
            raise ValueError("ranges must be [n, 2]")
        windows = windows.contiguous()
        ranges = ranges.to(torch.int32).contiguous()
        targets = targets.contiguous()
        weights = weights.contiguous()
        grad = torch.empty(N.CA_CNN_PARAMS, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        vp = C.c_void_p
        N.check(N.lib().ca_cnn_gradients(self._ctx, vp(windows.data_ptr()), vp(ranges.data_ptr()),
                                         vp(targets.data_ptr()), vp(weights.data_ptr()), n,
                                         float(scale), vp(grad.data_ptr()), vp(loss.data_ptr()),
                                         vp(s.cuda_stream)), "ca_cnn_gradients")
        return grad, loss

    def cnn_sgd_step(self, grad: torch.Tensor, lr: float, momentum: float, stream=None) -> None:
        """m = momentum m + grad; p -= lr m on the master weights; rebuild the model."""
        if grad.dtype != torch.float32 or grad.numel() != N.CA_CNN_PARAMS or not grad.is_contiguous():
            raise ValueError("grad must be a contiguous float32 tensor of CA_CNN_PARAMS values")
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        N.check(N.lib().ca_cnn_sgd_step(self._ctx, C.c_void_p(grad.data_ptr()), float(lr),
                                        float(momentum), C.c_void_p(s.cuda_stream)),
                "ca_cnn_sgd_step")

    # the paper's own 2-D scorer (CA_SCORER_LEARNED_2D)

    def set_model_2d(self, params) -> None:
        """Load the 2-D scorer (CA_CNN2D_PARAMS float32 values, model-file order)."""
        import numpy as np
        a = np.ascontiguousarray(params, dtype=np.float32).ravel()
        N.check(N.lib().ca_set_model_2d(self._ctx, a.ctypes.data_as(C.POINTER(C.c_float)),
                                        a.size), "ca_set_model_2d")

    def get_model_2d(self, with_momentum: bool = False):
        import numpy as np
        prm = np.empty(N.CA_CNN2D_PARAMS, dtype=np.float32)
        mom = np.empty(N.CA_CNN2D_PARAMS, dtype=np.float32) if with_momentum else None
        fp = C.POINTER(C.c_float)
        N.check(N.lib().ca_get_model_2d(self._ctx, prm.ctypes.data_as(fp),
                                        mom.ctypes.data_as(fp) if mom is not None else None,
                                        prm.size), "ca_get_model_2d")
        return (prm, mom) if with_momentum else prm

    def set_momentum_2d(self, momentum) -> None:
        import numpy as np
        a = np.ascontiguousarray(momentum, dtype=np.float32).ravel()
        N.check(N.lib().ca_set_momentum_2d(self._ctx, a.ctypes.data_as(C.POINTER(C.c_float)),
                                           a.size), "ca_set_momentum_2d")

    @staticmethod
    def _windows_2d(windows, geom, ranges):
        if windows.dtype != torch.uint8 or tuple(windows.shape[1:]) != (8, N.CA_CNN_WINDOW, 3):
            raise ValueError("windows must be uint8 [n, 8, 128, 3]")
        n = windows.shape[0]
        if tuple(geom.shape) != (n, 8) or tuple(ranges.shape) != (n, 2):
            raise ValueError("geom must be [n, 8] and ranges [n, 2]")
        return (windows.contiguous(), geom.to(torch.int32).contiguous(),
                ranges.to(torch.int32).contiguous(), n)

    def cnn2d_window_logits(self, windows: torch.Tensor, geom: torch.Tensor, ranges: torch.Tensor,
                            stream=None) -> torch.Tensor:
        """Logits [n, 112] of the 2-D scorer on uint8 windows [n, 8, 128, 3]
        with int32 geometry [n, 8] and ranges [n, 2]."""
        windows, geom, ranges, n = self._windows_2d(windows, geom, ranges)
        z = torch.empty((n, N.CA_CNN_OUTPUTS), dtype=torch.float32, device=self.device)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        vp = C.c_void_p
        N.check(N.lib().ca_cnn2d_window_logits(self._ctx, vp(windows.data_ptr()),
                                               vp(geom.data_ptr()), vp(ranges.data_ptr()), n,
                                               vp(z.data_ptr()), vp(s.cuda_stream)),
                "ca_cnn2d_window_logits")
        return z

    def cnn2d_gradients(self, windows: torch.Tensor, geom: torch.Tensor, ranges: torch.Tensor,
                        targets: torch.Tensor, weights: torch.Tensor, scale: float, stream=None):
        """(grad [CA_CNN2D_PARAMS], loss [1]) device tensors of the weighted soft BCE."""
        windows, geom, ranges, n = self._windows_2d(windows, geom, ranges)
        for t, name in ((targets, "targets"), (weights, "weights")):
            if t.dtype != torch.float32 or tuple(t.shape) != (n, N.CA_CNN_OUTPUTS):
                raise ValueError(f"{name} must be float32 [n, {N.CA_CNN_OUTPUTS}]")
        targets = targets.contiguous()
        weights = weights.contiguous()
        grad = torch.empty(N.CA_CNN2D_PARAMS, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        vp = C.c_void_p
        N.check(N.lib().ca_cnn2d_gradients(self._ctx, vp(windows.data_ptr()), vp(geom.data_ptr()),
                                           vp(ranges.data_ptr()), vp(targets.data_ptr()),
                                           vp(weights.data_ptr()), n, float(scale),
                                           vp(grad.data_ptr()), vp(loss.data_ptr()),
                                           vp(s.cuda_stream)), "ca_cnn2d_gradients")
        return grad, loss

    def cnn2d_sgd_step(self, grad: torch.Tensor, lr: float, momentum: float, stream=None) -> None:
        if grad.dtype != torch.float32 or grad.numel() != N.CA_CNN2D_PARAMS or not grad.is_contiguous():
            raise ValueError("grad must be a contiguous float32 tensor of CA_CNN2D_PARAMS values")
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        N.check(N.lib().ca_cnn2d_sgd_step(self._ctx, C.c_void_p(grad.data_ptr()), float(lr),
                                          float(momentum), C.c_void_p(s.cuda_stream)),
                "ca_cnn2d_sgd_step")

    def selftest_mfma(self) -> torch.Tensor:
        out = torch.empty((16, 16), dtype=torch.float32, device=self.device)
        s = torch.cuda.current_stream(self.device)
        N.check(N.lib().ca_selftest_mfma(self._ctx, C.c_void_p(out.data_ptr()),
                                         C.c_void_p(s.cuda_stream)), "ca_selftest_mfma")
        return out

    def profile_begin(self, max_calls: int) -> None:
        """Time each kernel of the next ``max_calls`` calls with HIP events."""
        N.check(N.lib().ca_profile_begin(self._ctx, max_calls), "ca_profile_begin")

    def profile_end(self) -> dict:
        """Average kernel durations (ms) of the calls timed since profile_begin."""
        t = N.KernelTimes()
        N.check(N.lib().ca_profile_end(self._ctx, C.byref(t)), "ca_profile_end")
        names = ("strips", "ransac", "gap")
        return {n: {"total_ms": t.total_ms[i], "launches": int(t.launches[i]),
                    "avg_ms": t.total_ms[i] / t.launches[i] if t.launches[i] else 0.0}
                for i, n in enumerate(names)}

    def _prep(self, frames, params, frame_uids, stream):
        base, descs, n, dev = _frames_layout(frames, frame_uids)
        if dev.index != self.device.index:
            raise ValueError(f"frames on {dev}, estimator on {self.device}")
        p = _as_params(params)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return base, descs, n, p, s

    def estimate_area(self, frames, params=None, frame_uids: Sequence[int] | None = None,
                      out: torch.Tensor | None = None, stream=None) -> Result:
        """Content area of each frame (Section 2.2); enqueued on the current stream."""
        base, descs, n, p, s = self._prep(frames, params, frame_uids, stream)
        if out is None:
            out = torch.empty((n, 8), dtype=torch.int32, device=self.device)
        rc = N.lib().ca_estimate_area(self._ctx, C.c_void_p(base), descs, n, C.byref(p),
                                      C.c_void_p(out.data_ptr()), C.c_void_p(s.cuda_stream))
        N.check(rc, "ca_estimate_area")
        return Result(out)

    def estimate_area_noalloc(self, frames, params=None, frame_uids: Sequence[int] | None = None,
                              out: torch.Tensor | None = None, stream=None) -> Result:
        """estimate_area over the library's fixed device scratch instead of
        allocated buffers (ca_estimate_area_noalloc); `out` is allocated here
        only when not given."""
        base, descs, n, p, s = self._prep(frames, params, frame_uids, stream)
        if out is None:
            out = torch.empty((n, 8), dtype=torch.int32, device=self.device)
        rc = N.lib().ca_estimate_area_noalloc(self._ctx, C.c_void_p(base), descs, n, C.byref(p),
                                              C.c_void_p(out.data_ptr()),
                                              C.c_void_p(s.cuda_stream))
        N.check(rc, "ca_estimate_area_noalloc")
        return Result(out)

    def autotune(self, frames, params=None, frame_uids=None, reps: int = 5) -> dict:
        """Tune the strip tile (strip items per workgroup) of every frame shape
        in the batch, then the batch's schedule (split in 1, 2 or 4 pipelined
        sub-batches, or persistent: last_tuned_schedule, last_tuned_pipeline);
        returns {(width, height): T}."""
        base, descs, n, p, s = self._prep(frames, params, frame_uids, None)
        sched = C.c_int32(-1)
        N.check(N.lib().ca_autotune(self._ctx, C.c_void_p(base), descs, n, C.byref(p), reps,
                                    C.c_void_p(s.cuda_stream), C.byref(sched)), "ca_autotune")
        out = {}
        for i in range(n):
            key = (descs[i].width, descs[i].height)
            if key not in out:
                out[key] = self.get_tuning(key[0], key[1], p.n_hstrips, p.n_vstrips)
        self.last_tuned_schedule = {0: "split", 1: "fused"}.get(sched.value)
        s2, pipe = C.c_int32(), C.c_int32()
        N.check(N.lib().ca_get_last_autotune(self._ctx, C.byref(s2), C.byref(pipe)),
                "ca_get_last_autotune")
        self.last_tuned_pipeline = int(pipe.value) if self.last_tuned_schedule == "split" else None
        return out

    def get_tuning(self, width: int, height: int, n_hstrips: int, n_vstrips: int) -> int:
        v = C.c_int32()
        N.check(N.lib().ca_get_tuning(self._ctx, width, height, n_hstrips, n_vstrips, C.byref(v)),
                "ca_get_tuning")
        return int(v.value)

    def capture(self, frames, params=None, frame_uids=None, out: torch.Tensor | None = None,
                calls: int = 1) -> "Graph":
        """A HIP graph replaying ``calls`` estimate calls on these buffers."""
        base, descs, n, p, _ = self._prep(frames, params, frame_uids, None)
        if out is None:
            out = torch.empty((n, 8), dtype=torch.int32, device=self.device)
        g = C.c_void_p()
        rc = N.lib().ca_graph_create(self._ctx, C.c_void_p(base), descs, n, C.byref(p),
                                     C.c_void_p(out.data_ptr()), calls, C.byref(g))
        N.check(rc, "ca_graph_create")
        return Graph(self, g, Result(out), frames)

    def debug_candidates(self, frames, params=None, frame_uids=None, stream=None):
        """(Result, points int16/float32 packed as int32 [B, P, 2])."""
        base, descs, n, p, s = self._prep(frames, params, frame_uids, stream)
        P = 2 * (p.n_hstrips + p.n_vstrips)
        out = torch.empty((n, 8), dtype=torch.int32, device=self.device)
        pts = torch.empty((n, P, 2), dtype=torch.int32, device=self.device)
        rc = N.lib().ca_debug_candidates(self._ctx, C.c_void_p(base), descs, n, C.byref(p),
                                         C.c_void_p(pts.data_ptr()), C.c_void_p(out.data_ptr()),
                                         C.c_void_p(s.cuda_stream))
        N.check(rc, "ca_debug_candidates")
        return Result(out), pts

    def debug_attempts(self, frames, params=None, frame_uids=None, stream=None):
        """(Result, attempts as raw bytes uint8 [B, A, 56])."""
        base, descs, n, p, s = self._prep(frames, params, frame_uids, stream)
        A = p.ransac_attempts
        out = torch.empty((n, 8), dtype=torch.int32, device=self.device)
        att = torch.empty((n, A, 56), dtype=torch.uint8, device=self.device)
        rc = N.lib().ca_debug_attempts(self._ctx, C.c_void_p(base), descs, n, C.byref(p),
                                       C.c_void_p(att.data_ptr()), C.c_void_p(out.data_ptr()),
                                       C.c_void_p(s.cuda_stream))
        N.check(rc, "ca_debug_attempts")
        return Result(out), att


class Graph:
    """Captured estimate calls (ca_graph); keeps its buffers alive."""

    def __init__(self, est: Estimator, handle, result: Result, frames):
        self._est, self._g, self.result, self._frames = est, handle, result, frames

    def launch(self, stream=None) -> Result:
        s = stream if stream is not None else torch.cuda.current_stream(self._est.device)
        N.check(N.lib().ca_graph_launch(self._g, C.c_void_p(s.cuda_stream)), "ca_graph_launch")
        return self.result

    def close(self):
        if self._g is not None and self._g.value:
            N.lib().ca_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


POINT_FIELDS = [("x", "<i2"), ("y", "<i2"), ("score", "<f4")]
ATTEMPT_FIELDS = [("status", "<i4"), ("fail_stage", "<i4"), ("i0", "<i4"), ("i1", "<i4"),
                  ("i2", "<i4"), ("inliers", "<i4"), ("qsum", "<u8"), ("cx", "<f8"),
                  ("cy", "<f8"), ("r2", "<f8")]


def points_numpy(pts: torch.Tensor):
    """Structured numpy view (x, y, score) of debug_candidates' points."""
    import numpy as np
    a = pts.cpu().contiguous().numpy()
    return a.view(np.dtype(POINT_FIELDS)).reshape(a.shape[0], a.shape[1])


def attempts_numpy(att: torch.Tensor):
    import numpy as np
    a = att.cpu().contiguous().numpy()
    return a.view(np.dtype(ATTEMPT_FIELDS)).reshape(a.shape[0], a.shape[1])


_default: dict[int, Estimator] = {}


def estimate_area(frames, params=None, frame_uids=None) -> Result:
    """Module-level convenience: one cached Estimator per device."""
    dev = frames.device.index if isinstance(frames, torch.Tensor) else frames[0].device.index
    est = _default.get(dev)
    if est is None:
        est = _default[dev] = Estimator(dev)
    return est.estimate_area(frames, params, frame_uids)


def strip_positions(extent: int, n: int, alpha: float = 8.0):
    import numpy as np
    out = np.zeros(max(n, 1), dtype=np.int32)
    N.check(N.lib().ca_strip_positions(extent, n, alpha,
                                       out.ctypes.data_as(C.POINTER(C.c_int32))),
            "ca_strip_positions")
    return out[:n]


def score_tables(params=None):
    """(SG[:sg_len], ST, SI) float32 tables exactly as the kernels use them."""
    import numpy as np
    p = _as_params(params)
    sg = np.zeros(N.CA_SG_CAPACITY, dtype=np.float32)
    st = np.zeros(2049, dtype=np.float32)
    si = np.zeros(256, dtype=np.float32)
    n = C.c_int32()
    f = lambda a: a.ctypes.data_as(C.POINTER(C.c_float))  # noqa: E731
    N.check(N.lib().ca_score_tables(C.byref(p), f(sg), C.byref(n), f(st), f(si)),
            "ca_score_tables")
    return sg[:n.value], st, si
