"""Device rendering of synthetic frames and training windows (libcasynth.so).

An input generator, like ``synth``: the host draws every frame's ground
truth, control grids and distractors with ``synth``'s seeded generators;
the device renders the pixels.  Used for the learned scorer's training set
(far too many frames for the CPU renderer) and for hard evaluation frames.
Frames drawn here are never fed to the oracle.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

from . import synth

_LIB = None

FRAME_DTYPE = np.dtype([
    ("width", "<i4"), ("height", "<i4"), ("kind", "<i4"), ("n_blobs", "<i4"),
    ("cx", "<f4"), ("cy", "<f4"), ("r", "<f4"), ("blur", "<f4"),
    ("border_sigma", "<f4"), ("vignette", "<f4"), ("mean_luma", "<f4"), ("edge_step", "<f4"),
    ("tint", "<f4", (3,)), ("grid_off", "<i4"),
    ("gh0", "<i4"), ("gw0", "<i4"), ("gh1", "<i4"), ("gw1", "<i4"),
    ("key0", "<u4"), ("key1", "<u4"), ("glyph_off", "<i4"), ("text_scale", "<i4"),
    ("text_x", "<f4"), ("text_y", "<f4"), ("text_lines", "<i4"), ("text_chars", "<i4"),
    ("blob", "<f4", (4, 4)), ("out_offset", "<i8"), ("flags", "<i4"), ("pad", "<i4"),
])
NO_NOISE = 1
assert FRAME_DTYPE.itemsize == 192

# seed streams of the device-rendered sets (disjoint from the CPU workloads)
TRAIN_PLAIN = 100
TRAIN_HARD = 101
VALID_PLAIN = 110
VALID_HARD = 111


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libcasynth.so")
        if not os.path.exists(path):
            raise RuntimeError("libcasynth.so is not built (run paper_2210_14771_amd/build.py)")
        L = C.CDLL(path)
        vp, i32 = C.c_void_p, C.c_int32
        L.synth_render_frames.argtypes = [vp, i32, i32, vp, vp, vp, vp]
        L.synth_render_windows.argtypes = [vp, vp, i32, vp, vp, C.c_float, vp, vp, vp, vp, vp]
        _LIB = L
    return _LIB


@dataclasses.dataclass
class Recipe:
    spec: synth.FrameSpec
    extras: synth.HardExtras | None
    grids: tuple          # base, fine, chroma list, tint
    key: tuple[int, int]


def draw_recipe(wl: synth.Workload, stream_id: int, idx: int, hard: bool,
                width: int | None = None, height: int | None = None) -> Recipe:
    """Frame ``idx`` of seed stream ``stream_id``: ground truth, distractors
    (hard frames), control grids and noise key."""
    rng = synth.frame_rng(stream_id, idx)
    w = wl.width if width is None else width
    h = wl.height if height is None else height
    spec = synth.draw_spec(rng, w, h, wl.mix, wl.border_sigma, wl.blur_sigma, wl.vignette,
                           wl.radius_frac)
    extras = synth.draw_hard(rng, spec) if hard else None
    grids = synth.smooth_grids(rng, spec)
    key = tuple(int(k) for k in rng.integers(0, 2 ** 32, 2, dtype=np.uint64))
    return Recipe(spec, extras, grids, key)


def pack(recipes: list[Recipe], frame_bytes_offsets=None):
    """Recipe records, concatenated control grids and glyphs (host arrays)."""
    n = len(recipes)
    rec = np.zeros(n, dtype=FRAME_DTYPE)
    grids, glyphs = [], []
    g_at, y_at, o_at = 0, 0, 0
    for i, rc in enumerate(recipes):
        s, ex = rc.spec, rc.extras
        base, fine, chroma, tint = rc.grids
        r = rec[i]
        r["width"], r["height"], r["kind"] = s.width, s.height, s.kind
        r["cx"], r["cy"], r["r"], r["blur"] = s.cx, s.cy, s.r, s.blur_sigma
        r["border_sigma"], r["vignette"], r["mean_luma"] = s.border_sigma, s.vignette, s.mean_luma
        r["tint"] = tint
        r["grid_off"] = g_at
        r["gh0"], r["gw0"] = base.shape
        r["gh1"], r["gw1"] = fine.shape
        for c in chroma:
            assert c.shape == base.shape
        block = np.concatenate([base.ravel(), fine.ravel()] + [c.ravel() for c in chroma])
        grids.append(block)
        g_at += block.size
        r["key0"], r["key1"] = rc.key
        if ex is not None:
            r["edge_step"] = ex.edge_step
            assert len(ex.blobs) <= 4
            r["n_blobs"] = len(ex.blobs)
            for j, b in enumerate(ex.blobs):
                r["blob"][j] = b
            if ex.text_scale > 0:
                assert ex.glyphs.size == ex.text_lines * ex.text_chars
                r["text_scale"], r["text_x"], r["text_y"] = ex.text_scale, ex.text_x, ex.text_y
                r["text_lines"], r["text_chars"] = ex.text_lines, ex.text_chars
                r["glyph_off"] = y_at
                glyphs.append(ex.glyphs.astype(np.uint64))
                y_at += ex.glyphs.size
        if frame_bytes_offsets is None:
            r["out_offset"] = o_at
            o_at += 3 * s.width * s.height
        else:
            r["out_offset"] = frame_bytes_offsets[i]
    g = np.concatenate(grids).astype(np.float32) if grids else np.zeros(1, np.float32)
    y = np.concatenate(glyphs) if glyphs else np.zeros(1, np.uint64)
    return rec, g, y, o_at


class DeviceRecipes:
    """Recipes uploaded to the device."""

    def __init__(self, recipes: list[Recipe], device="cuda", flags: int = 0):
        import torch
        rec, g, y, total = pack(recipes)
        rec["flags"] = flags
        self.recipes = recipes
        self.n = len(recipes)
        self.total_bytes = total
        self.rec = torch.from_numpy(rec.view(np.uint8).copy()).to(device)
        self.grids = torch.from_numpy(g).to(device)
        self.glyphs = torch.from_numpy(y.view(np.int64)).to(device)
        self.device = device

    def render_frames(self, stream=None):
        """uint8 device tensor: [n, H, W, 3] when all frames share a size,
        else a flat buffer with the frames at their out_offset."""
        import torch
        specs = [r.spec for r in self.recipes]
        out = torch.empty(self.total_bytes, dtype=torch.uint8, device=self.device)
        maxp = max(s.width * s.height for s in specs)
        st = stream if stream is not None else torch.cuda.current_stream()
        rc = lib().synth_render_frames(C.c_void_p(self.rec.data_ptr()), self.n, maxp,
                                       C.c_void_p(self.grids.data_ptr()),
                                       C.c_void_p(self.glyphs.data_ptr()),
                                       C.c_void_p(out.data_ptr()), C.c_void_p(st.cuda_stream))
        if rc != 0:
            raise RuntimeError(f"synth_render_frames failed ({rc})")
        if len({(s.width, s.height) for s in specs}) == 1:
            return out.view(self.n, specs[0].height, specs[0].width, 3)
        return out

    def render_windows(self, desc: np.ndarray, edge_boost: float = 0.0, stream=None):
        """(windows, ranges, targets, weights) device tensors for int32 desc [n, 4]."""
        import torch
        desc = np.ascontiguousarray(desc, dtype=np.int32)
        n = desc.shape[0]
        assert desc.ndim == 2 and desc.shape[1] == 4
        if n:
            assert desc[:, 0].min() >= 0 and desc[:, 0].max() < self.n
            for f in np.unique(desc[:, 0]):
                s = self.recipes[f].spec
                sel = desc[:, 0] == f
                ext = np.where(desc[sel, 1] != 0, s.height, s.width)
                assert np.all((desc[sel, 2] >= 0) & (desc[sel, 2] < ext))
        d = torch.from_numpy(desc).to(self.device)
        win = torch.empty((n, 8, 128, 3), dtype=torch.uint8, device=self.device)
        rng_ = torch.empty((n, 2), dtype=torch.int32, device=self.device)
        tgt = torch.empty((n, 112), dtype=torch.float32, device=self.device)
        wt = torch.empty((n, 112), dtype=torch.float32, device=self.device)
        st = stream if stream is not None else torch.cuda.current_stream()
        rc = lib().synth_render_windows(C.c_void_p(self.rec.data_ptr()), C.c_void_p(d.data_ptr()),
                                        n, C.c_void_p(self.grids.data_ptr()),
                                        C.c_void_p(self.glyphs.data_ptr()), float(edge_boost),
                                        C.c_void_p(win.data_ptr()), C.c_void_p(rng_.data_ptr()),
                                        C.c_void_p(tgt.data_ptr()), C.c_void_p(wt.data_ptr()),
                                        C.c_void_p(st.cuda_stream))
        if rc != 0:
            raise RuntimeError(f"synth_render_windows failed ({rc})")
        return win, rng_, tgt, wt


def strip_windows(frame: int, horizontal: bool, line: int, length: int) -> np.ndarray:
    """Descriptors of the windows that tile one whole strip (112 new
    positions each, 8 halo positions on both sides)."""
    starts = np.arange(0, length, 112) - 8
    return np.stack([np.full_like(starts, frame), np.full_like(starts, int(horizontal)),
                     np.full_like(starts, line), starts], axis=1).astype(np.int32)


def render_set(wl: synth.Workload, stream_id: int, n: int, hard: bool, first: int = 0,
               device="cuda"):
    """Render frames first .. first+n-1 of a seed stream on the device:
    (uint8 [n, H, W, 3] device tensor, their FrameSpecs)."""
    recs = [draw_recipe(wl, stream_id, i, hard) for i in range(first, first + n)]
    return DeviceRecipes(recs, device).render_frames(), [r.spec for r in recs]

