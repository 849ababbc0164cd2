"""Seeded synthetic endoscopic frames with a known content-area circle.

Input generator only: this module draws pixels and ground truth and holds
none of the estimator's arithmetic, so both the HIP path and the CPU oracle
can be fed from it.  It stands in for the paper's annotated datasets
(Section 2.1, Table 1), which are not available here.

Image model (Section 1.1, Figure 1): a circular projection of the scope's
field of view intersected with the sensor rectangle.  Inside the disc is a
smooth tissue-like colour field; outside is a dark grey border with Gaussian
noise.  The transition is an analytically Gaussian-blurred step, so the 50 %
level sits exactly on the ground-truth radius.  Coordinates are pixel-index
coordinates: pixel (x, y) has its centre at integer (x, y).

Every frame is generated from its own ``numpy.random.SeedSequence`` built
from ``(2210_14771, config_id, frame_idx)``, so any frame can be reproduced
alone, independent of batch composition.
"""
from __future__ import annotations

import dataclasses
import numpy as np
from scipy.special import ndtr

ROOT_SEED = 2210_14771

KIND_PARTIAL = 0   # circle clipped by the sensor, at least one corner outside
KIND_FULL = 1      # whole circle inside the sensor rectangle
KIND_NOBORDER = 2  # no border at all: content fills the rectangle
KIND_NAMES = {KIND_PARTIAL: "partial", KIND_FULL: "full", KIND_NOBORDER: "noborder"}


@dataclasses.dataclass
class FrameSpec:
    """Drawn parameters of one synthetic frame (the ground truth)."""
    width: int
    height: int
    kind: int
    cx: float
    cy: float
    r: float
    border_sigma: float
    blur_sigma: float
    vignette: float
    mean_luma: float

    @property
    def has_border(self) -> bool:
        return self.kind != KIND_NOBORDER


def _interp_matrix(n_out: int, n_in: int) -> np.ndarray:
    """Linear interpolation weights mapping n_in control values onto n_out samples."""
    pos = np.linspace(0.0, n_in - 1.0, n_out)
    i0 = np.clip(np.floor(pos).astype(np.int64), 0, n_in - 2)
    f = pos - i0
    m = np.zeros((n_out, n_in), dtype=np.float32)
    m[np.arange(n_out), i0] = 1.0 - f
    m[np.arange(n_out), i0 + 1] = f
    return m


def _smooth_field(rng: np.random.Generator, h: int, w: int, cell: float) -> np.ndarray:
    """Zero-mean, roughly unit-variance smooth random field of shape (h, w)."""
    gh = max(3, int(round(h / cell)) + 2)
    gw = max(3, int(round(w / cell)) + 2)
    g = rng.standard_normal((gh, gw), dtype=np.float32)
    # two passes of a small box blur on the control grid soften the lattice
    g = (g + np.roll(g, 1, 0) + np.roll(g, -1, 0)) / 3.0
    g = (g + np.roll(g, 1, 1) + np.roll(g, -1, 1)) / 3.0
    g /= max(float(g.std()), 1e-6)
    return _interp_matrix(h, gh) @ g @ _interp_matrix(w, gw).T


def _content_from_grids(spec: FrameSpec, grids, rho: np.ndarray | None) -> np.ndarray:
    """Noise-free tissue-like colour field, float32 (H, W, 3), mean luma near
    spec.mean_luma, from the control grids of ``smooth_grids``."""
    h, w = spec.height, spec.width
    base_g, fine_g, chroma_g, tint = grids

    def field(g):
        return _interp_matrix(h, g.shape[0]) @ g @ _interp_matrix(w, g.shape[1]).T

    lum = spec.mean_luma * (1.0 + 0.18 * field(base_g) + 0.06 * field(fine_g))
    chroma = [field(g) for g in chroma_g]
    img = np.empty((h, w, 3), dtype=np.float32)
    for c in range(3):
        img[..., c] = lum * np.float32(tint[c]) * (1.0 + np.float32(0.08) * chroma[c])
    if spec.vignette > 0.0:
        if rho is None:
            yy, xx = np.mgrid[0:h, 0:w].astype(np.float32)
            rho = np.hypot(xx - (w - 1) / 2.0, yy - (h - 1) / 2.0)
            scale = float(np.hypot(w, h) / 2.0)
        else:
            scale = spec.r
        fall = 1.0 - spec.vignette * np.minimum(rho / scale, 1.0) ** 2
        img *= fall[..., None]
    return img


def _content(rng: np.random.Generator, spec: FrameSpec, rho: np.ndarray | None) -> np.ndarray:
    """Tissue-like smooth colour field with pixel noise (sigma 2), float32 (H, W, 3)."""
    img = _content_from_grids(spec, smooth_grids(rng, spec), rho)
    img += 2.0 * rng.standard_normal(img.shape, dtype=np.float32)
    return img


def render_noise_free(spec: FrameSpec, grids) -> np.ndarray:
    """The frame of ``render`` without its pixel and border noise (float32,
    before rounding), from given control grids: the image model's
    deterministic part, against which a device renderer can be checked."""
    h, w = spec.height, spec.width
    if spec.kind == KIND_NOBORDER:
        return _content_from_grids(spec, grids, None)
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float32)
    rho = np.hypot(xx - np.float32(spec.cx), yy - np.float32(spec.cy))
    img = _content_from_grids(spec, grids, rho)
    alpha = ndtr((np.float32(spec.r) - rho) / np.float32(spec.blur_sigma)).astype(np.float32)
    return alpha[..., None] * img + (1.0 - alpha)[..., None] * np.float32(6.0)


def render(spec: FrameSpec, rng: np.random.Generator) -> np.ndarray:
    """Render one uint8 (H, W, 3) RGB frame for ``spec`` from ``rng``."""
    h, w = spec.height, spec.width
    if spec.kind == KIND_NOBORDER:
        img = _content(rng, spec, None)
        return np.clip(np.rint(img), 0, 255).astype(np.uint8)
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float32)
    rho = np.hypot(xx - np.float32(spec.cx), yy - np.float32(spec.cy))
    img = _content(rng, spec, rho)
    alpha = ndtr((np.float32(spec.r) - rho) / np.float32(spec.blur_sigma)).astype(np.float32)
    border = 6.0 + np.float32(spec.border_sigma) * rng.standard_normal((h, w), dtype=np.float32)
    out = alpha[..., None] * img + (1.0 - alpha)[..., None] * border[..., None]
    return np.clip(np.rint(out), 0, 255).astype(np.uint8)


def _corners_outside(cx: float, cy: float, r: float, w: int, h: int) -> int:
    corners = [(-0.5, -0.5), (w - 0.5, -0.5), (-0.5, h - 0.5), (w - 0.5, h - 0.5)]
    return sum(1 for (x, y) in corners if np.hypot(x - cx, y - cy) > r)


def draw_spec(rng: np.random.Generator, w: int, h: int, mix: tuple[float, float, float],
              border_sigma: tuple[float, float], blur_sigma: tuple[float, float],
              vignette: tuple[float, float], radius_frac: tuple[float, float] | None) -> FrameSpec:
    """Draw the ground truth of one frame.

    ``radius_frac`` fixes r ~ U(lo, hi) * H for every bordered frame (the
    small 640x480 workload); when it is None the kind decides the radius:
    partial circles r ~ U(0.55, 0.95) * H with at least one corner outside
    the disc, full circles r ~ U(0.30 H, distance to the nearest edge - 3 blur).
    """
    p = np.asarray(mix, dtype=np.float64)
    kind = int(rng.choice(3, p=p / p.sum()))
    bs = float(rng.uniform(*border_sigma))
    bl = float(rng.uniform(*blur_sigma))
    vg = float(rng.uniform(*vignette))
    luma = float(rng.uniform(90.0, 150.0))
    for _ in range(1000):
        cx = (w - 1) / 2.0 + float(rng.uniform(-0.08, 0.08)) * w
        cy = (h - 1) / 2.0 + float(rng.uniform(-0.08, 0.08)) * h
        if kind == KIND_NOBORDER:
            r = float(np.hypot(w, h))
            break
        if radius_frac is not None:
            r = float(rng.uniform(*radius_frac)) * h
            inside = min(cx + 0.5, w - 0.5 - cx, cy + 0.5, h - 0.5 - cy) >= r
            kind = KIND_FULL if inside else KIND_PARTIAL
            break
        if kind == KIND_PARTIAL:
            r = float(rng.uniform(0.55, 0.95)) * h
            if _corners_outside(cx, cy, r, w, h) >= 1:
                break
        else:
            rmax = min(cx + 0.5, w - 0.5 - cx, cy + 0.5, h - 0.5 - cy) - 3.0 * bl
            if rmax > 0.30 * h:
                r = float(rng.uniform(0.30 * h, rmax))
                break
    else:  # pragma: no cover - the rejection loop accepts within a few draws
        raise RuntimeError("could not draw a frame spec")
    return FrameSpec(w, h, kind, cx, cy, r, bs, bl, vg, luma)


@dataclasses.dataclass
class Workload:
    """Shape and distribution of one synthetic workload."""
    config_id: int
    width: int
    height: int
    n_frames: int
    mix: tuple[float, float, float]
    border_sigma: tuple[float, float]
    blur_sigma: tuple[float, float]
    vignette: tuple[float, float]
    radius_frac: tuple[float, float] | None
    n_hstrips: int
    n_vstrips: int
    attempts: int


# Small case: 8 x 640x480, every frame bordered, r ~ U(0.45, 0.75) H,
# border sigma 3, edge blur 1.5 px; 16+16 strips, 256 RANSAC attempts.
SMALL_640x480 = Workload(1, 640, 480, 8, (1.0, 0.0, 0.0), (3.0, 3.0), (1.5, 1.5), (0.0, 0.0),
                         (0.45, 0.75), 16, 16, 256)
# Headline case: 64 x 1920x1080, partial : full : no border = 60 : 25 : 10 (renormalised),
# border sigma U(2, 8), blur U(1, 3), vignetting up to 40 %; 32+32 strips, 1024 attempts.
HD_1080p = Workload(2, 1920, 1080, 64, (60.0, 25.0, 10.0), (2.0, 8.0), (1.0, 3.0), (0.0, 0.4),
                    None, 32, 32, 1024)
WORKLOADS = {1: SMALL_640x480, 2: HD_1080p}


def frame_rng(config_id: int, frame_idx: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([ROOT_SEED, config_id, frame_idx]))


def make_frame(wl: Workload, frame_idx: int, width: int | None = None,
               height: int | None = None) -> tuple[np.ndarray, FrameSpec]:
    """Frame ``frame_idx`` of workload ``wl`` (optionally at another resolution)."""
    rng = frame_rng(wl.config_id, frame_idx)
    w = wl.width if width is None else width
    h = wl.height if height is None else height
    spec = draw_spec(rng, w, h, wl.mix, wl.border_sigma, wl.blur_sigma, wl.vignette,
                     wl.radius_frac)
    return render(spec, rng), spec


def make_batch(wl: Workload, n_frames: int | None = None, start: int = 0,
               width: int | None = None, height: int | None = None
               ) -> tuple[np.ndarray, list[FrameSpec]]:
    """uint8 [B, H, W, 3] batch of frames start .. start+B-1 and their specs."""
    n = wl.n_frames if n_frames is None else n_frames
    frames, specs = [], []
    for i in range(start, start + n):
        f, s = make_frame(wl, i, width, height)
        frames.append(f)
        specs.append(s)
    return np.stack(frames), specs


# ------------------------------------------------------------ hard frames --
#
# Failure cases of the handcrafted score (Section 1.1, Figure 3): a dark rim
# that leaves only a small luma step at the edge, strong border noise,
# specular blobs and white text overlays in the border.  Hard frames are
# rendered on the device (the training set is far too large for a CPU
# renderer); this module draws their parameters.

GLYPH_W, GLYPH_H = 5, 7        # dot-matrix glyph cells


@dataclasses.dataclass
class HardExtras:
    """Extra ground-truth-free distractors of a hard frame."""
    edge_step: float                      # content luma at the rim = 6 + edge_step (0: off)
    blobs: list                           # (x, y, radius, amplitude) in the border
    text_x: float = 0.0                   # top-left corner of the text block
    text_y: float = 0.0
    text_scale: int = 0                   # pixels per glyph cell (0: no text)
    text_lines: int = 0
    text_chars: int = 0
    glyphs: np.ndarray | None = None      # uint64 [lines * chars], 35 bits each


def _in_border(spec: FrameSpec, x: float, y: float, margin: float) -> bool:
    return bool(np.hypot(x - spec.cx, y - spec.cy) > spec.r + margin)


def draw_hard(rng: np.random.Generator, spec: FrameSpec,
              edge_step: tuple[float, float] = (10.0, 25.0)) -> HardExtras:
    """Draw the distractors of a hard frame (none in a frame without border)."""
    ex = HardExtras(edge_step=float(rng.uniform(*edge_step)), blobs=[])
    if not spec.has_border:
        ex.edge_step = 0.0
        return ex
    w, h = spec.width, spec.height
    margin = 3.0 * spec.blur_sigma + 2.0
    for _ in range(int(rng.integers(0, 4))):
        for _ in range(50):
            x, y = float(rng.uniform(0, w - 1)), float(rng.uniform(0, h - 1))
            rad = float(rng.uniform(3.0, 15.0))
            if _in_border(spec, x, y, margin + 2.0 * rad):
                ex.blobs.append((x, y, rad, float(rng.uniform(120.0, 250.0))))
                break
    if rng.uniform() < 0.8:
        scale = int(rng.integers(2, 4))
        lines = int(rng.integers(1, 5))
        chars = int(rng.integers(4, 15))
        bw = chars * (GLYPH_W + 1) * scale
        bh = lines * (GLYPH_H + 2) * scale
        corners = [(4.0, 4.0), (w - 5.0 - bw, 4.0), (4.0, h - 5.0 - bh), (w - 5.0 - bw, h - 5.0 - bh)]
        order = rng.permutation(4)
        for ci in order:
            x0, y0 = corners[ci]
            if x0 < 0 or y0 < 0:
                continue
            box = [(x0, y0), (x0 + bw, y0), (x0, y0 + bh), (x0 + bw, y0 + bh)]
            if all(_in_border(spec, x, y, margin) for x, y in box) and \
                    _in_border(spec, x0 + bw / 2, y0 + bh / 2, margin):
                ex.text_x, ex.text_y = x0, y0
                ex.text_scale, ex.text_lines, ex.text_chars = scale, lines, chars
                bits = rng.integers(0, 2, (lines * chars, GLYPH_W * GLYPH_H), dtype=np.uint64)
                bits[rng.uniform(size=lines * chars) < 0.15] = 0     # spaces
                ex.glyphs = (bits << np.arange(GLYPH_W * GLYPH_H, dtype=np.uint64)).sum(
                    axis=1).astype(np.uint64)
                break
    return ex


def smooth_grids(rng: np.random.Generator, spec: FrameSpec):
    """Control grids of the content's smooth fields (base, fine, 3 chroma),
    blurred and normalised exactly as the CPU renderer does before its
    bilinear interpolation, and the per-frame channel tint."""
    h, w = spec.height, spec.width
    cell = max(h, w) / 10.0

    def grid(c):
        gh = max(3, int(round(h / c)) + 2)
        gw = max(3, int(round(w / c)) + 2)
        g = rng.standard_normal((gh, gw), dtype=np.float32)
        g = (g + np.roll(g, 1, 0) + np.roll(g, -1, 0)) / 3.0
        g = (g + np.roll(g, 1, 1) + np.roll(g, -1, 1)) / 3.0
        g /= max(float(g.std()), 1e-6)
        return g.astype(np.float32)

    base = grid(cell)
    fine = grid(cell / 4.0)
    tint = np.array([1.30, 0.88, 0.72], dtype=np.float32)
    tint = tint * (1.0 + 0.05 * rng.standard_normal(3).astype(np.float32))
    tint /= float(0.299 * tint[0] + 0.587 * tint[1] + 0.114 * tint[2])
    chroma = [grid(cell) for _ in range(3)]
    return base, fine, chroma, tint


# Uneven batch: 512 frames of four resolutions in ratio 2 : 3 : 4 : 1 with the
# headline distributions, shapes interleaved by a seeded permutation.
MIXED_512 = Workload(3, 1920, 1080, 512, (60.0, 25.0, 10.0), (2.0, 8.0), (1.0, 3.0), (0.0, 0.4),
                     None, 32, 32, 1024)
MIXED_SHAPES = ((720, 576, 2), (1280, 720, 3), (1920, 1080, 4), (3840, 2160, 1))
WORKLOADS[3] = MIXED_512


def mixed_shapes(n: int = 512) -> list[tuple[int, int]]:
    """(width, height) of frames 0 .. n-1 of the uneven batch."""
    total = sum(k for _, _, k in MIXED_SHAPES)
    # largest remainder: 102 / 154 / 205 / 51 at n = 512
    quota = [n * k / total for _, _, k in MIXED_SHAPES]
    counts = [int(q) for q in quota]
    for i in sorted(range(len(quota)), key=lambda i: counts[i] - quota[i])[:n - sum(counts)]:
        counts[i] += 1
    shapes = [(w, h) for (w, h, _), c in zip(MIXED_SHAPES, counts) for _ in range(c)]
    order = np.random.default_rng(np.random.SeedSequence([ROOT_SEED, 3])).permutation(n)
    return [shapes[i] for i in order]


def make_mixed_batch(n: int = 512, threads: int = 1):
    """Frames and specs of the uneven batch (a list: the shapes differ)."""
    shapes = mixed_shapes(n)

    def one(i):
        return make_frame(MIXED_512, i, *shapes[i])

    if threads > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(threads) as ex:
            out = list(ex.map(one, range(n)))
    else:
        out = [one(i) for i in range(n)]
    return [f for f, _ in out], [s for _, s in out]


# Hard 1080p frames: the headline mix with border noise sigma up to 12 and the
# distractors above.
HARD_1080p = Workload(4, 1920, 1080, 64, (60.0, 25.0, 10.0), (2.0, 12.0), (1.0, 3.0), (0.0, 0.4),
                      None, 32, 32, 1024)
WORKLOADS[4] = HARD_1080p

