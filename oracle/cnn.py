"""TEST INFRASTRUCTURE ONLY: plain numpy statement of the learned strip scorer.

The paper replaces the handcrafted edge score by a shallow CNN whose output
probability is the edge score (Section 2.2.4), trained with soft binary
cross entropy and SGD on edge maps blurred with a Gaussian of sigma 3.  The
network here follows the spec form of that idea: a 1-D CNN along each
strip whose input at every strip position is the 3 colours of 8 lines
(24 channels), four convolutions of width 5 (24 -> 16 -> 32 -> 32 -> 16,
ReLU), a 1x1 convolution to one logit, and a sigmoid.

Numeric definition (shared with the GPU kernels by definition, not by code):
  * input value (v - 128) / 64 for an 8-bit sample v (exact in bfloat16);
    lines pos-3 .. pos+4 around the strip's line, clamped to the frame;
  * weights are stored in bfloat16, biases in float32;
  * each hidden activation is stored in bfloat16 (round to nearest even);
  * positions outside the strip are zero in every layer's input ("same"
    zero padding);
  * logit z, score sigmoid(z).
The oracle evaluates every sum in float64; only the storage roundings are
emulated.  Gradients follow the chain rule through the stored values
(rounding is treated as identity), the loss being the mean soft BCE.  With
``grad_bf16`` the backward signal at each hidden pre-activation (ReLU mask
applied) is also stored in bfloat16, as a training pass that keeps its
backward activations in bfloat16 does; the 1x1 layer's logit gradient stays
exact.
"""
from __future__ import annotations

import numpy as np

LAYERS = [(24, 16, 5), (16, 32, 5), (32, 32, 5), (32, 16, 5), (16, 1, 1)]
N_LINES = 8
LINE_OFFSETS = tuple(range(-3, 5))  # across the strip: pos-3 .. pos+4


def n_params() -> int:
    return sum(co * ci * k + co for ci, co, k in LAYERS)


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest even) via float32; returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounding = ((u >> 16) & 1) + 0x7FFF
    u = ((u + rounding) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed: int = 0) -> list[tuple[np.ndarray, np.ndarray]]:
    """He-style random init; weights already rounded to bfloat16."""
    rng = np.random.default_rng(seed)
    out = []
    for ci, co, k in LAYERS:
        w = rng.standard_normal((co, ci, k)) * np.sqrt(2.0 / (ci * k))
        b = np.zeros(co)
        out.append((bf16(w), b.astype(np.float32).astype(np.float64)))
    return out


def strip_input(frame: np.ndarray, pos: int, horizontal: bool) -> np.ndarray:
    """X[24, L]: channel 3*j + colour is line pos + LINE_OFFSETS[j] (clamped)."""
    h, w = frame.shape[:2]
    extent = h if horizontal else w
    lines = [min(max(pos + o, 0), extent - 1) for o in LINE_OFFSETS]
    if horizontal:
        rows = frame[lines]                      # [8, W, 3]
    else:
        rows = frame[:, lines].transpose(1, 0, 2)  # [8, H, 3]
    x = (rows.astype(np.float64) - 128.0) / 64.0
    return x.transpose(0, 2, 1).reshape(N_LINES * 3, -1)


def conv_same(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[o, p] = b[o] + sum_c sum_t w[o, c, t] x[c, p + t - k//2], zero outside."""
    co, ci, k = w.shape
    L = x.shape[1]
    half = k // 2
    xp = np.zeros((ci, L + 2 * half))
    xp[:, half:half + L] = x
    y = np.tile(b[:, None], (1, L))
    for t in range(k):
        y += w[:, :, t] @ xp[:, t:t + L]
    return y


def forward(x: np.ndarray, params, store_bf16: bool = True, mask=None) -> dict:
    """Activations of one strip: h[0] = input, h[1..4] hidden, z logit, s score.

    `mask` (optional, boolean per position) marks the positions that belong
    to the strip; the others are zero in every layer's input, as beyond the
    ends of a strip."""
    if mask is not None:
        x = np.where(mask[None, :], x, 0.0)
    h = [x]
    pre = []
    for li, (w, b) in enumerate(params[:-1]):
        a = conv_same(h[-1], w, b)
        if mask is not None:
            a = np.where(mask[None, :], a, 0.0)
        pre.append(a)
        r = np.maximum(a, 0.0)
        h.append(bf16(r) if store_bf16 else r)
    w5, b5 = params[-1]
    z = conv_same(h[-1], w5, b5)[0]
    s = 1.0 / (1.0 + np.exp(-z))
    return {"h": h, "pre": pre, "z": z, "s": s}


def bce(s: np.ndarray, t: np.ndarray) -> float:
    eps = 1e-12
    return float(-np.mean(t * np.log(s + eps) + (1 - t) * np.log(1 - s + eps)))


def conv_backward(x: np.ndarray, w: np.ndarray, dy: np.ndarray):
    """Gradients of conv_same: (dx, dw, db)."""
    co, ci, k = w.shape
    L = x.shape[1]
    half = k // 2
    xp = np.zeros((ci, L + 2 * half))
    xp[:, half:half + L] = x
    dw = np.zeros_like(w)
    for t in range(k):
        dw[:, :, t] = dy @ xp[:, t:t + L].T
    db = dy.sum(axis=1)
    dxp = np.zeros_like(xp)
    for t in range(k):
        dxp[:, t:t + L] += w[:, :, t].T @ dy
    return dxp[:, half:half + L], dw, db


def backward(cache: dict, params, dz: np.ndarray, mask=None, grad_bf16: bool = False):
    """Parameter gradients for an upstream gradient dz on the logits."""
    h = cache["h"]
    grads = [None] * len(params)
    w5, b5 = params[-1]
    dx, dw, db = conv_backward(h[-1], w5, dz[None, :])
    grads[-1] = (dw, db)
    for li in range(len(params) - 2, -1, -1):
        w, b = params[li]
        dpre = dx * (cache["pre"][li] > 0)
        if mask is not None:
            dpre = np.where(mask[None, :], dpre, 0.0)
        if grad_bf16:
            dpre = bf16(dpre)
        dx, dw, db = conv_backward(h[li], w, dpre)
        grads[li] = (dw, db)
    return grads


def flat_params(params) -> np.ndarray:
    """Parameters in the model-file order: W1, b1, W2, b2, ..., W5, b5."""
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])


def unflat_params(v: np.ndarray):
    out, at = [], 0
    for ci, co, k in LAYERS:
        w = v[at:at + co * ci * k].reshape(co, ci, k)
        at += co * ci * k
        b = v[at:at + co]
        at += co
        out.append((np.asarray(w, dtype=np.float64), np.asarray(b, dtype=np.float64)))
    return out


WINDOW = 128      # positions of one window
HALO = 8          # receptive-field radius of the network
OUTPUTS = WINDOW - 2 * HALO


def window_forward(win_u8: np.ndarray, lo: int, hi: int, params) -> np.ndarray:
    """Logits of the OUTPUTS central positions of one window [8, WINDOW, 3]
    whose positions lo .. hi-1 belong to the strip (NaN where outside)."""
    x = (win_u8.astype(np.float64) - 128.0) / 64.0            # [8, W, 3]
    x = x.transpose(0, 2, 1).reshape(N_LINES * 3, WINDOW)
    mask = np.zeros(WINDOW, dtype=bool)
    mask[lo:hi] = True
    z = forward(x, params, True, mask)["z"][HALO:WINDOW - HALO]
    return np.where(mask[HALO:WINDOW - HALO], z, np.nan)


def loss_and_grads(xs, ts, params, store_bf16: bool = True, masks=None, weights=None,
                   scale=None, grad_bf16: bool = False):
    """Weighted soft-BCE over the positions of a list of strips, and its
    gradients: scale * sum of weight * BCE, scale = 1 / (sum of the weights)
    unless given (the mean when every weight is 1).  `weights` (optional, per
    strip, per position, >= 0) selects the positions that carry a loss;
    `masks` marks positions inside the strip."""
    if weights is None:
        weights = [np.ones(len(t)) for t in ts]
    if masks is None:
        masks = [None] * len(ts)
    total = sum(float(w.sum()) for w in weights) if scale is None else 1.0 / scale
    loss = 0.0
    acc = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
    for x, t, m, wt in zip(xs, ts, masks, weights):
        c = forward(x, params, store_bf16, m)
        eps = 1e-12
        s = c["s"]
        loss += float(np.sum(-wt * (t * np.log(s + eps) + (1 - t) * np.log(1 - s + eps)))) / total
        dz = wt * (s - t) / total
        g = backward(c, params, dz, m, grad_bf16)
        acc = [(a[0] + gw, a[1] + gb) for a, (gw, gb) in zip(acc, g)]
    return loss, acc


def edge_target(length: int, pos: int, horizontal: bool, circle, sigma: float = 3.0):
    """Soft edge label along a strip line: a Gaussian (sigma 3 px) of each
    pixel's distance to the content circle's boundary; zero without a circle."""
    if circle is None:
        return np.zeros(length)
    cx, cy, r = circle
    k = np.arange(length, dtype=np.float64)
    if horizontal:
        rho = np.hypot(k - cx, pos - cy)
    else:
        rho = np.hypot(pos - cx, k - cy)
    return np.exp(-((rho - r) ** 2) / (2.0 * sigma * sigma))


def strip_logits(frame: np.ndarray, pos: int, horizontal: bool, params) -> np.ndarray:
    """Logits of every position of one strip (the whole line, zero padded)."""
    return forward(strip_input(frame, pos, horizontal), params, True)["z"]


def learned_half_strip_scores(frame: np.ndarray, params, n_h: int, n_v: int, alpha: float = 8.0):
    """Per half strip, in canonical candidate order: (xs, ys, scores) of all
    pixels in scan order (k = 0 at the outer edge), scores = sigmoid(logit)."""
    import oracle as ora
    h, w = frame.shape[:2]
    rows = ora.strip_positions(h, n_h, alpha)
    cols = ora.strip_positions(w, n_v, alpha)
    out = []
    for i, r in enumerate(rows):
        s = 1.0 / (1.0 + np.exp(-strip_logits(frame, int(r), True, params)))
        k = np.arange(w // 2)
        out.append((k, np.full_like(k, r), s[k]))
        k2 = np.arange(w - w // 2)
        out.append((w - 1 - k2, np.full_like(k2, r), s[w - 1 - k2]))
    for j, c in enumerate(cols):
        s = 1.0 / (1.0 + np.exp(-strip_logits(frame, int(c), False, params)))
        k = np.arange(h // 2)
        out.append((np.full_like(k, c), k, s[k]))
        k2 = np.arange(h - h // 2)
        out.append((np.full_like(k2, c), h - 1 - k2, s[h - 1 - k2]))
    return out
