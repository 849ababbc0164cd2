"""TEST INFRASTRUCTURE ONLY: plain numpy statement of the paper's own learned
edge scorer (Section 2.2.4), for the parity tests of the library's 2-D CNN
kernels.  Nothing in the library imports it.

The network, as the paper gives it: three 3x3 convolutions with 8, 16 and 32
output features, each followed by a ReLU, then a 1x1 convolution to a single
feature and a sigmoid, giving an edge probability per pixel.  The input has
five channels per pixel, RGBXY: the colour channels normalised by the mean
and standard deviation of each channel over the training data, and the pixel
coordinates normalised to [-0.5, 0.5] with (0, 0) at the image centre.  The
network is applied only to the selected strips, seven pixels thick (its
receptive field), so a strip's scores are the full-image network's output
on the strip's centre line.

Numeric definition (shared with the GPU kernels by definition, not by code):
  * colour c of an 8-bit sample v: bf16((f32(v) - mean_c) * inv_std_c) in
    float32 arithmetic (mean_c and inv_std_c are float32 constants of the
    model); coordinates bf16(f32(2x - (W-1)) / f32(2(W-1))) and the same for
    y with H;
  * 3x3 convolutions with zero "same" padding: every layer's input is zero
    outside the frame (a strip's band sees zero rows beyond the frame edge
    and zero positions beyond the strip's ends);
  * weights stored in bfloat16, biases in float32, each hidden activation
    stored in bfloat16 (round to nearest even); the oracle evaluates every
    sum in float64;
  * logit z; score sigmoid(z).
Model-file order (float32): mean[3], inv_std[3], then W1[8][5][3][3], b1,
W2[16][8][3][3], b2, W3[32][16][3][3], b3, w4[32], b4: 6215 values, of which
the 6209 after the normaliser are trained.

A band is the strip's seven lines: for a horizontal strip through row r the
rows r-3 .. r+3, positions along the row; for a vertical strip through
column c the columns c-3 .. c+3, positions down the column (the weights'
two spatial axes then swap roles).
"""
from __future__ import annotations

import numpy as np

CONVS = [(5, 8), (8, 16), (16, 32)]   # 3x3 convolutions (in, out)
N_NORM = 6
BAND = 7                               # lines of a strip band
HALF = BAND // 2


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest even) via float32; returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounding = ((u >> 16) & 1) + 0x7FFF
    u = ((u + rounding) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def n_params() -> int:
    return N_NORM + sum(co * ci * 9 + co for ci, co in CONVS) + 32 + 1


def init_params(seed: int = 0):
    """He-style random weights (rounded to bfloat16), small random biases, and
    a normaliser of typical endoscopic statistics: (norm, [(W, b)] * 3, (w4, b4))."""
    rng = np.random.default_rng(seed)
    norm = (np.array([110.0, 70.0, 60.0]), np.array([1 / 50.0, 1 / 40.0, 1 / 40.0]))
    norm = tuple(np.asarray(v, dtype=np.float32).astype(np.float64) for v in norm)
    convs = []
    for ci, co in CONVS:
        w = bf16(rng.standard_normal((co, ci, 3, 3)) * np.sqrt(2.0 / (ci * 9)))
        b = rng.normal(0.0, 0.05, co).astype(np.float32).astype(np.float64)
        convs.append((w, b))
    w4 = bf16(rng.standard_normal(32) * np.sqrt(1.0 / 32))
    b4 = np.array([-1.0])
    return norm, convs, (w4, b4)


def flat_params(params) -> np.ndarray:
    norm, convs, (w4, b4) = params
    parts = [norm[0], norm[1]]
    for w, b in convs:
        parts += [w.ravel(), b.ravel()]
    parts += [w4.ravel(), b4.ravel()]
    return np.concatenate(parts)


def unflat_params(v: np.ndarray):
    """Inverse of flat_params; weights rounded to bfloat16 as the model
    stores them, the rest as float32 values."""
    v = np.asarray(v, dtype=np.float64)
    f32 = lambda a: a.astype(np.float32).astype(np.float64)   # noqa: E731
    norm = (f32(v[0:3]), f32(v[3:6]))
    at = N_NORM
    convs = []
    for ci, co in CONVS:
        w = bf16(v[at:at + co * ci * 9].reshape(co, ci, 3, 3))
        at += co * ci * 9
        b = f32(v[at:at + co])
        at += co
        convs.append((w, b))
    w4 = bf16(v[at:at + 32])
    b4 = f32(v[at + 32:at + 33])
    return norm, convs, (w4, b4)


# ---------------------------------------------------------------- input --

def input_image(frame: np.ndarray, norm) -> np.ndarray:
    """RGBXY [5, H, W] of a whole frame, every value a bfloat16 number."""
    h, w = frame.shape[:2]
    mean = norm[0].astype(np.float32)
    inv = norm[1].astype(np.float32)
    rgb = (frame.astype(np.float32) - mean[None, None, :]) * inv[None, None, :]
    x = np.float32(2 * np.arange(w) - (w - 1)) / np.float32(2 * (w - 1))
    y = np.float32(2 * np.arange(h) - (h - 1)) / np.float32(2 * (h - 1))
    out = np.empty((5, h, w))
    out[0:3] = bf16(rgb.transpose(2, 0, 1))
    out[3] = bf16(np.broadcast_to(x[None, :], (h, w)))
    out[4] = bf16(np.broadcast_to(y[:, None], (h, w)))
    return out


def band_input(frame: np.ndarray, line: int, horizontal: bool, norm):
    """Band [5, 7, L] of a strip through `line` (rows for a horizontal
    strip, columns for a vertical one) and which of its 7 lines lie in the
    frame; lines beyond the frame are zero."""
    img = input_image(frame, norm)
    if not horizontal:
        img = img.transpose(0, 2, 1)            # lines are columns
    extent, L = img.shape[1], img.shape[2]
    band = np.zeros((5, BAND, L))
    ok = np.zeros(BAND, dtype=bool)
    for j in range(BAND):
        r = line - HALF + j
        if 0 <= r < extent:
            band[:, j] = img[:, r]
            ok[j] = True
    return band, ok


# --------------------------------------------------------- whole image --

def conv3x3_same(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[o, i, j] = b[o] + sum_{c, dy, dx} w[o, c, dy, dx] x[c, i+dy-1, j+dx-1],
    zero outside x."""
    ci, h, wd = x.shape
    xp = np.zeros((ci, h + 2, wd + 2))
    xp[:, 1:h + 1, 1:wd + 1] = x
    y = np.tile(b[:, None, None], (1, h, wd)).astype(np.float64)
    for dy in range(3):
        for dx in range(3):
            y += np.einsum("oc,chw->ohw", w[:, :, dy, dx], xp[:, dy:dy + h, dx:dx + wd])
    return y


def forward_image(frame: np.ndarray, params, store_bf16: bool = True) -> np.ndarray:
    """Logits of every pixel of a (small) frame: the network as defined."""
    norm, convs, (w4, b4) = params
    h = input_image(frame, norm)
    for w, b in convs:
        a = np.maximum(conv3x3_same(h, w, b), 0.0)
        h = bf16(a) if store_bf16 else a
    return b4[0] + np.einsum("o,ohw->hw", w4, h)


# ---------------------------------------------------------------- bands --

def _oriented(w: np.ndarray, horizontal: bool) -> np.ndarray:
    """Weights indexed [o, c, across, along] for a band: the frame's (dy, dx)
    for a horizontal strip, (dx, dy) for a vertical one."""
    return w if horizontal else w.transpose(0, 1, 3, 2)


def _conv_band(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Across: valid (R lines in, R - 2 out); along: same, zero padded."""
    ci, R, L = x.shape
    xp = np.zeros((ci, R, L + 2))
    xp[:, :, 1:L + 1] = x
    y = np.tile(b[:, None, None], (1, R - 2, L)).astype(np.float64)
    for da in range(3):
        for dl in range(3):
            y += np.einsum("oc,crl->orl", w[:, :, da, dl], xp[:, da:da + R - 2, dl:dl + L])
    return y


def forward_band(x: np.ndarray, line_ok: np.ndarray, pos_ok: np.ndarray, params,
                 horizontal: bool, store_bf16: bool = True) -> dict:
    """Activations of one band: x [5, 7, L], line_ok [7] (line inside the
    frame), pos_ok [L] (position inside the strip).  Hidden layer k keeps the
    band's lines k .. 6-k; values outside the frame or strip are zero in every
    layer's input.  Returns h (inputs of each layer), pre (pre-activations),
    z (logits of the centre line), s."""
    _, convs, (w4, b4) = params
    keep = line_ok[:, None] & pos_ok[None, :]
    x = np.where(keep[None], x, 0.0)
    h, pre = [x], []
    for k, (w, b) in enumerate(convs):
        a = _conv_band(h[-1], _oriented(w, horizontal), b)
        a = np.where(keep[None, k + 1:BAND - k - 1], a, 0.0)
        pre.append(a)
        r = np.maximum(a, 0.0)
        h.append(bf16(r) if store_bf16 else r)
    z = b4[0] + w4 @ h[-1][:, 0, :]
    return {"h": h, "pre": pre, "z": z, "s": 1.0 / (1.0 + np.exp(-z))}


def _conv_band_backward(x: np.ndarray, w: np.ndarray, dy: np.ndarray):
    """Gradients of _conv_band: (dx, dw, db)."""
    ci, R, L = x.shape
    xp = np.zeros((ci, R, L + 2))
    xp[:, :, 1:L + 1] = x
    dw = np.zeros_like(w)
    dxp = np.zeros_like(xp)
    for da in range(3):
        for dl in range(3):
            win = xp[:, da:da + R - 2, dl:dl + L]
            dw[:, :, da, dl] = np.einsum("orl,crl->oc", dy, win)
            dxp[:, da:da + R - 2, dl:dl + L] += np.einsum("oc,orl->crl", w[:, :, da, dl], dy)
    return dxp[:, :, 1:L + 1], dw, dy.sum(axis=(1, 2))


def backward_band(cache: dict, line_ok, pos_ok, params, horizontal: bool, dz: np.ndarray,
                  grad_bf16: bool = False):
    """Gradients (frame orientation) of every trained parameter for an
    upstream gradient dz on the centre line's logits: [(dW, db)] * 3 and
    (dw4, db4).  With grad_bf16 the signal at each hidden pre-activation
    (ReLU and masks applied) is stored in bfloat16 before it is used."""
    _, convs, (w4, b4) = params
    keep = line_ok[:, None] & pos_ok[None, :]
    h = cache["h"]
    dw4 = h[-1][:, 0, :] @ dz
    db4 = np.array([dz.sum()])
    dh = (w4[:, None] * dz[None, :])[:, None, :]          # [32, 1, L]
    out = [None] * len(convs)
    for k in range(len(convs) - 1, -1, -1):
        w, b = convs[k]
        dpre = dh * (cache["pre"][k] > 0)
        dpre = np.where(keep[None, k + 1:BAND - k - 1], dpre, 0.0)
        if grad_bf16:
            dpre = bf16(dpre)
        dx, dw, db = _conv_band_backward(h[k], _oriented(w, horizontal), dpre)
        out[k] = (_oriented(dw, horizontal), db)
        dh = dx
    return out, (dw4, db4)


# --------------------------------------------------------------- strips --

def strip_logits(frame: np.ndarray, line: int, horizontal: bool, params) -> np.ndarray:
    """Logits of every position of one strip through `line`."""
    band, ok = band_input(frame, line, horizontal, params[0])
    return forward_band(band, ok, np.ones(band.shape[2], dtype=bool), params, horizontal)["z"]


def learned_half_strip_scores(frame: np.ndarray, params, n_h: int, n_v: int, alpha: float = 8.0):
    """Per half strip, in canonical candidate order: (xs, ys, scores) of all
    pixels in scan order (k = 0 at the outer edge)."""
    import oracle as ora
    h, w = frame.shape[:2]
    out = []
    for r in ora.strip_positions(h, n_h, alpha):
        s = 1.0 / (1.0 + np.exp(-strip_logits(frame, int(r), True, params)))
        k = np.arange(w // 2)
        out.append((k, np.full_like(k, r), s[k]))
        k2 = np.arange(w - w // 2)
        out.append((w - 1 - k2, np.full_like(k2, r), s[w - 1 - k2]))
    for c in ora.strip_positions(w, n_v, alpha):
        s = 1.0 / (1.0 + np.exp(-strip_logits(frame, int(c), False, params)))
        k = np.arange(h // 2)
        out.append((np.full_like(k, c), k, s[k]))
        k2 = np.arange(h - h // 2)
        out.append((np.full_like(k2, c), h - 1 - k2, s[h - 1 - k2]))
    return out


# -------------------------------------------------------------- windows --

WINDOW = 128      # positions of one training / test window
HALO = 8          # the window's first and last HALO positions carry no output
OUTPUTS = WINDOW - 2 * HALO


def window_band(win_u8: np.ndarray, geom, norm):
    """Band [5, 7, WINDOW] and line_ok of a rendered window: win_u8
    [8, WINDOW, 3] holds lines line-3 .. line+4 (clamped to the frame) of a
    strip, geom = (horizontal, line, start, width, height)."""
    hz, line, start, W, H = (int(v) for v in geom[:5])
    extent = H if hz else W
    mean = norm[0].astype(np.float32)
    inv = norm[1].astype(np.float32)
    rgb = (win_u8[:BAND].astype(np.float32) - mean[None, None, :]) * inv[None, None, :]
    band = np.zeros((5, BAND, WINDOW))
    band[0:3] = bf16(rgb.transpose(2, 0, 1))
    p = start + np.arange(WINDOW)
    lines = line - HALF + np.arange(BAND)
    xs = np.broadcast_to((p[None, :] if hz else lines[:, None]), (BAND, WINDOW))
    ys = np.broadcast_to((lines[:, None] if hz else p[None, :]), (BAND, WINDOW))
    band[3] = bf16(np.float32(2 * xs - (W - 1)) / np.float32(2 * (W - 1)))
    band[4] = bf16(np.float32(2 * ys - (H - 1)) / np.float32(2 * (H - 1)))
    ok = (lines >= 0) & (lines < extent)
    return band, ok


def window_forward(win_u8: np.ndarray, geom, lo: int, hi: int, params) -> np.ndarray:
    """Logits of the OUTPUTS central positions of one window whose positions
    lo .. hi-1 belong to the strip (NaN where outside)."""
    band, ok = window_band(win_u8, geom, params[0])
    mask = np.zeros(WINDOW, dtype=bool)
    mask[lo:hi] = True
    z = forward_band(band, ok, mask, params, bool(geom[0]))["z"][HALO:WINDOW - HALO]
    return np.where(mask[HALO:WINDOW - HALO], z, np.nan)


def loss_and_grads(wins, geoms, ranges, targets, weights, params, scale: float,
                   grad_bf16: bool = False):
    """scale * sum over windows and central positions of weight * soft BCE,
    and its gradients in model-file order (zeros for the normaliser)."""
    acc_c = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params[1]]
    acc4 = [np.zeros(32), np.zeros(1)]
    loss = 0.0
    for win, g, (lo, hi), t, wt in zip(wins, geoms, ranges, targets, weights):
        band, ok = window_band(win, g, params[0])
        mask = np.zeros(WINDOW, dtype=bool)
        mask[lo:hi] = True
        c = forward_band(band, ok, mask, params, bool(g[0]))
        tt = np.zeros(WINDOW)
        tt[HALO:WINDOW - HALO] = t
        ww = np.zeros(WINDOW)
        ww[HALO:WINDOW - HALO] = wt
        ww = np.where(mask, ww, 0.0)
        s = c["s"]
        eps = 1e-12
        loss += scale * float(np.sum(-ww * (tt * np.log(s + eps) + (1 - tt) * np.log(1 - s + eps))))
        dz = scale * ww * (s - tt)
        gc, (dw4, db4) = backward_band(c, ok, mask, params, bool(g[0]), dz, grad_bf16)
        acc_c = [(a[0] + gw, a[1] + gb) for a, (gw, gb) in zip(acc_c, gc)]
        acc4 = [acc4[0] + dw4, acc4[1] + db4]
    grads = (np.zeros(3), np.zeros(3)), acc_c, tuple(acc4)
    return loss, flat_params(grads)
