"""Pins of the oracle of the paper's own learned scorer (oracle/cnn2d.py):
torch's conv2d and autograd (library routines, float64, CPU) for the whole
image and for bands, the band of a strip equal to the whole-image network's
row or column (zero padding at the frame edges, the weights' spatial axes
swapped for vertical strips), the RGBXY encoding's closed forms, and a
rendered window equal to the band of the strip it was cut from."""
import numpy as np
import pytest
import torch

from oracle import cnn2d


def _torch_image(frame, params):
    norm, convs, (w4, b4) = params
    h = torch.tensor(cnn2d.input_image(frame, norm))[None]
    for w, b in convs:
        h = torch.relu(torch.nn.functional.conv2d(h, torch.tensor(w), torch.tensor(b), padding=1))
    return (torch.einsum("o,ohw->hw", torch.tensor(w4), h[0]) + float(b4[0])).numpy()


def _frame(seed, h=17, w=23):
    return np.random.default_rng(seed).integers(0, 256, (h, w, 3), dtype=np.uint8)


def test_parameter_count_and_layout():
    assert cnn2d.n_params() == 6 + (8 * 5 * 9 + 8) + (16 * 8 * 9 + 16) + (32 * 16 * 9 + 32) + 33
    assert cnn2d.n_params() == 6215
    p = cnn2d.init_params(3)
    v = cnn2d.flat_params(p)
    assert v.shape == (6215,)
    q = cnn2d.unflat_params(v)
    np.testing.assert_array_equal(cnn2d.flat_params(q), v)


def test_whole_image_matches_torch_conv2d():
    params = cnn2d.init_params(1)
    frame = _frame(2)
    z = cnn2d.forward_image(frame, params, store_bf16=False)
    np.testing.assert_allclose(z, _torch_image(frame, params), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_bands_equal_the_whole_image_rows_and_columns(seed):
    params = cnn2d.init_params(seed + 5)
    frame = _frame(seed + 7, 19, 26)
    full = cnn2d.forward_image(frame, params)
    H, W = frame.shape[:2]
    for r in range(H):
        np.testing.assert_allclose(cnn2d.strip_logits(frame, r, True, params), full[r],
                                   rtol=0, atol=1e-12, err_msg=f"row {r}")
    for c in range(W):
        np.testing.assert_allclose(cnn2d.strip_logits(frame, c, False, params), full[:, c],
                                   rtol=0, atol=1e-12, err_msg=f"column {c}")


def test_rgbxy_encoding_closed_forms():
    norm = (np.array([110.0, 70.0, 60.0]), np.array([0.02, 0.025, 0.025]))
    frame = np.zeros((5, 9, 3), dtype=np.uint8)
    frame[2, 4] = (128, 70, 255)
    x = cnn2d.input_image(frame, norm)
    assert x[0, 2, 4] == cnn2d.bf16(np.float32(18.0) * np.float32(0.02))
    assert x[1, 2, 4] == 0.0
    assert x[2, 2, 4] == cnn2d.bf16(np.float32(195.0) * np.float32(0.025))
    # coordinates: -0.5 at the first pixel, +0.5 at the last, 0 at the centre
    assert x[3, 0, 0] == -0.5 and x[3, 0, 8] == 0.5 and x[3, 0, 4] == 0.0
    assert x[4, 0, 0] == -0.5 and x[4, 4, 0] == 0.5 and x[4, 2, 0] == 0.0
    assert x[3, 0, 2] == cnn2d.bf16(-0.25)
    assert np.all(x == cnn2d.bf16(x))


@pytest.mark.parametrize("horizontal", [True, False])
def test_band_backward_matches_autograd(horizontal):
    params = cnn2d.init_params(4)
    frame = _frame(9, 21, 30)
    line = 1                                    # two band lines beyond the frame
    band, ok = cnn2d.band_input(frame, line, horizontal, params[0])
    L = band.shape[2]
    pos_ok = np.zeros(L, dtype=bool)
    pos_ok[2:L - 3] = True
    rng = np.random.default_rng(0)
    dz = rng.standard_normal(L)
    c = cnn2d.forward_band(band, ok, pos_ok, params, horizontal, store_bf16=False)
    gc, (dw4, db4) = cnn2d.backward_band(c, ok, pos_ok, params, horizontal, dz)

    _, convs, (w4, b4) = params
    ts = [torch.tensor(w, requires_grad=True) for w, _ in convs]
    tb = [torch.tensor(b, requires_grad=True) for _, b in convs]
    tw4 = torch.tensor(w4, requires_grad=True)
    tb4 = torch.tensor(b4, requires_grad=True)
    keep = torch.tensor(ok[:, None] & pos_ok[None, :], dtype=torch.float64)
    h = torch.tensor(band) * keep
    for k in range(3):
        w = ts[k] if horizontal else ts[k].transpose(2, 3)
        a = torch.nn.functional.conv2d(h[None], w, tb[k], padding=(0, 1))[0]
        a = a * keep[k + 1:cnn2d.BAND - k - 1]
        h = torch.relu(a)
    z = tw4 @ h[:, 0, :] + tb4[0]
    np.testing.assert_allclose(c["z"], z.detach().numpy(), rtol=1e-12, atol=1e-12)
    (z * torch.tensor(dz)).sum().backward()
    for k in range(3):
        np.testing.assert_allclose(gc[k][0], ts[k].grad.numpy(), rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(gc[k][1], tb[k].grad.numpy(), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(dw4, tw4.grad.numpy(), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(db4, tb4.grad.numpy(), rtol=1e-10, atol=1e-12)


def _cut_window(frame, horizontal, line, start):
    """The renderer's window layout: lines line-3 .. line+4 clamped to the
    frame, positions start .. start+127 clamped."""
    H, W = frame.shape[:2]
    ext, L = (H, W) if horizontal else (W, H)
    win = np.zeros((8, cnn2d.WINDOW, 3), dtype=np.uint8)
    for j in range(8):
        ln = min(max(line - 3 + j, 0), ext - 1)
        for p in range(cnn2d.WINDOW):
            q = min(max(start + p, 0), L - 1)
            win[j, p] = frame[ln, q] if horizontal else frame[q, ln]
    return win


@pytest.mark.parametrize("horizontal,line,start", [(True, 0, -8), (True, 9, 40), (False, 2, -8),
                                                   (False, 20, 100)])
def test_window_band_is_the_strip_band(horizontal, line, start):
    params = cnn2d.init_params(6)
    frame = _frame(11, 160, 200)
    H, W = frame.shape[:2]
    win = _cut_window(frame, horizontal, line, start)
    geom = (int(horizontal), line, start, W, H)
    band_w, ok_w = cnn2d.window_band(win, geom, params[0])
    band_s, ok_s = cnn2d.band_input(frame, line, horizontal, params[0])
    np.testing.assert_array_equal(ok_w, ok_s)
    L = band_s.shape[2]
    for p in range(cnn2d.WINDOW):
        q = start + p
        if 0 <= q < L:
            np.testing.assert_array_equal(band_w[:, ok_w, p], band_s[:, ok_s, q])
    # the window's logits are the strip's where the window has full context
    lo, hi = max(0, -start), min(cnn2d.WINDOW, L - start)
    z = cnn2d.window_forward(win, geom, lo, hi, params)
    ref = cnn2d.strip_logits(frame, line, horizontal, params)
    for i in range(cnn2d.OUTPUTS):
        q = start + cnn2d.HALO + i
        if lo <= cnn2d.HALO + i < hi:
            assert abs(z[i] - ref[q]) < 1e-12
        else:
            assert np.isnan(z[i])


def test_loss_gradients_match_autograd_of_windows():
    params = cnn2d.init_params(8)
    frame = _frame(12, 150, 190)
    H, W = frame.shape[:2]
    cases = [(True, 5, 0), (False, 1, 60), (True, 149, 70)]
    wins = [_cut_window(frame, hz, ln, st) for hz, ln, st in cases]
    geoms = [(int(hz), ln, st, W, H) for hz, ln, st in cases]
    ranges = [(0, 128), (0, 128 - 38), (3, 120)]
    rng = np.random.default_rng(1)
    targets = [rng.uniform(0, 1, cnn2d.OUTPUTS) for _ in cases]
    weights = [rng.uniform(0, 2, cnn2d.OUTPUTS) for _ in cases]
    scale = 0.01
    loss, g = cnn2d.loss_and_grads(wins, geoms, ranges, targets, weights, params, scale)
    # finite differences of the same loss (float64 activations: no bfloat16
    # storage, so the loss is smooth away from ReLU kinks)
    v = cnn2d.flat_params(params)

    # directional derivative along a random direction of the trained part
    d = np.zeros_like(v)
    d[6:] = rng.standard_normal(v.size - 6)
    eps = 1e-6

    def loss_at(vec):
        p = _unrounded(vec)
        total = 0.0
        for win, gm, (lo, hi), t, wt in zip(wins, geoms, ranges, targets, weights):
            band, ok = cnn2d.window_band(win, gm, p[0])
            mask = np.zeros(cnn2d.WINDOW, dtype=bool)
            mask[lo:hi] = True
            c = cnn2d.forward_band(band, ok, mask, p, bool(gm[0]), store_bf16=False)
            tt = np.zeros(cnn2d.WINDOW)
            tt[cnn2d.HALO:-cnn2d.HALO] = t
            ww = np.zeros(cnn2d.WINDOW)
            ww[cnn2d.HALO:-cnn2d.HALO] = wt
            ww = np.where(mask, ww, 0.0)
            s = c["s"]
            total += scale * float(np.sum(-ww * (tt * np.log(s) + (1 - tt) * np.log(1 - s))))
        return total

    def _unrounded(vec):
        at = cnn2d.N_NORM
        convs = []
        for ci, co in cnn2d.CONVS:
            w = vec[at:at + co * ci * 9].reshape(co, ci, 3, 3)
            at += co * ci * 9
            convs.append((w, vec[at:at + co]))
            at += co
        return params[0], convs, (vec[at:at + 32], vec[at + 32:at + 33])

    num = (loss_at(v + eps * d) - loss_at(v - eps * d)) / (2 * eps)
    # the analytic gradient of the unrounded network at the same point
    _, g_exact = _loss_unrounded(wins, geoms, ranges, targets, weights, params, scale)
    assert abs(num - g_exact @ d) <= 1e-6 * max(1.0, abs(num))
    # with bfloat16 storage the gradients stay close to the exact chain rule
    cos = g @ g_exact / (np.linalg.norm(g) * np.linalg.norm(g_exact))
    assert cos > 0.999
    assert np.all(g[:6] == 0)
    assert loss > 0


def _loss_unrounded(wins, geoms, ranges, targets, weights, params, scale):
    """loss_and_grads without bfloat16 storage of activations."""
    acc = None
    loss = 0.0
    for win, gm, (lo, hi), t, wt in zip(wins, geoms, ranges, targets, weights):
        band, ok = cnn2d.window_band(win, gm, params[0])
        mask = np.zeros(cnn2d.WINDOW, dtype=bool)
        mask[lo:hi] = True
        c = cnn2d.forward_band(band, ok, mask, params, bool(gm[0]), store_bf16=False)
        tt = np.zeros(cnn2d.WINDOW)
        tt[cnn2d.HALO:-cnn2d.HALO] = t
        ww = np.zeros(cnn2d.WINDOW)
        ww[cnn2d.HALO:-cnn2d.HALO] = wt
        ww = np.where(mask, ww, 0.0)
        s = c["s"]
        loss += scale * float(np.sum(-ww * (tt * np.log(s) + (1 - tt) * np.log(1 - s))))
        gc, g4 = cnn2d.backward_band(c, ok, mask, params, bool(gm[0]), scale * ww * (s - tt))
        flat = cnn2d.flat_params(((np.zeros(3), np.zeros(3)), gc, g4))
        acc = flat if acc is None else acc + flat
    return loss, acc
