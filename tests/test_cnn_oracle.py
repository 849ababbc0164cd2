"""Pins of the learned-scorer oracle (oracle/cnn.py): torch's conv1d and
autograd (library routines, float64, CPU), central finite differences, the
bfloat16 rounding against torch's bfloat16 conversion, and the soft edge
label's closed form."""
import math

import numpy as np
import pytest
import torch

from oracle import cnn


def _torch_forward(x, params):
    h = torch.tensor(x)[None]
    for w, b in params[:-1]:
        h = torch.relu(torch.nn.functional.conv1d(h, torch.tensor(w), torch.tensor(b), padding=2))
    w5, b5 = params[-1]
    z = torch.nn.functional.conv1d(h, torch.tensor(w5), torch.tensor(b5))[0, 0]
    return z


def test_parameter_count():
    assert cnn.n_params() == 12273


def test_bf16_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-8, 8, 5000),
                        [0.0, 1.0, -1.0, 1.00390625, 1.005859375, 3.0e38]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.bf16(x), ref)


def test_forward_matches_torch_conv1d():
    params = cnn.init_params(1)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((24, 137))
    c = cnn.forward(x, params, store_bf16=False)
    np.testing.assert_allclose(c["z"], _torch_forward(x, params).numpy(), rtol=1e-12, atol=1e-12)


def test_backward_matches_autograd():
    params = cnn.init_params(3)
    rng = np.random.default_rng(4)
    xs = [rng.standard_normal((24, n)) for n in (40, 71)]
    ts = [rng.uniform(0, 1, n) for n in (40, 71)]
    loss, grads = cnn.loss_and_grads(xs, ts, params, store_bf16=False)
    tp = [(torch.tensor(w, requires_grad=True), torch.tensor(b, requires_grad=True))
          for w, b in params]
    total = sum(len(t) for t in ts)
    tl = 0
    for x, t in zip(xs, ts):
        h = torch.tensor(x)[None]
        for w, b in tp[:-1]:
            h = torch.relu(torch.nn.functional.conv1d(h, w, b, padding=2))
        z = torch.nn.functional.conv1d(h, tp[-1][0], tp[-1][1])[0, 0]
        tl = tl + torch.nn.functional.binary_cross_entropy_with_logits(
            z, torch.tensor(t), reduction="sum") / total
    tl.backward()
    assert abs(tl.item() - loss) < 1e-9
    for (gw, gb), (w, b) in zip(grads, tp):
        np.testing.assert_allclose(gw, w.grad.numpy(), rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(gb, b.grad.numpy(), rtol=1e-9, atol=1e-12)


def test_backward_finite_differences():
    params = cnn.init_params(5)
    rng = np.random.default_rng(6)
    xs = [rng.standard_normal((24, 30))]
    ts = [rng.uniform(0, 1, 30)]
    _, grads = cnn.loss_and_grads(xs, ts, params, store_bf16=False)
    eps = 1e-6
    for li, idx in [(0, (3, 7, 1)), (1, (20, 5, 4)), (2, (0, 31, 2)), (3, (9, 12, 0)), (4, (0, 11, 0))]:
        w, b = params[li]
        wp = w.copy()
        wp[idx] += eps
        wm = w.copy()
        wm[idx] -= eps
        pp = list(params)
        pp[li] = (wp, b)
        lp, _ = cnn.loss_and_grads(xs, ts, pp, store_bf16=False)
        pp[li] = (wm, b)
        lm, _ = cnn.loss_and_grads(xs, ts, pp, store_bf16=False)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - grads[li][0][idx]) < 1e-6 * max(1.0, abs(fd)), (li, idx)


def test_strip_input_layout_and_exactness():
    frame = np.arange(20 * 30 * 3, dtype=np.int64).reshape(20, 30, 3) % 256
    frame = frame.astype(np.uint8)
    x = cnn.strip_input(frame, 1, True)           # rows -2..5 clamp to 0..5
    assert x.shape == (24, 30)
    assert np.array_equal(x[0], (frame[0, :, 0] - 128.0) / 64.0)     # row 1-3 -> 0
    assert np.array_equal(x[3 * 7 + 2], (frame[5, :, 2] - 128.0) / 64.0)
    assert np.array_equal(cnn.bf16(x), x)        # inputs are exact in bfloat16
    y = cnn.strip_input(frame, 28, False)         # columns 25..32 clamp to 25..29
    assert y.shape == (24, 20)
    assert np.array_equal(y[3 * 7 + 1], (frame[:, 29, 1] - 128.0) / 64.0)


def test_edge_target_closed_form():
    t = cnn.edge_target(200, 50, True, (100.0, 50.0, 30.0))
    assert t[70] == 1.0 and t[130] == 1.0
    assert abs(t[73] - math.exp(-9 / 18)) < 1e-12
    assert np.all(cnn.edge_target(50, 5, False, None) == 0)


class _RoundForward(torch.autograd.Function):
    """bfloat16 storage of an activation; the gradient passes unchanged."""

    @staticmethod
    def forward(ctx, x):
        return x.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    @staticmethod
    def backward(ctx, g):
        return g


class _RoundBackward(torch.autograd.Function):
    """Identity forward; the gradient is stored in bfloat16."""

    @staticmethod
    def forward(ctx, x):
        return x.clone()

    @staticmethod
    def backward(ctx, g):
        return g.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def test_bf16_backward_signals_match_autograd():
    """The grad_bf16 mode: autograd with explicit bfloat16 roundings of the
    stored activations and of the gradients at the hidden pre-activations,
    masked windows and per-position loss weights, a given scale."""
    rng = np.random.default_rng(8)
    params = [(w, b + rng.normal(0, 0.1, b.shape)) for w, b in cnn.init_params(9)]
    L = 64
    xs = [cnn.bf16(rng.standard_normal((24, L))) for _ in range(3)]
    ts = [rng.uniform(0, 1, L) for _ in range(3)]
    masks = [np.ones(L, bool), np.arange(L) < 40, np.arange(L) >= 11]
    weights = [rng.uniform(0, 2, L) * (rng.uniform(size=L) > 0.2) for _ in range(3)]
    scale = 1.0 / 77.0
    loss, grads = cnn.loss_and_grads(xs, ts, params, True, masks, weights, scale, grad_bf16=True)
    tp = [(torch.tensor(w, requires_grad=True), torch.tensor(b, requires_grad=True))
          for w, b in params]
    tl = 0
    for x, t, m, wt in zip(xs, ts, masks, weights):
        mt = torch.tensor(m)
        h = torch.where(mt, torch.tensor(x), torch.zeros(()))[None]
        for w, b in tp[:-1]:
            a = torch.nn.functional.conv1d(h, w, b, padding=2)
            a = torch.where(mt, a, torch.zeros(()))
            h = _RoundForward.apply(torch.relu(_RoundBackward.apply(a)))
        z = torch.nn.functional.conv1d(h, tp[-1][0], tp[-1][1])[0, 0]
        tl = tl + scale * (torch.tensor(wt) * torch.nn.functional.binary_cross_entropy_with_logits(
            z, torch.tensor(t), reduction="none")).sum()
    tl.backward()
    assert abs(tl.item() - loss) < 1e-9
    for (gw, gb), (w, b) in zip(grads, tp):
        np.testing.assert_allclose(gw, w.grad.numpy(), rtol=1e-9, atol=1e-15)
        np.testing.assert_allclose(gb, b.grad.numpy(), rtol=1e-9, atol=1e-15)
    # and the rounding matters: the exact chain rule differs
    _, exact = cnn.loss_and_grads(xs, ts, params, True, masks, weights, scale)
    assert any(not np.array_equal(a[0], b[0]) for a, b in zip(grads, exact))
