"""GPU parity of the learned strip scorer's kernels against the numpy oracle:
the MFMA lane layout, window logits, and the learned pipeline's candidates."""
import numpy as np
import pytest

from oracle import cnn
from paper_2210_14771_amd import api, synth

from gpu_helpers import say

pytestmark = pytest.mark.gpu

# bfloat16 storage of hidden activations makes GPU (float32 sums) and oracle
# (float64 sums) round an activation differently when a sum lies within
# rounding distance of a bfloat16 tie; such flips move a logit by a few 1e-3.
LOGIT_TOL = 0.03


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def est(torch_dev):
    e = api.Estimator(0)
    yield e
    e.close()


def test_mfma_16x16x32_bf16_layout(torch_dev, est):
    out = est.selftest_mfma()
    torch_dev.cuda.synchronize()
    m = np.arange(16)[:, None]
    k = np.arange(32)[None, :]
    A = (m * 7 + k * 3) % 11 - 5
    Bm = (np.arange(32)[:, None] * 5 + np.arange(16)[None, :] * 2) % 13 - 6
    np.testing.assert_array_equal(out.cpu().numpy(), (A @ Bm).astype(np.float32))


def _random_windows(rng, n):
    win = rng.integers(0, 256, (n, 8, 128, 3), dtype=np.uint8)
    ranges = np.tile(np.array([0, 128], dtype=np.int32), (n, 1))
    ranges[1] = (0, 60)       # strip ends inside the window
    ranges[2] = (20, 128)
    ranges[3] = (9, 100)
    return win, ranges


@pytest.mark.parametrize("seed", [0, 1])
def test_window_logits_match_oracle(torch_dev, est, seed):
    torch = torch_dev
    rng = np.random.default_rng(seed)
    params = cnn.init_params(seed + 10)
    # give the biases some spread so that ReLUs are not all open
    params = [(w, b + rng.normal(0, 0.1, b.shape)) for w, b in params]
    est.set_model(cnn.flat_params(params))
    win, ranges = _random_windows(rng, 6)
    say(f"window logits seed {seed}")
    z = est.cnn_window_logits(torch.from_numpy(win).cuda(), torch.from_numpy(ranges).cuda())
    torch.cuda.synchronize()
    z = z.cpu().numpy()
    for i in range(len(win)):
        ref = cnn.window_forward(win[i], int(ranges[i, 0]), int(ranges[i, 1]), params)
        ok = ~np.isnan(ref)
        d = np.abs(z[i][ok] - ref[ok])
        assert d.max() <= LOGIT_TOL, (i, d.max())
        assert np.median(d) <= 1e-3


def test_learned_candidates_are_valid_argmax(torch_dev, est):
    torch = torch_dev
    rng = np.random.default_rng(3)
    params = [(w, b + rng.normal(0, 0.1, b.shape)) for w, b in cnn.init_params(7)]
    est.set_model(cnn.flat_params(params))
    frames, _ = synth.make_batch(synth.SMALL_640x480, 2)
    kw = dict(n_hstrips=4, n_vstrips=3, ransac_attempts=64, scorer=1)
    say("learned candidates")
    res, pts = est.debug_candidates(torch.from_numpy(frames).cuda(), api.default_params(**kw), [0, 1])
    torch.cuda.synchronize()
    g = api.points_numpy(pts)
    tol = 0.01
    for f in range(2):
        halves = cnn.learned_half_strip_scores(frames[f], params, 4, 3)
        for c, (xs, ys, sc) in enumerate(halves):
            gx, gy, gs = int(g[f][c]["x"]), int(g[f][c]["y"]), float(g[f][c]["score"])
            idx = np.flatnonzero((xs == gx) & (ys == gy))
            assert idx.size == 1, (f, c, gx, gy)
            # the chosen pixel is a maximum within tolerance, with its own score
            assert sc[idx[0]] >= sc.max() - tol, (f, c, sc[idx[0]], sc.max())
            assert abs(gs - sc[idx[0]]) <= tol
