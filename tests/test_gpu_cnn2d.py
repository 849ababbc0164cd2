"""GPU parity of the paper's own learned scorer (three 3x3 convolutions on
RGBXY strip bands) against the numpy oracle (oracle/cnn2d.py): window
logits in both strip orientations and at the frame edges, the learned
candidates of whole strips, gradients of the soft cross entropy, and the
SGD step."""
import numpy as np
import pytest

from oracle import cnn2d
from paper_2210_14771_amd import _native as N
from paper_2210_14771_amd import api, synth

from gpu_helpers import say

pytestmark = pytest.mark.gpu

# bfloat16 storage of hidden activations: GPU (float32 sums) and oracle
# (float64 sums) round an activation differently when a sum lies within
# rounding distance of a bfloat16 tie; such flips move a logit by a few 1e-3
LOGIT_TOL = 0.03
GRAD_MAX_REL = 4e-3      # max |gpu - oracle| / max |oracle| per parameter tensor
GRAD_NORM_REL = 2e-3     # ||gpu - oracle|| / ||oracle||
LOSS_REL = 1e-5


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


def _params(seed):
    norm, convs, (w4, b4) = cnn2d.init_params(seed)
    rng = np.random.default_rng(seed + 50)
    convs = [(w, (b + rng.normal(0, 0.1, b.shape)).astype(np.float32).astype(np.float64))
             for w, b in convs]
    return norm, convs, (w4, b4)


def _windows(rng, n, W=640, H=480):
    """Random window bytes with the geometry of strips of a W x H frame:
    both orientations, lines at and near the frame edges, windows crossing
    the strip ends."""
    win = rng.integers(0, 256, (n, 8, 128, 3), dtype=np.uint8)
    geom = np.zeros((n, 8), dtype=np.int32)
    ranges = np.zeros((n, 2), dtype=np.int32)
    for i in range(n):
        hz = i % 2 == 0
        extent, L = (H, W) if hz else (W, H)
        line = [0, 1, 2, extent - 1, extent - 3][i % 5] if i % 3 == 0 else int(rng.integers(0, extent))
        start = [-8, L - 120, int(rng.integers(-8, L - 119))][i % 3]
        geom[i, :5] = (int(hz), line, start, W, H)
        ranges[i] = (max(0, -start), min(128, L - start))
    return win, geom, ranges


def _dev(torch, *arrays):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


@pytest.mark.parametrize("seed", [0, 1])
def test_window_logits_match_oracle(torch_dev, est, seed):
    torch = torch_dev
    params = _params(seed)
    est.set_model_2d(cnn2d.flat_params(params))
    rng = np.random.default_rng(seed)
    win, geom, ranges = _windows(rng, 12)
    say(f"2-D window logits seed {seed}")
    z = est.cnn2d_window_logits(*_dev(torch, win, geom, ranges))
    torch.cuda.synchronize()
    z = z.cpu().numpy()
    for i in range(len(win)):
        ref = cnn2d.window_forward(win[i], geom[i], int(ranges[i, 0]), int(ranges[i, 1]), params)
        ok = ~np.isnan(ref)
        d = np.abs(z[i][ok] - ref[ok])
        assert d.max() <= LOGIT_TOL, (i, d.max())
        assert np.median(d) <= 1e-3


def test_learned_2d_candidates_are_valid_argmax(torch_dev, est):
    torch = torch_dev
    params = _params(3)
    est.set_model_2d(cnn2d.flat_params(params))
    frames, _ = synth.make_batch(synth.SMALL_640x480, 2)
    kw = dict(n_hstrips=4, n_vstrips=3, ransac_attempts=64, scorer=N.CA_SCORER_LEARNED_2D)
    say("2-D learned candidates")
    res, pts = est.debug_candidates(torch.from_numpy(frames).cuda(), api.default_params(**kw),
                                    [0, 1])
    torch.cuda.synchronize()
    g = api.points_numpy(pts)
    tol = 0.01
    for f in range(2):
        halves = cnn2d.learned_half_strip_scores(frames[f], params, 4, 3)
        for c, (xs, ys, sc) in enumerate(halves):
            gx, gy, gs = int(g[f][c]["x"]), int(g[f][c]["y"]), float(g[f][c]["score"])
            idx = np.flatnonzero((xs == gx) & (ys == gy))
            assert idx.size == 1, (f, c, gx, gy)
            assert sc[idx[0]] >= sc.max() - tol, (f, c, sc[idx[0]], sc.max())
            assert abs(gs - sc[idx[0]]) <= tol


def _slices():
    out, at = [], cnn2d.N_NORM
    for k, (ci, co) in enumerate(cnn2d.CONVS):
        out.append((f"W{k + 1}", slice(at, at + co * ci * 9)))
        at += co * ci * 9
        out.append((f"b{k + 1}", slice(at, at + co)))
        at += co
    out.append(("w4", slice(at, at + 32)))
    out.append(("b4", slice(at + 32, at + 33)))
    return out


def _case(rng, n):
    win, geom, ranges = _windows(rng, n)
    targets = rng.uniform(0, 1, (n, 112)).astype(np.float32)
    weights = (rng.uniform(0, 2, (n, 112)) * (rng.uniform(size=(n, 112)) > 0.3)).astype(np.float32)
    return win, geom, ranges, targets, weights


@pytest.mark.parametrize("seed,n", [(0, 37), (1, 600)])
def test_gradients_match_oracle(torch_dev, est, seed, n):
    """n = 600 exceeds the gradient grid: workgroups accumulate several windows."""
    torch = torch_dev
    params = _params(seed + 10)
    est.set_model_2d(cnn2d.flat_params(params))
    rng = np.random.default_rng(seed)
    win, geom, ranges, targets, weights = _case(rng, n)
    scale = float(np.float32(1.0 / max(weights.sum(), 1.0)))
    say(f"2-D gradients seed {seed} n {n}")
    grad, loss = est.cnn2d_gradients(*_dev(torch, win, geom, ranges, targets, weights), scale)
    torch.cuda.synchronize()
    g = grad.cpu().numpy().astype(np.float64)
    ref_loss, ref = cnn2d.loss_and_grads(win, geom, ranges, targets, weights, params, scale,
                                         grad_bf16=True)
    assert abs(loss.item() - ref_loss) <= LOSS_REL * abs(ref_loss)
    assert np.all(g[:cnn2d.N_NORM] == 0)
    for name, sl in _slices():
        d = g[sl] - ref[sl]
        scale_t = np.abs(ref[sl]).max()
        assert scale_t > 0, name
        assert np.abs(d).max() <= GRAD_MAX_REL * scale_t, (name, np.abs(d).max() / scale_t)
        assert np.linalg.norm(d) <= GRAD_NORM_REL * np.linalg.norm(ref[sl]), name
    # the bfloat16 backward signals stay close to the exact chain rule
    _, exact = cnn2d.loss_and_grads(win, geom, ranges, targets, weights, params, scale,
                                    grad_bf16=False)
    cos = g @ exact / (np.linalg.norm(g) * np.linalg.norm(exact))
    assert cos > 0.9999


def test_gradients_of_no_windows_are_zero(torch_dev, est):
    torch = torch_dev
    est.set_model_2d(cnn2d.flat_params(_params(2)))
    e8 = torch.empty((0, 8, 128, 3), dtype=torch.uint8, device="cuda")
    g8 = torch.empty((0, 8), dtype=torch.int32, device="cuda")
    e2 = torch.empty((0, 2), dtype=torch.int32, device="cuda")
    ef = torch.empty((0, 112), dtype=torch.float32, device="cuda")
    grad, loss = est.cnn2d_gradients(e8, g8, e2, ef, ef, 1.0)
    torch.cuda.synchronize()
    assert not grad.cpu().numpy().any() and loss.item() == 0.0


def test_sgd_step_updates_master_and_model(torch_dev, est):
    """Two momentum steps are bit-exact float32 arithmetic (the normaliser
    receives zero gradient and stays); the rebuilt device model scores
    windows like the oracle with the new weights."""
    torch = torch_dev
    rng = np.random.default_rng(5)
    p0 = cnn2d.flat_params(_params(4)).astype(np.float32)
    est.set_model_2d(p0)
    g = (rng.standard_normal(p0.size) * 0.01).astype(np.float32)
    g[:cnn2d.N_NORM] = 0.0
    gd = torch.from_numpy(g).cuda()
    lr, mu = np.float32(0.5), np.float32(0.9)
    est.cnn2d_sgd_step(gd, float(lr), float(mu))
    est.cnn2d_sgd_step(gd, float(lr), float(mu))
    p, m = est.get_model_2d(with_momentum=True)
    m1 = mu * np.zeros_like(g) + g
    p1 = p0 - lr * m1
    m2 = mu * m1 + g
    p2 = p1 - lr * m2
    np.testing.assert_array_equal(m, m2)
    np.testing.assert_array_equal(p, p2)
    new = cnn2d.unflat_params(p.astype(np.float64))
    win, geom, ranges = _windows(rng, 6)
    z = est.cnn2d_window_logits(*_dev(torch, win, geom, ranges))
    torch.cuda.synchronize()
    z = z.cpu().numpy()
    for i in range(len(win)):
        ref = cnn2d.window_forward(win[i], geom[i], int(ranges[i, 0]), int(ranges[i, 1]), new)
        ok = ~np.isnan(ref)
        assert np.abs(z[i][ok] - ref[ok]).max() <= LOGIT_TOL


def test_trained_2d_scorer_1080p_candidates_ransac_and_fallback(torch_dev):
    """The committed trained 2-D network on two headline 1080p frames with
    32+32 strips: every candidate is a within-tolerance maximum of the
    oracle's half-strip scores; the RANSAC over the kept candidates equals the
    oracle's attempt by attempt; with the 0.5 inlier fallback a frame below
    the fraction carries the oracle's handcrafted result."""
    import os

    import oracle
    from paper_2210_14771_amd import train_scorer

    from gpu_helpers import assert_attempts_equal, assert_results_equal, oracle_params

    torch = torch_dev
    path = os.path.join(train_scorer.MODEL_DIR, train_scorer.MODEL_FILE_2D)
    if not os.path.exists(path):
        pytest.skip("no trained 2-D scorer model")
    flat = train_scorer.load_model_2d(path)
    params = cnn2d.unflat_params(flat.astype(np.float64))
    e = api.Estimator(0)
    e.set_model_2d(flat)
    frames, _ = synth.make_batch(synth.HD_1080p, 2)
    dev = torch.from_numpy(frames).cuda()
    uids = [0, 1]
    kw = dict(n_hstrips=32, n_vstrips=32, ransac_attempts=1024)
    say("trained 2-D scorer at 1080p")
    _, pts = e.debug_candidates(dev, api.default_params(**kw, scorer=2), uids)
    res_l, att = e.debug_attempts(dev, api.default_params(**kw, scorer=2), uids)
    res_f = e.estimate_area(dev, api.default_params(**kw, scorer=2, fallback_inlier_frac=0.5),
                            uids)
    torch.cuda.synchronize()
    g = api.points_numpy(pts)
    res_l, res_f = res_l.numpy(), res_f.numpy()
    att = api.attempts_numpy(att)
    op = oracle_params(**kw)
    for f in range(2):
        halves = cnn2d.learned_half_strip_scores(frames[f], params, 32, 32)
        for c, (xs, ys, sc) in enumerate(halves):
            gx, gy, gs = int(g[f][c]["x"]), int(g[f][c]["y"]), float(g[f][c]["score"])
            idx = np.flatnonzero((xs == gx) & (ys == gy))
            assert idx.size == 1, (f, c, gx, gy)
            assert sc[idx[0]] >= sc.max() - 0.01, (f, c, sc[idx[0]], sc.max())
            assert abs(gs - sc[idx[0]]) <= 0.01
        s32 = g[f]["score"].astype(np.float32)
        keep = s32 >= np.float32(op.t_ps)
        xs = g[f]["x"][keep].astype(np.int32)
        ys = g[f]["y"][keep].astype(np.int32)
        sq = (s32[keep].astype(np.float64) * 2.0 ** 24).astype(np.uint32)
        assert int(res_l[f]["n_points"]) == int(keep.sum())
        assert_attempts_equal([att[f]], [oracle.ransac_attempts(xs, ys, sq, 1920, 1080, uids[f], op)])
        n = int(res_l[f]["n_points"])
        if n < 3 or np.float32(res_l[f]["inliers"]) < np.float32(0.5) * np.float32(n):
            want = oracle.estimate(frames[f], op, uids[f]).copy()
            want["reason"] += 256
            assert_results_equal([res_f[f]], [want])
        else:
            assert res_f[f].tobytes() == res_l[f].tobytes()
    e.close()


def test_trained_2d_scorer_gains_on_hard_frames(torch_dev):
    """The paper's own network, trained here, against the handcrafted scorer
    on device-rendered hard frames (low-contrast rims, strong border noise,
    specular blobs, text in the border)."""
    import os

    from paper_2210_14771_amd import evaluate, synth_gpu, train_scorer

    path = os.path.join(train_scorer.MODEL_DIR, train_scorer.MODEL_FILE_2D)
    if not os.path.exists(path):
        pytest.skip("no trained 2-D scorer model")
    e = api.Estimator(0)
    e.set_model_2d(train_scorer.load_model_2d(path))
    frames, specs = synth_gpu.render_set(synth.HARD_1080p, synth.HARD_1080p.config_id, 64, True)
    kw = dict(n_hstrips=32, n_vstrips=32, ransac_attempts=1024)
    plain = evaluate.accuracy(e, frames, specs, api.default_params(**kw))
    learned = evaluate.accuracy(e, frames, specs, api.default_params(**kw, scorer=2))
    say(f"hard frames: plain {plain}  2-D learned {learned}")
    assert learned["frac_le_2px"] >= plain["frac_le_2px"] + 0.2
    assert learned["median_px"] < plain["median_px"]
    e.close()
