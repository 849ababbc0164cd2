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


def test_trained_scorer_1080p_candidates_ransac_and_fallback(torch_dev):
    """The committed trained network on two headline 1080p frames with 32+32
    strips: every candidate is a within-tolerance maximum of the numpy
    statement's half-strip scores; the RANSAC over the kept learned
    candidates equals the oracle's attempt by attempt; with the 0.5 inlier
    fallback a frame below the fraction carries the oracle's handcrafted
    result, any other frame the learned one."""
    import os

    import oracle
    from paper_2210_14771_amd import train_scorer

    from gpu_helpers import assert_attempts_equal, assert_results_equal, oracle_params

    torch = torch_dev
    path = os.path.join(train_scorer.MODEL_DIR, train_scorer.MODEL_FILE)
    if not os.path.exists(path):
        pytest.skip("no trained scorer model")
    flat = train_scorer.load_model(path)
    params = [(cnn.bf16(w), b) for w, b in cnn.unflat_params(flat.astype(np.float64))]
    e = api.Estimator(0)
    e.set_model(flat)
    frames, _ = synth.make_batch(synth.HD_1080p, 2)
    dev = torch.from_numpy(frames).cuda()
    uids = [0, 1]
    kw = dict(n_hstrips=32, n_vstrips=32, ransac_attempts=1024)
    say("trained scorer at 1080p: candidates")
    _, pts = e.debug_candidates(dev, api.default_params(**kw, scorer=1), uids)
    res_l, att = e.debug_attempts(dev, api.default_params(**kw, scorer=1), uids)
    res_f = e.estimate_area(dev, api.default_params(**kw, scorer=1, fallback_inlier_frac=0.5),
                            uids)
    torch.cuda.synchronize()
    g = api.points_numpy(pts)
    res_l, res_f = res_l.numpy(), res_f.numpy()
    att = api.attempts_numpy(att)
    tol = 0.01
    op = oracle_params(**kw)
    for f in range(2):
        halves = cnn.learned_half_strip_scores(frames[f], params, 32, 32)
        assert len(halves) == 128
        for c, (xs, ys, sc) in enumerate(halves):
            gx, gy, gs = int(g[f][c]["x"]), int(g[f][c]["y"]), float(g[f][c]["score"])
            idx = np.flatnonzero((xs == gx) & (ys == gy))
            assert idx.size == 1, (f, c, gx, gy)
            assert sc[idx[0]] >= sc.max() - tol, (f, c, sc[idx[0]], sc.max())
            assert abs(gs - sc[idx[0]]) <= tol
        # the learned form keeps points by score alone (no edge-distance filter)
        s32 = g[f]["score"].astype(np.float32)
        keep = s32 >= np.float32(op.t_ps)
        xs = g[f]["x"][keep].astype(np.int32)
        ys = g[f]["y"][keep].astype(np.int32)
        sq = (s32[keep].astype(np.float64) * 2.0 ** 24).astype(np.uint32)
        assert int(res_l[f]["n_points"]) == int(keep.sum())
        say(f"frame {f}: {int(keep.sum())} learned points kept, oracle RANSAC over them")
        ora_att = oracle.ransac_attempts(xs, ys, sq, 1920, 1080, uids[f], op)
        assert_attempts_equal([att[f]], [ora_att])
        n = int(res_l[f]["n_points"])
        if n < 3 or np.float32(res_l[f]["inliers"]) < np.float32(0.5) * np.float32(n):
            want = oracle.estimate(frames[f], op, uids[f]).copy()
            want["reason"] += 256
            say(f"frame {f}: fallback to the handcrafted pipeline")
            assert_results_equal([res_f[f]], [want])
        else:
            assert res_f[f].tobytes() == res_l[f].tobytes()
    e.close()


# ----------------------------------------------------------------- training --
#
# The GPU backward pass stores its signals in bfloat16 and sums in float32;
# the oracle (grad_bf16 mode) applies the same roundings with float64 sums.
# A rounding that falls differently (a float32 sum within rounding distance
# of a bfloat16 tie) changes one stored value by 2^-8 relative; a gradient
# entry sums thousands of such values, so whole-tensor errors stay far below
# that.  Bounds per parameter tensor, relative to the tensor's scale:
GRAD_MAX_REL = 4e-3      # max |gpu - oracle| / max |oracle|
GRAD_NORM_REL = 2e-3     # ||gpu - oracle|| / ||oracle||
LOSS_REL = 1e-5


def _train_case(rng, n):
    win = rng.integers(0, 256, (n, 8, 128, 3), dtype=np.uint8)
    ranges = np.tile(np.array([0, 128], dtype=np.int32), (n, 1))
    if n > 4:
        ranges[1] = (0, 60)
        ranges[2] = (20, 128)
        ranges[3] = (9, 100)
        ranges[4] = (0, 8)       # no central position inside the strip
    targets = rng.uniform(0, 1, (n, 112)).astype(np.float32)
    weights = (rng.uniform(0, 2, (n, 112)) * (rng.uniform(size=(n, 112)) > 0.3)).astype(np.float32)
    return win, ranges, targets, weights


def _oracle_window_grads(win, ranges, targets, weights, params, scale, grad_bf16=True):
    xs, ts, ms, ws = [], [], [], []
    for i in range(len(win)):
        x = (win[i].astype(np.float64) - 128.0) / 64.0
        xs.append(x.transpose(0, 2, 1).reshape(24, 128))
        m = np.zeros(128, dtype=bool)
        m[ranges[i, 0]:ranges[i, 1]] = True
        t = np.zeros(128)
        t[8:120] = targets[i]
        w = np.zeros(128)
        w[8:120] = weights[i]
        ms.append(m)
        ts.append(t)
        ws.append(np.where(m, w, 0.0))
    loss, grads = cnn.loss_and_grads(xs, ts, params, True, ms, ws, scale, grad_bf16)
    return loss, cnn.flat_params(grads)


def _param_slices():
    out, at = [], 0
    for li, (ci, co, k) in enumerate(cnn.LAYERS):
        out.append((f"W{li + 1}", slice(at, at + co * ci * k)))
        at += co * ci * k
        out.append((f"b{li + 1}", slice(at, at + co)))
        at += co
    return out


def _spread_params(seed):
    rng = np.random.default_rng(seed + 100)
    return [(w, (b + rng.normal(0, 0.1, b.shape)).astype(np.float32).astype(np.float64))
            for w, b in cnn.init_params(seed)]


@pytest.mark.parametrize("seed,n", [(0, 37), (1, 600)])
def test_gradients_match_oracle(torch_dev, est, seed, n):
    """n = 600 exceeds the gradient grid: workgroups accumulate several windows."""
    torch = torch_dev
    rng = np.random.default_rng(seed)
    params = _spread_params(seed)
    est.set_model(cnn.flat_params(params))
    win, ranges, targets, weights = _train_case(rng, n)
    scale = float(np.float32(1.0 / max(weights.sum(), 1.0)))
    say(f"gradients seed {seed} n {n}")
    grad, loss = est.cnn_gradients(torch.from_numpy(win).cuda(), torch.from_numpy(ranges).cuda(),
                                   torch.from_numpy(targets).cuda(),
                                   torch.from_numpy(weights).cuda(), scale)
    torch.cuda.synchronize()
    g = grad.cpu().numpy().astype(np.float64)
    ref_loss, ref = _oracle_window_grads(win, ranges, targets, weights, params, scale)
    assert abs(loss.item() - ref_loss) <= LOSS_REL * abs(ref_loss)
    for name, sl in _param_slices():
        d = g[sl] - ref[sl]
        scale_t = np.abs(ref[sl]).max()
        assert scale_t > 0, name
        assert np.abs(d).max() <= GRAD_MAX_REL * scale_t, (name, np.abs(d).max() / scale_t)
        assert np.linalg.norm(d) <= GRAD_NORM_REL * np.linalg.norm(ref[sl]), name
    # the bfloat16 backward signals stay close to the exact chain rule
    _, exact = _oracle_window_grads(win, ranges, targets, weights, params, scale, False)
    cos = g @ exact / (np.linalg.norm(g) * np.linalg.norm(exact))
    assert cos > 0.9999


def test_gradients_of_no_windows_are_zero(torch_dev, est):
    torch = torch_dev
    est.set_model(cnn.flat_params(_spread_params(2)))
    e8 = torch.empty((0, 8, 128, 3), dtype=torch.uint8, device="cuda")
    e2 = torch.empty((0, 2), dtype=torch.int32, device="cuda")
    ef = torch.empty((0, 112), dtype=torch.float32, device="cuda")
    grad, loss = est.cnn_gradients(e8, e2, ef, ef, 1.0)
    torch.cuda.synchronize()
    assert not grad.cpu().numpy().any() and loss.item() == 0.0


def test_sgd_step_updates_master_and_model(torch_dev, est):
    """Two momentum steps are bit-exact float32 arithmetic; the rebuilt
    device model scores windows like the oracle with the new weights."""
    torch = torch_dev
    rng = np.random.default_rng(5)
    params = _spread_params(3)
    p0 = cnn.flat_params(params).astype(np.float32)
    est.set_model(p0)
    g = (rng.standard_normal(p0.size) * 0.01).astype(np.float32)
    gd = torch.from_numpy(g).cuda()
    lr, mu = np.float32(0.5), np.float32(0.9)
    est.cnn_sgd_step(gd, float(lr), float(mu))
    est.cnn_sgd_step(gd, float(lr), float(mu))
    p, m = est.get_model(with_momentum=True)
    m1 = mu * np.zeros_like(g) + g
    p1 = p0 - lr * m1
    m2 = mu * m1 + g
    p2 = p1 - lr * m2
    np.testing.assert_array_equal(m, m2)
    np.testing.assert_array_equal(p, p2)
    new = cnn.unflat_params(p.astype(np.float64))
    new = [(cnn.bf16(w), b) for w, b in new[:-1]] + [(cnn.bf16(new[-1][0]), new[-1][1])]
    win, ranges = _random_windows(rng, 4)
    z = est.cnn_window_logits(torch.from_numpy(win).cuda(), torch.from_numpy(ranges).cuda())
    torch.cuda.synchronize()
    z = z.cpu().numpy()
    for i in range(len(win)):
        ref = cnn.window_forward(win[i], int(ranges[i, 0]), int(ranges[i, 1]), new)
        ok = ~np.isnan(ref)
        assert np.abs(z[i][ok] - ref[ok]).max() <= LOGIT_TOL


def test_training_resumes_from_checkpoint(torch_dev):
    """Three steps in one go equal one step, a checkpoint (master weights and
    momentum) restored into a fresh context, and two more steps."""
    torch = torch_dev
    rng = np.random.default_rng(6)
    win, ranges, targets, weights = _train_case(rng, 50)
    dev = [torch.from_numpy(a).cuda() for a in (win, ranges, targets, weights)]
    scale = float(np.float32(1.0 / weights.sum()))
    p0 = cnn.flat_params(_spread_params(4)).astype(np.float32)

    def steps(e, k):
        for _ in range(k):
            grad, _ = e.cnn_gradients(*dev, scale)
            e.cnn_sgd_step(grad, 0.05, 0.9)
        torch.cuda.synchronize()

    a = api.Estimator(0)
    a.set_model(p0)
    steps(a, 3)
    pa = a.get_model()
    a.close()
    b = api.Estimator(0)
    b.set_model(p0)
    steps(b, 1)
    ck_p, ck_m = b.get_model(with_momentum=True)
    b.close()
    c = api.Estimator(0)
    c.set_model(ck_p)
    c.set_momentum(ck_m)
    steps(c, 2)
    pc = c.get_model()
    c.close()
    np.testing.assert_array_equal(pa, pc)
    assert not np.array_equal(pa, p0)
