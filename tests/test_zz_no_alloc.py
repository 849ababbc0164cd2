"""The entry point without device allocation (ca_estimate_area_noalloc),
through the C ABI: its results equal ca_estimate_area's bit for bit on two
calls in a row (the second with a smaller batch of another shape, so the
shared scratch holds the first call's contents when the second starts), on
a batch of mixed shapes, and with the learned scorer and its fallback; a
batch beyond the scratch's limits is refused before anything runs."""
import os

import numpy as np
import pytest

from paper_2210_14771_amd import _native as N
from paper_2210_14771_amd import api, synth, train_scorer

from gpu_helpers import say

pytestmark = pytest.mark.gpu

HD = dict(n_hstrips=32, n_vstrips=32, ransac_attempts=1024)
SMALL = dict(n_hstrips=16, n_vstrips=16, ransac_attempts=256)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _raw(torch, res):
    torch.cuda.synchronize()
    return res.raw.cpu().numpy()


@pytest.mark.parametrize("schedule", ["split", "fused"])
def test_two_calls_in_a_row_equal_the_allocating_entry_point(torch_dev, schedule):
    torch = torch_dev
    hd, _ = synth.make_batch(synth.HD_1080p, 16)
    small, _ = synth.make_batch(synth.SMALL_640x480, 5)
    hd_dev = torch.from_numpy(hd).cuda()
    small_dev = torch.from_numpy(small).cuda()
    est = api.Estimator(0)
    est.set_option("schedule", schedule)
    say(f"noalloc {schedule}: 16 x 1080p, then 5 x 640x480")
    a1 = _raw(torch, est.estimate_area_noalloc(hd_dev, HD, list(range(100, 116))))
    a2 = _raw(torch, est.estimate_area_noalloc(small_dev, SMALL, list(range(5))))
    r1 = _raw(torch, est.estimate_area(hd_dev, HD, list(range(100, 116))))
    r2 = _raw(torch, est.estimate_area(small_dev, SMALL, list(range(5))))
    np.testing.assert_array_equal(a1, r1)
    np.testing.assert_array_equal(a2, r2)
    # back to the larger call: nothing of the smaller one leaks into it
    a3 = _raw(torch, est.estimate_area_noalloc(hd_dev, HD, list(range(100, 116))))
    np.testing.assert_array_equal(a3, r1)
    est.device_status()
    est.close()


def test_mixed_shapes_in_one_call(torch_dev):
    torch = torch_dev
    views = []
    for i, (w, h) in enumerate([(720, 576), (1280, 720), (1920, 1080), (720, 576), (3840, 2160)]):
        f, _ = synth.make_frame(synth.HD_1080p, 400 + i, w, h)
        views.append(torch.from_numpy(f).cuda())
    est = api.Estimator(0)
    uids = list(range(400, 405))
    say("noalloc: five frames of four shapes")
    a = _raw(torch, est.estimate_area_noalloc(views, HD, uids))
    r = _raw(torch, est.estimate_area(views, HD, uids))
    np.testing.assert_array_equal(a, r)
    est.close()


def test_learned_scorer_with_fallback(torch_dev):
    torch = torch_dev
    path = os.path.join(train_scorer.MODEL_DIR, train_scorer.MODEL_FILE)
    if not os.path.exists(path):
        pytest.skip("no trained scorer model")
    frames, _ = synth.make_batch(synth.HD_1080p, 8)
    dev = torch.from_numpy(frames).cuda()
    est = api.Estimator(0)
    est.set_model(train_scorer.load_model(path))
    p = api.default_params(**HD, scorer=1, fallback_inlier_frac=0.5)
    say("noalloc: learned scorer with fallback, 8 x 1080p")
    a = _raw(torch, est.estimate_area_noalloc(dev, p, list(range(8))))
    r = _raw(torch, est.estimate_area(dev, p, list(range(8))))
    np.testing.assert_array_equal(a, r)
    est.close()


def test_limits_are_refused_before_any_work(torch_dev):
    torch = torch_dev
    est = api.Estimator(0)
    one = torch.zeros((1, 32, 32, 3), dtype=torch.uint8, device="cuda")
    out = torch.zeros((N.CA_NOALLOC_MAX_FRAMES + 1, 8), dtype=torch.int32, device="cuda")
    # more frames than the scratch holds: every descriptor points at one frame
    many = one.expand(N.CA_NOALLOC_MAX_FRAMES + 1, 32, 32, 3)
    with pytest.raises(RuntimeError, match="scratch"):
        est.estimate_area_noalloc(list(many), SMALL, out=out)
    # more distinct frame shapes than it holds strip tables for
    shapes = [torch.zeros((16 + k, 16, 3), dtype=torch.uint8, device="cuda")
              for k in range(N.CA_NOALLOC_MAX_SHAPES + 1)]
    with pytest.raises(RuntimeError, match="scratch"):
        est.estimate_area_noalloc(shapes, SMALL, out=out)
    torch.cuda.synchronize()
    assert not out.cpu().numpy().any()
    est.close()
