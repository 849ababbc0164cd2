"""Host-side pieces of the next rows, on the CPU: the uneven batch's shape
mix, hard-frame distractors, device-renderer recipes, the training set's
window tiling and labels, the scorer's initialisation and the serving
simulation's arrivals.  (Input generators and plumbing: none of this is the
estimator's arithmetic.)"""
import math
from collections import Counter

import numpy as np
import pytest

from oracle import cnn
from paper_2210_14771_amd import serve, synth, synth_gpu, train_scorer


def test_mixed_batch_shapes_follow_the_ratio():
    shapes = synth.mixed_shapes(512)
    c = Counter(shapes)
    assert c[(720, 576)] == 102 and c[(1280, 720)] == 154
    assert c[(1920, 1080)] == 205 and c[(3840, 2160)] == 51
    # interleaved, reproducible
    assert shapes == synth.mixed_shapes(512)
    assert len({shapes[i] for i in range(16)}) > 1
    assert Counter(synth.mixed_shapes(10)) == Counter({(1920, 1080): 4, (1280, 720): 3,
                                                       (720, 576): 2, (3840, 2160): 1})


def test_hard_distractors_stay_in_the_border():
    wl = synth.HARD_1080p
    n_text = n_blob = 0
    for i in range(40):
        rng = synth.frame_rng(wl.config_id, i)
        spec = synth.draw_spec(rng, wl.width, wl.height, wl.mix, wl.border_sigma,
                               wl.blur_sigma, wl.vignette, wl.radius_frac)
        ex = synth.draw_hard(rng, spec)
        if not spec.has_border:
            assert ex.edge_step == 0 and not ex.blobs and ex.text_scale == 0
            continue
        assert 10.0 <= ex.edge_step <= 25.0
        for x, y, rad, amp in ex.blobs:
            n_blob += 1
            assert math.hypot(x - spec.cx, y - spec.cy) > spec.r + 2 * rad
            assert 3 <= rad <= 15 and 120 <= amp <= 250
        if ex.text_scale:
            n_text += 1
            bw = ex.text_chars * (synth.GLYPH_W + 1) * ex.text_scale
            bh = ex.text_lines * (synth.GLYPH_H + 2) * ex.text_scale
            for x, y in ((ex.text_x, ex.text_y), (ex.text_x + bw, ex.text_y),
                         (ex.text_x, ex.text_y + bh), (ex.text_x + bw, ex.text_y + bh)):
                assert 0 <= x < spec.width and 0 <= y < spec.height
                assert math.hypot(x - spec.cx, y - spec.cy) > spec.r
            assert ex.glyphs.size == ex.text_lines * ex.text_chars
            assert int(ex.glyphs.max()) < (1 << (synth.GLYPH_W * synth.GLYPH_H))
    assert n_text > 5 and n_blob > 5


def test_recipes_pack_consistently():
    recs = [synth_gpu.draw_recipe(synth.HARD_1080p, 7, i, True) for i in range(6)]
    rec, grids, glyphs, total = synth_gpu.pack(recs)
    assert rec.dtype.itemsize == 192 and len(rec) == 6
    assert total == sum(3 * r.spec.width * r.spec.height for r in recs)
    for i, r in enumerate(recs):
        base, fine, chroma, tint = r.grids
        o = int(rec[i]["grid_off"])
        n0, n1 = base.size, fine.size
        np.testing.assert_array_equal(grids[o:o + n0], base.ravel())
        np.testing.assert_array_equal(grids[o + n0:o + n0 + n1], fine.ravel())
        np.testing.assert_array_equal(grids[o + n0 + n1 + 2 * n0:o + n0 + n1 + 3 * n0],
                                      chroma[2].ravel())
        if r.extras.text_scale:
            g = int(rec[i]["glyph_off"])
            np.testing.assert_array_equal(glyphs[g:g + r.extras.glyphs.size], r.extras.glyphs)
        assert int(rec[i]["n_blobs"]) == len(r.extras.blobs) <= 4
    # the same recipe twice is the same frame description
    again = synth_gpu.draw_recipe(synth.HARD_1080p, 7, 3, True)
    assert again.key == recs[3].key and again.spec == recs[3].spec


@pytest.mark.parametrize("length", [16, 111, 112, 113, 1080, 1920, 3840])
def test_strip_windows_cover_each_position_once(length):
    desc = synth_gpu.strip_windows(2, True, 5, length)
    cover = np.zeros(length, dtype=int)
    for f, hz, line, start in desc:
        assert (f, hz, line) == (2, 1, 5)
        p = np.arange(start + 8, start + 120)
        cover[p[(p >= 0) & (p < length)]] += 1
    assert np.all(cover == 1)


def test_positions_inside_counts_the_loss_positions():
    recs = [synth_gpu.draw_recipe(synth.HD_1080p, 100, i, False) for i in range(2)]
    desc = np.concatenate([synth_gpu.strip_windows(0, True, 10, 1920),
                           synth_gpu.strip_windows(1, False, 10, 1080)])
    assert train_scorer.positions_inside(desc, recs) == 1920 + 1080


def test_initial_scorer_scale_and_bias():
    p = train_scorer.init_params(0)
    assert p.dtype == np.float32 and p.size == cnn.n_params()
    layers = cnn.unflat_params(p.astype(np.float64))
    for (ci, co, k), (w, b) in zip(cnn.LAYERS[:-1], layers[:-1]):
        bound = 1.0 / math.sqrt(ci * k)
        assert np.abs(w).max() <= bound and np.abs(b).max() <= bound
    assert layers[-1][1][0] == -4.0
    assert not np.array_equal(p, train_scorer.init_params(1))


def test_trained_model_file_is_a_model():
    p = train_scorer.load_model()
    assert p.shape == (cnn.n_params(),) and np.all(np.isfinite(p))


def test_serving_arrivals_are_poisson_like():
    rng = np.random.default_rng(0)
    fps = 45.0
    t, gaps = 0.0, []
    for _ in range(20000):
        g = float(rng.exponential(1.0 / fps))
        gaps.append(g)
        t += g
    gaps = np.array(gaps)
    # exponential gaps: mean 1/fps, standard deviation 1/fps
    assert abs(gaps.mean() * fps - 1.0) < 0.03 and abs(gaps.std() * fps - 1.0) < 0.03


def test_drifting_circle_steps():
    rng = np.random.default_rng(3)
    recs = serve.drifting_recipes(4, 1920, 1080, 200, rng)
    cx = np.array([r.spec.cx for r in recs])
    r = np.array([r.spec.r for r in recs])
    steps = np.diff(cx)
    assert 0.35 < steps.std() < 0.65                      # random walk, sigma 0.5 px
    jumps = np.abs(np.diff(r) / r[:-1])
    assert np.all((jumps < 1e-12) | (np.abs(jumps - 0.1) < 0.02) | (np.abs(jumps - 1 / 11) < 0.02))
    assert all(rr.grids is recs[0].grids for rr in recs)   # the same tissue
    assert len({rr.key for rr in recs}) == len(recs)       # fresh noise


def test_serving_accuracy_is_sampled_with_progress():
    """The serving benchmark evaluates accuracy on an evenly spaced sample of
    the served frames and logs every block of frames, so the host-side
    evaluation after a serving run never goes silent for long; the sample's
    errors are those of a direct evaluation of the same frames."""
    from paper_2210_14771_amd import evaluate, serve_bench

    rng = np.random.default_rng(7)
    streams, served = [], []
    for sid, (w, h) in enumerate(((96, 64), (128, 72), (80, 80))):
        recs = serve.drifting_recipes(sid, w, h, 4, rng)
        streams.append(serve.SimStream(sid, w, h, 30.0, [None] * 4, [r.spec for r in recs],
                                       np.zeros(0)))
        for seq in range(25):
            spec = recs[seq % 4].spec
            valid = int(seq % 3 != 0)
            res = (spec.cx + rng.normal(0, 2), spec.cy + rng.normal(0, 2), spec.r * 0.97, 0.5,
                   10, 20, valid, 0 if valid else 2)
            filt = (1, spec.cx + 1.0, spec.cy, spec.r + 0.5, 2.0)
            served.append({"stream": sid, "seq": seq, "result": res, "filtered": filt})
    rng.shuffle(served)
    sample = serve_bench.accuracy_sample(served, 20)
    keys = [(r["stream"], r["seq"]) for r in sample]
    assert len(sample) == 20 and keys == sorted(keys) and len(set(keys)) == 20
    assert keys[0] == (0, 0) and keys[-1] == (2, 24)            # both ends of the order
    assert serve_bench.accuracy_sample(served, 500) == sorted(
        served, key=lambda r: (r["stream"], r["seq"]))
    lines = []
    acc = serve_bench.accuracy(sample, streams, lines.append, block=6)
    assert len(lines) == 2 * 4                                   # ceil(20 / 6) per kind
    assert lines[3] == "accuracy (frame): 20 of 20 frames"
    specs = [streams[r["stream"]].specs[r["seq"] % 4] for r in sample]
    a = np.array([r["result"] for r in sample], dtype=np.float64)
    e = evaluate.frame_errors(specs, a[:, 0], a[:, 1], a[:, 2], a[:, 6] != 0)
    assert acc["frame"] == evaluate.summarise(e)
