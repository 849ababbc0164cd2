"""Uneven batches: 512 frames of 720x576, 1280x720, 1920x1080 and 3840x2160
in ratio 2:3:4:1 in one captured HIP graph, with autotuned strip tiles.
Every frame of the graph's output, under the split and the persistent
schedule, matches the oracle (results exact, circles within 1e-3 px), and
every frame's candidates match it bit for bit under each strip tile."""
import numpy as np
import pytest

from paper_2210_14771_amd import api, synth

from gpu_helpers import assert_points_equal, assert_results_equal, run_oracle, say

pytestmark = pytest.mark.gpu

N = 512
KW = dict(n_hstrips=32, n_vstrips=32, ransac_attempts=1024)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def batch(torch_dev):
    torch = torch_dev
    say(f"rendering {N} mixed-resolution frames")
    frames, specs = synth.make_mixed_batch(N, threads=16)
    sizes = [f.nbytes for f in frames]
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    flat = torch.empty(int(sum(sizes)), dtype=torch.uint8, device="cuda")
    views = []
    for f, o, nb in zip(frames, offs, sizes):
        v = flat[int(o):int(o) + nb].view(f.shape)
        v.copy_(torch.from_numpy(f))
        views.append(v)
    torch.cuda.synchronize()
    say("frames resident")
    return frames, specs, views


@pytest.fixture(scope="module")
def oracle_out(batch):
    frames, _, _ = batch
    say(f"oracle on all {N} frames")
    res, pts, _ = run_oracle(frames, KW, list(range(N)), threads=16)
    return res, pts


def _raw(res):
    import torch
    torch.cuda.synchronize()
    return res.raw.cpu().numpy()


def _as_results(raw):
    return raw.view(api.RESULT_DTYPE).reshape(-1)


def test_graph_with_autotuned_tiles_matches_oracle(torch_dev, batch, oracle_out):
    torch = torch_dev
    frames, specs, views = batch
    ores, opts = oracle_out
    est = api.Estimator(0)
    params = api.default_params(**KW)
    uids = list(range(N))
    est.set_option("strips_per_group", 1)
    ref = _raw(est.estimate_area(views, params, uids))
    assert_results_equal(_as_results(ref), ores)
    _, ref_pts = est.debug_candidates(views, params, uids)
    ref_pts = ref_pts.cpu().numpy()
    assert_points_equal(api.points_numpy(torch.from_numpy(ref_pts)), opts)
    est.set_option("strips_per_group", 0)
    say("autotuning")
    tuned = est.autotune(views, params, uids, reps=3)
    say(f"tuned strip items per workgroup: {tuned}, schedule {est.last_tuned_schedule}, "
        f"sub-batches {est.last_tuned_pipeline}")
    assert est.last_tuned_schedule in ("split", "fused")
    assert est.last_tuned_pipeline in ((1, 2, 4) if est.last_tuned_schedule == "split" else (None,))
    assert est.get_option("schedule") == 2            # auto: the graph takes the tuned one
    assert set(tuned) == {(w, h) for w, h, _ in synth.MIXED_SHAPES}
    assert all(t in (1, 2, 4, 8) for t in tuned.values())
    out = torch.empty((N, 8), dtype=torch.int32, device="cuda")
    # the tuned configuration (schedule and sub-batches), the split schedule
    # with the tuned tiles (one strip launch per frame shape), then the
    # persistent one (one kernel drawing strip and RANSAC work items from
    # per-XCD queues), each captured as one graph
    for sched in ("auto", "split", "fused"):
        est.set_option("schedule", sched)
        g = est.capture(views, params, uids, out=out)
        for rep in range(2):
            out.zero_()
            g.launch()
            got = _raw(api.Result(out))
            say(f"{sched} replay {rep}: all {N} frames against the oracle")
            assert_results_equal(_as_results(got), ores)
            np.testing.assert_array_equal(got, ref, err_msg=f"{sched} replay {rep}")
        g.close()
    est.device_status()        # raises if a wait hit its guard
    est.set_option("schedule", "split")
    # every forced tile gives the oracle's candidates
    for t in (2, 8):
        est.set_option("strips_per_group", t)
        _, pts = est.debug_candidates(views, params, uids)
        np.testing.assert_array_equal(pts.cpu().numpy(), ref_pts, err_msg=f"tile {t}")
    est.close()
