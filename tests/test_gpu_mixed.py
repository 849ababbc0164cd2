"""Uneven batches: 512 frames of 720x576, 1280x720, 1920x1080 and 3840x2160
in ratio 2:3:4:1 in one captured HIP graph, with autotuned strip tiles.
Results must not depend on the tile (bit-exact against one strip item per
workgroup), and sampled frames match the oracle one by one."""
import numpy as np
import pytest

from paper_2210_14771_amd import api, synth

from gpu_helpers import assert_points_equal, assert_results_equal, run_gpu, run_oracle, say

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


def _raw(res):
    import torch
    torch.cuda.synchronize()
    return res.raw.cpu().numpy()


def test_graph_with_autotuned_tiles_equals_single_item_tiles(torch_dev, batch):
    torch = torch_dev
    frames, specs, views = batch
    est = api.Estimator(0)
    params = api.default_params(**KW)
    uids = list(range(N))
    est.set_option("strips_per_group", 1)
    ref = _raw(est.estimate_area(views, params, uids))
    _, ref_pts = est.debug_candidates(views, params, uids)
    ref_pts = ref_pts.cpu().numpy()
    est.set_option("strips_per_group", 0)
    say("autotuning")
    tuned = est.autotune(views, params, uids, reps=3)
    say(f"tuned strip items per workgroup: {tuned}, schedule {est.last_tuned_schedule}")
    assert est.last_tuned_schedule in ("split", "fused")
    assert est.get_option("schedule") == 2            # auto: the graph takes the tuned one
    assert set(tuned) == {(w, h) for w, h, _ in synth.MIXED_SHAPES}
    assert all(t in (1, 2, 4, 8) for t in tuned.values())
    out = torch.empty((N, 8), dtype=torch.int32, device="cuda")
    g = est.capture(views, params, uids, out=out)
    for rep in range(3):
        out.zero_()
        g.launch()
        np.testing.assert_array_equal(_raw(api.Result(out)), ref, err_msg=f"replay {rep}")
    g.close()
    # the persistent schedule (one kernel drawing strip and RANSAC work
    # items from per-XCD queues), captured the same way
    est.set_option("schedule", "fused")
    g = est.capture(views, params, uids, out=out)
    for rep in range(2):
        out.zero_()
        g.launch()
        np.testing.assert_array_equal(_raw(api.Result(out)), ref, err_msg=f"fused replay {rep}")
    g.close()
    est.device_status()        # raises if a wait hit its guard
    est.set_option("schedule", "split")
    # every forced tile gives the same candidates
    for t in (2, 8):
        est.set_option("strips_per_group", t)
        _, pts = est.debug_candidates(views, params, uids)
        np.testing.assert_array_equal(pts.cpu().numpy(), ref_pts, err_msg=f"tile {t}")
    est.close()


def test_sampled_frames_match_oracle(torch_dev, batch):
    """Two frames of each resolution, from the 512-frame launch with tuned
    tiles: candidates bit-exact, results exact (circles within 1e-3 px)."""
    frames, specs, views = batch
    est = api.Estimator(0)
    uids = list(range(N))
    est.autotune(views, api.default_params(**KW), uids, reps=1)
    got = run_gpu(est, views, KW, uids, what=("pts",))
    shapes = synth.mixed_shapes(N)
    picks = []
    for w, h, _ in synth.MIXED_SHAPES:
        picks += [i for i in range(N) if shapes[i] == (w, h)][:2]
    say(f"oracle on frames {picks}")
    ores, opts, _ = run_oracle([frames[i] for i in picks], KW, picks, threads=8)
    assert_points_equal([got["pts"][i] for i in picks], opts)
    assert_results_equal([got["res"][i] for i in picks], ores)
    est.close()
