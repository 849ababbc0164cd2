"""Several batches in flight: independent contexts, each with its own plan
buffers, output and HIP stream, running the path concurrently on one GPU
(eager calls and captured graphs, taking turns; the handcrafted scorer under
both schedules and the learned scorer with its fallback) give bit-identical
results to one context running alone, on every call."""
import numpy as np
import pytest

from paper_2210_14771_amd import api, synth, train_scorer

from gpu_helpers import say

pytestmark = pytest.mark.gpu

KW = dict(n_hstrips=32, n_vstrips=32, ransac_attempts=1024)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _estimator(schedule, learned):
    e = api.Estimator(0)
    e.set_option("schedule", "split" if learned else schedule)
    if learned:
        e.set_model(train_scorer.load_model())
    return e


@pytest.mark.parametrize("schedule", ["split", "fused", "learned"])
def test_four_contexts_four_streams(torch_dev, schedule):
    torch = torch_dev
    learned = schedule == "learned"
    frames, _ = synth.make_batch(synth.SMALL_640x480, 8)
    batches = [torch.from_numpy(frames).cuda(),
               torch.from_numpy(np.ascontiguousarray(frames[:, ::-1])).cuda()]
    # the learned scorer with the handcrafted fallback: both paths per call
    params = (api.default_params(**KW, scorer=1, fallback_inlier_frac=0.5) if learned
              else api.default_params(**KW))
    uids = list(range(len(frames)))
    say(f"in flight: {schedule}")
    ref_est = _estimator(schedule, learned)
    refs = [ref_est.estimate_area(b, params, uids).raw.cpu() for b in batches]
    ref_est.close()
    n = 4
    ests = [_estimator(schedule, learned) for _ in range(n)]
    streams = [torch.cuda.Stream() for _ in range(n)]
    # eager: n x 6 calls taking turns over the contexts, each into its own output
    outs = [[torch.empty((len(frames), 8), dtype=torch.int32, device="cuda") for _ in range(6)]
            for _ in range(n)]
    torch.cuda.synchronize()
    for i in range(6):
        for k in range(n):
            ests[k].estimate_area(batches[(i + k) % 2], params, uids, out=outs[k][i],
                                  stream=streams[k])
    torch.cuda.synchronize()
    for i in range(6):
        for k in range(n):
            assert torch.equal(outs[k][i].cpu(), refs[(i + k) % 2]), (i, k)
    # graphs: each context replays its own graph on its own stream
    gouts = [torch.empty((len(frames), 8), dtype=torch.int32, device="cuda") for _ in range(n)]
    graphs = [ests[k].capture(batches[k % 2], params, uids, out=gouts[k], calls=3)
              for k in range(n)]
    for rep in range(3):
        for o in gouts:
            o.zero_()
        for k in range(n):
            graphs[k].launch(streams[k])
        torch.cuda.synchronize()
        for k in range(n):
            assert torch.equal(gouts[k].cpu(), refs[k % 2]), (rep, k)
    for g in graphs:
        g.close()
    for e in ests:
        e.device_status()
        e.close()
