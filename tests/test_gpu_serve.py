"""The serving loop: continuous batching of simulated video streams.  Every
frame's result equals the batch API's and the oracle's result for the same
frame and uid, whether the stream is served alone or among 47 others; the per-stream
temporal filter follows its definition; streams wait for memory and are
admitted as others close."""
import json
import os

import numpy as np
import pytest

from paper_2210_14771_amd import api, serve, train_scorer

from gpu_helpers import say

pytestmark = pytest.mark.gpu

KW = dict(n_hstrips=32, n_vstrips=32, ransac_attempts=1024)
MODEL = os.path.join(train_scorer.MODEL_DIR, train_scorer.MODEL_FILE)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def streams(torch_dev):
    say("rendering 48 streams")
    return serve.make_streams(48, frames_per_stream=6, duration_s=0.4, seed=1)


def _key(rec):
    return rec["stream"], rec["seq"]


def test_results_identical_alone_and_in_the_mix(torch_dev, streams):
    est = api.Estimator(0)
    srv = serve.Server(est, serve.server_config(max_batch=64, **KW))
    mix, wall = serve.run(srv, streams)
    srv.close()
    report = {"plain": serve.latency_summary(mix, wall)}
    say(f"mix: {report['plain']}")
    n_expected = sum(len(s.arrivals) for s in streams)
    assert len(mix) == n_expected
    assert max(r["batch"] for r in mix) > 1          # batches did form
    # the same arrivals served with the learned scorer (handcrafted fallback)
    if os.path.exists(MODEL):
        est.set_model(train_scorer.load_model())
        srv = serve.Server(est, serve.server_config(max_batch=64, scorer=1,
                                                    fallback_inlier_frac=0.5, **KW))
        learned, lwall = serve.run(srv, streams)
        srv.close()
        assert len(learned) == n_expected
        report["learned"] = serve.latency_summary(learned, lwall)
        say(f"learned: {report['learned']}")
    if os.environ.get("CA_SERVE_REPORT"):
        with open(os.environ["CA_SERVE_REPORT"], "w") as f:
            json.dump(dict(report, streams=len(streams),
                           arrival_fps=n_expected / 0.4), f, indent=1)
    by = {_key(r): r for r in mix}
    for sid in (0, 1, 2, 5):                          # 720p, 1080p, 4K, 4K
        srv = serve.Server(est, serve.server_config(max_batch=64, **KW))
        alone, _ = serve.run(srv, streams, only={sid})
        srv.close()
        assert len(alone) == len(streams[sid].arrivals)
        for r in alone:
            m = by[_key(r)]
            assert r["result"] == m["result"], (sid, r["seq"])
            assert r["filtered"] == m["filtered"], (sid, r["seq"])
    est.close()


def test_each_result_equals_the_batch_api_and_the_oracle(torch_dev, streams):
    """Every served frame: the batch API's result for the same frame and uid,
    and the oracle's (counts exact, circle within 1e-3 px)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    from gpu_helpers import assert_results_equal, oracle_params

    torch = torch_dev
    est = api.Estimator(0)
    srv = serve.Server(est, serve.server_config(max_batch=32, **KW))
    got, _ = serve.run(srv, streams[:6], realtime=False)
    srv.close()
    host = {}
    for r in got:
        st = streams[r["stream"]]
        frame = st.frames[r["seq"] % len(st.frames)]
        uid = (r["stream"] << 32) | r["seq"]
        res = est.estimate_area(frame, api.default_params(**KW), [uid])
        torch.cuda.synchronize()
        raw = res.raw.cpu().numpy()[0]
        want = tuple(raw[:4].view(np.float32)) + tuple(int(v) for v in raw[4:])
        assert r["result"] == want, (r["stream"], r["seq"])
        host[_key(r)] = (frame.cpu().numpy(), uid)
    est.close()
    op = oracle_params(**KW)
    keys = sorted(host)
    say(f"oracle on {len(keys)} served frames")
    with ThreadPoolExecutor(16) as ex:
        ora = list(ex.map(lambda k: oracle.estimate(host[k][0], op, host[k][1]), keys))
    by = {_key(r): r for r in got}
    gpu = np.zeros(len(keys), dtype=api.RESULT_DTYPE)
    for i, k in enumerate(keys):
        gpu[i] = by[k]["result"]
    assert_results_equal(gpu, ora)


def test_temporal_filter_follows_its_definition(torch_dev, streams):
    est = api.Estimator(0)
    decay = np.float32(0.8)
    srv = serve.Server(est, serve.server_config(max_batch=16, smooth=float(decay), **KW))
    got, _ = serve.run(srv, streams[:3], realtime=False)
    srv.close()
    for sid in range(3):
        recs = sorted((r for r in got if r["stream"] == sid), key=lambda r: r["seq"])
        x = y = rr = w = np.float32(0.0)
        for r in recs:
            cx, cy, rad, score, _, _, valid, _ = r["result"]
            wd = decay * w
            if valid and score > 0:
                s = np.float32(score)
                wn = wd + s
                x = (wd * x + s * np.float32(cx)) / wn
                y = (wd * y + s * np.float32(cy)) / wn
                rr = (wd * rr + s * np.float32(rad)) / wn
                w = wn
            else:
                w = wd
            fv, fx, fy, fr, fw = r["filtered"]
            assert (fx, fy, fr, fw) == (x, y, rr, w), (sid, r["seq"])
            assert fv == (1 if w > 0 else 0)
    est.close()


def test_streams_wait_for_memory(torch_dev, streams):
    est = api.Estimator(0)
    st = streams[1]                                    # 1080p
    ring = 2 * ((3 * st.width * st.height + 255) // 256 * 256)
    srv = serve.Server(est, serve.server_config(hbm_budget=2 * ring, max_batch=8, **KW))
    ids = [1, 4, 7, 10]                               # four 1080p streams
    adm = [srv.open(i, st.width, st.height) for i in ids]
    assert adm == [True, True, False, False]
    for i in ids:
        for k in range(3):
            srv.submit(i, k, streams[i].frames[k])
    served = []
    for _ in range(100000):
        served += [serve.served_record(s) for s in srv.step()]
        if sum(1 for r in served if r["stream"] in ids[:2]) == 6:
            break
    assert srv.stats()["streams_waiting"] == 2
    assert all(r["stream"] in ids[:2] for r in served)
    srv.close_stream(1)
    srv.close_stream(4)
    for _ in range(100000):
        served += [serve.served_record(s) for s in srv.step()]
        if len(served) == 12:
            break
    assert len(served) == 12
    st_ = srv.stats()
    assert st_["streams_waiting"] == 0 and st_["streams_admitted"] == 2
    srv.close()
    est.close()


def test_strided_and_contiguous_frames_in_one_backlog(torch_dev, streams):
    """Frames with padded rows (views into wider images) and contiguous ones
    submitted together as a backlog: the step's batched copy into ring slots
    takes the byte path for the first and the 16-byte path for the second;
    every result equals the batch API's on the same frame and uid."""
    torch = torch_dev
    est = api.Estimator(0)
    srv = serve.Server(est, serve.server_config(max_batch=16, **KW))
    src = [streams[0], streams[1]]                     # 720p and 1080p
    ids = [100, 101, 102, 103]
    frames = {}
    for k, sid in enumerate(ids):
        st = src[k % 2]
        base = st.frames[0]
        if k < 2:                                      # padded rows: a view into a wider image
            wide = torch.zeros((st.height, st.width + 7, 3), dtype=torch.uint8, device="cuda")
            wide[:, :st.width].copy_(base)
            f = wide[:, :st.width]
            assert f.stride(0) == 3 * (st.width + 7)
        else:
            f = base
        frames[sid] = (f, st)
        assert srv.open(sid, st.width, st.height)
    torch.cuda.synchronize()
    for seq in range(3):
        for sid in ids:
            srv.submit(sid, seq, frames[sid][0])
    served = []
    for _ in range(100000):
        served += [serve.served_record(s) for s in srv.step()]
        if len(served) == 3 * len(ids):
            break
    assert len(served) == 3 * len(ids)
    assert max(r["batch"] for r in served) > 1          # several frames per step
    for r in served:
        f, _ = frames[r["stream"]]
        uid = (r["stream"] << 32) | r["seq"]
        res = est.estimate_area(f, api.default_params(**KW), [uid])
        torch.cuda.synchronize()
        raw = res.raw.cpu().numpy()[0]
        want = tuple(raw[:4].view(np.float32)) + tuple(int(v) for v in raw[4:])
        assert r["result"] == want, (r["stream"], r["seq"])
    srv.close()
    est.close()


def test_learned_scorers_served_equal_the_batch_api(torch_dev, streams):
    """Both learned scorers with the handcrafted fallback behind the server:
    every served frame's result equals the batch API's on the same frame and
    uid (the server runs the same kernels on its own batches)."""
    torch = torch_dev
    model2d = os.path.join(train_scorer.MODEL_DIR, train_scorer.MODEL_FILE_2D)
    if not (os.path.exists(MODEL) and os.path.exists(model2d)):
        pytest.skip("no trained scorer models")
    est = api.Estimator(0)
    est.set_model(train_scorer.load_model())
    est.set_model_2d(train_scorer.load_model_2d(model2d))
    for scorer in (1, 2):
        kw = dict(KW, scorer=scorer, fallback_inlier_frac=0.5)
        srv = serve.Server(est, serve.server_config(max_batch=16, **kw))
        got, _ = serve.run(srv, streams[:4], realtime=False)
        srv.close()
        assert len(got) == sum(len(s.arrivals) for s in streams[:4])
        for r in got:
            st = streams[r["stream"]]
            frame = st.frames[r["seq"] % len(st.frames)]
            uid = (r["stream"] << 32) | r["seq"]
            res = est.estimate_area(frame, api.default_params(**kw), [uid])
            torch.cuda.synchronize()
            raw = res.raw.cpu().numpy()[0]
            want = tuple(raw[:4].view(np.float32)) + tuple(int(v) for v in raw[4:])
            assert r["result"] == want, (scorer, r["stream"], r["seq"])
    est.close()


def test_lent_frames_read_in_place(torch_dev, streams):
    """Frames lent to the server (read in place, no ring slot) mixed with
    copied ones in each stream, padded rows among them: each stream's frames
    are served in submission order, each result equals the batch API's on
    the same frame and uid, and results and filtered circles equal those of
    the same backlog with every frame copied."""
    torch = torch_dev
    est = api.Estimator(0)
    src = [streams[0], streams[1]]                     # 720p and 1080p
    ids = [200, 201, 202, 203]
    frames = {}
    for k, sid in enumerate(ids):
        st = src[k % 2]
        base = st.frames[1]
        if k < 2:                                      # padded rows: a view into a wider image
            wide = torch.zeros((st.height, st.width + 5, 3), dtype=torch.uint8, device="cuda")
            wide[:, :st.width].copy_(base)
            f = wide[:, :st.width]
        else:
            f = base
        frames[sid] = f
    torch.cuda.synchronize()

    def serve_all(lend_of):
        srv = serve.Server(est, serve.server_config(max_batch=16, **KW))
        for k, sid in enumerate(ids):
            assert srv.open(sid, src[k % 2].width, src[k % 2].height)
        for seq in range(6):
            for sid in ids:
                srv.submit(sid, seq, frames[sid], lend_of(sid, seq))
        served = []
        for _ in range(100000):
            served += [serve.served_record(s) for s in srv.step()]
            if len(served) == 6 * len(ids):
                break
        srv.close()
        assert len(served) == 6 * len(ids)
        return served

    say("lent and copied frames in one backlog")
    mixed = serve_all(lambda sid, seq: (seq + sid) % 2 == 0)
    copied = serve_all(lambda sid, seq: False)
    for sid in ids:
        seqs = [r["seq"] for r in mixed if r["stream"] == sid]
        assert seqs == sorted(seqs) == list(range(6)), sid
    by = {_key(r): r for r in copied}
    for r in mixed:
        assert r["result"] == by[_key(r)]["result"], _key(r)
        assert r["filtered"] == by[_key(r)]["filtered"], _key(r)
        uid = (r["stream"] << 32) | r["seq"]
        res = est.estimate_area(frames[r["stream"]], api.default_params(**KW), [uid])
        torch.cuda.synchronize()
        raw = res.raw.cpu().numpy()[0]
        want = tuple(raw[:4].view(np.float32)) + tuple(int(v) for v in raw[4:])
        assert r["result"] == want, _key(r)
    est.close()
