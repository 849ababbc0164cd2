"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs -- candidates and per-attempt inliers bit-exact, circles
within 1e-3 px -- at the small 640x480 size, the full 64 x 1080p batch,
brute-force enumeration on tiny frames, and edge cases."""
import numpy as np
import pytest

import oracle
from paper_2210_14771_amd import api, synth

from gpu_helpers import (assert_attempts_equal, assert_points_equal, assert_results_equal,
                         gen_batch, oracle_params, run_gpu, run_oracle, say)

pytestmark = pytest.mark.gpu

SMALL = dict(n_hstrips=16, n_vstrips=16, ransac_attempts=256)
HD = dict(n_hstrips=32, n_vstrips=32, ransac_attempts=1024)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


# split: one strip launch and one RANSAC launch per call; split_pipeN: the
# call cut into N sub-batches alternating over two side streams forked from
# and joined back into the caller's stream; fused: the persistent kernel
@pytest.fixture(scope="module", params=["split", "split_pipe2", "split_pipe4", "fused"])
def est(torch_dev, request):
    e = api.Estimator(0)
    e.set_option("schedule", "fused" if request.param == "fused" else "split")
    if request.param.startswith("split_pipe"):
        e.set_option("pipeline", int(request.param[len("split_pipe"):]))
    else:
        e.set_option("pipeline", 1)
    say(f"schedule: {request.param}")
    yield e
    e.device_status()
    e.close()


@pytest.fixture(scope="module")
def small_batch():
    return synth.make_batch(synth.SMALL_640x480)


@pytest.fixture(scope="module")
def hd_batch():
    return gen_batch(synth.HD_1080p, 64)


def _dev(torch, frames):
    return torch.from_numpy(np.ascontiguousarray(frames)).cuda()


def _full_parity(torch, est, frames, kw, uids=None, attempts=True):
    uids = list(range(len(frames))) if uids is None else uids
    say(f"parity case: {frames.shape} {kw}")
    fd = _dev(torch, frames)
    g = run_gpu(est, fd, kw, uids, what=("pts", "att", "res") if attempts else ("pts", "res"))
    r, p, a = run_oracle(frames, kw, uids, attempts=attempts)
    assert_points_equal(g["pts"], p)
    bits = None
    if attempts:
        bits = assert_attempts_equal(g["att"], a)
        assert_results_equal(g["res_att"], r)
    assert_results_equal(g["res"], r)
    return g, r, bits


def test_small_workload_parity(torch_dev, est, small_batch):
    frames, specs = small_batch
    g, r, bits = _full_parity(torch_dev, est, frames, SMALL)
    say(f"circle values bit-identical: {bits[0]}/{bits[1]}")
    assert bits[0] == bits[1]
    assert all(int(x["valid"]) == 1 for x in r)


def test_hd_workload_parity(torch_dev, est, hd_batch):
    frames, specs = hd_batch
    g, r, bits = _full_parity(torch_dev, est, frames, HD)
    say(f"circle values bit-identical: {bits[0]}/{bits[1]}")
    assert bits[0] == bits[1]


@pytest.mark.parametrize("lanes", [2, 4, 8, 16])
def test_ransac_lanes_per_attempt(torch_dev, small_batch, lanes):
    # the attempts of a small batch spread over more workgroups (more lanes
    # share an attempt's inlier passes): every attempt, candidate and result
    # still equals the oracle
    e = api.Estimator(0)
    e.set_option("schedule", "split")
    e.set_option("ransac_lanes", lanes)
    frames, _ = small_batch
    say(f"ransac lanes {lanes}")
    g, r, bits = _full_parity(torch_dev, e, frames, SMALL)
    assert bits[0] == bits[1]
    e.device_status()
    e.close()


WIDE = dict(n_hstrips=64, n_vstrips=64, ransac_attempts=256, t_ps=0.0, t_px=0)


@pytest.fixture(scope="module")
def wide_batch():
    return np.stack([synth.make_frame(synth.HD_1080p, 310 + i, 16384, 512)[0] for i in range(2)])


def test_large_extent_parity(torch_dev, est, wide_batch):
    # 16384 x 512 frames keeping all 256 candidates (no score or edge filter):
    # n^2 max(U, V) (U^2 + V^2) is 8 times 2^52, so the refits form the
    # centred moment sums in int64 rather than float64; both forms must agree
    # with the oracle bit for bit
    g, r, bits = _full_parity(torch_dev, est, wide_batch, WIDE, uids=[310, 311])
    W, H = 16384, 512
    U, V = W // 2, H // 2
    for x in r:
        n = int(x["n_points"])
        assert n == 256
        assert float(n) * n * max(U, V) * (U * U + V * V) >= 2.0 ** 52
    assert bits[0] == bits[1]


def test_enumeration_equals_brute_force(torch_dev, est):
    # tiny frames: every triple of the kept points is tried once
    frames, _ = synth.make_batch(synth.SMALL_640x480, 6)
    tiny = np.ascontiguousarray(frames[:, ::5, ::5])
    kw = dict(n_hstrips=4, n_vstrips=3, ransac_attempts=4096, sampler=1)
    g = run_gpu(est, _dev(torch_dev, tiny), kw, list(range(6)))
    for i in range(6):
        b = oracle.estimate_bruteforce(tiny[i], oracle.params(n_hstrips=4, n_vstrips=3,
                                                              attempts=4096, sampler=1), i)
        gr = g["res"][i]
        assert gr["valid"] == b["valid"] and gr["inliers"] == b["inliers"]
        assert gr["n_points"] == b["n_points"]
        if b["best_attempt"] >= 0:
            assert abs(float(gr["cx"]) - float(b["cx"])) <= 1e-3
            assert abs(float(gr["r"]) - float(b["r"])) <= 1e-3
    _full_parity(torch_dev, est, tiny, kw)


@pytest.mark.parametrize("case", ["blank", "odd_unaligned", "padded_stride", "paper_literal",
                                  "max_strips", "one_attempt", "no_refine", "tall",
                                  "minimum_size", "enumerate_small"])
def test_edge_cases(torch_dev, est, case):
    torch = torch_dev
    frames, _ = synth.make_batch(synth.SMALL_640x480, 3)
    kw = dict(SMALL)
    if case == "blank":
        frames = np.stack([np.zeros((120, 160, 3), np.uint8), np.full((120, 160, 3), 255, np.uint8),
                           np.full((120, 160, 3), 77, np.uint8)])
    elif case == "odd_unaligned":
        # odd width: rows are not 16-byte aligned, so the byte-wise load path runs
        frames = np.ascontiguousarray(frames[:, 3:470, 5:606])
    elif case == "paper_literal":
        kw["n_vstrips"] = 0
    elif case == "max_strips":
        kw.update(n_hstrips=64, n_vstrips=64, ransac_attempts=4096)
    elif case == "one_attempt":
        kw["ransac_attempts"] = 1
    elif case == "no_refine":
        kw["refine_iters"] = 0
    elif case == "tall":
        frames = np.ascontiguousarray(frames.transpose(0, 2, 1, 3))
    elif case == "minimum_size":
        frames = np.ascontiguousarray(frames[:, 200:216, 300:316])
    elif case == "enumerate_small":
        kw.update(sampler=1, ransac_attempts=300)
    if case == "padded_stride":
        # rows 7 bytes longer than the pixels, frames at unaligned offsets
        B, H, W, _ = frames.shape
        rs = 3 * W + 7
        buf = np.zeros(B * H * rs + 5, np.uint8)
        descs_frames = []
        for b in range(B):
            base = 5 + b * H * rs
            for y in range(H):
                buf[base + y * rs: base + y * rs + 3 * W] = frames[b, y].reshape(-1)
        dbuf = torch.from_numpy(buf).cuda()
        views = [torch.as_strided(dbuf, (H, W, 3), (rs, 3, 1), 5 + b * H * rs) for b in range(B)]
        say(f"edge case {case}")
        g = run_gpu(est, views, kw, [0, 1, 2], what=("pts", "att", "res"))
        r, p, a = run_oracle(frames, kw, [0, 1, 2], attempts=True)
        assert_points_equal(g["pts"], p)
        assert_attempts_equal(g["att"], a)
        assert_results_equal(g["res"], r)
        return
    say(f"edge case {case}")
    _full_parity(torch, est, np.ascontiguousarray(frames), kw)


def test_mixed_resolutions_in_one_batch(torch_dev, est):
    torch = torch_dev
    sizes = [(576, 720), (720, 1280), (1080, 1920), (480, 640), (2160, 3840)]
    frames = [synth.make_frame(synth.HD_1080p, 100 + i, w, h)[0] for i, (h, w) in enumerate(sizes)]
    devs = [torch.from_numpy(f).cuda() for f in frames]
    uids = [100 + i for i in range(len(frames))]
    say("mixed resolution batch")
    g = run_gpu(est, devs, HD, uids, what=("pts", "res"))
    for i, f in enumerate(frames):
        r, p = oracle.estimate(f, oracle.params(n_hstrips=32, n_vstrips=32, attempts=1024),
                               uids[i], with_points=True)
        assert_points_equal(g["pts"][i:i + 1], [p])
        assert_results_equal(g["res"][i:i + 1], [r])


@pytest.mark.parametrize("n_h,n_v", [(8, 12), (4, 3)], ids=["pairs", "single_strips"])
def test_odd_sizes_in_one_batch(torch_dev, est, n_h, n_v):
    # 20 frames of small and odd extents (from the 16-pixel minimum, odd
    # heights, half lines of odd length, a tall narrow frame) in one batch:
    # every candidate and result equals the oracle's.  The strip counts take
    # each strip kernel in turn: strips in pairs (8 + 12), one per workgroup
    # (4 + 3: an odd count).
    torch = torch_dev
    sizes = [(16, 40), (33, 64), (63, 48), (64, 96), (65, 80), (97, 120), (129, 64), (1000, 72),
             (480, 640), (31, 200)] * 2
    frames = [synth.make_frame(synth.SMALL_640x480, 700 + i, w, h)[0]
              for i, (h, w) in enumerate(sizes)]
    devs = [torch.from_numpy(f).cuda() for f in frames]
    uids = [700 + i for i in range(len(frames))]
    kw = dict(n_hstrips=n_h, n_vstrips=n_v, ransac_attempts=64)
    say(f"odd sizes in one batch, {n_h} + {n_v} strips")
    g = run_gpu(est, devs, kw, uids, what=("pts", "res"))
    for i, f in enumerate(frames):
        r, p = oracle.estimate(f, oracle_params(**kw), uids[i], with_points=True)
        assert_points_equal(g["pts"][i:i + 1], [p])
        assert_results_equal(g["res"][i:i + 1], [r])


def test_many_vertical_strips_on_odd_sizes(torch_dev, est):
    # 40 frames of small and odd extents with 32 vertical strips (on the
    # narrowest frames many strips share a column); under the pipelined
    # schedules sub-batches start mid-batch.  Every candidate and result
    # equals the oracle's
    torch = torch_dev
    sizes = [(16, 40), (33, 64), (63, 48), (64, 96), (65, 80), (97, 120), (129, 64), (1000, 72),
             (480, 640), (31, 200)] * 4
    frames = [synth.make_frame(synth.SMALL_640x480, 900 + i, w, h)[0]
              for i, (h, w) in enumerate(sizes)]
    devs = [torch.from_numpy(f).cuda() for f in frames]
    uids = [900 + i for i in range(len(frames))]
    kw = dict(n_hstrips=8, n_vstrips=32, ransac_attempts=64)
    say("odd sizes, 32 vertical strips")
    g = run_gpu(est, devs, kw, uids, what=("pts", "res"))
    for i, f in enumerate(frames):
        r, p = oracle.estimate(f, oracle_params(**kw), uids[i], with_points=True)
        assert_points_equal(g["pts"][i:i + 1], [p])
        assert_results_equal(g["res"][i:i + 1], [r])


def test_frame_result_independent_of_batch(torch_dev, est, small_batch):
    torch = torch_dev
    frames, _ = small_batch
    fd = _dev(torch, frames)
    uids = [1000 + i for i in range(len(frames))]
    whole = run_gpu(est, fd, SMALL, uids)["res"]
    for i in (0, 5):
        alone = run_gpu(est, fd[i:i + 1], SMALL, [uids[i]])["res"]
        assert alone.tobytes() == whole[i:i + 1].tobytes()
    # reversed batch order, same uids
    rev = run_gpu(est, fd.flip(0).contiguous(), SMALL, uids[::-1])["res"]
    assert rev[::-1].tobytes() == whole.tobytes()


def test_repeated_runs_bitwise_equal(torch_dev, est, small_batch):
    torch = torch_dev
    fd = _dev(torch, small_batch[0])
    a = run_gpu(est, fd, SMALL, list(range(8)), what=("pts", "att"))
    b = run_gpu(est, fd, SMALL, list(range(8)), what=("pts", "att"))
    assert a["pts"].tobytes() == b["pts"].tobytes()
    assert a["att"].tobytes() == b["att"].tobytes()


def test_errors_are_reported_before_enqueue(torch_dev, est):
    torch = torch_dev
    f = torch.zeros((1, 20, 20, 3), dtype=torch.uint8, device="cuda")
    with pytest.raises(Exception):
        est.estimate_area(f, {"ransac_attempts": 0})
    with pytest.raises(Exception):
        est.estimate_area(torch.zeros((1, 8, 8, 3), dtype=torch.uint8, device="cuda"))
    # the context stays usable
    r = est.estimate_area(f)
    torch.cuda.synchronize()
    assert int(r.valid[0]) == 0 and int(r.reason[0]) == 1


def test_tiny_budget_is_nomem_and_context_survives(torch_dev):
    torch = torch_dev
    from paper_2210_14771_amd import _native as N
    e = api.Estimator(0, workspace_budget=1024)
    f = torch.zeros((4, 64, 64, 3), dtype=torch.uint8, device="cuda")
    with pytest.raises(N.NativeError) as ei:
        e.estimate_area(f)
    assert ei.value.code == N.CA_E_NOMEM
    e.close()


@pytest.mark.parametrize("opts", [dict(lag=0), dict(lag=1000), dict(queues=1), dict(queues=8),
                                  dict(grid=8), dict(grid=8, queues=8, lag=0), dict(queues=3)])
def test_fused_schedule_variants(torch_dev, small_batch, opts):
    # every queue layout, lag and grid size must give the same bits
    torch = torch_dev
    frames, _ = small_batch
    frames = np.concatenate([frames, frames[::-1].copy()])        # 16 frames
    uids = list(range(16))
    ref_est = api.Estimator(0)
    ref_est.set_option("schedule", "split")
    fd = _dev(torch, frames)
    ref = run_gpu(ref_est, fd, SMALL, uids, what=("pts", "att", "res"))
    ref_est.close()
    e = api.Estimator(0)
    for k, v in opts.items():
        e.set_option(k, v)
    say(f"fused variant {opts}")
    for _ in range(2):          # a second call checks that the control words were rearmed
        got = run_gpu(e, fd, SMALL, uids, what=("pts", "att", "res"))
        assert got["pts"].tobytes() == ref["pts"].tobytes()
        assert got["att"].tobytes() == ref["att"].tobytes()
        assert got["res"].tobytes() == ref["res"].tobytes()
    e.device_status()
    e.close()


def test_fused_small_batches_and_plan_switching(torch_dev, small_batch):
    torch = torch_dev
    frames, _ = small_batch
    e = api.Estimator(0)
    fd = _dev(torch, frames)
    outs = {}
    for n in (1, 3, 8, 1, 8, 3):
        outs.setdefault(n, []).append(run_gpu(e, fd[:n], SMALL, list(range(n)))["res"].tobytes())
    for n, v in outs.items():
        assert all(x == v[0] for x in v), n
    r, p, a = run_oracle(frames[:3], SMALL, [0, 1, 2])
    assert_results_equal(np.frombuffer(outs[3][0], dtype=run_gpu(e, fd[:3], SMALL, [0, 1, 2])["res"].dtype), r)
    e.device_status()
    e.close()


@pytest.mark.parametrize("queues", [1, 8])
def test_fused_repeated_against_split(torch_dev, hd_batch, queues):
    # strip candidates and attempt records cross workgroups (and XCDs) inside
    # the fused kernel; repeated calls must reproduce the split schedule's bits
    torch = torch_dev
    frames, _ = hd_batch
    fd = _dev(torch, frames)
    uids = list(range(len(frames)))
    split = api.Estimator(0)
    split.set_option("schedule", "split")
    ref = run_gpu(split, fd, HD, uids, what=("pts", "res"))
    split.close()
    e = api.Estimator(0)
    e.set_option("queues", queues)
    say(f"fused x10, queues={queues}")
    for i in range(10):
        got = run_gpu(e, fd, HD, uids, what=("pts", "res"))
        assert got["pts"].tobytes() == ref["pts"].tobytes(), i
        assert got["res"].tobytes() == ref["res"].tobytes(), i
    e.device_status()
    e.close()


def test_graph_replays_match_eager(torch_dev, hd_batch):
    # several replays with eager work and synchronisation between them; every
    # replay must reproduce the eager results (no state leaks between replays)
    torch = torch_dev
    frames, _ = hd_batch
    fd = _dev(torch, frames[:16])
    fd2 = _dev(torch, frames[16:32])
    uids = list(range(16))
    for sched in ("split", "fused"):
        e = api.Estimator(0)
        e.set_option("schedule", sched)
        p = api.default_params(**HD)
        ref = e.estimate_area(fd, p, uids).numpy()
        ref2 = e.estimate_area(fd2, p, uids).numpy()
        out = torch.zeros((16, 8), dtype=torch.int32, device="cuda")
        g = e.capture(fd, p, uids, out=out, calls=3)
        say(f"graph replays ({sched})")
        for i in range(4):
            out.zero_()
            g.launch()
            torch.cuda.synchronize()
            assert g.result.numpy().tobytes() == ref.tobytes(), (sched, i)
            other = e.estimate_area(fd2, p, uids).numpy()      # eager work in between
            assert other.tobytes() == ref2.tobytes()
        g.close()
        e.device_status()
        e.close()
