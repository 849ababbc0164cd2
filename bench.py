"""Throughput benchmark of the content-area estimator on one MI355X.

One step = one call of the whole hot path (strip scoring, candidate
selection, RANSAC with refits, best-circle selection) on a batch of 64
synthetic 1920x1080 RGB frames already resident in HBM.  The timed steps
replay captured HIP graphs with six batches in flight (six contexts on
six HIP streams taking turns, so one batch's FP64 RANSAC overlaps other
batches' strip loads, and the strip loads of several batches together keep
more DRAM pages busy); the same steps with one batch in flight, and eager
calls, are reported beside.  Prints one JSON
line with frames/s, per-call latency percentiles, the dominant kernel's
roofline position (kernel time from HIP events recorded inside the library
on the launch stream), accuracy against the synthetic ground truth, and the
CPU oracle timed on the host cores as a reference point.

    python bench.py [--gpus 1] [--steps 1000] [--warmup 50]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "1080p frames/s + HBM GB/s, learned vs plain at ≤2 px circle err; p99 ms"
HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E, vendor figure
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X vector FP64


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--latency-calls", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate CPU work of the oracle sample")
    ap.add_argument("--batches", type=int, default=7,
                    help="distinct resident batches rotated (more than --inflight, so calls in "
                         "flight together read different batches)")
    ap.add_argument("--schedule", choices=["auto", "fused", "split"], default="auto",
                    help="auto: the schedule and strip tiles ca_autotune measures fastest for "
                         "the batch")
    ap.add_argument("--graph-calls", type=int, default=10,
                    help="estimate calls captured per HIP graph in the timed region")
    ap.add_argument("--inflight", type=int, default=6,
                    help="batches in flight in the timed region: contexts, each with its own "
                         "plan buffers, output and HIP stream, taking the graphs in turn")
    ap.add_argument("--pipeline", type=int, default=None, help="sub-batches per split call")
    ap.add_argument("--lag", type=int, default=None)
    ap.add_argument("--queues", type=int, default=None)
    ap.add_argument("--learned-steps", type=int, default=100,
                    help="timed calls of the learned scorer (0: skip the learned section)")
    ap.add_argument("--hard-frames", type=int, default=64,
                    help="device-rendered hard 1080p frames for the accuracy comparison")
    ap.add_argument("--mixed-steps", type=int, default=20,
                    help="timed graph replays of the 512-frame uneven batch (0: skip)")
    ap.add_argument("--small-steps", type=int, default=20,
                    help="timed graph launches (100 calls each) of the 8 x 640x480 case (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=0.4,
                    help="seconds of simulated arrivals of the 48-stream serving loop, plain "
                         "and learned side by side, in a child process (0: skip)")
    ap.add_argument("--small-only", action="store_true",
                    help="run only the small case (8 x 640x480) and print its JSON (profiling)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def graph_calls(steps: int, wanted: int, cycle: int) -> int:
    """Calls per captured graph: the largest G <= wanted dividing `steps`
    that still leaves steps // G >= cycle launches (with cycle = the contexts
    in flight, every context runs); 1 when no such G exists.  The contexts
    and resident batches a run touches are reported (rotation_used)."""
    for g in range(min(wanted, steps), 0, -1):
        if steps % g == 0 and steps // g >= cycle:
            return g
    return 1


def contexts_in_flight(steps: int, wanted: int, graph_max: int, min_graph: int = 4) -> int:
    """Contexts for a timed region of `steps` calls: the most, up to `wanted`,
    whose graphs (graph_calls) still hold at least `min_graph` calls, so short
    runs trade a context for fewer graph launches (at 20 steps: 5 contexts
    with 4-call graphs rather than 6 with 2-call ones)."""
    for c in range(max(1, wanted), 1, -1):
        if steps >= c and graph_calls(steps, graph_max, c) >= min(min_graph, steps // c):
            return c
    return 1


def rotation_used(launches: int, contexts: int, batches: int) -> dict:
    """Contexts and resident batches a run of `launches` graph launches
    actually touches when launch i goes to context i % contexts and reads
    batch i % batches."""
    return {"contexts": min(contexts, launches), "batches": min(batches, launches)}


def strip_bytes_per_frame(w: int, h: int, n_h: int, n_v: int) -> int:
    """Bytes the method must read: 3 full rows per horizontal strip and
    3 pixels of every row per vertical strip (RGB, 3 bytes per pixel)."""
    return n_h * 3 * (3 * w) + n_v * h * 9


def ransac_flops(n_points, attempts: int, refine: int) -> float:
    """FP64 operations the method itself asks for in the inlier passes: per
    attempt, point and pass (K refits and the final count) the squared
    distance to the centre (2 sub, 2 mul, 1 add); the band test is two
    compares and the moment sums over inliers are integer additions, so
    neither is counted."""
    return float(sum(attempts * n * (refine + 1) * 5 for n in n_points if n >= 3))


def ransac_issued_flops(n_points, attempts: int, refine: int) -> float:
    """FP64 operations the kernel issues for the same passes: per point and
    refit pass the squared distance (5) and 9 moment FMAs accumulating the
    integer sums exactly in float64 (18), masked rather than branched; per
    point in the final pass the distance and 2 FMAs (9)."""
    return float(sum(attempts * n * (refine * 23 + 9) for n in n_points if n >= 3))


def measured_traffic(kernel: str, source: str = "ca_kernels.hip"):
    """HBM bytes per launch of `kernel` from its committed rocprofv3 counter
    summary (profiles/<kernel>_64x1080p_hbm_traffic.md), or None when the
    kernel source changed since the counters were taken."""
    import hashlib
    import re
    src = os.path.join(ROOT, "paper_2210_14771_amd", "csrc", source)
    summary = os.path.join(ROOT, "profiles", f"{kernel}_64x1080p_hbm_traffic.md")
    try:
        text = open(summary).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch " + kernel + r" (\d+)", text)
    h = re.search(r"source_sha256_prefix ([0-9a-f]+)", text)
    if not m or not h or not sha.startswith(h.group(1)):
        return None
    return int(m.group(1))


def strip_kernel(n_h: int, n_v: int, tiles: int = 1) -> str:
    """The strip kernel a split call launches: strips in pairs (one
    workgroup per two strips) when both counts are even and each workgroup
    takes one item, else one strip per workgroup item."""
    return "k_strips_pair" if tiles <= 1 and n_h % 2 == 0 and n_v % 2 == 0 else "k_strips"


BF16_MFMA_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 matrix


def cnn_flops_per_frame(w: int, h: int, n_h: int, n_v: int) -> float:
    """Multiply-adds x 2 of the learned scorer at every strip position once:
    four width-5 convolutions 24-16-32-32-16 and the 1x1 layer."""
    macs = 5 * (24 * 16 + 16 * 32 + 32 * 32 + 32 * 16) + 16
    return 2.0 * macs * (n_h * w + n_v * h)


def cnn2d_flops_per_frame(w: int, h: int, n_h: int, n_v: int) -> float:
    """Multiply-adds x 2 of the paper's 2-D network per strip position: layer
    1 on the band's 5 inner lines (8 x 5 x 9 each), layer 2 on 3 lines
    (16 x 8 x 9), layer 3 on the strip line (32 x 16 x 9), the 1x1 layer."""
    macs = 5 * 8 * 5 * 9 + 3 * 16 * 8 * 9 + 32 * 16 * 9 + 32
    return 2.0 * macs * (n_h * w + n_v * h)


def learned_section(args, est, resident, specs, params_plain, kw, uids, out):
    """The learned scorer (with the handcrafted fallback) on the same frames:
    throughput, kernel roofline, accuracy next to the plain scorer on the
    headline batch and on device-rendered hard frames."""
    import numpy as np
    import torch
    from paper_2210_14771_amd import api, evaluate, synth, synth_gpu, train_scorer
    path = os.path.join(train_scorer.MODEL_DIR, train_scorer.MODEL_FILE)
    if args.learned_steps <= 0 or not os.path.exists(path):
        return None
    B, W, H = len(specs), specs[0].width, specs[0].height
    est.set_model(train_scorer.load_model(path))
    lp = api.default_params(**kw, scorer=1, fallback_inlier_frac=0.5)
    lp_nofb = api.default_params(**kw, scorer=1)
    K = args.learned_steps
    for i in range(5):
        est.estimate_area(resident[i % len(resident)], lp, uids, out=out)
    torch.cuda.synchronize()
    saved_pipeline = est.get_option("pipeline")
    est.set_option("pipeline", 1)
    est.profile_begin(K)
    for i in range(K):
        est.estimate_area(resident[i % len(resident)], lp_nofb, uids, out=out)
    torch.cuda.synchronize()
    kt = est.profile_end()
    est.set_option("pipeline", saved_pipeline)
    # as in the headline step: up to `args.inflight` contexts (each with the
    # model, its own buffers, output and stream) take the graph launches in turn
    n_inflight = contexts_in_flight(K, args.inflight, 10)
    G = graph_calls(K, 10, n_inflight)

    def inflight_timing(params, load_model):
        """Elapsed time of K calls with one context, then with n_inflight
        (graphs of G calls taken in turn), the rotation each touched, and
        whether every context gives the first one's results."""
        extra = []
        for _ in range(n_inflight - 1):
            e = api.Estimator(0)
            load_model(e)
            extra.append(e)
        ests = [est] + extra
        outs = [out] + [torch.empty_like(out) for _ in extra]
        streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in extra]
        used = {}

        def graph_region(n):
            graphs = [[ests[k].capture(r, params, uids, out=outs[k], calls=G) for r in resident]
                      for k in range(n)]
            for k in range(n):
                for g in graphs[k]:
                    g.launch(streams[k])
            torch.cuda.synchronize()
            t = time.perf_counter()
            for i in range(K // G):
                graphs[i % n][i % len(resident)].launch(streams[i % n])
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            for gs in graphs:
                for g in gs:
                    g.close()
            used[n] = rotation_used(K // G, n, len(resident))
            return dt

        one = graph_region(1)
        many = graph_region(n_inflight) if n_inflight > 1 else one
        ref = est.estimate_area(resident[0], params, uids).raw
        same = all(torch.equal(e.estimate_area(resident[0], params, uids).raw, ref)
                   for e in extra)
        for e in extra:
            e.close()
        return one, many, used, same

    elapsed_one, elapsed, used, identical = inflight_timing(
        lp, lambda e: e.set_model(train_scorer.load_model(path)))
    lat = []
    for i in range(min(args.latency_calls, 100)):
        t1 = time.perf_counter()
        est.estimate_area(resident[i % len(resident)], lp, uids, out=out)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
    cnn_ms = kt["strips"]["avg_ms"]
    flops = B * cnn_flops_per_frame(W, H, kw["n_hstrips"], kw["n_vstrips"])
    rl = {"kernel": "k_cnn_strips", "bound": "mfma",
          "achieved": flops / (cnn_ms * 1e-3) / 1e12, "peak": BF16_MFMA_PEAK_TFLOPS,
          "unit": "TFLOP/s", "traffic": measured_traffic("k_cnn_strips", "ca_cnn.hip")}
    rl["frac"] = rl["achieved"] / rl["peak"]
    print("# learned: accuracy", file=sys.stderr, flush=True)
    hard, hard_specs = synth_gpu.render_set(synth.HARD_1080p, synth.HARD_1080p.config_id,
                                            args.hard_frames, True)
    acc = {}
    path2d = os.path.join(train_scorer.MODEL_DIR, train_scorer.MODEL_FILE_2D)
    has2d = os.path.exists(path2d)
    if has2d:
        est.set_model_2d(train_scorer.load_model_2d(path2d))
    lp2 = api.default_params(**kw, scorer=2, fallback_inlier_frac=0.5)
    lp2_nofb = api.default_params(**kw, scorer=2)
    for name, fr, sp in (("accuracy_1080p", resident[0], specs),
                         ("accuracy_hard_1080p", hard, hard_specs)):
        acc[name] = {"plain": evaluate.accuracy(est, fr, sp, params_plain, by=True),
                     "learned": evaluate.accuracy(est, fr, sp, lp_nofb, by=True),
                     "learned_fallback": evaluate.accuracy(est, fr, sp, lp, by=True)}
        if has2d:
            acc[name]["learned_2d"] = evaluate.accuracy(est, fr, sp, lp2_nofb, by=True)
            acc[name]["learned_2d_fallback"] = evaluate.accuracy(est, fr, sp, lp2, by=True)
    learned_2d = None
    if has2d:
        # the paper's own network: kernel time (dispatch events) and whole-call
        # throughput from graph replays, one and n_inflight batches in flight
        print("# learned 2-D scorer", file=sys.stderr, flush=True)
        saved_pipeline = est.get_option("pipeline")
        est.set_option("pipeline", 1)
        est.profile_begin(K)
        for i in range(K):
            est.estimate_area(resident[i % len(resident)], lp2_nofb, uids, out=out)
        torch.cuda.synchronize()
        kt2 = est.profile_end()
        est.set_option("pipeline", saved_pipeline)
        model2d = train_scorer.load_model_2d(path2d)
        el2_one, el2, used2, same2 = inflight_timing(lp2, lambda e: e.set_model_2d(model2d))
        ms2 = kt2["strips"]["avg_ms"]
        fl2 = B * cnn2d_flops_per_frame(W, H, kw["n_hstrips"], kw["n_vstrips"])
        rl2 = {"kernel": "k_cnn2d_strips", "bound": "mfma",
               "achieved": fl2 / (ms2 * 1e-3) / 1e12, "peak": BF16_MFMA_PEAK_TFLOPS,
               "unit": "TFLOP/s", "traffic": measured_traffic("k_cnn2d_strips", "ca_cnn2d.hip")}
        rl2["frac"] = rl2["achieved"] / rl2["peak"]
        learned_2d = {"value": B * K / el2, "unit": "frames/s", "ms_per_step": el2 / K * 1e3,
                      "timing": f"{K // G} launches of HIP graphs of {G} calls on "
                                f"{used2[n_inflight]['contexts']} contexts taking the launches "
                                f"in turn, over {used2[n_inflight]['batches']} distinct resident "
                                f"batches, with the handcrafted fallback",
                      "inflight": dict(used2[n_inflight], graph_calls=G, launches=K // G,
                                       results_identical=bool(same2)),
                      "one_in_flight_value": B * K / el2_one,
                      "scorer": "the paper's 2-D CNN (3x3 convolutions 8/16/32 on RGBXY bands, "
                                "BF16 MFMA), handcrafted fallback below 0.5 inlier fraction",
                      "kernels": {"k_cnn2d_strips": {"avg_us": ms2 * 1e3},
                                  "k_ransac": {"avg_us": kt2["ransac"]["avg_ms"] * 1e3}},
                      "roofline": rl2}
    return {
        "value": B * K / elapsed, "unit": "frames/s", "ms_per_step": elapsed / K * 1e3,
        "steps": K,
        "timing": f"{K // G} launches of HIP graphs of {G} calls on "
                  f"{used[n_inflight]['contexts']} contexts taking the launches in turn, over "
                  f"{used[n_inflight]['batches']} distinct resident batches",
        "inflight": dict(used[n_inflight], graph_calls=G, launches=K // G,
                         results_identical=bool(identical)),
        "one_in_flight_value": B * K / elapsed_one,
        "scorer": "learned 1-D CNN (BF16 MFMA), handcrafted fallback below 0.5 inlier fraction",
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "kernels": {"k_cnn_strips": {"avg_us": cnn_ms * 1e3},
                    "k_ransac": {"avg_us": kt["ransac"]["avg_ms"] * 1e3}},
        "kernel_timing": "learned scorer without fallback, one launch per kernel",
        "roofline": rl,
        "learned_2d": learned_2d,
        "accuracy_1080p": acc["accuracy_1080p"],
        "accuracy_hard_1080p": dict(acc["accuracy_hard_1080p"], frames=args.hard_frames,
                                    note="device-rendered: dark rims (edge step 10-25 luma), "
                                         "border noise sigma 2-12, specular blobs and white "
                                         "text in the border"),
    }


def small_section(args):
    """The small case (8 x 640x480, 16+16 strips, 256 attempts): launch-bound,
    so its steady state is taken from HIP graphs of 100 back-to-back calls,
    with one call in flight and with `args.inflight` contexts (each its own
    buffers, output, graph and stream) taking the graph launches in turn."""
    import torch
    from paper_2210_14771_amd import api, synth
    if args.small_steps <= 0:
        return None
    wl = synth.SMALL_640x480
    frames, _ = synth.make_batch(wl)
    dev = torch.from_numpy(frames).cuda()
    kw = dict(n_hstrips=wl.n_hstrips, n_vstrips=wl.n_vstrips, ransac_attempts=wl.attempts)
    params = api.default_params(**kw)
    uids = list(range(len(frames)))
    n = max(1, args.inflight)
    ests, outs, graphs = [], [], []
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(n - 1)]
    for k in range(n):
        est = api.Estimator(0)
        est.set_option("schedule", "auto")
        est.autotune(dev, params, uids, reps=20)
        out = torch.empty((len(frames), 8), dtype=torch.int32, device="cuda")
        ests.append(est)
        outs.append(out)
        graphs.append(est.capture(dev, params, uids, out=out, calls=100))
    for k in range(n):
        graphs[k].launch(streams[k])
    torch.cuda.synchronize()

    def region(m):
        t0 = time.perf_counter()
        for i in range(args.small_steps):
            graphs[i % m].launch(streams[i % m])
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    dt1 = region(1)
    dtn = region(n) if n > 1 else dt1
    identical = all(torch.equal(o, outs[0]) for o in outs[1:])
    schedule = ests[0].last_tuned_schedule
    for g in graphs:
        g.close()
    for e in ests:
        e.close()
    calls = 100 * args.small_steps
    return {"workload": f"plain pipeline, {len(frames)} x {wl.width}x{wl.height} frames per call, "
                        f"{kw['n_hstrips']}+{kw['n_vstrips']} strips, {kw['ransac_attempts']} "
                        f"RANSAC attempts, HIP graphs of 100 back-to-back calls",
            "value": len(frames) * calls / dtn, "unit": "frames/s", "us_per_call": dtn / calls * 1e6,
            "inflight": {"contexts": min(n, args.small_steps), "results_identical": identical},
            "one_in_flight_value": len(frames) * calls / dt1,
            "one_in_flight_us_per_call": dt1 / calls * 1e6,
            "calls": calls, "schedule": schedule}


def mixed_section(args, est, kw):
    """The uneven batch: 512 frames of 720x576, 1280x720, 1920x1080 and
    3840x2160 (2:3:4:1) in one captured graph, strip tiles autotuned."""
    import numpy as np
    import torch
    from paper_2210_14771_amd import api, synth
    if args.mixed_steps <= 0:
        return None
    n = synth.MIXED_512.n_frames
    print(f"# mixed: generating {n} frames", file=sys.stderr, flush=True)
    frames, specs = synth.make_mixed_batch(n, threads=min(16, os.cpu_count() or 1))
    sizes = [f.nbytes for f in frames]
    flat = torch.empty(int(sum(sizes)), dtype=torch.uint8, device="cuda")
    views, at = [], 0
    for f in frames:
        v = flat[at:at + f.nbytes].view(f.shape)
        v.copy_(torch.from_numpy(f))
        views.append(v)
        at += f.nbytes
    del frames
    uids = list(range(n))
    params = api.default_params(**kw)
    est.set_option("strips_per_group", 0)
    est.set_option("schedule", "auto")
    tuned = est.autotune(views, params, uids, reps=5)
    chosen = est.last_tuned_schedule
    chosen_pipeline = est.last_tuned_pipeline
    out = torch.empty((n, 8), dtype=torch.int32, device="cuda")
    K = args.mixed_steps

    def timed(schedule, tiles):
        est.set_option("schedule", schedule)
        est.set_option("strips_per_group", tiles)
        g1 = est.capture(views, params, uids, out=out, calls=1)
        g1.launch()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(K):
            g1.launch()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        g1.close()
        return dt

    elapsed = timed("auto", 0)
    split_t1 = timed("split", 1)
    split_tuned = timed("split", 0)
    persistent = timed("fused", 0)
    est.set_option("schedule", "auto")
    est.set_option("strips_per_group", 0)
    est.device_status()
    algo = sum(strip_bytes_per_frame(s.width, s.height, kw["n_hstrips"], kw["n_vstrips"])
               for s in specs)
    return {"workload": "512 frames 720x576 : 1280x720 : 1920x1080 : 3840x2160 = 2:3:4:1, "
                        "one HIP graph launch per step",
            "value": n * K / elapsed, "unit": "frames/s", "ms_per_step": elapsed / K * 1e3,
            "steps": K, "hbm_gbps_algorithmic": algo * K / elapsed / 1e9,
            "autotuned": {"schedule": chosen, "pipeline": chosen_pipeline,
                          "strips_per_group": {f"{w}x{h}": t for (w, h), t in sorted(tuned.items())}},
            "ms_per_step_by_schedule": {"split_tile1": split_t1 / K * 1e3,
                                        "split_tuned_tiles": split_tuned / K * 1e3,
                                        "persistent_fused": persistent / K * 1e3},
            "note": "value: the autotuned configuration in one HIP graph per step; split: strip "
                    "kernel per frame shape then RANSAC; persistent: one fused kernel",
            "frame_bytes": int(sum(sizes))}


def serving_section(args):
    """The serving loop (48 streams of 720p, 1080p and 4K, Poisson arrivals at
    30-60 frames/s each, continuous batching): p50/p99 latency and frames/s
    with the plain and the learned scorer, from serve_bench in a child
    process with a time limit of its own; its progress lines pass through to
    this program's stderr."""
    import subprocess
    if args.serve_seconds <= 0:
        return None
    cmd = [sys.executable, "-u", "-m", "paper_2210_14771_amd.serve_bench", "--seconds",
           str(args.serve_seconds)]
    limit_s = 240
    try:
        r = subprocess.run(cmd, cwd=ROOT, stdout=subprocess.PIPE, stderr=None, text=True,
                           timeout=limit_s)
    except subprocess.TimeoutExpired:
        return {"status": "timeout", "limit_s": limit_s}
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    if r.returncode != 0 or not lines:
        return {"status": "failed", "rc": r.returncode}
    return json.loads(lines[-1])


def run_environment(params) -> dict:
    import torch
    try:
        rocm = open("/opt/rocm/.info/version").read().strip()
    except OSError:
        rocm = None
    return {"rocm": rocm, "torch": torch.__version__, "hip": torch.version.hip,
            "device": torch.cuda.get_device_name(0), "host_cpus": os.cpu_count(),
            "seed": int(params.seed), "data_seed": "SeedSequence([2210_14771, config, frame])"}


def cpu_baseline(frames, kw, target_cpu_s: float, threads: int | None = None):
    """The oracle on the host cores, on the headline frames: one pass to
    size the sample, then enough passes for about target_cpu_s of CPU time."""
    import oracle
    if threads is None:
        threads = max(1, min(os.cpu_count() or 1, 16))
    p = oracle.params(n_hstrips=kw["n_hstrips"], n_vstrips=kw["n_vstrips"],
                      attempts=kw["ransac_attempts"])
    sample = frames if threads > 1 else frames[:8]
    t0 = time.perf_counter()
    oracle.estimate_batch(sample, p, threads=threads)
    t1 = time.perf_counter() - t0
    reps = max(1, min(1000, math.ceil(target_cpu_s / max(t1 * threads, 1e-6))))
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.estimate_batch(sample, p, threads=threads)
    wall = time.perf_counter() - t0
    n = reps * len(sample)
    return {"value": n / wall, "unit": "frames/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(sample)} x {frames.shape[2]}x{frames.shape[1]} frames x {reps} "
                      f"passes ({n} frame estimates, {wall:.1f} s wall, {threads} threads)"}


def copy_bandwidth(dev, mib: int = 1024, reps: int = 20) -> dict:
    """A plain device-to-device copy on the same GPU (bytes read + written
    per second): the practical HBM ceiling beside the published 8 TB/s."""
    import torch
    src = torch.ones(mib << 20, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return {"value": 2 * (mib << 20) / (ms * 1e-3) / 1e9, "unit": "GB/s",
            "what": f"torch copy_ of {mib} MiB, read + write bytes, mean of {reps}"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the estimator has no cross-GPU step "
              "(frames are independent); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from concurrent.futures import ThreadPoolExecutor

    from paper_2210_14771_amd import api, evaluate, synth

    if args.small_only:
        print(json.dumps(small_section(args)), flush=True)
        return

    wl = synth.HD_1080p
    B, W, H = wl.n_frames, wl.width, wl.height
    kw = dict(n_hstrips=wl.n_hstrips, n_vstrips=wl.n_vstrips, ransac_attempts=wl.attempts)
    print(f"# generating {B} synthetic {W}x{H} frames", file=sys.stderr, flush=True)
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        gen = list(ex.map(lambda i: synth.make_frame(wl, i), range(B)))
    frames = np.stack([g[0] for g in gen])
    specs = [g[1] for g in gen]

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    resident = [torch.from_numpy(frames).to(dev)]
    for k in range(1, args.batches):
        # further resident batches: mirrored copies (different bytes, same work)
        resident.append(resident[0].flip(2 if k % 2 else 1).contiguous())
    uids = list(range(B))
    params = api.default_params(**kw)

    def make_estimator():
        e = api.Estimator(0)
        e.set_option("schedule", args.schedule)
        if args.lag is not None:
            e.set_option("lag", args.lag)
        if args.queues is not None:
            e.set_option("queues", args.queues)
        if args.pipeline is not None:
            e.set_option("pipeline", args.pipeline)
        tiles = {}
        if args.schedule == "auto":
            for r in resident:
                tiles = e.autotune(r, params, uids, reps=20)
        return e, tiles

    print("# autotune", file=sys.stderr, flush=True)
    est, tiles = make_estimator()
    pipeline = est.get_option("pipeline")
    out = torch.empty((B, 8), dtype=torch.int32, device=dev)
    tuning = None
    if args.schedule == "auto":
        schedule_used = est.last_tuned_schedule or "split"
        tuning = {"schedule": schedule_used, "pipeline": est.last_tuned_pipeline,
                  "strips_per_group": {f"{w}x{h}": t for (w, h), t in tiles.items()}}
    else:
        schedule_used = args.schedule
    print("# warmup", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        est.estimate_area(resident[i % len(resident)], params, uids, out=out)
    torch.cuda.synchronize()

    K = args.steps
    # kernel durations: HIP events recorded by the library around each kernel
    # on the launch stream, with the whole batch in one launch per kernel
    if schedule_used == "split":
        est.set_option("pipeline", 1)
    est.profile_begin(K)
    torch.cuda.synchronize()
    for i in range(K):
        est.estimate_area(resident[i % len(resident)], params, uids, out=out)
    torch.cuda.synchronize()
    kt = est.profile_end()
    est.set_option("pipeline", pipeline)
    # eager calls as configured
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        est.estimate_area(resident[i % len(resident)], params, uids, out=out)
    torch.cuda.synchronize()
    elapsed_eager = time.perf_counter() - t0
    print("# eager region done", file=sys.stderr, flush=True)

    # timed region: the same K calls replayed from captured HIP graphs (G
    # calls per graph, one graph per resident batch per context).  With
    # several batches in flight, each context (its own plan buffers, output
    # and HIP stream) takes the graphs in turn, so one batch's RANSAC (FP64
    # ALU) overlaps the next one's strip loads (HBM); every batch still runs
    # the whole path.
    n_inflight = contexts_in_flight(K, args.inflight, args.graph_calls)
    G = graph_calls(K, args.graph_calls, n_inflight)
    extra = [make_estimator()[0] for _ in range(n_inflight - 1)]
    ests = [est] + extra
    outs = [out] + [torch.empty_like(out) for _ in extra]
    streams = [torch.cuda.current_stream(dev)] + [torch.cuda.Stream(dev) for _ in extra]
    used = {}

    def graph_region(n):
        # launch i goes to context i % n and reads resident batch
        # i % len(resident): with more batches than contexts, calls in flight
        # together read distinct batches and every context meets every batch
        graphs = [[ests[k].capture(r, params, uids, out=outs[k], calls=G) for r in resident]
                  for k in range(n)]
        for k in range(n):
            for g in graphs[k]:
                g.launch(streams[k])
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(K // G):
            graphs[i % n][i % len(resident)].launch(streams[i % n])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        for gs in graphs:
            for g in gs:
                g.close()
        used[n] = rotation_used(K // G, n, len(resident))
        return dt

    elapsed_one = graph_region(1)
    elapsed = graph_region(n_inflight) if n_inflight > 1 else elapsed_one
    # warm case: every step on the first resident batch (its strip lines may
    # stay in the Infinity Cache between steps), one in flight
    g_warm = est.capture(resident[0], params, uids, out=out, calls=G)
    g_warm.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K // G):
        g_warm.launch()
    torch.cuda.synchronize()
    elapsed_warm = time.perf_counter() - t0
    g_warm.close()
    for e in ests:
        e.device_status()
    # every context gives the same results
    ref = est.estimate_area(resident[0], params, uids).raw
    inflight_identical = all(
        torch.equal(e.estimate_area(resident[0], params, uids).raw, ref) for e in extra)
    for e in extra:
        e.close()
    print("# graph region done", file=sys.stderr, flush=True)

    # per-call latency: each call waited for on its own
    lat = []
    for i in range(args.latency_calls):
        t1 = time.perf_counter()
        est.estimate_area(resident[i % len(resident)], params, uids, out=out)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
    lat = np.array(lat)

    # accuracy of the same computation (not timed)
    res = est.estimate_area(resident[0], params, uids).numpy()
    errs = evaluate.frame_errors(specs, res["cx"], res["cy"], res["r"], res["valid"])
    acc = evaluate.summarise(errs)
    acc["valid_frac"] = float(np.mean(res["valid"] != 0))

    fps = B * K / elapsed
    algo_bytes = B * strip_bytes_per_frame(W, H, kw["n_hstrips"], kw["n_vstrips"])
    flops = ransac_flops(res["n_points"], kw["ransac_attempts"], params.refine_iters)
    if schedule_used == "fused":
        # one kernel runs the whole path: its HBM position on the strip bytes,
        # and its FP64 position on the RANSAC work, over the same duration
        fused_ms = kt["strips"]["avg_ms"]
        kernels = {"k_fused": {"avg_us": fused_ms * 1e3, "launches": kt["strips"]["launches"]}}
        strips_ms = ransac_ms = fused_ms
        dominant = "fused"
    else:
        strips_ms = kt["strips"]["avg_ms"]
        ransac_ms = kt["ransac"]["avg_ms"]
        kernels = {"k_" + k: {"avg_us": v["avg_ms"] * 1e3, "launches": v["launches"]}
                   for k, v in kt.items() if k != "gap"}
        dominant = "strips" if strips_ms >= ransac_ms else "ransac"
    skern = strip_kernel(kw["n_hstrips"], kw["n_vstrips"], max(tiles.values(), default=1))
    if schedule_used != "fused" and "k_strips" in kernels:
        kernels[skern] = kernels.pop("k_strips")
    traffic = measured_traffic(skern) if schedule_used == "split" else None
    rl_strips = {"bound": "hbm", "achieved": algo_bytes / (strips_ms * 1e-3) / 1e9,
                 "peak": HBM_PEAK_GBPS, "unit": "GB/s", "traffic": traffic,
                 "traffic_note": "bytes per launch from rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                 f"copy-calibrated (profiles/{skern}_64x1080p_hbm_traffic.md)"}
    if traffic:
        rl_strips["traffic_gbps"] = traffic / (strips_ms * 1e-3) / 1e9
    rl_strips["frac"] = rl_strips["achieved"] / rl_strips["peak"]
    issued = ransac_issued_flops(res["n_points"], kw["ransac_attempts"], params.refine_iters)
    rl_ransac = {"bound": "alu", "achieved": flops / (ransac_ms * 1e-3) / 1e12,
                 "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "traffic": None,
                 "flops_note": "the method's FP64 work: one squared distance (5 flops) per "
                               "attempt, point and pass (3 refits + final count); band compares "
                               "and integer moment sums not counted",
                 "issued_tflops": issued / (ransac_ms * 1e-3) / 1e12,
                 "issued_note": "FP64 operations the kernel issues (23 per point and refit "
                                "pass, 9 per point in the final pass)"}
    rl_ransac["frac"] = rl_ransac["achieved"] / rl_ransac["peak"]
    roofline = dict(rl_ransac if dominant == "ransac" else rl_strips)
    roofline["kernel"] = {"fused": "k_fused", "strips": skern, "ransac": "k_ransac"}[dominant]

    line = {
        "metric": METRIC,
        "value": fps,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": elapsed / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8/f32/f64",
        "data": "synthetic",
        "config": {"workload": f"plain handcrafted pipeline, {B} x {W}x{H} uint8 RGB frames per "
                               f"step (60:25:10 partial/full/no-border mix), "
                               f"{kw['n_hstrips']}+{kw['n_vstrips']} strips, "
                               f"{kw['ransac_attempts']} RANSAC attempts",
                   "frames_per_step": B, "width": W, "height": H,
                   "n_hstrips": kw["n_hstrips"], "n_vstrips": kw["n_vstrips"],
                   "ransac_attempts": kw["ransac_attempts"], "scorer": "plain"},
        "hbm_gbps_algorithmic": algo_bytes * K / elapsed / 1e9,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "latency_note": "per call of 64 frames, each call synchronised on its own",
        "timing": f"K steps replayed from {K // G} launches of HIP graphs of {G} calls on "
                  f"{used[n_inflight]['contexts']} contexts and HIP streams taking the launches "
                  f"in turn, over {used[n_inflight]['batches']} distinct resident batches; one "
                  f"batch in flight and eager calls below",
        "inflight": dict(used[n_inflight], graph_calls=G, launches=K // G,
                         results_identical=bool(inflight_identical)),
        "one_in_flight_value": B * K / elapsed_one,
        "one_in_flight_ms_per_step": elapsed_one / K * 1e3,
        "warm_value": B * K / elapsed_warm,
        "warm_note": "one resident batch for every step, one in flight",
        "eager_value": B * K / elapsed_eager,
        "eager_ms_per_step": elapsed_eager / K * 1e3,
        "schedule": schedule_used,
        "autotune": tuning,
        "pipeline": ((pipeline or (est.last_tuned_pipeline if args.schedule == "auto" else 1) or 1)
                     if schedule_used == "split" else None),
        "kernel_timing": "one launch per kernel for the whole batch (pipeline 1)",
        "kernels": kernels,
        "roofline": roofline,
        "roofline_other": rl_strips if dominant == "ransac" else rl_ransac,
        "accuracy": acc,
    }
    print("# learned scorer", file=sys.stderr, flush=True)
    learned = learned_section(args, est, resident, specs, params, kw, uids, out)
    if learned is not None:
        line["learned"] = learned
    mixed = mixed_section(args, est, kw)
    if mixed is not None:
        line["mixed_512"] = mixed
    print("# small case", file=sys.stderr, flush=True)
    small = small_section(args)
    if small is not None:
        line["small_640x480"] = small
    print("# serving", file=sys.stderr, flush=True)
    serving = serving_section(args)
    if serving is not None:
        line["serving"] = serving
    line["env"] = run_environment(params)
    line["hbm_copy_gbps"] = copy_bandwidth(dev)
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(frames, kw, args.cpu_seconds)
        line["cpu_baseline_1thread"] = cpu_baseline(frames, kw, args.cpu_seconds / 3, threads=1)
    if args.calibrate_copy:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE per dispatch
        # scale the counters of the estimator's kernels to bytes
        src = torch.ones(args.calibrate_copy << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = src.numel()
    est.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
