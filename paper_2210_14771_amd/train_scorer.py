"""Train the learned strip scorer on the GPU (Section 2.2.4, training).

The paper trains its CNN with a soft binary cross entropy against edge maps
blurred with a Gaussian of sigma 3, by SGD, and keeps the model with the
best validation loss.  Here every step draws a fresh batch of synthetic
1080p frames (plain and hard, device-rendered), cuts the 8-line strips of
random rows and columns into windows, labels each strip pixel with the soft
edge label of the ground-truth circle, and runs the library's own forward,
backward and SGD kernels (ca_cnn_gradients, ca_cnn_sgd_step).  Nothing of
the step runs on the host except drawing the frames' parameters.

    python -m paper_2210_14771_amd.train_scorer --out paper_2210_14771_amd/models

(the committed model: these defaults, 3125 steps of 64 frames = 200,000
frames, 83 s on one MI355X; its log is models/scorer_1d_training.json).
With --model 2d the same loop trains the paper's own network (three 3x3
convolutions on RGBXY bands seven lines thick) through ca_cnn2d_gradients
and ca_cnn2d_sgd_step, its input normaliser taken from the colour
statistics of rendered training frames; at the 1-D network's rate it barely
moves, at lr 0.3 it diverges once it starts fitting edges, so its default is
lr 0.3 with each step's gradient clipped to a global norm of 0.0065 (about
twice the early norm): models/scorer_2d.npy, 200,000 frames, 90 s.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

from . import api, synth, synth_gpu

LAYERS = [(24, 16, 5), (16, 32, 5), (32, 32, 5), (32, 16, 5), (16, 1, 1)]
MODEL_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "models")
MODEL_FILE = "scorer_1d.npy"
# the paper's own network: three 3x3 convolutions 5 -> 8 -> 16 -> 32, 1x1 -> 1
LAYERS_2D = [(5, 8, 9), (8, 16, 9), (16, 32, 9), (32, 1, 1)]
MODEL_FILE_2D = "scorer_2d.npy"
N_PARAMS_2D = 6215


def init_params(seed: int, out_bias: float = -4.0) -> np.ndarray:
    """Weights and biases uniform in +-1/sqrt(fan_in), in model-file order
    (float32); the output bias starts at `out_bias` (edge pixels are rare,
    so the network starts by predicting a small probability everywhere)."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co, k in LAYERS:
        b = 1.0 / math.sqrt(ci * k)
        parts.append(rng.uniform(-b, b, co * ci * k).astype(np.float32))
        parts.append(rng.uniform(-b, b, co).astype(np.float32))
    parts[-1][:] = out_bias
    return np.concatenate(parts)


def init_params_2d(seed: int, mean, std, out_bias: float = -4.0) -> np.ndarray:
    """The 2-D network's model-file vector: the input normaliser (mean and
    1 / std per colour channel), then weights and biases uniform in
    +-1/sqrt(fan_in) (float32); the output bias starts at `out_bias`."""
    rng = np.random.default_rng(seed)
    parts = [np.asarray(mean, dtype=np.float32),
             (1.0 / np.asarray(std, dtype=np.float64)).astype(np.float32)]
    for ci, co, k in LAYERS_2D:
        b = 1.0 / math.sqrt(ci * k)
        parts.append(rng.uniform(-b, b, co * ci * k).astype(np.float32))
        parts.append(rng.uniform(-b, b, co).astype(np.float32))
    parts[-1][:] = out_bias
    v = np.concatenate(parts)
    assert v.size == N_PARAMS_2D
    return v


def load_model(path: str | None = None) -> np.ndarray:
    """The committed trained scorer (float32, model-file order)."""
    path = path or os.path.join(MODEL_DIR, MODEL_FILE)
    p = np.load(path, allow_pickle=False)
    if p.dtype != np.float32 or p.shape != (12273,):
        raise ValueError(f"{path}: not a scorer model")
    return p


def load_model_2d(path: str | None = None) -> np.ndarray:
    """The committed trained 2-D scorer (float32, model-file order)."""
    path = path or os.path.join(MODEL_DIR, MODEL_FILE_2D)
    p = np.load(path, allow_pickle=False)
    if p.dtype != np.float32 or p.shape != (N_PARAMS_2D,):
        raise ValueError(f"{path}: not a 2-D scorer model")
    return p


def colour_statistics(recs) -> tuple[np.ndarray, np.ndarray]:
    """Per-channel mean and standard deviation of the pixels of rendered
    training frames (the paper normalises by these over its training set)."""
    import torch
    frames = synth_gpu.DeviceRecipes(recs).render_frames()
    x = frames.reshape(-1, 3).to(torch.float64)
    mean = x.mean(dim=0)
    std = x.std(dim=0)
    return mean.cpu().numpy(), std.cpu().numpy()


def draw_frames(stream_plain: int, stream_hard: int, first: int, n: int, hard_frac: float,
                rng: np.random.Generator):
    """n frame recipes: a hard_frac share from the hard stream, the rest plain."""
    recs = []
    for i in range(first, first + n):
        if rng.uniform() < hard_frac:
            recs.append(synth_gpu.draw_recipe(synth.HARD_1080p, stream_hard, i, True))
        else:
            recs.append(synth_gpu.draw_recipe(synth.HD_1080p, stream_plain, i, False))
    return recs


def draw_windows(recs, strips_per_frame: int, rng: np.random.Generator) -> np.ndarray:
    """Windows tiling strips through random rows and columns of every frame."""
    out = []
    for f, rc in enumerate(recs):
        w, h = rc.spec.width, rc.spec.height
        for _ in range(strips_per_frame):
            hz = bool(rng.uniform() < 0.5)
            line = int(rng.integers(0, h if hz else w))
            out.append(synth_gpu.strip_windows(f, hz, line, w if hz else h))
    return np.concatenate(out)


def positions_inside(desc: np.ndarray, recs) -> int:
    """Central window positions that lie inside their strips."""
    L = np.array([recs[f].spec.width if hz else recs[f].spec.height for f, hz, _, _ in desc])
    lo = np.maximum(desc[:, 3] + 8, 0)
    hi = np.minimum(desc[:, 3] + 120, L)
    return int(np.maximum(hi - lo, 0).sum())


def window_geometry(desc: np.ndarray, recs) -> np.ndarray:
    """int32 [n, 8] (horizontal, line, start, width, height, 0, 0, 0) of the
    windows of desc (frame, horizontal, line, start)."""
    g = np.zeros((len(desc), 8), dtype=np.int32)
    g[:, 0] = desc[:, 1]
    g[:, 1] = desc[:, 2]
    g[:, 2] = desc[:, 3]
    g[:, 3] = [recs[f].spec.width for f in desc[:, 0]]
    g[:, 4] = [recs[f].spec.height for f in desc[:, 0]]
    return g


# the handcrafted pipeline that labels frames for --labels pseudo (the
# headline configuration)
PSEUDO_PARAMS = dict(n_hstrips=32, n_vstrips=32, ransac_attempts=1024)


def pseudo_targets(est, dev, desc: np.ndarray, wt):
    """Soft edge labels of the windows from the handcrafted pipeline's own
    circle of each frame (the paper trains on such pseudo-labels, Section
    2.2.4): the library's estimate on the rendered frames, whose results equal
    the oracle's; frames it finds no valid circle in get no edge label.
    Returns (targets, share of frames with a valid circle)."""
    import torch
    frames = dev.render_frames()
    n = frames.shape[0]
    raw = est.estimate_area(frames, api.default_params(**PSEUDO_PARAMS), list(range(n))).raw
    cx, cy, r = (raw[:, k].view(torch.float32) for k in range(3))
    valid = (raw[:, 6] != 0).to(torch.float32)
    d = torch.from_numpy(np.ascontiguousarray(desc, dtype=np.int64)).to(frames.device)
    f, hz = d[:, 0], d[:, 1] != 0
    line = d[:, 2].to(torch.float32)[:, None]
    p = (d[:, 3][:, None] + 8 + torch.arange(112, device=frames.device)[None, :]).to(torch.float32)
    x = torch.where(hz[:, None], p, line)
    y = torch.where(hz[:, None], line, p)
    rho = torch.sqrt((x - cx[f][:, None]) ** 2 + (y - cy[f][:, None]) ** 2)
    t = torch.exp(-(rho - r[f][:, None]) ** 2 / 18.0) * valid[f][:, None]
    t = torch.where(wt > 0, t, torch.zeros_like(t))
    return t.contiguous(), float(valid.mean().item())


class Batch:
    def __init__(self, recs, desc, edge_boost, kind: str = "1d", labels: str = "truth", est=None):
        import torch
        self.dev = synth_gpu.DeviceRecipes(recs)
        self.win, self.rng, self.tgt, self.wt = self.dev.render_windows(desc, edge_boost)
        self.scale = 1.0 / max(positions_inside(desc, recs), 1)
        self.kind = kind
        self.geom = (torch.from_numpy(window_geometry(desc, recs)).to(self.win.device)
                     if kind == "2d" else None)
        self.pseudo_valid = None
        if labels == "pseudo":
            self.tgt, self.pseudo_valid = pseudo_targets(est, self.dev, desc, self.wt)

    def tensors(self):
        if self.kind == "2d":
            return self.win, self.geom, self.rng, self.tgt, self.wt
        return self.win, self.rng, self.tgt, self.wt


def train(steps: int = 3125, frames_per_step: int = 64, strips_per_frame: int = 16,
          lr: float = 0.05, momentum: float = 0.9, warmup: int = 100, hard_frac: float = 0.5,
          edge_boost: float = 0.0, seed: int = 0, valid_every: int = 50, valid_frames: int = 128,
          log=print, est: api.Estimator | None = None, kind: str = "1d",
          labels: str = "truth", clip: float = 0.0):
    """Returns (best master weights, log dict).  kind "1d": the 1-D strip
    network; "2d": the paper's 3x3 network on RGBXY bands.  labels "truth":
    the generator's circle; "pseudo": the handcrafted pipeline's circle of
    each training frame (validation keeps the true labels).  clip > 0 scales
    a step's gradient down to that global norm when it is larger."""
    import torch
    own = est is None
    est = est or api.Estimator(0)
    rng = np.random.default_rng(seed)
    info_extra = {}
    if kind == "2d":
        srng = np.random.default_rng(seed + 2)
        mean, std = colour_statistics(draw_frames(synth_gpu.TRAIN_PLAIN, synth_gpu.TRAIN_HARD,
                                                  10 ** 7, 32, hard_frac, srng))
        info_extra = {"colour_mean": [float(v) for v in mean],
                      "colour_std": [float(v) for v in std], "statistics_frames": 32}
        est.set_model_2d(init_params_2d(seed, mean, std))
        grads_of, sgd, get_model = est.cnn2d_gradients, est.cnn2d_sgd_step, est.get_model_2d
    else:
        est.set_model(init_params(seed))
        grads_of, sgd, get_model = est.cnn_gradients, est.cnn_sgd_step, est.get_model
    vrng = np.random.default_rng(seed + 1)
    vrecs = draw_frames(synth_gpu.VALID_PLAIN, synth_gpu.VALID_HARD, 0, valid_frames, hard_frac,
                        vrng)
    valid = Batch(vrecs, draw_windows(vrecs, strips_per_frame, vrng), edge_boost, kind)
    history = []
    pseudo_valid = []
    last_norm = 0.0
    best = (math.inf, None, -1)
    t0 = time.time()
    frames_seen = 0
    for step in range(steps + 1):
        if step % valid_every == 0 or step == steps:
            _, vloss = grads_of(*valid.tensors(), valid.scale)
            v = float(vloss.item())
            history.append({"step": step, "valid_loss": v, "frames": frames_seen,
                            "seconds": round(time.time() - t0, 1)})
            if step > 0:
                history[-1]["last_grad_norm"] = last_norm
            log(f"step {step} valid loss {v:.5f} frames {frames_seen} "
                f"grad {last_norm:.3g} ({time.time() - t0:.0f} s)")
            if v < best[0]:
                best = (v, get_model(), step)
        if step == steps:
            break
        recs = draw_frames(synth_gpu.TRAIN_PLAIN, synth_gpu.TRAIN_HARD, step * frames_per_step,
                           frames_per_step, hard_frac, rng)
        b = Batch(recs, draw_windows(recs, strips_per_frame, rng), edge_boost, kind, labels, est)
        if b.pseudo_valid is not None:
            pseudo_valid.append(b.pseudo_valid)
        grad, loss = grads_of(*b.tensors(), b.scale)
        if clip > 0:
            # clipped on the device (no host round trip): g *= min(1, clip / |g|)
            norm = torch.linalg.vector_norm(grad)
            grad.mul_(torch.clamp(clip / (norm + 1e-30), max=1.0))
        if step < warmup:
            lr_t = lr * (step + 1) / warmup
        else:
            lr_t = 0.5 * lr * (1.0 + math.cos(math.pi * (step - warmup) / max(steps - warmup, 1)))
        sgd(grad, lr_t, momentum)
        if (step + 1) % valid_every == 0:
            last_norm = float(torch.linalg.vector_norm(grad).item())
        frames_seen += frames_per_step
        if step % 25 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    if pseudo_valid:
        info_extra["pseudo_label_valid_frac"] = float(np.mean(pseudo_valid))
    info = {"model": kind, "labels": labels, "steps": steps, "frames": frames_seen, "frames_per_step": frames_per_step,
            "strips_per_frame": strips_per_frame, "lr": lr, "momentum": momentum,
            "warmup": warmup, "hard_frac": hard_frac, "edge_boost": edge_boost, "seed": seed,
            "clip": clip,
            "best_step": best[2], "best_valid_loss": best[0], "history": history,
            "seconds": round(time.time() - t0, 1), **info_extra}
    if own:
        est.close()
    return best[1], info


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--steps", type=int, default=3125)
    ap.add_argument("--frames-per-step", type=int, default=64)
    ap.add_argument("--strips-per-frame", type=int, default=16)
    ap.add_argument("--lr", type=float, default=None,
                    help="peak learning rate (default 0.05 for 1d, 0.3 for 2d)")
    ap.add_argument("--momentum", type=float, default=0.9)
    ap.add_argument("--hard-frac", type=float, default=0.5)
    ap.add_argument("--edge-boost", type=float, default=0.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--valid-every", type=int, default=50)
    ap.add_argument("--out", default=MODEL_DIR)
    ap.add_argument("--model", choices=["1d", "2d"], default="1d",
                    help="1d: the 1-D strip network; 2d: the paper's 3x3 network on RGBXY bands")
    ap.add_argument("--labels", choices=["truth", "pseudo"], default="truth",
                    help="truth: the generator's circle; pseudo: the handcrafted pipeline's")
    ap.add_argument("--name", default=None, help="model file name (default per model kind)")
    ap.add_argument("--clip", type=float, default=None,
                    help="clip each step's gradient to this global norm (0: off; default off "
                         "for 1d, 0.0065 for 2d)")
    a = ap.parse_args()
    if a.lr is None:
        a.lr = 0.05 if a.model == "1d" else 0.3
    if a.clip is None:
        # the 2-D network diverges at this rate once it starts fitting edges
        # unless its steps are bounded: about twice the early gradient norm
        a.clip = 0.0 if a.model == "1d" else 0.0065
    params, info = train(a.steps, a.frames_per_step, a.strips_per_frame, a.lr, a.momentum,
                         hard_frac=a.hard_frac, edge_boost=a.edge_boost, seed=a.seed,
                         valid_every=a.valid_every,
                         log=lambda s: print(s, flush=True), kind=a.model, labels=a.labels, clip=a.clip)
    os.makedirs(a.out, exist_ok=True)
    name = a.name or (MODEL_FILE if a.model == "1d" else MODEL_FILE_2D)
    np.save(os.path.join(a.out, name), params.astype(np.float32), allow_pickle=False)
    with open(os.path.join(a.out, name.replace(".npy", "_training.json")), "w") as f:
        json.dump(info, f, indent=1)
    print(json.dumps({k: v for k, v in info.items() if k != "history"}), flush=True)


if __name__ == "__main__":
    main()
