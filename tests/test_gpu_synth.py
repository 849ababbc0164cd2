"""The device renderer of synthetic frames (an input generator): it renders
the image model the CPU renderer defines, windows cut from a rendered frame
equal windows rendered directly, and the soft edge labels follow their
closed form."""
import numpy as np
import pytest

from oracle import cnn
from paper_2210_14771_amd import synth, synth_gpu

from gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _recipes(n, wl=synth.HD_1080p, stream=synth_gpu.VALID_PLAIN, hard=False):
    return [synth_gpu.draw_recipe(wl, stream, i, hard) for i in range(n)]


@pytest.mark.parametrize("wl", [synth.SMALL_640x480, synth.HD_1080p], ids=["640x480", "1080p"])
def test_noise_free_frames_match_cpu_image_model(torch_dev, wl):
    torch = torch_dev
    recs = _recipes(6, wl)
    say(f"noise-free frames {wl.width}x{wl.height}")
    dev = synth_gpu.DeviceRecipes(recs, flags=synth_gpu.NO_NOISE)
    frames = dev.render_frames().cpu().numpy()
    kinds = set()
    for i, rc in enumerate(recs):
        ref = np.clip(np.rint(synth.render_noise_free(rc.spec, rc.grids)), 0, 255)
        d = np.abs(frames[i].astype(np.int32) - ref.astype(np.int32))
        # float32 rounding may move a value across a .5 boundary, nothing more
        assert d.max() <= 1, (i, d.max())
        assert (d > 0).mean() < 1e-3, (i, (d > 0).mean())
        kinds.add(rc.spec.kind)
    if wl.mix[2] > 0:
        assert synth.KIND_NOBORDER in kinds and len(kinds) >= 2


def test_windows_equal_crops_of_rendered_frames(torch_dev):
    torch = torch_dev
    recs = _recipes(3, synth.HD_1080p, synth_gpu.VALID_HARD, hard=True)
    dev = synth_gpu.DeviceRecipes(recs)
    say("windows vs frames")
    frames = dev.render_frames().cpu().numpy()
    desc = np.concatenate([synth_gpu.strip_windows(0, True, 3, 1920),
                           synth_gpu.strip_windows(1, False, 1917, 1080),
                           synth_gpu.strip_windows(2, True, 700, 1920)])
    win, rng_, tgt, wt = [t.cpu().numpy() for t in dev.render_windows(desc, edge_boost=2.0)]
    for i, (f, hz, line, start) in enumerate(desc):
        img = frames[f]
        H, W = img.shape[:2]
        L, E = (W, H) if hz else (H, W)
        lines = [min(max(line + o, 0), E - 1) for o in range(-3, 5)]
        strip = img[lines] if hz else img[:, lines].transpose(1, 0, 2)     # [8, L, 3]
        lo, hi = max(0, -start), min(128, L - start)
        assert tuple(rng_[i]) == (lo, hi)
        np.testing.assert_array_equal(win[i][:, lo:hi], strip[:, start + lo:start + hi])
        spec = recs[f].spec
        full = cnn.edge_target(L, line, bool(hz), (spec.cx, spec.cy, spec.r))
        for j in range(112):
            p = start + 8 + j
            if 0 <= p < L:
                assert abs(tgt[i, j] - full[p]) <= 2e-4   # float32 circle and distance
                assert abs(wt[i, j] - (1.0 + 2.0 * tgt[i, j])) <= 1e-5
            else:
                assert wt[i, j] == 0.0


def test_border_noise_statistics(torch_dev):
    """Border pixels far from the circle: mean 6 and the drawn sigma (when
    clipping at 0 is negligible), content noise sigma 2 per channel."""
    torch = torch_dev
    wl = synth.Workload(9, 640, 480, 1, (0.0, 1.0, 0.0), (2.0, 2.0), (1.0, 1.0), (0.0, 0.0),
                        None, 8, 8, 64)
    recs = [synth_gpu.draw_recipe(wl, 120, i, False) for i in range(4)]
    frames = synth_gpu.DeviceRecipes(recs).render_frames().cpu().numpy().astype(np.float64)
    quiet = synth_gpu.DeviceRecipes(recs, flags=synth_gpu.NO_NOISE).render_frames()
    quiet = quiet.cpu().numpy().astype(np.float64)
    for i, rc in enumerate(recs):
        s = rc.spec
        yy, xx = np.mgrid[0:s.height, 0:s.width]
        rho = np.hypot(xx - s.cx, yy - s.cy)
        far = rho > s.r + 6 * s.blur_sigma
        b = frames[i][far][:, 0]
        assert abs(b.mean() - 6.0) < 0.15 and abs(b.std() - 2.0) < 0.15, (b.mean(), b.std())
        # content pixels away from the clipping limits
        inner = (rho < s.r - 6 * s.blur_sigma)[..., None] & (quiet[i] > 12) & (quiet[i] < 243)
        resid = (frames[i] - quiet[i])[inner]
        assert abs(resid.std() - np.sqrt(4.0 + 1.0 / 12.0)) < 0.1, resid.std()
