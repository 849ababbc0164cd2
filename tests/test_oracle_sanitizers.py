"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code, gcc): synthetic frames, a blank frame and a tiny frame run through the
whole pipeline with every diagnostic fatal, and the results equal the
regular build's."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2210_14771_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    out = tmp_path_factory.mktemp("san") / "driver"
    cmd = ["gcc", "-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "oracle"),
           os.path.join(HERE, "csrc", "oracle_sanitize_driver.c"),
           os.path.join(ROOT, "oracle", "ca_oracle.c"), "-lm", "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail("sanitizer build failed:\n" + r.stderr)
    return out


def _run(driver, tmp_path, frames, attempts, nh, nv):
    h, w = frames[0].shape[:2]
    files = []
    for i, f in enumerate(frames):
        path = tmp_path / f"f{i}.rgb"
        path.write_bytes(np.ascontiguousarray(f).tobytes())
        files.append(str(path))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(driver), str(w), str(h), str(attempts), str(nh), str(nv), *files],
                       capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    return [tuple(int(v) for v in line.split()) for line in r.stdout.split("\n") if line]


def test_oracle_clean_under_sanitizers(driver, tmp_path):
    frames, _ = synth.make_batch(synth.SMALL_640x480, 3)
    blank = np.zeros_like(frames[0])
    got = _run(driver, tmp_path, list(frames) + [blank], 256, 16, 16)
    p = oracle.params(n_hstrips=16, n_vstrips=16, attempts=256)
    for i, f in enumerate(list(frames) + [blank]):
        res, _ = oracle.estimate(f, p, 6 + i, with_points=True)
        assert got[i] == (int(res["valid"]), int(res["inliers"]), int(res["n_points"]))


def test_tiny_odd_frame_clean_under_sanitizers(driver, tmp_path):
    rng = np.random.default_rng(0)
    tiny = rng.integers(0, 256, (17, 19, 3), dtype=np.uint8)
    got = _run(driver, tmp_path, [tiny], 64, 4, 4)
    assert len(got) == 1
