"""The library's host core (ca_api.cpp, ca_server.cpp) under AddressSanitizer
and UndefinedBehaviorSanitizer, built with g++ against a stand-in HIP runtime
(tests/csrc/hip_stub) and driven without a GPU by tests/csrc/host_harness.cpp:
the batch API over mixed shapes, plan eviction, every schedule option and
graphs; the serving loop fed a whole backlog at once and then in real
time by a second server on the same context (per scorer, as the serving
benchmark runs them, in the other order), with more stream shapes than
frames per batch, and with streams waiting for memory.  The stand-in kernels check that every frame byte, strip table and
output they would touch lies inside its allocation, and any synchronous
runtime call inside ca_server_step aborts the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2210_14771_amd", "csrc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = tmp_path_factory.mktemp("hostsan") / "host_harness"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall",
           "-I", os.path.join(HERE, "csrc", "hip_stub"), "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, os.path.join(HERE, "csrc", "host_harness.cpp"),
           os.path.join(CSRC, "ca_api.cpp"), os.path.join(CSRC, "ca_server.cpp"), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail("harness build failed:\n" + r.stderr[-4000:])
    return out


def _run(harness, *args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(harness), *args], capture_output=True, text=True, env=env,
                       timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    return r.stdout


def test_batch_api(harness):
    out = _run(harness, "batch_api")
    assert "ok batch api" in out


def test_streams_wait_for_memory(harness):
    assert "ok memory wait" in _run(harness, "memory_wait")


def test_more_stream_shapes_than_batch_frames(harness):
    out = _run(harness, "few_slots")
    assert out.count("ok one frame per batch") == 2 and "ok pipelined sub-batches" in out


def test_serve_bench_sequence_never_blocks(harness):
    # two simulated seconds of 48 streams, a backlog server then a real-time
    # one per scorer; no call inside step may block
    out = _run(harness, "serve_sequence", "2.0")
    for name in ("plain warm-up", "plain realtime", "learned warm-up", "learned realtime"):
        assert f"ok {name}" in out, name
