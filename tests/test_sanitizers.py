"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the trie builder with every device-image variant, the oracle's three
matchers, and the serving loop's ring placement.  Each is built into its own test binary with g++ / gcc (no GPU
code is compiled with a sanitizer); a memory or UB error aborts the run."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _run(cmd, tmp_path, name):
    exe = str(tmp_path / name)
    build = subprocess.run(cmd + ["-o", exe], capture_output=True, text=True)
    if build.returncode != 0 and "fsanitize" in build.stderr and "unrecognized" in build.stderr:
        pytest.skip("compiler without sanitizers")
    assert build.returncode == 0, build.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert run.returncode == 0, (run.stdout + run.stderr)[-4000:]
    assert "runtime error" not in run.stderr
    return run.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_builder_under_sanitizers(tmp_path):
    out = _run(["g++", "-std=c++17", *SAN, os.path.join(NATIVE, "sanitize_builder.cpp"),
                os.path.join(ROOT, "paper_1702_03657_amd", "csrc", "trie_build.cpp")],
               tmp_path, "sanitize_builder")
    assert "ok" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_sanitizers(tmp_path):
    out = _run(["gcc", "-std=gnu11", *SAN, os.path.join(NATIVE, "sanitize_oracle.c"),
                os.path.join(ROOT, "oracle", "oracle.c"), "-lpthread", "-lm"],
               tmp_path, "sanitize_oracle")
    assert "ok" in out


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_serving_ring_placement(tmp_path):
    """The serving loop's ring placement (the server's own host class) in a
    randomized simulation: arrivals, completions in any order, cancellations
    of queued requests, release in placement order; every ring byte is
    tracked, so an overlap, a budget overrun or a refused empty ring fails."""
    out = _run(["g++", "-std=c++17", *SAN, os.path.join(NATIVE, "ring_sim.cpp")],
               tmp_path, "ring_sim")
    assert "ok" in out and "wrapped" in out
