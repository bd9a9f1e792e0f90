"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the oracle (oracle/oracle.c, every entry point, through
tests/oracle_sanitize_main.c) and the library's host-side edge-tile layout
builder (csrc/tiles.h, through tests/tile_layout_main.hip, device code not
instrumented and not run). A memory error, a leak or undefined arithmetic
ends the run with a non-zero status."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1503_07241_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "orc_san")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "tests", "oracle_sanitize_main.c"),
           os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stderr[-4000:]


def test_tile_layout_builder_under_sanitizers(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "tile_layout_san")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", CSRC, os.path.join(ROOT, "tests", "tile_layout_main.hip"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    rng = np.random.default_rng(7)
    degs = [np.zeros(5, np.int64), np.array([0], np.int64), np.array([1023, 1, 1024, 1025]),
            np.array([5000, 3, 0, 0]), rng.integers(0, 50, 3000)]
    for deg in degs:
        deg = np.sort(deg)[::-1]  # rows with edges first, as the layouts order them
        noff = np.concatenate([[0], np.cumsum(deg)])
        inp = "%d %d\n%s\n" % (len(deg), int(noff[-1]), " ".join(map(str, noff)))
        r = subprocess.run([exe], input=inp, capture_output=True, text=True, timeout=120,
                           env=ENV)
        assert r.returncode == 0, r.stderr[-4000:]
