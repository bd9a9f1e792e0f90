"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the oracle (oracle/oracle.c, every entry point, through
tests/oracle_sanitize_main.c) and the library's Matrix Market reader
(csrc/mtx.hip, through tests/mtx_sanitize_main.cpp, on valid, malformed and
adversarial files; its statuses and edge lists must match the library's).
A memory error, a leak or undefined arithmetic ends the run with a non-zero
status."""
import os
import shutil
import subprocess

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


MTX_FILES = {
    "weighted": "%%MatrixMarket matrix coordinate integer general\n% comment\n5 5 3\n"
                "1 2 7\n\n3 2 1\n5 5 9\n",
    "symmetric": "%%MatrixMarket matrix coordinate pattern symmetric\n3 3 3\n2 1\n3 2\n3 3\n",
    "real": "%%MatrixMarket matrix coordinate real general\n2 4 2\n1 4 0.25\n2 1 -1.5e1\n",
    "empty": "",
    "banner_only": "%%MatrixMarket matrix coordinate pattern general\n",
    "short": "%%MatrixMarket matrix coordinate pattern general\n2 2 5\n1 1\n",
    "outside": "%%MatrixMarket matrix coordinate pattern general\n2 2 1\n3 1\n",
    "zero_index": "%%MatrixMarket matrix coordinate pattern general\n2 2 1\n0 1\n",
    "nan_value": "%%MatrixMarket matrix coordinate integer general\n2 2 1\n1 2 nan\n",
    "inf_value": "%%MatrixMarket matrix coordinate integer general\n2 2 1\n1 2 inf\n",
    "huge_value": "%%MatrixMarket matrix coordinate integer general\n2 2 1\n1 2 1e300\n",
    "huge_index": "%%MatrixMarket matrix coordinate pattern general\n2 2 1\n"
                  "99999999999999999999 1\n",
    "huge_size": "%%MatrixMarket matrix coordinate pattern general\n"
                 "99999999999999999999 2 1\n1 1\n",
    "negative_size": "%%MatrixMarket matrix coordinate pattern general\n-2 2 1\n1 1\n",
    "no_value": "%%MatrixMarket matrix coordinate real general\n2 2 1\n1 2\n",
    "long_line": "%%MatrixMarket matrix coordinate pattern general\n3 3 2\n1 2" + " " * 3000
                 + "\n2 3\n",
    "long_banner": "%%MatrixMarket " + "x" * 5000 + "\n1 1 0\n",
    "garbage": "\x00\xff%%MatrixMarket\n\x01\x02\n",
}


def test_mtx_reader_under_sanitizers(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    from paper_1503_07241_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libgm.so is not built")
    import paper_1503_07241_amd as gm
    exe = str(tmp_path / "mtx_san")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           os.path.join(CSRC, "mtx.hip"), os.path.join(ROOT, "tests", "mtx_sanitize_main.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    paths = []
    for name, text in MTX_FILES.items():
        p = tmp_path / (name + ".mtx")
        p.write_bytes(text.encode("latin-1"))
        paths.append(str(p))
    paths.append(str(tmp_path / "missing.mtx"))
    r = subprocess.run([exe] + paths, capture_output=True, text=True, timeout=120, env=ENV)
    assert r.returncode == 0, r.stderr[-4000:]
    lines = r.stdout.split("\n")[:len(paths)]
    assert len(lines) == len(paths)
    for path, line in zip(paths, lines):
        st, n, m, _ = (int(x) for x in line.split())
        try:
            nn, s, d, w = gm.read_mtx(path)
            want = (0, nn, len(s))
        except gm.GmError as e:
            want = (e.status,)
        assert (st, n, m)[:len(want)] == want, (path, line, want)
    assert [int(x) for x in lines[0].split()[:3]] == [0, 5, 3]
    assert [int(x) for x in lines[1].split()[:3]] == [0, 3, 5]
