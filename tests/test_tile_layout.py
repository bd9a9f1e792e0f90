"""Host logic of the edge-tile layout shared by PageRank's pull superstep and
its reverse pass (csrc/tiles.h), checked on the CPU: a host-only driver built
with hipcc prints the layout, and every field is compared with its plain
definition restated here (row-start bitmap, first row of each tile, rows
spanning tiles), on degree sequences that end on, just before and just after
tile boundaries, rows longer than several tiles, ragged tails and empty
graphs."""
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1503_07241_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def tile_edges():
    text = open(os.path.join(CSRC, "tiles.h")).read()
    return int(re.search(r"constexpr int kRounds = (\d+);", text).group(1)) * 256


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("tiles") / "tile_layout")
    cmd = [HIPCC if os.path.exists(HIPCC) else "hipcc", "--offload-arch=gfx950", "-O1",
           "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", CSRC, os.path.join(ROOT, "tests", "tile_layout_main.hip"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


def run_driver(exe, deg):
    noff = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    n, m = len(deg), int(noff[-1])
    inp = "%d %d\n%s\n" % (n, m, " ".join(map(str, noff)))
    r = subprocess.run([exe], input=inp, capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    lines = r.stdout.split("\n")
    rows, ntiles, mpad = map(int, lines[0].split())
    starts = [int(x) for x in lines[1].split()]
    tile_row = [int(x) for x in lines[2].split()]
    cross = [int(x) for x in lines[3].split()]
    return noff, m, (rows, ntiles, mpad, starts, tile_row, [tuple(cross[i:i + 3])
                                                             for i in range(0, len(cross), 3)])


def reference(noff, n, m, kt):
    """The layout by definition: rows with edges are the labels [0, rows)."""
    deg = np.diff(noff)
    rows = int(np.argmax(deg == 0)) if (deg == 0).any() else n
    ntiles = -(-m // kt)
    mpad = ntiles * kt
    bits = np.zeros(mpad // 32 * 32 + 32, dtype=bool)
    bits[noff[:rows]] = True
    bits[m] = True
    starts = [int(sum(1 << i for i in range(32) if bits[32 * wd + i]))
              for wd in range(mpad // 32 + 1)]
    # the row holding edge t * kt
    tile_row = [int(np.searchsorted(noff[1:rows + 1], t * kt, side="right")) for t in range(ntiles)]
    cross = [(u, int(noff[u] // kt), int((noff[u + 1] - 1) // kt)) for u in range(rows)
             if noff[u] // kt != (noff[u + 1] - 1) // kt]
    return rows, ntiles, mpad, starts, tile_row, cross


def cases(kt):
    rng = np.random.default_rng(3)
    pl = np.sort(np.minimum((rng.pareto(1.2, 3000) * 3 + 1).astype(int), 9000))[::-1]
    return {
        "empty": [0, 0, 0, 0, 0],
        "one_long_row": [5 * kt + 17],
        "rows_of_exactly_one_tile": [kt, kt, kt],
        "end_before_after_boundary": sorted([kt - 1, 2, kt + 1, kt - 3, 3, 1], reverse=True) + [0, 0],
        "ragged_last_tile": [700, 300, 25, 1] + [0] * 4,
        "exact_fill": [kt // 2] * 4,
        "power_law": list(pl) + [0] * 500,
    }


@pytest.mark.parametrize("name", list(cases(1024)))
def test_tile_layout_matches_definition(driver, name):
    kt = tile_edges()
    deg = cases(kt)[name]
    noff, m, got = run_driver(driver, deg)
    assert got == reference(noff, len(deg), m, kt)
