"""Matrix Market input (App. A, ReadMTX) through the C ABI's host-only
reader: hand-written files, symmetric expansion, value types, and the errors
of malformed input. The GPU test in test_gpu_graph.py builds graphs from
such files and checks programs against the oracle."""
import os

import numpy as np
import pytest

import paper_1503_07241_amd as gm
from paper_1503_07241_amd import _lib

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libgm.so is not built")
    return _lib.load()


def test_weighted_general(lib):
    n, s, d, w = gm.read_mtx(os.path.join(HERE, "small_weighted.mtx"))
    assert n == 5
    assert s.tolist() == [0, 0, 2, 1, 3, 4]
    assert d.tolist() == [1, 2, 1, 3, 4, 4]
    assert w.dtype == np.uint32 and w.tolist() == [7, 2, 1, 4, 3, 9]


def test_symmetric_pattern(lib):
    n, s, d, w = gm.read_mtx(os.path.join(HERE, "small_symmetric.mtx"))
    assert n == 3 and w is None
    # off-diagonal entries in both directions, the diagonal entry once
    assert sorted(zip(s.tolist(), d.tolist())) == [(0, 1), (1, 0), (1, 2), (2, 1), (2, 2)]


def test_real_values_and_rectangular(tmp_path, lib):
    p = tmp_path / "r.mtx"
    p.write_text("%%MatrixMarket matrix coordinate real general\n2 4 2\n1 4 0.25\n2 1 -1.5e1\n")
    n, s, d, w = gm.read_mtx(str(p))
    assert n == 4 and s.tolist() == [0, 1] and d.tolist() == [3, 0]
    assert w.dtype == np.float32 and w.tolist() == [0.25, -15.0]


@pytest.mark.parametrize("text,status", [
    ("%%MatrixMarket matrix array real general\n2 2\n1\n2\n3\n4\n", _lib.GM_EINVAL),
    ("%%MatrixMarket matrix coordinate complex general\n2 2 1\n1 1 1 0\n", _lib.GM_EUNSUPPORTED),
    ("%%MatrixMarket matrix coordinate pattern hermitian\n2 2 1\n1 1\n", _lib.GM_EUNSUPPORTED),
    ("%%MatrixMarket matrix coordinate pattern general\n2 2 2\n1 1\n", _lib.GM_EINVAL),
    ("%%MatrixMarket matrix coordinate pattern general\n2 2 1\n3 1\n", _lib.GM_EINVAL),
    ("%%MatrixMarket matrix coordinate integer general\n2 2 1\n1 2 -4\n", _lib.GM_EUNSUPPORTED),
    ("%%MatrixMarket matrix coordinate integer general\n2 2 1\n1 2\n", _lib.GM_EINVAL),
    ("not a matrix market file\n", _lib.GM_EINVAL),
])
def test_malformed_files(tmp_path, lib, text, status):
    p = tmp_path / "bad.mtx"
    p.write_text(text)
    with pytest.raises(gm.GmError) as e:
        gm.read_mtx(str(p))
    assert e.value.status == status


def test_missing_file_and_short_arrays(tmp_path, lib):
    with pytest.raises(gm.GmError) as e:
        gm.read_mtx(str(tmp_path / "none.mtx"))
    assert e.value.status == _lib.GM_EINVAL
    import ctypes
    n, m, wt = ctypes.c_int64(0), ctypes.c_int64(2), ctypes.c_int32(0)
    src = np.empty(2, np.int32)
    st = lib.gm_mtx_read(os.path.join(HERE, "small_weighted.mtx").encode(), ctypes.byref(n),
                         ctypes.byref(m), src.ctypes.data, None, None, ctypes.byref(wt))
    assert st == _lib.GM_EINVAL
