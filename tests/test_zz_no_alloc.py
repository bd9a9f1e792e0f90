"""The allocation-free PageRank entry point (gm_pagerank_noalloc) through the
C ABI against gm_run_vertex_program with GM_PROG_PAGERANK: two calls in a
row on one GPU (the second on a smaller graph, so the shared scratch array
holds the first call's larger contents), each within the PageRank tolerance
of the regular entry point (the same kernels in the same order give equal
bits), plus its error cases."""
import ctypes

import numpy as np
import pytest
import torch

import graphgen as gg
import paper_1503_07241_amd as gm
from paper_1503_07241_amd import _lib

pytestmark = pytest.mark.gpu
DEV = "cuda"
R = 0.15


def noalloc(g, iters, rank):
    st = _lib.load().gm_pagerank_noalloc(g.handle, ctypes.c_float(R), iters, rank.data_ptr(),
                                         torch.cuda.current_stream().cuda_stream)
    return st


def regular(g, n, iters):
    rank = torch.ones(n, dtype=torch.float32, device=DEV)
    gm.run_vertex_program(g, gm.GM_PROG_PAGERANK, None, iters, rank)
    return rank


def test_noalloc_pagerank_two_calls_second_smaller():
    for scale, seed, w in ((16, 1, False), (11, 7, True)):
        n, s, d = gg.rmat(scale, seed=seed)
        wf = gg.weights_f32(s, d, 13, 0.5, 1.5) if w else None
        g = gm.Graph.from_coo(n, s, d, w=wf)
        g.prepare(gm.GM_PROG_PAGERANK)
        rank = torch.ones(n, dtype=torch.float32, device=DEV)
        assert noalloc(g, 20, rank) == _lib.GM_OK, _lib.load().gm_last_error()
        ref = regular(g, n, 20)
        torch.cuda.synchronize()
        err = float(((rank.double() - ref.double()).abs() / ref.double()).max())
        assert err <= 1e-5, err
        assert torch.equal(rank, ref)


def test_noalloc_pagerank_errors():
    n, s, d = gg.rmat(10)
    g = gm.Graph.from_coo(n, s, d)
    rank = torch.ones(n, dtype=torch.float32, device=DEV)
    assert noalloc(g, 20, rank) == _lib.GM_ESTATE  # layout not built: nothing is allocated
    g.prepare(gm.GM_PROG_PAGERANK)
    assert noalloc(g, 0, rank) == _lib.GM_EINVAL
    # a graph whose vectors exceed the fixed array: refused with a clear error
    big = 6_000_000
    gb = gm.Graph.from_coo(big, np.array([0, 1], np.int32), np.array([1, 2], np.int32))
    gb.prepare(gm.GM_PROG_PAGERANK)
    rb = torch.ones(big, dtype=torch.float32, device=DEV)
    assert noalloc(gb, 20, rb) == _lib.GM_EUNSUPPORTED
    assert b"scratch" in _lib.load().gm_last_error()
