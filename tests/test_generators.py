"""Pins of the seeded input generators (no method arithmetic lives there)."""
import numpy as np
import pytest

import graphgen as gg


def test_rmat_range_and_determinism():
    n, s, d = gg.rmat(12, seed=7)
    assert n == 4096 and len(s) == 16 * 4096
    assert s.min() >= 0 and s.max() < n and d.min() >= 0 and d.max() < n
    _, s2, d2 = gg.rmat(12, seed=7)
    assert np.array_equal(s, s2) and np.array_equal(d, d2)
    _, s3, _ = gg.rmat(12, seed=8)
    assert not np.array_equal(s, s3)


@pytest.mark.parametrize("scale", [10, 14])
def test_rmat_quadrant_probabilities(scale):
    """Closed forms of the quadrant recursion: P(self-loop) = (a+d)^scale,
    P(src = 0) = (a+b)^scale, P(src bit l set) = c + d for every level."""
    a, b, c = gg.RMAT_A, gg.RMAT_B, gg.RMAT_C
    dd = 1 - a - b - c
    n, s, d = gg.rmat(scale)
    m = len(s)
    for p, count in [((a + dd) ** scale, int((s == d).sum())), ((a + b) ** scale, int((s == 0).sum()))]:
        mu, sd = m * p, np.sqrt(m * p * (1 - p))
        assert abs(count - mu) <= 4 * sd + 1, (count, mu, sd)
    for bit in range(scale):
        frac = ((s >> bit) & 1).mean()
        assert abs(frac - (c + dd)) < 4 * np.sqrt((c + dd) * (a + b) / m)


def test_weights_per_pair_and_range():
    src = np.array([0, 1, 0, 5, 0], dtype=np.int32)
    dst = np.array([1, 0, 1, 6, 1], dtype=np.int32)
    w = gg.weights_u32(src, dst)
    assert w[0] == w[2] == w[4]  # same ordered pair, same weight
    _, s, d = gg.rmat(14)
    w = gg.weights_u32(s, d)
    assert w.min() >= 1 and w.max() <= 255
    # uniform on 1..255: every value shows up, mean near 128
    assert len(np.unique(w)) == 255 and abs(w.mean() - 128.0) < 1.0
    wf = gg.weights_f32(s, d, 11, 0.5, 1.5)
    assert wf.min() >= 0.5 and wf.max() < 1.5


def test_sources_distinct_with_out_edges():
    n, s, d = gg.rmat(12)
    src = gg.sources(n, s, d, 64, gg.SEED_BATCH_SOURCES)
    assert len(src) == 64 and src[0] == 0 and len(set(src.tolist())) == 64
    has_out = np.zeros(n, dtype=bool)
    has_out[s[s != d]] = True
    assert has_out[src].all()


def test_cf_ratings_shape():
    R = gg.cf_ratings(n_users=3000, n_items=500, total=120_000)
    deg = np.bincount(R.user, minlength=R.n_users)
    assert R.m == 120_000 and deg.sum() == 120_000
    assert deg.min() >= gg.CF_DMIN and deg.max() <= R.n_items
    assert R.rating.min() >= 1 and R.rating.max() <= 5
    key = R.user.astype(np.int64) * R.n_items + R.item
    assert (np.diff(key) > 0).all()  # sorted, no repeated (user, item)
    assert R.item.min() >= 0 and R.item.max() < R.n_items
