"""Seeded generators: determinism and the shape of the synthetic workloads."""
import numpy as np

from paper_2404_19638_amd import synth


def test_uniform_stream_is_deterministic_and_in_range():
    a = synth.uniform_f32(99, 100_000)
    b = synth.uniform_f32(99, 100_000)
    assert a.tobytes() == b.tobytes()
    assert a.min() >= -1.0 and a.max() < 1.0
    assert abs(float(a.mean())) < 0.01
    # offsets address the same stream
    np.testing.assert_array_equal(synth.uniform_f32(99, 10, ctr0=500), a[500:510])


def test_dense_indexing_by_global_row():
    full = synth.dense_f32(5, 0, 64, 8)
    part = synth.dense_f32(5, 40, 10, 8)
    np.testing.assert_array_equal(full[40:50], part)


def test_uniform_block_exact_count_distinct():
    r, c = synth.uniform_block(4096, 4096, 40_000, 2404)
    assert r.size == 40_000
    assert np.unique(r * 4096 + c).size == 40_000
    r2, c2 = synth.uniform_block(4096, 4096, 40_000, 2404)
    assert np.array_equal(r, r2) and np.array_equal(c, c2)


def test_rmat_block_distinct_in_range_and_skewed():
    rr, cr = (1 << 12, 2 << 12), (0, 1 << 12)
    r, c = synth.rmat_block(14, 16 << 14, 77, rr, cr)
    assert r.size > 0
    assert r.min() >= rr[0] and r.max() < rr[1] and c.min() >= cr[0] and c.max() < cr[1]
    assert np.unique((r - rr[0]) * (1 << 12) + (c - cr[0])).size == r.size
    deg = np.bincount(r - rr[0])
    deg = deg[deg > 0]
    assert deg.max() > 8 * deg.mean()          # power-law hubs
    r2, c2 = synth.rmat_block(14, 16 << 14, 77, rr, cr)
    assert np.array_equal(r, r2) and np.array_equal(c, c2)


def test_banded_block_distinct_in_band_and_deterministic():
    lo, n, w = 1000, 5000, 40
    r1, c1 = synth.banded_block(lo, n, 3, w, 77)
    r2, c2 = synth.banded_block(lo, n, 3, w, 77)
    np.testing.assert_array_equal(r1, r2)
    np.testing.assert_array_equal(c1, c2)
    assert r1.min() >= lo and r1.max() < lo + n and c1.min() >= lo and c1.max() < lo + n
    assert np.abs(c1 - r1).max() <= w
    assert np.unique((r1 - lo) * n + (c1 - lo)).size == r1.size          # distinct
    assert np.unique(r1).size == n                                       # every row drawn
    assert r1.size > 0.9 * 3 * n                                         # few duplicates
    # offsets cover the band on both sides
    assert (c1 - r1).min() == -w and (c1 - r1).max() == w
