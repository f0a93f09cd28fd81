"""Seeded generators: reproducible, chunk-independent, with the stated shapes and ranges."""

import numpy as np

from synth import workloads as wl


def test_same_seed_same_data_and_chunking_does_not_matter(monkeypatch):
    a = wl.gaussian_mixture(3, 5000, 16, 10)
    b = wl.gaussian_mixture(3, 5000, 16, 10)
    np.testing.assert_array_equal(a, b)
    monkeypatch.setattr(wl, "CHUNK_ROWS", 1000)
    c = wl.gaussian_mixture(3, 1000, 16, 10)
    np.testing.assert_array_equal(a[:1000], c)
    assert not np.array_equal(a, wl.gaussian_mixture(4, 5000, 16, 10))


def test_integer_workload_is_integer_valued_in_range():
    w = wl.integer_pq(n=20_000, n_train=5000)
    assert w.x.dtype == np.float32 and w.x.shape == (20_000, 128)
    assert np.all(w.x == np.rint(w.x)) and w.x.min() >= 0 and w.x.max() <= 255
    assert len(np.unique(w.train_rows)) == 5000
    assert w.init_rows.shape == (16, 256)
    for j in range(16):
        assert len(np.unique(w.init_rows[j])) == 256 and w.init_rows[j].max() < 5000


def test_sphere_workload_rows_are_unit_norm_and_sizes_in_range():
    b = wl.batched_uneven(n_prob=4, n_lo=300, n_hi=900, n_comp=20, ks=32)
    for p in b.problems:
        assert 300 <= p.x.shape[0] <= 900
        np.testing.assert_allclose(np.linalg.norm(p.x, axis=1), 1.0, rtol=1e-5)


def test_queries_differ_from_rows_but_share_the_mixture():
    w = wl.ivf_adc(n=2000, d=16, n_comp=8, kc=8, n_query=50, m=4, ks=16, n_train=500)
    assert w.queries.shape == (50, 16)
    assert not np.array_equal(w.queries, w.x[:50])
    assert len(np.unique(w.coarse_init)) == 8
