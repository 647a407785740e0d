"""Sanity of the seeded generators (shapes, determinism, CSR validity,
statistics of the stand-in corpora).  CPU only."""
import numpy as np

import datagen


def _check_csr(m):
    assert m.rowptr.dtype == np.int32 and m.col.dtype == np.int32 and m.val.dtype == np.float32
    assert m.rowptr[0] == 0 and np.all(np.diff(m.rowptr) >= 0)
    assert m.col.min() >= 0 and m.col.max() < m.cols
    for r in range(0, m.rows, max(1, m.rows // 50)):
        c = m.col[m.rowptr[r]:m.rowptr[r + 1]]
        assert np.all(np.diff(c) > 0)


def test_dense_c0_deterministic_and_shaped():
    a = datagen.c0()
    b = datagen.c0()
    assert a.shape == (1000, 800) and a.dtype == np.float32
    assert np.array_equal(a, b)
    assert a.min() > 0
    W, H = datagen.uniform_init(1000, 800, 16, seed=1)
    assert W.shape == (1000, 16) and H.shape == (16, 800) and W.dtype == np.float32


def test_bag_of_words_statistics():
    c = datagen.bag_of_words(3000, 1200, 1.1, 77.0, seed=2)
    _check_csr(c.A)
    _check_csr(c.At)
    assert c.A.nnz == c.At.nnz
    # every document (column of A) has unit L2 norm
    norms = np.sqrt(np.add.reduceat(c.At.val.astype(np.float64) ** 2, c.At.rowptr[:-1]))
    np.testing.assert_allclose(norms, 1.0, rtol=1e-5)
    # Zipf skew: the most popular term appears in most documents
    df = np.diff(c.A.rowptr)
    assert df.max() > 0.8 * 1200
    # A and At hold the same matrix
    np.testing.assert_array_equal(c.A.to_dense(), c.At.to_dense().T)


def test_c1_size_matches_recipe():
    c = datagen.c1()
    assert (c.A.rows, c.A.cols) == (26000, 11000)
    assert 0.8e6 < c.A.nnz < 0.92e6  # about 0.3% dense


def test_matched_init_scales_h_only():
    W, H = datagen.uniform_init(300, 200, 10, seed=1)
    Wm, Hm = datagen.uniform_init_matched(300, 200, 10, 0.5, seed=1)
    assert np.array_equal(W, Wm)
    h = 0.5 * np.sqrt(300 / 3.0) / 2.5
    np.testing.assert_allclose(Hm, H.astype(np.float64) * h, rtol=1e-6)
