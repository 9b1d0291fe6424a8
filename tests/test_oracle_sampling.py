"""Pins of the oracle's bulk sampling (paper Section V-C): inverse transform
sampling by hand and by its draw frequencies, EXTRACT against scipy's
row/column selection, and P = Q A against the SpGEMM oracle."""
import numpy as np

import oracle
from paper_2512_12036_amd import gen


def test_its_hand_example():
    rpt = np.array([0, 4, 4, 5])
    col = np.array([3, 5, 8, 9, 2], dtype=np.int32)
    val = np.array([1, 2, 3, 4, 0], dtype=np.float32)
    # S = 10: x = 0.5 -> 3; x = 1.0 (not exceeded by 1) -> 5; x = 9.9 -> 9
    u = np.array([[0.05, 0.1, 0.99], [0.3, 0.3, 0.3], [0.7, 0.2, 0.0]], dtype=np.float32)
    out = oracle.its_sample(rpt, col, val, u, 3, np.array([40, 41, 42]))
    assert list(out[:3]) == [3, 5, 9]
    assert list(out[3:6]) == [41] * 3          # empty row: its own vertex
    assert list(out[6:]) == [42] * 3           # zero weight: its own vertex


def test_its_frequencies_follow_the_weights():
    rng = np.random.default_rng(3)
    w = rng.random(12).astype(np.float32)
    n = 200_000
    u = rng.random(n).astype(np.float32)
    out = oracle.its_sample(np.array([0, 12]), np.arange(12, dtype=np.int32), w, u, n,
                            np.array([0]))
    freq = np.bincount(out, minlength=12) / n
    p = w.astype(np.float64) / w.sum(dtype=np.float64)
    sigma = np.sqrt(p * (1 - p) / n)
    assert np.all(np.abs(freq - p) <= 5 * sigma + 1e-12)


def test_extract_matches_scipy_selection():
    from scipy.sparse import csr_matrix
    a = gen.rmat(9, 8, seed=5)
    rng = np.random.default_rng(4)
    rows = rng.integers(0, a.nrows, 60)
    cols = rng.integers(0, a.ncols, 90)
    rpt, col, val = oracle.induced(a, rows, cols)
    sp = csr_matrix((a.val.astype(np.float64), a.col, a.rpt), shape=(a.nrows, a.ncols))
    want = sp[rows][:, cols].toarray()
    got = np.zeros_like(want)
    rid = np.repeat(np.arange(len(rows)), np.diff(rpt))
    got[rid, col] = val
    assert np.array_equal(got, want)
    # an entry exactly where A stores one
    assert rpt[-1] == sp[rows][:, cols].nnz


def test_rows_of_equal_the_one_hot_product():
    a = gen.rmat(9, 8, seed=6)
    v = np.array([5, 0, 511, 5, 17])
    q = gen.selector(v.astype(np.int32), a.nrows)
    ref = oracle.product(q, a)
    prpt, pcol, pval = oracle.product_rows_of(a, v)
    for r in range(len(v)):
        s, e = prpt[r], prpt[r + 1]
        o = np.argsort(pcol[s:e])
        assert np.array_equal(pcol[s:e][o], ref.col[ref.rpt[r]:ref.rpt[r + 1]])
        assert np.array_equal(pval[s:e][o].astype(np.float64), ref.val[ref.rpt[r]:ref.rpt[r + 1]])
