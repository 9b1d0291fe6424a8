"""Pins of the oracle's Markov-clustering pieces (paper Algorithm 6): the
top-k pruning step, the change between iterates and the cluster
interpretation, against hand-worked examples, a dense computation, scipy's
connected components and the properties each step must have."""
import numpy as np
import pytest

import oracle
from paper_2512_12036_amd import gen


def test_topk_hand_example_with_ties():
    # one row: x = [.1, .3, .3, .2, .05, .3] (columns 0..5), power 1, theta .1
    rpt = np.array([0, 6])
    col = np.arange(6, dtype=np.int32)
    val = np.array([.1, .3, .3, .2, .05, .3])
    # y = x / 1.25: .08 .24 .24 .16 .04 .24; >= .1: columns 1 2 3 5
    # top-2 of {1: .24, 2: .24, 3: .16, 5: .24}: ties at .24 -> columns 1, 2
    nrpt, ncol, nval, before = oracle.mcl_prune_topk(rpt, col, val, 1.0, 0.1, 2)
    assert list(ncol) == [1, 2]
    assert np.allclose(nval, [0.5, 0.5])
    assert np.allclose(before, val / 1.25)
    # top-3 keeps the three .24 entries; top-4 all four
    assert list(oracle.mcl_prune_topk(rpt, col, val, 1.0, 0.1, 3)[1]) == [1, 2, 5]
    assert list(oracle.mcl_prune_topk(rpt, col, val, 1.0, 0.1, 4)[1]) == [1, 2, 3, 5]
    # power 2: x^2 = .01 .09 .09 .04 .0025 .09 (sum .3225); theta .2 keeps 1 2 5
    r = oracle.mcl_prune_topk(rpt, col, val, 2.0, 0.2, 0)
    assert list(r[1]) == [1, 2, 5] and np.allclose(r[2], [1 / 3] * 3)


def test_topk_zero_is_the_threshold_step():
    t = gen.planted_partition(20, 30, seed=3)
    a = oracle.mcl_prune_topk(t.rpt, t.col, t.val, 2.0, 1e-2, 0)
    b = oracle.mcl_inflate_normalize_prune(t.rpt, t.col, t.val, 2.0, 1e-2)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("k", [1, 3, 8])
def test_topk_keeps_the_largest(k):
    rng = np.random.default_rng(k)
    m = gen.random_csr(40, 60, 0.4, 5, lo=0.0, hi=1.0)
    # plant ties: round values to a coarse grid
    v = np.round(np.abs(m.val.astype(np.float64)) * 8) / 8 + 1.0 / 64
    nrpt, ncol, nval, before = oracle.mcl_prune_topk(m.rpt, m.col, v, 1.0, 0.02, k)
    for i in range(m.nrows):
        s, e = m.rpt[i], m.rpt[i + 1]
        kept = set(ncol[nrpt[i]:nrpt[i + 1]].tolist())
        elig = [(before[j], int(m.col[j])) for j in range(s, e) if before[j] >= 0.02]
        assert len(kept) == min(k, len(elig))
        if not kept:
            continue
        lo = min(y for y, c in elig if c in kept)
        for y, c in elig:
            if c in kept:
                continue
            # a dropped eligible entry is not larger than any kept one, and
            # on a tie it has a larger column than every kept entry of that value
            assert y <= lo
            if y == lo:
                assert all(c > kc for yy, kc in elig if kc in kept and yy == y)
        z = nval[nrpt[i]:nrpt[i + 1]]
        assert abs(z.sum() - 1.0) < 1e-12
        assert np.all(np.diff(ncol[nrpt[i]:nrpt[i + 1]]) > 0)


def _dense(n, rpt, col, val):
    d = np.zeros((n, n))
    for i in range(n):
        d[i, col[rpt[i]:rpt[i + 1]]] = val[rpt[i]:rpt[i + 1]]
    return d


def test_change_matches_dense_difference():
    a = gen.random_csr(30, 30, 0.2, 1, lo=0.0, hi=1.0)
    b = gen.random_csr(30, 30, 0.2, 2, lo=0.0, hi=1.0)
    got = oracle.mcl_change(a.rpt, a.col, a.val, b.rpt, b.col, b.val)
    want = np.abs(_dense(30, a.rpt, a.col, a.val) - _dense(30, b.rpt, b.col, b.val)).max()
    assert got == pytest.approx(want, abs=0)
    assert oracle.mcl_change(a.rpt, a.col, a.val, a.rpt, a.col, a.val) == 0.0
    assert oracle.mcl_change(b.rpt, b.col, b.val, a.rpt, a.col, a.val) == got


def test_components_hand_example():
    # 0-1-2 a path, 3 alone, 4->5 one directed entry, 6 self loop only
    coo = [(0, 1), (2, 1), (4, 5), (6, 6), (3, 3)]
    m = gen.from_coo(7, 7, [r for r, _ in coo], [c for _, c in coo], None, merge=True)
    assert list(oracle.components(7, m.rpt, m.col)) == [0, 0, 0, 3, 4, 4, 6]


def test_components_match_scipy():
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    for seed in range(4):
        m = gen.random_csr(300, 300, 0.004 + 0.002 * seed, seed, lo=0.0, hi=1.0)
        got = oracle.components(300, m.rpt, m.col)
        sp = csr_matrix((np.ones(m.nnz), m.col, m.rpt), shape=(300, 300))
        nc, lab = connected_components(sp, directed=False)
        # canonical labels: the smallest vertex of each scipy component
        first = np.full(nc, 300)
        for v in range(300):
            first[lab[v]] = min(first[lab[v]], v)
        assert np.array_equal(got, first[lab])
        assert len(set(got.tolist())) == nc
