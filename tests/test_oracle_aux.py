"""Pins for the oracle's row grouping, Markov-clustering steps and transpose.

* grouping (paper Section III-B, Table I): brute-force per-row loop, keys on
  both sides of every bound, the map is a permutation that is stable inside
  each group, offsets are the running group sizes;
* MCL step (paper Algorithm 6, on the transposed matrix): a hand-computed
  row, row sums equal one after renormalisation, nothing below theta is kept,
  power 1 with theta 0 is the identity on a stochastic matrix;
* transpose (paper Algorithm 7 needs S^T): scipy's transpose and the
  involution property.
"""
import numpy as np
import scipy.sparse as sp

import oracle
from paper_2512_12036_amd import gen

UPPER = [0, 31, 511, 8191]          # Table I bounds (group 0 = empty rows)


def test_bins_brute_force_and_boundaries():
    keys = []
    for t in UPPER[1:]:
        keys += [t - 1, t, t + 1]
    keys += [0, 0, 1, 10**9, 5, 0, 8191, 70000]
    keys = np.array(keys, dtype=np.int64)
    bins, order, offsets = oracle.bins_reference(keys, UPPER)
    for i, k in enumerate(keys):
        if k == 0:
            want = 0
        elif k <= 31:
            want = 1
        elif k <= 511:
            want = 2
        elif k <= 8191:
            want = 3
        else:
            want = 4
        assert bins[i] == want, (k, bins[i], want)
    assert sorted(order.tolist()) == list(range(keys.shape[0]))
    for b in range(5):
        seg = order[offsets[b]:offsets[b + 1]]
        assert np.all(bins[seg] == b)
        assert np.all(np.diff(seg) > 0)
    assert offsets[-1] == keys.shape[0]


def test_bins_copy_rule_brute_force():
    """Single-nonzero rows past the copy group take the copy group; every
    other row keeps its bound-derived group (brute force over all rows)."""
    upper = [0, 16, 64, 64, 256, 1024, 1024]
    rng = np.random.default_rng(3)
    keys = rng.integers(0, 5000, 400)
    keys[:20] = 0
    single = rng.random(400) < 0.4
    bins, order, offsets = oracle.bins_reference(keys, upper, single, 5)
    plain, _, _ = oracle.bins_reference(keys, upper)
    for i in range(400):
        want = 5 if (single[i] and plain[i] > 5) else plain[i]
        assert bins[i] == want, (i, keys[i], single[i], bins[i])
    assert np.any(single & (plain > 5)) and np.any(~single & (plain > 5))
    for b in range(len(upper) + 1):
        seg = order[offsets[b]:offsets[b + 1]]
        assert np.all(bins[seg] == b) and np.all(np.diff(seg) > 0)


def test_mcl_step_hand_example():
    rpt = np.array([0, 3, 3, 4])
    col = np.array([0, 1, 2, 5], dtype=np.int32)
    val = np.array([0.5, 0.3, 0.2, 0.7])
    nrpt, ncol, nval, before = oracle.mcl_inflate_normalize_prune(rpt, col, val, 2.0, 0.11)
    # row 0: squares 0.25 0.09 0.04 sum 0.38 -> 0.6579 0.2368 0.1053; the
    # last is below 0.11 and goes; renormalised 0.25/0.34, 0.09/0.34
    assert np.array_equal(nrpt, [0, 2, 2, 3])
    assert np.array_equal(ncol, [0, 1, 5])
    assert np.allclose(nval, [0.25 / 0.34, 0.09 / 0.34, 1.0], rtol=1e-14)
    assert np.allclose(before[:3], [0.25 / 0.38, 0.09 / 0.38, 0.04 / 0.38], rtol=1e-14)


def test_mcl_step_invariants():
    t = gen.planted_partition(n_comm=20, comm_size=30, intra_deg=8, inter_deg=2, seed=9)
    nrpt, ncol, nval, _ = oracle.mcl_inflate_normalize_prune(t.rpt, t.col, t.val, 2.0, 1e-2)
    sums = np.add.reduceat(nval, nrpt[:-1][np.diff(nrpt) > 0])
    assert np.allclose(sums, 1.0, rtol=1e-12)
    assert np.all(nval > 0)
    same = oracle.mcl_inflate_normalize_prune(t.rpt, t.col, t.val.astype(np.float64), 1.0, 0.0)
    assert np.array_equal(same[0], t.rpt) and np.array_equal(same[1], t.col)
    assert np.allclose(same[2], t.val, rtol=1e-6)


def test_transpose_matches_scipy():
    a = gen.er(50, 400, seed=3, ncols=70)
    trpt, tcol, tval = oracle.transpose(a.nrows, a.ncols, a.rpt, a.col, a.val)
    s = sp.csr_matrix((a.val, a.col, a.rpt), shape=(a.nrows, a.ncols)).T.tocsr()
    s.sort_indices()
    assert np.array_equal(trpt, s.indptr) and np.array_equal(tcol, s.indices)
    assert np.array_equal(tval, s.data)
    r2 = oracle.transpose(a.ncols, a.nrows, trpt, tcol, tval)
    assert np.array_equal(r2[0], a.rpt) and np.array_equal(r2[1], a.col)


def test_selector_transpose_groups_vertices():
    labels = gen.contraction_labels(1000, 16, seed=1)
    s = gen.selector(labels, 16)
    trpt, tcol, _ = oracle.transpose(s.nrows, s.ncols, s.rpt, s.col, s.val)
    for c in range(16):
        assert np.array_equal(tcol[trpt[c]:trpt[c + 1]], np.nonzero(labels == c)[0])
