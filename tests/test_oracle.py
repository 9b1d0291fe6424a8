"""Pins for the CPU oracle (no GPU).

The oracle is the definition of C = A*B (paper Section III-A) and of the
intermediate-product count (paper Algorithm 1).  It is checked here against
things other than itself:

* brute force: dense FP64 matrix products of small random matrices, with
  non-square shapes so that a transposed operand cannot pass;
* an independent library routine: scipy's sparse product on all-ones values
  (path counts, exact integers) for the structure;
* special cases with closed forms: B = I, permutation A, empty rows and
  matrices, cancellation to an explicit zero;
* the closed form sum_i IP_i = sum_k indeg_A(k) * len_B(k);
* a hand-worked fixture (tests/golden/hand_product.txt);
* planted mistakes: variants of the product with a dropped term, a flipped
  sign or a wrong row index fail the dense pin.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp
from hypothesis import given, settings, strategies as st

import oracle
from paper_2512_12036_amd import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense(m: gen.Csr) -> np.ndarray:
    d = np.zeros((m.nrows, m.ncols), dtype=np.float64)
    rid = np.repeat(np.arange(m.nrows), np.diff(m.rpt))
    np.add.at(d, (rid, m.col.astype(np.int64)), m.val.astype(np.float64))
    return d


def pattern(m: gen.Csr) -> np.ndarray:
    d = np.zeros((m.nrows, m.ncols), dtype=np.int64)
    rid = np.repeat(np.arange(m.nrows), np.diff(m.rpt))
    np.add.at(d, (rid, m.col.astype(np.int64)), 1)
    return d


def to_scipy(m: gen.Csr, ones=False):
    v = np.ones(m.nnz) if ones else m.val.astype(np.float64)
    return sp.csr_matrix((v, m.col, m.rpt), shape=(m.nrows, m.ncols))


def check_against_dense(a, b, ref):
    want = dense(a) @ dense(b)
    structure = (pattern(a) @ pattern(b)) > 0
    got = np.zeros_like(want)
    got_struct = np.zeros(want.shape, dtype=bool)
    rid = np.repeat(np.arange(a.nrows), np.diff(ref.rpt))
    got[rid, ref.col] = ref.val
    got_struct[rid, ref.col] = True
    assert np.array_equal(got_struct, structure)
    bound = np.abs(dense(a)) @ np.abs(dense(b))
    assert np.all(np.abs(got - want) <= 1e-12 * bound + 1e-300)
    babs = np.zeros_like(want)
    babs[rid, ref.col] = ref.absb
    assert np.allclose(babs, bound, rtol=1e-12, atol=0)
    for i in range(a.nrows):
        cols = ref.col[ref.rpt[i]:ref.rpt[i + 1]]
        assert np.all(np.diff(cols) > 0), "rows must be strictly ascending"


@settings(max_examples=60, deadline=None)
@given(m=st.integers(0, 23), k=st.integers(0, 29), n=st.integers(0, 31),
       da=st.floats(0.0, 0.6), db=st.floats(0.0, 0.6), seed=st.integers(0, 10_000))
def test_oracle_matches_dense_product(m, k, n, da, db, seed):
    a = gen.random_csr(m, k, da, seed)
    b = gen.random_csr(k, n, db, seed + 1)
    ref = oracle.product(a, b)
    check_against_dense(a, b, ref)


def test_oracle_structure_matches_scipy_boolean_product():
    a = gen.rmat(10, 8, seed=11)
    ref = oracle.product(gen.ones_valued(a), gen.ones_valued(a))
    s = to_scipy(a, ones=True) @ to_scipy(a, ones=True)
    s.sort_indices()
    assert np.array_equal(ref.rpt, s.indptr)
    assert np.array_equal(ref.col, s.indices)
    assert np.array_equal(ref.val, s.data)      # path counts, exact


def test_oracle_rectangular_scipy_values():
    a = gen.er(300, 2000, seed=5, ncols=450)
    b = gen.er(450, 3000, seed=6, ncols=170)
    ref = oracle.product(a, b)
    s = (to_scipy(a) @ to_scipy(b)).tocsr()
    s.sort_indices()
    # scipy drops nothing here (random reals never cancel exactly)
    assert np.array_equal(ref.rpt, s.indptr)
    assert np.array_equal(ref.col, s.indices)
    assert np.allclose(ref.val, s.data, rtol=1e-12, atol=1e-14)


def test_identity_and_permutation_are_exact():
    a = gen.rmat(9, 8, seed=3)
    n = a.ncols
    eye = gen.from_coo(n, n, np.arange(n), np.arange(n), np.ones(n, np.float32))
    r = oracle.product(a, eye)
    assert np.array_equal(r.rpt, a.rpt) and np.array_equal(r.col, a.col)
    assert np.array_equal(r.val, a.val.astype(np.float64))
    perm = np.random.default_rng(0).permutation(a.nrows)
    p = gen.from_coo(a.nrows, a.nrows, np.arange(a.nrows), perm, np.ones(a.nrows, np.float32))
    r = oracle.product(p, a)
    for i in range(a.nrows):
        c, v = a.row(perm[i])
        assert np.array_equal(r.col[r.rpt[i]:r.rpt[i + 1]], c)
        assert np.array_equal(r.val[r.rpt[i]:r.rpt[i + 1]], v.astype(np.float64))


def test_cancellation_keeps_explicit_zero():
    a = gen.from_coo(1, 2, [0, 0], [0, 1], np.array([1, 1], np.float32))
    b = gen.from_coo(2, 1, [0, 1], [0, 0], np.array([1, -1], np.float32))
    r = oracle.product(a, b)
    assert r.nnz == 1 and r.col[0] == 0 and r.val[0] == 0.0 and r.absb[0] == 2.0


def test_empty_shapes():
    for (m, k, n) in [(0, 5, 7), (5, 0, 7), (5, 7, 0), (1, 1, 1), (0, 0, 0)]:
        a = gen.random_csr(m, k, 0.5, 1)
        b = gen.random_csr(k, n, 0.5, 2)
        r = oracle.product(a, b)
        assert r.rpt.shape == (m + 1,)
        check_against_dense(a, b, r)


def test_duplicates_and_unsorted_rows():
    a = gen.rmat(8, 8, seed=21)
    b = gen.rmat(8, 4, seed=22)
    base = oracle.product(a, b)
    sh = oracle.product(gen.shuffle_rows(a, 1), gen.shuffle_rows(b, 2))
    assert np.array_equal(base.rpt, sh.rpt) and np.array_equal(base.col, sh.col)
    assert np.allclose(base.val, sh.val, rtol=1e-12, atol=1e-14)
    # a duplicated coordinate is summed: A with entry split in two halves
    rid = np.repeat(np.arange(a.nrows), np.diff(a.rpt))
    rows = np.concatenate([rid, rid])
    cols = np.concatenate([a.col, a.col])
    vals = np.concatenate([a.val / 2, a.val / 2]).astype(np.float32)
    dup = gen.from_coo(a.nrows, a.ncols, rows, cols, vals, merge=False)
    rd = oracle.product(dup, b)
    assert np.array_equal(rd.col, base.col)
    assert np.allclose(rd.val, base.val, rtol=1e-12, atol=1e-14)


def test_ip_closed_form_and_brute_force():
    a = gen.rmat(11, 8, seed=4)
    b = gen.rmat(11, 4, seed=5)
    ip = oracle.ip(a, b)
    indeg = np.bincount(a.col, minlength=a.ncols).astype(np.int64)
    assert ip.sum() == int((indeg * np.diff(b.rpt)).sum())
    for i in range(0, a.nrows, 37):
        want = sum(int(b.rpt[k + 1] - b.rpt[k]) for k in a.col[a.rpt[i]:a.rpt[i + 1]])
        assert ip[i] == want
    counts = oracle.row_counts(a, b)
    assert np.all(counts <= np.minimum(ip, b.ncols))


def test_er_ip_expectation():
    # n d^2 expected intermediate products for a G(n, n d) self-product
    a = gen.er(2000, 16000, seed=1)
    ip = oracle.ip(a, a).sum()
    assert abs(ip - 2000 * 8 * 8) < 0.05 * 128000


def test_row_selection_matches_full():
    a = gen.rmat(10, 8, seed=8)
    full = oracle.product(a, a)
    rows = np.array([5, 0, 1023, 17, 17, 600])
    part = oracle.product(a, a, rows)
    for s, i in enumerate(rows):
        assert np.array_equal(part.col[part.rpt[s]:part.rpt[s + 1]],
                              full.col[full.rpt[i]:full.rpt[i + 1]])
        assert np.array_equal(part.val[part.rpt[s]:part.rpt[s + 1]],
                              full.val[full.rpt[i]:full.rpt[i + 1]])


def _read_golden(path):
    sections, cur = {}, None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                cur = line.strip("[]")
                sections[cur] = []
            else:
                sections[cur].append([float(x) for x in line.split()])
    return sections


def _golden_csr(trip, shape):
    t = np.array(trip)
    return gen.from_coo(shape[0], shape[1], t[:, 0].astype(np.int64),
                        t[:, 1].astype(np.int64), t[:, 2].astype(np.float32), merge=False)


def test_hand_worked_fixture():
    s = _read_golden(os.path.join(GOLDEN, "hand_product.txt"))
    a = _golden_csr(s["A 3x3"], (3, 3))
    b = _golden_csr(s["B 3x4"], (3, 4))
    c = _golden_csr(s["C 3x4"], (3, 4))
    r = oracle.product(a, b)
    assert np.array_equal(r.rpt, c.rpt) and np.array_equal(r.col, c.col)
    assert np.array_equal(r.val, c.val.astype(np.float64))
    ip = oracle.ip(a, b)
    assert [int(x) for x in ip] == [int(v) for _, v in s["IP"]]


# ---- planted mistakes: the dense pin must reject each of them -------------
def _mutant_product(a, b, mode):
    """Python Gustavson product with one deliberate mistake."""
    da = dense(a)
    db = dense(b)
    if mode == "drop_last_term":
        out = np.zeros((a.nrows, b.ncols))
        for i in range(a.nrows):
            cols = a.col[a.rpt[i]:a.rpt[i + 1]]
            for k in cols[:-1]:
                out[i] += da[i, k] * db[k]
        return out
    if mode == "sign":
        return -(da @ db)
    if mode == "wrong_index":      # row i of B instead of row k
        out = np.zeros((a.nrows, b.ncols))
        for i in range(a.nrows):
            for k in a.col[a.rpt[i]:a.rpt[i + 1]]:
                out[i] += da[i, k] * db[i]
        return out
    raise ValueError(mode)


@pytest.mark.parametrize("mode", ["drop_last_term", "sign", "wrong_index"])
def test_dense_pin_rejects_planted_mistakes(mode):
    a = gen.random_csr(7, 9, 0.5, 3)
    b = gen.random_csr(9, 5, 0.5, 4)
    want = dense(a) @ dense(b)
    got = _mutant_product(a, b, mode)
    bound = np.abs(dense(a)) @ np.abs(dense(b))
    assert not np.all(np.abs(got - want) <= 1e-12 * bound + 1e-300)


def test_compare_detects_mismatches():
    a = gen.rmat(8, 8, seed=30)
    ref = oracle.product(a, a)
    rpt, col, val = ref.rpt.copy(), ref.col.copy(), ref.val.astype(np.float32)
    assert oracle.compare(ref, rpt, col, val) is None
    c2 = col.copy()
    c2[3] += 1
    assert "col_idx" in oracle.compare(ref, rpt, c2, val)
    v2 = val.copy()
    v2[5] += 1e-3 * max(1.0, abs(v2[5]))
    assert "tolerance" in oracle.compare(ref, rpt, col, v2)
    r2 = rpt.copy()
    r2[4] += 1
    assert "row_ptr" in oracle.compare(ref, r2, col, val)


def test_compare_row_selection_branch():
    """compare(rows=...) checks exactly the selected rows of the full arrays:
    a wrong column, a wrong row length or an out-of-tolerance value inside a
    selected row is reported; the same mistakes outside the selection are
    not looked at."""
    a = gen.rmat(8, 8, seed=31)
    full = oracle.product(a, a)
    rpt, col, val = full.rpt.copy(), full.col.copy(), full.val.astype(np.float32)
    lens = np.diff(rpt)
    busy = np.nonzero(lens >= 3)[0]
    sel = np.sort(busy[::3][:20])
    other = np.setdiff1d(busy, sel)[0]
    ref = oracle.product(a, a, sel)
    assert oracle.compare(ref, rpt, col, val, rows=sel) is None
    # wrong column in the middle of a selected row
    r = sel[len(sel) // 2]
    c2 = col.copy()
    c2[rpt[r] + 1] = c2[rpt[r]]
    msg = oracle.compare(ref, rpt, c2, val, rows=sel)
    assert msg is not None and "col_idx" in msg
    # the same mistake in a row outside the selection is not looked at
    c3 = col.copy()
    c3[rpt[other] + 1] = c3[rpt[other]]
    assert oracle.compare(ref, rpt, c3, val, rows=sel) is None
    # a selected row one entry shorter (its last entry handed to the next row)
    r2 = rpt.copy()
    r2[r + 1] -= 1
    msg = oracle.compare(ref, r2, col, val, rows=sel)
    assert msg is not None and "row lengths" in msg
    # a value outside the tolerance in a selected row
    v2 = val.copy()
    j = rpt[r] + 2
    v2[j] = np.float32(v2[j] + 1e-3 * max(1.0, abs(float(v2[j]))))
    msg = oracle.compare(ref, rpt, col, v2, rows=sel)
    assert msg is not None and "tolerance" in msg


def test_compare_exact_branch_rejects_one_ulp():
    """exact_values=True demands equal values: a one-ULP change of a single
    FP32 entry (well inside the 1e-5 tolerance) is reported, and the same
    arrays pass the tolerance check."""
    a = gen.int_valued(gen.rmat(8, 8, seed=32), 5)
    ref = oracle.product(a, a)
    rpt, col = ref.rpt.copy(), ref.col.copy()
    val = ref.val.astype(np.float32)
    assert np.array_equal(val.astype(np.float64), ref.val)   # integers: exact in FP32
    assert oracle.compare(ref, rpt, col, val, exact_values=True) is None
    big = int(np.argmax(np.abs(val)))
    for direction in (np.float32(np.inf), np.float32(-np.inf)):
        v2 = val.copy()
        v2[big] = np.nextafter(v2[big], direction)
        msg = oracle.compare(ref, rpt, col, v2, exact_values=True)
        assert msg is not None and "value differs" in msg
        assert oracle.compare(ref, rpt, col, v2) is None
    # selected rows with exact values
    sel = np.array([big_row for big_row in range(a.nrows) if rpt[big_row] <= big < rpt[big_row + 1]])
    part = oracle.product(a, a, sel)
    v3 = val.copy()
    v3[big] = np.nextafter(v3[big], np.float32(np.inf))
    assert oracle.compare(part, rpt, col, val, rows=sel, exact_values=True) is None
    assert "value differs" in oracle.compare(part, rpt, col, v3, rows=sel, exact_values=True)


def test_compare_contiguous_block_slice():
    """A block of consecutive rows is checked from slices of the full arrays:
    row pointers rebased at the block's first entry."""
    a = gen.rmat(9, 8, seed=33)
    full = oracle.product(a, a)
    val = full.val.astype(np.float32)
    r0, r1 = 100, 260
    blk = oracle.product(a, a, np.arange(r0, r1))
    s0, s1 = full.rpt[r0], full.rpt[r1]
    local = full.rpt[r0:r1 + 1] - s0
    assert oracle.compare(blk, local, full.col[s0:s1], val[s0:s1]) is None
    # or the block's pointers into the full arrays
    assert oracle.compare(blk, full.rpt[r0:r1 + 1], full.col, val) is None
    c2 = full.col[s0:s1].copy()
    c2[-1] += 1
    assert "col_idx" in oracle.compare(blk, local, c2, val[s0:s1])
