"""Chained products on the GPU: graph contraction C = S^T (A S) and the
Markov-clustering loop, checked against the oracle step by step (teacher
forcing: each oracle step starts from the GPU's previous result)."""
import numpy as np
import pytest

import oracle
from paper_2512_12036_amd import apps, gen, spgemm

from gpu_util import compare_all_rows, log, structure_invariants

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    spgemm.load()


def host(c):
    return c.to_host()


def sorted_rows(m):
    """Same matrix with every row's entries in ascending column order."""
    rid = np.repeat(np.arange(m.nrows), np.diff(m.rpt))
    order = np.lexsort((m.col, rid))
    return gen.Csr(m.nrows, m.ncols, m.rpt.copy(), m.col[order], m.val[order])


def test_selector_transpose_matches_host():
    import torch
    n, k = 50_000, 3_000
    labels = gen.contraction_labels(n, k, seed=4)
    st = spgemm.selector_transpose(torch.from_numpy(labels).cuda(), k)
    trpt, tcol, tval = oracle.transpose(n, k, np.arange(n + 1), labels, np.ones(n, np.float32))
    g = sorted_rows(host(st))
    assert np.array_equal(g.rpt, trpt) and np.array_equal(g.col, tcol)
    assert np.all(g.val == 1.0)
    bad = torch.from_numpy(labels).cuda()
    bad[7] = k
    with pytest.raises(spgemm.SpgemmError) as e:
        spgemm.selector_transpose(bad, k)
    assert e.value.code == 3


def check_contraction(a, labels, k, p, c, rows_p=None, rows_c=None):
    s = gen.selector(labels, k)
    ph = host(p)
    ref_p = oracle.product(a, s, rows_p)
    assert oracle.compare(ref_p, ph.rpt, ph.col, ph.val, rows=rows_p) is None
    st = sorted_rows(gen.Csr(k, a.nrows, *oracle.transpose(a.nrows, k, s.rpt, s.col, s.val)))
    ch = host(c)
    ref_c = oracle.product(st, ph, rows_c)        # teacher forced on the GPU's P
    assert oracle.compare(ref_c, ch.rpt, ch.col, ch.val, rows=rows_c) is None
    # total weight is preserved: 1^T C 1 = 1^T A 1
    tot = float(np.sum(ch.val, dtype=np.float64))
    want = float(np.sum(a.val, dtype=np.float64))
    assert abs(tot - want) <= 1e-4 * want


def test_contraction_small():
    import torch
    a = gen.rmat(14, 8, seed=21)
    k = a.nrows // 16
    labels = gen.contraction_labels(a.nrows, k, seed=22)
    p, c = apps.contract(spgemm.to_device(a), torch.from_numpy(labels).cuda(), k)
    torch.cuda.synchronize()
    check_contraction(a, labels, k, p, c)


def test_contraction_full_size_every_row():
    # R-MAT scale 20, edge factor 8, 65,536 clusters: P and C on the device,
    # every row of both against the oracle (C teacher-forced on the GPU's P)
    import torch
    a = gen.rmat(20, 8, seed=23)
    k = a.nrows // 16
    labels = gen.contraction_labels(a.nrows, k, seed=24)
    log(f"[gpu] contraction scale 20: nnz(A) {a.nnz}")
    p, c = apps.contract(spgemm.to_device(a), torch.from_numpy(labels).cuda(), k)
    torch.cuda.synchronize()
    log(f"[gpu] nnz(P) {p.nnz} nnz(C) {c.nnz}")
    check_contraction(a, labels, k, p, c)


def check_prune(e, t, power, theta, rows=None):
    """GPU prune step against the oracle's, on the GPU's expansion (device or
    host CSR).  Entries whose normalised value lies within 1e-5 * theta of
    theta may be kept by one side only; everything else must agree (values to
    1e-5 relative)."""
    eh = e if isinstance(e, gen.Csr) else host(e)
    th = t if isinstance(t, gen.Csr) else host(t)
    rows = np.arange(eh.nrows) if rows is None else rows
    band = 1e-5 * theta
    for i in rows:
        s, f = eh.rpt[i], eh.rpt[i + 1]
        nrpt, ncol, nval, before = oracle.mcl_inflate_normalize_prune(
            np.array([0, f - s]), eh.col[s:f], eh.val[s:f].astype(np.float64), power, theta)
        g0, g1 = th.rpt[i], th.rpt[i + 1]
        gcol, gval = th.col[g0:g1], th.val[g0:g1]
        if np.array_equal(gcol, ncol):
            assert np.all(np.abs(gval - nval) <= 1e-5 * nval + 1e-9), f"row {i}"
        else:
            diff = np.setxor1d(gcol, ncol)
            pos = np.searchsorted(eh.col[s:f], diff)
            assert np.all(np.abs(before[pos] - theta) <= band), f"row {i}: {diff}"


def test_mcl_small_teacher_forced():
    t = spgemm.to_device(gen.planted_partition(40, 100, seed=31))
    for it in range(4):
        e = spgemm.matmul(t, t)
        th = host(t)
        eh = host(e)
        ref = oracle.product(th, th)
        assert oracle.compare(ref, eh.rpt, eh.col, eh.val) is None, f"expansion {it}"
        nt = spgemm.mcl_prune(e, 2.0, 1e-4)
        check_prune(e, nt, 2.0, 1e-4)
        # rows of the pruned matrix are stochastic
        nh = host(nt)
        sums = np.add.reduceat(nh.val.astype(np.float64), nh.rpt[:-1])[np.diff(nh.rpt) > 0]
        assert np.all(np.abs(sums - 1.0) <= 1e-5)
        t = nt


_MCL = {}


@pytest.mark.parametrize("it", [1, 2, 3, 4, 5])
def test_mcl_full_size_iteration(it):
    """The Markov-clustering workload (1,000 communities x 100 nodes), one
    iteration per test, teacher-forced: the oracle's expansion starts from the
    GPU's previous pruned matrix.  Every expansion's row lengths are compared
    with the oracle's distinct counts; every row of the expansion and of the
    prune step is compared for iterations 1, 3, 4 and 5.  Iteration 2's
    expansion has ~4.8e9 entries: its rows are compared on a stratified 5 %
    sample (every 20th row) plus the 100 longest rows."""
    import torch
    if it == 1:
        _MCL.clear()
        _MCL["t"] = spgemm.to_device(gen.planted_partition(1000, 100, seed=5))
        _MCL["it"] = 0
    assert _MCL.get("it") == it - 1, "the previous iteration did not complete"
    t = _MCL["t"]
    th = host(t)
    e = spgemm.matmul(t, t)
    torch.cuda.synchronize()
    log(f"[gpu] mcl iteration {it}: nnz(T) {t.nnz} nnz(E) {e.nnz}")
    er = e.rpt.cpu().numpy()
    lens = np.diff(er)
    assert np.array_equal(lens, oracle.row_counts(th, th)), f"iteration {it} row lengths"
    structure_invariants(e)
    if it != 2:
        compare_all_rows(th, th, e, label=f"mcl expansion {it}")
        nt = spgemm.mcl_prune(e, 2.0, 1e-4)
        torch.cuda.synchronize()
        check_prune(e, nt, 2.0, 1e-4)
    else:
        rows = np.union1d(np.arange(0, th.nrows, 20), np.argsort(lens, kind="stable")[-100:])
        ref = oracle.product(th, th, rows)
        sub = [(er[r], er[r + 1]) for r in rows]
        col = np.concatenate([e.col[s:f].cpu().numpy() for s, f in sub])
        val = np.concatenate([e.val[s:f].cpu().numpy() for s, f in sub])
        srpt = np.zeros(len(rows) + 1, np.int64)
        np.cumsum(lens[rows], out=srpt[1:])
        assert oracle.compare(ref, srpt, col, val) is None, f"iteration {it}"
        log(f"[gpu] mcl expansion 2: {len(rows)} rows, {srpt[-1]} entries match the oracle")
        nt = spgemm.mcl_prune(e, 2.0, 1e-4)
        torch.cuda.synchronize()
        # prune step on the sampled rows, from the GPU's expansion rows
        e_rows = gen.Csr(len(rows), th.ncols, srpt, col, val)
        nr = nt.rpt.cpu().numpy()
        tcol = [nt.col[nr[r]:nr[r + 1]].cpu().numpy() for r in rows]
        tval = [nt.val[nr[r]:nr[r + 1]].cpu().numpy() for r in rows]
        t_rows = gen.Csr(len(rows), th.ncols,
                         np.concatenate([[0], np.cumsum([len(x) for x in tcol])]).astype(np.int64),
                         np.concatenate(tcol), np.concatenate(tval))
        check_prune(e_rows, t_rows, 2.0, 1e-4)
    del e
    torch.cuda.empty_cache()
    assert nt.nnz > 0
    _MCL["t"] = nt
    _MCL["it"] = it
    if it == 5:
        _MCL.clear()
