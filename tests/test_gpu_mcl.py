"""The whole Markov-clustering algorithm on the GPU (paper Algorithm 6):
the pruning step with its top-k part, the convergence measure and the
cluster interpretation, each against the oracle (teacher-forced: every
oracle step starts from the GPU's previous result), and the loop end to end
on a planted partition."""
import numpy as np
import pytest

import oracle
from paper_2512_12036_amd import apps, gen, spgemm

from gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    spgemm.load()


def check_prune_topk(eh, th, power, theta, k):
    """GPU prune step (th) against the oracle's on the GPU's input rows
    (eh).  Entries whose normalised value lies within 1e-5 * theta of theta
    may be kept by one side only; the top-k choice itself is made on the
    input order on both sides, so everything else must agree exactly, with
    values to 1e-5 relative."""
    band = 1e-5 * theta
    for i in range(eh.nrows):
        s, f = eh.rpt[i], eh.rpt[i + 1]
        nrpt, ncol, nval, before = oracle.mcl_prune_topk(
            np.array([0, f - s]), eh.col[s:f], eh.val[s:f].astype(np.float64), power, theta, k)
        g0, g1 = th.rpt[i], th.rpt[i + 1]
        gcol, gval = th.col[g0:g1], th.val[g0:g1]
        if np.array_equal(gcol, ncol):
            assert np.all(np.abs(gval - nval) <= 1e-5 * nval + 1e-9), f"row {i}"
        else:
            diff = np.setxor1d(gcol, ncol)
            pos = np.searchsorted(eh.col[s:f], diff)
            assert np.all(np.abs(before[pos] - theta) <= band), f"row {i}: {diff}"


@pytest.mark.parametrize("k", [1, 5, 40])
def test_prune_topk_teacher_forced(k):
    t = spgemm.to_device(gen.planted_partition(60, 50, seed=41))
    for it in range(3):
        e = spgemm.matmul(t, t)
        nt = spgemm.mcl_prune(e, 2.0, 1e-4, k)
        eh, nh = e.to_host(), nt.to_host()
        check_prune_topk(eh, nh, 2.0, 1e-4, k)
        assert np.all(np.diff(nh.rpt) <= k)
        t = nt
    log(f"[gpu] top-{k} prune matches the oracle over 3 iterations")


def test_prune_topk_ties_broken_by_column():
    # the planted partition's rows hold equal values (1 / degree): every
    # selection is a tie, resolved in column order
    th = gen.planted_partition(30, 40, seed=42)
    t = spgemm.to_device(th)
    for k in (1, 3, 7):
        nt = spgemm.mcl_prune(t, 1.0, 0.0, k).to_host()
        for i in range(th.nrows):
            want = th.col[th.rpt[i]:th.rpt[i + 1]][:k]
            assert np.array_equal(nt.col[nt.rpt[i]:nt.rpt[i + 1]], want), (k, i)
            assert np.allclose(nt.val[nt.rpt[i]:nt.rpt[i + 1]], 1.0 / len(want))


def test_change_matches_oracle_exactly():
    import torch
    for seed in range(3):
        a = gen.random_csr(300, 280, 0.05, 10 + seed, lo=0.0, hi=1.0)
        b = gen.random_csr(300, 280, 0.05, 20 + seed, lo=0.0, hi=1.0)
        # shared entries with different values, and identical ones
        b = gen.Csr(b.nrows, b.ncols, b.rpt, b.col, b.val)
        da, db = spgemm.to_device(a), spgemm.to_device(b)
        want = oracle.mcl_change(a.rpt, a.col, a.val, b.rpt, b.col, b.val)
        assert spgemm.mcl_change(da, db) == want
        assert spgemm.mcl_change(db, da) == want
        assert spgemm.mcl_change(da, da) == 0.0
    empty = spgemm.to_device(gen.random_csr(50, 50, 0.0, 1))
    torch.cuda.synchronize()
    assert spgemm.mcl_change(empty, empty) == 0.0


@pytest.mark.parametrize("density", [0.0005, 0.002, 0.01])
def test_components_match_oracle(density):
    m = gen.random_csr(3000, 3000, density, 5, lo=0.0, hi=1.0)
    lab, rounds = spgemm.components(spgemm.to_device(m))
    want = oracle.components(m.nrows, m.rpt, m.col)
    assert np.array_equal(lab.cpu().numpy(), want)
    log(f"[gpu] components: {len(set(want.tolist()))} clusters, {rounds} rounds")


def test_mcl_end_to_end_planted_partition():
    """Algorithm 6 to convergence on 40 planted communities of 50 nodes:
    every iteration teacher-forced against the oracle, the change measure
    exact, the final clusters equal to the oracle's components of the GPU's
    final matrix, and each recovered cluster inside one planted community for
    nearly every vertex."""
    import torch
    th0 = gen.planted_partition(40, 50, intra_deg=20.0, inter_deg=1.0, seed=43)
    t = spgemm.to_device(th0)
    changes = []
    for it in range(60):
        th = t.to_host()
        e = spgemm.matmul(t, t)
        eh = e.to_host()
        ref = oracle.product(th, th)
        assert oracle.compare(ref, eh.rpt, eh.col, eh.val) is None, f"expansion {it}"
        nt = spgemm.mcl_prune(e, 2.0, 1e-4, 0)
        nh = nt.to_host()
        check_prune_topk(eh, nh, 2.0, 1e-4, 0)
        ch = spgemm.mcl_change(t, nt)
        assert ch == oracle.mcl_change(th.rpt, th.col, th.val, nh.rpt, nh.col, nh.val)
        changes.append(ch)
        t = nt
        if ch <= 1e-6:
            break
    assert changes[-1] <= 1e-6, changes[-5:]
    lab, _ = spgemm.components(t)
    th = t.to_host()
    want = oracle.components(th.nrows, th.rpt, th.col)
    assert np.array_equal(lab.cpu().numpy(), want)
    comm = np.arange(th.nrows) // 50
    # the library loop gives the same result
    labels2, t2, iters, ch2 = apps.mcl_cluster(spgemm.to_device(th0), tol=1e-6, max_iter=60)
    assert iters == len(changes)
    assert np.array_equal(labels2.cpu().numpy(), want)
    # each cluster's vertices mostly share one planted community
    agree = 0
    for c in np.unique(want):
        members = comm[want == c]
        agree += np.bincount(members).max()
    assert agree >= 0.95 * th.nrows
    log(f"[gpu] mcl converged in {len(changes)} iterations: {len(np.unique(want))} clusters")
    torch.cuda.synchronize()
