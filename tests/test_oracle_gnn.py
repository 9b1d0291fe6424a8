"""Pins of the oracle's GNN layer (paper Section V-C, Eq. 1-3): the TopK
mask by hand and by its defining property, the forward product against a
fully dense evaluation, and the gradients against the change of the loss
L = sum(G (.) X_l) under unit perturbations (L is linear in X on a fixed
mask, and in W, so the change is the gradient exactly)."""
import numpy as np

import oracle
from paper_2512_12036_amd import gen


def test_topk_hand_example():
    x = np.array([[0.5, -2.0, 1.0, -1.0, 2.0],
                  [0.0, 0.0, 0.0, 0.0, 0.0],
                  [3.0, 1.0, -3.0, 1.0, 1.0]])
    rpt, col, val = oracle.topk_rows(x, 2)
    assert list(rpt) == [0, 2, 4, 6]
    # row 0: |-2| and |2| (columns 1 and 4); row 1: ties, lowest columns 0, 1;
    # row 2: |3| at columns 0 and 2
    assert list(col) == [1, 4, 0, 1, 0, 2]
    assert list(val) == [-2.0, 2.0, 0.0, 0.0, 3.0, -3.0]
    rpt, col, val = oracle.topk_rows(x, 3)
    assert list(col[6:9]) == [0, 1, 2]   # row 2: 3, 1 (first of the ties), -3
    rpt, col, _ = oracle.topk_rows(x, 9)
    assert list(np.diff(rpt)) == [5, 5, 5]


def test_topk_keeps_largest_magnitudes():
    rng = np.random.default_rng(1)
    x = np.round(rng.normal(size=(40, 30)) * 4) / 4      # many equal magnitudes
    rpt, col, val = oracle.topk_rows(x, 7)
    for i in range(40):
        kept = set(col[rpt[i]:rpt[i + 1]].tolist())
        lo = min(abs(x[i, j]) for j in kept)
        for j in range(30):
            if j in kept:
                continue
            assert abs(x[i, j]) <= lo
            if abs(x[i, j]) == lo:
                assert all(j > c for c in kept if abs(x[i, c]) == lo)


def _problem(seed, n=30, f=12, fo=5, k=4):
    rng = np.random.default_rng(seed)
    a = gen.random_csr(n, n, 0.15, seed, lo=-1.0, hi=1.0)
    x = rng.normal(size=(n, f)).astype(np.float32).astype(np.float64)
    w = rng.normal(size=(f, fo))
    g = rng.normal(size=(n, fo))
    return a, x, w, g, k


def _dense(a):
    d = np.zeros((a.nrows, a.ncols))
    rid = np.repeat(np.arange(a.nrows), np.diff(a.rpt))
    np.add.at(d, (rid, a.col), a.val.astype(np.float64))
    return d


def test_forward_matches_dense_evaluation():
    for seed in range(3):
        a, x, w, g, k = _problem(seed)
        out, xk, hd, hb = oracle.gnn_forward(a, x, w, k)
        mask = np.zeros_like(x)
        rid = np.repeat(np.arange(xk.nrows), np.diff(xk.rpt))
        mask[rid, xk.col] = 1.0
        want = _dense(a) @ (x * mask) @ w
        assert np.allclose(out, want, rtol=1e-12, atol=1e-12)
        assert np.all(mask.sum(axis=1) == k)


def test_gradients_match_loss_differences():
    a, x, w, g, k = _problem(7)
    out, xk, hd, _ = oracle.gnn_forward(a, x, w, k)
    dx, _, dw, _ = oracle.gnn_backward(a, g, w, xk, hd)
    mask = np.zeros_like(x)
    rid = np.repeat(np.arange(xk.nrows), np.diff(xk.rpt))
    mask[rid, xk.col] = 1.0
    ad = _dense(a)

    def loss(xx, ww):
        return float(np.sum(g * (ad @ (xx * mask) @ ww)))

    base = loss(x, w)
    for e in range(0, xk.nnz, 3):
        i, j = rid[e], xk.col[e]
        xp = x.copy()
        xp[i, j] += 1.0
        assert abs((loss(xp, w) - base) - dx[e]) <= 1e-9 * (1 + abs(dx[e]))
    for p in range(w.shape[0]):
        for q in range(w.shape[1]):
            wp = w.copy()
            wp[p, q] += 1.0
            assert abs((loss(x, wp) - base) - dw[p, q]) <= 1e-9 * (1 + abs(dw[p, q]))
    # gradients vanish off the mask: a perturbation there leaves L unchanged
    off = np.argwhere(mask == 0)[:10]
    for i, j in off:
        xp = x.copy()
        xp[i, j] += 1.0
        assert loss(xp, w) == base
