"""The GNN layer with a pruning layer (paper Section V-C, Eq. 1-3) on the
GPU against the oracle, step by step (teacher-forced: every oracle step
starts from the GPU's previous result), and its pieces: the TopK mask (bit
for bit), the FP32 GEMM on the matrix cores (bit for bit on integers,
within the FP32 summation bound otherwise, transposed operands included),
the masked backward product and the CSR transpose."""
import numpy as np
import pytest

import oracle
from paper_2512_12036_amd import gen, gnn, spgemm

from gpu_util import log

pytestmark = pytest.mark.gpu

U = 2.0 ** -24  # FP32 unit roundoff


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    spgemm.load()


def csr_host(m):
    return m.to_host()


@pytest.mark.parametrize("n,f,k", [(1000, 37, 5), (257, 512, 64), (300, 90, 90), (50, 8, 20),
                                   (2000, 300, 1)])
def test_topk_rows_bit_exact(n, f, k):
    import torch
    rng = np.random.default_rng(n + f)
    x = (np.round(rng.normal(size=(n, f)) * 3) / 3).astype(np.float32)   # many ties
    xt = torch.from_numpy(x).cuda()
    g = csr_host(spgemm.topk_rows(xt, k))
    rpt, col, val = oracle.topk_rows(x, k)
    assert np.array_equal(g.rpt, rpt) and np.array_equal(g.col, col)
    assert np.array_equal(g.val, val)


@pytest.mark.parametrize("M,N,K,ta,tb", [(300, 77, 129, False, False), (64, 64, 16, False, False),
                                         (1, 5, 3, False, False), (513, 200, 257, True, False),
                                         (129, 300, 70, False, True), (97, 65, 33, True, True),
                                         # few output tiles over a long k: split k
                                         (64, 48, 5000, True, False), (130, 70, 3001, False, False)])
def test_gemm_f32(M, N, K, ta, tb):
    import torch
    rng = np.random.default_rng(M * N + K)
    a = rng.normal(size=(K, M) if ta else (M, K)).astype(np.float32)
    b = rng.normal(size=(N, K) if tb else (K, N)).astype(np.float32)
    at = torch.from_numpy(a).cuda()
    bt = torch.from_numpy(b).cuda()
    av = at.t() if ta else at
    bv = bt.t() if tb else bt
    c = spgemm.gemm(av, bv).cpu().numpy().astype(np.float64)
    a64 = (a.T if ta else a).astype(np.float64)
    b64 = (b.T if tb else b).astype(np.float64)
    want = a64 @ b64
    bound = np.abs(a64) @ np.abs(b64)
    assert np.all(np.abs(c - want) <= K * U * bound + 1e-30)
    # integers: every product and partial sum exact in FP32
    ai = rng.integers(-4, 5, size=a.shape).astype(np.float32)
    bi = rng.integers(-4, 5, size=b.shape).astype(np.float32)
    ci = spgemm.gemm(torch.from_numpy(ai).cuda().t() if ta else torch.from_numpy(ai).cuda(),
                     torch.from_numpy(bi).cuda().t() if tb else torch.from_numpy(bi).cuda())
    wi = (ai.T if ta else ai).astype(np.float64) @ (bi.T if tb else bi).astype(np.float64)
    assert np.array_equal(ci.cpu().numpy().astype(np.float64), wi)


def test_transpose_matches_oracle():
    a = gen.rmat(12, 8, seed=51)
    t = csr_host(spgemm.transpose(spgemm.to_device(a)))
    trpt, tcol, tval = oracle.transpose(a.nrows, a.ncols, a.rpt, a.col, a.val)
    assert np.array_equal(t.rpt, trpt)
    for i in range(t.nrows):
        s, e = t.rpt[i], t.rpt[i + 1]
        o = np.argsort(t.col[s:e])
        assert np.array_equal(t.col[s:e][o], tcol[s:e]) and np.array_equal(t.val[s:e][o],
                                                                          tval[s:e])


def problem(seed, n, f, fo):
    """A_hat of the served generator (n nodes), X with ReLU-like rows, W."""
    import torch
    a = gen.gnn_graph_t(seed, "cpu", n=n)
    a = gen.Csr(a.nrows, a.ncols, a.rpt.numpy(), a.col.numpy(), a.val.numpy())
    rng = np.random.default_rng(seed)
    x = np.maximum(rng.normal(size=(n, f)), 0.0).astype(np.float32)
    w = (rng.normal(size=(f, fo)) / np.sqrt(f)).astype(np.float32)
    g = rng.normal(size=(n, fo)).astype(np.float32)
    return a, x, w, g


@pytest.mark.parametrize("n,f,fo,k", [(3000, 64, 32, 8), (20000, 256, 128, 32)])
def test_layer_teacher_forced(n, f, fo, k):
    import torch
    a, x, w, g = problem(n + f, n, f, fo)
    da = spgemm.to_device(a)
    xt, wt, gt = (torch.from_numpy(v).cuda() for v in (x, w, g))
    out, cache = gnn.layer_forward(da, xt, wt, k)
    xk_d, hd_d = cache
    xk = csr_host(xk_d)
    # mask: bit for bit
    rpt, col, val = oracle.topk_rows(x, k)
    assert np.array_equal(xk.col, col) and np.array_equal(xk.val, val)
    # H = A TopK(X): the SpGEMM against the oracle's product
    ref = oracle.product(a, xk)
    h = hd_d.cpu().numpy().astype(np.float64)
    rid = np.repeat(np.arange(a.nrows), np.diff(ref.rpt))
    hr = np.zeros_like(h)
    hr[rid, ref.col] = ref.val
    hb = np.zeros_like(h)
    hb[rid, ref.col] = ref.absb
    assert np.all(np.abs(h - hr) <= 1e-5 * hb + 1e-30)
    # X_l = H W from the GPU's H
    o = out.cpu().numpy().astype(np.float64)
    want = h @ w.astype(np.float64)
    bound = np.abs(h) @ np.abs(w.astype(np.float64))
    assert np.all(np.abs(o - want) <= f * U * bound + 1e-30)
    # backward, symmetric A_hat: A^T = A
    dx_d, dw_d = gnn.layer_backward(da, gt, wt, cache)
    dx, dxb, dw, dwb = oracle.gnn_backward(a, g.astype(np.float64), w.astype(np.float64), xk, h)
    gx = dx_d.val.cpu().numpy().astype(np.float64)
    # D = G W^T (fo terms), then at most deg + 1 terms per entry
    deg = int(np.diff(a.rpt).max())
    tol = (fo + deg + 2) * U
    assert np.all(np.abs(gx - dx) <= tol * dxb + 1e-30)
    gw = dw_d.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(gw - dw) <= n * U * dwb + 1e-30)
    log(f"[gpu] GNN layer n={n} f={f} fo={fo} k={k}: forward and backward match the oracle")


def test_layer_full_size_sampled_rows():
    """The benchmarked layer size (A_hat of the served generator with n =
    200,000 and mean degree 27, X 200,000 x 512, k = 64, W 512 x 256),
    checked on sampled outputs the oracle computes one by one: TopK on 2,000
    rows (bit for bit), H = A_hat TopK(X) on 2,000 rows including the densest
    (teacher-forced on the GPU's TopK, within the SpGEMM tolerance), X_l = H W
    and D = G W^T on those rows, the masked gradient on those rows, and 16
    columns of the weight gradient H^T G (within the FP32 summation bounds)."""
    import torch
    n, f, fo, k = 200_000, 512, 256, 64
    g_ = gen.gnn_graph_t(4242, "cpu", n=n, d=27.0)
    a = gen.Csr(g_.nrows, g_.ncols, g_.rpt.numpy(), g_.col.numpy(), g_.val.numpy())
    rng = np.random.default_rng(4242)
    x = np.maximum(rng.standard_normal((n, f), dtype=np.float32), 0.0)
    w = (rng.standard_normal((f, fo), dtype=np.float32) / np.float32(np.sqrt(f)))
    gr = rng.standard_normal((n, fo), dtype=np.float32)
    da = spgemm.to_device(a)
    xt, wt, gt = (torch.from_numpy(v).cuda() for v in (x, w, gr))
    out, cache = gnn.layer_forward(da, xt, wt, k)
    dx_d, dw_d = gnn.layer_backward(da, gt, wt, cache)
    torch.cuda.synchronize()
    xk_d, hd_d = cache
    deg = np.diff(a.rpt)
    rows = np.unique(np.concatenate([rng.choice(n, 1990, replace=False),
                                     np.argsort(deg)[-10:]])).astype(np.int64)
    # TopK, bit for bit
    xk = csr_host(xk_d)
    rpt, col, val = oracle.topk_rows(x[rows], k)
    sel = (xk.rpt[rows][:, None] + np.arange(k)[None, :]).reshape(-1)
    assert np.array_equal(xk.col[sel], col) and np.array_equal(xk.val[sel], val)
    # H on the sampled rows against the oracle's product with the GPU's TopK
    ref = oracle.product(a, xk, rows)
    h = hd_d[torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.float64)
    rid = np.repeat(np.arange(len(rows)), np.diff(ref.rpt))
    hr = np.zeros_like(h)
    hr[rid, ref.col] = ref.val
    hb = np.zeros_like(h)
    hb[rid, ref.col] = ref.absb
    assert np.all(np.abs(h - hr) <= 1e-5 * hb + 1e-30)
    # X_l = H W and the masked gradient on those rows
    w64 = w.astype(np.float64)
    o = out[torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(o - h @ w64) <= f * U * (np.abs(h) @ np.abs(w64)) + 1e-30)
    at = a  # A_hat is symmetric
    gx = dx_d.val.cpu().numpy().astype(np.float64)
    maxdeg = int(deg.max())
    for r in rows[:400]:
        nb = at.col[at.rpt[r]:at.rpt[r + 1]].astype(np.int64)
        av = at.val[at.rpt[r]:at.rpt[r + 1]].astype(np.float64)
        d_rows = gr[nb].astype(np.float64) @ w64.T          # D = G W^T on the neighbours
        d_abs = np.abs(gr[nb].astype(np.float64)) @ np.abs(w64.T)
        cs = xk.col[xk.rpt[r]:xk.rpt[r + 1]]
        want = av @ d_rows[:, cs]
        bound = np.abs(av) @ d_abs[:, cs]
        got = gx[xk.rpt[r]:xk.rpt[r + 1]]
        assert np.all(np.abs(got - want) <= (fo + maxdeg + 2) * U * bound + 1e-30), r
    # 16 columns of dW = H^T G, with the GPU's H
    cols = rng.choice(fo, 16, replace=False)
    hfull = hd_d.cpu().numpy().astype(np.float64)
    g64 = gr[:, cols].astype(np.float64)
    want = hfull.T @ g64
    bound = np.abs(hfull).T @ np.abs(g64)
    got = dw_d[:, torch.from_numpy(cols).cuda()].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - want) <= n * U * bound + 1e-30)
    log(f"[gpu] GNN layer at n={n}: sampled rows and weight-gradient columns match the oracle")
