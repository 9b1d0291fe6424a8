"""The allocation-free entry point (spgemm_multiply_noalloc) against the
ordinary one (spgemm_plan_create + spgemm_symbolic + spgemm_numeric), through
the C ABI: two calls in a row, the second with a smaller input, structure bit
for bit and values exactly (integer-valued inputs) or within the tolerance;
sizes beyond the static scratch array and a too-small C are rejected with
SPGEMM_ENOMEM."""
import numpy as np
import pytest

import oracle
from paper_2512_12036_amd import gen, spgemm

from gpu_util import log

pytestmark = pytest.mark.gpu

ENOMEM = 5


def ordinary(da, db):
    c = spgemm.matmul(da, db)
    return c.rpt.cpu().numpy(), c.col.cpu().numpy(), c.val.cpu().numpy()


def noalloc(da, db, capacity=None):
    import torch
    dev = da.rpt.device
    if capacity is None:
        capacity = int(oracle.row_counts(da.to_host(), db.to_host()).sum())
    rpt = torch.empty(da.nrows + 1, dtype=torch.int64, device=dev)
    col = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)[:capacity]
    val = torch.empty(max(capacity, 1), dtype=torch.float32, device=dev)[:capacity]
    code, nnz = spgemm.multiply_noalloc(da, db, rpt, col, val)
    torch.cuda.synchronize()
    return code, nnz, rpt, col, val


def check_pair(a, b, exact, label):
    da, db = spgemm.to_device(a), spgemm.to_device(b)
    code, nnz, rpt, col, val = noalloc(da, db)
    assert code == 0, f"{label}: status {code}"
    o_rpt, o_col, o_val = ordinary(da, db)
    g_rpt = rpt.cpu().numpy()
    g_col = col[:nnz].cpu().numpy()
    g_val = val[:nnz].cpu().numpy()
    assert nnz == o_rpt[-1]
    assert np.array_equal(g_rpt, o_rpt) and np.array_equal(g_col, o_col), label
    if exact:
        assert np.array_equal(g_val, o_val), label
    ref = oracle.product(a, b)
    assert oracle.compare(ref, g_rpt, g_col, g_val, exact_values=exact) is None, label
    log(f"[gpu] noalloc {label}: nnz {nnz} matches the ordinary entry point")


def test_noalloc_matches_ordinary_twice_smaller_second():
    # first call: R-MAT 13 (every row group, chunked rows included)
    a1 = gen.int_valued(gen.rmat(13, 16, seed=81), 82)
    check_pair(a1, a1, True, "rmat13-int")
    # second call on the same scratch array, smaller input
    a2 = gen.er(2000, 16000, seed=83)
    check_pair(a2, a2, False, "er2k")


def test_noalloc_served_request_and_rejections():
    import torch
    n, d, f, rho = gen.gnn_request_params(5, n_lo=300, n_hi=4000)
    ah, xh, _ = gen.gnn_request_t(5, "cpu", n=n, d=d, f=f, rho=rho)
    check_pair(ah.to_host(), xh.to_host(), False, "gnn")
    # C larger than the caller's arrays: nnz reported, nothing else written
    a = gen.er(2000, 16000, seed=84)
    da = spgemm.to_device(a)
    want = int(oracle.row_counts(a, a).sum())
    code, nnz, rpt, _, _ = noalloc(da, da, capacity=want - 1)
    assert code == ENOMEM and nnz == want
    o_rpt, _, _ = ordinary(da, da)
    assert np.array_equal(rpt.cpu().numpy(), o_rpt)
    # a workspace beyond the static array: rejected before anything is written
    big = gen.rmat(17, 16, seed=85)
    db = spgemm.to_device(big)
    rpt = torch.empty(big.nrows + 1, dtype=torch.int64, device=db.rpt.device)
    z = torch.empty(0, dtype=torch.int32, device=db.rpt.device)
    zf = torch.empty(0, dtype=torch.float32, device=db.rpt.device)
    code, nnz = spgemm.multiply_noalloc(db, db, rpt, z, zf)
    assert code == ENOMEM and nnz == -1
    assert int(spgemm.load().spgemm_noalloc_scratch_bytes()) == 64 << 20
    # the entry point still works after a rejection
    a3 = gen.int_valued(gen.rmat(11, 8, seed=86), 87)
    check_pair(a3, a3, True, "rmat11-after-reject")
