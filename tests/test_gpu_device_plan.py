"""Device-driven batch plans (spgemm_plan_create_device / spgemm_execute_arena):
the whole product with no host synchronisation, C in one arena sized from the
row-size estimate.  Checked against the oracle and the ordinary batch plan,
with a too-small arena (ENOMEM, nothing written), the captured graph replayed
with new values, and plan creation + execution returning while the stream is
still busy."""
import numpy as np
import pytest

import oracle
from paper_2512_12036_amd import gen, serve, spgemm

from gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    spgemm.load()


def batch_inputs(int_values=False):
    """Products whose B has at most 1,024 columns: served requests, an
    Erdos-Renyi product, skewed rows reaching the block groups, an empty A."""
    reqs = []
    for k in range(5):
        n, d, f, rho = gen.gnn_request_params(800 + k, n_lo=300, n_hi=3000)
        reqs += serve.gnn_requests([800 + k], "cuda", n=n, d=d, f=f, rho=rho)
    As = [r.a.to_host() for r in reqs]
    Bs = [r.b.to_host() for r in reqs]
    As.append(gen.er(1000, 8000, seed=81, ncols=900))
    Bs.append(gen.er(900, 9000, seed=82, ncols=1000))
    As.append(gen.skewed_csr(800, 700, seed=83, max_len=40, heavy_rows=5, heavy_len=500))
    Bs.append(gen.skewed_csr(700, 1024, seed=84, max_len=30, heavy_rows=3, heavy_len=600))
    As.append(gen.random_csr(50, 60, 0.0, 85))
    Bs.append(gen.random_csr(60, 70, 0.2, 86))
    if int_values:
        As = [gen.int_valued(a, 90 + q) for q, a in enumerate(As)]
        Bs = [gen.int_valued(b, 95 + q) for q, b in enumerate(Bs)]
    return As, Bs


def run_device(plan, As, capacity):
    import torch
    rpts = [torch.empty(a.nrows + 1, dtype=torch.int64, device="cuda") for a in As]
    off = torch.empty(len(As) + 1, dtype=torch.int64, device="cuda")
    col = torch.full((max(capacity, 1),), -7, dtype=torch.int32, device="cuda")[:capacity]
    val = torch.full((max(capacity, 1),), -7.0, dtype=torch.float32, device="cuda")[:capacity]
    plan.execute(rpts, off, col, val)
    return rpts, off, col, val


def check(As, Bs, rpts, off, col, val, exact):
    o = off.cpu().numpy()
    for q, (a, b) in enumerate(zip(As, Bs)):
        ref = oracle.product(a, b)
        r = rpts[q].cpu().numpy()
        c = col[o[q]:o[q + 1]].cpu().numpy()
        v = val[o[q]:o[q + 1]].cpu().numpy()
        assert o[q + 1] - o[q] == ref.nnz
        assert oracle.compare(ref, r, c, v, exact_values=exact) is None, q


@pytest.mark.parametrize("exact", [False, True])
def test_device_plan_matches_oracle(exact):
    import torch
    As, Bs = batch_inputs(exact)
    dA = [spgemm.to_device(a) for a in As]
    dB = [spgemm.to_device(b) for b in Bs]
    est = serve.estimate_many(list(zip(dA, dB)))
    capacity = sum(nb for _, nb in est)
    plan = spgemm.DevicePlan(dA, dB)
    rpts, off, col, val = run_device(plan, As, capacity)
    plan.sync()
    torch.cuda.synchronize()
    check(As, Bs, rpts, off, col, val, exact)
    if exact:  # the ordinary batch plan gives the same bits
        res = spgemm.matmul_batch(dA, dB)
        o = off.cpu().numpy()
        for q, c in enumerate(res):
            assert np.array_equal(c.col.cpu().numpy(), col[o[q]:o[q + 1]].cpu().numpy())
            assert np.array_equal(c.val.cpu().numpy(), val[o[q]:o[q + 1]].cpu().numpy())
    plan.free()


def test_device_plan_arena_too_small():
    import torch
    As, Bs = batch_inputs()
    dA = [spgemm.to_device(a) for a in As]
    dB = [spgemm.to_device(b) for b in Bs]
    want = sum(oracle.product(a, b).nnz for a, b in zip(As, Bs))
    plan = spgemm.DevicePlan(dA, dB)
    rpts, off, col, val = run_device(plan, As, want - 1)
    with pytest.raises(spgemm.SpgemmError) as e:
        plan.sync()
    assert e.value.code == 5
    torch.cuda.synchronize()
    assert int(off[-1]) == want                       # the size it needs
    assert bool(torch.all(col == -7)) and bool(torch.all(val == -7.0))   # nothing written
    plan.free()
    # B wider than the block groups take: refused at creation
    wide = spgemm.to_device(gen.random_csr(30, 5000, 0.01, 87))
    with pytest.raises(spgemm.SpgemmError) as e:
        spgemm.DevicePlan([spgemm.to_device(gen.random_csr(20, 30, 0.2, 88))], [wide])
    assert e.value.code == 1


def test_device_plan_row_limit():
    """A batch of 2^26 rows or more is refused (EOVERFLOW) before anything
    is allocated or read: descriptors only, their arrays never touched."""
    import ctypes
    import torch
    lib = spgemm.load()
    small = spgemm.to_device(gen.random_csr(20, 30, 0.2, 89))
    b = small.desc(False)
    a = spgemm.CsrDesc(1 << 25, 20, 0, small.rpt.data_ptr(), None, None, 0)
    da = (spgemm.CsrDesc * 2)(a, a)
    db = (spgemm.CsrDesc * 2)(spgemm.CsrDesc(20, 30, b.nnz, b.row_ptr, b.col_idx, b.values, 0),
                              spgemm.CsrDesc(20, 30, b.nnz, b.row_ptr, b.col_idx, b.values, 0))
    h = ctypes.c_void_p()
    st = lib.spgemm_plan_create_device(ctypes.byref(h), 2, da, db, None,
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                       spgemm.ALLOC_FN(), spgemm.FREE_FN(), None)
    assert st == 4 and not h.value  # SPGEMM_EOVERFLOW, no plan


def test_device_plan_graph_replays():
    """options.graph = 1: the first call captures every launch of the plan
    (grouping to accumulation) into one graph; replays with new integer
    values, with eager work and synchronisations between them, each equal to
    the oracle bit for bit; a new arena capacity is re-captured."""
    import torch
    As, Bs = batch_inputs(True)
    dA = [spgemm.to_device(a) for a in As]
    dB = [spgemm.to_device(b) for b in Bs]
    cap = sum(oracle.product(a, b).nnz for a, b in zip(As, Bs))
    opt = spgemm.make_options(graph=1)
    plan = spgemm.DevicePlan(dA, dB, opt)
    rpts = [torch.empty(a.nrows + 1, dtype=torch.int64, device="cuda") for a in As]
    off = torch.empty(len(As) + 1, dtype=torch.int64, device="cuda")
    for rep in range(4):
        capacity = cap + (0 if rep < 3 else 1000)
        col = torch.empty(capacity, dtype=torch.int32, device="cuda")
        val = torch.empty(capacity, dtype=torch.float32, device="cuda")
        a2 = [gen.int_valued(a, 200 + 10 * rep + q) for q, a in enumerate(As)]
        b2 = [gen.int_valued(b, 300 + 10 * rep + q) for q, b in enumerate(Bs)]
        av = [torch.from_numpy(a.val).cuda() for a in a2]
        bv = [torch.from_numpy(b.val).cuda() for b in b2]
        plan.execute(rpts, off, col, val, av, bv)
        plan.sync()
        torch.cuda.synchronize()
        check(a2, b2, rpts, off, col, val, True)
        _ = (torch.ones(1000, device="cuda") * rep).sum().item()   # eager work between replays
    plan.free()


def test_device_plan_does_not_synchronise():
    import torch
    if not hasattr(torch.cuda, "_sleep"):
        pytest.skip("no device sleep in this torch build")
    As, Bs = batch_inputs()
    dA = [spgemm.to_device(a) for a in As]
    dB = [spgemm.to_device(b) for b in Bs]
    cap = sum(oracle.product(a, b).nnz for a, b in zip(As, Bs))
    rpts = [torch.empty(a.nrows + 1, dtype=torch.int64, device="cuda") for a in As]
    off = torch.empty(len(As) + 1, dtype=torch.int64, device="cuda")
    col = torch.empty(cap, dtype=torch.int32, device="cuda")
    val = torch.empty(cap, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    torch.cuda._sleep(int(2e9))       # about a second of device time, ends by itself
    plan = spgemm.DevicePlan(dA, dB)
    plan.execute(rpts, off, col, val)
    busy = not torch.cuda.current_stream().query()
    torch.cuda.synchronize()
    plan.sync()
    plan.free()
    check(As, Bs, rpts, off, col, val, False)
    assert busy, "plan creation or execution waited for the stream"
    log("[gpu] device-driven plan: created and executed while the stream was busy")
