"""Error paths of the C ABI on the GPU: an allocator that fails (ENOMEM, and
the plan stays freeable with every successful allocation returned), calls
out of order (ESTATE), and the chunk-item limit (EOVERFLOW).  Each failure is
forced from the host: no kernel is made to fail."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2512_12036_amd import gen, spgemm

from gpu_util import forced_options, log

pytestmark = pytest.mark.gpu

ENOMEM, EOVERFLOW, ESTATE = 5, 4, 7


class CountingAllocator:
    """torch-backed allocator callbacks that fail from the k-th request on."""

    def __init__(self, fail_at):
        import torch
        self.fail_at = fail_at
        self.live = {}
        self.calls = 0

        def _alloc(ctx, nbytes, stream):
            self.calls += 1
            if self.calls >= self.fail_at:
                return None
            p = torch.cuda.caching_allocator_alloc(int(nbytes), 0, stream or None)
            self.live[p] = nbytes
            return p

        def _free(ctx, ptr, stream):
            assert ptr in self.live, "freed a pointer the allocator never gave"
            del self.live[ptr]
            torch.cuda.caching_allocator_delete(ptr)

        self.alloc = spgemm.ALLOC_FN(_alloc)
        self.free = spgemm.FREE_FN(_free)


def create(da, db, opt, al):
    import torch
    lib = spgemm.load()
    h = ctypes.c_void_p()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    code = lib.spgemm_plan_create(ctypes.byref(h), ctypes.byref(da.desc(False)),
                                  ctypes.byref(db.desc(False)), ctypes.byref(opt), st,
                                  al.alloc, al.free, None)
    return code, h


def test_allocator_failure_at_every_point():
    """The allocator fails at its k-th call, for every k the plan reaches:
    plan creation or the symbolic phase returns ENOMEM, nothing leaks, and
    the plan (when one was returned) can still be freed."""
    import torch
    lib = spgemm.load()
    a = gen.rmat(12, 16, seed=91)
    da = spgemm.to_device(a)
    opt = spgemm.default_options()
    # number of allocations of a successful plan + symbolic phase
    ok = CountingAllocator(10 ** 9)
    code, h = create(da, da, opt, ok)
    assert code == 0
    rpt = torch.empty(a.nrows + 1, dtype=torch.int64, device="cuda")
    nnz = ctypes.c_int64()
    assert lib.spgemm_symbolic(h, ctypes.c_void_p(rpt.data_ptr()), ctypes.byref(nnz), None) == 0
    total = ok.calls
    lib.spgemm_free(h)
    assert not ok.live and total >= 2   # one reservation per planning stage
    log(f"[gpu] a plan + symbolic phase makes {total} allocations")
    saw_create, saw_symbolic = False, False
    for k in range(1, total + 1):
        al = CountingAllocator(k)
        code, h = create(da, da, opt, al)
        if code != 0:
            assert code == ENOMEM and not h.value
            saw_create = True
        else:
            c2 = lib.spgemm_symbolic(h, ctypes.c_void_p(rpt.data_ptr()), ctypes.byref(nnz), None)
            assert c2 == ENOMEM, (k, c2)
            saw_symbolic = True
            # a failed call leaves the plan freeable; numeric is out of order
            assert lib.spgemm_numeric(h, None, None, None, None) in (ESTATE, 1)
            lib.spgemm_free(h)
        torch.cuda.synchronize()
        assert not al.live, f"allocation {k}: {len(al.live)} buffers leaked"
    assert saw_create and saw_symbolic


def test_calls_out_of_order():
    import torch
    lib = spgemm.load()
    a = gen.rmat(10, 8, seed=92)
    da = spgemm.to_device(a)
    plan = spgemm.Plan(da, da)
    h = plan._handle
    col = torch.empty(1, dtype=torch.int32, device="cuda")
    val = torch.empty(1, dtype=torch.float32, device="cuda")
    vp = ctypes.c_void_p
    # numeric before symbolic
    assert lib.spgemm_numeric(h, vp(da.val.data_ptr()), vp(da.val.data_ptr()),
                              vp(col.data_ptr()), vp(val.data_ptr())) == ESTATE
    plan.symbolic()
    # symbolic twice
    rpt = torch.empty(a.nrows + 1, dtype=torch.int64, device="cuda")
    nnz = ctypes.c_int64()
    assert lib.spgemm_symbolic(h, vp(rpt.data_ptr()), ctypes.byref(nnz), None) == ESTATE
    # the plan still works after the rejected calls
    cols, vals = plan.allocate_outputs()
    plan.numeric(cols, vals)
    plan.sync()
    k = plan.nnz[0]
    ref = oracle.product(a, a)
    assert oracle.compare(ref, plan.rpts[0].cpu().numpy(), cols[0][:k].cpu().numpy(),
                          vals[0][:k].cpu().numpy()) is None
    plan.free()
    # single-product symbolic on a batch plan
    bp = spgemm.Plan([da, da], [da, da])
    assert lib.spgemm_symbolic(bp._handle, vp(rpt.data_ptr()), ctypes.byref(nnz), None) == ESTATE
    bp.free()
    # export of the numeric map before the symbolic phase
    p2 = spgemm.Plan(da, da)
    with pytest.raises(spgemm.SpgemmError) as e:
        p2.export(2)
    assert e.value.code == ESTATE
    p2.free()


def test_item_limit_overflow():
    """A plan whose chunk items exceed the item limit fails with EOVERFLOW at
    plan creation (the numeric items never outnumber the symbolic ones); at
    the limit it succeeds."""
    a = gen.rmat(12, 16, seed=93)
    da = spgemm.to_device(a)
    base = forced_options(7, 256)
    plan = spgemm.Plan(da, da, base)
    nsym = int(plan.info().sym_group_rows[7]) * int(plan.info().chunks_per_row)
    plan.symbolic()
    plan.free()
    assert nsym > 8
    for lim, where in ((nsym - 1, "create"), (1, "create")):
        o = forced_options(7, 256)
        o.item_limit = lim
        with pytest.raises(spgemm.SpgemmError) as e:
            spgemm.Plan(da, da, o)
        assert e.value.code == EOVERFLOW, where
    o = forced_options(7, 256)
    o.item_limit = nsym
    c = spgemm.matmul(da, da, o)
    ref = oracle.product(a, a)
    assert oracle.compare(ref, c.rpt.cpu().numpy(), c.col.cpu().numpy(),
                          c.val.cpu().numpy()) is None
