"""Full-size parity on the benchmarked workload (R-MAT scale 18 self-product,
1.28e9 output entries) in the launch configuration the benchmark uses, and on
R-MAT scale 16, whose B has 65,536 columns: the same chunk width (8,192
columns), rank cap and merging, so the same kernel instantiations run as in
the benchmark.

Every row of every result is compared with the oracle: the oracle computes
consecutive row blocks of C and each block is checked against the device
arrays (structure bit for bit, values within 1e-5 * sum |a||b| per entry, or
exactly for integer-valued inputs).  Properties that hold at any size are
checked on all of C as well: monotone row pointers, strictly ascending columns
inside rows, and the row-sum identity C 1 = A (B 1) within the summed
per-entry tolerance.
"""
import numpy as np
import pytest

import oracle
from paper_2512_12036_amd import gen, spgemm

from gpu_util import compare_all_rows, log, structure_invariants

pytestmark = pytest.mark.gpu


def row_sum_identity(a, b, c):
    import torch
    dev = c.col.device
    m = c.nrows
    rid = torch.repeat_interleave(torch.arange(m, device=dev), c.rpt[1:] - c.rpt[:-1])
    got = torch.zeros(m, dtype=torch.float64, device=dev)
    got.index_add_(0, rid, c.val.double())
    del rid
    b_rid = np.repeat(np.arange(b.nrows), np.diff(b.rpt))
    b1 = np.bincount(b_rid, weights=b.val.astype(np.float64), minlength=b.nrows)
    b1a = np.bincount(b_rid, weights=np.abs(b.val.astype(np.float64)), minlength=b.nrows)
    a_rid = np.repeat(np.arange(a.nrows), np.diff(a.rpt))
    av = a.val.astype(np.float64)
    want = np.bincount(a_rid, weights=av * b1[a.col], minlength=a.nrows)
    bound = np.bincount(a_rid, weights=np.abs(av) * b1a[a.col], minlength=a.nrows)
    err = np.abs(got.cpu().numpy() - want)
    assert np.all(err <= 1e-5 * bound + 1e-30), int(np.argmax(err - 1e-5 * bound))


def used_group_bounds():
    """Every group bound the default options use, plus the rank cap and half
    of it (the split points of the chunk launches)."""
    o = spgemm.default_options()
    t = set(int(v) for v in o.sym_upper[1:]) | set(int(v) for v in o.num_upper[1:])
    t |= {int(o.num_rank_cap), int(o.num_rank_cap) // 2}
    return sorted(v for v in t if v > 0)


def test_rmat18_full_size_every_row():
    """The benchmark's product, default options: every row of C against the
    oracle."""
    import torch
    a = gen.rmat(18, 16, seed=2)
    log(f"[gpu] R-MAT 18: {a.nnz} nnz")
    da = spgemm.to_device(a)
    c = spgemm.matmul(da, da)
    torch.cuda.synchronize()
    log(f"[gpu] nnz(C) = {c.nnz}")
    counts = np.diff(c.rpt.cpu().numpy())
    # rows close to both sides of every bound in use exist in this workload
    # (so the block compare below covers both sides of each)
    for t in used_group_bounds():
        assert np.any((counts > t - 8) & (counts <= t)), t
        assert np.any((counts > t) & (counts <= t + 8)), t
    structure_invariants(c)
    row_sum_identity(a, a, c)
    compare_all_rows(a, a, c, label="R-MAT 18")


@pytest.mark.parametrize("values", ["ones", "int", "float"])
def test_rmat16_full_size_every_row(values):
    """R-MAT 16 self-product (B: 65,536 columns, chunk width 8,192, rank cap
    2,048, merged items) with default options, every row compared.  With
    all-ones values every entry is an exact path count, and with integer
    values in [-3, 3] every partial sum is an integer below 2^24: both are
    compared bit for bit; uniform (0, 1] values within the tolerance."""
    import torch
    base = gen.rmat(16, 16, seed=2)
    a = {"ones": lambda: gen.ones_valued(base), "int": lambda: gen.int_valued(base, 61),
         "float": lambda: base}[values]()
    da = spgemm.to_device(a)
    plan = spgemm.Plan(da, da)
    plan.symbolic()
    inf = plan.info()
    assert inf.chunk_cols == 8192 and inf.num_group_rows[7] > 0
    cols, vals = plan.allocate_outputs()
    plan.numeric(cols, vals)
    plan.sync()
    c = plan.results(cols, vals)[0]
    plan.free()
    torch.cuda.synchronize()
    structure_invariants(c)
    compare_all_rows(a, a, c, exact=(values != "float"), label=f"R-MAT 16 {values}")


@pytest.mark.parametrize("m,kper", [(70_000, 1), (140_000, 2)])
def test_chunk_items_beyond_one_grid(m, kper):
    """More column-chunk work than one 1-D grid holds (the dispatch packet
    counts work-items in 32 bits): rows of about 1,800 products each against
    a B of 2^21 columns, 256 chunks per row.  B's rows are stored out of
    order, so the plan sorts them first.  With one chunk per item the
    pipelined kernels take the 17.9 million items with a capped grid; with
    two chunks per item (140,000 rows) the one-workgroup-per-item kernels
    take 17.9 million 256-lane workgroups, a grid split over two dimensions.
    Every row against the oracle, exactly (integer values)."""
    import torch
    rng = np.random.default_rng(2024)
    nb, ncols, blen = 16, 1 << 21, 900
    b_col = np.concatenate([rng.choice(ncols, blen, replace=False) for _ in range(nb)])
    b = gen.Csr(nb, ncols, np.arange(nb + 1, dtype=np.int64) * blen, b_col.astype(np.int32),
                rng.integers(1, 4, nb * blen).astype(np.float32))
    a_col = np.sort(np.stack([rng.choice(nb, 2, replace=False) for _ in range(m)]), axis=1)
    a = gen.Csr(m, nb, np.arange(m + 1, dtype=np.int64) * 2, a_col.reshape(-1).astype(np.int32),
                rng.integers(1, 4, 2 * m).astype(np.float32))
    da, db = spgemm.to_device(a), spgemm.to_device(b, sorted_rows=False)
    opt = spgemm.make_options(chunks_per_item=kper)
    plan = spgemm.Plan(da, db, opt)
    info = plan.info()
    items = info.chunks_per_row * m // kper
    assert info.sym_group_rows[7] == m and items * 256 >= 1 << 32
    plan.free()
    c = spgemm.matmul(da, db, opt)
    torch.cuda.synchronize()
    log(f"[gpu] beyond one grid (kper {kper}): nnz(C) = {c.nnz}, {items} chunk items")
    structure_invariants(c)
    compare_all_rows(a, b, c, exact=True, label=f"beyond one grid, kper {kper}")
