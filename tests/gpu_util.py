"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
compare with the CPU oracle (structure bit-exact, FP32 values within
1e-5 * sum |a||b| per entry)."""
import sys

import numpy as np

import oracle
from paper_2512_12036_amd import gen, spgemm

SYM_CAP = [0, 32, 64, 128, 256, 4096, 16384]
NUM_CAP = [0, 32, 64, 128, 256, 2048, 8192]


def forced_options(group: int, chunk_cols: int | None = None, chunks_per_item: int | None = None,
                   chunk_wgs_per_cu: int | None = None, chunk_threads: int | None = None,
                   num_rank_cap: int | None = None, sym_chunk_threads: int | None = None,
                   chunk_merge: int | None = None):
    """Options that send every row whose key fits to `group` (1..7)."""
    sym = [0] * 7
    num = [0] * 7
    for g in range(1, 7):
        if g >= group:
            sym[g] = SYM_CAP[g]
            num[g] = NUM_CAP[g]
    # sym_upper[6] <= num_upper[6]
    sym[6] = min(sym[6], num[6])
    for g in range(1, 7):
        sym[g] = max(sym[g], sym[g - 1])
        num[g] = max(num[g], num[g - 1])
    return spgemm.make_options(sym, num, chunk_cols=chunk_cols, chunks_per_item=chunks_per_item,
                               chunk_wgs_per_cu=chunk_wgs_per_cu, chunk_threads=chunk_threads,
                               num_rank_cap=num_rank_cap, sym_chunk_threads=sym_chunk_threads,
                               chunk_merge=chunk_merge)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_and_compare(a, b, options=None, exact=False, rows=None, b_sorted=None, label=""):
    """Runs C = A*B on the GPU and checks it against the oracle.  Returns the
    DeviceCsr result."""
    import torch
    log(f"[gpu] {label} A {a.nrows}x{a.ncols} nnz {a.nnz}  B {b.nrows}x{b.ncols} nnz {b.nnz}")
    da = spgemm.to_device(a)
    db = spgemm.to_device(b, sorted_rows=b_sorted)
    c = spgemm.matmul(da, db, options)
    torch.cuda.synchronize()
    ref = oracle.product(a, b, rows)
    rpt = c.rpt.cpu().numpy()
    col = c.col.cpu().numpy()
    val = c.val.cpu().numpy()
    msg = oracle.compare(ref, rpt, col, val, rows=rows, exact_values=exact)
    assert msg is None, f"{label}: {msg}"
    return c


def structure_invariants(c):
    """Properties of any CSR product output: monotone row pointers and
    strictly ascending columns inside every row (checked on the GPU)."""
    import torch
    rpt = c.rpt
    assert int(rpt[0]) == 0 and int(rpt[-1]) == c.nnz
    assert bool(torch.all(rpt[1:] >= rpt[:-1]))
    if c.nnz > 1:
        col = c.col.long()
        inner = torch.ones(c.nnz - 1, dtype=torch.bool, device=col.device)
        ends = rpt[1:-1]
        ends = ends[(ends > 0) & (ends < c.nnz)]
        inner[ends - 1] = False
        d = col[1:] - col[:-1]
        assert bool(torch.all(d[inner] > 0))
        assert int(col.min()) >= 0 and int(col.max()) < c.ncols
