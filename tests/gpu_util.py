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


def structure_invariants(c, chunk=1 << 28):
    """Properties of any CSR product output: monotone row pointers and
    strictly ascending columns inside every row (checked on the GPU, in
    chunks of entries so that outputs of billions of entries fit)."""
    import torch
    rpt = c.rpt
    nnz = c.nnz
    assert int(rpt[0]) == 0 and int(rpt[-1]) == nnz
    assert bool(torch.all(rpt[1:] >= rpt[:-1]))
    if nnz == 0:
        return
    col = c.col
    assert int(col.min()) >= 0 and int(col.max()) < c.ncols
    if nnz < 2:
        return
    # first entry of every nonempty row
    start = torch.zeros(nnz, dtype=torch.bool, device=col.device)
    starts = rpt[:-1][rpt[1:] > rpt[:-1]]
    start[starts] = True
    for s in range(0, nnz - 1, chunk):
        e = min(nnz, s + chunk + 1)
        d = col[s + 1:e] - col[s:e - 1]          # int32: columns are below 2^31
        assert bool(torch.all((d > 0) | start[s + 1:e])), f"entries [{s}, {e})"
    del start


def compare_all_rows(a, b, c, exact=False, block_entries=40_000_000, label=""):
    """Checks EVERY row of the device result c = A*B against the oracle, in
    blocks of consecutive rows of about block_entries output entries: each
    block's columns and values are copied to the host, the oracle computes
    the same rows, and oracle.compare checks them (structure bit for bit,
    values within the tolerance or exactly)."""
    import time
    import torch
    t0 = time.perf_counter()
    rpt = c.rpt.cpu().numpy()
    assert rpt.shape[0] == a.nrows + 1 and int(rpt[0]) == 0
    m = a.nrows
    # block bounds: consecutive rows, at most block_entries entries unless one
    # row alone is larger
    cuts = [0]
    while cuts[-1] < m:
        r0 = cuts[-1]
        r1 = int(np.searchsorted(rpt, rpt[r0] + block_entries, side="right")) - 1
        cuts.append(min(m, max(r1, r0 + 1)))
    for k in range(len(cuts) - 1):
        r0, r1 = cuts[k], cuts[k + 1]
        s0, s1 = int(rpt[r0]), int(rpt[r1])
        col = c.col[s0:s1].cpu().numpy()
        val = c.val[s0:s1].cpu().numpy()
        ref = oracle.product(a, b, np.arange(r0, r1, dtype=np.int64))
        msg = oracle.compare(ref, rpt[r0:r1 + 1] - s0, col, val, exact_values=exact)
        assert msg is None, f"{label} rows [{r0}, {r1}): {msg}"
        del col, val, ref
    torch.cuda.synchronize()
    log(f"[gpu] {label}: all {m} rows ({int(rpt[-1])} entries) match the oracle in "
        f"{len(cuts) - 1} blocks, {time.perf_counter() - t0:.1f} s")
