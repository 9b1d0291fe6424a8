"""Row-block sharding of one product C = A * B, rehearsed on one GPU.

Several GPUs would split C = A * B by contiguous row blocks of A (and so of
C), with B replicated: the rows are cut into P ranges of about equal
intermediate-product sums, from the prefix sum of the per-row counts that
the plan already computes (paper Algorithm 1), and every GPU runs the
unchanged pipeline on its range.  Here the P row-block products run as one
batch plan on one GPU and their results are concatenated, which checks the
split and the reassembly against the whole product; the broadcast of B and
the cross-GPU balance are not exercised.
"""
from __future__ import annotations

from . import spgemm


def row_ranges(ip, parts: int) -> list[tuple[int, int]]:
    """Contiguous row ranges [r0, r1) covering every row, cut where the
    prefix sum of `ip` (int64 tensor, one entry per row) crosses k/parts of
    the total, k = 1 .. parts - 1.  Empty ranges are dropped."""
    import torch
    if parts < 1:
        raise ValueError("parts must be positive")
    m = int(ip.numel())
    if m == 0:
        return []
    prefix = torch.cumsum(ip.to(torch.int64), 0)
    total = int(prefix[-1])
    targets = torch.tensor([(total * k + parts - 1) // parts for k in range(1, parts)],
                           dtype=torch.int64, device=prefix.device)
    # first row whose inclusive prefix reaches the target ends the range
    cuts = (torch.searchsorted(prefix, targets) + 1).clamp(max=m).tolist() if parts > 1 else []
    bounds = [0] + cuts + [m]
    return [(r0, r1) for r0, r1 in zip(bounds[:-1], bounds[1:]) if r1 > r0]


def row_block(a: spgemm.DeviceCsr, r0: int, r1: int) -> spgemm.DeviceCsr:
    """Rows [r0, r1) of A as a CSR matrix of its own (row pointers rebased,
    columns and values viewed in place)."""
    j0, j1 = int(a.rpt[r0]), int(a.rpt[r1])
    return spgemm.DeviceCsr(r1 - r0, a.ncols, a.rpt[r0:r1 + 1] - j0, a.col[j0:j1],
                            a.val[j0:j1], a.sorted_rows)


def sharded_matmul(a: spgemm.DeviceCsr, b: spgemm.DeviceCsr, parts: int,
                   options: spgemm.Options | None = None):
    """C = A * B computed as `parts` row-block products (one batch plan) and
    concatenated.  Returns (C as DeviceCsr, the row ranges used)."""
    import torch
    whole = spgemm.Plan(a, b, options)
    ip, _ = whole.export(0)
    whole.free()
    ranges = row_ranges(ip, parts)
    if not ranges:
        return spgemm.matmul(a, b, options), ranges
    blocks = [row_block(a, r0, r1) for r0, r1 in ranges]
    parts_c = spgemm.matmul_batch(blocks, [b] * len(blocks), options)
    rpts, off = [], 0
    for c in parts_c:
        rpts.append(c.rpt[:-1] + off)
        off += c.nnz
    dev = parts_c[0].rpt.device
    rpt = torch.cat(rpts + [torch.tensor([off], dtype=torch.int64, device=dev)])
    col = torch.cat([c.col for c in parts_c])
    val = torch.cat([c.val for c in parts_c])
    return spgemm.DeviceCsr(a.nrows, b.ncols, rpt, col, val, True), ranges
