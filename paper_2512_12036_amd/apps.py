"""Applications that chain products on the device (paper Section V).

* Graph contraction (Algorithm 7): C = S^T (A S) with the selector S
  (n x k, one 1.0 per row at the vertex's cluster); S^T is built on the
  device from the labels by a counting sort, and the intermediate P = A S
  never leaves the GPU.
* Markov clustering (Algorithm 6) on row-stochastic storage T = M^T: the
  expansion (M M)^T = T T is a product, then the device prune step raises
  entries to the inflation power, normalises each row, drops entries below
  the threshold, keeps the k largest (optional) and renormalises.  The loop
  stops when the largest entry change between successive iterates falls to
  the tolerance (or after max_iter iterations); the clusters are the
  connected components of the final matrix's pattern.
"""
from __future__ import annotations

from . import spgemm


def selector(labels, k: int) -> spgemm.DeviceCsr:
    """S (n x k) with S[v, labels[v]] = 1 on the device (rows sorted: one entry)."""
    import torch
    n = int(labels.numel())
    dev = labels.device
    rpt = torch.arange(n + 1, dtype=torch.int64, device=dev)
    return spgemm.DeviceCsr(n, k, rpt, labels.to(torch.int32),
                            torch.ones(n, dtype=torch.float32, device=dev), True)


def contract(a: spgemm.DeviceCsr, labels, k: int, options=None):
    """(P, C) with P = A S and C = S^T P, both computed and kept on the GPU."""
    s = selector(labels, k)
    st = spgemm.selector_transpose(labels, k)
    p = spgemm.matmul(a, s, options)
    c = spgemm.matmul(st, p, options)
    return p, c


def mcl(t: spgemm.DeviceCsr, iterations: int = 5, power: float = 2.0, theta: float = 1e-4,
        options=None, keep_history: bool = False, k: int = 0):
    """Runs a fixed number of iterations on T = M^T; returns the final T and,
    when asked, the list of (expansion, pruned) pairs of every iteration."""
    history = []
    for _ in range(iterations):
        e = spgemm.matmul(t, t, options)
        t = spgemm.mcl_prune(e, power, theta, k)
        if keep_history:
            history.append((e, t))
        else:
            del e
    return t, history


def mcl_cluster(t: spgemm.DeviceCsr, power: float = 2.0, theta: float = 1e-4, k: int = 0,
                tol: float = 1e-6, max_iter: int = 100, options=None):
    """The whole of Algorithm 6 on T = M^T (row-stochastic, self loops
    included): iterate expansion and pruning/inflation while the largest
    entry change between successive iterates exceeds tol (at most max_iter
    times), then interpret the final matrix.  Returns (labels, final T,
    iterations, changes): labels[v] = smallest vertex of v's cluster."""
    import torch
    changes = []
    out = torch.empty(1, dtype=torch.float64, device=t.rpt.device)
    it = 0
    while it < max_iter:
        e = spgemm.matmul(t, t, options)
        nt = spgemm.mcl_prune(e, power, theta, k)
        del e
        spgemm.mcl_change_async(t, nt, out)
        ch = float(out.item())
        changes.append(ch)
        t = nt
        it += 1
        if ch <= tol:
            break
    labels, _ = spgemm.components(t)
    return labels, t, it, changes
