"""CPU oracle for the hash-based multi-phase SpGEMM path.

TEST INFRASTRUCTURE ONLY.  The pytest suite, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package; the product
path (``paper_2512_12036_amd``) never does, and shares no code with it.

* ``product`` / ``row_counts`` / ``ip`` wrap the plain C + OpenMP Gustavson
  product in ``spgemm_oracle.c`` (FP64 dense accumulator, paper Section
  III-A; intermediate products per row, paper Algorithm 1).
* ``bins_reference`` is the definition of row grouping (paper Section III-B):
  every row gets the group its key falls in, and the map lists rows group by
  group, in row order inside a group.
* ``mcl_*`` are the Markov-clustering steps applied between products (paper
  Algorithm 6): Hadamard power, column normalisation and pruning, written on
  the transposed (row-stochastic) matrix so that column operations are row
  operations.
* ``mcl_prune_topk``, ``mcl_change`` and ``components`` are the top-k
  pruning, the convergence measure and the cluster interpretation of
  Algorithm 6.
* ``topk_rows``, ``gnn_forward`` and ``gnn_backward`` are the GNN layer
  with a pruning layer (paper Section V-C, Eq. 1-3).
* ``its_sample``, ``induced`` and ``graphsage_bulk`` are matrix-based bulk
  sampling (paper Section V-C).
* ``transpose`` builds S^T for graph contraction (paper Algorithm 7).

Every function here is pinned by ``tests/test_oracle*.py`` against closed
forms, brute force and library routines (see the test docstrings).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spgemm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_I64P = ctypes.POINTER(ctypes.c_int64)
_I32P = ctypes.POINTER(ctypes.c_int32)
_F32P = ctypes.POINTER(ctypes.c_float)
_F64P = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (portable x86-64 code, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c99", "-fopenmp", "-fPIC",
                               "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_ip.argtypes = [ctypes.c_int64, _I64P, _I32P, _I64P, _I64P]
        lib.oracle_row_counts.argtypes = [ctypes.c_int64, _I64P, _I32P, _I64P, _I32P,
                                          ctypes.c_int64, _I64P, _I64P]
        lib.oracle_row_values.argtypes = [ctypes.c_int64, _I64P, _I32P, _F32P, _I64P,
                                          _I32P, _F32P, ctypes.c_int64, _I64P, _I64P,
                                          _I32P, _F64P, _F64P]
        lib.oracle_max_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def _check_pair(a, b):
    if a.ncols != b.nrows:
        raise ValueError(f"inner dimensions differ: {a.ncols} vs {b.nrows}")


def ip(a, b) -> np.ndarray:
    """Intermediate products of every row of A*B (int64)."""
    _check_pair(a, b)
    out = np.zeros(a.nrows, dtype=np.int64)
    rpt_a = np.ascontiguousarray(a.rpt, dtype=np.int64)
    col_a = np.ascontiguousarray(a.col, dtype=np.int32)
    rpt_b = np.ascontiguousarray(b.rpt, dtype=np.int64)
    _load().oracle_ip(a.nrows, _p(rpt_a, _I64P), _p(col_a, _I32P), _p(rpt_b, _I64P),
                      _p(out, _I64P))
    return out


def row_counts(a, b, rows: np.ndarray | None = None) -> np.ndarray:
    """Distinct output columns of the selected rows (int64)."""
    _check_pair(a, b)
    sel = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nsel = a.nrows if sel is None else sel.shape[0]
    out = np.zeros(nsel, dtype=np.int64)
    arrs = [np.ascontiguousarray(x) for x in (a.rpt, a.col, b.rpt, b.col)]
    rc = _load().oracle_row_counts(
        b.ncols, _p(arrs[0], _I64P), _p(arrs[1], _I32P), _p(arrs[2], _I64P),
        _p(arrs[3], _I32P), nsel, None if sel is None else _p(sel, _I64P),
        _p(out, _I64P))
    if rc != 0:
        raise MemoryError("oracle_row_counts failed")
    return out


@dataclasses.dataclass
class Product:
    """Oracle rows of C: row_ptr over the selected rows, sorted columns, FP64
    values and FP64 absolute bounds."""

    rpt: np.ndarray
    col: np.ndarray
    val: np.ndarray
    absb: np.ndarray
    rows: np.ndarray | None

    @property
    def nnz(self) -> int:
        return int(self.rpt[-1])


def product(a, b, rows: np.ndarray | None = None) -> Product:
    """C = A*B (all rows, or the selected rows in the given order)."""
    _check_pair(a, b)
    counts = row_counts(a, b, rows)
    rpt = np.zeros(counts.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=rpt[1:])
    nnz = int(rpt[-1])
    col = np.zeros(nnz, dtype=np.int32)
    val = np.zeros(nnz, dtype=np.float64)
    absb = np.zeros(nnz, dtype=np.float64)
    sel = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    arrs = [np.ascontiguousarray(x) for x in (a.rpt, a.col, a.val, b.rpt, b.col, b.val)]
    rc = _load().oracle_row_values(
        b.ncols, _p(arrs[0], _I64P), _p(arrs[1], _I32P), _p(arrs[2], _F32P),
        _p(arrs[3], _I64P), _p(arrs[4], _I32P), _p(arrs[5], _F32P),
        counts.shape[0], None if sel is None else _p(sel, _I64P), _p(rpt, _I64P),
        _p(col, _I32P), _p(val, _F64P), _p(absb, _F64P))
    if rc != 0:
        raise RuntimeError(f"oracle_row_values failed ({rc})")
    return Product(rpt, col, val, absb, sel)


# --------------------------------------------------------------------------
# Row grouping (paper Section III-B): group of each row by its key, and the
# map from sorted position to original row.
# --------------------------------------------------------------------------
def bin_of(key: np.ndarray, upper: list[int]) -> np.ndarray:
    """Group id per row.  Group 0 holds rows whose key is 0; group b >= 1 the
    rows with upper[b-1] < key <= upper[b] (upper[0] = 0); keys beyond the
    last bound land in the last group, len(upper) + 1 groups in all."""
    key = np.asarray(key, dtype=np.int64)
    nb = len(upper) + 1
    bins = np.full(key.shape[0], nb - 1, dtype=np.int64)
    for t in range(nb - 2, 0, -1):      # smallest fitting group wins
        bins[key <= upper[t]] = t
    bins[key == 0] = 0
    return bins


def bins_reference(key: np.ndarray, upper: list[int], single=None, copy_group: int = 5):
    """(bins, map, offsets): map lists rows group by group, ascending row
    order inside a group; offsets[b] is where group b starts.  single: rows
    that hold one A nonzero against strictly ascending B rows; those the
    bounds would put past copy_group go to copy_group (a scaled copy of one B
    row needs no table, so the smallest block group's kernel takes it)."""
    bins = bin_of(key, upper)
    if single is not None:
        move = np.asarray(single, dtype=bool) & (bins > copy_group)
        bins[move] = copy_group
    nb = len(upper) + 1
    order = np.argsort(bins, kind="stable").astype(np.int64)
    offsets = np.zeros(nb + 1, dtype=np.int64)
    np.cumsum(np.bincount(bins, minlength=nb), out=offsets[1:])
    return bins, order, offsets


# --------------------------------------------------------------------------
# Markov clustering steps (paper Algorithm 6) on T = M^T: every column
# operation of the algorithm becomes a row operation on T.
# --------------------------------------------------------------------------
def mcl_inflate_normalize_prune(rpt, col, val, power: float, theta: float):
    """One post-expansion step on row-stochastic storage, in FP64:
    x -> x**power, divide each row by its sum, drop entries below theta
    (strictly), divide each row by the sum of what is left.  Returns the new
    (rpt, col, val) and the FP64 values before pruning (for the tolerance
    band at theta)."""
    rpt = np.asarray(rpt, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    m = rpt.shape[0] - 1
    new_cols, new_vals, counts = [], [], np.zeros(m, dtype=np.int64)
    before = np.zeros_like(val)
    for i in range(m):
        s, e = rpt[i], rpt[i + 1]
        x = val[s:e] ** power
        tot = x.sum()
        y = x / tot if tot > 0 else x
        before[s:e] = y
        keep = y >= theta
        z = y[keep]
        tz = z.sum()
        z = z / tz if tz > 0 else z
        new_cols.append(np.asarray(col[s:e])[keep])
        new_vals.append(z)
        counts[i] = z.shape[0]
    nrpt = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=nrpt[1:])
    ncol = np.concatenate(new_cols).astype(np.int32) if m else np.zeros(0, np.int32)
    nval = np.concatenate(new_vals) if m else np.zeros(0)
    return nrpt, ncol, nval, before


def mcl_prune_topk(rpt, col, val, power: float, theta: float, k: int):
    """The pruning step of Algorithm 6 with its top-k part, on row-stochastic
    storage, in FP64: x -> x**power, divide each row by its sum, drop entries
    below theta (strictly), keep only the k largest of what is left (k = 0:
    no limit; among equal values the lower columns first), divide each row
    by the sum of what it keeps.  Returns (rpt, col, val, before) like
    mcl_inflate_normalize_prune."""
    rpt = np.asarray(rpt, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    col = np.asarray(col)
    m = rpt.shape[0] - 1
    new_cols, new_vals, counts = [], [], np.zeros(m, dtype=np.int64)
    before = np.zeros_like(val)
    for i in range(m):
        s, e = rpt[i], rpt[i + 1]
        x = val[s:e] ** power
        tot = x.sum()
        y = x / tot if tot > 0 else x
        before[s:e] = y
        keep = np.nonzero(y >= theta)[0]
        if k > 0 and keep.shape[0] > k:
            # largest first; equal values in ascending column order
            order = sorted(keep, key=lambda j: (-y[j], col[s + j]))
            keep = np.sort(np.asarray(order[:k], dtype=np.int64))
        z = y[keep]
        tz = z.sum()
        z = z / tz if tz > 0 else z
        new_cols.append(col[s:e][keep])
        new_vals.append(z)
        counts[i] = z.shape[0]
    nrpt = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=nrpt[1:])
    ncol = np.concatenate(new_cols).astype(np.int32) if m else np.zeros(0, np.int32)
    nval = np.concatenate(new_vals) if m else np.zeros(0)
    return nrpt, ncol, nval, before


def mcl_change(rpt_a, col_a, val_a, rpt_b, col_b, val_b) -> float:
    """The change between successive iterates of Algorithm 6: the largest
    |a_ij - b_ij| over the union of the two patterns (an entry missing from
    one side counts as 0)."""
    m = len(rpt_a) - 1
    worst = 0.0
    for i in range(m):
        da = dict(zip(col_a[rpt_a[i]:rpt_a[i + 1]], val_a[rpt_a[i]:rpt_a[i + 1]]))
        db = dict(zip(col_b[rpt_b[i]:rpt_b[i + 1]], val_b[rpt_b[i]:rpt_b[i + 1]]))
        for c in set(da) | set(db):
            worst = max(worst, abs(float(da.get(c, 0.0)) - float(db.get(c, 0.0))))
    return worst


def components(n: int, rpt, col) -> np.ndarray:
    """Cluster interpretation of Algorithm 6's final matrix: the connected
    components of the undirected graph with an edge {i, j} for every stored
    entry (i, j) of the n x n matrix, by breadth-first search.  Each vertex
    is labelled with the smallest vertex of its component (int32)."""
    rpt = np.asarray(rpt, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    adj = [[] for _ in range(n)]
    for i in range(n):
        for j in col[rpt[i]:rpt[i + 1]]:
            adj[i].append(int(j))
            adj[int(j)].append(i)
    label = np.full(n, -1, dtype=np.int64)
    for v in range(n):              # ascending: v is its component's smallest
        if label[v] >= 0:
            continue
        label[v] = v
        frontier = [v]
        while frontier:
            nxt = []
            for u in frontier:
                for w in adj[u]:
                    if label[w] < 0:
                        label[w] = v
                        nxt.append(w)
            frontier = nxt
    return label.astype(np.int32)


# --------------------------------------------------------------------------
# GNN layer with a pruning layer (paper Section V-C, Eq. 1-3), in FP64.
# --------------------------------------------------------------------------
def topk_rows(x, k: int):
    """TopK(X, k) per row of the dense matrix x: the k entries of largest
    magnitude (equal magnitudes: lower column first), as (rpt, col, val) with
    ascending columns; the pattern is the mask M_k of Eq. 2."""
    x = np.asarray(x)
    n, f = x.shape
    kk = min(k, f)
    cols = np.zeros((n, kk), dtype=np.int32)
    for i in range(n):
        order = sorted(range(f), key=lambda j: (-abs(float(x[i, j])), j))[:kk]
        cols[i] = np.sort(order)
    rpt = np.arange(n + 1, dtype=np.int64) * kk
    col = cols.reshape(-1)
    val = x[np.repeat(np.arange(n), kk), col]
    return rpt, col, val


def gnn_forward(a, x, w, k: int):
    """X_l = A TopK(X, k) W (Eq. 1-2) with the sparse product by the
    definition (``product``) and the dense one by numpy, in FP64.  Returns
    (X_l, TopK(X) as a Csr with the input's precision, H = A TopK(X) as a
    dense FP64 array, |A| |TopK(X)| for the bounds)."""
    from paper_2512_12036_amd import gen
    rpt, col, val = topk_rows(x, k)
    xk = gen.Csr(x.shape[0], x.shape[1], rpt, col, val.astype(np.float32))
    h = product(a, xk)
    hd = np.zeros((a.nrows, x.shape[1]))
    hb = np.zeros((a.nrows, x.shape[1]))
    rid = np.repeat(np.arange(a.nrows), np.diff(h.rpt))
    hd[rid, h.col] = h.val
    hb[rid, h.col] = h.absb
    return hd @ np.asarray(w, dtype=np.float64), xk, hd, hb


def gnn_backward(a, g, w, xk, hd):
    """Eq. 3: dL/dX = M_k (.) (A^T (G W^T)), on the mask's pattern (values in
    xk's order), and dL/dW = H^T G, in FP64.  Also the bounds sum |.||.| of
    every result entry."""
    from scipy.sparse import csr_matrix
    g = np.asarray(g, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    d = g @ w.T
    db = np.abs(g) @ np.abs(w.T)
    at = csr_matrix((np.asarray(a.val, dtype=np.float64), a.col, a.rpt),
                    shape=(a.nrows, a.ncols)).T.tocsr()
    full = at @ d
    fullb = abs(at) @ db
    rid = np.repeat(np.arange(xk.nrows), np.diff(xk.rpt))
    dx = np.asarray(full)[rid, xk.col]
    dxb = np.asarray(fullb)[rid, xk.col]
    dw = hd.T @ g
    dwb = np.abs(hd).T @ np.abs(g)
    return dx, dxb, dw, dwb


# --------------------------------------------------------------------------
# Matrix-based bulk sampling (paper Section V-C), GraphSAGE form.
# --------------------------------------------------------------------------
def its_sample(rpt, col, val, u, s: int, self_v):
    """Inverse transform sampling, s draws per row: with S the FP32 sum of
    the row's weights in storage order, draw t of row r takes the column of
    the first entry whose FP32 running sum exceeds u[r, t] * S (FP32), the
    last entry if none does, and self_v[r] for a row of zero weight.  The
    sums are sequential FP32 sums, the same arithmetic the device performs,
    so the drawn integers are decided identically."""
    rpt = np.asarray(rpt, dtype=np.int64)
    val = np.asarray(val, dtype=np.float32)
    col = np.asarray(col)
    u = np.asarray(u, dtype=np.float32).reshape(-1)
    m = rpt.shape[0] - 1
    out = np.zeros(m * s, dtype=np.int32)
    for r in range(m):
        w = val[rpt[r]:rpt[r + 1]]
        c = col[rpt[r]:rpt[r + 1]]
        run = np.cumsum(w, dtype=np.float32)       # sequential FP32
        tot = run[-1] if w.shape[0] else np.float32(0)
        if not tot > 0:
            out[r * s:(r + 1) * s] = self_v[r]
            continue
        x = u[r * s:(r + 1) * s] * tot             # FP32 products
        # first entry whose running sum exceeds x (sums never decrease)
        hit = np.searchsorted(run, x, side="right")
        out[r * s:(r + 1) * s] = c[np.minimum(hit, w.shape[0] - 1)]
    return out


def induced(a, rows, cols):
    """EXTRACT(A, Q^l, Q^{l-1}): the len(rows) x len(cols) matrix with entry
    (r, c) = A[rows[r], cols[c]] wherever A stores that entry, columns
    ascending; values in FP64.  Every stored entry of a selected row is
    repeated once for each position c at which its column was drawn."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    prpt, pcol, pval = product_rows_of(a, rows)
    order = np.argsort(cols, kind="stable")
    first = np.searchsorted(cols[order], pcol, side="left")
    mult = np.searchsorted(cols[order], pcol, side="right") - first
    rid = np.repeat(np.repeat(np.arange(len(rows)), np.diff(prpt)), mult)
    base = np.repeat(first, mult)
    step = np.arange(mult.sum()) - np.repeat(np.cumsum(mult) - mult, mult)
    c = order[base + step]
    v = np.repeat(np.asarray(pval, dtype=np.float64), mult)
    srt = np.lexsort((c, rid))
    rpt = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(np.bincount(rid, minlength=len(rows)), out=rpt[1:])
    return rpt, c[srt].astype(np.int32), v[srt]


def graphsage_bulk(a, batch, fanouts, uniforms):
    """The layers of bulk sampling from the batch down: per layer the
    frontier, the drawn vertices and EXTRACT(A, frontier, draws)."""
    frontier = np.asarray(batch, dtype=np.int64)
    layers = []
    for s, u in zip(fanouts, uniforms):
        rows = product_rows_of(a, frontier)
        drawn = its_sample(rows[0], rows[1], rows[2], u, s, frontier)
        layers.append(dict(frontier=frontier, sampled=drawn,
                           a_l=induced(a, frontier, drawn)))
        frontier = drawn.astype(np.int64)
    return layers


def product_rows_of(a, vertices):
    """P = Q A for the one-hot Q of `vertices`: A's rows, in that order."""
    vertices = np.asarray(vertices, dtype=np.int64)
    rpt = np.asarray(a.rpt, dtype=np.int64)
    lens = rpt[vertices + 1] - rpt[vertices]
    prpt = np.zeros(len(vertices) + 1, dtype=np.int64)
    np.cumsum(lens, out=prpt[1:])
    idx = np.repeat(rpt[vertices] - prpt[:-1], lens) + np.arange(prpt[-1])
    return prpt, np.asarray(a.col)[idx], np.asarray(a.val)[idx]


def transpose(nrows: int, ncols: int, rpt, col, val):
    """CSR transpose with ascending columns in every output row."""
    rpt = np.asarray(rpt, dtype=np.int64)
    rid = np.repeat(np.arange(nrows, dtype=np.int64), np.diff(rpt))
    col = np.asarray(col, dtype=np.int64)
    order = np.lexsort((rid, col))
    trpt = np.zeros(ncols + 1, dtype=np.int64)
    np.cumsum(np.bincount(col, minlength=ncols), out=trpt[1:])
    return trpt, rid[order].astype(np.int32), np.asarray(val)[order]


# --------------------------------------------------------------------------
# Acceptance check shared by every parity test.
# --------------------------------------------------------------------------
FP32_REL_TOL = 1e-5


def compare(ref: Product, rpt, col, val, rows: np.ndarray | None = None,
            tol: float = FP32_REL_TOL, exact_values: bool = False):
    """Structure bit-exact; |c - c*| <= tol * sum|a||b| per entry (or exact
    equality when ``exact_values``).  ``rpt/col/val`` are the full GPU
    arrays; with ``rows`` only those rows are checked against ``ref``.
    Returns None or a message naming the first mismatch."""
    rpt = np.asarray(rpt, dtype=np.int64)
    col = np.asarray(col)
    val = np.asarray(val)
    sel = np.arange(rpt.shape[0] - 1) if rows is None else np.asarray(rows)
    if rows is None:
        if not np.array_equal(rpt - rpt[0], ref.rpt):
            bad = np.nonzero((np.diff(rpt)) != np.diff(ref.rpt))[0]
            return f"row_ptr differs (first row {bad[:5]})"
        s0, s1 = int(rpt[0]), int(rpt[-1])
        g_col = col[s0:s1]
        g_val = val[s0:s1].astype(np.float64)
    else:
        starts = rpt[sel]
        lens = rpt[sel + 1] - starts
        if not np.array_equal(lens, np.diff(ref.rpt)):
            bad = sel[np.nonzero(lens != np.diff(ref.rpt))[0]]
            return f"row lengths differ (rows {bad[:5]})"
        idx = np.concatenate([np.arange(s, s + n, dtype=np.int64)
                              for s, n in zip(starts, lens)]) if len(sel) else \
            np.zeros(0, dtype=np.int64)
        g_col = col[idx]
        g_val = val[idx].astype(np.float64)
    same = (np.array_equal(g_col, ref.col) if g_col.dtype == ref.col.dtype else
            np.array_equal(g_col.astype(np.int64), ref.col.astype(np.int64)))
    if not same:
        pos = int(np.nonzero(g_col.astype(np.int64) != ref.col)[0][0])
        return f"col_idx differs at entry {pos}"
    if exact_values:
        bad = np.nonzero(g_val != ref.val)[0]
        if bad.shape[0]:
            return f"value differs at entry {int(bad[0])}: {g_val[bad[0]]} vs {ref.val[bad[0]]}"
        return None
    err = np.abs(g_val - ref.val)
    bad = np.nonzero(err > tol * ref.absb)[0]
    if bad.shape[0]:
        i = int(bad[0])
        return (f"value out of tolerance at entry {i}: {g_val[i]} vs {ref.val[i]} "
                f"(bound {tol * ref.absb[i]})")
    return None
