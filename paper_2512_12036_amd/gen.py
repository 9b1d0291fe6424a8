"""Seeded synthetic inputs for the SpGEMM path.

This module only *builds inputs*: sparsity patterns and the values stored in
them.  It holds none of the product's arithmetic and is shared by the CPU
oracle tests and the GPU path alike.  Every generator is deterministic in its
seed (numpy PCG64).

Workload recipes (shapes follow the paper's evaluation workloads, see the
paper's Table II for the self-product matrices, Algorithms 6/7 for the graph
applications and Eq. 1-2 for the pruned GNN aggregation):

* ``er``: Erdos-Renyi G(n, M) with exactly M distinct positions (diagonal
  allowed), FP32 values uniform in [-1, 1].
* ``rmat``: recursive-matrix graph, directed, one quadrant draw per level with
  probabilities (a, b, c, d), no noise, no vertex permutation, self loops kept,
  duplicate edges merged before values are drawn; FP32 values in (0, 1].
* ``planted_partition``: undirected community graph with self loops,
  column-stochastic (unit weights divided by the column sum).  Stored
  transposed (row-stochastic), so that column operations become row
  operations.
* ``contraction_labels``: one uniform cluster id per vertex, and the n x k
  selector matrix S with a single 1.0 per row.
* ``gnn_request``: symmetric-normalised adjacency D^-1/2 (A + I) D^-1/2 of an
  undirected G(n, M = n d / 2) graph and a structurally pruned feature matrix
  X whose kept columns K are dense with values in (0, 1].
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Csr:
    """Host CSR matrix: int64 row pointers, int32 columns, FP32 values."""

    nrows: int
    ncols: int
    rpt: np.ndarray  # int64 [nrows + 1]
    col: np.ndarray  # int32 [nnz]
    val: np.ndarray  # float32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.rpt[-1])

    def row(self, i: int):
        s, e = int(self.rpt[i]), int(self.rpt[i + 1])
        return self.col[s:e], self.val[s:e]

    def with_values(self, val: np.ndarray) -> "Csr":
        return Csr(self.nrows, self.ncols, self.rpt, self.col,
                   np.ascontiguousarray(val, dtype=np.float32))


def from_coo(nrows: int, ncols: int, rows: np.ndarray, cols: np.ndarray,
             vals: np.ndarray | None = None, merge: bool = True) -> Csr:
    """Build a row-sorted CSR from coordinates.  With ``merge`` duplicate
    coordinates are collapsed to one entry (keeping the first value)."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    key = rows * np.int64(ncols) + cols
    if merge:
        key, first = np.unique(key, return_index=True)
        if vals is not None:
            vals = np.asarray(vals)[first]
    else:
        order = np.argsort(key, kind="stable")
        key = key[order]
        if vals is not None:
            vals = np.asarray(vals)[order]
    r = key // ncols
    c = key - r * ncols
    rpt = np.zeros(nrows + 1, dtype=np.int64)
    np.add.at(rpt, r + 1, 1)
    rpt = np.cumsum(rpt)
    if vals is None:
        vals = np.ones(key.shape[0], dtype=np.float32)
    return Csr(nrows, ncols, rpt.astype(np.int64), c.astype(np.int32),
               np.ascontiguousarray(vals, dtype=np.float32))


def _unit_open_low(rng: np.random.Generator, size) -> np.ndarray:
    """FP32 values in (0, 1]."""
    return (1.0 - rng.random(size)).astype(np.float32)


def er(n: int, nnz: int, seed: int, ncols: int | None = None,
       lo: float = -1.0, hi: float = 1.0) -> Csr:
    """G(n, M): exactly ``nnz`` distinct positions uniform over n x ncols."""
    ncols = n if ncols is None else ncols
    rng = np.random.default_rng(seed)
    total = n * ncols
    if nnz > total:
        raise ValueError("more nonzeros than positions")
    if total <= 50_000_000:
        pos = rng.choice(total, size=nnz, replace=False)
    else:
        got = np.empty(0, dtype=np.int64)
        while got.shape[0] < nnz:
            extra = rng.integers(0, total, size=int((nnz - got.shape[0]) * 1.1) + 16)
            got = np.unique(np.concatenate([got, extra]))
        pos = rng.permutation(got)[:nnz]
    pos = np.sort(pos)
    rows = pos // ncols
    cols = pos - rows * ncols
    vals = rng.uniform(lo, hi, size=nnz).astype(np.float32)
    return from_coo(n, ncols, rows, cols, vals, merge=False)


def rmat_edges(scale: int, edge_factor: int, abcd=(0.57, 0.19, 0.19, 0.05),
               seed: int = 2) -> tuple[np.ndarray, np.ndarray]:
    """Raw R-MAT samples (duplicates not merged), highest bit first."""
    a, b, c, _ = abcd
    n_edges = edge_factor * (1 << scale)
    rng = np.random.default_rng(seed)
    rows = np.zeros(n_edges, dtype=np.int64)
    cols = np.zeros(n_edges, dtype=np.int64)
    for _ in range(scale):
        u = rng.random(n_edges)
        rbit = u >= (a + b)
        cbit = ((u >= a) & (u < a + b)) | (u >= (a + b + c))
        rows = (rows << 1) | rbit
        cols = (cols << 1) | cbit
    return rows, cols


def rmat(scale: int, edge_factor: int, abcd=(0.57, 0.19, 0.19, 0.05),
         seed: int = 2) -> Csr:
    """Directed R-MAT, duplicates merged, FP32 values in (0, 1]."""
    n = 1 << scale
    rows, cols = rmat_edges(scale, edge_factor, abcd, seed)
    m = from_coo(n, n, rows, cols, None, merge=True)
    rng = np.random.default_rng(seed + 1_000_003)
    m.val = _unit_open_low(rng, m.nnz)
    return m


def planted_partition(n_comm: int = 1000, comm_size: int = 100,
                      intra_deg: float = 25.0, inter_deg: float = 5.0,
                      seed: int = 5) -> Csr:
    """Undirected community graph + self loops, column-stochastic, returned
    transposed (row i holds column i of the column-stochastic matrix)."""
    rng = np.random.default_rng(seed)
    n = n_comm * comm_size
    p_in = intra_deg / (comm_size - 1)
    p_out = inter_deg / (n - comm_size)
    iu, ju = np.triu_indices(comm_size, k=1)
    keep = rng.random((n_comm, iu.shape[0])) < p_in
    cidx, pidx = np.nonzero(keep)
    u_in = cidx * comm_size + iu[pidx]
    v_in = cidx * comm_size + ju[pidx]
    inter_pairs = n * (n - comm_size) // 2
    m_out = rng.binomial(inter_pairs, p_out)
    got_u = np.empty(0, dtype=np.int64)
    got_v = np.empty(0, dtype=np.int64)
    while got_u.shape[0] < m_out:
        need = int((m_out - got_u.shape[0]) * 1.05) + 64
        u = rng.integers(0, n, size=need)
        v = rng.integers(0, n, size=need)
        ok = (u // comm_size) != (v // comm_size)
        u, v = np.minimum(u[ok], v[ok]), np.maximum(u[ok], v[ok])
        key = np.concatenate([got_u * n + got_v, u * n + v])
        _, first = np.unique(key, return_index=True)
        first = np.sort(first)
        key = key[first]
        got_u, got_v = key // n, key % n
    got_u, got_v = got_u[:m_out], got_v[:m_out]
    diag = np.arange(n, dtype=np.int64)
    rows = np.concatenate([u_in, v_in, got_u, got_v, diag])
    cols = np.concatenate([v_in, u_in, got_v, got_u, diag])
    g = from_coo(n, n, rows, cols, None, merge=True)
    # The graph is symmetric, so column sums equal row lengths; the
    # transposed column-stochastic matrix is the row-normalised adjacency.
    deg = np.diff(g.rpt).astype(np.float64)
    rid = np.repeat(np.arange(n), np.diff(g.rpt))
    g.val = (1.0 / deg[rid]).astype(np.float32)
    return g


def contraction_labels(n: int, k: int, seed: int = 3) -> np.ndarray:
    """One uniform cluster id in [0, k) per vertex (int32)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, k, size=n).astype(np.int32)


def selector(labels: np.ndarray, k: int) -> Csr:
    """n x k matrix with S[v, labels[v]] = 1.0."""
    n = labels.shape[0]
    rpt = np.arange(n + 1, dtype=np.int64)
    return Csr(n, k, rpt, labels.astype(np.int32), np.ones(n, dtype=np.float32))


@dataclasses.dataclass
class GnnRequest:
    """One served aggregation request C = A_hat X."""

    a_hat: Csr
    x: Csr
    n: int
    avg_degree: float
    features: int
    kept: np.ndarray  # int32 sorted kept columns


def gnn_request_params(seed: int, n_lo: int = 1000, n_hi: int = 200_000):
    rng = np.random.default_rng(seed)
    n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
    d = float(rng.uniform(5.0, 50.0))
    f = int(rng.integers(64, 513))
    rho = float(rng.uniform(0.1, 0.5))
    return n, d, f, rho


def gnn_request(seed: int, n: int | None = None, d: float | None = None,
                f: int | None = None, rho: float | None = None) -> GnnRequest:
    pn, pd, pf, prho = gnn_request_params(seed)
    n = pn if n is None else n
    d = pd if d is None else d
    f = pf if f is None else f
    rho = prho if rho is None else rho
    rng = np.random.default_rng(seed * 7919 + 17)
    m_edges = int(round(n * d / 2.0))
    m_edges = min(m_edges, n * (n - 1) // 2)
    got = np.empty(0, dtype=np.int64)
    while got.shape[0] < m_edges:
        need = int((m_edges - got.shape[0]) * 1.05) + 16
        u = rng.integers(0, n, size=need)
        v = rng.integers(0, n, size=need)
        ok = u != v
        u, v = np.minimum(u[ok], v[ok]), np.maximum(u[ok], v[ok])
        key = np.concatenate([got, u * n + v])
        _, first = np.unique(key, return_index=True)
        got = key[np.sort(first)]
    got = got[:m_edges]
    u, v = got // n, got % n
    diag = np.arange(n, dtype=np.int64)
    rows = np.concatenate([u, v, diag])
    cols = np.concatenate([v, u, diag])
    a = from_coo(n, n, rows, cols, None, merge=True)
    deg = np.diff(a.rpt).astype(np.float64)
    rid = np.repeat(np.arange(n), np.diff(a.rpt))
    dinv = 1.0 / np.sqrt(deg)
    a.val = (dinv[rid] * dinv[a.col.astype(np.int64)]).astype(np.float32)
    nk = max(1, int(round(rho * f)))
    kept = np.sort(rng.choice(f, size=nk, replace=False)).astype(np.int32)
    xrpt = np.arange(n + 1, dtype=np.int64) * nk
    xcol = np.tile(kept, n)
    xval = _unit_open_low(rng, n * nk)
    x = Csr(n, f, xrpt, xcol, xval)
    return GnnRequest(a, x, n, d, f, kept)


def int_valued(m: Csr, seed: int, lo: int = -3, hi: int = 3) -> Csr:
    """Same structure, nonzero integer values in [lo, hi] (exact in FP32)."""
    rng = np.random.default_rng(seed)
    choices = np.array([v for v in range(lo, hi + 1) if v != 0], dtype=np.float32)
    return m.with_values(rng.choice(choices, size=m.nnz))


def ones_valued(m: Csr) -> Csr:
    return m.with_values(np.ones(m.nnz, dtype=np.float32))


def shuffle_rows(m: Csr, seed: int) -> Csr:
    """Same matrix with the entries of every row stored in random order."""
    rng = np.random.default_rng(seed)
    rid = np.repeat(np.arange(m.nrows), np.diff(m.rpt))
    order = np.lexsort((rng.random(m.nnz), rid))
    return Csr(m.nrows, m.ncols, m.rpt.copy(), m.col[order].copy(), m.val[order].copy())


def random_csr(nrows: int, ncols: int, density: float, seed: int,
               lo: float = -1.0, hi: float = 1.0) -> Csr:
    """Small Bernoulli(density) matrix for brute-force checks."""
    rng = np.random.default_rng(seed)
    mask = rng.random((nrows, ncols)) < density
    r, c = np.nonzero(mask)
    v = rng.uniform(lo, hi, size=r.shape[0]).astype(np.float32)
    return from_coo(nrows, ncols, r, c, v, merge=False)


def skewed_csr(nrows: int, ncols: int, seed: int, max_len: int,
               heavy_rows: int = 4, heavy_len: int | None = None) -> Csr:
    """Rows with geometric lengths plus a few very long rows; used to reach
    every bin of the multi-phase path at small size."""
    rng = np.random.default_rng(seed)
    lens = np.minimum(rng.geometric(0.15, size=nrows) - 1, max_len)
    if heavy_rows:
        idx = rng.choice(nrows, size=min(heavy_rows, nrows), replace=False)
        lens[idx] = min(ncols, heavy_len or ncols // 2)
    rows, cols = [], []
    for i, ln in enumerate(lens):
        if ln:
            cols.append(rng.choice(ncols, size=int(ln), replace=False))
            rows.append(np.full(int(ln), i, dtype=np.int64))
    if rows:
        rows = np.concatenate(rows)
        cols = np.concatenate(cols)
    else:
        rows = np.zeros(0, dtype=np.int64)
        cols = np.zeros(0, dtype=np.int64)
    vals = rng.uniform(-1.0, 1.0, size=rows.shape[0]).astype(np.float32)
    return from_coo(nrows, ncols, rows, cols, vals, merge=False)


# ---------------------------------------------------------------------------
# Device-agnostic generator for the served workload.  Built from torch integer
# and float64 operations whose results are exact (wrapping 64-bit integer
# arithmetic, correctly rounded float64 sqrt and division, exact conversions),
# so the same seed yields bit-identical matrices on the CPU and on the GPU:
# requests are generated in device memory for serving, and any of them can be
# regenerated on the host for the oracle.

def _i64(v: int) -> int:
    """An unsigned 64-bit constant as the equal-bits signed value."""
    return v - (1 << 64) if v >= (1 << 63) else v


_SM_GAMMA = _i64(0x9E3779B97F4A7C15)
_SM_M1 = _i64(0xBF58476D1CE4E5B9)
_SM_M2 = _i64(0x94D049BB133111EB)


def _lsr(x, s: int):
    """Logical right shift of an int64 tensor."""
    return (x >> s) & ((1 << (64 - s)) - 1)


def hash64(x):
    """SplitMix64 finaliser of (x + golden gamma), elementwise on an int64
    tensor (Steele, Lea and Flood, OOPSLA 2014)."""
    z = x + _SM_GAMMA
    z = (z ^ _lsr(z, 30)) * _SM_M1
    z = (z ^ _lsr(z, 27)) * _SM_M2
    return z ^ _lsr(z, 31)


def _stream(seed: int, tag: int, n: int, device):
    import torch
    idx = torch.arange(n, dtype=torch.int64, device=device)
    off = ((((seed & 0xFFFFFFFF) << 24) + (tag << 2) + 1) * 0x100000001) % (1 << 64)
    return hash64(idx * 4 + _i64(off))


def _unit_open_low_t(h):
    """(0, 1] with 24 random bits: k / 2^24, k in [1, 2^24] (exact in FP32)."""
    import torch
    return ((_lsr(h, 40) + 1).to(torch.float64) * (1.0 / (1 << 24))).to(torch.float32)


@dataclasses.dataclass
class TorchCsr:
    nrows: int
    ncols: int
    rpt: "object"  # int64 [nrows + 1]
    col: "object"  # int32 [nnz]
    val: "object"  # float32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def to_host(self) -> Csr:
        return Csr(self.nrows, self.ncols, self.rpt.cpu().numpy(), self.col.cpu().numpy(),
                   self.val.cpu().numpy())


def gnn_graph_t(seed: int, device="cpu", n: int | None = None, d: float | None = None):
    """A_hat = D^-1/2 (A + I) D^-1/2 of the served request `seed`, built on
    `device`: an undirected graph with round(n d / 2) distinct random edges
    (the first distinct ones of a hashed stream of vertex pairs)."""
    import torch
    pn, pd, _, _ = gnn_request_params(seed)
    n = pn if n is None else n
    d = pd if d is None else d
    m_edges = min(int(round(n * d / 2.0)), n * (n - 1) // 2)
    cand = int(m_edges * 1.15) + 64
    hu = _stream(seed, 1, cand, device)
    hv = _stream(seed, 2, cand, device)
    u = _lsr(hu, 1) % n
    v = _lsr(hv, 1) % n
    ok = u != v
    u, v = u[ok], v[ok]
    key = torch.minimum(u, v) * n + torch.maximum(u, v)
    uniq, inv = torch.unique(key, return_inverse=True)
    pos = torch.arange(key.shape[0], dtype=torch.int64, device=device)
    first = torch.full((uniq.shape[0],), key.shape[0], dtype=torch.int64, device=device)
    first = first.scatter_reduce(0, inv, pos, reduce="amin")
    order = torch.argsort(first)[:m_edges]
    edges = uniq[order]
    eu, ev = edges // n, edges % n
    diag = torch.arange(n, dtype=torch.int64, device=device)
    rows = torch.cat([eu, ev, diag])
    cols = torch.cat([ev, eu, diag])
    k2, _ = torch.sort(rows * n + cols)
    rows, cols = k2 // n, k2 % n
    cnt = torch.bincount(rows, minlength=n)
    rpt = torch.zeros(n + 1, dtype=torch.int64, device=device)
    rpt[1:] = torch.cumsum(cnt, 0)
    deg = cnt.to(torch.float64)
    val = (1.0 / torch.sqrt(deg[rows] * deg[cols])).to(torch.float32)
    return TorchCsr(n, n, rpt, cols.to(torch.int32), val)


def gnn_features_shape(seed: int, n: int | None = None, f: int | None = None,
                       rho: float | None = None):
    """(rows, columns, kept columns) of the served request's X."""
    pn, _, pf, prho = gnn_request_params(seed)
    n = pn if n is None else n
    f = pf if f is None else f
    rho = prho if rho is None else rho
    return n, f, max(1, int(round(rho * f)))


def gnn_features_t(seed: int, device="cpu", n: int | None = None, f: int | None = None,
                   rho: float | None = None, structure_only: bool = False):
    """X of the served request `seed` on `device`: n x f with round(rho f)
    kept columns, dense with values in (0, 1], every other column zero.  With
    structure_only, only the row pointers are built (col / val empty)."""
    import torch
    n, f, nk = gnn_features_shape(seed, n, f, rho)
    xrpt = torch.arange(n + 1, dtype=torch.int64, device=device) * nk
    if structure_only:
        empty_c = torch.zeros(0, dtype=torch.int32, device=device)
        return TorchCsr(n, f, xrpt, empty_c, torch.zeros(0, dtype=torch.float32, device=device))
    rank = torch.argsort(_stream(seed, 3, f, device))
    kept = torch.sort(rank[:nk])[0].to(torch.int32)
    xcol = kept.repeat(n)
    xval = _unit_open_low_t(_stream(seed, 4, n * nk, device))
    return TorchCsr(n, f, xrpt, xcol, xval)


def gnn_request_t(seed: int, device="cpu", n: int | None = None, d: float | None = None,
                  f: int | None = None, rho: float | None = None):
    """The served aggregation request C = A_hat X for `seed`, built on
    `device` (gnn_graph_t and gnn_features_t).  Returns (A_hat, X, (n, d, f,
    rho))."""
    pn, pd, pf, prho = gnn_request_params(seed)
    n = pn if n is None else n
    d = pd if d is None else d
    f = pf if f is None else f
    rho = prho if rho is None else rho
    a_hat = gnn_graph_t(seed, device, n, d)
    x = gnn_features_t(seed, device, n, f, rho)
    return a_hat, x, (n, d, f, rho)


# ---------------------------------------------------------------------------
# The same streams with numpy (host metadata), and the served request's
# features built in one device kernel (libspgemm_gen.so, a generator library
# of its own); both bit-identical to gnn_features_t.

_M64 = (1 << 64) - 1


def _hash64_np(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser on a uint64 array (wrapping arithmetic)."""
    with np.errstate(over="ignore"):
        z = x + np.uint64(_SM_GAMMA & _M64)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_SM_M1 & _M64)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_SM_M2 & _M64)
        return z ^ (z >> np.uint64(31))


def _stream_offset(seed: int, tag: int) -> int:
    return ((((seed & 0xFFFFFFFF) << 24) + (tag << 2) + 1) * 0x100000001) % (1 << 64)


def _stream_np(seed: int, tag: int, n: int) -> np.ndarray:
    """_stream on the host: int64 values with the same bits."""
    idx = np.arange(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        x = idx * np.uint64(4) + np.uint64(_stream_offset(seed, tag))
    return _hash64_np(x).view(np.int64)


def gnn_kept_columns(seed: int, f: int, nk: int) -> np.ndarray:
    """The kept columns of the request's X (sorted int32), as gnn_features_t
    chooses them: the nk columns of smallest stream value."""
    rank = np.argsort(_stream_np(seed, 3, f), kind="stable")
    return np.sort(rank[:nk]).astype(np.int32)


_genlib = None


def _gen_lib():
    global _genlib
    if _genlib is None:
        import ctypes
        import os
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libspgemm_gen.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
        import torch  # noqa: F401  (the HIP runtime torch holds is the one shared)
        lib = ctypes.CDLL(path)
        vp = ctypes.c_void_p
        lib.gen_gnn_features.argtypes = [ctypes.c_int64, ctypes.c_int32, vp, ctypes.c_uint64,
                                         vp, vp, vp, vp]
        lib.gen_gnn_features.restype = ctypes.c_int
        _genlib = lib
    return _genlib


def gnn_features_device(seed: int, kept, n: int, f: int, stream=None) -> TorchCsr:
    """X of the served request `seed` built by one device kernel on the
    current (or given) stream; kept: device int32 tensor of its kept columns
    (gnn_kept_columns).  Equal bit for bit to gnn_features_t."""
    import ctypes
    import torch
    dev = kept.device
    nk = int(kept.numel())
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    rpt = torch.empty(n + 1, dtype=torch.int64, device=dev)
    col = torch.empty(n * nk, dtype=torch.int32, device=dev)
    val = torch.empty(n * nk, dtype=torch.float32, device=dev)
    vp = ctypes.c_void_p
    rc = _gen_lib().gen_gnn_features(n, nk, vp(kept.data_ptr()), _stream_offset(seed, 4),
                                     vp(rpt.data_ptr()), vp(col.data_ptr()) if n else None,
                                     vp(val.data_ptr()) if n else None, vp(st.cuda_stream))
    if rc != 0:
        raise RuntimeError(f"gen_gnn_features failed ({rc})")
    return TorchCsr(n, f, rpt, col, val)
