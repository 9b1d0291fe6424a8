"""GNN layer with a pruning layer (paper Section V-C, Eq. 1-3) on the GPU.

Forward, X_l = A TopK(X_{l-1}, k) W_l:
  1. TopK(X, k) per row (spgemm_topk_rows): the sparse X (.) M_k; its
     pattern is the mask M_k;
  2. H = A TopK(X): the SpGEMM of this library (sparse times sparse);
  3. H made dense and multiplied by W on the matrix cores (spgemm_gemm_f32).
Backward, dL/dX_{l-1} = M_k (.) (A^T (dL/dX_l) W_l^T):
  1. D = G W^T on the matrix cores;
  2. A^T D evaluated only on the mask's entries (spgemm_masked_spmm), so the
     gradient is sparse with the mask's pattern;
  and the weight gradient dL/dW_l = H^T G (matrix cores, H^T as a strided
  view).  Every step runs in the library's kernels; torch holds the memory.
"""
from __future__ import annotations

from . import spgemm


def layer_forward(a_hat: spgemm.DeviceCsr, x, w, k: int, options=None):
    """Returns (X_l dense, cache) for the backward pass."""
    xk = spgemm.topk_rows(x, k)
    h = spgemm.matmul(a_hat, xk, options)
    hd = spgemm.to_dense(h)
    out = spgemm.gemm(hd, w)
    return out, (xk, hd)


def layer_backward(a_hat_t: spgemm.DeviceCsr, g, w, cache):
    """(dL/dX_{l-1} as a DeviceCsr on the mask's pattern, dL/dW_l dense).
    a_hat_t is A^T (A itself for a symmetric normalised adjacency)."""
    xk, hd = cache
    d = spgemm.gemm(g, w.t())
    dx = spgemm.masked_spmm(a_hat_t, d, xk)
    dw = spgemm.gemm(hd.t(), g)
    return spgemm.DeviceCsr(xk.nrows, xk.ncols, xk.rpt, xk.col, dx, True), dw
