"""Matrix-based bulk sampling for mini-batch GNN training (paper Section
V-C), GraphSAGE form, on the GPU.

Every layer l, from L down to 1, takes the frontier Q^l (one one-hot row per
frontier vertex; several minibatches are simply stacked, so they are sampled
in bulk by the same launches):
  1. P = Q^l A: the SpGEMM of this library; row r is the neighbourhood
     distribution of frontier vertex r (a copy of A's row);
  2. NORM(P): rows divided by their sums (GraphSAGE);
  3. Q^{l-1} = SAMPLE(P, s): s inverse-transform draws per row (random
     numbers passed in); every draw becomes a frontier vertex of the next
     layer, in row-major order;
  4. A^l = EXTRACT(A, Q^l, Q^{l-1}) = (Q^l A) (Q^{l-1})^T: the rows of the
     frontier against the columns of the sampled vertices, a second SpGEMM
     with the transposed selector of the draws.
"""
from __future__ import annotations

from . import apps, spgemm


def one_hot(vertices, n: int) -> spgemm.DeviceCsr:
    """Q: one row per entry of `vertices` (int32 device tensor), a single
    1.0 at that vertex."""
    return apps.selector(vertices, n)


def graphsage_bulk(a: spgemm.DeviceCsr, batch, fanouts, uniforms, options=None):
    """batch: int32 device tensor of the (stacked) minibatch vertices;
    fanouts: [s_L, ..., s_1]; uniforms: one float32 device tensor per layer
    with len(frontier) * s uniforms in [0, 1).  Returns, per layer from L
    down: dict(frontier, p (NORM(P)), sampled, a_l (EXTRACT))."""
    n = a.nrows
    frontier = batch
    layers = []
    for s, u in zip(fanouts, uniforms):
        q = one_hot(frontier, n)
        p = spgemm.matmul(q, a, options)
        pn = spgemm.mcl_prune(p, 1.0, 0.0, 0)   # NORM: row normalisation
        sampled = spgemm.its_sample(p, s, u, frontier)
        qt = spgemm.selector_transpose(sampled, n)   # (Q^{l-1})^T, n x (rows * s)
        a_l = spgemm.matmul(p, qt, options)
        layers.append(dict(frontier=frontier, p=pn, sampled=sampled, a_l=a_l))
        frontier = sampled
    return layers
