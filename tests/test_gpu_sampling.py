"""Matrix-based bulk sampling (paper Section V-C) on the GPU against the
oracle: two stacked minibatches sampled in bulk through two layers; the
drawn vertices are compared bit for bit (both sides take each draw with the
same sequential FP32 sums), EXTRACT's structure and values exactly (every
entry is one product 1 * a * 1), and NORM(P) within the FP32 tolerance."""
import numpy as np
import pytest

import oracle
from paper_2512_12036_amd import gen, sampling, spgemm

from gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("scale,batches,b,fanouts", [(12, 2, 256, [10, 5]), (14, 2, 512, [8, 4])])
def test_graphsage_bulk_matches_oracle(scale, batches, b, fanouts):
    import torch
    a = gen.rmat(scale, 16, seed=70 + scale)
    rng = np.random.default_rng(scale)
    batch = np.concatenate([rng.choice(a.nrows, b, replace=False) for _ in range(batches)])
    sizes = [len(batch)]
    for s in fanouts[:-1]:
        sizes.append(sizes[-1] * s)
    uniforms = [rng.random(m * s).astype(np.float32) for m, s in zip(sizes, fanouts)]
    da = spgemm.to_device(a)
    layers = sampling.graphsage_bulk(da, torch.from_numpy(batch.astype(np.int32)).cuda(), fanouts,
                                     [torch.from_numpy(u).cuda() for u in uniforms])
    torch.cuda.synchronize()
    ref = oracle.graphsage_bulk(a, batch, fanouts, uniforms)
    for l, (g, r) in enumerate(zip(layers, ref)):
        assert np.array_equal(g["frontier"].cpu().numpy(), r["frontier"]), l
        assert np.array_equal(g["sampled"].cpu().numpy(), r["sampled"]), l
        al = g["a_l"].to_host()
        rpt, col, val = r["a_l"]
        assert np.array_equal(al.rpt, rpt) and np.array_equal(al.col, col), l
        assert np.array_equal(al.val.astype(np.float64), val), l
        # NORM(P): rows of A at the frontier, divided by their sums
        pn = g["p"].to_host()
        prpt, pcol, pval = oracle.product_rows_of(a, r["frontier"])
        assert np.array_equal(pn.rpt, prpt) and np.array_equal(pn.col, pcol)
        lens = np.diff(prpt)
        rid = np.repeat(np.arange(len(lens)), lens)
        p64 = pval.astype(np.float64)
        sums = np.bincount(rid, weights=p64, minlength=len(lens))
        want = p64 / sums[rid]
        assert np.all(np.abs(pn.val - want) <= 1e-5 * want + 1e-12), l
    log(f"[gpu] bulk sampling scale {scale}: {batches} x {b} vertices, fanouts {fanouts}: "
        f"frontiers {[len(x['sampled']) for x in ref]} match the oracle")


def test_graphsage_bulk_full_size():
    """The benchmarked sampling workload: the served generator's graph with
    2^20 vertices (mean degree about 16), 8 x 1,024 batch vertices, fanouts
    25 and 10.  Both layers against the oracle: frontiers and draws bit for
    bit, EXTRACT's structure and values exactly."""
    import torch
    g_ = gen.gnn_graph_t(90, "cpu", n=1 << 20, d=15.0)
    a = gen.Csr(g_.nrows, g_.ncols, g_.rpt.numpy(), g_.col.numpy(), g_.val.numpy())
    rng = np.random.default_rng(90)
    batch = np.concatenate([rng.choice(a.nrows, 1024, replace=False) for _ in range(8)])
    fanouts = [25, 10]
    sizes = [len(batch), len(batch) * 25]
    uniforms = [rng.random(m * s).astype(np.float32) for m, s in zip(sizes, fanouts)]
    da = spgemm.to_device(a)
    layers = sampling.graphsage_bulk(da, torch.from_numpy(batch.astype(np.int32)).cuda(),
                                     fanouts, [torch.from_numpy(u).cuda() for u in uniforms])
    torch.cuda.synchronize()
    ref = oracle.graphsage_bulk(a, batch, fanouts, uniforms)
    for l, (g, r) in enumerate(zip(layers, ref)):
        assert np.array_equal(g["frontier"].cpu().numpy(), r["frontier"]), l
        assert np.array_equal(g["sampled"].cpu().numpy(), r["sampled"]), l
        al = g["a_l"].to_host()
        rpt, col, val = r["a_l"]
        assert np.array_equal(al.rpt, rpt) and np.array_equal(al.col, col), l
        assert np.array_equal(al.val.astype(np.float64), val), l
    log(f"[gpu] bulk sampling at 2^20 vertices: {[int(r['a_l'][0][-1]) for r in ref]} "
        f"extracted entries per layer match the oracle")
