"""Serving layer on the GPU: every request's result is the same alone and in
the mix (structure bit for bit, values within the tolerance of each other and
of the oracle), admission by HBM budget splits the stream into batches, and
Poisson arrivals are served with overlapping batches."""
import numpy as np
import pytest

import oracle
from paper_2512_12036_amd import gen, serve, spgemm

from gpu_util import log

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    spgemm.load()


def small_requests(count, seed0=100):
    # request parameters drawn per seed, with the node count kept small so
    # the oracle finishes quickly
    reqs = []
    for k in range(count):
        n, d, f, rho = gen.gnn_request_params(seed0 + k, n_lo=300, n_hi=4000)
        reqs += serve.gnn_requests([seed0 + k], "cuda", n=n, d=d, f=f, rho=rho)
        reqs[-1].rid = k
    return reqs


def alone(req):
    plan = spgemm.Plan(req.a, req.b)
    try:
        plan.symbolic()
        cols, vals = plan.allocate_outputs()
        plan.numeric(cols, vals)
        plan.sync()
        k = plan.nnz[0]
        return plan.rpts[0].cpu().numpy(), cols[0][:k].cpu().numpy(), vals[0][:k].cpu().numpy()
    finally:
        plan.free()


def test_gpu_generator_matches_host():
    import torch
    a_d, x_d, p = gen.gnn_request_t(7, "cuda", n=3000)
    a_h, x_h, _ = gen.gnn_request_t(7, "cpu", n=3000)
    for dv, hv in [(a_d, a_h), (x_d, x_h)]:
        assert torch.equal(dv.rpt.cpu(), hv.rpt)
        assert torch.equal(dv.col.cpu(), hv.col)
        assert torch.equal(dv.val.cpu(), hv.val)


def test_same_alone_and_in_the_mix():
    reqs = small_requests(14)
    solo = {r.rid: alone(r) for r in reqs}
    srv = serve.Server(budget_bytes=8 << 30, max_batch=5, n_streams=2, keep_results=True)
    stats, done = srv.run(reqs)
    log(f"[gpu] serve mix: {stats}")
    assert stats["requests"] == len(reqs) and stats["batches"] >= 3
    by = {d.rid: d for d in done}
    for r in reqs:
        d = by[r.rid]
        rpt_s, col_s, val_s = solo[r.rid]
        k = d.nnz
        rpt_m = d.rpt.cpu().numpy()
        col_m = d.col[:k].cpu().numpy()
        val_m = d.val[:k].cpu().numpy()
        assert np.array_equal(rpt_m, rpt_s) and np.array_equal(col_m, col_s)
        ref = oracle.product(r.a.to_host(), r.b.to_host())
        # both runs within the tolerance of the oracle, hence of each other
        assert oracle.compare(ref, rpt_m, col_m, val_m) is None
        assert oracle.compare(ref, rpt_s, col_s, val_s) is None
        assert np.all(np.abs(val_m.astype(np.float64) - val_s) <= 2e-5 * ref.absb)


def test_admission_budget_splits_batches():
    reqs = small_requests(8, seed0=300)
    need = max(r.bound_bytes for r in reqs)
    srv = serve.Server(budget_bytes=int(need * 1.5), max_batch=64, n_streams=2,
                       keep_results=True)
    stats, done = srv.run(reqs)
    log(f"[gpu] serve budget: {stats}")
    assert stats["requests"] == len(reqs)
    assert stats["batches"] >= len(reqs) // 2
    assert stats["budget_waits"] + stats["budget_cuts"] >= 1
    assert stats["peak_admitted_bytes"] <= int(need * 1.5)
    # the admission bound holds: no batch's exact footprint exceeds it
    for bound, exact in stats["batch_bytes"]:
        assert exact <= bound, (exact, bound)
    with pytest.raises(ValueError):
        serve.Server(budget_bytes=need // 2).run(reqs)


def test_poisson_arrivals_and_plain_baseline():
    reqs = small_requests(24, seed0=500)
    arr = serve.poisson_arrivals(len(reqs), 400.0, seed=1)
    for r, t in zip(reqs, arr):
        r.arrival = float(t)
    stats, done = serve.Server(max_batch=8).run(reqs)
    log(f"[gpu] serve poisson: {stats}")
    assert stats["requests"] == len(reqs)
    assert stats["p99_ms"] >= stats["p50_ms"] > 0
    pstats, pdone = serve.run_plain(reqs)
    log(f"[gpu] plain: {pstats}")
    assert sorted(d.nnz for d in pdone) == sorted(d.nnz for d in done)


def test_features_built_on_admission_same_alone_and_in_the_mix():
    """B built on the device when the request is admitted (and released when
    it completes): same results as with B resident, and alone."""
    reqs = []
    for k in range(10):
        n, d, f, rho = gen.gnn_request_params(700 + k, n_lo=300, n_hi=4000)
        reqs += serve.gnn_requests([700 + k], "cuda", features_on_admission=True,
                                   n=n, d=d, f=f, rho=rho)
        reqs[-1].rid = k
    assert all(r.b is None and r.make_b is not None for r in reqs)
    stats, done = serve.Server(budget_bytes=4 << 30, max_batch=4, n_streams=2,
                               keep_results=True).run(reqs)
    assert stats["requests"] == len(reqs)
    for bound, exact in stats["batch_bytes"]:
        assert exact <= bound, (exact, bound)
    for d in done:
        r = reqs[d.rid]
        xb = d.b.to_host()
        ref = oracle.product(r.a.to_host(), xb)
        k = d.nnz
        assert oracle.compare(ref, d.rpt.cpu().numpy(), d.col[:k].cpu().numpy(),
                              d.val[:k].cpu().numpy()) is None


@pytest.mark.slow
def test_config5_full_trace_sampled_results():
    """The served workload as configured: 4,096 GNN aggregation requests,
    graphs resident, features built on admission, backlogged under a 200 GB
    HBM budget that binds (admission waits on it).  Every 64th result is
    compared with the oracle after the run."""
    import torch
    reqs = serve.gnn_requests(range(4096), "cuda", features_on_admission=True, log=log)
    keep = set(range(0, 4096, 64))
    budget = 200 * 10 ** 9
    srv = serve.Server(budget_bytes=budget, max_batch=1024, max_batch_ip=128 << 30, n_streams=4)
    stats, done = srv.run(reqs, keep_rids=keep)
    log(f"[gpu] config 5: {dict((k, v) for k, v in stats.items() if k != 'batch_bytes')}")
    assert stats["requests"] == 4096
    # the budget binds: batches closed early or admission waiting on it
    assert stats["budget_waits"] + stats["budget_cuts"] >= 1
    assert stats["peak_admitted_bytes"] <= budget
    for bound, exact in stats["batch_bytes"]:
        assert exact <= bound, (exact, bound)
    checked = 0
    for d in done:
        if d.rid not in keep:
            assert d.col is None
            continue
        r = reqs[d.rid]
        ref = oracle.product(r.a.to_host(), d.b.to_host())
        k = d.nnz
        msg = oracle.compare(ref, d.rpt.cpu().numpy(), d.col[:k].cpu().numpy(),
                             d.val[:k].cpu().numpy())
        assert msg is None, f"request {d.rid}: {msg}"
        checked += 1
    assert checked == len(keep)
    log(f"[gpu] config 5: {checked} sampled results match the oracle")
    del reqs, done
    torch.cuda.empty_cache()


def test_device_feature_generator_matches_host():
    """The one-kernel feature generator of the served requests equals the
    reference generator run on the host, bit for bit."""
    import torch
    odd = 0
    for seed, n in ((3, 5000), (900, 5000), (4095, 5000), (17, 4999), (18, 4999), (19, 1),
                    (20, 0)):
        n, f, nk = gen.gnn_features_shape(seed, n=n)
        odd += (n * nk) % 2
        kept = torch.from_numpy(gen.gnn_kept_columns(seed, f, nk)).cuda()
        xd = gen.gnn_features_device(seed, kept, n, f)
        xh = gen.gnn_features_t(seed, "cpu", n=n)
        torch.cuda.synchronize()
        assert torch.equal(xd.rpt.cpu(), xh.rpt)
        assert torch.equal(xd.col.cpu(), xh.col)
        assert torch.equal(xd.val.cpu(), xh.val)
    assert odd > 0, "no case with an odd entry count"


def test_device_driven_server_same_results():
    """Batches as device-driven plans (no host synchronisation, C in one
    arena per batch): every result equals the oracle and the ordinary
    server's, request by request."""
    reqs = []
    for k in range(12):
        n, d, f, rho = gen.gnn_request_params(900 + k, n_lo=300, n_hi=4000)
        reqs += serve.gnn_requests([900 + k], "cuda", features_on_admission=True,
                                   n=n, d=d, f=f, rho=rho)
        reqs[-1].rid = k
    stats, done = serve.Server(budget_bytes=4 << 30, max_batch=4, n_streams=2,
                               keep_results=True, device_driven=True).run(reqs)
    assert stats["requests"] == len(reqs)
    for bound, exact in stats["batch_bytes"]:
        assert exact <= bound, (exact, bound)
    for d in done:
        r = reqs[d.rid]
        ref = oracle.product(r.a.to_host(), d.b.to_host())
        assert d.nnz == ref.nnz
        assert oracle.compare(ref, d.rpt.cpu().numpy(), d.col.cpu().numpy(),
                              d.val.cpu().numpy()) is None, d.rid
