"""The numeric phase captured once into a HIP graph (options.graph = 1) and
replayed for value-only re-runs: every replay, with eager GPU work and host
synchronisations between replays, must give the oracle's product for that
call's values (integer-valued inputs, so the values are exact)."""
import pytest

import oracle
from paper_2512_12036_amd import gen, spgemm

from gpu_util import forced_options, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    spgemm.load()


def _check(plan, cols, vals, As, Bs):
    plan.sync()
    for q, (a, b) in enumerate(zip(As, Bs)):
        k = plan.nnz[q]
        msg = oracle.compare(oracle.product(a, b), plan.rpts[q].cpu().numpy(),
                             cols[q][:k].cpu().numpy(), vals[q][:k].cpu().numpy(),
                             exact_values=True)
        assert msg is None, f"product {q}: {msg}"


def _replays(As, Bs, opt, label, reps=4):
    import torch
    opt.graph = 1
    log(f"[gpu] graph replays: {label}, {len(As)} product(s), {reps} calls")
    da = [spgemm.to_device(a) for a in As]
    db = [spgemm.to_device(b) for b in Bs]
    batch = len(As) > 1
    plan = spgemm.Plan(da if batch else da[0], db if batch else db[0], opt)
    try:
        plan.symbolic()
        cols, vals = plan.allocate_outputs()
        for r in range(reps):
            a_r = [gen.int_valued(a, 100 * r + q) for q, a in enumerate(As)]
            b_r = [gen.int_valued(b, 100 * r + q + 50) for q, b in enumerate(Bs)]
            if r == 2:  # fresh output buffers: the pointers travel in the descriptors
                cols, vals = plan.allocate_outputs()
            plan.numeric(cols, vals, a_vals=[torch.from_numpy(x.val).cuda() for x in a_r],
                         b_vals=[torch.from_numpy(x.val).cuda() for x in b_r])
            _check(plan, cols, vals, a_r, b_r)
            # eager work and a synchronisation between replays
            x = torch.randn(1 << 20, device="cuda")
            assert torch.isfinite(x.sum())
            torch.cuda.synchronize()
    finally:
        plan.free()


def test_graph_default_groups():
    # R-MAT reaches the small, block and chunk groups with the defaults
    a = gen.rmat(13, 16, seed=71)
    _replays([a], [a], spgemm.make_options(), "rmat13 defaults")


@pytest.mark.parametrize("merge", [1, 2])
def test_graph_chunk_launches(merge):
    # every row as column chunks: dense and rank launches, single and merged
    a = gen.rmat(12, 16, seed=72)
    _replays([a], [a], forced_options(7, chunk_cols=512, chunk_merge=merge),
             f"rmat12 chunks merge {merge}")


def test_graph_batch():
    As = [gen.rmat(11, 8, seed=80 + i) for i in range(3)]
    Bs = [gen.random_csr(a.ncols, 300 + 100 * i, 0.02, 90 + i) for i, a in enumerate(As)]
    _replays(As, Bs, spgemm.make_options(), "batch of 3")


def test_graph_ignored_when_profiling():
    a = gen.rmat(10, 8, seed=5)
    opt = spgemm.make_options(profile=1)
    _replays([a], [a], opt, "profile on", reps=2)


def test_library_loaded_before_torch():
    # options built (so the library loaded) before torch is imported: the
    # binding must still end with one HIP runtime in the process
    import subprocess
    import sys
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2512_12036_amd import gen, spgemm\n"
            "opt = spgemm.make_options(graph=1)\n"
            "import torch\n"
            "a = spgemm.to_device(gen.rmat(9, 8, seed=4))\n"
            "c = spgemm.matmul(a, a, opt)\n"
            "torch.cuda.synchronize()\n"
            "print('nnz', c.nnz)\n") % root
    log("[gpu] fresh process: library loaded before torch")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       timeout=100)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "nnz" in r.stdout


def test_graph_unsorted_b():
    # rows of B stored out of order: the chunk kernels without sub-range
    # tables, captured the same way
    a = gen.rmat(12, 16, seed=73)
    b = gen.shuffle_rows(a, 9)
    _replays([a], [b], forced_options(7, chunk_cols=1024), "rmat12 unsorted B")


def test_graph_degenerate_products():
    # empty shapes and an all-zero A capture a graph with nothing to launch;
    # every call must still succeed and give the (empty) product
    for (m, k, n) in [(0, 5, 7), (5, 0, 7), (5, 7, 0), (1, 1, 1)]:
        a = gen.random_csr(m, k, 0.5, 1)
        b = gen.random_csr(k, n, 0.5, 2)
        _replays([a], [b], spgemm.make_options(), f"degenerate {(m, k, n)}", reps=2)
    z = gen.random_csr(100, 80, 0.0, 1)
    _replays([z], [gen.random_csr(80, 90, 0.3, 2)], spgemm.make_options(), "zero A", reps=2)
