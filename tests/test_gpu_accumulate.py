"""FP64 accumulation of the column-chunked rows (options.accumulate = 1)
against the CPU oracle, through the C ABI.

Structure must match bit for bit.  Each value must be the oracle's FP64 sum
rounded once to FP32, up to FP64 summation error:
    |c - c*| <= 2^-24 |c*| + 2^-36 sum|a||b|.
FP32 accumulation (the default) meets the ordinary 1e-5 sum|a||b| bound but
not this one on inputs with many signed products per output, which the
tests check too, so that the tight bound tells the two modes apart.
"""
import numpy as np
import pytest

import oracle
from paper_2512_12036_amd import gen, spgemm

from gpu_util import forced_options, log, run_and_compare

pytestmark = pytest.mark.gpu

TIGHT = 2.0 ** -36


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    spgemm.load()


def signed(m, seed):
    """Same structure, values uniform in [-1, 1) (FP32)."""
    rng = np.random.default_rng(seed)
    return m.with_values(rng.uniform(-1.0, 1.0, m.nnz).astype(np.float32))


def excess(a, b, c, ref=None):
    """Largest (|c - c*| - 2^-24 |c*|) / sum|a||b| over the entries of C."""
    ref = oracle.product(a, b) if ref is None else ref
    val = c.val.cpu().numpy().astype(np.float64)
    assert val.shape == ref.val.shape
    e = np.abs(val - ref.val) - 2.0 ** -24 * np.abs(ref.val)
    return float(np.max(e / np.maximum(ref.absb, 1e-300))) if e.size else 0.0


def with_accumulate(o, acc):
    o.accumulate = acc
    return o


@pytest.mark.parametrize("chunk_cols", [256, 2048])
def test_chunked_rows_fp64(chunk_cols):
    # every row with a key above the lane groups' goes to group 7
    a = signed(gen.rmat(12, 16, seed=41), 1)
    o = with_accumulate(forced_options(7, chunk_cols), 1)
    c = run_and_compare(a, a, options=o, label=f"f64 chunk{chunk_cols}")
    ref = oracle.product(a, a)
    e64 = excess(a, a, c, ref)
    c32 = run_and_compare(a, a, options=forced_options(7, chunk_cols), label="f32 same")
    e32 = excess(a, a, c32, ref)
    log(f"[gpu] excess over one rounding / sum|a||b|: FP64 {e64:.3g}, FP32 {e32:.3g}")
    assert e64 <= TIGHT
    assert e32 > TIGHT


def test_wide_chunks_lowered():
    # chunk_cols above 2048 is lowered to 2048 by the option (the width used
    # is then at most that: a row takes a multiple of 8 chunks)
    a = signed(gen.rmat(13, 16, seed=42), 2)
    o = with_accumulate(forced_options(7, 8192), 1)
    c = run_and_compare(a, a, options=o, label="f64 chunk8192")
    assert excess(a, a, c) <= TIGHT
    plan = spgemm.Plan(spgemm.to_device(a), spgemm.to_device(a), o)
    info = plan.info()
    plan.free()
    assert 0 < info.chunk_cols <= 2048


def test_default_groups_fp64():
    a = signed(gen.rmat(13, 16, seed=43), 3)
    o = with_accumulate(spgemm.default_options(), 1)
    c = run_and_compare(a, a, options=o, label="f64 default groups")
    ref = oracle.product(a, a)
    # rows of group 7 (the chunked ones) meet the tight bound
    plan = spgemm.Plan(spgemm.to_device(a), spgemm.to_device(a), o)
    plan.symbolic()
    m, gs = plan.export(2)  # numeric row map, group by group
    heavy = (m.cpu().numpy()[gs[7]:gs[8]] & 0xffffffff).astype(np.int64)
    assert heavy.size > 0
    rpt = ref.rpt
    sel = np.concatenate([np.arange(rpt[r], rpt[r + 1]) for r in heavy])
    val = c.val.cpu().numpy().astype(np.float64)[sel]
    e = np.abs(val - ref.val[sel]) - 2.0 ** -24 * np.abs(ref.val[sel])
    assert float(np.max(e / ref.absb[sel])) <= TIGHT
    plan.free()


def test_unsorted_b_fp64():
    a = signed(gen.rmat(12, 16, seed=44), 4)
    b = gen.shuffle_rows(a, 5)
    o = with_accumulate(forced_options(7, 512), 1)
    c = run_and_compare(a, b, options=o, b_sorted=False, label="f64 unsorted B")
    assert excess(a, a, c) <= TIGHT


def test_integer_exact_fp64():
    a = gen.int_valued(gen.rmat(12, 16, seed=45), 6)
    o = with_accumulate(forced_options(7, 1024), 1)
    run_and_compare(a, a, options=o, exact=True, label="f64 integer")


def test_batch_plan_fp64():
    # three products of different widths in one batched plan
    mats = [signed(gen.rmat(11, 16, seed=46), 7), signed(gen.rmat(12, 16, seed=47), 8),
            signed(gen.skewed_csr(900, 900, seed=48, max_len=300, heavy_rows=4,
                                  heavy_len=800), 9)]
    o = with_accumulate(forced_options(7, 512), 1)
    log("[gpu] f64 batch of 3")
    cs = spgemm.matmul_batch([spgemm.to_device(m) for m in mats],
                             [spgemm.to_device(m) for m in mats], o)
    for m, c in zip(mats, cs):
        ref = oracle.product(m, m)
        msg = oracle.compare(ref, c.rpt.cpu().numpy(), c.col.cpu().numpy(), c.val.cpu().numpy())
        assert msg is None, msg
        assert excess(m, m, c, ref) <= TIGHT
