"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Structure (row_ptr, col_idx, explicit zeros included) must match the oracle
bit for bit; FP32 values must satisfy |c - c*| <= 1e-5 * sum|a||b| per entry;
integer-valued inputs must match exactly.  Every row group (kernel) is forced
in turn on inputs that span several workgroups and a ragged tail.
"""
import numpy as np
import pytest

import oracle
from paper_2512_12036_amd import gen, spgemm

from gpu_util import forced_options, log, run_and_compare, structure_invariants

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    spgemm.load()


def test_er_config_small():
    a = gen.er(2000, 16000, seed=1)
    c = run_and_compare(a, a, label="er2k")
    structure_invariants(c)


@pytest.mark.parametrize("group", [1, 2, 3, 4, 5, 6, 7])
def test_forced_group_ragged(group):
    # rows of every length up to a few hundred, plus empty rows
    a = gen.skewed_csr(3001, 2500, seed=10 + group, max_len=12, heavy_rows=0)
    b = gen.skewed_csr(2500, 2700, seed=20 + group, max_len=9, heavy_rows=0)
    run_and_compare(a, b, options=forced_options(group), label=f"group{group}")


@pytest.mark.parametrize("group", [1, 4, 5, 6, 7])
def test_forced_group_integer_exact(group):
    a = gen.int_valued(gen.skewed_csr(1500, 1200, seed=31, max_len=10, heavy_rows=0), 1)
    b = gen.int_valued(gen.skewed_csr(1200, 1300, seed=32, max_len=10, heavy_rows=0), 2)
    run_and_compare(a, b, options=forced_options(group), exact=True, label=f"int{group}")


def test_rmat_default_groups():
    a = gen.rmat(13, 16, seed=7)
    c = run_and_compare(a, a, label="rmat13")
    structure_invariants(c)


@pytest.mark.parametrize("chunk_cols", [64, 256, 4096])
def test_chunk_widths(chunk_cols):
    a = gen.rmat(12, 16, seed=9)
    run_and_compare(a, a, options=forced_options(7, chunk_cols), label=f"chunk{chunk_cols}")


@pytest.mark.parametrize("kper", [1, 2, 4, 8])
def test_chunks_per_item(kper):
    a = gen.rmat(12, 16, seed=10)
    run_and_compare(a, a, options=forced_options(7, 256, kper), label=f"kper{kper}")
    b = gen.shuffle_rows(a, 7)
    run_and_compare(a, b, options=forced_options(7, 512, kper), b_sorted=False,
                    label=f"kper{kper}-unsorted")


@pytest.mark.parametrize("chunk_cols,wgs", [(256, 1), (2048, 2), (4096, 4), (8192, 8),
                                             (16384, 3)])
def test_chunk_resident_workgroups(chunk_cols, wgs):
    # a fixed grid of resident workgroups walking the chunk items (several
    # items per workgroup, next item's inputs prefetched)
    a = gen.rmat(12, 16, seed=14)
    run_and_compare(a, a, options=forced_options(7, chunk_cols, 1, wgs, None, 0),
                    label=f"wgs{wgs}")
    ai = gen.int_valued(a, 3)
    run_and_compare(ai, ai, options=forced_options(7, chunk_cols, 1, wgs, None, 512), exact=True,
                    label=f"wgs{wgs}-int")


@pytest.mark.parametrize("chunk_cols,threads", [(2048, 256), (4096, 64), (8192, 64),
                                                 (8192, 512), (16384, 128)])
def test_chunk_workgroup_sizes(chunk_cols, threads):
    a = gen.rmat(12, 16, seed=15)
    # rank accumulator off: every chunk takes the dense kernel
    run_and_compare(a, a, options=forced_options(7, chunk_cols, 1, None, threads, 0),
                    label=f"thr{threads}")
    run_and_compare(a, a, options=forced_options(7, chunk_cols, 1, 2, threads, 0),
                    label=f"thr{threads}-wgs2")


@pytest.mark.parametrize("chunk_cols,cap,sym_threads", [(256, 512, 64), (2048, 1024, 128),
                                                        (8192, 2048, 256), (16384, 1024, 512),
                                                        (4096, 512, 0)])
def test_chunk_rank_accumulator(chunk_cols, cap, sym_threads):
    # chunks with at most `cap` outputs go to the compact rank accumulator,
    # the others to the dense one
    a = gen.rmat(13, 16, seed=16)
    run_and_compare(a, a, options=forced_options(7, chunk_cols, 1, None, None, cap, sym_threads),
                    label=f"rank{cap}")
    ai = gen.int_valued(gen.rmat(12, 16, seed=17), 4)
    run_and_compare(ai, ai, options=forced_options(7, chunk_cols, 1, None, None, cap,
                                                   sym_threads), exact=True, label=f"rank{cap}-int")


@pytest.mark.parametrize("chunk_cols,cap,merge", [(256, 512, 2), (256, 1024, 4), (512, 2048, 8),
                                                   (2048, 1024, 8), (8192, 1024, 4),
                                                   (16384, 2048, 8), (4096, 512, 1)])
def test_chunk_merging(chunk_cols, cap, merge):
    # adjacent light chunks of a row merged into one item (products within the
    # rank cap, at most `merge` chunks, at most 65536 columns)
    a = gen.rmat(13, 16, seed=18)
    run_and_compare(a, a, options=forced_options(7, chunk_cols, 1, None, None, cap,
                                                 chunk_merge=merge), label=f"merge{merge}")
    ai = gen.int_valued(gen.rmat(12, 16, seed=19), 5)
    run_and_compare(ai, ai, options=forced_options(7, chunk_cols, 1, None, None, cap,
                                                   chunk_merge=merge), exact=True,
                    label=f"merge{merge}-int")
    # ragged: B's columns not a multiple of the chunk width
    b = gen.skewed_csr(a.ncols, 7001, seed=20, max_len=40, heavy_rows=5, heavy_len=3000)
    run_and_compare(a, b, options=forced_options(7, chunk_cols, 1, None, None, cap,
                                                 chunk_merge=merge), label=f"merge{merge}-ragged")


def test_chunk_merging_many_chunks():
    # rows with more chunks than the merge table holds (512 chunks of 64
    # columns) keep one item per chunk, next to merged rows of a second
    # product (64 chunks) in the same batch
    import torch
    a1 = gen.rmat(15, 8, seed=21)
    a2 = gen.rmat(12, 16, seed=22)
    opt = forced_options(7, 64, 1, None, None, 1024, chunk_merge=8)
    log("[gpu] merge batch: rmat15 (512 chunks per row) + rmat12 (64 chunks per row)")
    d1, d2 = spgemm.to_device(a1), spgemm.to_device(a2)
    plan = spgemm.Plan([d1, d2], [d1, d2], opt)
    plan.symbolic()
    cols, vals = plan.allocate_outputs()
    plan.numeric(cols, vals)
    torch.cuda.synchronize()
    for a, rpt, col, val, rows in ((a1, plan.rpts[0], cols[0], vals[0], np.arange(0, a1.nrows, 97)),
                                   (a2, plan.rpts[1], cols[1], vals[1], None)):
        ref = oracle.product(a, a, rows)
        msg = oracle.compare(ref, rpt.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy(),
                             rows=rows)
        assert msg is None, msg
    plan.free()


def test_chunk_unsorted_b():
    a = gen.rmat(11, 16, seed=12)
    b = gen.shuffle_rows(a, 3)
    run_and_compare(a, b, options=forced_options(7, 128), b_sorted=False, label="unsortedB")
    run_and_compare(a, b, options=None, b_sorted=False, label="unsortedB-default")


def test_unsorted_b_detected_on_device():
    a = gen.rmat(11, 16, seed=13)
    b = gen.shuffle_rows(a, 4)
    # flag absent: the library detects the order itself
    run_and_compare(a, b, options=forced_options(7, 256), b_sorted=False, label="detect")


def test_heavy_rows_mixed():
    a = gen.skewed_csr(2000, 3000, seed=40, max_len=30, heavy_rows=6, heavy_len=1500)
    b = gen.skewed_csr(3000, 5000, seed=41, max_len=40, heavy_rows=3, heavy_len=2500)
    run_and_compare(a, b, label="heavy-mixed")
    run_and_compare(a, b, options=forced_options(7, 512), label="heavy-chunks")


def with_duplicates(m, seed, frac=0.3):
    """Same matrix plus a second stored copy of a random fraction of its
    entries (same row and column, its own value), appended at the row's end:
    duplicate coordinates that the product must sum."""
    rng = np.random.default_rng(seed)
    rid = np.repeat(np.arange(m.nrows), np.diff(m.rpt))
    pick = np.nonzero(rng.random(m.nnz) < frac)[0]
    rows = np.concatenate([rid, rid[pick]])
    cols = np.concatenate([m.col, m.col[pick]])
    vals = np.concatenate([m.val, rng.choice(np.array([-2, -1, 1, 2], np.float32), pick.size)])
    order = np.argsort(rows, kind="stable")
    out = gen.from_coo(m.nrows, m.ncols, rows[order], cols[order], vals[order], merge=False)
    # from_coo sorts by (row, col): the copies sit next to their originals
    assert out.nnz == m.nnz + pick.size
    return out


@pytest.mark.parametrize("group", [None, 1, 4, 5, 7])
def test_duplicate_entries_are_summed(group):
    """Duplicate (row, col) entries in A and in B (valid input per the
    header: they are summed).  B's rows are then not strictly ascending, so
    the unsorted-B paths run.  Integer values: compared exactly."""
    a = with_duplicates(gen.int_valued(gen.rmat(11, 8, seed=71), 72), 73)
    b = with_duplicates(gen.int_valued(gen.rmat(11, 8, seed=74), 75), 76)
    opt = None if group is None else forced_options(group, 256 if group == 7 else None)
    c = run_and_compare(a, b, options=opt, exact=True, b_sorted=False, label=f"dup{group}")
    structure_invariants(c)


def test_cancellation_explicit_zeros():
    a = gen.from_coo(3, 2, [0, 0, 1, 2], [0, 1, 1, 0], np.array([1, 1, 2, 3], np.float32))
    b = gen.from_coo(2, 3, [0, 1, 0, 1], [0, 0, 2, 2], np.array([1, -1, 4, -4], np.float32))
    for g in range(1, 8):
        c = run_and_compare(a, b, options=forced_options(g), exact=True, label=f"cancel{g}")
        assert c.nnz == 6


def test_empty_inputs():
    for (m, k, n) in [(0, 5, 7), (5, 0, 7), (5, 7, 0), (1, 1, 1)]:
        a = gen.random_csr(m, k, 0.5, 1)
        b = gen.random_csr(k, n, 0.5, 2)
        run_and_compare(a, b, label=f"empty{(m, k, n)}")
    z = gen.random_csr(100, 80, 0.0, 1)
    run_and_compare(z, gen.random_csr(80, 90, 0.3, 2), label="zero-A")


def test_identity_exact():
    a = gen.rmat(12, 8, seed=5)
    n = a.ncols
    eye = gen.from_coo(n, n, np.arange(n), np.arange(n), np.ones(n, np.float32))
    c = run_and_compare(a, eye, exact=True, label="identity")
    assert np.array_equal(c.val.cpu().numpy(), a.val)


def test_ip_and_maps_bit_exact():
    import torch
    a = gen.rmat(13, 16, seed=21)
    da, db = spgemm.to_device(a), spgemm.to_device(a)
    opt = spgemm.default_options()
    plan = spgemm.Plan(da, db, opt)
    try:
        ip, _ = plan.export(0)
        assert np.array_equal(ip.cpu().numpy(), oracle.ip(a, a))
        m, gs = plan.export(1)
        # symbolic key: intermediate products capped at B's column count
        key = np.minimum(oracle.ip(a, a), a.ncols)
        # rows of one A nonzero (B's rows strictly ascending) go no further
        # than the first block group
        single = np.diff(a.rpt) == 1
        assert np.any(single & (key > opt.sym_upper[5]))
        _, order, offs = oracle.bins_reference(key, list(opt.sym_upper), single)
        mm = m.cpu().numpy()
        assert np.all((mm >> 32) == 0)
        assert np.array_equal(mm & 0xffffffff, order)
        assert gs == offs.tolist()
        plan.symbolic()
        m2, gs2 = plan.export(2)
        counts = oracle.row_counts(a, a)
        # numeric key: output length, raised to ceil(IP / 16) capped at B's columns
        key2 = np.maximum(counts, np.minimum((oracle.ip(a, a) + 15) // 16, a.ncols))
        _, order2, offs2 = oracle.bins_reference(key2, list(opt.num_upper), single)
        assert np.array_equal(m2.cpu().numpy() & 0xffffffff, order2)
        assert gs2 == offs2.tolist()
        assert np.array_equal(np.diff(plan.rpts[0].cpu().numpy()), counts)
        info = plan.info()
        assert info.ip_total == int(oracle.ip(a, a).sum())
        assert info.nnz_c == int(counts.sum())
    finally:
        plan.free()
    torch.cuda.synchronize()


def test_symbolic_key_capped_at_columns():
    # B with few columns: rows with many intermediate products but at most
    # ncols(B) outputs take a small-table group
    a = gen.skewed_csr(3000, 2000, seed=51, max_len=40, heavy_rows=5, heavy_len=1500)
    b = gen.random_csr(2000, 100, 0.3, 52)
    da, db = spgemm.to_device(a), spgemm.to_device(b)
    opt = spgemm.default_options()
    plan = spgemm.Plan(da, db, opt)
    try:
        m, gs = plan.export(1)
        key = np.minimum(oracle.ip(a, b), b.ncols)
        _, order, offs = oracle.bins_reference(key, list(opt.sym_upper), np.diff(a.rpt) == 1)
        assert np.array_equal(m.cpu().numpy() & 0xffffffff, order)
        assert gs == offs.tolist()
        assert gs[7] == gs[8]      # no chunked rows although IP reaches ~10^4
    finally:
        plan.free()
    run_and_compare(a, b, label="capped-key")


@pytest.mark.parametrize("group", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("ncols", [48, 200, 1000])
def test_direct_mapped_tables(group, ncols):
    # B with few columns: tables indexed by the column itself where they fit
    a = gen.int_valued(gen.skewed_csr(1200, 900, seed=60 + group, max_len=30, heavy_rows=2,
                                      heavy_len=600), 3)
    b = gen.int_valued(gen.random_csr(900, ncols, min(0.5, 40.0 / ncols), 61 + group), 4)
    run_and_compare(a, b, options=forced_options(group), exact=True,
                    label=f"direct g{group} n{ncols}")


def test_value_only_rerun():
    import torch
    a = gen.rmat(11, 16, seed=33)
    da, db = spgemm.to_device(a), spgemm.to_device(a)
    plan = spgemm.Plan(da, db)
    try:
        plan.symbolic()
        cols, vals = plan.allocate_outputs()
        plan.numeric(cols, vals)
        a2 = gen.int_valued(a, 5)
        v2 = torch.from_numpy(a2.val).cuda()
        plan.numeric(cols, vals, a_vals=[v2], b_vals=[v2])
        plan.sync()
        ref = oracle.product(a2, a2)
        k = plan.nnz[0]
        msg = oracle.compare(ref, plan.rpts[0].cpu().numpy(), cols[0][:k].cpu().numpy(),
                             vals[0][:k].cpu().numpy(), exact_values=True)
        assert msg is None, msg
    finally:
        plan.free()


def test_validation_rejects_malformed():
    import torch
    a = gen.rmat(8, 8, seed=1)
    da = spgemm.to_device(a)
    bad = spgemm.DeviceCsr(da.nrows, da.ncols, da.rpt.clone(), da.col.clone(), da.val, True)
    bad.col[3] = da.ncols + 5          # column out of range
    opt = spgemm.make_options(validate=2)
    with pytest.raises(spgemm.SpgemmError) as e:
        spgemm.Plan(da, bad, opt)
    assert e.value.code == 3
    # the cheap level checks row pointers only: the column is not looked at
    spgemm.Plan(da, bad, spgemm.make_options(validate=1)).free()
    bad2 = spgemm.DeviceCsr(da.nrows, da.ncols, da.rpt.clone(), da.col, da.val, True)
    bad2.rpt[5] = bad2.rpt[6] + 1      # non-monotone row pointers
    for level in (1, 2):
        with pytest.raises(spgemm.SpgemmError) as e:
            spgemm.Plan(bad2, da, spgemm.make_options(validate=level))
        assert e.value.code == 3
    torch.cuda.synchronize()


def test_dimension_mismatch():
    a = spgemm.to_device(gen.random_csr(10, 12, 0.3, 1))
    b = spgemm.to_device(gen.random_csr(13, 9, 0.3, 2))
    with pytest.raises(spgemm.SpgemmError) as e:
        spgemm.Plan(a, b)
    assert e.value.code == 2


@pytest.mark.parametrize("exact", [False, True])
def test_row_thread_group1(exact):
    """Group 1 handled one thread per row with the gathered range stream
    (options.row_thread), on rows of every length the group takes, empty
    rows included; integer values compared exactly."""
    a = gen.skewed_csr(5001, 3000, seed=81, max_len=6, heavy_rows=0)
    b = gen.skewed_csr(3000, 4000, seed=82, max_len=5, heavy_rows=0)
    if exact:
        a, b = gen.int_valued(a, 83), gen.int_valued(b, 84)
    opt = forced_options(1)
    opt.row_thread = 1
    c = run_and_compare(a, b, options=opt, exact=exact, label=f"rowthread-{exact}")
    structure_invariants(c)
    # default grouping with the option on: group 1 rows only take the new path
    o2 = spgemm.make_options(row_thread=1)
    run_and_compare(gen.er(2000, 16000, seed=85), gen.er(2000, 16000, seed=85), options=o2,
                    label="rowthread-er2k")
    # unsorted B and columns of B fewer than the table (ncols <= 32)
    bs = gen.shuffle_rows(b, 86)
    run_and_compare(a, bs, options=opt, exact=exact, b_sorted=False, label="rowthread-unsorted")
    narrow = gen.random_csr(3000, 20, 0.3, 87)
    run_and_compare(a, narrow, options=opt, label="rowthread-narrow")


def test_row_thread_batch_and_graph():
    import torch
    As = [gen.int_valued(gen.skewed_csr(700 + 37 * q, 900, seed=90 + q, max_len=5,
                                        heavy_rows=0), q) for q in range(5)]
    Bs = [gen.int_valued(gen.skewed_csr(900, 1000 + q, seed=95 + q, max_len=4,
                                        heavy_rows=0), q + 7) for q in range(5)]
    opt = forced_options(1)
    opt.row_thread = 1
    for graph in (0, 1):
        opt.graph = graph
        plan = spgemm.Plan([spgemm.to_device(a) for a in As], [spgemm.to_device(b) for b in Bs],
                           opt)
        try:
            plan.symbolic()
            cols, vals = plan.allocate_outputs()
            for rep in range(3):
                plan.numeric(cols, vals)
                plan.sync()
                torch.cuda.synchronize()
                for q in range(5):
                    ref = oracle.product(As[q], Bs[q])
                    k = plan.nnz[q]
                    assert oracle.compare(ref, plan.rpts[q].cpu().numpy(),
                                          cols[q][:k].cpu().numpy(), vals[q][:k].cpu().numpy(),
                                          exact_values=True) is None, (graph, rep, q)
        finally:
            plan.free()


@pytest.mark.parametrize("group,nk", [(1, 5), (1, 40), (2, 9), (2, 100), (3, 70), (4, 20),
                                      (4, 64), (4, 100), (4, 300)])
def test_direct_mapped_shared_columns(group, nk):
    # every B row holds the same columns (the layout of the served GNN
    # features): one lane's products of a round name the same column when
    # they come from different B rows
    ncols = 8 * (8, 16, 32, 64)[group - 1]   # the group's table size
    rng = np.random.default_rng(70 + group)
    n = 700
    kept = np.sort(rng.choice(ncols, min(nk, ncols), replace=False)).astype(np.int32)
    k = kept.size
    b = gen.Csr(n, ncols, np.arange(n + 1, dtype=np.int64) * k, np.tile(kept, n),
                rng.integers(1, 4, n * k).astype(np.float32))
    a = gen.int_valued(gen.skewed_csr(1100, n, seed=80 + group, max_len=40, heavy_rows=0), 5)
    run_and_compare(a, b, options=forced_options(group), exact=True,
                    label=f"shared g{group} nk{k}")
    af = a.with_values(rng.uniform(-1, 1, a.nnz).astype(np.float32))
    run_and_compare(af, b, options=forced_options(group), label=f"shared f32 g{group} nk{k}")


@pytest.mark.parametrize("group,ncols", [(1, 64), (2, 100), (3, 256), (4, 300), (4, 512),
                                         (None, 512), (None, 513)])
def test_row_bitmap_counts(group, ncols):
    """B of at most 512 columns is also kept as row bitmaps, from which the
    symbolic phase of direct-mapped rows counts the row's columns (the OR of
    the bitmaps of the B rows named).  B with duplicate entries, rows stored
    out of order and empty rows; 513 columns: no bitmaps (the ordinary
    walk).  Integer values: compared exactly."""
    rng = np.random.default_rng(ncols)
    b = gen.random_csr(800, ncols, min(0.5, 30.0 / ncols), 90 + ncols)
    b = gen.shuffle_rows(with_duplicates(gen.int_valued(b, 91), 92), 93)
    cnt = np.diff(b.rpt)
    empty = rng.random(b.nrows) < 0.1                # some B rows emptied
    keep = ~np.repeat(empty, cnt)
    rpt = np.zeros(b.nrows + 1, dtype=np.int64)
    np.cumsum(np.where(empty, 0, cnt), out=rpt[1:])
    b = gen.Csr(b.nrows, ncols, rpt, b.col[keep], b.val[keep])
    a = gen.int_valued(gen.skewed_csr(1500, b.nrows, seed=94, max_len=40, heavy_rows=0), 95)
    opt = None if group is None else forced_options(group)
    run_and_compare(a, b, options=opt, exact=True, b_sorted=False,
                    label=f"bitmap g{group} n{ncols}")


@pytest.mark.parametrize("group", [1, 2, 3, 4, None])
def test_direct_mapped_nan_values(group):
    """The group kernels' direct-mapped tables mark an untouched value slot
    with the all-ones bit pattern (a NaN) instead of a key.  B values that
    are NaN, and B values with exactly that bit pattern, must still leave
    their outputs in the structure (the structure never depends on values):
    row pointers and columns equal the oracle's, NaN outputs sit where the
    oracle's are, and every other (integer-valued) output is exact."""
    import torch
    ncols = 8 * (8, 16, 32, 64)[(group or 4) - 1]   # fits the table: direct-mapped
    rng = np.random.default_rng(100 + (group or 0))
    a = gen.int_valued(gen.skewed_csr(1300, 700, seed=110 + (group or 0), max_len=25,
                                      heavy_rows=0), 6)
    b = gen.int_valued(gen.random_csr(700, ncols, min(0.5, 24.0 / ncols), 120 + (group or 0)),
                       7)
    bv = b.val.copy()
    pick = rng.random(bv.size)
    bv[pick < 0.02] = np.float32("nan")
    bits = bv.view(np.uint32)
    bits[(pick >= 0.02) & (pick < 0.04)] = np.uint32(0xFFFFFFFF)
    b = b.with_values(bv)
    opts = forced_options(group) if group else None
    log(f"[gpu] direct nan g{group}: B {b.nrows}x{b.ncols} nnz {b.nnz}, "
        f"{int((pick < 0.04).sum())} NaN values")
    c = spgemm.matmul(spgemm.to_device(a), spgemm.to_device(b), opts)
    torch.cuda.synchronize()
    ref = oracle.product(a, b)
    rpt, col, val = c.rpt.cpu().numpy(), c.col.cpu().numpy(), c.val.cpu().numpy()
    assert np.array_equal(rpt, ref.rpt), "row pointers"
    assert np.array_equal(col, ref.col), "columns"
    gnan, rnan = np.isnan(val), np.isnan(ref.val)
    assert rnan.any(), "the case holds NaN outputs"
    assert np.array_equal(gnan, rnan), "NaN outputs"
    assert np.array_equal(val[~gnan].astype(np.float64), ref.val[~rnan]), "values"
