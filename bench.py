"""Benchmark of the hash-based multi-phase SpGEMM on one MI355X.

A step is one pass of the whole path on one product: plan (intermediate
products per row + row grouping), symbolic phase (+ row-pointer scan),
allocation of C, numeric phase (+ gather and sort), kernel flag check, plan
release.  The headline workload is C = A*A with A an R-MAT graph of scale 18,
edge factor 16, (a, b, c, d) = (0.57, 0.19, 0.19, 0.05), duplicates merged,
FP32 values in (0, 1]; the inputs are resident in HBM before timing starts.
The other workloads are reported under "configs" (Erdos-Renyi 2k
self-product, graph contraction, Markov clustering) and "served" (4,096
GNN aggregation requests under continuous batching against plain
per-request plans).

Prints one JSON line.  Throughput is 2 * sum(intermediate products) / time
(paper Section VI).  The roofline entry is for the dominant kernel, timed with
HIP events on the library's stream inside the timed region.  Its algorithmic
bytes apply a per-unit model to the rows that kernel handles: numeric 8 B per
intermediate product (B column + value), 8 B per output entry, 24 B per A
nonzero (column, value, B row-pointer pair), 24 B per row; symbolic 4 B per
intermediate product, 20 B per A nonzero, 28 B per row.  The CPU baseline is
the CPU oracle timed on a bounded row sample on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SpGEMM GFLOP/s + HBM GB/s; batched-serve vs plain speedup, p50/p99 latency"
HBM_PEAK_GBS = 8000.0

# algorithmic bytes per unit: intermediate product, output entry, A nonzero, row
NUM_BYTES = dict(ip=8, nnz=8, alen=24, row=24)
SYM_BYTES = dict(ip=4, nnz=0, alen=20, row=28)
PLAN_BYTES = dict(ip=0, nnz=0, alen=20, row=24)


# HBM traffic of the dominant kernel, from rocprofv3 FETCH_SIZE / WRITE_SIZE
# passes over this benchmark, scaled by what the same counters read for a plain
# device copy of known size.  Only used while the kernel sources are unchanged.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "num_chunk_rmat18_traffic.json")
KERNEL_SOURCES = ["paper_2512_12036_amd/csrc/k_chunk.hip", "paper_2512_12036_amd/csrc/dev.hpp",
                  "paper_2512_12036_amd/csrc/common.hpp"]


def kernel_source_digest():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(group, chunk_cols):
    """Bytes per launch of `group` from the committed counter summary, or None
    when there is none for this kernel, these options and these sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("group") != group or t.get("chunk_cols") != chunk_cols:
        return None
    if t.get("source_sha256") != kernel_source_digest():
        return None
    return int(t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def rmat18():
    from paper_2512_12036_amd import gen
    return gen.rmat(18, 16, seed=2)


def group_units(plan, rpt_a):
    """Per-group (rows, sum ip, sum nnz, sum alen) of the symbolic (1) and
    numeric (2) row maps of a single-product plan after its symbolic phase,
    and the totals.  rpt_a: A's row pointers (device tensor)."""
    ip, _ = plan.export(0)
    alen = (rpt_a[1:] - rpt_a[:-1])
    nnz = plan.rpts[0][1:] - plan.rpts[0][:-1]
    res = []
    for what in (1, 2):
        m, gs = plan.export(what)
        rows = (m & 0xffffffff).long()
        out = {}
        for g in range(8):
            sel = rows[gs[g]:gs[g + 1]]
            out[g] = dict(rows=int(sel.numel()), ip=int(ip[sel].sum()), nnz=int(nnz[sel].sum()),
                          alen=int(alen[sel].sum()))
        res.append(out)
    tot = dict(rows=int(alen.numel()), ip=int(ip.sum()), nnz=int(nnz.sum()),
               alen=int(alen.sum()))
    return res[0], res[1], tot


def model_bytes(model, u):
    return (model["ip"] * u["ip"] + model["nnz"] * u["nnz"] + model["alen"] * u["alen"]
            + model["row"] * u["rows"])


def launch_groups(timings, steps):
    """Average duration per step of every launch group (HIP events on the
    plan's stream), and the same with the dense and rank launches of the
    numeric chunk group (num.g7, num.g7r: disjoint chunks) taken as one."""
    agg = {}
    for tl in timings:
        for name, t in tl:
            agg.setdefault(name, []).append(t)
    avg = {k: float(np.sum(v)) / steps for k, v in agg.items()}
    per_launch = {}
    for k, v in avg.items():
        key = "num.g7" if k.startswith("num.g7") else k
        per_launch[key] = per_launch.get(key, 0.0) + v
    return avg, per_launch


def alg_bytes_of(name, units):
    """Algorithmic bytes of launch group `name` ("sym.g5", "num.g7",
    "plan.ipcount", ...) from the per-group units of its plan."""
    sym_u, num_u, tot = units
    phase, grp = name.split(".")
    if phase == "num" and grp.startswith("g"):
        return model_bytes(NUM_BYTES, num_u[int(grp[1])])
    if phase == "sym" and grp.startswith("g"):
        return model_bytes(SYM_BYTES, sym_u[int(grp[1])])
    return model_bytes(PLAN_BYTES, tot)


def roofline_entry(name, ms, nbytes, traffic=None, kernel=None):
    achieved = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": kernel or name, "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "alg_bytes_per_launch": int(nbytes),
            "avg_launch_ms": round(ms, 4)}


def plan_units(da, db):
    """Group units of C = A * B under the default options."""
    from paper_2512_12036_amd import spgemm
    plan = spgemm.Plan(da, db, spgemm.make_options())
    plan.symbolic()
    u = group_units(plan, da.rpt)
    plan.free()
    return u


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def time_oracle(fn, reps: int = 3) -> list[float]:
    """Wall seconds of `reps` runs of fn() (the oracle on a fixed sample)."""
    out = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        out.append(time.perf_counter() - t0)
    return out


def cpu_baseline_of(a, b, rows, flops: float, sample: str, rows_1core=None,
                    flops_1core: float = 0.0):
    """The oracle timed on this host: the median of 3 runs on all threads over
    `rows` of A*B (flops = 2 x their intermediate products), and one run on a
    single thread over rows_1core."""
    import oracle
    nthreads = oracle.max_threads()
    t_all = time_oracle(lambda: oracle.product(a, b, rows))
    med = float(np.median(t_all))
    out = {"value": round(flops / med / 1e9, 3), "unit": "GFLOP/s", "cores": nthreads,
           "kind": "oracle", "sample": f"{sample}; median of {len(t_all)} runs "
                                       f"({', '.join(f'{t:.2f}' for t in t_all)} s)",
           "cpu_model": cpu_model()}
    if rows_1core is not None:
        oracle.set_threads(1)
        try:
            t1 = time_oracle(lambda: oracle.product(a, b, rows_1core), reps=1)[0]
        finally:
            oracle.set_threads(nthreads)
        out["one_core"] = {"value": round(flops_1core / t1 / 1e9, 3), "unit": "GFLOP/s",
                           "seconds": round(t1, 2)}
    return out


def cpu_baseline(a):
    """The CPU oracle on the R-MAT 18 self-product over row slices (rows i
    with i mod 8 = k): three slices (3/8 of the product, about 3 s on 16
    threads) for the median of 3, one slice on one thread."""
    import oracle
    ip = oracle.ip(a, a)
    rows = np.concatenate([np.arange(k, a.nrows, 8, dtype=np.int64) for k in range(3)])
    rows1 = np.arange(3, a.nrows, 64, dtype=np.int64)
    return cpu_baseline_of(a, a, rows, 2.0 * float(ip[rows].sum()),
                           f"rows i with i mod 8 in {{0, 1, 2}} ({int(ip[rows].sum())} "
                           f"intermediate products = 3/8 of the product), FP64 Gustavson",
                           rows1, 2.0 * float(ip[rows1].sum()))


def measure_product(da, db, steps: int, warmup: int, label: str, opt=None):
    """Times `steps` whole passes (plan, symbolic, allocation of C, numeric,
    flag check, release) of C = A * B after `warmup` untimed ones, with the
    launch groups timed by HIP events on the plan's stream."""
    import torch
    from paper_2512_12036_amd import spgemm
    opt = opt if opt is not None else spgemm.make_options(profile=1)
    stream = torch.cuda.current_stream(da.rpt.device)

    def step():
        plan = spgemm.Plan(da, db, opt, stream)
        plan.symbolic()
        cols, vals = plan.allocate_outputs()
        plan.numeric(cols, vals)
        return plan, cols, vals

    for w in range(warmup):
        plan, cols, vals = step()
        torch.cuda.synchronize()
        plan.sync()
        plan.free()
        del cols, vals
    log(f"[bench] {label}: {warmup} warmup steps done")
    info = None
    timings = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        plan, cols, vals = step()
        torch.cuda.synchronize()
        plan.sync()                     # kernel error flags of this step
        timings.append(plan.timings())
        if k == 0:
            info = plan.info()
        plan.free()
        del cols, vals
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"[bench] {label}: {steps} timed steps done")
    ms = (t1 - t0) * 1e3 / steps
    avg, per_launch = launch_groups(timings, steps)
    return dict(ms=ms, info=info, avg=avg, per_launch=per_launch, opt=opt)


def dominant_roofline(per_launch, avg, units, chunk_cols=None):
    dom = max(per_launch, key=lambda k: per_launch[k])
    traffic = measured_traffic(dom, chunk_cols) if chunk_cols is not None else None
    kernel = dom + (" (k_num_chunk_pipe + k_num_chunk_rank)"
                    if dom == "num.g7" and "num.g7r" in avg else "")
    return roofline_entry(dom, per_launch[dom], alg_bytes_of(dom, units), traffic, kernel)


# Counter calibration (--calib-copy-mib): kernels of known HBM traffic, run
# before the steps so that a counter pass sees them beside the kernels it
# measures.  Their buffers are far larger than the 256 MB last-level cache.
#  * a plain copy of CALIB MiB: CALIB MiB read, CALIB MiB written;
#  * a 4 GiB float32 buffer read at a 64-byte stride (one float of every
#    64-byte segment, a float32 strided copy): every segment, so every byte
#    of the buffer, is fetched; 256 MiB written;
#  * the same buffer as int32 at a 128-byte stride (an int32 strided copy):
#    one word per 128-byte line, so 2 GiB fetched if lines are fetched in
#    64-byte halves and 4 GiB if whole; 128 MiB written.
CALIB_GATHER_BYTES = 4 << 30


def calibration_kernels(copy_mib, dev):
    import torch
    n = copy_mib * (1 << 20) // 4
    src = torch.rand(n, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    g = torch.rand(CALIB_GATHER_BYTES // 4, device=dev)
    torch.cuda.synchronize()
    s64 = g.view(-1, 16)[:, 0].contiguous()
    torch.cuda.synchronize()
    s128 = g.view(torch.int32).view(-1, 32)[:, 0].contiguous()
    torch.cuda.synchronize()
    del g, s64, s128
    torch.cuda.empty_cache()
    log(f"[bench] calibration copy of {copy_mib} MiB and strided reads of 4 GiB done")


def run_rmat18(args):
    import torch
    from paper_2512_12036_amd import spgemm
    torch.cuda.init()
    dev = torch.device("cuda:0")
    log("[bench] generating R-MAT scale 18 ...")
    a = rmat18()
    da = spgemm.to_device(a, dev)
    torch.cuda.synchronize()
    if args.calib_copy_mib:
        calibration_kernels(args.calib_copy_mib, dev)
    r = measure_product(da, da, args.steps, args.warmup, "R-MAT 18")
    info, avg, per_launch = r["info"], r["avg"], r["per_launch"]
    ms = r["ms"]
    flops = info.flops
    gflops = flops / (ms * 1e-3) / 1e9
    units = plan_units(da, da)
    roof = dominant_roofline(per_launch, avg, units, r["opt"].chunk_cols)
    num_u = units[1]
    num_total_bytes = sum(model_bytes(NUM_BYTES, v) for g, v in num_u.items() if g > 0)
    num_ms = sum(t for k, t in avg.items() if k.startswith("num."))
    out = {
        "metric": METRIC, "value": round(gflops, 2), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "C = A*A, A R-MAT scale 18 (262,144 vertices), edge factor 16, "
                               "(a,b,c,d) = (.57,.19,.19,.05), duplicates merged, FP32 in (0,1]",
                   "nnz_a": a.nnz, "intermediate_products": info.ip_total,
                   "nnz_c": info.nnz_c, "flops": flops},
        "roofline": roof,
        "numeric_phase": {"ms": round(num_ms, 3), "alg_bytes": int(num_total_bytes),
                          "alg_GBps": round(num_total_bytes / (num_ms * 1e-3) / 1e9, 1)
                          if num_ms > 0 else None},
        "phases_ms": {k: round(v, 4) for k, v in sorted(avg.items())},
    }
    if not args.no_cpu:
        log("[bench] timing the CPU oracle on a row sample ...")
        out["cpu_baseline"] = cpu_baseline(a)
    del da
    torch.cuda.empty_cache()
    return out


def run_unsorted(args):
    """The R-MAT 18 self-product with every row of B stored in a random
    order (A unchanged): the plan sorts B's rows on the device first (a
    segmented radix sort) and gathers B's values into that order at the
    numeric call, so the column-chunked rows keep the tabulated chunk bounds.
    Compared with the sorted input's step."""
    import torch
    from paper_2512_12036_amd import gen, spgemm
    a = rmat18()
    b = gen.shuffle_rows(a, seed=5)
    da = spgemm.to_device(a)
    db = spgemm.to_device(b, sorted_rows=False)
    r = measure_product(da, db, args.steps, args.warmup, "R-MAT 18, B unsorted")
    out = {"workload": "C = A*B, A R-MAT scale 18, B = A with every row stored in a random order",
           "ms_per_step": round(r["ms"], 3),
           "gflops": round(r["info"].flops / (r["ms"] * 1e-3) / 1e9, 2),
           "phases_ms": {k: round(v, 4) for k, v in sorted(r["avg"].items())}}
    del da, db
    torch.cuda.empty_cache()
    return out


def run_er2k(args):
    """Erdos-Renyi 2,000 x 2,000 with 16,000 nonzeros, C = A*A: the latency
    floor of one whole pass."""
    import torch
    from paper_2512_12036_amd import gen, spgemm
    a = gen.er(2000, 16000, seed=1)
    da = spgemm.to_device(a)
    steps = max(20, 4 * args.steps)
    r = measure_product(da, da, steps, max(5, args.warmup), "ER 2k")
    units = plan_units(da, da)
    out = {"workload": "C = A*A, A 2,000 x 2,000 Erdos-Renyi G(n, M), M = 16,000, FP32 U[-1, 1]",
           "steps": steps, "ms_per_step": round(r["ms"], 4),
           "gflops": round(r["info"].flops / (r["ms"] * 1e-3) / 1e9, 3),
           "intermediate_products": r["info"].ip_total, "nnz_c": r["info"].nnz_c,
           "roofline": dominant_roofline(r["per_launch"], r["avg"], units),
           "phases_ms": {k: round(v, 4) for k, v in sorted(r["avg"].items())}}
    # the same product through the one-call allocation-free entry point (plan,
    # symbolic and numeric in one C call, C into arrays sized by the IP bound)
    cap = int(r["info"].ip_total)
    c_rpt = torch.empty(a.nrows + 1, dtype=torch.int64, device="cuda")
    c_col = torch.empty(cap, dtype=torch.int32, device="cuda")
    c_val = torch.empty(cap, dtype=torch.float32, device="cuda")
    per = []
    for k in range(steps + 5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        code, _ = spgemm.multiply_noalloc(da, da, c_rpt, c_col, c_val)
        per.append((time.perf_counter() - t0) * 1e3)
        assert code == 0, code
    out["one_call_ms"] = round(float(np.median(per[5:])), 4)
    if not args.no_cpu:
        rows = np.arange(a.nrows, dtype=np.int64)
        out["cpu_baseline"] = cpu_baseline_of(a, a, rows, float(r["info"].flops),
                                              "the whole product", rows, float(r["info"].flops))
    return out


def run_tiny(args):
    """Rows of a few products each (the smallest group): C = A*A with A an
    Erdos-Renyi 2^20 x 2^20 matrix of 4 nonzeros per row (about 16 products
    per row), with the lane-group kernels and with the thread-per-row
    range-stream kernels (options.row_thread)."""
    from paper_2512_12036_amd import gen, spgemm
    log("[bench] generating the tiny-row workload ...")
    a = gen.er(1 << 20, 4 << 20, seed=61, lo=0.0, hi=1.0)
    da = spgemm.to_device(a)
    out = {"workload": "C = A*A, A Erdos-Renyi 2^20 x 2^20 with 4 nonzeros per row, FP32 (0,1]"}
    for rt in (0, 1):
        r = measure_product(da, da, max(10, args.steps), max(3, args.warmup), f"tiny rt={rt}",
                            spgemm.make_options(profile=1, row_thread=rt))
        out["row_thread" if rt else "lane_groups"] = {
            "ms_per_step": round(r["ms"], 3),
            "gflops": round(r["info"].flops / (r["ms"] * 1e-3) / 1e9, 2),
            "phases_ms": {k: round(v, 4) for k, v in sorted(r["avg"].items())}}
    return out


def _cuda_timed(fn, steps, warmup):
    """Median ms of fn() between HIP events on the current stream."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def run_gnn(args):
    """One GNN layer with a pruning layer (paper Section V-C, Eq. 1-3),
    forward and backward, at the largest served graph size: A_hat of the
    served generator with n = 200,000 nodes (mean degree about 28 with the
    self loop), X dense n x 512 with ReLU-like rows (half zero), TopK k = 64
    per row, W 512 x 256.  Forward: TopK, the SpGEMM A_hat TopK(X), dense H,
    H W on the matrix cores; backward: G W^T, the masked SpMM on TopK's
    pattern, H^T G.  Each step is timed on its own (median of the steps)."""
    import torch
    from paper_2512_12036_amd import gen, gnn, spgemm
    n, f, fo, k = 200_000, 512, 256, 64
    log("[bench] generating the GNN layer problem ...")
    g_ = gen.gnn_graph_t(4242, "cuda", n=n, d=27.0)
    a = spgemm.DeviceCsr(g_.nrows, g_.ncols, g_.rpt, g_.col, g_.val, True)
    gen_t = torch.Generator(device="cuda").manual_seed(4242)
    x = torch.relu(torch.randn(n, f, device="cuda", generator=gen_t))
    w = torch.randn(f, fo, device="cuda", generator=gen_t) / f ** 0.5
    g = torch.randn(n, fo, device="cuda", generator=gen_t)
    torch.cuda.synchronize()
    steps, warm = max(10, args.steps), max(3, args.warmup)
    st = {}
    xk = spgemm.topk_rows(x, k)
    st["topk"] = _cuda_timed(lambda: spgemm.topk_rows(x, k), steps, warm)
    h = spgemm.matmul(a, xk)
    st["spgemm"] = _cuda_timed(lambda: spgemm.matmul(a, xk), steps, warm)
    hd = spgemm.to_dense(h)
    st["to_dense"] = _cuda_timed(lambda: spgemm.to_dense(h), steps, warm)
    st["gemm_hw"] = _cuda_timed(lambda: spgemm.gemm(hd, w), steps, warm)
    d = spgemm.gemm(g, w.t())
    st["gemm_gwt"] = _cuda_timed(lambda: spgemm.gemm(g, w.t()), steps, warm)
    st["masked_spmm"] = _cuda_timed(lambda: spgemm.masked_spmm(a, d, xk), steps, warm)
    st["gemm_htg"] = _cuda_timed(lambda: spgemm.gemm(hd.t(), g), steps, warm)
    fwd = _cuda_timed(lambda: gnn.layer_forward(a, x, w, k), steps, warm)
    _, cache = gnn.layer_forward(a, x, w, k)
    bwd = _cuda_timed(lambda: gnn.layer_backward(a, g, w, cache), steps, warm)
    deg = (a.rpt[1:] - a.rpt[:-1]).to(torch.int64)
    # every A nonzero (i, j) meets TopK row j, which holds k entries
    ip = int(deg.sum()) * k
    gemm_flops = 2.0 * n * f * fo
    mask_flops = 2.0 * int(deg.sum()) * k  # one multiply-add per (mask entry, A^T entry)
    best_gemm = min(st["gemm_hw"], st["gemm_gwt"], st["gemm_htg"])
    out = {
        "workload": f"GNN layer, A_hat of the served generator n = {n}, nnz = {int(deg.sum())}; "
                    f"X {n} x {f} ReLU(N(0,1)); TopK k = {k}; W {f} x {fo}; FP32",
        "forward_ms": round(fwd, 3), "backward_ms": round(bwd, 3),
        "steps_ms": {k_: round(v, 4) for k_, v in st.items()},
        "spgemm_gflops": round(2.0 * ip / (st["spgemm"] * 1e-3) / 1e9, 2),
        "masked_spmm_gflops": round(mask_flops / (st["masked_spmm"] * 1e-3) / 1e9, 2),
        "gemm_tflops": {k_: round(gemm_flops / (st[k_] * 1e-3) / 1e12, 2)
                        for k_ in ("gemm_hw", "gemm_gwt", "gemm_htg")},
        "roofline": {"bound": "mfma", "kernel": "spgemm_gemm_f32 (v_mfma_f32_16x16x4_f32)",
                     "achieved": round(gemm_flops / (best_gemm * 1e-3) / 1e12, 2),
                     "peak": 157.3, "unit": "TFLOP/s",
                     "frac": round(gemm_flops / (best_gemm * 1e-3) / 1e12 / 157.3, 4),
                     "traffic": None},
    }
    del a, x, w, g, xk, h, hd, d, cache
    torch.cuda.empty_cache()
    return out


def run_sampling(args):
    """Matrix-based bulk sampling (paper Section V-C, GraphSAGE form): 8
    stacked minibatches of 1,024 vertices of a graph of 2^20 vertices (the
    served generator's normalised adjacency, mean degree about 16), fanouts
    25 then 10, every layer's P = Q A, NORM, SAMPLE and EXTRACT on the
    device; uniforms drawn beforehand.  Reports draws and extracted entries
    per second."""
    import torch
    from paper_2512_12036_amd import gen, sampling, spgemm
    log("[bench] generating the sampling graph ...")
    g_ = gen.gnn_graph_t(90, "cuda", n=1 << 20, d=15.0)
    da = spgemm.DeviceCsr(g_.nrows, g_.ncols, g_.rpt, g_.col, g_.val, True)
    a = da
    rng = np.random.default_rng(90)
    batch = np.concatenate([rng.choice(a.nrows, 1024, replace=False) for _ in range(8)])
    fanouts = [25, 10]
    sizes = [len(batch)]
    for s_ in fanouts[:-1]:
        sizes.append(sizes[-1] * s_)
    uniforms = [torch.from_numpy(rng.random(m * s_).astype(np.float32)).cuda()
                for m, s_ in zip(sizes, fanouts)]
    bt = torch.from_numpy(batch.astype(np.int32)).cuda()
    torch.cuda.synchronize()
    layers = sampling.graphsage_bulk(da, bt, fanouts, uniforms)
    torch.cuda.synchronize()
    draws = sum(int(l["sampled"].numel()) for l in layers)
    extracted = sum(int(l["a_l"].nnz) for l in layers)
    del layers
    ms = _cuda_timed(lambda: sampling.graphsage_bulk(da, bt, fanouts, uniforms),
                     max(10, args.steps), max(3, args.warmup))
    out = {"workload": "GraphSAGE bulk sampling, 2^20-vertex graph of the served generator (mean "
                       "degree about 16, + self loops), 8 x 1,024 batch vertices, fanouts 25, 10",
           "ms": round(ms, 3), "draws": draws, "extracted_entries": extracted,
           "draws_per_s": round(draws / (ms * 1e-3), 1),
           "extracted_per_s": round(extracted / (ms * 1e-3), 1)}
    del da, a, g_, uniforms, bt
    torch.cuda.empty_cache()
    return out


def run_contraction(args):
    """Graph contraction C = S^T (A S), A R-MAT scale 20 edge factor 8, S the
    n x n/16 selector of uniform labels.  A step: S and S^T built on the
    device from the labels, then the two products, both kept on the GPU."""
    import torch
    from paper_2512_12036_amd import apps, gen, spgemm
    log("[bench] generating R-MAT scale 20 (contraction) ...")
    a = gen.rmat(20, 8, seed=23)
    k = a.nrows // 16
    labels_h = gen.contraction_labels(a.nrows, k, seed=24)
    da = spgemm.to_device(a)
    labels = torch.from_numpy(labels_h).cuda()
    opt = spgemm.make_options(profile=1)

    def product(x, y):
        plan = spgemm.Plan(x, y, opt)
        plan.symbolic()
        cols, vals = plan.allocate_outputs()
        plan.numeric(cols, vals)
        torch.cuda.synchronize()
        plan.sync()
        c = plan.results(cols, vals)[0]
        t = plan.timings()
        plan.free()
        return c, t

    def step():
        s = apps.selector(labels, k)
        st = spgemm.selector_transpose(labels, k)
        p, tp = product(da, s)
        c, tc = product(st, p)
        return p, c, tp, tc, s, st

    for _ in range(max(2, args.warmup)):
        step()
    torch.cuda.synchronize()
    steps = max(5, args.steps)
    tps, tcs = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        p, c, tp, tc, s, st = step()
        tps.append(tp)
        tcs.append(tc)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    log(f"[bench] contraction: {steps} timed steps done")
    up = plan_units(da, s)
    uc = plan_units(st, p)
    avg_p, pl_p = launch_groups(tps, steps)
    avg_c, pl_c = launch_groups(tcs, steps)
    ip_p, ip_c = up[2]["ip"], uc[2]["ip"]
    flops = 2 * (ip_p + ip_c)
    rp = dominant_roofline(pl_p, avg_p, up)
    rc = dominant_roofline(pl_c, avg_c, uc)
    roof = rp if rp["avg_launch_ms"] >= rc["avg_launch_ms"] else rc
    roof["kernel"] = ("A*S " if roof is rp else "S^T*P ") + roof["kernel"]
    out = {"workload": "C = S^T (A S), A R-MAT scale 20 (1,048,576 vertices), edge factor 8, "
                       "FP32 in (0,1]; S n x n/16, one 1.0 per row at a uniform cluster id",
           "steps": steps, "ms_per_step": round(ms, 3),
           "ms_products": {"A*S": round(sum(pl_p.values()), 3),
                           "S^T*P": round(sum(pl_c.values()), 3)},
           "gflops": round(flops / (ms * 1e-3) / 1e9, 2),
           "intermediate_products": [ip_p, ip_c], "nnz": [p.nnz, c.nnz],
           "roofline": roof}
    if not args.no_cpu:
        import oracle
        sh = gen.selector(labels_h, k)
        sth = gen.Csr(k, a.nrows, *oracle.transpose(a.nrows, k, sh.rpt, sh.col, sh.val))
        ph = oracle.product(a, sh)
        ph = gen.Csr(a.nrows, k, ph.rpt, ph.col, ph.val.astype(np.float32))

        def both(sel_a, sel_c):
            oracle.product(a, sh, sel_a)
            oracle.product(sth, ph, sel_c)
        import functools
        rows_a = np.arange(a.nrows, dtype=np.int64)
        rows_c = np.arange(k, dtype=np.int64)
        t_all = time_oracle(functools.partial(both, rows_a, rows_c))
        nthreads = oracle.max_threads()
        oracle.set_threads(1)
        try:
            t1 = time_oracle(functools.partial(both, rows_a, rows_c), reps=1)[0]
        finally:
            oracle.set_threads(nthreads)
        med = float(np.median(t_all))
        out["cpu_baseline"] = {
            "value": round(flops / med / 1e9, 3), "unit": "GFLOP/s", "cores": nthreads,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": "both products, all rows (the oracle's own P feeds S^T P); median of 3 "
                      f"runs ({', '.join(f'{t:.2f}' for t in t_all)} s)",
            "one_core": {"value": round(flops / t1 / 1e9, 3), "unit": "GFLOP/s",
                         "seconds": round(t1, 2)}}
    del da, p, c, s, st
    torch.cuda.empty_cache()
    return out


def run_mcl(args):
    """Markov clustering: 100,000-node planted partition (1,000 communities),
    5 iterations of expansion T*T, inflation x^2, row normalisation, prune at
    1e-4, renormalisation, on the row-stochastic transpose T = M^T.  A step is
    the whole 5-iteration loop; throughput counts the expansions' products."""
    import torch
    from paper_2512_12036_amd import gen, spgemm
    log("[bench] generating the planted-partition graph (MCL) ...")
    t0h = gen.planted_partition(1000, 100, seed=5)
    t0 = spgemm.to_device(t0h)
    opt = spgemm.make_options(profile=1)

    def loop(record):
        t = t0
        it_ms, tl, ips, units, pr_ms = [], [], [], [], []
        for it in range(5):
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            evp = torch.cuda.Event(enable_timing=True)
            ev0.record()
            plan = spgemm.Plan(t, t, opt)
            plan.symbolic()
            cols, vals = plan.allocate_outputs()
            plan.numeric(cols, vals)
            torch.cuda.synchronize()
            plan.sync()
            e = plan.results(cols, vals)[0]
            tl.append(plan.timings())
            ips.append(plan.info().ip_total)
            plan.free()
            del cols, vals
            if record:
                units.append(plan_units(t, t))
            evp.record()
            nt = spgemm.mcl_prune(e, 2.0, 1e-4)
            ev1.record()
            del e
            t = nt
            torch.cuda.synchronize()
            it_ms.append(ev0.elapsed_time(ev1))
            pr_ms.append(evp.elapsed_time(ev1))
        return it_ms, tl, ips, units, t, pr_ms

    loop(False)
    torch.cuda.empty_cache()
    log("[bench] mcl: warmup loop done")
    steps = 2
    all_ms, all_tl, all_pr = [], [], []
    torch.cuda.synchronize()
    tt = time.perf_counter()
    for _ in range(steps):
        it_ms, tl, ips, _, tfin, pr_ms = loop(False)
        all_ms.append(it_ms)
        all_tl.append(tl)
        all_pr.append(pr_ms)
        torch.cuda.empty_cache()
    ms = (time.perf_counter() - tt) * 1e3 / steps
    log(f"[bench] mcl: {steps} timed loops done")
    _, _, _, units, _, _ = loop(True)
    torch.cuda.empty_cache()
    # the whole of Algorithm 6: iterations until the change between iterates
    # reaches 1e-6 (at most 40), then the clusters as connected components
    from paper_2512_12036_amd import apps
    torch.cuda.synchronize()
    tc = time.perf_counter()
    labels, tcl, iters, changes = apps.mcl_cluster(t0, 2.0, 1e-4, 0, 1e-6, 40)
    torch.cuda.synchronize()
    cl_ms = (time.perf_counter() - tc) * 1e3
    n_clusters = int(torch.unique(labels).numel())
    del tcl
    torch.cuda.empty_cache()
    flops = 2 * sum(ips)
    # dominant launch group over the iterations
    best = None
    for it in range(5):
        avg, pl = launch_groups([all_tl[s][it] for s in range(steps)], steps)
        r = dominant_roofline(pl, avg, units[it])
        if best is None or r["avg_launch_ms"] > best["avg_launch_ms"]:
            best = r
            best["kernel"] = f"iteration {it + 1} " + r["kernel"]
    out = {"workload": "MCL on a 100,000-node planted partition (1,000 communities of 100, "
                       "~25 intra + ~5 inter edges per node, + self loops), column-stochastic "
                       "FP32; 5 iterations of expansion, inflation power 2, prune at 1e-4, "
                       "renormalisation",
           "steps": steps, "ms_per_step": round(ms, 2),
           "ms_per_iteration": [round(float(np.mean([m[i] for m in all_ms])), 3)
                                for i in range(5)],
           "prune_ms_per_iteration": [round(float(np.mean([m[i] for m in all_pr])), 3)
                                      for i in range(5)],
           "gflops": round(flops / (ms * 1e-3) / 1e9, 2),
           "intermediate_products": ips, "nnz_final": tfin.nnz, "roofline": best,
           "clustering": {"iterations": iters, "ms": round(cl_ms, 2), "clusters": n_clusters,
                          "last_change": changes[-1] if changes else None,
                          "what": "iterations until the largest entry change <= 1e-6 (at most "
                                  "40), then connected components of the final pattern"}}
    if not args.no_cpu:
        import oracle
        ip1 = oracle.ip(t0h, t0h)
        rows = np.arange(t0h.nrows, dtype=np.int64)
        rows1 = np.arange(0, t0h.nrows, 4, dtype=np.int64)
        out["cpu_baseline"] = cpu_baseline_of(
            t0h, t0h, rows, 2.0 * float(ip1.sum()),
            f"iteration 1's expansion, all rows ({int(ip1.sum())} intermediate products)",
            rows1, 2.0 * float(ip1[rows1].sum()))
    del t0, tfin
    torch.cuda.empty_cache()
    return out


# server configurations: (max requests per batch, max intermediate products
# per batch, streams, device-driven plans)
SERVE_CONFIGS = [(64, 8 << 30, 4, False), (128, 16 << 30, 4, True), (1024, 128 << 30, 4, False)]
SERVE_PASSES = 3


def _median_pass(runs):
    """The stats of the pass with the median makespan (an odd count)."""
    return sorted(runs, key=lambda r: r["makespan_s"])[len(runs) // 2]


def run_served(n_req: int, configs):
    """Served GNN aggregation trace: n_req requests C = A_hat X (seeds 0 ..
    n_req - 1).  The graphs A_hat are generated in device memory first (the
    resident graph store, untimed); each request's features X are built on
    the device when it is admitted and released when it completes, inside the
    HBM budget of 200 GB.  Served with continuous batching and, for
    comparison, one request after another on single-product plans (which
    build X the same way).  For each server configuration (max requests and
    products per batch, streams) the backlogged trace (all requests waiting
    at t = 0; on each side the median of SERVE_PASSES timed passes) gives the
    throughput and the speedup, and a further pass with
    Poisson arrivals at 0.7 x that configuration's capacity the latency
    percentiles."""
    import torch
    from paper_2512_12036_amd import serve
    log(f"[bench] generating {n_req} served requests (graphs on the GPU) ...")
    reqs = serve.gnn_requests(range(n_req), "cuda", features_on_admission=True,
                              log=log if n_req > 512 else None)
    torch.cuda.synchronize()
    ip_total = sum(r.ip for r in reqs)
    budget = 200 * 10 ** 9
    # both sides in steady state: an untimed pass first (see below)
    log("[bench] plain warm-up pass ...")
    serve.run_plain(reqs)
    # each side's figure is the median of SERVE_PASSES timed passes (the
    # GPU's rate drifts by a few percent from pass to pass)
    p_runs = []
    for k in range(SERVE_PASSES):
        log(f"[bench] plain run {k + 1}/{SERVE_PASSES} ...")
        p_runs.append(serve.run_plain(reqs)[0])
    p_stats = _median_pass(p_runs)
    out = {"requests": n_req, "intermediate_products": ip_total,
           "workload": "C = A_hat X, A_hat sym-normalised G(n, n d / 2) + I, n log-uniform "
                       "[1e3, 2e5], d U[5, 50]; X n x F, F U{64..512}, round(rho F) kept "
                       "dense columns, rho U[0.1, 0.5]; FP32; graphs resident, X built on "
                       "admission and released on completion",
           "hbm_budget_gb": budget / 1e9,
           "plain_gflops": round(p_stats["gflops"], 2),
           "plain_makespan_s": round(p_stats["makespan_s"], 4),
           "plain_backlogged_p50_ms": round(p_stats["p50_ms"], 3),
           "plain_pass_gflops": [round(r["gflops"], 2) for r in p_runs],
           "timed_passes": SERVE_PASSES, "servers": []}
    for max_batch, max_batch_ip, n_streams, device_driven in configs:
        srv = serve.Server(budget_bytes=budget, max_batch=max_batch, max_batch_ip=max_batch_ip,
                           n_streams=n_streams, device_driven=device_driven)
        for r in reqs:
            r.arrival = 0.0
        # a server in steady state: one untimed pass over the trace brings
        # PyTorch's caching allocator to the trace's peak, so the timed pass
        # makes no hipMalloc calls (each of those takes milliseconds)
        log(f"[bench] served warm-up pass (batches of <= {max_batch}"
            f"{', device-driven' if device_driven else ''}) ...")
        srv.run(reqs)
        s_runs = []
        for k in range(SERVE_PASSES):
            log(f"[bench] served run {k + 1}/{SERVE_PASSES} (backlogged) ...")
            s_runs.append(srv.run(reqs)[0])
        s_stats = _median_pass(s_runs)
        rate = 0.7 * n_req / s_stats["makespan_s"]
        arr = serve.poisson_arrivals(n_req, rate, seed=11)
        for r, t in zip(reqs, arr):
            r.arrival = float(t)
        log(f"[bench] served run (Poisson arrivals, {rate:.0f}/s) ...")
        l_stats, _ = srv.run(reqs)
        torch.cuda.empty_cache()
        out["servers"].append({
            "max_batch": max_batch, "max_batch_ip": max_batch_ip, "streams": n_streams,
            "device_driven": device_driven,
            "batches": s_stats["batches"], "served_gflops": round(s_stats["gflops"], 2),
            "pass_gflops": [round(r["gflops"], 2) for r in s_runs],
            "speedup_vs_plain": round(p_stats["makespan_s"] / s_stats["makespan_s"], 3),
            "served_makespan_s": round(s_stats["makespan_s"], 4),
            "peak_admitted_gb": round(s_stats["peak_admitted_bytes"] / 1e9, 2),
            "budget_waits": s_stats["budget_waits"], "budget_cuts": s_stats["budget_cuts"],
            "arrival_rate_per_s": round(rate, 1),
            "p50_ms": round(l_stats["p50_ms"], 3), "p99_ms": round(l_stats["p99_ms"], 3),
            "poisson_peak_admitted_gb": round(l_stats["peak_admitted_bytes"] / 1e9, 2)})
    best = max(out["servers"], key=lambda x: x["served_gflops"])
    out.update({k: best[k] for k in ("served_gflops", "speedup_vs_plain", "p50_ms", "p99_ms")})
    del reqs
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# Reduction of the counter passes (rocprofv3 --pmc, csv output) of
#   bench.py --steps 1 --warmup 0 --no-cpu --serve-requests 0 --no-configs
#            --calib-copy-mib 1024
# into profiles/num_chunk_rmat18_hbm_traffic.md and the traffic file.
COUNTER_PASSES = {
    "fetch": ["FETCH_SIZE"],
    "write": ["WRITE_SIZE"],
    "req": ["TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum",
            "TCC_EA0_RDREQ_128B_sum"],
    "tcc": ["TCC_BUBBLE_sum", "TCC_HIT_sum", "TCC_MISS_sum", "TCC_EA0_RDREQ_DRAM_sum"],
    "td": ["TD_TD_BUSY_sum", "TA_TA_BUSY_sum", "GRBM_GUI_ACTIVE"],
}
NUM_G7_PREFIXES = ("spg::k_num_chunk_pipe", "spg::k_num_chunk_rank")


def _read_counter_pass(folder):
    """{dispatch id: {"name", "grid", "ns", counter: value}} of one pass."""
    import csv
    import glob
    out = {}
    files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {folder}")
    for f in files:
        with open(f) as fh:
            for r in csv.DictReader(fh):
                d = out.setdefault(int(r["Dispatch_Id"]), {
                    "name": r["Kernel_Name"], "grid": int(r["Grid_Size"]),
                    "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
                d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return out


def _short_name(name):
    n = name.replace("spg::", "").replace("void ", "").replace("(anonymous namespace)::", "")
    return n.split("(")[0]


def summarize_counters(root, copy_mib):
    passes = {k: _read_counter_pass(os.path.join(root, k)) for k in COUNTER_PASSES}
    # every pass ran the same program: dispatches line up by order
    order = {k: sorted(v) for k, v in passes.items()}
    n = min(len(v) for v in order.values())
    names = [passes["fetch"][order["fetch"][i]]["name"] for i in range(n)]
    for k in passes:
        for i in range(n):
            if passes[k][order[k][i]]["name"] != names[i]:
                raise SystemExit(f"pass {k} dispatch {i} is {passes[k][order[k][i]]['name']}, "
                                 f"not {names[i]}")

    def rec(i):
        r = {"name": names[i], "ns": passes["td"][order["td"][i]]["ns"]}
        for k in passes:
            r.update({c: v for c, v in passes[k][order[k][i]].items()
                      if c not in ("name", "grid", "ns")})
        r["grid"] = passes["fetch"][order["fetch"][i]]["grid"]
        return r

    recs = [rec(i) for i in range(n)]
    # calibration: the largest copyBuffer dispatch, then the first two
    # elementwise copies after it (float 64-byte stride, int 128-byte stride)
    ci = max((i for i in range(n) if "copyBuffer" in recs[i]["name"]),
             key=lambda i: recs[i]["FETCH_SIZE"])
    # PyTorch cuts each strided copy into launches of 32-bit offsets: merge the
    # consecutive launches of one kernel and grid
    strided = []
    for i in range(ci + 1, n):
        if "copy" not in recs[i]["name"] or "rocclr" in recs[i]["name"]:
            continue
        if strided and strided[-1][-1] == i - 1 and recs[i - 1]["grid"] == recs[i]["grid"] \
                and recs[i - 1]["name"] == recs[i]["name"]:
            strided[-1].append(i)
        elif len(strided) < 2:
            strided.append([i])
        else:
            break
    for grp in strided:
        merged = dict(recs[grp[0]])
        for i in grp[1:]:
            for c, v in recs[i].items():
                if isinstance(v, float):
                    merged[c] += v
        merged["launches"] = len(grp)
        recs.append(merged)
    strided = [len(recs) - len(strided) + k for k in range(len(strided))]
    copy_b = copy_mib << 20
    gather_b = [CALIB_GATHER_BYTES, CALIB_GATHER_BYTES]

    def req_bytes(r):
        return (32 * r["TCC_EA0_RDREQ_32B_sum"] + 64 * r["TCC_EA0_RDREQ_64B_sum"]
                + 128 * r["TCC_EA0_RDREQ_128B_sum"])

    fscale = copy_b / (recs[ci]["FETCH_SIZE"] * 1024)
    wscale = copy_b / (recs[ci]["WRITE_SIZE"] * 1024)
    lines = ["# HBM traffic of the dominant kernel, R-MAT scale 18 self-product", "",
             "Five counter passes, each its own run of the same program (one step of the "
             "R-MAT 18 product after the calibration kernels):", ""]
    for k, ctrs in COUNTER_PASSES.items():
        lines.append(f"    cd /tmp && export TMPDIR=/tmp && timeout -s KILL 300 rocprofv3 --pmc "
                     f"{' '.join(ctrs)} -d <out>/{k} -o run --output-format csv -- python3 "
                     f"/root/repo/bench.py --steps 1 --warmup 0 --no-cpu --serve-requests 0 "
                     f"--no-configs --calib-copy-mib {copy_mib}")
    lines += ["", "reduced by", "",
              f"    python3 bench.py --summarize-counters <out> --calib-copy-mib {copy_mib}", "",
              "## Calibration", "",
              "FETCH_SIZE is defined as (128 TCC_BUBBLE + 64 (TCC_EA0_RDREQ - TCC_BUBBLE - "
              "TCC_EA0_RDREQ_32B) + 32 TCC_EA0_RDREQ_32B) / 1024 KiB.  The request-size column "
              "counts the read requests the L2 sends to memory by their size instead: "
              "32 RDREQ_32B + 64 RDREQ_64B + 128 RDREQ_128B bytes.", "",
              "| calibration kernel | known read | known write | FETCH_SIZE | request sizes "
              "(32/64/128 B) | read by request size | TCC_BUBBLE | WRITE_SIZE |",
              "|---|---|---|---|---|---|---|---|"]
    cal = [("plain copy, 1 GiB", ci, copy_b, copy_b)]
    if len(strided) == 2:
        cal += [("4 GiB read at a 64-byte stride (float32)", strided[0], gather_b[0],
                 CALIB_GATHER_BYTES // 16),
                ("4 GiB read at a 128-byte stride (int32)", strided[1], None,
                 CALIB_GATHER_BYTES // 32)]
    for label, i, rd, wr in cal:
        r = recs[i]
        nl = r.get("launches", 1)
        lines.append(
            f"| {label} (`{_short_name(r['name'])[:48]}...`"
            f"{', %d launches' % nl if nl > 1 else ''}) | "
            f"{'%.2f GiB' % (rd / 2**30) if rd else '2 or 4 GiB'} | {wr / 2**20:.0f} MiB | "
            f"{r['FETCH_SIZE'] / 2**20:.3f} GiB | {r['TCC_EA0_RDREQ_32B_sum']:.0f} / "
            f"{r['TCC_EA0_RDREQ_64B_sum']:.0f} / {r['TCC_EA0_RDREQ_128B_sum']:.0f} | "
            f"{req_bytes(r) / 2**30:.3f} GiB | {r['TCC_BUBBLE_sum']:.0f} | "
            f"{r['WRITE_SIZE'] / 2**20:.3f} GiB |")
    lines += ["", f"Copy-based scale factors: fetch {fscale:.4f}, write {wscale:.4f}.", "",
              "Why the fetch factor is 2: on this GPU the L2 sends its reads to memory as "
              "128-byte requests, counted by TCC_EA0_RDREQ_128B, while TCC_BUBBLE, the term "
              "FETCH_SIZE's formula weights by 128 bytes, reads 0; every 128-byte request is "
              "then counted as 64 bytes.  The copy and both strided reads are (nearly) all "
              "128-byte requests, so FETCH_SIZE reads half their traffic.  The int32 read at "
              "a 128-byte stride fetches 4 GiB for 128 MiB of data: the L2 fetches whole "
              "128-byte lines.  The measured kernels' requests are 128-byte too (above 99.9 % "
              "of them), so the copy-scaled FETCH_SIZE and the request-size count agree for "
              "them (below).  WRITE_SIZE needs no scale (64-byte write requests, counted "
              "right).  'DRAM read requests' are those sent towards memory; the 256 MB "
              "last-level cache sits on that path, so part of them is served there.", ""]
    # the numeric chunk group
    g7 = [r for r in recs[:n] if r["name"].replace("void ", "").startswith(NUM_G7_PREFIXES)]
    lines += ["## The numeric chunk group (num.g7)", "",
              "| kernel | ms | FETCH_SIZE x scale | read by request size | WRITE_SIZE x scale | "
              "L2 hit | DRAM read requests / all | TD busy | TA busy |",
              "|---|---|---|---|---|---|---|---|---|"]
    tot = dict(fetch=0.0, req=0.0, write=0.0, ns=0)
    for r in g7:
        f_b = r["FETCH_SIZE"] * 1024 * fscale
        w_b = r["WRITE_SIZE"] * 1024 * wscale
        q_b = req_bytes(r)
        hit = r["TCC_HIT_sum"] / max(1.0, r["TCC_HIT_sum"] + r["TCC_MISS_sum"])
        dram = r["TCC_EA0_RDREQ_DRAM_sum"] / max(1.0, r["TCC_EA0_RDREQ_sum"])
        cyc = r["GRBM_GUI_ACTIVE"] / 8  # summed over the 8 dies: busy clocks of one
        td = r["TD_TD_BUSY_sum"] / max(1.0, cyc * 256)
        ta = r["TA_TA_BUSY_sum"] / max(1.0, cyc * 256)
        tot["fetch"] += f_b
        tot["req"] += q_b
        tot["write"] += w_b
        tot["ns"] += r["ns"]
        lines.append(f"| `{_short_name(r['name'])}` | {r['ns'] / 1e6:.3f} | {f_b / 1e9:.2f} GB | "
                     f"{q_b / 1e9:.2f} GB | {w_b / 1e9:.2f} GB | {100 * hit:.1f} % | "
                     f"{100 * dram:.1f} % | {100 * td:.0f} % | {100 * ta:.0f} % |")
    lines += ["", f"Per launch of the group: {tot['fetch'] / 1e9:.2f} GB fetched (copy-scaled "
                  f"FETCH_SIZE) or {tot['req'] / 1e9:.2f} GB (request sizes), "
                  f"{tot['write'] / 1e9:.2f} GB written.  TD and TA busy: the counters summed "
                  f"over the 256 compute units, divided by 256 times the dispatch's busy "
                  f"clocks (GRBM_GUI_ACTIVE, which sums the 8 dies' clocks: it reads about "
                  f"19 per ns, 8 x 2.4 GHz, so it is divided by 8).  For scale, the 1 GiB "
                  f"copy keeps TD busy {100 * recs[ci]['TD_TD_BUSY_sum'] / max(1.0, recs[ci]['GRBM_GUI_ACTIVE'] / 8 * 256):.0f} % "
                  f"of its time.  Times are the counter runs' own dispatch durations "
                  f"(serialised, so a little longer than in the timed bench).",
              f"Kernel sources at measurement (sha256 of {', '.join(os.path.basename(f) for f in KERNEL_SOURCES)}): "
              f"`{kernel_source_digest()}`.", ""]
    md = os.path.join(ROOT, "profiles", "num_chunk_rmat18_hbm_traffic.md")
    with open(md, "w") as fh:
        fh.write("\n".join(lines))
    chunk_cols = None
    m = [r for r in g7 if "k_num_chunk_pipe" in r["name"]]
    if m:
        chunk_cols = int(_short_name(m[0]["name"]).split(",")[1].strip(" >"))
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump({"group": "num.g7",
                   "kernel": " + ".join(_short_name(r["name"]) for r in g7),
                   "chunk_cols": chunk_cols, "source_sha256": kernel_source_digest(),
                   "fetch_bytes_per_launch": int(tot["fetch"]),
                   "write_bytes_per_launch": int(tot["write"]),
                   "fetch_bytes_by_request_size": int(tot["req"]),
                   "fetch_scale": fscale, "write_scale": wscale,
                   "summary": os.path.basename(md)}, fh, indent=1)
        fh.write("\n")
    print("\n".join(lines))


KERNEL_STATS = {
    "rmat18": {
        "file": "rmat18_kernel_stats.md",
        "title": "Kernel time, R-MAT scale 18 self-product (bench.py default workload)",
        "what": "one MI355X, 5 timed + 2 warm-up steps, so 7 launches of each per-step kernel; "
                "the symbolic-phase kernels run once more, for the group statistics",
        "args": "--steps 5 --warmup 2 --no-cpu --serve-requests 0 --no-configs",
        "note": "Launch groups named in bench.py's `phases_ms`: `num.g7` = `k_num_chunk_pipe` "
                "(dense chunks), `num.g7r` = `k_num_chunk_rank` (four launches: single light "
                "chunks, 8192 columns, and merged light chunks, 16384 columns, each with a "
                "2048- and a 1024-slot accumulator), `sym.g7` = `k_sym_chunk_pipe`, "
                "`num.g5`/`num.g6` = `k_num_block`, `sym.g5`/`sym.g6` = `k_sym_block`, "
                "`plan.ipcount` = `k_ipcount` + `k_ip_groups`, `plan.split` = `k_bsplit` + "
                "`k_sabs` + `k_chunk_items` + item descriptors and scans."},
    "served": {
        "file": "served_gnn_kernel_stats.md",
        "title": "Kernel time, served GNN aggregation trace (1,024 requests C = A_hat X)",
        "what": "one MI355X; the plain loop (one warm-up and three timed passes) and the three "
                "server configurations (each a warm-up, three timed backlogged passes and a "
                "Poisson pass) over the same 1,024 requests, so every request's product runs "
                "20 times; the graph store's generation runs once",
        "args": "--only served --no-cpu --serve-requests 1024",
        "note": "Every B (X) of this trace has at most 512 columns, so every row takes the "
                "group kernels with direct-mapped tables: `k_num_group<G, ..., true>` is the "
                "instantiation without a key table, and the symbolic phase counts from B's row "
                "bitmaps (`k_sym_group`, built by `k_brow_bitmap_batch`).  `k_gnn_features` "
                "builds each X when its request is admitted.  Batches on the server's four "
                "streams overlap, so a dispatch's duration includes time shared with other "
                "streams' kernels, and the totals add up to more than the run's wall time."},
}


def summarize_kernel_stats(path, workload="rmat18"):
    """profiles/<workload>_kernel_stats.md from a rocprofv3 --stats
    kernel_stats.csv of the bench command named in KERNEL_STATS."""
    import csv
    k = KERNEL_STATS[workload]
    with open(path) as fh:
        rows = list(csv.DictReader(fh))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# {k['title']}", "", f"Command ({k['what']}):", "",
             "    cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats -d <out> -o run "
             f"--output-format csv -- python3 /root/repo/bench.py {k['args']}", "",
             "reduced by", "",
             f"    python3 bench.py --summarize-kernel-stats <out>/run_kernel_stats.csv "
             f"--kernel-stats-workload {workload}", "",
             f"`rocprofv3 --stats` summary, kernels above 0.05 % of GPU time "
             f"({total / 1e6:.1f} ms of kernel time in all):", "",
             "| kernel | calls | total (ms) | average (ms) | min (ms) | max (ms) | share |",
             "|---|---|---|---|---|---|---|"]
    for r in rows:
        if float(r["Percentage"]) < 0.05:
            continue
        lines.append(f"| `{_short_name(r['Name'])[:140]}` | {r['Calls']} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e6:.3f} | {float(r['MinNs']) / 1e6:.3f} | "
                     f"{float(r['MaxNs']) / 1e6:.3f} | {float(r['Percentage']):.2f} % |")
    lines += ["", k["note"], ""]
    with open(os.path.join(ROOT, "profiles", k["file"]), "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
    ap.add_argument("--serve-requests", type=int, default=4096,
                    help="requests of the served GNN trace (0: skip it)")

    ap.add_argument("--no-configs", action="store_true",
                    help="skip the ER, contraction and MCL workloads")
    ap.add_argument("--only", default="",
                    help="comma-separated subset of rmat18, er2k, contraction, mcl, tiny, gnn, "
                         "sampling, unsorted, served "
                         "(a study run: the JSON line then holds only those)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this size, and strided reads of a 4 GiB "
                         "buffer, first (counter calibration)")
    ap.add_argument("--summarize-counters", default="",
                    help="no GPU work: reduce the rocprofv3 counter passes under this folder "
                         "(subfolders fetch, write, req, tcc, td) to the traffic summary in "
                         "profiles/")
    ap.add_argument("--summarize-kernel-stats", default="",
                    help="no GPU work: write profiles/<workload>_kernel_stats.md from this "
                         "rocprofv3 kernel_stats.csv")
    ap.add_argument("--kernel-stats-workload", default="rmat18", choices=sorted(KERNEL_STATS),
                    help="which profiled command the kernel_stats.csv comes from")
    args = ap.parse_args()
    if args.summarize_kernel_stats:
        summarize_kernel_stats(args.summarize_kernel_stats, args.kernel_stats_workload)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.calib_copy_mib or 1024)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the row-block "
              f"sharding over several GPUs is designed but not built", file=sys.stderr)
        sys.exit(2)
    if args.only:
        runs = {"rmat18": run_rmat18, "er2k": run_er2k, "contraction": run_contraction,
                "mcl": run_mcl, "tiny": run_tiny, "gnn": run_gnn, "sampling": run_sampling,
                "unsorted": run_unsorted,
                "served": lambda a: run_served(a.serve_requests,
                                               SERVE_CONFIGS)}
        out = {}
        for name in args.only.split(","):
            out[name] = runs[name](args)
        print(json.dumps(out), flush=True)
        return
    out = run_rmat18(args)
    if not args.no_configs:
        out["configs"] = {"er2k": run_er2k(args), "contraction": run_contraction(args),
                          "mcl": run_mcl(args), "tiny_rows": run_tiny(args),
                          "gnn_layer": run_gnn(args), "bulk_sampling": run_sampling(args)}
    if args.serve_requests > 0:
        # small batches (latency, throughput) and large ones (the HBM budget
        # binds: batches are closed by it)
        out["served"] = run_served(args.serve_requests, SERVE_CONFIGS)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
