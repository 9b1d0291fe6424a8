"""Continuous-batching server for streams of SpGEMM requests.

Every request is one product C = A * B.  A is in device memory when the
request arrives (for the GNN aggregation requests: the graph's normalised
adjacency, held resident like a model's graph store); B either is too, or is
built on the device when the request is admitted (the request's features,
from their seed) and released when it completes.  The server admits the
requests that have arrived, as HBM budget and stream slots free up, into
batches; a batch is one batch plan of the C ABI (spgemm_plan_create_batch):
each phase of the method (intermediate-product count, grouping, symbolic,
numeric) runs as one launch per row group over the rows of every product in
the batch, a global bin queue of (product, row) entries.  Batches run on
their own HIP streams, so the numeric phase of one batch overlaps the planning
of the next, and requests that arrive while others are on the GPU join the
next batch (continuous batching).

With device_driven, a batch is a device-driven plan (spgemm_plan_create_device
and spgemm_execute_arena): the whole batch runs with no host synchronisation,
C in one arena sized by the requests' nnz bounds, and the host only reads the
batch's error flags and output offsets once it has completed.

Admission control: each request carries an upper bound of its device
footprint, taken before it is admitted: the plan workspace bound
(``workspace_bound``, from the plan's allocations), C's arrays at the bound
nnz(C) <= sum over rows of min(IP_i, ncols) and, when B is built on
admission, B's arrays.  IP and the nnz bound come from the library's
row-size estimation (spgemm_estimate, Algorithm 1).  A batch is admitted only
while the sum over admitted, unfinished requests stays within the budget.
After the symbolic phase the batch's bound is replaced by its exact footprint
(plan workspace + C + B), whichever is larger.  When a batch completes, its
kernel error flags are read (spgemm_sync) and an error raises.

The plain baseline runs the same requests one after another, each with its
own single-product plan: (build B,) plan, symbolic (synchronises), allocation,
numeric, synchronise, release.

Both loops run with Python's cyclic garbage collector paused (its full
collections would stall the host thread, and with it the GPU's feed).
"""
from __future__ import annotations

import collections
import dataclasses
import functools
import gc
import time
from typing import Callable

import numpy as np

from . import spgemm


def _collector_paused(fn):
    """Runs fn with Python's cyclic garbage collector paused.  Its full
    collections stop the host thread for tens of milliseconds once a trace's
    request objects are alive (36-51 ms measured with 4,096 requests), and
    while the host thread is stopped no work is enqueued and the GPU drains.
    Reference counting still frees every acyclic object at once; the
    collector resumes when fn returns."""
    @functools.wraps(fn)
    def wrapper(*args, **kwargs):
        was = gc.isenabled()
        gc.disable()
        try:
            return fn(*args, **kwargs)
        finally:
            if was:
                gc.enable()
    return wrapper

WS_BYTES_FIXED = 1 << 20      # per-plan descriptors, statistics, scan tiles, rounding
SYM_CHUNK_MIN = 1024          # default sym_upper[6]: rows above it are column-chunked
BITMAP_COLS = 512             # B of at most this many columns is also kept as row bitmaps


_STREAMS: dict = {}


def _server_streams(device, n: int):
    """The first n of the process's server streams on `device`.  Servers
    share them: PyTorch's caching allocator keeps one pool of cached
    segments per stream, so servers on fresh streams could not reuse what
    earlier ones cached, and reserved memory would grow with every server."""
    import torch
    pool = _STREAMS.setdefault(str(device), [])
    while len(pool) < n:
        pool.append(torch.cuda.Stream(device))
    return pool[:n]


@dataclasses.dataclass
class Request:
    rid: int
    a: spgemm.DeviceCsr
    b: spgemm.DeviceCsr | None     # None: built by make_b when admitted
    arrival: float = 0.0           # seconds after the start of the trace
    ip: int = 0                    # sum of intermediate products
    bound_bytes: int = 0           # admission bound of the device footprint
    make_b: Callable | None = None  # builds B on the current stream
    b_bytes: int = 0               # device bytes of B when built on admission
    nnz_bound: int = 0             # sum over rows of min(IP, ncols) >= nnz(C)


@dataclasses.dataclass
class Done:
    rid: int
    rpt: object
    col: object
    val: object
    nnz: int
    t_admit: float
    t_done: float
    batch: int
    b: object = None               # B, when it was built on admission and kept


def workspace_bound(m: int, nnz_a: int, k: int, ncols: int, ip_total: int,
                    chunk_cols: int = 8192) -> int:
    """Upper bound of a single product's plan workspace in bytes, from the
    arrays the plan allocates: per row 8-byte IP, output count, C row
    pointer, two row-map entries, a 4-byte slot and the grouping histograms;
    for the column-chunked rows (more than SYM_CHUNK_MIN possible outputs,
    so at most ip_total / (SYM_CHUNK_MIN + 1) of them) the chunk bounds of
    B's rows, the sub-range tables, the per-chunk counts, bitmaps and the
    item descriptors of both phases; for a B of at most BITMAP_COLS columns,
    its rows as column bitmaps."""
    per_row = 8 * 3 + 8 * 2 + 4 + 8
    total = WS_BYTES_FIXED + per_row * (m + 1) + 16 * (m // 256 + 1) * 8
    if 0 < ncols <= BITMAP_COLS:
        total += 4 * (-(-ncols // 32)) * k + 256          # B's rows as column bitmaps
    if ncols > SYM_CHUNK_MIN and ip_total > SYM_CHUNK_MIN:
        nch = 8 * max(1, -(-ncols // (8 * chunk_cols)))
        w = max(64, -(-(-(-ncols // nch)) // 64) * 64)
        wpc = -(-w // 32)
        nh = min(m, ip_total // (SYM_CHUNK_MIN + 1))
        items = nh * nch
        total += 4 * k * (nch + 1)                     # chunk bounds of B's rows
        total += 4 * nnz_a * (nch + 1)                 # sub-range tables
        total += nh * 8 * 12                           # per-row chunk-row arrays
        total += items * (8 * 4 + 4 * 4 + 56 * 3 + 4 * wpc + 8 * 4)
    return int(total)


def estimate_many(pairs, device="cuda"):
    """(IP, nnz bound) of every (A, B) in `pairs` (B may carry row pointers
    only), from the library's Algorithm 1 on the device, one synchronisation
    for all of them."""
    import torch
    out = torch.zeros((max(len(pairs), 1), 4), dtype=torch.int64, device=device)
    for q, (a, b) in enumerate(pairs):
        spgemm.estimate_async(a, b, out[q])
    h = out.cpu().numpy()
    return [(int(h[q, 0]), int(h[q, 1])) for q in range(len(pairs))]


def footprint(a, b_nrows: int, b_ncols: int, ip: int, nnz_bound: int, b_bytes: int = 0) -> int:
    """Admission bound of C = A * B in bytes: plan workspace bound, C's row
    pointers, columns and values at the nnz bound, and B when it is built on
    admission."""
    return (workspace_bound(a.nrows, a.nnz, b_nrows, b_ncols, ip) + 8 * (a.nrows + 1)
            + 8 * nnz_bound + b_bytes)


class Server:
    def __init__(self, budget_bytes: int = 200 * 10 ** 9, max_batch: int = 64,
                 max_batch_ip: int = 8 << 30, n_streams: int = 4,
                 options: spgemm.Options | None = None, keep_results: bool = False,
                 device="cuda", device_driven: bool = False):
        import torch
        self.device_driven = device_driven
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.max_batch_ip = max_batch_ip
        self.options = options
        self.keep = keep_results
        self.device = torch.device(device)
        self.streams = _server_streams(self.device, n_streams)

    @_collector_paused
    def run(self, requests: list[Request], keep_rids=None):
        """Serves the trace; returns (stats dict, list of Done).  Results
        (and B when built on admission) are kept for the requests in
        keep_rids, or for all of them with keep_results."""
        import torch
        torch.cuda.synchronize(self.device)
        keep_rids = set(keep_rids) if keep_rids is not None else None
        order = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in order:
            if r.bound_bytes > self.budget:
                raise ValueError(f"request {r.rid} alone exceeds the HBM budget")
        pending = collections.deque(order)
        waiting: collections.deque = collections.deque()
        inflight = []          # dicts: stream index, plan, reqs, outputs, event, bytes, t_admit
        free_streams = list(range(len(self.streams)))
        in_use = 0
        peak = 0
        budget_waits = 0       # times nothing could be admitted for the budget
        budget_cuts = 0        # batches closed early because the next request did not fit
        blocked = False
        done: list[Done] = []
        t_evt = []             # (rid, done event) for exact completion times
        nbatch = 0
        ref = torch.cuda.Event(enable_timing=True)
        ref.record(torch.cuda.current_stream(self.device))
        t0 = time.perf_counter()

        def kept(rid):
            return self.keep or (keep_rids is not None and rid in keep_rids)

        def finish(fl):
            nonlocal in_use
            fl["plan"].sync()          # raises on a kernel error flag
            fl["plan"].free()
            if "arena" in fl:          # device-driven: each request's slice of the arena
                rpts, off, col, val = fl.pop("arena")
                o = off.cpu().tolist()
                fl["rpts"] = rpts
                fl["nnz"] = [o[k + 1] - o[k] for k in range(len(fl["reqs"]))]
                fl["cols"] = [col[o[k]:o[k + 1]] for k in range(len(fl["reqs"]))]
                fl["vals"] = [val[o[k]:o[k + 1]] for k in range(len(fl["reqs"]))]
            for k, r in enumerate(fl["reqs"]):
                keep = kept(r.rid)
                done.append(Done(r.rid, fl["rpts"][k] if keep else None,
                                 fl["cols"][k] if keep else None,
                                 fl["vals"][k] if keep else None,
                                 fl["nnz"][k], fl["t_admit"], 0.0, fl["batch"],
                                 fl["bs"][k] if (keep and r.make_b) else None))
                t_evt.append((len(done) - 1, fl["event"]))
            fl.clear()
            in_use -= fl_bytes.pop(id(fl))
            free_streams.append(stream_of.pop(id(fl)))

        fl_bytes, stream_of = {}, {}
        batch_bytes = []       # (admission bound, exact footprint) per batch
        while pending or waiting or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            still = []
            for fl in inflight:
                if fl["event"].query():
                    finish(fl)
                else:
                    still.append(fl)
            inflight[:] = still
            if waiting and free_streams:
                batch, ip_sum, need = [], 0, 0
                while waiting and len(batch) < self.max_batch:
                    r = waiting[0]
                    if batch and (ip_sum + r.ip > self.max_batch_ip):
                        break
                    if in_use + need + r.bound_bytes > self.budget:
                        if not batch and not blocked:
                            budget_waits += 1
                        if batch:
                            budget_cuts += 1
                        blocked = not batch
                        break
                    batch.append(waiting.popleft())
                    ip_sum += r.ip
                    need += r.bound_bytes
                if batch:
                    blocked = False
                    si = free_streams.pop(0)
                    s = self.streams[si]
                    in_use += need
                    peak = max(peak, in_use)
                    t_admit = time.perf_counter() - t0
                    arena = None
                    with torch.cuda.stream(s):
                        bs = [r.b if r.b is not None else r.make_b() for r in batch]
                        if self.device_driven:
                            # no host synchronisation: C of the whole batch in
                            # one arena sized by the requests' nnz bounds
                            plan = spgemm.DevicePlan([r.a for r in batch], bs, self.options, s)
                            cap = sum(r.nnz_bound for r in batch)
                            rpts = [torch.empty(r.a.nrows + 1, dtype=torch.int64, device=s.device)
                                    for r in batch]
                            off = torch.empty(len(batch) + 1, dtype=torch.int64, device=s.device)
                            col = torch.empty(max(cap, 1), dtype=torch.int32, device=s.device)
                            val = torch.empty(max(cap, 1), dtype=torch.float32, device=s.device)
                            plan.execute(rpts, off, col[:cap], val[:cap])
                            arena = (rpts, off, col, val)
                            nnz = [r.nnz_bound for r in batch]
                        else:
                            plan = spgemm.Plan([r.a for r in batch], bs, self.options, s)
                            nnz = plan.symbolic()
                            cols, vals = plan.allocate_outputs()
                            plan.numeric(cols, vals)
                        ev = torch.cuda.Event(enable_timing=True)
                        ev.record(s)
                    exact = plan.info().workspace_bytes + sum(
                        8 * (r.a.nrows + 1) + 8 * k + (r.b_bytes if r.make_b else 0)
                        for r, k in zip(batch, nnz))
                    held = max(exact, need)
                    batch_bytes.append((need, exact))
                    in_use += held - need
                    peak = max(peak, in_use)
                    if arena is not None:
                        fl = dict(plan=plan, reqs=batch, arena=arena, event=ev,
                                  t_admit=t_admit, batch=nbatch, bs=bs)
                    else:
                        fl = dict(plan=plan, reqs=batch, rpts=plan.rpts, cols=cols, vals=vals,
                                  nnz=nnz, event=ev, t_admit=t_admit, batch=nbatch, bs=bs)
                    fl_bytes[id(fl)] = held
                    stream_of[id(fl)] = si
                    inflight.append(fl)
                    nbatch += 1
                    del bs, plan, arena
                    if not self.device_driven:
                        del cols, vals
                    continue
            if inflight:
                if pending and not waiting:
                    nxt = pending[0].arrival - (time.perf_counter() - t0)
                    if nxt > 0:
                        time.sleep(min(nxt, 2e-4))
                else:
                    time.sleep(5e-5)
            elif pending:
                time.sleep(max(0.0, min(pending[0].arrival - (time.perf_counter() - t0), 1e-3)))
        torch.cuda.synchronize(self.device)
        wall = time.perf_counter() - t0
        for k, ev in t_evt:
            done[k].t_done = ref.elapsed_time(ev) * 1e-3
        arr = {r.rid: r.arrival for r in requests}
        lat = np.array([d.t_done - arr[d.rid] for d in done])
        makespan = max(d.t_done for d in done) if done else 0.0
        ip_total = sum(r.ip for r in requests)
        stats = {"requests": len(done), "batches": nbatch, "makespan_s": makespan,
                 "wall_s": wall, "p50_ms": float(np.percentile(lat, 50) * 1e3) if done else None,
                 "p99_ms": float(np.percentile(lat, 99) * 1e3) if done else None,
                 "gflops": 2.0 * ip_total / makespan / 1e9 if makespan > 0 else None,
                 "peak_admitted_bytes": int(peak), "budget_waits": int(budget_waits),
                 "budget_cuts": int(budget_cuts),
                 "batch_bytes": batch_bytes}
        return stats, done


@_collector_paused
def run_plain(requests: list[Request], options: spgemm.Options | None = None,
              keep_results: bool = False):
    """The plain baseline: one request after another, each on its own plan.
    Returns (stats, list of Done)."""
    import torch
    dev = requests[0].a.rpt.device
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    done = []
    lat = []
    for r in sorted(requests, key=lambda r: (r.arrival, r.rid)):
        t_start = time.perf_counter() - t0
        b = r.b if r.b is not None else r.make_b()
        plan = spgemm.Plan(r.a, b, options)
        nnz = plan.symbolic()
        cols, vals = plan.allocate_outputs()
        plan.numeric(cols, vals)
        plan.sync()
        t_end = time.perf_counter() - t0
        rpt = plan.rpts[0]
        plan.free()
        done.append(Done(r.rid, rpt if keep_results else None, cols[0] if keep_results else None,
                         vals[0] if keep_results else None, nnz[0], t_start, t_end, -1,
                         b if (keep_results and r.make_b) else None))
        del b, cols, vals, rpt
        lat.append(t_end - max(r.arrival, 0.0))
    torch.cuda.synchronize(dev)
    makespan = time.perf_counter() - t0
    ip_total = sum(r.ip for r in requests)
    stats = {"requests": len(done), "makespan_s": makespan,
             "p50_ms": float(np.percentile(lat, 50) * 1e3),
             "p99_ms": float(np.percentile(lat, 99) * 1e3),
             "gflops": 2.0 * ip_total / makespan / 1e9}
    return stats, done


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def _dev(m) -> spgemm.DeviceCsr:
    return spgemm.DeviceCsr(m.nrows, m.ncols, m.rpt, m.col, m.val, True)


def gnn_requests(seeds, device="cuda", features_on_admission: bool = False,
                 log=None, **overrides) -> list[Request]:
    """Served GNN aggregation requests C = A_hat X (one per seed).  A_hat is
    generated in device memory now (the resident graph store); X too, or,
    with features_on_admission, only when the request is admitted, by one
    generator kernel (and it is released when the request completes).
    Admission bounds come from the library's Algorithm 1 (spgemm_estimate) on
    A_hat and X's row pointers."""
    import torch
    from . import gen
    seeds = [int(s) for s in seeds]
    out = []
    step = 256
    for g0 in range(0, len(seeds), step):
        group = seeds[g0:g0 + step]
        pairs, items = [], []
        kept_all = [gen.gnn_kept_columns(seed, *gen.gnn_features_shape(
            seed, overrides.get("n"), overrides.get("f"), overrides.get("rho"))[1:])
            for seed in group] if features_on_admission else []
        kept_dev = (torch.from_numpy(np.concatenate(kept_all)).to(device)
                    if features_on_admission else None)
        koff = 0
        for k, seed in enumerate(group):
            n, f, nk = gen.gnn_features_shape(seed, overrides.get("n"), overrides.get("f"),
                                              overrides.get("rho"))
            a = _dev(gen.gnn_graph_t(seed, device, overrides.get("n"), overrides.get("d")))
            if features_on_admission:
                kept = kept_dev[koff:koff + nk]
                koff += nk
                xs = _dev(gen.TorchCsr(n, f, torch.arange(n + 1, dtype=torch.int64,
                                                          device=device) * nk,
                                       torch.zeros(0, dtype=torch.int32, device=device),
                                       torch.zeros(0, dtype=torch.float32, device=device)))
                x = None

                def make(seed=seed, kept=kept, n=n, f=f):
                    return _dev(gen.gnn_features_device(seed, kept, n, f))
                b_bytes = 8 * (n + 1) + 8 * n * nk
            else:
                x = xs = _dev(gen.gnn_features_t(seed, device, overrides.get("n"),
                                                 overrides.get("f"), overrides.get("rho")))
                make, b_bytes = None, 0
            pairs.append((a, xs))
            items.append((g0 + k, a, x, make, b_bytes, f, n))
        est = estimate_many(pairs, device)
        for (rid, a, x, make, b_bytes, f, n), (ip, nnz_bound) in zip(items, est):
            out.append(Request(rid, a, x, 0.0, ip, footprint(a, n, f, ip, nnz_bound, b_bytes),
                               make, b_bytes, nnz_bound))
        del pairs
        if log is not None:
            log(f"[serve] {len(out)} / {len(seeds)} requests generated")
    torch.cuda.synchronize()
    return out
