"""Continuous-batching server for streams of SpGEMM requests.

Every request is one product C = A * B whose operands are already in device
memory.  The server admits the requests that have arrived, as HBM budget and
stream slots free up, into batches; a batch is one batch plan of the C ABI
(spgemm_plan_create_batch): each phase of the method (intermediate-product
count, grouping, symbolic, numeric) runs as one launch per row group over the
rows of every product in the batch, a global bin queue of (product, row)
entries.  Batches run on their own HIP streams, so the numeric phase of one
batch overlaps the planning of the next, and requests that arrive while
others are on the GPU join the next batch (continuous batching).

Admission control: each request carries an upper bound of its device
footprint (workspace estimate plus C's arrays at the bound
nnz(C_i) <= min(IP_i, ncols) per row); a batch is admitted only while the sum
over admitted, unfinished requests stays within the budget.  After the
symbolic phase the bound is replaced by the exact output size.

The plain baseline runs the same requests one after another, each with its
own single-product plan: plan, symbolic (synchronises), allocation, numeric,
synchronise, release.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import spgemm

WS_BYTES_PER_ROW = 112        # per-row plan arrays (IP, counts, maps, pointers)
WS_BYTES_FIXED = 1 << 20      # per-plan scan tiles, descriptors, statistics


@dataclasses.dataclass
class Request:
    rid: int
    a: spgemm.DeviceCsr
    b: spgemm.DeviceCsr
    arrival: float = 0.0       # seconds after the start of the trace
    ip: int = 0                # sum of intermediate products
    bound_bytes: int = 0       # admission bound of the device footprint


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


def footprint_bound(a: spgemm.DeviceCsr, b: spgemm.DeviceCsr):
    """(sum of intermediate products, upper bound of the device footprint in
    bytes) of C = A * B, from a few torch reductions on the device."""
    import torch
    if a.nnz == 0:
        return 0, WS_BYTES_FIXED + WS_BYTES_PER_ROW * a.nrows + 8 * (a.nrows + 1)
    blen = b.rpt[1:] - b.rpt[:-1]
    per = blen[a.col.long()]
    rid = torch.repeat_interleave(torch.arange(a.nrows, device=a.rpt.device),
                                  a.rpt[1:] - a.rpt[:-1])
    ip_row = torch.zeros(a.nrows, dtype=torch.int64, device=a.rpt.device)
    ip_row.index_add_(0, rid, per)
    ip = int(ip_row.sum())
    nnz_bound = int(torch.clamp(ip_row, max=b.ncols).sum())
    return ip, (WS_BYTES_FIXED + WS_BYTES_PER_ROW * a.nrows + 8 * (a.nrows + 1)
                + 8 * nnz_bound + 16 * a.nnz)


class Server:
    def __init__(self, budget_bytes: int = 200 << 30, max_batch: int = 64,
                 max_batch_ip: int = 8 << 30, n_streams: int = 4,
                 options: spgemm.Options | None = None, keep_results: bool = False,
                 device="cuda"):
        import torch
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.max_batch_ip = max_batch_ip
        self.options = options
        self.keep = keep_results
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(self.device) for _ in range(n_streams)]

    def run(self, requests: list[Request]):
        """Serves the trace; returns (stats dict, list of Done)."""
        import torch
        torch.cuda.synchronize(self.device)
        order = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in order:
            if r.bound_bytes > self.budget:
                raise ValueError(f"request {r.rid} alone exceeds the HBM budget")
        pending = collections.deque(order)
        waiting: collections.deque = collections.deque()
        inflight = []          # dicts: stream index, plan, reqs, outputs, event, bytes, t_admit
        free_streams = list(range(len(self.streams)))
        in_use = 0
        done: list[Done] = []
        t_evt = []             # (rid, done event) for exact completion times
        nbatch = 0
        ref = torch.cuda.Event(enable_timing=True)
        ref.record(torch.cuda.current_stream(self.device))
        t0 = time.perf_counter()

        def finish(fl):
            nonlocal in_use
            fl["plan"].free()
            for k, r in enumerate(fl["reqs"]):
                done.append(Done(r.rid, fl["rpts"][k] if self.keep else None,
                                 fl["cols"][k] if self.keep else None,
                                 fl["vals"][k] if self.keep else None,
                                 fl["nnz"][k], fl["t_admit"], 0.0, fl["batch"]))
                t_evt.append((len(done) - 1, fl["event"]))
            in_use -= fl["bytes"]
            free_streams.append(fl["stream"])

        while pending or waiting or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            for fl in list(inflight):
                if fl["event"].query():
                    inflight.remove(fl)
                    finish(fl)
            if waiting and free_streams:
                batch, ip_sum, need = [], 0, 0
                while waiting and len(batch) < self.max_batch:
                    r = waiting[0]
                    if batch and (ip_sum + r.ip > self.max_batch_ip):
                        break
                    if in_use + need + r.bound_bytes > self.budget:
                        break
                    batch.append(waiting.popleft())
                    ip_sum += r.ip
                    need += r.bound_bytes
                if batch:
                    si = free_streams.pop(0)
                    s = self.streams[si]
                    in_use += need
                    t_admit = time.perf_counter() - t0
                    with torch.cuda.stream(s):
                        plan = spgemm.Plan([r.a for r in batch], [r.b for r in batch],
                                           self.options, s)
                        nnz = plan.symbolic()
                        cols, vals = plan.allocate_outputs()
                        plan.numeric(cols, vals)
                        ev = torch.cuda.Event(enable_timing=True)
                        ev.record(s)
                    exact = plan.info().workspace_bytes + sum(
                        8 * (r.a.nrows + 1) + 8 * k for r, k in zip(batch, nnz))
                    exact = min(exact, need)
                    in_use -= need - exact
                    inflight.append(dict(stream=si, plan=plan, reqs=batch, rpts=plan.rpts,
                                         cols=cols, vals=vals, nnz=nnz, event=ev, bytes=exact,
                                         t_admit=t_admit, batch=nbatch))
                    nbatch += 1
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
                 "gflops": 2.0 * ip_total / makespan / 1e9 if makespan > 0 else None}
        return stats, done


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
        plan = spgemm.Plan(r.a, r.b, options)
        nnz = plan.symbolic()
        cols, vals = plan.allocate_outputs()
        plan.numeric(cols, vals)
        plan.sync()
        t_end = time.perf_counter() - t0
        rpt = plan.rpts[0]
        plan.free()
        done.append(Done(r.rid, rpt if keep_results else None, cols[0] if keep_results else None,
                         vals[0] if keep_results else None, nnz[0], t_start, t_end, -1))
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


def gnn_requests(seeds, device="cuda", **overrides) -> list[Request]:
    """Served GNN aggregation requests C = A_hat X (one per seed), generated
    in device memory, with their admission bounds."""
    from . import gen
    out = []
    for k, seed in enumerate(seeds):
        a, x, _ = gen.gnn_request_t(int(seed), device, **overrides)
        da = spgemm.DeviceCsr(a.nrows, a.ncols, a.rpt, a.col, a.val, True)
        dx = spgemm.DeviceCsr(x.nrows, x.ncols, x.rpt, x.col, x.val, True)
        ip, bound = footprint_bound(da, dx)
        out.append(Request(k, da, dx, 0.0, ip, bound))
    return out
