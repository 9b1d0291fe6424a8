"""Autotuner for the row-group bounds, the table sizes they imply, the chunk
parameters and the small-row kernel on the current GPU; its result is the
library's default options for the architecture.

Paper Table I fixes four groups with hand-picked bounds for the paper's GPU.
Here the bounds of the eight gfx950 groups (include/spgemm.h) decide which
kernel, and so which LDS table size, handles each row; they and the chunk
parameters are chosen by timing whole products (plan + symbolic + numeric)
and keeping the fastest candidate.  Every candidate produces the same C
(grouping only changes which kernel handles a row), so tuning never trades
accuracy.

The search is a coordinate descent: starting from the current defaults, each
parameter in turn is moved through its legal values with the others fixed,
and a move is kept when it lowers the objective by more than 1 % without
slowing any single workload by more than 1 % (the run-to-run spread of the
medians).  The objective is the geometric mean, over the workloads, of the
time relative to the starting point:
  * rmat18: the R-MAT scale 18 self-product (single product);
  * served: one batch plan of 64 served GNN aggregation requests;
  * er2k:   the Erdos-Renyi 2,000 self-product (latency floor).

    python -m paper_2512_12036_amd.autotune --write

writes paper_2512_12036_amd/tuned/<arch>.json, from which the build compiles
the library's defaults (spgemm_default_options).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TUNED_DIR = os.path.join(HERE, "tuned")

SYM_CAP = [0, 32, 64, 128, 256, 4096, 16384]
NUM_CAP = [0, 32, 64, 128, 256, 2048, 8192]

# parameters searched, with their legal values
SPACE = {
    "chunk_cols": [4096, 8192, 16384],
    "num_rank_cap": [0, 512, 1024, 2048],
    "chunk_merge": [1, 2, 4],
    "sym_chunk_threads": [64, 128],
    "row_thread": [0, 1],
}
BOUND_VALUES = {1: [8, 16, 32], 2: [32, 48, 64], 3: [64, 96, 128], 4: [128, 192, 256],
                5: [512, 768, 1024, 2048], 6: [1024, 2048, 4096, 8192]}


def options_dict(o) -> dict:
    """The tunable fields of an Options struct."""
    return {"sym_upper": [int(x) for x in o.sym_upper], "num_upper": [int(x) for x in o.num_upper],
            "chunk_cols": int(o.chunk_cols), "chunks_per_item": int(o.chunks_per_item),
            "chunk_wgs_per_cu": int(o.chunk_wgs_per_cu), "chunk_threads": int(o.chunk_threads),
            "sym_chunk_threads": int(o.sym_chunk_threads), "num_rank_cap": int(o.num_rank_cap),
            "chunk_merge": int(o.chunk_merge), "row_thread": int(o.row_thread)}


def legal(c: dict) -> bool:
    s, n = c["sym_upper"], c["num_upper"]
    for g in range(1, 7):
        if s[g] < s[g - 1] or n[g] < n[g - 1] or s[g] > SYM_CAP[g] or n[g] > NUM_CAP[g]:
            return False
    if s[6] > n[6]:
        return False
    if c["row_thread"] and (s[1] > 32 or n[1] > 32):
        return False
    if c["num_rank_cap"] == 0 and c["chunk_merge"] > 1:
        return False
    return True


def make(c: dict, profile: int = 0):
    from . import spgemm
    return spgemm.make_options(profile=profile, **c)


def time_product(da, db, opt, steps: int = 7) -> float:
    """Median wall ms of plan + symbolic + allocation + numeric."""
    import torch
    from . import spgemm
    per = []
    for k in range(steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = spgemm.Plan(da, db, opt)
        plan.symbolic()
        cols, vals = plan.allocate_outputs()
        plan.numeric(cols, vals)
        torch.cuda.synchronize()
        if k > 0:
            per.append((time.perf_counter() - t0) * 1e3)
        plan.free()
        del cols, vals
    return float(np.median(per))


def workloads(names):
    from . import gen, serve, spgemm
    out = {}
    for name in names:
        if name == "rmat18":
            a = spgemm.to_device(gen.rmat(18, 16, seed=2))
            out[name] = (a, a)
        elif name == "rmat16":
            a = spgemm.to_device(gen.rmat(16, 16, seed=2))
            out[name] = (a, a)
        elif name == "er2k":
            a = spgemm.to_device(gen.er(2000, 16000, seed=1))
            out[name] = (a, a)
        elif name == "served":
            reqs = serve.gnn_requests(range(64), "cuda")
            out[name] = ([r.a for r in reqs], [r.b for r in reqs])
        else:
            raise ValueError(name)
    return out


def score(c: dict, loads, base=None, log=None):
    t = {name: time_product(a, b, make(c)) for name, (a, b) in loads.items()}
    if base is None:
        return t, 1.0
    g = math.exp(sum(math.log(t[k] / base[k]) for k in t) / len(t))
    if log:
        log(json.dumps({"score": round(g, 4), "ms": {k: round(v, 3) for k, v in t.items()},
                        "cand": c}))
    return t, g


def tune(loads, start: dict, rounds: int = 2, log=None):
    """Coordinate descent from `start`; returns (best, its times, the
    starting times, every trial)."""
    base, _ = score(start, loads)
    best, best_g, best_t0 = dict(start), 1.0, base
    trials = []
    for _ in range(rounds):
        improved = False
        moves = [(k, v) for k, vals in SPACE.items() for v in vals]
        moves += [(("sym", g), v) for g, vals in BOUND_VALUES.items() for v in vals]
        moves += [(("num", g), v) for g, vals in BOUND_VALUES.items() for v in vals]
        for key, v in moves:
            c = json.loads(json.dumps(best))
            if isinstance(key, tuple):
                side, g = key
                arr = c["sym_upper" if side == "sym" else "num_upper"]
                if arr[g] == v:
                    continue
                arr[g] = v
            else:
                if c[key] == v:
                    continue
                c[key] = v
            if not legal(c):
                continue
            t, g = score(c, loads, base, log)
            trials.append({"cand": c, "ms": t, "score": g})
            # a move must win by more than the run-to-run spread, and may not
            # slow any workload down by more than that spread
            worse = any(t[k] > 1.01 * best_t0[k] for k in t)
            if g < best_g * 0.99 and not worse:
                best, best_g, best_t0, improved = c, g, t, True
        if not improved:
            break
    best_t, _ = score(best, loads)
    return best, best_t, base, trials


def arch_name() -> str:
    import torch
    name = torch.cuda.get_device_properties(0).gcnArchName
    return name.split(":")[0]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", default="rmat18,served,er2k")
    ap.add_argument("--rounds", type=int, default=2)
    ap.add_argument("--write", action="store_true",
                    help="write tuned/<arch>.json (the library's compiled-in defaults)")
    ap.add_argument("--write-dir", default=TUNED_DIR,
                    help="folder of the tuned file (default: the package's tuned/)")
    ap.add_argument("--out", default=None, help="also write every trial to this file")
    args = ap.parse_args()
    from . import spgemm

    def log(msg):
        print(msg, flush=True)

    loads = workloads(args.workloads.split(","))
    start = options_dict(spgemm.default_options())
    best, best_t, base, trials = tune(loads, start, args.rounds, log)
    log("BEST " + json.dumps({"options": best, "ms": best_t, "start_ms": base}))
    arch = arch_name()
    if args.write:
        os.makedirs(args.write_dir, exist_ok=True)
        with open(os.path.join(args.write_dir, f"{arch}.json"), "w") as f:
            json.dump({"arch": arch, "options": best,
                       "tuned_on": {"workloads": list(loads), "ms": best_t,
                                    "start_ms": base, "trials": len(trials)},
                       "command": "python -m paper_2512_12036_amd.autotune --write"},
                      f, indent=1)
            f.write("\n")
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"arch": arch, "best": best, "trials": trials}, f, indent=1)


if __name__ == "__main__":
    sys.exit(main())
