"""Autotuner for the row-group bounds, the chunk width, the rank cap and the
chunk merging on the current GPU.

Paper Table I fixes four groups with hand-picked bounds for the paper's GPU;
here the bounds of the eight gfx950 groups (see include/spgemm.h) and the
column-chunk width are chosen by timing whole products (plan + symbolic +
numeric) on a workload and keeping the fastest candidate.  Every candidate
produces the same C (grouping only changes which kernel handles a row), so
tuning never trades accuracy.

    python -m paper_2512_12036_amd.autotune --workload rmat18 --out tuned.json
"""
from __future__ import annotations

import argparse
import itertools
import json
import sys
import time

import numpy as np

SYM_CAP = [0, 32, 64, 128, 256, 4096, 16384]
NUM_CAP = [0, 32, 64, 128, 256, 2048, 8192]


def candidates(quick: bool = False):
    """Candidate option sets (keyword arguments of spgemm.make_options)."""
    small = [0, 32, 64, 128, 256]
    out = []
    for cc, cap, sthr, merge in itertools.product([4096, 8192, 16384], [0, 512, 1024, 2048],
                                                  [64, 128], [1, 2, 4]):
        if cap == 0 and merge > 1:
            continue  # merging needs the rank accumulator
        out.append(dict(chunk_cols=cc, sym_upper=small + [1024, 1024],
                        num_upper=small + [1024, 1024], chunks_per_item=1, chunk_wgs_per_cu=0,
                        chunk_threads=0, sym_chunk_threads=sthr, num_rank_cap=cap,
                        chunk_merge=merge))
    if quick:
        out = [c for c in out if c["chunk_cols"] == 8192 and c["sym_chunk_threads"] == 64]
    return out


def time_product(da, db, opt, steps: int = 3):
    import torch
    from . import spgemm
    per = []
    groups = {}
    for k in range(steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = spgemm.Plan(da, db, opt)
        plan.symbolic()
        cols, vals = plan.allocate_outputs()
        plan.numeric(cols, vals)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if k > 0:
            per.append((t1 - t0) * 1e3)
            for name, ms in plan.timings():
                groups[name] = groups.get(name, 0.0) + ms / steps
        plan.free()
        del cols, vals
    return float(np.median(per)), groups


def tune(a, b=None, quick=False, log=None):
    from . import spgemm
    da = spgemm.to_device(a)
    db = da if b is None else spgemm.to_device(b)
    results = []
    for cand in candidates(quick):
        opt = spgemm.make_options(profile=1, **cand)
        ms, groups = time_product(da, db, opt)
        rec = dict(cand)
        rec["ms"] = round(ms, 3)
        rec["groups_ms"] = {k: round(v, 3) for k, v in sorted(groups.items())}
        results.append(rec)
        if log:
            log(json.dumps(rec))
    best = min(results, key=lambda r: r["ms"])
    return best, results


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="rmat18", choices=["rmat18", "rmat16", "er2k"])
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    from . import gen
    if args.workload == "rmat18":
        a = gen.rmat(18, 16, seed=2)
    elif args.workload == "rmat16":
        a = gen.rmat(16, 16, seed=2)
    else:
        a = gen.er(2000, 16000, seed=1)

    def log(msg):
        print(msg, flush=True)

    best, results = tune(a, quick=args.quick, log=log)
    print("BEST " + json.dumps(best), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"arch": "gfx950", "workload": args.workload, "best": best,
                       "all": results}, f, indent=1)


if __name__ == "__main__":
    sys.exit(main())
