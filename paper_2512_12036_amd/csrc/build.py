"""Builds libspgemm.so for gfx950 with hipcc (in-tree, next to the package).

Every HIP translation unit is compiled with packed-FP32 instruction
selection disabled (-packed-fp32-ops): the kernels are scalar FP32 code and
must not be turned into v_pk_* forms.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libspgemm.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = ["k_plan.hip", "k_hash.hip", "k_chunk.hip", "k_apps.hip", "k_gnn.hip", "k_rowthread.hip",
           "k_bsort.hip", "api.cpp"]
# the device input generator of the served workload: a library of its own
GEN_SOURCES = ["k_gen.hip"]
GEN_LIB = os.path.join(PKG, "libspgemm_gen.so")
ARCH = os.environ.get("SPGEMM_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


TUNED = os.path.join(PKG, "tuned")


def write_tuned_defaults() -> str:
    """The library's default options, compiled in from tuned/<arch>.json
    (written by the autotuner): a C++ include in the build folder."""
    import json
    with open(os.path.join(TUNED, f"{ARCH}.json")) as f:
        o = json.load(f)["options"]
    lines = ["// Generated from paper_2512_12036_amd/tuned/%s.json by csrc/build.py." % ARCH,
             "constexpr int64_t kTunedSym[kGroups - 1] = {%s};" % ", ".join(map(str, o["sym_upper"])),
             "constexpr int64_t kTunedNum[kGroups - 1] = {%s};" % ", ".join(map(str, o["num_upper"]))]
    for k in ("chunk_cols", "chunks_per_item", "chunk_wgs_per_cu", "chunk_threads",
              "sym_chunk_threads", "num_rank_cap", "chunk_merge", "row_thread"):
        lines.append("constexpr int32_t kTuned_%s = %d;" % (k, int(o[k])))
    os.makedirs(BUILD, exist_ok=True)
    path = os.path.join(BUILD, "tuned_defaults.inc")
    text = "\n".join(lines) + "\n"
    if not os.path.exists(path) or open(path).read() != text:
        with open(path, "w") as f:
            f.write(text)
    return path


def common_flags() -> list[str]:
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", "-I", INCLUDE, "-I", HERE, "-I", BUILD]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *common_flags(), "-x", "hip", "-c", os.path.join(HERE, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip():
        msgs = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if msgs:
            sys.stderr.write("\n".join(msgs) + "\n")
    return obj


def _link(objs, lib):
    tmp = lib + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    write_tuned_defaults()
    with ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES + GEN_SOURCES))
    _link(objs[:len(SOURCES)], LIB)
    _link(objs[len(SOURCES):], GEN_LIB)
    if verbose:
        print(f"built {LIB} and {GEN_LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
