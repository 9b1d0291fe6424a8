"""Host-only checks of the C ABI (no GPU): the library loads, exports every
entry point that include/spgemm.h declares, the ctypes structures have the C
layout, and argument errors are reported before any device work."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2512_12036_amd import spgemm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spgemm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(spgemm_[a-z0-9_]+)\s*\(", text)
    return sorted(set(n for n in names if not n.endswith("_fn")))


def test_library_exports_every_declared_symbol():
    lib = spgemm.load()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), f"missing export {n}"
    assert sorted(spgemm.EXPORTED) == names


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include "spgemm.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu\\n", sizeof(spgemm_csr),'
                   ' sizeof(spgemm_options), sizeof(spgemm_info),'
                   ' offsetof(spgemm_options, chunk_cols));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src),
                           "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    assert [int(x) for x in out] == [ctypes.sizeof(spgemm.CsrDesc),
                                     ctypes.sizeof(spgemm.Options),
                                     ctypes.sizeof(spgemm.Info),
                                     spgemm.Options.chunk_cols.offset]


def test_header_compiles_as_cxx(tmp_path):
    src = tmp_path / "h.cpp"
    src.write_text('#include "spgemm.h"\nint main(){spgemm_options o; (void)o; return 0;}\n')
    subprocess.check_call(["g++", "-std=c++17", "-fsyntax-only", "-I",
                           os.path.join(ROOT, "include"), str(src)])


def test_default_options_are_consistent():
    o = spgemm.default_options()
    sym, num = list(o.sym_upper), list(o.num_upper)
    assert sym[0] == 0 and num[0] == 0
    assert sym == sorted(sym) and num == sorted(num)
    assert sym[6] <= num[6]
    assert o.chunk_cols % 64 == 0 and 64 <= o.chunk_cols <= 16384


def _create(a, b, o):
    lib = spgemm.load()
    h = ctypes.c_void_p()
    code = lib.spgemm_plan_create(ctypes.byref(h), ctypes.byref(a), ctypes.byref(b),
                                  ctypes.byref(o), None, spgemm.ALLOC_FN(), spgemm.FREE_FN(), None)
    assert not h.value
    return code


@pytest.mark.parametrize("field,value", [("chunk_cols", 100), ("chunk_cols", 0),
                                         ("chunk_cols", 32768), ("validate", 7),
                                         ("chunks_per_item", 3), ("chunk_wgs_per_cu", -1),
                                         ("chunk_wgs_per_cu", 65), ("chunk_threads", 96),
                                         ("sym_chunk_threads", 32), ("num_rank_cap", 300),
                                         ("chunk_merge", 3), ("chunk_merge", 16),
                                         ("graph", 2), ("graph", -1), ("validate", 3),
                                         ("item_limit", -1), ("row_thread", 2),
                                         ("accumulate", 2), ("accumulate", -1)])
def test_bad_options_rejected(field, value):
    o = spgemm.default_options()
    setattr(o, field, value)
    a = spgemm.CsrDesc(4, 4, 0, 1, None, None, 0)
    assert _create(a, a, o) == 1


def test_bad_group_bounds_rejected():
    a = spgemm.CsrDesc(4, 4, 0, 1, None, None, 0)
    o = spgemm.default_options()
    o.sym_upper[2] = 10                 # decreasing
    assert _create(a, a, o) == 1
    o = spgemm.default_options()
    o.num_upper[1] = 1000               # over the group's table capacity
    assert _create(a, a, o) == 1
    o = spgemm.default_options()
    o.sym_upper[6] = o.num_upper[6] + 1  # chunked numeric rows must be chunked symbolic rows
    o.sym_upper[6] = min(o.sym_upper[6], 16384)
    assert _create(a, a, o) == 1


def test_dimension_and_argument_errors():
    o = spgemm.default_options()
    a = spgemm.CsrDesc(10, 12, 0, 1, None, None, 0)
    b = spgemm.CsrDesc(13, 9, 0, 1, None, None, 0)
    assert _create(a, b, o) == 2                       # EDIM
    big = spgemm.CsrDesc(1 << 31, 4, 0, 1, None, None, 0)
    assert _create(big, spgemm.CsrDesc(4, 4, 0, 1, None, None, 0), o) == 2
    neg = spgemm.CsrDesc(-1, 4, 0, 1, None, None, 0)
    assert _create(neg, spgemm.CsrDesc(4, 4, 0, 1, None, None, 0), o) == 1
    nul = spgemm.CsrDesc(4, 4, 3, None, None, None, 0)
    assert _create(nul, nul, o) == 1
    lib = spgemm.load()
    assert lib.spgemm_symbolic(None, None, None, None) == 1
    assert lib.spgemm_numeric(None, None, None, None, None) == 1
    lib.spgemm_free(None)              # NULL-safe
    assert lib.spgemm_status_string(8) == b"kernel error flag raised"


def test_product_path_fails_loudly_without_library(tmp_path):
    with pytest.raises(RuntimeError):
        spgemm.load.__wrapped__ if hasattr(spgemm.load, "__wrapped__") else None
        import importlib
        mod = importlib.reload(spgemm)
        mod._lib = None
        mod.load(str(tmp_path / "missing.so"))
    import importlib
    importlib.reload(spgemm)


def test_library_has_no_unresolved_internal_symbols():
    lib = os.path.join(ROOT, "paper_2512_12036_amd", "libspgemm.so")
    out = subprocess.check_output(["nm", "-D", "--undefined-only", lib]).decode()
    missing = [l for l in out.splitlines() if "spg" in l]
    assert not missing, missing


def test_defaults_come_from_the_tuned_file():
    """spgemm_default_options returns what the autotuner wrote for gfx950
    (paper_2512_12036_amd/tuned/gfx950.json), compiled in by the build."""
    import json
    with open(os.path.join(ROOT, "paper_2512_12036_amd", "tuned", "gfx950.json")) as f:
        want = json.load(f)["options"]
    from paper_2512_12036_amd import autotune
    assert autotune.options_dict(spgemm.default_options()) == want
    assert autotune.legal(want)
