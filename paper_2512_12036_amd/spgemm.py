"""Thin Python binding of libspgemm.so (include/spgemm.h).

Argument marshalling only: every step of the product runs in the library's
HIP kernels.  PyTorch provides device memory (its caching allocator backs
the library's workspace through the allocator callbacks) and the stream
(``torch.cuda.current_stream()``).  There is no CPU fallback: if the
library is not built, or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspgemm.so")
NGROUPS = 8
ROWS_SORTED = 1

_I64 = ctypes.c_int64
_VP = ctypes.c_void_p


class CsrDesc(ctypes.Structure):
    _fields_ = [("nrows", _I64), ("ncols", _I64), ("nnz", _I64), ("row_ptr", _VP),
                ("col_idx", _VP), ("values", _VP), ("flags", ctypes.c_uint32)]


class Options(ctypes.Structure):
    _fields_ = [("sym_upper", _I64 * (NGROUPS - 1)), ("num_upper", _I64 * (NGROUPS - 1)),
                ("chunk_cols", ctypes.c_int32), ("validate", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("chunks_per_item", ctypes.c_int32),
                ("chunk_wgs_per_cu", ctypes.c_int32), ("chunk_threads", ctypes.c_int32),
                ("sym_chunk_threads", ctypes.c_int32), ("num_rank_cap", ctypes.c_int32),
                ("chunk_merge", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("item_limit", _I64), ("row_thread", ctypes.c_int32),
                ("accumulate", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("flops", _I64), ("ip_total", _I64), ("ip_max", _I64), ("nnz_c", _I64),
                ("sym_group_rows", _I64 * NGROUPS), ("num_group_rows", _I64 * NGROUPS),
                ("chunk_cols", _I64), ("chunks_per_row", _I64),
                ("workspace_bytes", ctypes.c_size_t)]


ALLOC_FN = ctypes.CFUNCTYPE(_VP, _VP, ctypes.c_size_t, _VP)
FREE_FN = ctypes.CFUNCTYPE(None, _VP, _VP, _VP)

STATUS = {0: "SPGEMM_OK", 1: "SPGEMM_EINVAL", 2: "SPGEMM_EDIM", 3: "SPGEMM_EINDEX",
          4: "SPGEMM_EOVERFLOW", 5: "SPGEMM_ENOMEM", 6: "SPGEMM_EHIP", 7: "SPGEMM_ESTATE",
          8: "SPGEMM_EINTERNAL"}

EXPORTED = ["spgemm_default_options", "spgemm_plan_create", "spgemm_plan_create_batch",
            "spgemm_symbolic", "spgemm_symbolic_batch", "spgemm_numeric",
            "spgemm_numeric_batch", "spgemm_sync", "spgemm_get_info", "spgemm_export",
            "spgemm_timing_count", "spgemm_timing", "spgemm_free", "spgemm_status_string",
            "spgemm_selector_transpose_workspace", "spgemm_selector_transpose",
            "spgemm_mcl_prune_workspace", "spgemm_mcl_prune_count", "spgemm_mcl_prune_write",
            "spgemm_estimate", "spgemm_noalloc_scratch_bytes", "spgemm_multiply_noalloc",
            "spgemm_mcl_change", "spgemm_components_workspace", "spgemm_components",
            "spgemm_topk_rows", "spgemm_csr_to_dense", "spgemm_gemm_f32", "spgemm_masked_spmm",
            "spgemm_transpose_workspace", "spgemm_transpose", "spgemm_its_sample",
            "spgemm_plan_create_device", "spgemm_execute_arena"]


class SpgemmError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)}")


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads the HIP library (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    # torch first: its HIP libraries ask for the runtime by its unversioned
    # name, so a runtime that this library pulled in earlier (by its
    # versioned name) would not be shared, and the second runtime of the
    # process finds no device.  Loaded after torch, the library binds to the
    # runtime torch already holds.
    _torch()
    lib = ctypes.CDLL(path)
    pp = ctypes.POINTER(_VP)
    lib.spgemm_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.spgemm_default_options.restype = None
    lib.spgemm_plan_create.argtypes = [pp, ctypes.POINTER(CsrDesc), ctypes.POINTER(CsrDesc),
                                       ctypes.POINTER(Options), _VP, ALLOC_FN, FREE_FN, _VP]
    lib.spgemm_plan_create_batch.argtypes = [pp, ctypes.c_int32, ctypes.POINTER(CsrDesc),
                                             ctypes.POINTER(CsrDesc), ctypes.POINTER(Options),
                                             _VP, ALLOC_FN, FREE_FN, _VP]
    lib.spgemm_symbolic.argtypes = [_VP, _VP, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]
    lib.spgemm_symbolic_batch.argtypes = [_VP, ctypes.POINTER(_VP), ctypes.POINTER(_I64)]
    lib.spgemm_numeric.argtypes = [_VP, _VP, _VP, _VP, _VP]
    lib.spgemm_numeric_batch.argtypes = [_VP, ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                                         ctypes.POINTER(_VP), ctypes.POINTER(_VP)]
    lib.spgemm_sync.argtypes = [_VP]
    lib.spgemm_estimate.argtypes = [ctypes.POINTER(CsrDesc), ctypes.POINTER(CsrDesc), _VP, _VP]
    lib.spgemm_noalloc_scratch_bytes.argtypes = []
    lib.spgemm_noalloc_scratch_bytes.restype = ctypes.c_size_t
    lib.spgemm_multiply_noalloc.argtypes = [ctypes.POINTER(CsrDesc), ctypes.POINTER(CsrDesc),
                                            ctypes.POINTER(Options), _VP, _VP, _VP, _VP, _I64,
                                            ctypes.POINTER(_I64)]
    lib.spgemm_get_info.argtypes = [_VP, ctypes.POINTER(Info)]
    lib.spgemm_export.argtypes = [_VP, ctypes.c_int32, _VP, ctypes.POINTER(_I64)]
    lib.spgemm_timing_count.argtypes = [_VP]
    lib.spgemm_timing_count.restype = ctypes.c_int32
    lib.spgemm_timing.argtypes = [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_char_p),
                                  ctypes.POINTER(ctypes.c_float)]
    lib.spgemm_timing.restype = ctypes.c_int
    lib.spgemm_free.argtypes = [_VP]
    lib.spgemm_free.restype = None
    lib.spgemm_status_string.argtypes = [ctypes.c_int]
    lib.spgemm_status_string.restype = ctypes.c_char_p
    lib.spgemm_selector_transpose_workspace.argtypes = [_I64]
    lib.spgemm_selector_transpose_workspace.restype = ctypes.c_size_t
    lib.spgemm_selector_transpose.argtypes = [_VP, _I64, _I64, _VP, _VP, _VP, _VP, _VP]
    lib.spgemm_mcl_prune_workspace.argtypes = [_I64]
    lib.spgemm_mcl_prune_workspace.restype = ctypes.c_size_t
    lib.spgemm_mcl_prune_count.argtypes = [_I64, _VP, _VP, ctypes.c_float, ctypes.c_float,
                                           ctypes.c_int32, _VP, _VP, ctypes.POINTER(_I64), _VP]
    lib.spgemm_mcl_prune_write.argtypes = [_I64, _VP, _VP, _VP, ctypes.c_float, ctypes.c_float,
                                           ctypes.c_int32, _VP, _VP, _VP, _VP, _VP]
    lib.spgemm_mcl_change.argtypes = [_I64, _VP, _VP, _VP, _VP, _VP, _VP, _I64, _I64, _VP, _VP]
    lib.spgemm_components_workspace.argtypes = []
    lib.spgemm_components_workspace.restype = ctypes.c_size_t
    lib.spgemm_components.argtypes = [_I64, _VP, _VP, _I64, _VP, _VP, _VP,
                                      ctypes.POINTER(ctypes.c_int32)]
    lib.spgemm_topk_rows.argtypes = [_I64, _I64, _VP, _I64, ctypes.c_int32, _VP, _VP, _VP, _VP]
    lib.spgemm_csr_to_dense.argtypes = [_I64, _I64, _VP, _VP, _VP, _VP, _I64, _VP]
    lib.spgemm_gemm_f32.argtypes = [_I64, _I64, _I64, _VP, _I64, _I64, _VP, _I64, _I64, _VP, _I64,
                                    _VP]
    lib.spgemm_masked_spmm.argtypes = [_I64, _VP, _VP, _VP, _VP, _I64, _VP, _VP, _VP, _VP]
    lib.spgemm_transpose_workspace.argtypes = [_I64]
    lib.spgemm_transpose_workspace.restype = ctypes.c_size_t
    lib.spgemm_transpose.argtypes = [_I64, _I64, _VP, _VP, _VP, _I64, _VP, _VP, _VP, _VP, _VP]
    lib.spgemm_its_sample.argtypes = [_I64, ctypes.c_int32, _VP, _VP, _VP, _VP, _VP, _VP, _VP]
    lib.spgemm_plan_create_device.argtypes = [pp, ctypes.c_int32, ctypes.POINTER(CsrDesc),
                                              ctypes.POINTER(CsrDesc), ctypes.POINTER(Options),
                                              _VP, ALLOC_FN, FREE_FN, _VP]
    lib.spgemm_execute_arena.argtypes = [_VP, ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                                         ctypes.POINTER(_VP), _VP, _VP, _VP, _I64]
    for name in ("spgemm_plan_create", "spgemm_plan_create_batch", "spgemm_symbolic",
                 "spgemm_symbolic_batch", "spgemm_numeric", "spgemm_numeric_batch",
                 "spgemm_sync", "spgemm_get_info", "spgemm_export", "spgemm_selector_transpose",
                 "spgemm_mcl_prune_count", "spgemm_mcl_prune_write", "spgemm_estimate",
                 "spgemm_multiply_noalloc", "spgemm_mcl_change", "spgemm_components"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(code: int, where: str):
    if code != 0:
        raise SpgemmError(code, where)


def default_options() -> Options:
    o = Options()
    load().spgemm_default_options(ctypes.byref(o))
    return o


def make_options(sym_upper=None, num_upper=None, chunk_cols=None, validate=None,
                 profile=None, chunks_per_item=None, chunk_wgs_per_cu=None,
                 chunk_threads=None, sym_chunk_threads=None, num_rank_cap=None,
                 chunk_merge=None, graph=None, item_limit=None, row_thread=None,
                 accumulate=None) -> Options:
    o = default_options()
    if sym_upper is not None:
        for g, v in enumerate(sym_upper):
            o.sym_upper[g] = int(v)
    if num_upper is not None:
        for g, v in enumerate(num_upper):
            o.num_upper[g] = int(v)
    if chunk_cols is not None:
        o.chunk_cols = int(chunk_cols)
    if validate is not None:
        o.validate = int(validate)
    if profile is not None:
        o.profile = int(profile)
    if chunks_per_item is not None:
        o.chunks_per_item = int(chunks_per_item)
    if chunk_wgs_per_cu is not None:
        o.chunk_wgs_per_cu = int(chunk_wgs_per_cu)
    if chunk_threads is not None:
        o.chunk_threads = int(chunk_threads)
    if sym_chunk_threads is not None:
        o.sym_chunk_threads = int(sym_chunk_threads)
    if num_rank_cap is not None:
        o.num_rank_cap = int(num_rank_cap)
    if chunk_merge is not None:
        o.chunk_merge = int(chunk_merge)
    if graph is not None:
        o.graph = int(graph)
    if item_limit is not None:
        o.item_limit = int(item_limit)
    if row_thread is not None:
        o.row_thread = int(row_thread)
    if accumulate is not None:
        o.accumulate = int(accumulate)
    return o


# ---------------------------------------------------------------------------
# torch glue
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


class _TorchAllocator:
    """Routes the library's workspace through PyTorch's caching allocator."""

    def __init__(self, device):
        torch = _torch()
        self.device = torch.device(device)

        def _alloc(ctx, nbytes, stream):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), self.device.index,
                                                          stream or None)
            except Exception:
                return None

        delete = torch.cuda.caching_allocator_delete

        def _free(ctx, ptr, stream):
            try:
                delete(ptr)
            except (AttributeError, TypeError):
                pass  # interpreter shutdown: torch's modules are gone already

        self.alloc = ALLOC_FN(_alloc)
        self.free = FREE_FN(_free)


@dataclasses.dataclass
class DeviceCsr:
    """CSR matrix resident on the GPU (torch tensors)."""

    nrows: int
    ncols: int
    rpt: "object"   # torch.int64 [nrows + 1]
    col: "object"   # torch.int32 [nnz]
    val: "object"   # torch.float32 [nnz]
    sorted_rows: bool = True

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    def desc(self, with_values: bool = True) -> CsrDesc:
        return CsrDesc(self.nrows, self.ncols, self.nnz, self.rpt.data_ptr(),
                       self.col.data_ptr() if self.nnz else None,
                       self.val.data_ptr() if (with_values and self.nnz) else None,
                       ROWS_SORTED if self.sorted_rows else 0)

    def to_host(self):
        from . import gen
        return gen.Csr(self.nrows, self.ncols, self.rpt.cpu().numpy(), self.col.cpu().numpy(),
                       self.val.cpu().numpy())


def to_device(m, device="cuda", sorted_rows: bool | None = None) -> DeviceCsr:
    """Host gen.Csr -> DeviceCsr.  Row sortedness is checked on the host
    unless given."""
    torch = _torch()
    if sorted_rows is None:
        sorted_rows = _rows_sorted(m)
    return DeviceCsr(m.nrows, m.ncols,
                     torch.from_numpy(np.ascontiguousarray(m.rpt, dtype=np.int64)).to(device),
                     torch.from_numpy(np.ascontiguousarray(m.col, dtype=np.int32)).to(device),
                     torch.from_numpy(np.ascontiguousarray(m.val, dtype=np.float32)).to(device),
                     bool(sorted_rows))


def _rows_sorted(m) -> bool:
    if m.nnz < 2:
        return True
    d = np.diff(m.col.astype(np.int64))
    inner = np.ones(m.nnz - 1, dtype=bool)
    ends = m.rpt[1:-1]
    ends = ends[(ends > 0) & (ends < m.nnz)]
    inner[ends - 1] = False
    return bool(np.all(d[inner] > 0))


class Plan:
    """One plan (single product or batch) on the current torch stream."""

    def __init__(self, As, Bs, options: Options | None = None, stream=None,
                 use_torch_allocator: bool = True):
        torch = _torch()
        lib = load()
        self._lib = lib
        self.batch = isinstance(As, (list, tuple))
        self.As = list(As) if self.batch else [As]
        self.Bs = list(Bs) if self.batch else [Bs]
        if len(self.As) != len(self.Bs) or not self.As:
            raise ValueError("need equally many A and B")
        dev = self.As[0].rpt.device
        self.device = dev
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self._alloc = _TorchAllocator(dev) if use_torch_allocator else None
        self._handle = _VP()
        n = len(self.As)
        da = (CsrDesc * n)(*[a.desc(False) for a in self.As])
        db = (CsrDesc * n)(*[b.desc(False) for b in self.Bs])
        opt = options if options is not None else default_options()
        afn = self._alloc.alloc if self._alloc else ALLOC_FN()
        ffn = self._alloc.free if self._alloc else FREE_FN()
        sh = _VP(self.stream.cuda_stream)
        if self.batch:
            code = lib.spgemm_plan_create_batch(ctypes.byref(self._handle), n, da, db,
                                                ctypes.byref(opt), sh, afn, ffn, None)
        else:
            code = lib.spgemm_plan_create(ctypes.byref(self._handle), da, db, ctypes.byref(opt),
                                          sh, afn, ffn, None)
        _check(code, "spgemm_plan_create")
        self.nnz = None
        self.rpts = None

    # -- phases ------------------------------------------------------------
    def symbolic(self):
        torch = _torch()
        lib = self._lib
        if not self.batch:
            rpt = torch.empty(self.As[0].nrows + 1, dtype=torch.int64, device=self.device)
            nnz = _I64()
            flops = _I64()
            _check(lib.spgemm_symbolic(self._handle, _VP(rpt.data_ptr()), ctypes.byref(nnz),
                                       ctypes.byref(flops)), "spgemm_symbolic")
            self.rpts = [rpt]
            self.nnz = [int(nnz.value)]
        else:
            n = len(self.As)
            self.rpts = [torch.empty(a.nrows + 1, dtype=torch.int64, device=self.device)
                         for a in self.As]
            ptrs = (_VP * n)(*[r.data_ptr() for r in self.rpts])
            nnz = (_I64 * n)()
            _check(lib.spgemm_symbolic_batch(self._handle, ptrs, nnz), "spgemm_symbolic_batch")
            self.nnz = [int(x) for x in nnz]
        return self.nnz

    def allocate_outputs(self):
        torch = _torch()
        cols = [torch.empty(max(k, 1), dtype=torch.int32, device=self.device) for k in self.nnz]
        vals = [torch.empty(max(k, 1), dtype=torch.float32, device=self.device) for k in self.nnz]
        return cols, vals

    def numeric(self, cols, vals, a_vals=None, b_vals=None):
        lib = self._lib
        a_vals = a_vals if a_vals is not None else [a.val for a in self.As]
        b_vals = b_vals if b_vals is not None else [b.val for b in self.Bs]
        if not self.batch:
            _check(lib.spgemm_numeric(self._handle, _VP(a_vals[0].data_ptr()),
                                      _VP(b_vals[0].data_ptr()), _VP(cols[0].data_ptr()),
                                      _VP(vals[0].data_ptr())), "spgemm_numeric")
        else:
            n = len(self.As)
            _check(lib.spgemm_numeric_batch(
                self._handle, (_VP * n)(*[t.data_ptr() for t in a_vals]),
                (_VP * n)(*[t.data_ptr() for t in b_vals]),
                (_VP * n)(*[t.data_ptr() for t in cols]),
                (_VP * n)(*[t.data_ptr() for t in vals])), "spgemm_numeric_batch")

    def sync(self):
        _check(self._lib.spgemm_sync(self._handle), "spgemm_sync")

    def info(self) -> Info:
        inf = Info()
        _check(self._lib.spgemm_get_info(self._handle, ctypes.byref(inf)), "spgemm_get_info")
        return inf

    def export(self, what: int):
        torch = _torch()
        total = sum(a.nrows for a in self.As)
        dst = torch.empty(max(total, 1), dtype=torch.int64, device=self.device)
        gs = (_I64 * (NGROUPS + 1))()
        _check(self._lib.spgemm_export(self._handle, what, _VP(dst.data_ptr()), gs),
               "spgemm_export")
        return dst[:total], [int(x) for x in gs]

    def timings(self) -> list[tuple[str, float]]:
        """(name, ms) of every profiled launch group (options.profile = 1)."""
        lib = self._lib
        out = []
        for k in range(lib.spgemm_timing_count(self._handle)):
            name = ctypes.c_char_p()
            ms = ctypes.c_float()
            _check(lib.spgemm_timing(self._handle, k, ctypes.byref(name), ctypes.byref(ms)),
                   "spgemm_timing")
            out.append((name.value.decode(), float(ms.value)))
        return out

    def free(self):
        if self._handle:
            self._lib.spgemm_free(self._handle)
            self._handle = _VP()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def results(self, cols, vals):
        out = []
        for q in range(len(self.As)):
            k = self.nnz[q]
            out.append(DeviceCsr(self.As[q].nrows, self.Bs[q].ncols, self.rpts[q],
                                 cols[q][:k], vals[q][:k], True))
        return out


def matmul(A: DeviceCsr, B: DeviceCsr, options: Options | None = None, stream=None) -> DeviceCsr:
    """C = A * B on the GPU (plan, symbolic, allocate, numeric, free)."""
    plan = Plan(A, B, options, stream)
    try:
        plan.symbolic()
        cols, vals = plan.allocate_outputs()
        plan.numeric(cols, vals)
        plan.sync()  # surfaces a kernel-raised error flag
        return plan.results(cols, vals)[0]
    finally:
        plan.free()


def matmul_batch(As, Bs, options: Options | None = None, stream=None):
    """C_p = A_p * B_p for every p in one batched plan."""
    plan = Plan(list(As), list(Bs), options, stream)
    try:
        plan.symbolic()
        cols, vals = plan.allocate_outputs()
        plan.numeric(cols, vals)
        plan.sync()
        return plan.results(cols, vals)
    finally:
        plan.free()


def estimate_async(A: DeviceCsr, B: DeviceCsr, out, stream=None):
    """Enqueues Algorithm 1 alone for C = A * B: out (device int64[3]) gets
    [sum of intermediate products, sum over rows of min(ip, B.ncols), largest
    row].  Needs only A's structure and B's row pointers (B.col may be
    empty); no synchronisation."""
    torch = _torch()
    st = stream if stream is not None else torch.cuda.current_stream(out.device)
    da = A.desc(False)
    db = CsrDesc(B.nrows, B.ncols, B.nnz, B.rpt.data_ptr(), None, None, 0)
    _check(load().spgemm_estimate(ctypes.byref(da), ctypes.byref(db), _VP(out.data_ptr()),
                                  _VP(st.cuda_stream)), "spgemm_estimate")


def multiply_noalloc(A: DeviceCsr, B: DeviceCsr, c_rpt, c_col, c_val,
                     options: Options | None = None, stream=None):
    """spgemm_multiply_noalloc into caller tensors (c_rpt int64 [A.nrows + 1],
    c_col int32 / c_val float32 of equal capacity).  Returns (status code,
    nnz(C) or -1); does not raise on ENOMEM so that callers can retry."""
    torch = _torch()
    st = stream if stream is not None else torch.cuda.current_stream(c_rpt.device)
    nnz = _I64(-1)
    cap = int(c_col.numel())
    code = load().spgemm_multiply_noalloc(
        ctypes.byref(A.desc()), ctypes.byref(B.desc()),
        ctypes.byref(options) if options is not None else None, _VP(st.cuda_stream),
        _VP(c_rpt.data_ptr()), _VP(c_col.data_ptr()) if cap else None,
        _VP(c_val.data_ptr()) if cap else None, cap, ctypes.byref(nnz))
    return int(code), int(nnz.value)


def _ptr(t):
    return _VP(t.data_ptr()) if t is not None and t.numel() else None


def selector_transpose(labels, k: int, stream=None) -> DeviceCsr:
    """S^T (k x n) of the selector S[v, labels[v]] = 1, built on the device
    (graph contraction, paper Algorithm 7).  labels: int32 device tensor."""
    torch = _torch()
    lib = load()
    dev = labels.device
    n = int(labels.numel())
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    rpt = torch.empty(k + 1, dtype=torch.int64, device=dev)
    col = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    val = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
    ws = torch.empty(int(lib.spgemm_selector_transpose_workspace(k)), dtype=torch.uint8,
                     device=dev)
    _check(lib.spgemm_selector_transpose(_ptr(labels), n, k, _VP(rpt.data_ptr()),
                                         _VP(col.data_ptr()), _VP(val.data_ptr()),
                                         _VP(ws.data_ptr()), _VP(st.cuda_stream)),
           "spgemm_selector_transpose")
    return DeviceCsr(k, n, rpt, col[:n], val[:n], False)


def mcl_prune(E: DeviceCsr, power: float = 2.0, theta: float = 1e-4, k: int = 0,
              stream=None) -> DeviceCsr:
    """Markov-clustering step after an expansion, on row-stochastic storage:
    x -> x^power, row-normalise, drop entries below theta, keep the k largest
    (k = 0: all), row-normalise."""
    torch = _torch()
    lib = load()
    dev = E.rpt.device
    m = E.nrows
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    ws = torch.empty(max(int(lib.spgemm_mcl_prune_workspace(m)), 1), dtype=torch.uint8,
                     device=dev)
    rpt = torch.empty(m + 1, dtype=torch.int64, device=dev)
    nnz = _I64()
    _check(lib.spgemm_mcl_prune_count(m, _VP(E.rpt.data_ptr()), _ptr(E.val), float(power),
                                      float(theta), int(k), _VP(rpt.data_ptr()),
                                      _VP(ws.data_ptr()), ctypes.byref(nnz),
                                      _VP(st.cuda_stream)), "spgemm_mcl_prune_count")
    n = int(nnz.value)
    col = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    val = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
    _check(lib.spgemm_mcl_prune_write(m, _VP(E.rpt.data_ptr()), _ptr(E.col), _ptr(E.val),
                                      float(power), float(theta), int(k), _VP(rpt.data_ptr()),
                                      _VP(ws.data_ptr()), _VP(col.data_ptr()),
                                      _VP(val.data_ptr()), _VP(st.cuda_stream)),
           "spgemm_mcl_prune_write")
    return DeviceCsr(m, E.ncols, rpt, col[:n], val[:n], E.sorted_rows)


def mcl_change_async(A: DeviceCsr, B: DeviceCsr, out, stream=None):
    """Enqueues the largest |a_ij - b_ij| over both patterns into out (device
    float64 tensor of one element)."""
    torch = _torch()
    st = stream if stream is not None else torch.cuda.current_stream(out.device)
    _check(load().spgemm_mcl_change(A.nrows, _VP(A.rpt.data_ptr()), _ptr(A.col), _ptr(A.val),
                                    _VP(B.rpt.data_ptr()), _ptr(B.col), _ptr(B.val), A.nnz,
                                    B.nnz, _VP(out.data_ptr()), _VP(st.cuda_stream)),
           "spgemm_mcl_change")


def mcl_change(A: DeviceCsr, B: DeviceCsr) -> float:
    torch = _torch()
    out = torch.empty(1, dtype=torch.float64, device=A.rpt.device)
    mcl_change_async(A, B, out)
    return float(out.item())


def components(M: DeviceCsr, stream=None):
    """Connected components of the undirected graph of M's pattern (square):
    (labels int32 device tensor, each the smallest vertex of its component;
    rounds)."""
    torch = _torch()
    lib = load()
    dev = M.rpt.device
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    lab = torch.empty(max(M.nrows, 1), dtype=torch.int32, device=dev)
    ws = torch.empty(int(lib.spgemm_components_workspace()), dtype=torch.uint8, device=dev)
    rounds = ctypes.c_int32()
    _check(lib.spgemm_components(M.nrows, _VP(M.rpt.data_ptr()), _ptr(M.col), M.nnz,
                                 _VP(lab.data_ptr()), _VP(ws.data_ptr()), _VP(st.cuda_stream),
                                 ctypes.byref(rounds)), "spgemm_components")
    return lab[:M.nrows], int(rounds.value)


# ---------------------------------------------------------------------------
# GNN layer pieces (paper Section V-C)
# ---------------------------------------------------------------------------
def _st(dev, stream):
    torch = _torch()
    return _VP((stream if stream is not None else torch.cuda.current_stream(dev)).cuda_stream)


def topk_rows(x, k: int, stream=None) -> DeviceCsr:
    """TopK(X, k) per row of a dense row-major float32 device tensor, as CSR
    with ascending columns (its pattern is the mask M_k)."""
    torch = _torch()
    n, f = x.shape
    kk = min(int(k), f)
    dev = x.device
    rpt = torch.empty(n + 1, dtype=torch.int64, device=dev)
    col = torch.empty(max(n * kk, 1), dtype=torch.int32, device=dev)
    val = torch.empty(max(n * kk, 1), dtype=torch.float32, device=dev)
    _check(load().spgemm_topk_rows(n, f, _VP(x.data_ptr()) if x.numel() else None, x.stride(0),
                                   int(k), _VP(rpt.data_ptr()), _VP(col.data_ptr()),
                                   _VP(val.data_ptr()), _st(dev, stream)), "spgemm_topk_rows")
    return DeviceCsr(n, f, rpt, col[:n * kk], val[:n * kk], True)


def to_dense(m: DeviceCsr, stream=None):
    torch = _torch()
    d = torch.empty((m.nrows, m.ncols), dtype=torch.float32, device=m.rpt.device)
    _check(load().spgemm_csr_to_dense(m.nrows, m.ncols, _VP(m.rpt.data_ptr()), _ptr(m.col),
                                      _ptr(m.val), _VP(d.data_ptr()) if d.numel() else None,
                                      max(m.ncols, 0), _st(m.rpt.device, stream)),
           "spgemm_csr_to_dense")
    return d


def gemm(a, b, stream=None):
    """a @ b for 2-D float32 device tensors (any strides, e.g. transposed
    views) on the matrix cores; returns a new row-major tensor."""
    torch = _torch()
    M, K = a.shape
    K2, N = b.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    c = torch.empty((M, N), dtype=torch.float32, device=a.device)
    _check(load().spgemm_gemm_f32(M, N, K, _VP(a.data_ptr()) if a.numel() else None,
                                  a.stride(0), a.stride(1),
                                  _VP(b.data_ptr()) if b.numel() else None, b.stride(0),
                                  b.stride(1), _VP(c.data_ptr()) if c.numel() else None, N,
                                  _st(a.device, stream)), "spgemm_gemm_f32")
    return c


def masked_spmm(at: DeviceCsr, d, mask: DeviceCsr, stream=None):
    """Values, on mask's pattern, of (A^T d) given at = A^T (CSR) and the
    dense row-major d."""
    torch = _torch()
    out = torch.empty(max(mask.nnz, 1), dtype=torch.float32, device=d.device)
    _check(load().spgemm_masked_spmm(at.nrows, _VP(at.rpt.data_ptr()), _ptr(at.col),
                                     _ptr(at.val), _VP(d.data_ptr()) if d.numel() else None,
                                     d.stride(0), _VP(mask.rpt.data_ptr()), _ptr(mask.col),
                                     _VP(out.data_ptr()), _st(d.device, stream)),
           "spgemm_masked_spmm")
    return out[:mask.nnz]


def transpose(m: DeviceCsr, stream=None) -> DeviceCsr:
    """CSR transpose on the device (rows of the result not column-sorted)."""
    torch = _torch()
    lib = load()
    dev = m.rpt.device
    rpt = torch.empty(m.ncols + 1, dtype=torch.int64, device=dev)
    col = torch.empty(max(m.nnz, 1), dtype=torch.int32, device=dev)
    val = torch.empty(max(m.nnz, 1), dtype=torch.float32, device=dev)
    ws = torch.empty(int(lib.spgemm_transpose_workspace(m.ncols)), dtype=torch.uint8, device=dev)
    _check(lib.spgemm_transpose(m.nrows, m.ncols, _VP(m.rpt.data_ptr()), _ptr(m.col),
                                _ptr(m.val), m.nnz, _VP(rpt.data_ptr()), _VP(col.data_ptr()),
                                _VP(val.data_ptr()), _VP(ws.data_ptr()), _st(dev, stream)),
           "spgemm_transpose")
    return DeviceCsr(m.ncols, m.nrows, rpt, col[:m.nnz], val[:m.nnz], False)


def its_sample(p: DeviceCsr, s: int, u, self_v, stream=None):
    """s inverse-transform draws per row of p (weights); u: float32 device
    tensor of p.nrows * s uniforms in [0, 1); self_v: int32 device tensor of
    each row's own vertex (drawn when the row has no weight).  Returns the
    drawn columns, int32 [p.nrows * s]."""
    torch = _torch()
    out = torch.empty(max(p.nrows * s, 1), dtype=torch.int32, device=p.rpt.device)
    _check(load().spgemm_its_sample(p.nrows, int(s), _VP(p.rpt.data_ptr()), _ptr(p.col),
                                    _ptr(p.val), _ptr(u), _ptr(self_v), _VP(out.data_ptr()),
                                    _st(p.rpt.device, stream)), "spgemm_its_sample")
    return out[:p.nrows * s]


class DevicePlan:
    """A device-driven batch plan (spgemm_plan_create_device): the whole
    product runs with no host synchronisation, C in one arena."""

    def __init__(self, As, Bs, options: Options | None = None, stream=None):
        torch = _torch()
        lib = load()
        self._lib = lib
        self.As, self.Bs = list(As), list(Bs)
        dev = self.As[0].rpt.device
        self.device = dev
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self._alloc = _TorchAllocator(dev)
        self._handle = _VP()
        n = len(self.As)
        da = (CsrDesc * n)(*[a.desc(False) for a in self.As])
        db = (CsrDesc * n)(*[b.desc(False) for b in self.Bs])
        opt = options if options is not None else default_options()
        _check(lib.spgemm_plan_create_device(ctypes.byref(self._handle), n, da, db,
                                             ctypes.byref(opt), _VP(self.stream.cuda_stream),
                                             self._alloc.alloc, self._alloc.free, None),
               "spgemm_plan_create_device")

    def execute(self, rpts, offsets, col, val, a_vals=None, b_vals=None):
        """Enqueues the whole product into caller tensors: rpts (one int64
        tensor of A_p.nrows + 1 per product), offsets (int64, nprod + 1),
        the arena col (int32) / val (float32) of equal capacity."""
        n = len(self.As)
        a_vals = a_vals if a_vals is not None else [a.val for a in self.As]
        b_vals = b_vals if b_vals is not None else [b.val for b in self.Bs]
        cap = int(col.numel())
        _check(self._lib.spgemm_execute_arena(
            self._handle, (_VP * n)(*[t.data_ptr() for t in a_vals]),
            (_VP * n)(*[t.data_ptr() for t in b_vals]),
            (_VP * n)(*[r.data_ptr() for r in rpts]), _VP(offsets.data_ptr()),
            _VP(col.data_ptr()) if cap else None, _VP(val.data_ptr()) if cap else None, cap),
            "spgemm_execute_arena")

    def sync(self):
        _check(self._lib.spgemm_sync(self._handle), "spgemm_sync")

    def info(self) -> Info:
        return Plan.info(self)

    def timings(self):
        return Plan.timings(self)

    def free(self):
        if self._handle:
            self._lib.spgemm_free(self._handle)
            self._handle = _VP()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
