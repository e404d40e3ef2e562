"""EBBkC k-clique counting and listing on MI355X (gfx950) -- Python binding of libebbkc.

Argument marshalling only: every step of the computation runs in the HIP kernels of
``libebbkc.so`` (sources in ``csrc/``).  The functions below carry the names of the C entry points
declared in ``include/ebbkc.h``; :class:`Graph` is a small convenience wrapper over a handle.
PyTorch is used only for device memory and the current stream.  There is no CPU fallback: if the
library is missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libebbkc.so")

OK, E_INVALID_ARG, E_BAD_CSR, E_OOM, E_K_RANGE, E_BUFFER_TOO_SMALL, E_OVERFLOW, E_WIDTH, E_HIP, E_CANCELLED = (
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9)
E_SCRATCH = -10
NOALLOC_SCRATCH_BYTES = 256 << 20  # the fixed scratch of ebbkc_count_noalloc
PTR_HOST, PTR_DEVICE = 0, 1
LIST_SORTED = 1
ARR_SUPPORT, ARR_RANK, ARR_LEVEL, ARR_SUBSIZE, ARR_VERTEX_POS, ARR_VERTEX_COLOR = 0, 1, 2, 3, 4, 5
ORDER_HYBRID, ORDER_COLOR, ORDER_DEGEN_VERTEX, ORDER_TRUSS, ORDER_DEGEN_VERTEX_NP = 0, 1, 2, 3, 4
BATCH_AUTO, BATCH_ARENA, BATCH_BUILD = 0, 1, 2


class EbbkcError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str = ""):
        super().__init__(f"{what}: {detail} (status {status})")
        self.status = status


class ebbkc_options(ctypes.Structure):
    _fields_ = [("early_termination", ctypes.c_int32), ("t_plex", ctypes.c_int32), ("rule1", ctypes.c_int32),
                ("rule2", ctypes.c_int32), ("waves_per_block", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("split_threshold", ctypes.c_int32), ("count_work", ctypes.c_int32),
                ("dense_k4", ctypes.c_int32), ("ordering", ctypes.c_int32), ("batch_build", ctypes.c_int32),
                ("node_split", ctypes.c_int32), ("adj_max_n", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class ebbkc_result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("graph", ctypes.c_int32), ("k", ctypes.c_int32), ("status", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("count", ctypes.c_uint64), ("arrival_ms", ctypes.c_double),
                ("admit_ms", ctypes.c_double), ("done_ms", ctypes.c_double)]


class ebbkc_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64), ("tau", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("max_degree", ctypes.c_int32), ("device_bytes", ctypes.c_int64), ("prepare_ms", ctypes.c_double)]


EXPORTED = ("ebbkc_default_options", "ebbkc_prepare", "ebbkc_count", "ebbkc_count_noalloc", "ebbkc_count128", "ebbkc_max_clique_size",
            "ebbkc_count_range", "ebbkc_count_seeds",
            "ebbkc_list", "ebbkc_export", "ebbkc_info_get", "ebbkc_last_timing", "ebbkc_last_work",
            "ebbkc_last_work_class", "ebbkc_destroy", "ebbkc_strerror", "ebbkc_batch_create", "ebbkc_batch_run", "ebbkc_batch_tune", "ebbkc_batch_info",
            "ebbkc_batch_destroy", "ebbkc_server_create", "ebbkc_server_submit", "ebbkc_server_cancel", "ebbkc_server_poll",
            "ebbkc_server_stats", "ebbkc_server_destroy")

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libebbkc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2311_13798_amd/build.py (no CPU fallback exists)")
    lib = ctypes.CDLL(path)
    vp, i32, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    pu64 = ctypes.POINTER(ctypes.c_uint64)
    lib.ebbkc_default_options.argtypes = [ctypes.POINTER(ebbkc_options)]
    lib.ebbkc_default_options.restype = None
    lib.ebbkc_prepare.argtypes = [vp, vp, i32, i64, i32, ctypes.POINTER(ebbkc_options), vp, ctypes.POINTER(vp)]
    lib.ebbkc_count.argtypes = [vp, i32, pu64, vp]
    lib.ebbkc_count_noalloc.argtypes = [vp, i32, pu64, vp]
    lib.ebbkc_count_range.argtypes = [vp, i32, i64, i64, pu64, vp]
    lib.ebbkc_count128.argtypes = [vp, i32, pu64, vp]
    lib.ebbkc_max_clique_size.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), vp]
    lib.ebbkc_count_seeds.argtypes = [vp, i32, vp, i64, i32, vp, vp]
    lib.ebbkc_list.argtypes = [vp, i32, i64, i64, vp, u64, u32, pu64, vp, vp]
    lib.ebbkc_export.argtypes = [vp, i32, vp, i32, vp]
    lib.ebbkc_info_get.argtypes = [vp, ctypes.POINTER(ebbkc_info)]
    lib.ebbkc_last_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.ebbkc_last_work.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
    lib.ebbkc_last_work_class.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_uint64)]
    lib.ebbkc_destroy.argtypes = [vp]
    lib.ebbkc_destroy.restype = None
    lib.ebbkc_batch_create.argtypes = [vp, vp, i32, ctypes.POINTER(ebbkc_options), vp, ctypes.POINTER(vp)]
    lib.ebbkc_batch_run.argtypes = [vp, i32, vp, vp]
    lib.ebbkc_batch_tune.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)]
    lib.ebbkc_batch_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
    lib.ebbkc_batch_destroy.argtypes = [vp]
    lib.ebbkc_batch_destroy.restype = None
    for f in ("ebbkc_batch_create", "ebbkc_batch_run", "ebbkc_batch_tune", "ebbkc_batch_info"):
        getattr(lib, f).restype = ctypes.c_int
    lib.ebbkc_server_create.argtypes = [vp, i32, ctypes.POINTER(ebbkc_options), i64, ctypes.POINTER(vp)]
    lib.ebbkc_server_submit.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_int64)]
    lib.ebbkc_server_cancel.argtypes = [vp, i64]
    lib.ebbkc_server_poll.argtypes = [vp, ctypes.POINTER(ebbkc_result), i32, i32, ctypes.POINTER(ctypes.c_int32)]
    lib.ebbkc_server_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.ebbkc_server_destroy.argtypes = [vp]
    lib.ebbkc_server_destroy.restype = None
    for f in ("ebbkc_server_create", "ebbkc_server_submit", "ebbkc_server_cancel", "ebbkc_server_poll",
              "ebbkc_server_stats"):
        getattr(lib, f).restype = ctypes.c_int
    lib.ebbkc_strerror.argtypes = [i32]
    lib.ebbkc_strerror.restype = ctypes.c_char_p
    for f in ("ebbkc_prepare", "ebbkc_count", "ebbkc_count_noalloc", "ebbkc_count_range", "ebbkc_count128", "ebbkc_max_clique_size", "ebbkc_count_seeds", "ebbkc_list",
              "ebbkc_export", "ebbkc_info_get", "ebbkc_last_timing", "ebbkc_last_work", "ebbkc_last_work_class"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(st: int, what: str):
    if st != OK:
        raise EbbkcError(st, what, load_library().ebbkc_strerror(st).decode())


def _stream(stream=None):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:  # pragma: no cover
        pass
    return ctypes.c_void_p(0)


def _ptr(a):
    """(pointer, kind) of a numpy array or torch tensor."""
    if isinstance(a, np.ndarray):
        return ctypes.c_void_p(a.ctypes.data), PTR_HOST
    import torch
    if isinstance(a, torch.Tensor):
        return ctypes.c_void_p(a.data_ptr()), (PTR_DEVICE if a.is_cuda else PTR_HOST)
    raise TypeError(f"unsupported array type {type(a)}")


# ---------------------------------------------------------------- C entry points

def ebbkc_default_options() -> ebbkc_options:
    o = ebbkc_options()
    load_library().ebbkc_default_options(ctypes.byref(o))
    return o


def ebbkc_prepare(row_ptr, col_idx, n: int, nnz: int, options: ebbkc_options | None = None, stream=None):
    rp, kind = _ptr(row_ptr)
    ci, kind2 = _ptr(col_idx)
    if kind != kind2:
        raise ValueError("row_ptr and col_idx must both be host or both be device arrays")
    h = ctypes.c_void_p()
    st = load_library().ebbkc_prepare(rp, ci, n, nnz, kind, ctypes.byref(options) if options else None,
                                      _stream(stream), ctypes.byref(h))
    _check(st, "ebbkc_prepare")
    return h


def ebbkc_count(h, k: int, stream=None) -> int:
    out = ctypes.c_uint64()
    _check(load_library().ebbkc_count(h, k, ctypes.byref(out), _stream(stream)), "ebbkc_count")
    return int(out.value)


def ebbkc_count_noalloc(h, k: int, stream=None) -> int:
    out = ctypes.c_uint64()
    _check(load_library().ebbkc_count_noalloc(h, k, ctypes.byref(out), _stream(stream)), "ebbkc_count_noalloc")
    return int(out.value)


def ebbkc_count128(h, k: int, stream=None) -> int:
    out = (ctypes.c_uint64 * 2)()
    _check(load_library().ebbkc_count128(h, k, out, _stream(stream)), "ebbkc_count128")
    return int(out[0]) | (int(out[1]) << 64)


def ebbkc_max_clique_size(h, stream=None) -> int:
    out = ctypes.c_int32()
    _check(load_library().ebbkc_max_clique_size(h, ctypes.byref(out), _stream(stream)), "ebbkc_max_clique_size")
    return int(out.value)


def ebbkc_count_range(h, k: int, r_begin: int, r_end: int, stream=None) -> int:
    out = ctypes.c_uint64()
    _check(load_library().ebbkc_count_range(h, k, r_begin, r_end, ctypes.byref(out), _stream(stream)),
           "ebbkc_count_range")
    return int(out.value)


def ebbkc_count_seeds(h, k: int, eids, out, stream=None):
    pe, kind = _ptr(eids)
    po, _ = _ptr(out)
    _check(load_library().ebbkc_count_seeds(h, k, pe, len(eids), kind, po, _stream(stream)), "ebbkc_count_seeds")
    return out


def ebbkc_list(h, k: int, buf, cap: int, flags: int = LIST_SORTED, r_begin: int = 0, r_end: int = -1,
               stream=None):
    """Returns (written, ordered_checksum, unordered_checksum)."""
    pb, kind = _ptr(buf)
    if kind != PTR_DEVICE:
        raise ValueError("the listing buffer must be device memory")
    w = ctypes.c_uint64()
    cs = (ctypes.c_uint64 * 2)()
    st = load_library().ebbkc_list(h, k, r_begin, r_end, pb, cap, flags, ctypes.byref(w), cs, _stream(stream))
    if st == E_BUFFER_TOO_SMALL:
        raise EbbkcError(st, "ebbkc_list", f"buffer too small: {int(w.value)} tuples needed")
    _check(st, "ebbkc_list")
    return int(w.value), int(cs[0]), int(cs[1])


def ebbkc_export(h, which: int, dst, stream=None):
    pd, kind = _ptr(dst)
    _check(load_library().ebbkc_export(h, which, pd, kind, _stream(stream)), "ebbkc_export")
    return dst


def ebbkc_info_get(h) -> ebbkc_info:
    info = ebbkc_info()
    _check(load_library().ebbkc_info_get(h, ctypes.byref(info)), "ebbkc_info_get")
    return info


def ebbkc_last_timing(h):
    out = (ctypes.c_double * 4)()
    _check(load_library().ebbkc_last_timing(h, out), "ebbkc_last_timing")
    return list(out)


def ebbkc_last_work(h):
    out = (ctypes.c_uint64 * 4)()
    _check(load_library().ebbkc_last_work(h, out), "ebbkc_last_work")
    return [int(x) for x in out]


def ebbkc_last_work_class(h, width_class: int):
    out = (ctypes.c_uint64 * 4)()
    _check(load_library().ebbkc_last_work_class(h, width_class, out), "ebbkc_last_work_class")
    return [int(x) for x in out]


def ebbkc_destroy(h):
    load_library().ebbkc_destroy(h)


def ebbkc_strerror(status: int) -> str:
    return load_library().ebbkc_strerror(status).decode()


def ebbkc_batch_create(handles, ks, options: ebbkc_options | None = None, stream=None):
    n = len(handles)
    arr = (ctypes.c_void_p * n)(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in handles])
    kk = (ctypes.c_int32 * n)(*ks)
    b = ctypes.c_void_p()
    _check(load_library().ebbkc_batch_create(arr, kk, n, ctypes.byref(options) if options else None, _stream(stream),
                                             ctypes.byref(b)), "ebbkc_batch_create")
    return b


def ebbkc_batch_run(b, use_graph: bool = True, stream=None):
    n = _batch_sizes.get(b.value, 0)
    out = (ctypes.c_uint64 * max(n, 1))()
    _check(load_library().ebbkc_batch_run(b, int(use_graph), out, _stream(stream)), "ebbkc_batch_run")
    return [int(x) for x in out[:n]]


def ebbkc_batch_tune(b, stream=None):
    sp, bp, ns = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load_library().ebbkc_batch_tune(b, _stream(stream), ctypes.byref(sp), ctypes.byref(bp), ctypes.byref(ns)),
           "ebbkc_batch_tune")
    return int(sp.value), int(bp.value), int(ns.value)


def ebbkc_batch_info(b):
    t, ms = ctypes.c_int64(), ctypes.c_double()
    _check(load_library().ebbkc_batch_info(b, ctypes.byref(t), ctypes.byref(ms)), "ebbkc_batch_info")
    return int(t.value), float(ms.value)


def ebbkc_batch_destroy(b):
    _batch_sizes.pop(b.value, None)
    load_library().ebbkc_batch_destroy(b)


_batch_sizes: dict = {}


class Batch:
    """Several (prepared graph, k) counts run as one fused launch per width class."""

    def __init__(self, graphs, ks, options: ebbkc_options | None = None):
        self._graphs = list(graphs)  # keep the handles alive
        self._b = ebbkc_batch_create([G.handle for G in self._graphs], list(ks), options)
        _batch_sizes[self._b.value] = len(self._graphs)

    def run(self, use_graph: bool = True):
        return ebbkc_batch_run(self._b, use_graph)

    def tune(self):
        return ebbkc_batch_tune(self._b)

    def info(self):
        return ebbkc_batch_info(self._b)

    def close(self):
        if getattr(self, "_b", None):
            ebbkc_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ebbkc_server_create(handles, budget_bytes: int, options: ebbkc_options | None = None):
    n = len(handles)
    arr = (ctypes.c_void_p * n)(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in handles])
    s = ctypes.c_void_p()
    _check(load_library().ebbkc_server_create(arr, n, ctypes.byref(options) if options else None, int(budget_bytes),
                                              ctypes.byref(s)), "ebbkc_server_create")
    return s


def ebbkc_server_submit(s, graph: int, k: int) -> int:
    rid = ctypes.c_int64()
    _check(load_library().ebbkc_server_submit(s, graph, k, ctypes.byref(rid)), "ebbkc_server_submit")
    return int(rid.value)


def ebbkc_server_cancel(s, rid: int):
    _check(load_library().ebbkc_server_cancel(s, rid), "ebbkc_server_cancel")


def ebbkc_server_poll(s, max_results: int = 4096, wait: bool = False):
    buf = (ebbkc_result * max_results)()
    n = ctypes.c_int32()
    _check(load_library().ebbkc_server_poll(s, buf, max_results, int(wait), ctypes.byref(n)), "ebbkc_server_poll")
    return [dict(id=r.id, graph=r.graph, k=r.k, status=r.status, count=int(r.count), arrival_ms=r.arrival_ms,
                 admit_ms=r.admit_ms, done_ms=r.done_ms) for r in buf[: n.value]]


def ebbkc_server_stats(s):
    out = (ctypes.c_int64 * 4)()
    _check(load_library().ebbkc_server_stats(s, out), "ebbkc_server_stats")
    return [int(x) for x in out]


def ebbkc_server_destroy(s):
    load_library().ebbkc_server_destroy(s)


# ---------------------------------------------------------------- convenience wrapper

class Graph:
    """A prepared graph on the current device (owns the handle)."""

    def __init__(self, row_ptr, col_idx, n: int | None = None, options: ebbkc_options | None = None, stream=None,
                 nnz: int | None = None):
        n = int(len(row_ptr) - 1) if n is None else n
        nnz = int(len(col_idx)) if nnz is None else nnz
        self._h = ebbkc_prepare(row_ptr, col_idx, n, nnz, options, stream)
        self.info = ebbkc_info_get(self._h)

    @classmethod
    def from_csr(cls, g, device: bool = True, options=None):
        """From a graphgen.Graph-like object (n, row_ptr, col_idx numpy arrays)."""
        if device:
            import torch
            rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr, dtype=np.int32)).cuda()
            nnz = int(len(g.col_idx))
            ci = torch.from_numpy(np.ascontiguousarray(g.col_idx, dtype=np.int32)).cuda()
            if nnz == 0:
                ci = torch.zeros(1, dtype=torch.int32, device="cuda")
            return cls(rp, ci, g.n, options, nnz=nnz)
        ci = np.ascontiguousarray(g.col_idx, np.int32)
        nnz = int(len(ci))
        if nnz == 0:
            ci = np.zeros(1, np.int32)
        return cls(np.ascontiguousarray(g.row_ptr, np.int32), ci, g.n, options, nnz=nnz)

    @property
    def handle(self):
        return self._h

    def count(self, k: int) -> int:
        return ebbkc_count(self._h, k)

    def count128(self, k: int) -> int:
        return ebbkc_count128(self._h, k)

    def max_clique_size(self) -> int:
        return ebbkc_max_clique_size(self._h)

    def count_range(self, k: int, r_begin: int, r_end: int) -> int:
        return ebbkc_count_range(self._h, k, r_begin, r_end)

    def export(self, which: int) -> np.ndarray:
        size = int(self.info.n) if which in (ARR_VERTEX_POS, ARR_VERTEX_COLOR) else int(self.info.m)
        out = np.zeros(max(size, 1), np.int32)
        ebbkc_export(self._h, which, out)
        return out[:size]

    def last_timing(self):
        return ebbkc_last_timing(self._h)

    def last_work(self):
        return ebbkc_last_work(self._h)

    def last_work_class(self, width_class: int):
        return ebbkc_last_work_class(self._h, width_class)

    def close(self):
        if getattr(self, "_h", None):
            ebbkc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
