"""CPU oracle for exact k-clique counting and listing -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this
package.  The GPU library (``paper_2311_13798_amd``) never imports it and shares no code with it.

The arithmetic lives in ``oracle.c`` (plain C, compiled with gcc); this module only marshals
numpy arrays.  What each function computes, and from which passage of the paper, is stated in
the header of ``oracle.c``:

* ``count``            N_k by degeneracy-ordered vertex branching (Algorithm VBBkC, Section 3).
* ``count_brute``      N_k by testing every k-subset (n <= 62).
* ``list_lex``         all k-cliques, lexicographic, with the two listing checksums.
* ``edge_support``     common-neighbour count of every edge (Section 4.2).
* ``truss_levelsync``  level-synchronous truss-based edge ordering (Section 4.2): level, rank, tau.
* ``truss_sequential`` the sequential greedy of Eq. truss-based-edge.
* ``degeneracy``       degeneracy order and delta.
* ``seed_sizes`` / ``seed_counts``  per-edge sub-branch size and (k-2)-clique count of
  Eq. edge-oriented-branching at the initial branch, for a given edge ranking.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

OK, BAD_CSR, OOM, BAD_ARG, BUFFER_TOO_SMALL, OVERFLOW = 0, -2, -3, -4, -5, -6


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC, "-lpthread"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        sig = {
            "orc_validate_csr": [i32, i64, vp, vp],
            "orc_edge_support": [i32, vp, vp, vp],
            "orc_edge_list": [i32, vp, vp, vp, vp],
            "orc_truss_levelsync": [i32, vp, vp, vp, vp, vp, vp, vp],
            "orc_truss_sequential": [i32, vp, vp, vp, vp],
            "orc_degeneracy": [i32, vp, vp, vp, vp],
            "orc_count_vbb": [i32, vp, vp, i32, i32, i32, vp],
            "orc_count_brute": [i32, vp, vp, i32, vp],
            "orc_list_lex": [i32, vp, vp, i32, i32, vp, u64, vp, vp, vp],
            "orc_seed_sizes": [i32, vp, vp, vp, vp],
            "orc_seed_counts": [i32, vp, vp, vp, i32, vp, i64, vp],
            "orc_binom": [u64, u64, vp],
            "orc_tuple_hash": [vp, i32],
            "orc_num_edges": [i32, vp, vp],
        }
        for name, args in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        lib.orc_tuple_hash.restype = u64
        lib.orc_num_edges.restype = i64
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data if a.size else None


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    if ci.size == 0:
        ci = np.zeros(1, np.int32)
    return g.n, rp, ci


def _chk(rc: int, what: str):
    if rc != OK:
        raise OracleError(rc, what)


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def validate(g) -> int:
    n, rp, ci = _csr(g)
    return _load().orc_validate_csr(n, g.nnz, rp.ctypes.data, ci.ctypes.data)


def num_edges(g) -> int:
    n, rp, ci = _csr(g)
    return int(_load().orc_num_edges(n, rp.ctypes.data, ci.ctypes.data))


def edge_list(g):
    n, rp, ci = _csr(g)
    m = num_edges(g)
    eu = np.zeros(max(m, 1), np.int32)
    ev = np.zeros(max(m, 1), np.int32)
    _chk(_load().orc_edge_list(n, rp.ctypes.data, ci.ctypes.data, eu.ctypes.data, ev.ctypes.data), "edge_list")
    return eu[:m], ev[:m]


def binom(n: int, r: int) -> int:
    out = ctypes.c_uint64()
    _chk(_load().orc_binom(n, r, ctypes.byref(out)), "binom")
    return int(out.value)


def tuple_hash(t) -> int:
    a = np.ascontiguousarray(t, dtype=np.int32)
    return int(_load().orc_tuple_hash(a.ctypes.data, a.size))


def count(g, k: int, threads: int | None = None, shortcut: bool = True) -> int:
    n, rp, ci = _csr(g)
    out = ctypes.c_uint64()
    _chk(_load().orc_count_vbb(n, rp.ctypes.data, ci.ctypes.data, k, threads or default_threads(),
                               int(shortcut), ctypes.byref(out)), "count")
    return int(out.value)


def count_brute(g, k: int) -> int:
    n, rp, ci = _csr(g)
    out = ctypes.c_uint64()
    _chk(_load().orc_count_brute(n, rp.ctypes.data, ci.ctypes.data, k, ctypes.byref(out)), "count_brute")
    return int(out.value)


def list_lex(g, k: int, threads: int | None = None, want_tuples: bool = True):
    """Returns (count, ordered_checksum, unordered_checksum, tuples or None)."""
    n, rp, ci = _csr(g)
    lib = _load()
    cnt, ho, hu = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    th = threads or default_threads()
    if not want_tuples:
        _chk(lib.orc_list_lex(n, rp.ctypes.data, ci.ctypes.data, k, th, None, 0,
                              ctypes.byref(cnt), ctypes.byref(ho), ctypes.byref(hu)), "list_lex")
        return int(cnt.value), int(ho.value), int(hu.value), None
    c = count(g, k, th)
    buf = np.zeros((max(c, 1), k), np.int32)
    _chk(lib.orc_list_lex(n, rp.ctypes.data, ci.ctypes.data, k, th, buf.ctypes.data, c,
                          ctypes.byref(cnt), ctypes.byref(ho), ctypes.byref(hu)), "list_lex")
    assert cnt.value == c
    return int(cnt.value), int(ho.value), int(hu.value), buf[:c]


def edge_support(g) -> np.ndarray:
    n, rp, ci = _csr(g)
    m = num_edges(g)
    sup = np.zeros(max(m, 1), np.int32)
    _chk(_load().orc_edge_support(n, rp.ctypes.data, ci.ctypes.data, sup.ctypes.data), "edge_support")
    return sup[:m]


def truss_levelsync(g):
    """Returns dict(level, rank, round, rounds, tau), arrays indexed by edge id."""
    n, rp, ci = _csr(g)
    m = num_edges(g)
    level = np.zeros(max(m, 1), np.int32)
    rank = np.zeros(max(m, 1), np.int32)
    rnd = np.zeros(max(m, 1), np.int32)
    nr, tau = ctypes.c_int32(), ctypes.c_int32()
    _chk(_load().orc_truss_levelsync(n, rp.ctypes.data, ci.ctypes.data, level.ctypes.data, rank.ctypes.data,
                                     rnd.ctypes.data, ctypes.byref(nr), ctypes.byref(tau)), "truss_levelsync")
    return dict(level=level[:m], rank=rank[:m], round=rnd[:m], rounds=int(nr.value), tau=int(tau.value))


def truss_sequential(g):
    """Returns (order, peel): order[i] = id of the i-th removed edge, peel[e] = its support then."""
    n, rp, ci = _csr(g)
    m = num_edges(g)
    order = np.zeros(max(m, 1), np.int32)
    peel = np.zeros(max(m, 1), np.int32)
    _chk(_load().orc_truss_sequential(n, rp.ctypes.data, ci.ctypes.data, order.ctypes.data, peel.ctypes.data),
         "truss_sequential")
    return order[:m], peel[:m]


def degeneracy(g):
    n, rp, ci = _csr(g)
    order = np.zeros(max(n, 1), np.int32)
    d = ctypes.c_int32()
    _chk(_load().orc_degeneracy(n, rp.ctypes.data, ci.ctypes.data, order.ctypes.data, ctypes.byref(d)),
         "degeneracy")
    return order[:n], int(d.value)


def seed_sizes(g, rank: np.ndarray) -> np.ndarray:
    n, rp, ci = _csr(g)
    m = num_edges(g)
    r = np.ascontiguousarray(rank, dtype=np.int32)
    out = np.zeros(max(m, 1), np.int32)
    _chk(_load().orc_seed_sizes(n, rp.ctypes.data, ci.ctypes.data, _ptr(r), out.ctypes.data), "seed_sizes")
    return out[:m]


def seed_counts(g, rank: np.ndarray, k: int, eids=None) -> np.ndarray:
    n, rp, ci = _csr(g)
    m = num_edges(g)
    r = np.ascontiguousarray(rank, dtype=np.int32)
    e = np.arange(m, dtype=np.int64) if eids is None else np.ascontiguousarray(eids, dtype=np.int64)
    out = np.zeros(max(e.size, 1), np.uint64)
    _chk(_load().orc_seed_counts(n, rp.ctypes.data, ci.ctypes.data, _ptr(r), k, _ptr(e), e.size,
                                 out.ctypes.data), "seed_counts")
    return out[:e.size]
