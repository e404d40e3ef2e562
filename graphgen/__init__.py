"""Seeded synthetic graph inputs shared by the oracle, the HIP path, the tests and the bench.

This package only prepares inputs: it draws random edges (``graphgen.c``) and returns a clean
CSR (sorted rows, symmetric, no self-loops or duplicates), the simple undirected graph model of
the paper's problem statement (Section 2; Section 6.1 drops directions, weights and loops).
It contains none of the k-clique method's arithmetic.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgraphgen.so")
_SRC = os.path.join(_HERE, "graphgen.c")


def build(force: bool = True) -> str:
    """Compile graphgen.c into libgraphgen.so next to it (gcc, host code only)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.POINTER(ctypes.c_int32)), ("col_idx", ctypes.POINTER(ctypes.c_int32))]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        P = ctypes.POINTER(_CSR)
        i32, i64, u64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        lib.gg_er.argtypes = [i32, dbl, u64, P]
        lib.gg_rmat.argtypes = [i32, i64, dbl, dbl, dbl, u64, P]
        lib.gg_chung_lu.argtypes = [i32, dbl, dbl, i32, i32, i32, u64, P]
        lib.gg_er_planted.argtypes = [i32, dbl, i32, i32, i32, u64, P]
        lib.gg_from_edges.argtypes = [i32, i64, ctypes.c_void_p, ctypes.c_void_p, P]
        lib.gg_permute.argtypes = [P, u64, P]
        lib.gg_free.argtypes = [P]
        lib.gg_splitmix64.argtypes = [u64]
        lib.gg_splitmix64.restype = u64
        for f in ("gg_er", "gg_rmat", "gg_chung_lu", "gg_er_planted", "gg_from_edges", "gg_permute"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class Graph:
    """Undirected simple graph as int32 CSR with sorted rows (both directions stored)."""
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        h.update(np.ascontiguousarray(self.row_ptr, dtype=np.int32).tobytes())
        h.update(np.ascontiguousarray(self.col_idx, dtype=np.int32).tobytes())
        return h.hexdigest()

    def edges(self) -> np.ndarray:
        """(m,2) array of undirected edges (u<v) in lexicographic order."""
        src = np.repeat(np.arange(self.n, dtype=np.int32), self.degrees())
        mask = src < self.col_idx
        return np.stack([src[mask], self.col_idx[mask]], axis=1)


def _take(c: _CSR, name: str) -> Graph:
    lib = _load()
    n, nnz = int(c.n), int(c.nnz)
    rp = np.ctypeslib.as_array(c.row_ptr, shape=(n + 1,)).copy() if n + 1 > 0 else np.zeros(1, np.int32)
    ci = (np.ctypeslib.as_array(c.col_idx, shape=(nnz,)).copy() if nnz > 0
          else np.zeros(0, np.int32))
    lib.gg_free(ctypes.byref(c))
    return Graph(n, rp.astype(np.int32, copy=False), ci.astype(np.int32, copy=False), name)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"graphgen {what} failed with code {rc}")


def splitmix64(x: int) -> int:
    return int(_load().gg_splitmix64(ctypes.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


def er(n: int, p: float, seed: int = 1) -> Graph:
    c = _CSR()
    _check(_load().gg_er(n, p, seed, ctypes.byref(c)), "er")
    return _take(c, f"er_n{n}_p{p}_s{seed}")


def rmat(scale: int, edge_factor: int = 16, a=0.57, b=0.19, c=0.19, seed: int = 1) -> Graph:
    cs = _CSR()
    _check(_load().gg_rmat(scale, edge_factor << scale, a, b, c, seed, ctypes.byref(cs)), "rmat")
    return _take(cs, f"rmat_s{scale}_ef{edge_factor}_s{seed}")


def chung_lu(n: int, gamma: float = 2.1, mean_deg: float = 30.0, nplant: int = 0,
             smin: int = 30, smax: int = 60, seed: int = 1) -> Graph:
    cs = _CSR()
    _check(_load().gg_chung_lu(n, gamma, mean_deg, nplant, smin, smax, seed, ctypes.byref(cs)), "chung_lu")
    return _take(cs, f"cl_n{n}_g{gamma}_d{mean_deg}_p{nplant}_s{seed}")


def er_planted(n: int, p: float, nplant: int, smin: int, smax: int, seed: int) -> Graph:
    cs = _CSR()
    _check(_load().gg_er_planted(n, p, nplant, smin, smax, seed, ctypes.byref(cs)), "er_planted")
    return _take(cs, f"erp_n{n}_p{p}_{nplant}x{smin}-{smax}_s{seed}")


def from_edges(n: int, edges, name: str = "") -> Graph:
    e = np.asarray(edges, dtype=np.int32).reshape(-1, 2)
    src = np.ascontiguousarray(e[:, 0])
    dst = np.ascontiguousarray(e[:, 1])
    cs = _CSR()
    _check(_load().gg_from_edges(n, e.shape[0], src.ctypes.data, dst.ctypes.data, ctypes.byref(cs)),
           "from_edges")
    return _take(cs, name)


def permute(g: Graph, seed: int) -> Graph:
    src = _CSR(g.n, g.nnz, g.row_ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
               g.col_idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    out = _CSR()
    _check(_load().gg_permute(ctypes.byref(src), seed, ctypes.byref(out)), "permute")
    return _take(out, g.name + f"_perm{seed}")


# ---------------------------------------------------------------- structured families
def complete(n: int) -> Graph:
    iu = np.triu_indices(n, 1)
    return from_edges(n, np.stack(iu, 1), f"K{n}")


def complete_multipartite(parts) -> Graph:
    lab = np.concatenate([np.full(a, i) for i, a in enumerate(parts)]) if parts else np.zeros(0)
    n = int(len(lab))
    iu = np.triu_indices(n, 1)
    keep = lab[iu[0]] != lab[iu[1]]
    return from_edges(n, np.stack([iu[0][keep], iu[1][keep]], 1), "K_" + "_".join(map(str, parts)))


def cocktail_party(p: int) -> Graph:
    """K_{2p} minus a perfect matching (vertex 2i is not adjacent to 2i+1)."""
    return complete_multipartite([2] * p)


def disjoint_cliques(sizes) -> Graph:
    edges, off = [], 0
    for s in sizes:
        iu = np.triu_indices(s, 1)
        edges.append(np.stack(iu, 1) + off)
        off += s
    e = np.concatenate(edges) if edges else np.zeros((0, 2), np.int32)
    return from_edges(off, e, "cliques_" + "_".join(map(str, sizes)))


def empty(n: int) -> Graph:
    return from_edges(n, np.zeros((0, 2), np.int32), f"empty{n}")


def random_small(n: int, p: float, seed: int) -> Graph:
    """Tiny G(n,p) drawn pair by pair with SplitMix64 (for brute-force pins)."""
    return er(n, p, seed)
