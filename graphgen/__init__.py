"""Seeded synthetic inputs: permutations and positive-edge graphs in CSR.

This package only creates inputs (no clustering arithmetic).  The CPU oracle
and the GPU library both consume its arrays, so each test or benchmark case
hands the same bytes to both sides.

The C sources live next to this file (``graphgen.c``); ``build()`` compiles
them into ``libgraphgen.so`` in this directory.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile graphgen.c into libgraphgen.so (portable x86-64, OpenMP)."""
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
           "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("off", ctypes.POINTER(ctypes.c_int64)),
                ("col", ctypes.POINTER(ctypes.c_int32)),
                ("ngraphs", ctypes.c_int64),
                ("vtx_ptr", ctypes.POINTER(ctypes.c_int64))]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    i64, u64, f64, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
    lib.gg_free.argtypes = [P(_CSR)]
    lib.gg_permutation.argtypes = [u64, i64, ctypes.c_void_p]
    lib.gg_stream_outputs.argtypes = [u64, u64, i64, ctypes.c_void_p]
    lib.gg_bounded_outputs.argtypes = [u64, u64, u64, i64, ctypes.c_void_p]
    lib.gg_splitmix64_at.argtypes = [u64, u64]
    lib.gg_splitmix64_at.restype = u64
    lib.gg_erdos_renyi.argtypes = [i64, f64, u64]
    lib.gg_erdos_renyi.restype = P(_CSR)
    lib.gg_chung_lu_weights.argtypes = [i64, f64, f64, ctypes.c_void_p]
    lib.gg_chung_lu.argtypes = [i64, f64, f64, u64]
    lib.gg_chung_lu.restype = P(_CSR)
    lib.gg_rmat.argtypes = [i32, i64, f64, f64, f64, u64]
    lib.gg_rmat.restype = P(_CSR)
    lib.gg_sbm_shapes.argtypes = [i64, f64, f64, i64, i64, i64, i64, u64, ctypes.c_void_p, ctypes.c_void_p]
    lib.gg_sbm_batch.argtypes = [i64, ctypes.c_void_p, ctypes.c_void_p, f64, f64, u64]
    lib.gg_sbm_batch.restype = P(_CSR)
    lib.gg_from_edges.argtypes = [i64, i64, ctypes.c_void_p, ctypes.c_void_p]
    lib.gg_from_edges.restype = P(_CSR)
    lib.gg_num_threads.restype = i32
    _lib = lib
    return lib


@dataclass
class Graph:
    """Symmetric CSR of the positive edges.

    ``off`` int64[n+1], ``col`` int32[nnz]; rows sorted, no self-loops, no
    duplicates.  For a batch, ``vtx_ptr`` int64[ngraphs+1] gives each graph's
    first row and ``col`` holds local ids of the same graph.
    """
    n: int
    off: np.ndarray
    col: np.ndarray
    vtx_ptr: np.ndarray | None = None
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.off[-1])

    @property
    def m(self) -> int:
        """Undirected positive edges."""
        return self.nnz // 2

    @property
    def ngraphs(self) -> int:
        return 1 if self.vtx_ptr is None else len(self.vtx_ptr) - 1

    def degrees(self) -> np.ndarray:
        return np.diff(self.off)


class _Owner:
    """Frees a generator-owned CSR once no array views it any more."""

    def __init__(self, ptr):
        self._ptr = ptr

    def __del__(self):
        if self._ptr is not None and _lib is not None:
            _lib.gg_free(self._ptr)
            self._ptr = None


class _View:
    def __init__(self, addr: int, count: int, typestr: str, owner: _Owner):
        self.__array_interface__ = {"data": (addr, False), "shape": (count,),
                                    "typestr": typestr, "version": 3}
        self._owner = owner


def _take(ptr) -> Graph:
    """Wraps the C buffers in NumPy arrays without copying them."""
    c = ptr.contents
    n, nnz = int(c.n), int(c.nnz)
    owner = _Owner(ptr)
    off = np.asarray(_View(ctypes.addressof(c.off.contents), n + 1, "<i8", owner))
    col = (np.asarray(_View(ctypes.addressof(c.col.contents), nnz, "<i4", owner)) if nnz > 0
           else np.zeros(0, dtype=np.int32))
    vp = None
    if c.vtx_ptr:
        vp = np.asarray(_View(ctypes.addressof(c.vtx_ptr.contents), int(c.ngraphs) + 1, "<i8", owner))
    return Graph(n=n, off=off, col=col, vtx_ptr=vp)


def permutation(n: int, seed: int) -> np.ndarray:
    """order[k] = vertex of rank k, uniform over permutations of range(n)."""
    out = np.empty(n, dtype=np.int32)
    _load().gg_permutation(seed, n, out.ctypes.data)
    return out


def stream_outputs(seed: int, sid: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _load().gg_stream_outputs(seed, sid, count, out.ctypes.data)
    return out


def bounded_outputs(seed: int, sid: int, rng: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _load().gg_bounded_outputs(seed, sid, rng, count, out.ctypes.data)
    return out


def splitmix64_at(key: int, i: int) -> int:
    return int(_load().gg_splitmix64_at(key, i))


def erdos_renyi(n: int, mean_degree: float, seed: int) -> Graph:
    p = mean_degree / (n - 1) if n > 1 else 0.0
    g = _take(_load().gg_erdos_renyi(n, p, seed))
    g.name = f"er_n{n}_d{mean_degree:g}_s{seed}"
    return g


def chung_lu_weights(n: int, gamma: float, total: float) -> np.ndarray:
    w = np.empty(n, dtype=np.float64)
    _load().gg_chung_lu_weights(n, gamma, total, w.ctypes.data)
    return w


def chung_lu(n: int, gamma: float, mean_degree: float, seed: int) -> Graph:
    """Chung-Lu with sum of weights n * mean_degree (so ~n*mean_degree/2 edges)."""
    g = _take(_load().gg_chung_lu(n, gamma, float(n) * mean_degree, seed))
    g.name = f"chunglu_n{n}_g{gamma:g}_d{mean_degree:g}_s{seed}"
    return g


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int) -> Graph:
    ptr = _load().gg_rmat(scale, edge_factor, a, b, c, seed)
    if not ptr:
        raise MemoryError("R-MAT generation ran out of host memory")
    g = _take(ptr)
    g.name = f"rmat_s{scale}_ef{edge_factor}_s{seed}"
    return g


def sbm_shapes(ngraphs: int, seed: int, median: float = 500.0, sigma: float = 0.8,
               nmin: int = 50, nmax: int = 5000, kmin: int = 2, kmax: int = 40):
    sizes = np.empty(ngraphs, dtype=np.int64)
    blocks = np.empty(ngraphs, dtype=np.int64)
    _load().gg_sbm_shapes(ngraphs, math.log(median), sigma, nmin, nmax, kmin, kmax, seed,
                          sizes.ctypes.data, blocks.ctypes.data)
    return sizes, blocks


def sbm_batch(sizes: np.ndarray, blocks: np.ndarray, p_in: float, p_out: float, seed: int) -> Graph:
    sizes = np.ascontiguousarray(sizes, dtype=np.int64)
    blocks = np.ascontiguousarray(blocks, dtype=np.int64)
    g = _take(_load().gg_sbm_batch(len(sizes), sizes.ctypes.data, blocks.ctypes.data,
                                   p_in, p_out, seed))
    g.name = f"sbm_x{len(sizes)}_s{seed}"
    return g


def batch_permutations(vtx_ptr: np.ndarray, seed: int) -> np.ndarray:
    """Concatenated local permutations, one per graph, graph g seeded (seed, g)."""
    parts = []
    for gi in range(len(vtx_ptr) - 1):
        ng = int(vtx_ptr[gi + 1] - vtx_ptr[gi])
        parts.append(permutation(ng, seed * 1_000_003 + gi))
    return np.concatenate(parts) if parts else np.zeros(0, dtype=np.int32)


def from_edges(n: int, edges) -> Graph:
    """Symmetric CSR from an undirected edge list (self-loops, duplicates dropped)."""
    e = np.asarray(edges, dtype=np.int32).reshape(-1, 2)
    u = np.ascontiguousarray(e[:, 0])
    v = np.ascontiguousarray(e[:, 1])
    return _take(_load().gg_from_edges(n, len(e), u.ctypes.data, v.ctypes.data))


def num_threads() -> int:
    return int(_load().gg_num_threads())


# ---- the named workloads -------------------------------------------------

def workload(name: str) -> Graph:
    """Graphs of the five workloads (small ones only for tests)."""
    if name == "er20k":
        return erdos_renyi(20_000, 10.0, seed=1)
    if name == "chunglu2m":
        return chung_lu(2_000_000, 2.1, 40.0, seed=2)
    if name.startswith("rmat"):
        scale = int(name[4:])
        return rmat(scale, 16, 0.57, 0.19, 0.19, seed=3 if scale == 26 else 100 + scale)
    if name.startswith("sbm"):
        # planted blocks: lognormal sizes (median 500) clipped to [50, 5000],
        # 2-40 blocks, p_in = 0.3, p_out = 0.01
        count = int(name[3:])
        sizes, blocks = sbm_shapes(count, seed=4)
        return sbm_batch(sizes, blocks, 0.3, 0.01, seed=4)
    raise KeyError(name)
