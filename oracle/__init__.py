"""CPU oracle for C4 / ClusterWild! (arXiv 1507.05086).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py`` -- never by the GPU library in
``paper_1507_05086_amd``.  The two share no code; both read the arrays that
``graphgen`` writes.

``cc_oracle.c`` holds the plain serial algorithms (KwikCluster, the BSP
simulator of C4 and ClusterWild!, the objective counted three ways, and the
any-size KwikCluster checker); ``mlp.py`` holds the float64 reference of the
small epsilon-policy network.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libcc_oracle.so")
_lib = None

C4, CW = 0, 1
TRACE_FIELDS = ("n_i", "delta_i", "b_i", "r_i", "centers", "claimed", "conflicts")


def build(verbose: bool = False) -> str:
    """Compile the oracle (serial, -O3 for any x86-64 CPU with AVX2 -- the
    library travels to other hosts, so not -march=native; no fused
    multiply-add contraction, so every floating-point step rounds as written)
    into libcc_oracle.so."""
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11", "-Wall",
           "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Round(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in TRACE_FIELDS]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.orc_kwikcluster.argtypes = [i64, vp, vp, vp, vp]
    lib.orc_kwikcluster.restype = i32
    lib.orc_bsp.argtypes = [i32, i64, vp, vp, vp, i64, vp, i64, vp, vp, i64, vp]
    lib.orc_bsp.restype = i64
    lib.orc_quantize_eps.argtypes = [ctypes.c_double]
    lib.orc_quantize_eps.restype = i64
    lib.orc_cost.argtypes = [i64, vp, vp, vp]
    lib.orc_cost.restype = i64
    lib.orc_cost_pairs.argtypes = [i64, vp, vp, vp]
    lib.orc_cost_pairs.restype = i64
    lib.orc_kc_stepwise_cost.argtypes = [i64, vp, vp, vp]
    lib.orc_kc_stepwise_cost.restype = i64
    lib.orc_check_kc.argtypes = [i64, vp, vp, vp, vp, vp]
    lib.orc_check_kc.restype = i64
    u64, f64 = ctypes.c_uint64, ctypes.c_double
    lib.orc_binomial.argtypes = [u64, u64, i64, f64]
    lib.orc_binomial.restype = i64
    lib.orc_halving_period.argtypes = [i64, i64, f64, f64]
    lib.orc_halving_period.restype = i64
    lib.orc_binomial_schedule.argtypes = [i64, i64, f64, f64, u64, vp, i64]
    lib.orc_binomial_schedule.restype = i64
    lib.orc_bsp_binomial.argtypes = [i32, i64, vp, vp, vp, f64, f64, u64, vp, vp, i64, vp]
    lib.orc_bsp_binomial.restype = i64
    lib.orc_bsp_positions.argtypes = [i32, i64, vp, vp, vp, vp, i64, i64, i64, vp, vp, i64, vp]
    lib.orc_bsp_positions.restype = i64
    _lib = lib
    return lib


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


@dataclass
class BSPResult:
    labels: np.ndarray
    rounds: int
    trace: np.ndarray  # structured array with TRACE_FIELDS
    round_of: np.ndarray = None  # round in which each vertex was clustered (if asked for)

    def trace_dict(self, i: int) -> dict:
        return {f: int(self.trace[f][i]) for f in TRACE_FIELDS}


def kwikcluster(off, col, order) -> np.ndarray:
    """KwikCluster with order pi (Algorithm 1): labels = center vertex ids."""
    off, po = _c(off, np.int64)
    col, pc = _c(col, np.int32)
    order, pr = _c(order, np.int32)
    n = len(off) - 1
    labels = np.empty(n, dtype=np.int32)
    rc = _load().orc_kwikcluster(n, po, pc, pr, labels.ctypes.data)
    if rc != 0:
        raise ValueError(f"orc_kwikcluster failed ({rc})")
    return labels


def quantize_eps(eps: float) -> int:
    return int(_load().orc_quantize_eps(eps))


def bsp(algo: int, off, col, order, eps: float = 0.5, sched=None, trace_cap: int = 1 << 16,
        with_round_of: bool = False) -> BSPResult:
    """Serial simulation of the BSP round loop (Algorithm 2), C4 or ClusterWild!."""
    off, po = _c(off, np.int64)
    col, pc = _c(col, np.int32)
    order, pr = _c(order, np.int32)
    n = len(off) - 1
    labels = np.empty(n, dtype=np.int32)
    trace = np.zeros(trace_cap, dtype=[(f, np.int64) for f in TRACE_FIELDS])
    if sched is None:
        sp, slen = None, 0
    else:
        sched, sp = _c(sched, np.int64)
        slen = len(sched)
    round_of = np.full(n, -1, dtype=np.int32) if with_round_of else None
    rounds = _load().orc_bsp(algo, n, po, pc, pr, quantize_eps(eps), sp, slen,
                             labels.ctypes.data, trace.ctypes.data, trace_cap,
                             round_of.ctypes.data if with_round_of else None)
    if rounds < 0:
        raise ValueError(f"orc_bsp failed ({rounds})")
    return BSPResult(labels=labels, rounds=int(rounds), trace=trace[:min(rounds, trace_cap)],
                     round_of=round_of)


def c4(off, col, order, eps=0.5, sched=None, trace_cap=1 << 16) -> BSPResult:
    return bsp(C4, off, col, order, eps, sched, trace_cap)


def clusterwild(off, col, order, eps=0.5, sched=None, trace_cap=1 << 16) -> BSPResult:
    return bsp(CW, off, col, order, eps, sched, trace_cap)


def cost(off, col, labels) -> int:
    """Disagreements (objective of Section 2) in closed form."""
    off, po = _c(off, np.int64)
    col, pc = _c(col, np.int32)
    labels, pl = _c(labels, np.int32)
    r = _load().orc_cost(len(off) - 1, po, pc, pl)
    if r < 0:
        raise ValueError("labels out of range")
    return int(r)


def cost_pairs(off, col, labels) -> int:
    """Disagreements counted pair by pair (O(n^2); small graphs)."""
    off, po = _c(off, np.int64)
    col, pc = _c(col, np.int32)
    labels, pl = _c(labels, np.int32)
    return int(_load().orc_cost_pairs(len(off) - 1, po, pc, pl))


def kc_stepwise_cost(off, col, order) -> int:
    """KwikCluster's cost summed per peeling step (bad-triangle lemma)."""
    off, po = _c(off, np.int64)
    col, pc = _c(col, np.int32)
    order, pr = _c(order, np.int32)
    return int(_load().orc_kc_stepwise_cost(len(off) - 1, po, pc, pr))


def check_kc(off, col, order, labels):
    """(violations, first_bad_vertex): 0 violations iff labels == KwikCluster(G, pi)."""
    off, po = _c(off, np.int64)
    col, pc = _c(col, np.int32)
    order, pr = _c(order, np.int32)
    labels, pl = _c(labels, np.int32)
    first = ctypes.c_int64(-1)
    r = _load().orc_check_kc(len(off) - 1, po, pc, pr, pl, ctypes.byref(first))
    if r < 0:
        raise ValueError(f"orc_check_kc failed ({r})")
    return int(r), int(first.value)


# ------------------------------------------- the paper's practical schedule

DEFAULT_DELTA = 0.1  # failure probability in the halving period of Delta-hat (a reading)


def binomial(seed: int, stream: int, n: int, p: float) -> int:
    """One Binomial(n, p) variate from uniform stream `stream` of `seed`."""
    return int(_load().orc_binomial(seed, stream, n, p))


def halving_period(n: int, delta0: int, eps: float, delta: float = DEFAULT_DELTA) -> int:
    """Rounds between two halvings of Delta-hat."""
    return int(_load().orc_halving_period(n, delta0, eps, delta))


def binomial_schedule(n: int, delta0: int, eps: float, seed: int, delta: float = DEFAULT_DELTA) -> np.ndarray:
    """B_0, B_1, ...: pi positions taken by each round until none is left."""
    lib = _load()
    rounds = lib.orc_binomial_schedule(n, delta0, eps, delta, seed, None, 0)
    if rounds < 0:
        raise ValueError(f"orc_binomial_schedule failed ({rounds})")
    out = np.zeros(max(rounds, 1), dtype=np.int64)
    lib.orc_binomial_schedule(n, delta0, eps, delta, seed, out.ctypes.data, rounds)
    return out[:rounds]


def bsp_binomial(algo: int, off, col, order, eps: float = 0.5, seed: int = 0, delta: float = DEFAULT_DELTA,
                 trace_cap: int = 1 << 20, with_round_of: bool = False) -> BSPResult:
    """C4 or ClusterWild! with Delta-hat and Binomial batches over pi positions."""
    off, po = _c(off, np.int64)
    col, pc = _c(col, np.int32)
    order, pr = _c(order, np.int32)
    n = len(off) - 1
    labels = np.empty(n, dtype=np.int32)
    trace = np.zeros(trace_cap, dtype=[(f, np.int64) for f in TRACE_FIELDS])
    round_of = np.full(n, -1, dtype=np.int32) if with_round_of else None
    rounds = _load().orc_bsp_binomial(algo, n, po, pc, pr, eps, delta, seed, labels.ctypes.data,
                                      trace.ctypes.data, trace_cap,
                                      round_of.ctypes.data if with_round_of else None)
    if rounds < 0:
        raise ValueError(f"orc_bsp_binomial failed ({rounds})")
    return BSPResult(labels=labels, rounds=int(rounds), trace=trace[:min(rounds, trace_cap)],
                     round_of=round_of)


def bsp_positions(algo: int, off, col, order, sched, trace_cap: int = 1 << 20) -> BSPResult:
    """Rounds taking the next sched[i] positions of pi (must cover all of them)."""
    off, po = _c(off, np.int64)
    col, pc = _c(col, np.int32)
    order, pr = _c(order, np.int32)
    sched, ps = _c(sched, np.int64)
    n = len(off) - 1
    labels = np.empty(n, dtype=np.int32)
    trace = np.zeros(trace_cap, dtype=[(f, np.int64) for f in TRACE_FIELDS])
    rounds = _load().orc_bsp_positions(algo, n, po, pc, pr, ps, len(sched), 0, 0, labels.ctypes.data,
                                       trace.ctypes.data, trace_cap, None)
    if rounds < 0:
        raise ValueError(f"orc_bsp_positions failed ({rounds})")
    return BSPResult(labels=labels, rounds=int(rounds), trace=trace[:min(rounds, trace_cap)])
