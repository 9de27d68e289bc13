"""Python binding of the gfx950 correlation-clustering library (``libcc.so``).

The functions keep the C ABI's names (``include/cc.h``) and only marshal
arguments: every step of C4 / ClusterWild! runs in the library's HIP kernels.
Device tensors (torch, ``device="cuda"``) are passed as device pointers on
torch's current stream; NumPy arrays are passed as host pointers.

Importing this package fails loudly when ``libcc.so`` has not been built: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcc.so")

CC_OK = 0
CC_ERR_INVALID_ARG = 1
CC_ERR_NOT_SYMMETRIC = 2
CC_ERR_SELF_LOOP = 3
CC_ERR_DUPLICATE_EDGE = 4
CC_ERR_NOT_PERMUTATION = 5
CC_ERR_OUT_OF_MEMORY = 6
CC_ERR_DEVICE = 7
CC_ERR_NO_PROGRESS = 8
CC_ERR_POLICY = 9
CC_ERR_OUT_OF_RANGE = 10

CC_VALIDATE = 1
CC_INPUT_ON_DEVICE = 2
CC_BORROW = 4
CC_OUTPUT_ON_DEVICE = 8

CC_EPS_FIXED = 0
CC_EPS_LEARNED = 1
CC_EPS_TRACE = 2
CC_EPS_BINOMIAL = 3

CC_MLP_IN, CC_MLP_HIDDEN = 6, 64
CC_MLP_PARAMS = CC_MLP_HIDDEN * CC_MLP_IN + CC_MLP_HIDDEN + CC_MLP_HIDDEN + 1

CC_ALGO_C4, CC_ALGO_CLUSTERWILD = 0, 1
CC_BATCH_MAX_N = 7168

ABI_FUNCTIONS = ("cc_graph_from_csr", "cc_graph_destroy", "cc_graph_info", "cc_c4",
                 "cc_clusterwild", "cc_c4_async", "cc_clusterwild_async", "cc_cost", "cc_batch_set_config", "cc_batch_autotune",
                 "cc_mlp_forward", "cc_mlp_train_step", "cc_mlp_train_step_noalloc", "cc_set_eps_policy",
                 "cc_binomial_schedule",
                 "cc_last_error")

TRACE_FIELDS = ("n_i", "delta_i", "b_i", "r_i", "centers", "claimed", "conflicts", "eps_used", "t_ns")


class CCError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"cc error {code}: {message}")
        self.code = code


class _RoundRecord(ctypes.Structure):
    _fields_ = [("n_i", ctypes.c_int64), ("delta_i", ctypes.c_int64), ("b_i", ctypes.c_int64),
                ("r_i", ctypes.c_int64), ("centers", ctypes.c_int64), ("claimed", ctypes.c_int64),
                ("conflicts", ctypes.c_int64), ("eps_used", ctypes.c_double), ("t_ns", ctypes.c_int64)]


class _RunStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int64), ("scanned_elect", ctypes.c_int64),
                ("scanned_claim", ctypes.c_int64), ("scanned_peel", ctypes.c_int64),
                ("scanned_delta", ctypes.c_int64),
                ("blocked", ctypes.c_int64), ("atomics", ctypes.c_int64),
                ("loop_ms", ctypes.c_double), ("policy_fallback", ctypes.c_int32),
                ("truncated", ctypes.c_int32), ("trace", ctypes.POINTER(_RoundRecord)),
                ("trace_capacity", ctypes.c_int64), ("graph_rounds", ctypes.POINTER(ctypes.c_int32)),
                ("max_rounds", ctypes.c_int64), ("fault_round", ctypes.c_int64),
                ("async_waves", ctypes.c_int64)]


class _BinomialParams(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("delta", ctypes.c_double)]


class _BatchConfig(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("wave_max_n", ctypes.c_int32), ("quad_max_n", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("ms", ctypes.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1507_05086_amd.build.build() "
                          "(hipcc, gfx950); there is no CPU fallback")
    # torch first: the library then binds to the HIP runtime torch has loaded,
    # so both see the same devices, streams and memory
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double
    sig = {
        "cc_graph_from_csr": ([i32, vp, i64, vp, vp, u32, vp, ctypes.POINTER(vp)], i32),
        "cc_graph_destroy": ([vp], i32),
        "cc_graph_info": ([vp, vp, vp, vp], i32),
        "cc_c4": ([vp, vp, f64, vp, ctypes.POINTER(_RunStats), u32, vp], i32),
        "cc_clusterwild": ([vp, vp, f64, vp, ctypes.POINTER(_RunStats), u32, vp], i32),
        "cc_c4_async": ([vp, vp, vp, ctypes.POINTER(_RunStats), u32, vp], i32),
        "cc_clusterwild_async": ([vp, vp, vp, ctypes.POINTER(_RunStats), u32, vp], i32),
        "cc_cost": ([vp, vp, vp, u32, vp], i32),
        "cc_batch_set_config": ([vp, ctypes.POINTER(_BatchConfig)], i32),
        "cc_batch_autotune": ([vp, i32, vp, f64, u32, vp, ctypes.POINTER(_BatchConfig)], i32),
        "cc_mlp_forward": ([vp, vp, i64, vp, vp], i32),
        "cc_mlp_train_step": ([vp, vp, vp, vp, vp, i64, i64, ctypes.c_float, vp, vp, vp], i32),
        "cc_mlp_train_step_noalloc": ([vp, vp, vp, vp, vp, i64, i64, ctypes.c_float, vp, vp, vp], i32),
        "cc_set_eps_policy": ([i32, vp, ctypes.c_size_t, f64, f64], i32),
        "cc_binomial_schedule": ([i64, i64, f64, ctypes.c_uint64, f64, vp, i64, vp, vp], i32),
        "cc_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


def _check(rc: int):
    if rc != CC_OK:
        raise CCError(rc, _lib.cc_last_error().decode(errors="replace"))


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x, dtype):
    """(pointer, on_device, keepalive) of a torch tensor or array-like."""
    if x is None:
        return None, False, None
    if _is_torch(x):
        import torch
        want = {np.int32: torch.int32, np.int64: torch.int64, np.float32: torch.float32}[dtype]
        if x.dtype != want:
            raise TypeError(f"expected {want}, got {x.dtype}")
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(x.data_ptr()), x.is_cuda, x
    a = np.ascontiguousarray(x, dtype=dtype)
    return ctypes.c_void_p(a.ctypes.data), False, a


def _stream(stream, *tensors):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    for t in tensors:
        if t is not None and _is_torch(t) and t.is_cuda:
            import torch
            return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)
    return ctypes.c_void_p(0)


class Graph:
    """A graph handle (device CSR + run workspace)."""

    def __init__(self, handle, n, nnz, num_graphs, keep):
        self._h = handle
        self.n = n
        self.nnz = nnz
        self.num_graphs = num_graphs
        self._keep = keep  # borrowed device tensors stay alive with the handle

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            _lib.cc_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cc_graph_from_csr(offsets, cols, vtx_ptr=None, validate=False, borrow=False, stream=None) -> Graph:
    """Upload a symmetric CSR of positive edges (int64 offsets, int32 cols)."""
    po, od, ko = _ptr(offsets, np.int64)
    pc, cd, kc = _ptr(cols, np.int32)
    if od != cd:
        raise ValueError("offsets and cols must both be host arrays or both device tensors")
    n = (offsets.numel() if _is_torch(offsets) else len(ko)) - 1
    flags = (CC_VALIDATE if validate else 0)
    if od:
        flags |= CC_BORROW if borrow else CC_INPUT_ON_DEVICE
    ng = 1
    pv = None
    kv = None
    if vtx_ptr is not None:
        kv = np.ascontiguousarray(np.asarray(vtx_ptr), dtype=np.int64)
        ng = len(kv) - 1
        pv = ctypes.c_void_p(kv.ctypes.data)
    h = ctypes.c_void_p()
    _check(_lib.cc_graph_from_csr(ng, pv, n, po, pc, flags, _stream(stream, offsets), ctypes.byref(h)))
    nn, nnz, gg = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    _check(_lib.cc_graph_info(h, ctypes.byref(nn), ctypes.byref(nnz), ctypes.byref(gg)))
    return Graph(h, nn.value, nnz.value, gg.value, (ko, kc) if borrow else None)


@dataclass
class RunStats:
    rounds: int = 0
    scanned_elect: int = 0
    scanned_claim: int = 0
    scanned_peel: int = 0
    scanned_delta: int = 0
    blocked: int = 0
    atomics: int = 0
    loop_ms: float = 0.0
    policy_fallback: int = 0
    truncated: int = 0
    trace: np.ndarray = field(default_factory=lambda: np.zeros(0))
    graph_rounds: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))


def _run(fn, graph: Graph, order, eps, labels=None, trace_capacity=1 << 14, stream=None, max_rounds=0,
         fault_round=0):
    po, odev, _ko = _ptr(order, np.int32)
    if labels is None:
        if odev:
            import torch
            labels = torch.empty(graph.n, dtype=torch.int32, device=order.device)
        else:
            labels = np.empty(graph.n, dtype=np.int32)
    pl, ldev, _kl = _ptr(labels, np.int32)
    flags = (CC_INPUT_ON_DEVICE if odev else 0) | (CC_OUTPUT_ON_DEVICE if ldev else 0)
    st = _RunStats()
    rec = None
    if trace_capacity > 0:
        rec = (_RoundRecord * trace_capacity)()
        st.trace = ctypes.cast(rec, ctypes.POINTER(_RoundRecord))
        st.trace_capacity = trace_capacity
    st.max_rounds = int(max_rounds)
    st.fault_round = int(fault_round)
    gr = np.zeros(max(graph.num_graphs, 1), dtype=np.int32)
    st.graph_rounds = gr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    _check(fn(graph.handle, po, float(eps), pl, ctypes.byref(st), flags, _stream(stream, order, labels)))
    out = RunStats(rounds=st.rounds, scanned_elect=st.scanned_elect, scanned_claim=st.scanned_claim,
                   scanned_peel=st.scanned_peel, scanned_delta=st.scanned_delta, blocked=st.blocked,
                   atomics=st.atomics,
                   loop_ms=st.loop_ms, policy_fallback=st.policy_fallback,
                   truncated=st.truncated, graph_rounds=gr)
    if rec is not None:
        k = min(st.rounds, trace_capacity)
        dt = np.dtype([(f, np.float64 if f == "eps_used" else np.int64) for f in TRACE_FIELDS])
        arr = np.frombuffer(bytes(rec)[: k * ctypes.sizeof(_RoundRecord)], dtype=dt) if k else np.zeros(0, dt)
        out.trace = arr.copy()
    return labels, out


def cc_c4(graph: Graph, order, eps: float = 0.5, labels=None, trace_capacity: int = 1 << 14, stream=None,
          max_rounds: int = 0, fault_round: int = 0):
    """C4 (labels equal KwikCluster's under the same order).  Returns (labels, RunStats).
    max_rounds > 0 stops after that many rounds (unclustered vertices get -1);
    fault_round > 0 is the error-path test hook of cc_run_stats."""
    return _run(_lib.cc_c4, graph, order, eps, labels, trace_capacity, stream, max_rounds, fault_round)


def cc_clusterwild(graph: Graph, order, eps: float = 0.5, labels=None, trace_capacity: int = 1 << 14,
                   stream=None, max_rounds: int = 0, fault_round: int = 0):
    """ClusterWild!.  Returns (labels, RunStats)."""
    return _run(_lib.cc_clusterwild, graph, order, eps, labels, trace_capacity, stream, max_rounds, fault_round)


def _run_async(fn, graph: Graph, order, labels=None, waves=0, stream=None):
    po, odev, _ko = _ptr(order, np.int32)
    if labels is None:
        if odev:
            import torch
            labels = torch.empty(graph.n, dtype=torch.int32, device=order.device)
        else:
            labels = np.empty(graph.n, dtype=np.int32)
    pl, ldev, _kl = _ptr(labels, np.int32)
    flags = (CC_INPUT_ON_DEVICE if odev else 0) | (CC_OUTPUT_ON_DEVICE if ldev else 0)
    st = _RunStats()
    st.async_waves = int(waves)
    _check(fn(graph.handle, po, pl, ctypes.byref(st), flags, _stream(stream, order, labels)))
    return labels, RunStats(scanned_elect=st.scanned_elect, scanned_claim=st.scanned_claim, atomics=st.atomics,
                            loop_ms=st.loop_ms)


def cc_c4_async(graph: Graph, order, labels=None, waves: int = 0, stream=None):
    """Asynchronous C4 (Algorithm 3): KwikCluster's labels, no rounds.  Returns (labels, RunStats)."""
    return _run_async(_lib.cc_c4_async, graph, order, labels, waves, stream)


def cc_clusterwild_async(graph: Graph, order, labels=None, waves: int = 0, stream=None):
    """Asynchronous ClusterWild! (Algorithm 3); waves=1 makes the interleaving reproducible."""
    return _run_async(_lib.cc_clusterwild_async, graph, order, labels, waves, stream)


def cc_cost(graph: Graph, labels, stream=None) -> np.ndarray:
    """Disagreements per graph (int64[num_graphs])."""
    pl, ldev, _k = _ptr(labels, np.int32)
    out = np.zeros(graph.num_graphs, dtype=np.int64)
    _check(_lib.cc_cost(graph.handle, pl, ctypes.c_void_p(out.ctypes.data),
                        CC_INPUT_ON_DEVICE if ldev else 0, _stream(stream, labels)))
    return out


@dataclass
class BatchConfig:
    block: int
    wave_max_n: int
    quad_max_n: int = 0
    ms: float = 0.0


def cc_batch_set_config(graph: Graph, block: int, wave_max_n: int, quad_max_n: int = 0):
    """Fix a batch's launch shape: `block` threads per workgroup, graphs of at
    most `wave_max_n` vertices one per wave, then (block >= 512) graphs of at
    most `quad_max_n` vertices one per 4-wave sub-group."""
    c = _BatchConfig(int(block), int(wave_max_n), int(quad_max_n), 0, 0.0)
    _check(_lib.cc_batch_set_config(graph.handle, ctypes.byref(c)))


def cc_batch_autotune(graph: Graph, order, algo: int = CC_ALGO_C4, eps: float = 0.5, stream=None) -> BatchConfig:
    """Time every launch shape that fits on this batch and keep the fastest."""
    po, odev, _ko = _ptr(order, np.int32)
    c = _BatchConfig()
    _check(_lib.cc_batch_autotune(graph.handle, int(algo), po, float(eps), CC_INPUT_ON_DEVICE if odev else 0,
                                  _stream(stream, order), ctypes.byref(c)))
    return BatchConfig(c.block, c.wave_max_n, c.quad_max_n, c.ms)


def _dev(t, name):
    if t is None:
        return None
    if not (_is_torch(t) and t.is_cuda and str(t.dtype) == "torch.float32" and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def cc_mlp_forward(params, x, y=None, stream=None):
    """Network outputs for x[n, 6] (device tensors).  Returns y[n]."""
    import torch
    n = x.shape[0]
    if y is None:
        y = torch.empty(n, dtype=torch.float32, device=x.device)
    _check(_lib.cc_mlp_forward(_dev(params, "params"), _dev(x, "x"), n, _dev(y, "y"), _stream(stream, x)))
    return y


def cc_mlp_train_step(params, adam_m, adam_v, x, target, step: int, lr: float, grad=None, loss=None, stream=None):
    """Gradient of mean((y - target)^2) and, if lr > 0, one Adam step in place
    (device tensors).  grad / loss, when given, receive the gradient and loss."""
    n = x.shape[0]
    _check(_lib.cc_mlp_train_step(_dev(params, "params"), _dev(adam_m, "adam_m"), _dev(adam_v, "adam_v"),
                                  _dev(x, "x"), _dev(target, "target"), n, int(step), float(lr),
                                  _dev(grad, "grad"), _dev(loss, "loss"), _stream(stream, x)))


def cc_mlp_train_step_noalloc(params, adam_m, adam_v, x, target, step: int, lr: float, grad=None, loss=None,
                              stream=None):
    """cc_mlp_train_step with the library's static device buffer: allocates nothing."""
    n = x.shape[0]
    _check(_lib.cc_mlp_train_step_noalloc(_dev(params, "params"), _dev(adam_m, "adam_m"), _dev(adam_v, "adam_v"),
                                          _dev(x, "x"), _dev(target, "target"), n, int(step), float(lr),
                                          _dev(grad, "grad"), _dev(loss, "loss"), _stream(stream, x)))


def cc_set_eps_policy(kind: int, params=None, eps_min: float = 1.0 / 16, eps_max: float = 16.0):
    """Process-wide epsilon policy: FIXED, LEARNED (float32 MLP weights), TRACE
    (int64 schedule) or BINOMIAL (params = (seed, delta): the practical schedule)."""
    if kind == CC_EPS_BINOMIAL:
        seed, delta = params
        bp = _BinomialParams(int(seed), float(delta))
        _check(_lib.cc_set_eps_policy(kind, ctypes.byref(bp), ctypes.sizeof(bp), float(eps_min), float(eps_max)))
        return
    if kind == CC_EPS_LEARNED:
        a = np.ascontiguousarray(params, dtype=np.float32)
    elif kind == CC_EPS_TRACE:
        a = np.ascontiguousarray(params, dtype=np.int64)
    else:
        a = None
    p = ctypes.c_void_p(a.ctypes.data) if a is not None else None
    nbytes = a.nbytes if a is not None else 0
    _check(_lib.cc_set_eps_policy(kind, p, nbytes, float(eps_min), float(eps_max)))


def cc_binomial_schedule(n: int, delta0: int, eps: float, seed: int, delta: float = 0.1):
    """(B_0, B_1, ... as int64, K): the practical schedule the library draws."""
    rounds, period = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.cc_binomial_schedule(n, delta0, float(eps), int(seed), float(delta), None, 0,
                                     ctypes.byref(rounds), ctypes.byref(period)))
    out = np.zeros(max(rounds.value, 1), dtype=np.int64)
    _check(_lib.cc_binomial_schedule(n, delta0, float(eps), int(seed), float(delta),
                                     ctypes.c_void_p(out.ctypes.data), rounds.value, None, None))
    return out[:rounds.value], period.value
