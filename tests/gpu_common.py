"""Shared helpers of the GPU tests: device upload and oracle comparison."""
import numpy as np

import oracle

TRACE_INT_FIELDS = ("n_i", "delta_i", "b_i", "r_i", "centers", "claimed", "conflicts")


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def upload(g, validate=True, device=True):
    import paper_1507_05086_amd as cc
    if device:
        torch = torch_cuda()
        off = torch.from_numpy(np.ascontiguousarray(g.off)).cuda()
        col = torch.from_numpy(np.ascontiguousarray(g.col) if g.nnz else np.zeros(1, np.int32)).cuda()
        return cc.cc_graph_from_csr(off, col[: g.nnz] if g.nnz else col[:0], vtx_ptr=g.vtx_ptr,
                                    validate=validate)
    return cc.cc_graph_from_csr(g.off, g.col, vtx_ptr=g.vtx_ptr, validate=validate)


def run_gpu(algo, gh, order, eps, device=True, trace_capacity=1 << 16):
    import paper_1507_05086_amd as cc
    fn = cc.cc_c4 if algo == oracle.C4 else cc.cc_clusterwild
    if device:
        torch = torch_cuda()
        o = torch.from_numpy(np.ascontiguousarray(order)).cuda()
        lab, st = fn(gh, o, eps, trace_capacity=trace_capacity)
        torch.cuda.synchronize()
        return lab.cpu().numpy(), st
    lab, st = fn(gh, np.ascontiguousarray(order), eps, trace_capacity=trace_capacity)
    return lab, st


def assert_trace_equal(gpu_trace, orc_trace, rounds):
    assert len(gpu_trace) == rounds == len(orc_trace)
    for f in TRACE_INT_FIELDS:
        a = np.asarray(gpu_trace[f], dtype=np.int64)
        b = np.asarray(orc_trace[f], dtype=np.int64)
        if not np.array_equal(a, b):
            i = int(np.flatnonzero(a != b)[0])
            raise AssertionError(f"trace field {f} differs first at round {i}: gpu {a[i]} oracle {b[i]}")


def assert_labels_equal(gpu, ref, what=""):
    if not np.array_equal(gpu, ref):
        bad = np.flatnonzero(gpu != ref)
        raise AssertionError(f"{what}: {len(bad)} labels differ, first at v={bad[0]}: "
                             f"gpu {gpu[bad[0]]} oracle {ref[bad[0]]}")


def check_against_oracle(algo, g, gh, order, eps, device=True, cost=True):
    import paper_1507_05086_amd as cc
    ref = oracle.bsp(algo, g.off, g.col, order, eps)
    lab, st = run_gpu(algo, gh, order, eps, device=device)
    name = "C4" if algo == oracle.C4 else "CW"
    assert_labels_equal(lab, ref.labels, f"{name} eps={eps}")
    assert st.rounds == ref.rounds
    assert_trace_equal(st.trace, ref.trace, ref.rounds)
    if cost:
        assert int(cc.cc_cost(gh, lab)[0]) == oracle.cost(g.off, g.col, ref.labels)
    return lab, st, ref
