"""GPU parity of the batched path: many small graphs in one persistent launch.

Every graph of the batch is compared with the oracle run on that graph alone:
labels (local center ids) and rounds must match exactly, for C4 and
ClusterWild!, for launch shapes that put graphs on whole workgroups, on single
waves, and both.  Batches have the planted-block shape of the batched
workload (lognormal sizes in [50, 5000], 2-40 blocks, p_in = 0.3,
p_out = 0.01) plus degenerate members.
"""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_common import assert_labels_equal, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cc():
    torch_cuda()
    import paper_1507_05086_amd as cc
    cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
    return cc


def split(g):
    """Per-graph (off, col) with offsets rebased to 0."""
    out = []
    for i in range(g.ngraphs):
        a, b = int(g.vtx_ptr[i]), int(g.vtx_ptr[i + 1])
        off = np.asarray(g.off[a:b + 1], dtype=np.int64)
        out.append((off - off[0], np.asarray(g.col[off[0]:off[-1]], dtype=np.int32)))
    return out


def stack(graphs):
    """One batch from single graphs (local column ids kept)."""
    ns = [h.n for h in graphs]
    vtx = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    offs, base = [np.zeros(1, np.int64)], 0
    for h in graphs:
        offs.append(np.asarray(h.off[1:], np.int64) + base)
        base += h.nnz
    off = np.concatenate(offs)
    col = np.concatenate([np.asarray(h.col, np.int32) for h in graphs]) if base else np.zeros(0, np.int32)
    return graphgen.Graph(n=int(vtx[-1]), off=off, col=col, vtx_ptr=vtx)


def upload_batch(cc, g):
    torch = torch_cuda()
    off = torch.from_numpy(np.ascontiguousarray(g.off)).cuda()
    col = torch.from_numpy(np.ascontiguousarray(g.col) if g.nnz else np.zeros(1, np.int32)).cuda()
    return cc.cc_graph_from_csr(off, col[: g.nnz], vtx_ptr=g.vtx_ptr, validate=True)


def run_batch(cc, algo, gh, order, eps):
    torch = torch_cuda()
    fn = cc.cc_c4 if algo == oracle.C4 else cc.cc_clusterwild
    lab, st = fn(gh, torch.from_numpy(order).cuda(), eps)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), st


def check_batch(cc, algo, g, gh, order, eps, parts=None):
    lab, st = run_batch(cc, algo, gh, order, eps)
    parts = parts or split(g)
    name = "C4" if algo == oracle.C4 else "CW"
    max_rounds = 0
    for i, (off, col) in enumerate(parts):
        a, b = int(g.vtx_ptr[i]), int(g.vtx_ptr[i + 1])
        ref = oracle.bsp(algo, off, col, order[a:b], eps)
        assert_labels_equal(lab[a:b], ref.labels, f"{name} graph {i} (n={b - a}) eps={eps}")
        assert st.graph_rounds[i] == ref.rounds, f"graph {i}: rounds {st.graph_rounds[i]} vs {ref.rounds}"
        max_rounds = max(max_rounds, ref.rounds)
    assert st.rounds == max_rounds
    return lab, st


def sbm(ngraphs, seed, nmax=5000):
    sizes, blocks = graphgen.sbm_shapes(ngraphs, seed, nmax=nmax)
    return graphgen.sbm_batch(sizes, blocks, 0.3, 0.01, seed)


# (block, wave_max_n[, quad_max_n]); every shape fits 160 KB of LDS for graphs up
# to 5000 vertices (four 4-wave sub-groups of a 1024 workgroup hold <= ~1900 each)
SHAPES = [(256, 0), (1024, 0), (256, 1500), (512, 300), (1024, 400), (256, 128),
          (512, 256, 2048), (1024, 200, 1500), (512, 0, 3000), (1024, 0, 1800)]


@pytest.fixture(scope="module")
def sbm200(cc):
    g = sbm(200, 5)
    return g, upload_batch(cc, g), split(g), graphgen.batch_permutations(g.vtx_ptr, 5)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
def test_sbm_shapes(cc, sbm200, shape, algo):
    g, gh, parts, order = sbm200
    cc.cc_batch_set_config(gh, *shape)
    check_batch(cc, algo, g, gh, order, 0.5, parts)


@pytest.mark.parametrize("eps", [0.1, 0.9, 4.0])
@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
def test_sbm_eps(cc, sbm200, eps, algo):
    g, gh, parts, order = sbm200
    cc.cc_batch_set_config(gh, 512, 256)
    check_batch(cc, algo, g, gh, order, eps, parts)


def test_c4_batch_is_kwikcluster_and_cost(cc, sbm200):
    g, gh, parts, order = sbm200
    cc.cc_batch_set_config(gh, 256, 256)
    lab, _ = run_batch(cc, oracle.C4, gh, order, 0.5)
    costs = cc.cc_cost(gh, lab)
    for i, (off, col) in enumerate(parts):
        a, b = int(g.vtx_ptr[i]), int(g.vtx_ptr[i + 1])
        kc = oracle.kwikcluster(off, col, order[a:b])
        assert_labels_equal(lab[a:b], kc, f"graph {i} vs KwikCluster")
        assert int(costs[i]) == oracle.cost(off, col, kc)


def _complete(n):
    return graphgen.from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def test_degenerate_members(cc):
    members = [graphgen.from_edges(0, []), graphgen.from_edges(1, []), graphgen.from_edges(2, [(0, 1)]),
               graphgen.from_edges(700, []), _complete(90), graphgen.erdos_renyi(3000, 12.0, seed=3),
               graphgen.from_edges(0, []), graphgen.from_edges(4000, [(0, i) for i in range(1, 4000)]),
               graphgen.from_edges(65, [(i, i + 1) for i in range(64)]), graphgen.from_edges(1, [])]
    g = stack(members)
    gh = upload_batch(cc, g)
    order = graphgen.batch_permutations(g.vtx_ptr, 9)
    for shape in ((256, 0), (1024, 100), (256, 1000), (1024, 100, 1500), (512, 0, 3100)):
        cc.cc_batch_set_config(gh, *shape)
        for algo in (oracle.C4, oracle.CW):
            for eps in (0.5, 0.05, 20.0):
                check_batch(cc, algo, g, gh, order, eps)


@pytest.mark.parametrize("block", [256, 1024])
def test_all_on_waves(cc, block):
    g = sbm(500, 29, nmax=400)
    gh = upload_batch(cc, g)
    order = graphgen.batch_permutations(g.vtx_ptr, 29)
    cc.cc_batch_set_config(gh, block, cc.CC_BATCH_MAX_N)
    for algo in (oracle.C4, oracle.CW):
        check_batch(cc, algo, g, gh, order, 0.5)


def test_largest_member(cc):
    big = graphgen.erdos_renyi(cc.CC_BATCH_MAX_N, 30.0, seed=4)
    g = stack([big, graphgen.erdos_renyi(500, 8.0, seed=5), big])
    gh = upload_batch(cc, g)
    order = graphgen.batch_permutations(g.vtx_ptr, 4)
    for shape in ((1024, 0), (256, 600), (512, 400, 600)):
        cc.cc_batch_set_config(gh, *shape)
        for algo in (oracle.C4, oracle.CW):
            check_batch(cc, algo, g, gh, order, 0.5)


def test_autotune_then_run(cc):
    g = sbm(300, 17)
    gh = upload_batch(cc, g)
    order = graphgen.batch_permutations(g.vtx_ptr, 17)
    torch = torch_cuda()
    best = cc.cc_batch_autotune(gh, torch.from_numpy(order).cuda(), cc.CC_ALGO_C4, 0.5)
    assert best.block in (256, 512, 1024) and best.wave_max_n >= 0 and best.quad_max_n >= 0 and best.ms > 0
    check_batch(cc, oracle.C4, g, gh, order, 0.5)
    # a new handle of the same size class picks the tuned shape up
    gh2 = upload_batch(cc, g)
    check_batch(cc, oracle.CW, g, gh2, order, 0.5)


def test_batch_errors(cc):
    torch = torch_cuda()
    g = sbm(20, 23, nmax=800)
    gh = upload_batch(cc, g)
    order = graphgen.batch_permutations(g.vtx_ptr, 23)
    bad = order.copy()
    a = int(g.vtx_ptr[7])
    bad[a + 1] = bad[a + 2]  # graph 7 is no longer a permutation
    out = torch.full((g.n,), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(cc.CCError) as ei:
        cc.cc_c4(gh, torch.from_numpy(bad).cuda(), 0.5, labels=out)
    assert ei.value.code == cc.CC_ERR_NOT_PERMUTATION
    assert bool((out == -7).all())
    with pytest.raises(cc.CCError) as ei:
        cc.cc_batch_set_config(gh, 300, 0)
    assert ei.value.code == cc.CC_ERR_INVALID_ARG
    cc.cc_set_eps_policy(cc.CC_EPS_TRACE, np.array([5], np.int64))
    try:
        with pytest.raises(cc.CCError) as ei:
            cc.cc_clusterwild(gh, order, 0.5)
        assert ei.value.code == cc.CC_ERR_POLICY
    finally:
        cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
    too_big = stack([graphgen.from_edges(cc.CC_BATCH_MAX_N + 1, []), graphgen.from_edges(3, [])])
    gb = upload_batch(cc, too_big)
    with pytest.raises(cc.CCError) as ei:
        cc.cc_c4(gb, graphgen.batch_permutations(too_big.vtx_ptr, 1), 0.5)
    assert ei.value.code == cc.CC_ERR_INVALID_ARG


@pytest.fixture(scope="module")
def sbm4096(cc):
    g = graphgen.workload("sbm4096")
    return g, upload_batch(cc, g), split(g), graphgen.batch_permutations(g.vtx_ptr, 4096)


# the default shape, then shapes the autotuner picked for this workload
FULL_SHAPES = [None, (1024, 384, 1792), (1024, 256, 1792), (512, 256, 2048)]


@pytest.mark.parametrize("shape", FULL_SHAPES)
def test_batched_workload_full(cc, sbm4096, shape):
    """The batched workload at full size: 4096 planted-block graphs, with the
    default launch shape and the autotuned ones the benchmark runs."""
    g, gh, parts, order = sbm4096
    if shape is not None:
        cc.cc_batch_set_config(gh, *shape)
    for algo in (oracle.C4, oracle.CW):
        check_batch(cc, algo, g, gh, order, 0.5, parts)


def test_batched_workload_autotuned(cc, sbm4096):
    """Whatever shape the autotuner picks on this device is checked too."""
    g, gh, parts, order = sbm4096
    for algo in (oracle.C4, oracle.CW):
        best = cc.cc_batch_autotune(gh, order, algo, 0.5)
        assert best.block in (256, 512, 1024) and best.ms > 0
        check_batch(cc, algo, g, gh, order, 0.5, parts)
