"""Parity at the full sizes of the two large single-graph workloads, in the
launch configuration the benchmark times (graph, order and labels resident on
the device, fixed rule).

- Chung-Lu power law, n = 2,000,000, gamma = 2.1, mean degree 40 (about 40 M
  positive edges): labels and the whole round trace against the oracle for
  C4 and ClusterWild! at eps 0.1, 0.5 and 0.9 (order 21), and at eps 0.5 for
  orders 22-25.
- R-MAT scale 26 (about 1.05 G positive edges), eps = 0.5, orders 31-33:
  labels, round count and every trace field against the oracle's round loop
  for C4 and ClusterWild!, C4's labels also by the any-size KwikCluster
  checker, and the cost; and both algorithms under the paper's practical
  schedule (Delta-hat halving, Binomial batches over pi positions) against
  the oracle's loop with the same schedule.
"""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_common import assert_labels_equal, assert_trace_equal, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cc():
    torch_cuda()
    import paper_1507_05086_amd as cc
    cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
    return cc


def resident(cc, g, seed):
    torch = torch_cuda()
    off = torch.from_numpy(np.ascontiguousarray(g.off)).cuda()
    col = torch.from_numpy(np.ascontiguousarray(g.col)).cuda()
    gh = cc.cc_graph_from_csr(off, col, borrow=True)
    order = graphgen.permutation(g.n, seed)
    return gh, (off, col), order, torch.from_numpy(order).cuda()


def run(cc, algo, gh, dorder, eps):
    torch = torch_cuda()
    fn = cc.cc_c4 if algo == oracle.C4 else cc.cc_clusterwild
    lab = torch.empty(dorder.numel(), dtype=torch.int32, device="cuda")
    _, st = fn(gh, dorder, eps, labels=lab, trace_capacity=1 << 16)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), st


@pytest.fixture(scope="module")
def chunglu(cc):
    g = graphgen.workload("chunglu2m")
    return (g, *resident(cc, g, 21))


@pytest.mark.timeout(300)
@pytest.mark.parametrize("eps", [0.1, 0.5, 0.9])
@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
def test_chunglu_2m(cc, chunglu, algo, eps):
    g, gh, _keep, order, dorder = chunglu
    lab, st = run(cc, algo, gh, dorder, eps)
    ref = oracle.bsp(algo, g.off, g.col, order, eps)
    assert_labels_equal(lab, ref.labels, f"Chung-Lu 2M eps={eps}")
    assert st.rounds == ref.rounds
    assert_trace_equal(st.trace, ref.trace, ref.rounds)
    if algo == oracle.C4:
        assert oracle.check_kc(g.off, g.col, order, lab) == (0, -1)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("seed", [22, 23, 24, 25])
@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
def test_chunglu_2m_orders(cc, chunglu, algo, seed):
    g, gh, _keep, _order, _dorder = chunglu
    order = graphgen.permutation(g.n, seed)
    lab, st = run(cc, algo, gh, torch_cuda().from_numpy(order).cuda(), 0.5)
    ref = oracle.bsp(algo, g.off, g.col, order, 0.5)
    assert_labels_equal(lab, ref.labels, f"Chung-Lu 2M order {seed}")
    assert st.rounds == ref.rounds
    assert_trace_equal(st.trace, ref.trace, ref.rounds)


@pytest.fixture(scope="module")
def rmat26(cc):
    torch = torch_cuda()
    g = graphgen.workload("rmat26")
    off = torch.from_numpy(np.ascontiguousarray(g.off)).cuda()
    col = torch.from_numpy(np.ascontiguousarray(g.col)).cuda()
    gh = cc.cc_graph_from_csr(off, col, borrow=True)
    return g, gh, (off, col)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("seed", [31, 32, 33])
@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
def test_rmat26(cc, rmat26, algo, seed):
    g, gh, _keep = rmat26
    order = graphgen.permutation(g.n, seed)
    name = ("C4" if algo == oracle.C4 else "ClusterWild!") + f" on R-MAT 26, order {seed}"
    print(f"{name}: GPU run", flush=True)
    lab, st = run(cc, algo, gh, torch_cuda().from_numpy(order).cuda(), 0.5)
    print(f"{name}: oracle run", flush=True)
    ref = oracle.bsp(algo, g.off, g.col, order, 0.5)
    assert_labels_equal(lab, ref.labels, name)
    assert st.rounds == ref.rounds
    assert_trace_equal(st.trace, ref.trace, ref.rounds)
    if algo == oracle.C4:
        bad, first = oracle.check_kc(g.off, g.col, order, lab)
        assert bad == 0, f"{name}: {bad} vertices break KwikCluster, first {first}"
    assert int(cc.cc_cost(gh, lab)[0]) == oracle.cost(g.off, g.col, ref.labels)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
def test_rmat26_practical_schedule(cc, rmat26, algo):
    g, gh, _keep = rmat26
    order = graphgen.permutation(g.n, 31)
    name = ("C4" if algo == oracle.C4 else "ClusterWild!") + " on R-MAT 26, practical schedule"
    cc.cc_set_eps_policy(cc.CC_EPS_BINOMIAL, (31, 0.1))
    try:
        print(f"{name}: GPU run", flush=True)
        lab, st = run(cc, algo, gh, torch_cuda().from_numpy(order).cuda(), 0.5)
    finally:
        cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
    print(f"{name}: oracle run", flush=True)
    ref = oracle.bsp_binomial(algo, g.off, g.col, order, 0.5, seed=31, delta=0.1)
    assert_labels_equal(lab, ref.labels, name)
    assert st.rounds == ref.rounds
    assert_trace_equal(st.trace, ref.trace, ref.rounds)


@pytest.mark.timeout(600)
def test_rmat26_async(cc, rmat26):
    """Asynchronous C4 gives KwikCluster's labels on R-MAT 26; asynchronous
    ClusterWild! gives a clustering whose every label is a center, with its
    objective counted right."""
    torch = torch_cuda()
    g, gh, _keep = rmat26
    order = graphgen.permutation(g.n, 31)
    dorder = torch.from_numpy(order).cuda()
    print("async C4 on R-MAT 26: GPU run", flush=True)
    lab, st = cc.cc_c4_async(gh, dorder)
    torch.cuda.synchronize()
    lab = lab.cpu().numpy()
    print(f"  {st.loop_ms:.2f} ms; KwikCluster on the CPU", flush=True)
    assert_labels_equal(lab, oracle.kwikcluster(g.off, g.col, order), "async C4 on R-MAT 26")
    kc_cost = oracle.cost(g.off, g.col, lab)
    print("async ClusterWild! on R-MAT 26: GPU run", flush=True)
    labw, stw = cc.cc_clusterwild_async(gh, dorder)
    torch.cuda.synchronize()
    labw = labw.cpu().numpy()
    assert ((labw >= 0) & (labw < g.n)).all() and (labw[labw] == labw).all()
    cw_cost = int(cc.cc_cost(gh, labw)[0])
    assert cw_cost == oracle.cost(g.off, g.col, labw)
    print(f"  {stw.loop_ms:.2f} ms; cost {cw_cost} vs KwikCluster {kc_cost}", flush=True)
    # with the device full, millions of vertices are in flight at once and
    # rule 1 is broken often: the objective is unpinned, this only guards
    # against nonsense (it was 2.7 times KwikCluster's when measured)
    assert kc_cost / 4 < cw_cost < 5 * kc_cost
