"""GPU parity of the paper's practical schedule (Delta-hat halving and
Binomial batches over pi positions; policy CC_EPS_BINOMIAL) against the
oracle's round loop with the same schedule: labels, round count and every
trace field, bit for bit.  C4's labels must still be KwikCluster's."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_common import assert_labels_equal, assert_trace_equal, run_gpu, torch_cuda, upload

pytestmark = pytest.mark.gpu

DELTA = 0.1


@pytest.fixture(scope="module")
def cc():
    torch_cuda()
    import paper_1507_05086_amd as cc
    return cc


@pytest.fixture(autouse=True)
def fixed_after(cc):
    yield
    cc.cc_set_eps_policy(cc.CC_EPS_FIXED)


def check(cc, algo, g, gh, order, eps, seed):
    cc.cc_set_eps_policy(cc.CC_EPS_BINOMIAL, (seed, DELTA))
    ref = oracle.bsp_binomial(algo, g.off, g.col, order, eps, seed=seed, delta=DELTA)
    lab, st = run_gpu(algo, gh, order, eps)
    name = ("C4" if algo == oracle.C4 else "CW") + f" binomial eps={eps} seed={seed}"
    assert_labels_equal(lab, ref.labels, name)
    assert st.rounds == ref.rounds, name
    assert not st.truncated
    assert_trace_equal(st.trace, ref.trace, ref.rounds)
    assert int(cc.cc_cost(gh, lab)[0]) == oracle.cost(g.off, g.col, ref.labels)
    if algo == oracle.C4:
        assert_labels_equal(lab, oracle.kwikcluster(g.off, g.col, order), "C4 binomial vs KwikCluster")
    return lab, st, ref


FAMILIES = {
    "er20k": lambda: graphgen.workload("er20k"),
    "chunglu": lambda: graphgen.chung_lu(200_000, 2.1, 20.0, seed=7),
    "rmat16": lambda: graphgen.rmat(16, 16, 0.57, 0.19, 0.19, seed=8),
    "er_dense": lambda: graphgen.erdos_renyi(5_000, 60.0, seed=9),
}


@pytest.mark.parametrize("fam", list(FAMILIES))
@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
@pytest.mark.parametrize("eps", [0.1, 0.5, 0.9])
def test_families(cc, fam, algo, eps):
    g = FAMILIES[fam]()
    gh = upload(g)
    order = graphgen.permutation(g.n, 21)
    check(cc, algo, g, gh, order, eps, seed=101)


EDGE_CASES = {
    "single": lambda: graphgen.from_edges(1, []),
    "pair": lambda: graphgen.from_edges(2, [(0, 1)]),
    "edgeless": lambda: graphgen.from_edges(5000, []),
    "complete60": lambda: graphgen.from_edges(60, [(i, j) for i in range(60) for j in range(i + 1, 60)]),
    "star100k": lambda: graphgen.from_edges(100_001, [(0, i) for i in range(1, 100_001)]),
    "path3000": lambda: graphgen.from_edges(3000, [(i, i + 1) for i in range(2999)]),
    "isolated_mix": lambda: graphgen.from_edges(9000, [(i, i + 1) for i in range(0, 3000, 2)]),
}


@pytest.mark.parametrize("case", list(EDGE_CASES))
@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
def test_edge_cases(cc, case, algo):
    g = EDGE_CASES[case]()
    gh = upload(g)
    for seed, eps in ((1, 0.5), (2, 0.05), (3, 20.0)):
        order = graphgen.permutation(g.n, seed)
        check(cc, algo, g, gh, order, eps, seed=seed)


def test_seeds_and_cached_schedule(cc):
    """Repeated calls reuse the drawn schedule; another seed draws another one
    (ClusterWild!'s labels follow it, C4's do not)."""
    g = graphgen.chung_lu(100_000, 2.1, 12.0, seed=33)
    gh = upload(g)
    order = graphgen.permutation(g.n, 33)
    a1, s1, _ = check(cc, oracle.CW, g, gh, order, 0.5, seed=5)
    a2, s2, _ = check(cc, oracle.CW, g, gh, order, 0.5, seed=5)
    assert np.array_equal(a1, a2) and np.array_equal(s1.trace["b_i"], s2.trace["b_i"])
    b1, t1, _ = check(cc, oracle.CW, g, gh, order, 0.5, seed=6)
    assert not np.array_equal(s1.trace["b_i"], t1.trace["b_i"])
    c5, _, _ = check(cc, oracle.C4, g, gh, order, 0.5, seed=5)
    c6, _, _ = check(cc, oracle.C4, g, gh, order, 0.5, seed=6)
    assert np.array_equal(c5, c6)
    # back to the fixed rule on the same handle: the exact-Delta loop again
    cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
    ref = oracle.bsp(oracle.CW, g.off, g.col, order, 0.5)
    lab, st = run_gpu(oracle.CW, gh, order, 0.5)
    assert_labels_equal(lab, ref.labels, "fixed rule after the practical schedule")
    assert_trace_equal(st.trace, ref.trace, ref.rounds)


@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
def test_random_sweep(cc, algo):
    """Seeded cases: graph family, size, order, eps and schedule seed."""
    rng = np.random.default_rng(77 + algo)
    for i in range(24):
        n = int(rng.integers(1, 6000))
        kind = i % 3
        if kind == 0:
            g = graphgen.erdos_renyi(n, float(rng.uniform(0.2, 15.0)), seed=500 + i)
        elif kind == 1:
            g = graphgen.chung_lu(n, float(rng.uniform(1.9, 2.8)), float(rng.uniform(1.0, 20.0)), seed=500 + i)
        else:
            g = graphgen.rmat(max(1, int(np.log2(n))), int(rng.integers(1, 16)), 0.57, 0.19, 0.19, seed=500 + i)
        eps = float(np.exp(rng.uniform(np.log(0.05), np.log(8.0))))
        gh = upload(g)
        check(cc, algo, g, gh, graphgen.permutation(g.n, 600 + i), eps, seed=int(rng.integers(0, 2**62)))


@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
def test_partial_runs(cc, algo):
    g = graphgen.chung_lu(40_000, 2.1, 12.0, seed=52)
    gh = upload(g)
    order = graphgen.permutation(g.n, 52)
    _, stf, _ = check(cc, algo, g, gh, order, 0.5, seed=9)
    fn = cc.cc_c4 if algo == oracle.C4 else cc.cc_clusterwild
    full, _ = fn(gh, order, 0.5)
    for k in (1, stf.rounds // 3, stf.rounds - 1):
        lab, st = fn(gh, order, 0.5, max_rounds=k)
        assert st.rounds == k
        for f in ("n_i", "delta_i", "b_i", "r_i", "centers", "claimed", "conflicts"):
            assert np.array_equal(st.trace[f], stf.trace[f][:k])
        done = lab >= 0
        assert np.array_equal(lab[done], full[done])
        assert int((~done).sum()) == int(stf.trace["n_i"][k])


def test_batches_reject_the_practical_schedule(cc):
    g1, g2 = graphgen.from_edges(5, [(0, 1)]), graphgen.from_edges(4, [(1, 2)])
    off = np.concatenate([g1.off, g2.off[1:] + g1.off[-1]])
    col = np.concatenate([g1.col, g2.col])
    gh = cc.cc_graph_from_csr(off, col, vtx_ptr=np.array([0, 5, 9], np.int64))
    cc.cc_set_eps_policy(cc.CC_EPS_BINOMIAL, (1, DELTA))
    with pytest.raises(cc.CCError) as ei:
        cc.cc_c4(gh, np.array([0, 1, 2, 3, 4, 0, 1, 2, 3], np.int32), 0.5)
    assert ei.value.code == cc.CC_ERR_POLICY
