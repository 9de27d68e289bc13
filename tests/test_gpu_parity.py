"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Labels, round traces and costs are integer results and must match exactly.
Sizes span many scan tiles and edge tiles with ragged tails; the graph
families have the shapes of the workloads (Erdos-Renyi, power-law Chung-Lu,
R-MAT with hubs, planted blocks) plus the degenerate cases.
"""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_common import (assert_labels_equal, check_against_oracle, run_gpu, torch_cuda, upload)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cc():
    torch_cuda()
    import paper_1507_05086_amd as cc
    return cc


@pytest.fixture(autouse=True)
def fixed_policy(cc):
    cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
    yield
    cc.cc_set_eps_policy(cc.CC_EPS_FIXED)


# ------------------------------------------- the small workload (ER 20k)

@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
@pytest.mark.parametrize("eps", [0.1, 0.5, 0.9])
def test_er20k(cc, algo, eps):
    g = graphgen.workload("er20k")
    gh = upload(g)
    for seed in (11, 12, 13):
        order = graphgen.permutation(g.n, seed)
        lab, _, _ = check_against_oracle(algo, g, gh, order, eps)
        if algo == oracle.C4:
            assert_labels_equal(lab, oracle.kwikcluster(g.off, g.col, order), "C4 vs KwikCluster")


@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
def test_er20k_host_buffers(cc, algo):
    g = graphgen.workload("er20k")
    gh = upload(g, device=False)
    order = graphgen.permutation(g.n, 14)
    check_against_oracle(algo, g, gh, order, 0.5, device=False)


# ------------------------------------------------------ graph families

FAMILIES = {
    "chunglu": lambda: graphgen.chung_lu(200_000, 2.1, 20.0, seed=7),
    "rmat16": lambda: graphgen.rmat(16, 16, 0.57, 0.19, 0.19, seed=8),
    "er_dense": lambda: graphgen.erdos_renyi(5_000, 60.0, seed=9),
}


@pytest.mark.parametrize("fam", list(FAMILIES))
@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
@pytest.mark.parametrize("eps", [0.1, 0.5, 0.9, 4.0])
def test_families(cc, fam, algo, eps):
    g = FAMILIES[fam]()
    gh = upload(g)
    order = graphgen.permutation(g.n, 21)
    check_against_oracle(algo, g, gh, order, eps)


# --------------------------------------------------------- edge cases

def _cliques(sizes):
    edges, base = [], 0
    for s in sizes:
        edges += [(base + i, base + j) for i in range(s) for j in range(i + 1, s)]
        base += s
    return graphgen.from_edges(base, edges)


EDGE_CASES = {
    "single": lambda: graphgen.from_edges(1, []),
    "pair": lambda: graphgen.from_edges(2, [(0, 1)]),
    "edgeless": lambda: graphgen.from_edges(5000, []),
    "complete60": lambda: graphgen.from_edges(60, [(i, j) for i in range(60) for j in range(i + 1, 60)]),
    "star100k": lambda: graphgen.from_edges(100_001, [(0, i) for i in range(1, 100_001)]),
    "path3000": lambda: graphgen.from_edges(3000, [(i, i + 1) for i in range(2999)]),
    "cliques": lambda: _cliques([1, 2, 3, 50, 7, 200, 4, 1, 1]),
    "isolated_mix": lambda: graphgen.from_edges(9000, [(i, i + 1) for i in range(0, 3000, 2)]),
}


@pytest.mark.parametrize("case", list(EDGE_CASES))
@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
def test_edge_cases(cc, case, algo):
    g = EDGE_CASES[case]()
    gh = upload(g)
    for seed, eps in ((1, 0.5), (2, 0.05), (3, 20.0)):
        order = graphgen.permutation(g.n, seed)
        check_against_oracle(algo, g, gh, order, eps)


def test_empty_graph(cc):
    g = graphgen.from_edges(0, [])
    gh = cc.cc_graph_from_csr(np.zeros(1, np.int64), np.zeros(0, np.int32))
    lab, st = cc.cc_c4(gh, np.zeros(0, np.int32), 0.5)
    assert len(lab) == 0 and st.rounds == 0
    assert g.n == 0


# ----------------------------------------------------------- schedules

@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
def test_trace_schedule_replay(cc, algo):
    g = graphgen.chung_lu(30_000, 2.1, 12.0, seed=31)
    gh = upload(g)
    order = graphgen.permutation(g.n, 31)
    rng = np.random.default_rng(31)
    sched = rng.integers(1, 4000, size=60).astype(np.int64)
    cc.cc_set_eps_policy(cc.CC_EPS_TRACE, sched)
    ref = oracle.bsp(algo, g.off, g.col, order, 0.5, sched=sched)
    lab, st = run_gpu(algo, gh, order, 0.5)
    assert_labels_equal(lab, ref.labels, "schedule replay")
    assert st.rounds == ref.rounds
    assert np.array_equal(st.trace["b_i"], ref.trace["b_i"])


def test_unit_batches_clusterwild_is_kwikcluster(cc):
    g = graphgen.erdos_renyi(1500, 8.0, seed=5)
    gh = upload(g)
    order = graphgen.permutation(g.n, 5)
    cc.cc_set_eps_policy(cc.CC_EPS_TRACE, np.ones(g.n, dtype=np.int64))
    lab, st = run_gpu(oracle.CW, gh, order, 0.5)
    kc = oracle.kwikcluster(g.off, g.col, order)
    assert_labels_equal(lab, kc, "CW with B=1")
    assert st.rounds == int((kc == np.arange(g.n)).sum())  # one round per KwikCluster center


# ------------------------------------------------------ determinism

def test_repeat_and_streams(cc):
    torch = torch_cuda()
    g = graphgen.rmat(15, 16, 0.57, 0.19, 0.19, seed=41)
    gh = upload(g)
    order = torch.from_numpy(graphgen.permutation(g.n, 41)).cuda()
    outs = []
    for i in range(3):
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            lab, st = cc.cc_clusterwild(gh, order, 0.5)
        s.synchronize()
        outs.append((lab.cpu().numpy(), st.trace["b_i"].copy()))
    for lab, b in outs[1:]:
        assert np.array_equal(lab, outs[0][0]) and np.array_equal(b, outs[0][1])


# ------------------------------------------------ seeded random sweep

def _random_case(i):
    """Case i of a seeded sweep: a graph family, a size from 1 to a few
    thousand vertices (often with many isolated or low-degree vertices; every
    eighth case a power-law graph of 40-80 thousand with hubs), an order and
    an eps drawn log-uniformly from [0.05, 8]."""
    rng = np.random.default_rng(1000 + i)
    n = int(rng.integers(1, 4000))
    kind = i % 4 if i % 8 != 7 else 4
    if kind == 4:  # hubs: the lazy degree search, then the switch to exact degrees
        g = graphgen.chung_lu(int(rng.integers(40_000, 80_000)), float(rng.uniform(2.0, 2.3)),
                              float(rng.uniform(8.0, 16.0)), seed=2000 + i)
    elif kind == 0:
        g = graphgen.erdos_renyi(n, float(rng.uniform(0.2, 12.0)), seed=2000 + i)
    elif kind == 1:
        g = graphgen.chung_lu(n, float(rng.uniform(1.9, 2.8)), float(rng.uniform(1.0, 20.0)), seed=2000 + i)
    elif kind == 2:
        scale = max(1, int(np.log2(n)))
        g = graphgen.rmat(scale, int(rng.integers(1, 16)), 0.57, 0.19, 0.19, seed=2000 + i)
    else:
        g = graphgen.erdos_renyi(n, float(rng.uniform(0.0, 1.5)), seed=2000 + i)  # mostly isolated vertices
    eps = float(np.exp(rng.uniform(np.log(0.05), np.log(8.0))))
    return g, graphgen.permutation(g.n, 3000 + i), eps


@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
def test_random_sweep(cc, algo):
    """Labels, round traces and costs against the oracle over 48 seeded cases
    (every settled-vertex path: isolated, no neighbour left, listed)."""
    for i in range(48):
        g, order, eps = _random_case(i)
        gh = upload(g)
        check_against_oracle(algo, g, gh, order, eps)


# ------------------------------------------------------------ errors

def test_errors_leave_outputs_untouched(cc):
    g = graphgen.erdos_renyi(1000, 5.0, seed=2)
    gh = upload(g, device=False)
    bad = graphgen.permutation(g.n, 2)
    bad[5] = bad[6]
    out = np.full(g.n, -7, dtype=np.int32)
    with pytest.raises(cc.CCError) as ei:
        cc.cc_c4(gh, bad, 0.5, labels=out)
    assert ei.value.code == cc.CC_ERR_NOT_PERMUTATION
    assert (out == -7).all()
    bad[5] = g.n + 3  # out of range
    with pytest.raises(cc.CCError) as ei:
        cc.cc_clusterwild(gh, bad, 0.5, labels=out)
    assert ei.value.code == cc.CC_ERR_NOT_PERMUTATION and (out == -7).all()
    for eps in (0.0, -1.0, float("nan"), 5000.0):
        with pytest.raises(cc.CCError) as ei:
            cc.cc_c4(gh, graphgen.permutation(g.n, 3), eps, labels=out)
        assert ei.value.code == cc.CC_ERR_INVALID_ARG
    # the handle is still good after the rejected calls
    good = graphgen.permutation(g.n, 4)
    lab, _ = cc.cc_c4(gh, good, 0.5)
    assert np.array_equal(lab, oracle.kwikcluster(g.off, g.col, good))


@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
def test_device_outputs_untouched_on_failure(cc, algo):
    """A failure inside the round loop (forced from the host through the
    fault_round test hook: every kernel still exits normally) and a bad
    permutation found on the device both leave a device label buffer as it
    was; the handle keeps working afterwards."""
    torch = torch_cuda()
    g = graphgen.erdos_renyi(20_000, 10.0, seed=6)
    gh = upload(g)
    fn = cc.cc_c4 if algo == oracle.C4 else cc.cc_clusterwild
    order = graphgen.permutation(g.n, 6)
    dorder = torch.from_numpy(order).cuda()
    out = torch.full((g.n,), -7, dtype=torch.int32, device="cuda")
    for k in (1, 2, 5):
        with pytest.raises(cc.CCError) as ei:
            fn(gh, dorder, 0.5, labels=out, fault_round=k)
        assert ei.value.code == cc.CC_ERR_DEVICE
        torch.cuda.synchronize()
        assert bool((out == -7).all())
    bad = order.copy()
    bad[10] = bad[11]
    with pytest.raises(cc.CCError) as ei:
        fn(gh, torch.from_numpy(bad).cuda(), 0.5, labels=out)
    assert ei.value.code == cc.CC_ERR_NOT_PERMUTATION
    torch.cuda.synchronize()
    assert bool((out == -7).all())
    lab, st = fn(gh, dorder, 0.5, labels=out)
    ref = oracle.bsp(algo, g.off, g.col, order, 0.5)
    assert_labels_equal(out.cpu().numpy(), ref.labels, "after the failed calls")
    assert st.rounds == ref.rounds


# ----------------------------------------- settling the blocked vertices

def _path(n):
    return graphgen.from_edges(n, [(i, i + 1) for i in range(n - 1)])


@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
def test_blocked_chain_identity_order(cc, algo):
    """A path with the identity order: round 0's 5000 active vertices form one
    chain of blocked vertices that settles one link at a time."""
    g = _path(20_000)
    gh = upload(g)
    order = np.arange(g.n, dtype=np.int32)
    _, st, ref = check_against_oracle(algo, g, gh, order, 0.5)
    assert ref.trace["conflicts"][0] == ref.trace["b_i"][0] - 1


def test_blocked_many_listed_edges(cc):
    """Half of a dense random graph active at once: about 0.4 M conflict edges,
    settled from the listed edges."""
    g = graphgen.erdos_renyi(30_000, 100.0, seed=12)
    gh = upload(g)
    order = graphgen.permutation(g.n, 12)
    sched = np.array([g.n // 2], dtype=np.int64)
    cc.cc_set_eps_policy(cc.CC_EPS_TRACE, sched)
    ref = oracle.bsp(oracle.C4, g.off, g.col, order, 0.5, sched=sched)
    lab, st = run_gpu(oracle.C4, gh, order, 0.5)
    assert_labels_equal(lab, ref.labels, "C4, half the graph active")
    assert st.rounds == ref.rounds
    assert np.array_equal(st.trace["conflicts"], ref.trace["conflicts"])
    assert np.array_equal(st.trace["centers"], ref.trace["centers"])


@pytest.mark.parametrize("case", ["complete1500", "er30k_d100"])
def test_blocked_too_many_edges_to_list(cc, case):
    """Every vertex active in round 0 gives more conflict edges than the list
    holds (max(n, 2^20)): the blocked vertices are settled by row sweeps."""
    if case == "complete1500":
        n = 1500
        g = graphgen.from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)])
    else:
        g = graphgen.erdos_renyi(30_000, 100.0, seed=13)
    assert g.m > max(g.n, 1 << 20)  # conflict edges of an all-active round = m
    gh = upload(g)
    order = graphgen.permutation(g.n, 13)
    sched = np.array([g.n], dtype=np.int64)
    cc.cc_set_eps_policy(cc.CC_EPS_TRACE, sched)
    ref = oracle.bsp(oracle.C4, g.off, g.col, order, 0.5, sched=sched)
    lab, st = run_gpu(oracle.C4, gh, order, 0.5)
    assert_labels_equal(lab, ref.labels, case)
    assert st.rounds == ref.rounds == 1
    assert np.array_equal(st.trace["conflicts"], ref.trace["conflicts"])
    assert np.array_equal(lab, oracle.kwikcluster(g.off, g.col, order))


@pytest.mark.parametrize("validate", [False, True])
def test_graph_errors(cc, validate):
    off = np.array([0, 1, 2], dtype=np.int64)
    with pytest.raises(cc.CCError) as ei:  # column out of range: always checked
        cc.cc_graph_from_csr(off, np.array([1, 5], np.int32), validate=validate)
    assert ei.value.code == cc.CC_ERR_OUT_OF_RANGE
    with pytest.raises(cc.CCError) as ei:
        cc.cc_graph_from_csr(np.array([0, 2, 1], np.int64), np.array([1, 0], np.int32), validate=validate)
    assert ei.value.code == cc.CC_ERR_INVALID_ARG
    if not validate:
        return
    cases = {
        cc.CC_ERR_NOT_SYMMETRIC: (np.array([0, 1, 1], np.int64), np.array([1], np.int32)),
        cc.CC_ERR_SELF_LOOP: (np.array([0, 2, 3], np.int64), np.array([0, 1, 0], np.int32)),
        cc.CC_ERR_DUPLICATE_EDGE: (np.array([0, 2, 4], np.int64), np.array([1, 1, 0, 0], np.int32)),
    }
    for code, (o, c) in cases.items():
        with pytest.raises(cc.CCError) as ei:
            cc.cc_graph_from_csr(o, c, validate=True)
        assert ei.value.code == code


# --------------------------------------------------------------- cost

def test_cost_arbitrary_labels(cc):
    g = graphgen.chung_lu(50_000, 2.1, 16.0, seed=3)
    gh = upload(g)
    rng = np.random.default_rng(3)
    for k in (1, 7, 1000, g.n):
        lab = rng.integers(0, k, size=g.n).astype(np.int32)
        assert int(cc.cc_cost(gh, lab)[0]) == oracle.cost(g.off, g.col, lab)
    with pytest.raises(cc.CCError):
        cc.cc_cost(gh, np.full(g.n, g.n, np.int32))


@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
def test_partial_run_max_rounds(cc, algo):
    """Stopping after k rounds gives the first k records of the full run; a
    vertex clustered by then already has its final label, the rest get -1."""
    g = graphgen.chung_lu(40_000, 2.1, 12.0, seed=51)
    iso = np.diff(g.off) == 0
    assert iso.sum() > 500  # isolated vertices are settled without a label until the end
    gh = upload(g)
    order = graphgen.permutation(g.n, 51)
    fn = cc.cc_c4 if algo == oracle.C4 else cc.cc_clusterwild
    full, stf = fn(gh, order, 0.5)
    assert np.array_equal(full[iso], np.flatnonzero(iso))  # each its own cluster
    mixed = False
    for k in (1, 3, stf.rounds // 2, stf.rounds - 1, stf.rounds, stf.rounds + 5):
        lab, st = fn(gh, order, 0.5, max_rounds=k)
        kk = min(k, stf.rounds)
        assert st.rounds == kk
        for f in ("n_i", "delta_i", "b_i", "centers", "claimed"):
            assert np.array_equal(st.trace[f], stf.trace[f][:kk])
        done = lab >= 0
        assert np.array_equal(lab[done], full[done])
        left = int(stf.trace["n_i"][kk]) if kk < stf.rounds else 0
        assert int((~done).sum()) == left
        mixed |= bool(done[iso].any() and (~done[iso]).any())
    assert mixed  # some partial run stopped between isolated vertices
    with pytest.raises(cc.CCError):
        fn(gh, order, 0.5, max_rounds=-1)
