"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: worked
examples derived by hand from Algorithm 2, closed forms, a brute-force
optimum with the expected 3-approximation of KwikCluster, three independent
ways of counting the objective, and the serializability claim of Section 3
(C4's output equals KwikCluster's for every eps and every schedule).
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _graph(n, edges):
    return graphgen.from_edges(n, edges)


# ---------------------------------------------------------------- fixtures

def test_path5_worked_example():
    fx = _load("path5.json")
    g = _graph(fx["n"], fx["edges"])
    order = np.array(fx["order"], dtype=np.int32)
    assert oracle.kwikcluster(g.off, g.col, order).tolist() == fx["kwikcluster_labels"]
    for algo, key in ((oracle.C4, "c4"), (oracle.CW, "clusterwild")):
        r = oracle.bsp(algo, g.off, g.col, order, fx["eps"])
        exp = fx[key]
        assert r.labels.tolist() == exp["labels"]
        assert r.rounds == exp["rounds"]
        assert r.trace["b_i"].tolist() == exp["b"]
        assert r.trace["delta_i"].tolist() == exp["delta"]
        assert r.trace["n_i"].tolist() == exp["n"]
        assert r.trace["r_i"].tolist() == exp["r"]
        assert r.trace["conflicts"].tolist() == exp["conflicts"]
        assert r.trace["centers"].tolist() == exp["centers"]
        assert r.trace["claimed"].tolist() == exp["claimed"]
        assert oracle.cost(g.off, g.col, r.labels) == exp["cost"]


def test_star_example_and_opt():
    fx = _load("star5.json")
    g = _graph(fx["n"], fx["edges"])
    order = np.array(fx["order"], dtype=np.int32)
    lab = oracle.kwikcluster(g.off, g.col, order)
    assert lab.tolist() == fx["kwikcluster_labels"]
    assert oracle.cost(g.off, g.col, lab) == fx["cost"]
    assert brute_force_opt(g) == fx["opt"]


# ------------------------------------------------------------ closed forms

def _cliques(sizes):
    edges, base = [], 0
    for s in sizes:
        edges += [(base + i, base + j) for i in range(s) for j in range(i + 1, s)]
        base += s
    return base, edges


@pytest.mark.parametrize("seed", range(5))
def test_disjoint_cliques_zero_cost(seed):
    n, edges = _cliques([1, 2, 3, 5, 8, 4])
    g = _graph(n, edges)
    order = graphgen.permutation(n, seed)
    rank = np.argsort(order)
    starts = np.cumsum([0, 1, 2, 3, 5, 8, 4])
    for lab in (oracle.kwikcluster(g.off, g.col, order),
                *(oracle.c4(g.off, g.col, order, e).labels for e in (0.1, 0.5, 3.0))):
        assert oracle.cost(g.off, g.col, lab) == 0
        for a, b in zip(starts[:-1], starts[1:]):
            members = np.arange(a, b)
            center = members[np.argmin(rank[members])]  # lowest rank in the clique
            assert (lab[a:b] == center).all()


@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
def test_edgeless_one_round(algo):
    n = 37
    g = _graph(n, [])
    order = graphgen.permutation(n, 3)
    r = oracle.bsp(algo, g.off, g.col, order, 0.5)
    assert r.rounds == 1
    assert r.labels.tolist() == list(range(n))
    assert r.trace["b_i"].tolist() == [n] and r.trace["delta_i"].tolist() == [0]
    assert oracle.cost(g.off, g.col, r.labels) == 0


def _complete(n):
    return _graph(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


@pytest.mark.parametrize("n,eps", [(10, 0.5), (10, 0.9), (17, 3.0), (6, 40.0)])
def test_complete_graph_fixed_rule(n, eps):
    g = _complete(n)
    order = graphgen.permutation(n, 5)
    r = oracle.c4(g.off, g.col, order, eps)
    b0 = min(n, math.ceil(eps * n / (n - 1)))
    assert r.trace["b_i"][0] == b0
    assert (r.labels == order[0]).all() and r.rounds == 1
    assert oracle.cost(g.off, g.col, r.labels) == 0


@pytest.mark.parametrize("n,b", [(10, 3), (10, 1), (8, 8), (12, 5)])
def test_complete_graph_clusterwild_schedule(n, b):
    g = _complete(n)
    order = graphgen.permutation(n, 9)
    r = oracle.clusterwild(g.off, g.col, order, sched=[b])
    sizes = np.bincount(r.labels, minlength=n)
    assert sizes[order[0]] == n - b + 1
    assert sorted(sizes[sizes > 0].tolist()) == sorted([1] * (b - 1) + [n - b + 1])
    assert oracle.cost(g.off, g.col, r.labels) == math.comb(n, 2) - math.comb(n - b + 1, 2)
    if (n, b) == (10, 3):
        assert oracle.cost(g.off, g.col, r.labels) == 17


# -------------------------------------------- brute force: 3-approximation

def brute_force_opt(g):
    """Minimum disagreements over all set partitions (restricted growth strings)."""
    n = g.n
    adj = np.zeros((n, n), dtype=bool)
    for v in range(n):
        adj[v, g.col[g.off[v]:g.off[v + 1]]] = True
    iu = np.triu_indices(n, 1)
    pos = adj[iu]
    best = None
    a = [0] * n

    def rec(i, k):
        nonlocal best
        if i == n:
            lab = np.array(a)
            same = (lab[:, None] == lab[None, :])[iu]
            c = int(np.count_nonzero(same != pos))
            best = c if best is None else min(best, c)
            return
        for x in range(k + 1):
            a[i] = x
            rec(i + 1, max(k, x + 1))

    rec(0, 0)
    return best


def _random_small_graph(n, p, seed):
    rng = np.random.default_rng(seed)
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    return _graph(n, edges)


@pytest.mark.parametrize("n,p,seed", [(5, 0.5, 1), (6, 0.4, 2), (7, 0.5, 3), (7, 0.3, 4), (8, 0.45, 5)])
def test_kwikcluster_expected_three_approx(n, p, seed):
    g = _random_small_graph(n, p, seed)
    opt = brute_force_opt(g)
    total = 0
    for perm in itertools.permutations(range(n)):
        order = np.array(perm, dtype=np.int32)
        lab = oracle.kwikcluster(g.off, g.col, order)
        c = oracle.cost(g.off, g.col, lab)
        assert c >= opt
        total += c
    assert total <= 3 * opt * math.factorial(n)


# -------------------------------------------------- the objective, 3 ways

@pytest.mark.parametrize("seed", range(6))
def test_cost_three_ways(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 150))
    g = graphgen.erdos_renyi(n, float(rng.uniform(0.5, 12)), seed=seed)
    order = graphgen.permutation(n, seed + 50)
    lab = oracle.kwikcluster(g.off, g.col, order)
    c1 = oracle.cost(g.off, g.col, lab)
    assert c1 == oracle.cost_pairs(g.off, g.col, lab)
    assert c1 == oracle.kc_stepwise_cost(g.off, g.col, order)
    # arbitrary (non-center) cluster ids: closed form against pair count
    arb = rng.integers(0, max(1, n // 3), size=n).astype(np.int32)
    assert oracle.cost(g.off, g.col, arb) == oracle.cost_pairs(g.off, g.col, arb)
    cw = oracle.clusterwild(g.off, g.col, order, 0.9).labels
    assert oracle.cost(g.off, g.col, cw) == oracle.cost_pairs(g.off, g.col, cw)


# ---------------------------------------- serializability (Section 3)

def _graphs_small():
    yield graphgen.erdos_renyi(3000, 10.0, seed=11)
    yield graphgen.chung_lu(4000, 2.1, 12.0, seed=12)
    yield graphgen.rmat(12, 16, 0.57, 0.19, 0.19, seed=13)
    n, e = _cliques([3, 7, 1, 20, 2])
    yield _graph(n, e)


@pytest.mark.parametrize("gi,g", list(enumerate(_graphs_small())))
def test_c4_equals_kwikcluster_every_eps(gi, g):
    for seed in (1, 2):
        order = graphgen.permutation(g.n, 100 * gi + seed)
        kc = oracle.kwikcluster(g.off, g.col, order)
        assert oracle.check_kc(g.off, g.col, order, kc) == (0, -1)
        for eps in (0.05, 0.1, 0.5, 0.9, 2.0, 16.0):
            r = oracle.c4(g.off, g.col, order, eps)
            assert np.array_equal(r.labels, kc), eps
            assert int(r.trace["centers"].sum() + r.trace["claimed"].sum()) == g.n


@pytest.mark.parametrize("seed", range(4))
def test_c4_equals_kwikcluster_any_schedule(seed):
    g = graphgen.rmat(11, 8, 0.57, 0.19, 0.19, seed=seed)
    order = graphgen.permutation(g.n, seed)
    kc = oracle.kwikcluster(g.off, g.col, order)
    rng = np.random.default_rng(seed)
    for sched in (np.ones(g.n, dtype=np.int64), [g.n],
                  rng.integers(1, 300, size=40), rng.integers(1, 5, size=7)):
        r = oracle.c4(g.off, g.col, order, 0.5, sched=sched)
        assert np.array_equal(r.labels, kc)


@pytest.mark.parametrize("seed", range(3))
def test_clusterwild_unit_batches_is_kwikcluster(seed):
    g = graphgen.chung_lu(3000, 2.1, 10.0, seed=seed)
    order = graphgen.permutation(g.n, seed + 7)
    r = oracle.clusterwild(g.off, g.col, order, sched=np.ones(g.n, dtype=np.int64))
    assert np.array_equal(r.labels, oracle.kwikcluster(g.off, g.col, order))


def test_check_kc_detects_planted_mistakes():
    g = graphgen.erdos_renyi(500, 6.0, seed=4)
    order = graphgen.permutation(g.n, 4)
    kc = oracle.kwikcluster(g.off, g.col, order)
    rng = np.random.default_rng(0)
    non_centers = np.flatnonzero(kc != np.arange(g.n))
    centers = np.flatnonzero(kc == np.arange(g.n))
    # a non-center moved to another center
    bad = kc.copy()
    v = non_centers[0]
    bad[v] = centers[centers != kc[v]][0]
    assert oracle.check_kc(g.off, g.col, order, bad)[0] > 0
    # a non-center promoted to center
    bad = kc.copy()
    bad[v] = v
    assert oracle.check_kc(g.off, g.col, order, bad)[0] > 0
    # a center demoted: its members keep pointing to it
    bad = kc.copy()
    c = centers[rng.integers(len(centers))]
    bad[c] = kc[(c + 1) % g.n] if kc[(c + 1) % g.n] != c else 0
    assert oracle.check_kc(g.off, g.col, order, bad)[0] > 0
    # a different order gives a different answer
    other = graphgen.permutation(g.n, 99)
    assert oracle.check_kc(g.off, g.col, other, kc)[0] > 0


# ------------------------------------------------------------- invariants

@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
@pytest.mark.parametrize("eps", [0.1, 0.5, 0.9, 4.0])
def test_invariants(algo, eps):
    g = graphgen.chung_lu(5000, 2.1, 16.0, seed=21)
    order = graphgen.permutation(g.n, 21)
    r = oracle.bsp(algo, g.off, g.col, order, eps)
    lab = r.labels
    n = g.n
    assert ((lab >= 0) & (lab < n)).all()
    assert (lab[lab] == lab).all()  # every label is a center of itself
    for v in range(n):  # v is its center or adjacent to it
        if lab[v] != v:
            row = g.col[g.off[v]:g.off[v + 1]]
            assert lab[v] in row
    tr = r.trace
    assert tr["n_i"][0] == n
    assert (tr["n_i"][1:] == tr["n_i"][:-1] - tr["centers"][:-1] - tr["claimed"][:-1]).all()
    assert tr["n_i"][-1] == tr["centers"][-1] + tr["claimed"][-1]
    assert tr["delta_i"][0] == g.degrees().max()
    assert (np.diff(tr["delta_i"]) <= 0).all()  # remaining max degree never grows
    assert (np.diff(tr["r_i"]) > 0).all()  # the cursor only moves forward
    # B_i from its definition in integers (eps in millionths, ceil, clamp)
    q = oracle.quantize_eps(eps)
    for ni, di, bi in zip(tr["n_i"], tr["delta_i"], tr["b_i"]):
        want = ni if di == 0 else min(ni, max(1, -(-q * ni // (10**6 * di))))
        assert bi == want
    if algo == oracle.C4:
        centers = np.flatnonzero(lab == np.arange(n))
        is_c = np.zeros(n, dtype=bool)
        is_c[centers] = True
        for c in centers:  # centers form an independent set
            assert not is_c[g.col[g.off[c]:g.off[c + 1]]].any()
        # an active non-center always had an earlier active neighbour (it was blocked)
        assert (tr["b_i"] - tr["centers"] <= tr["conflicts"]).all()


def test_rounds_soft_bound():
    g = graphgen.rmat(14, 16, 0.57, 0.19, 0.19, seed=5)
    order = graphgen.permutation(g.n, 5)
    dmax = int(g.degrees().max())
    for eps in (0.1, 0.5, 0.9):
        r = oracle.c4(g.off, g.col, order, eps)
        # O((1/eps) log n log Delta) rounds (Section 3.1), constant 2 as a soft check
        assert r.rounds <= 2 * (1 / eps) * math.log(g.n) * math.log(dmax)


def test_invalid_inputs_rejected():
    g = _graph(4, [(0, 1)])
    with pytest.raises(ValueError):
        oracle.c4(g.off, g.col, np.array([0, 1, 1, 2], dtype=np.int32))
    with pytest.raises(ValueError):
        oracle.c4(g.off, g.col, np.arange(4, dtype=np.int32), sched=[2, 0])
    with pytest.raises(ValueError):
        oracle.cost(g.off, g.col, np.array([0, 1, 2, 9], dtype=np.int32))


# ------------------------------- every trace field from its definition

def _replay_checks(g, order, algo, eps):
    """Re-derive every field of the oracle's round trace from its definition,
    round by round, with plain full scans over the graph.  The only things
    taken from the oracle are the round in which each vertex was clustered,
    the labels and the trace itself."""
    r = oracle.bsp(algo, g.off, g.col, order, eps, with_round_of=True)
    n, lab, ro, tr = g.n, r.labels, r.round_of, r.trace
    assert (ro >= 0).all() and (ro < r.rounds).all()
    rank = np.empty(n, dtype=np.int64)
    rank[order] = np.arange(n)
    src = np.repeat(np.arange(n), np.diff(g.off))  # row of every adjacency entry
    is_center = lab == np.arange(n)
    prev_r = -1
    for i in range(r.rounds):
        unc = ro >= i  # unclustered when round i starts
        assert tr["n_i"][i] == np.count_nonzero(unc)
        # Delta_i: the largest number of unclustered neighbours of an unclustered vertex
        live = unc[src] & unc[g.col]
        deg = np.bincount(src[live], minlength=n)
        assert tr["delta_i"][i] == (deg[unc].max() if unc.any() else 0)
        # the active set: the unclustered vertices at pi positions (r_{i-1}, r_i]
        ri = int(tr["r_i"][i])
        assert unc[order[ri]]  # the last active vertex was still unclustered
        assert not unc[order[:prev_r + 1]].any()  # every earlier position is settled
        act = np.zeros(n, dtype=bool)
        seg = order[prev_r + 1:ri + 1]
        act[seg[unc[seg]]] = True
        assert tr["b_i"][i] == np.count_nonzero(act)
        # blocked: active vertices with an earlier-ranked active neighbour
        e = act[src] & act[g.col] & (rank[g.col] < rank[src])
        assert tr["conflicts"][i] == np.unique(src[e]).size
        done = ro == i
        ncent = np.count_nonzero(done & is_center)
        assert tr["centers"][i] == ncent
        assert tr["claimed"][i] == np.count_nonzero(done) - ncent
        assert not (done & ~unc).any()
        assert (ro[lab[done]] == i).all()  # a vertex joins a center made in the same round
        if algo == oracle.CW:
            assert is_center[act].all()  # ClusterWild! makes every active vertex a center
        else:
            assert not (done & is_center & ~act).any()  # C4's centers come from the active set
        prev_r = ri
    assert prev_r < n


@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
@pytest.mark.parametrize("eps", [0.1, 0.5, 2.0])
@pytest.mark.parametrize("family", ["rmat14", "chunglu5k"])
def test_trace_fields_from_definitions(family, algo, eps):
    g = (graphgen.rmat(14, 16, 0.57, 0.19, 0.19, seed=114) if family == "rmat14"
         else graphgen.chung_lu(5000, 2.1, 16.0, seed=51))
    order = graphgen.permutation(g.n, 7)
    _replay_checks(g, order, algo, eps)


# ----------------------- ClusterWild! as a peeling of the graph without the
# edges among same-round active vertices (the paper's analysis of CW)

def _peel(n, adj, centers):
    """Greedy peeling: each center in turn takes itself and its unclustered
    neighbours in `adj`.  Returns the labels and the number of bad triangles
    (three vertices, exactly two pairs adjacent) that contain the center and
    two vertices still unclustered at its turn."""
    unc = set(range(n))
    labels = [-1] * n
    bad = 0
    for c in centers:
        assert c in unc, "a center was already clustered at its turn"
        rest = sorted(unc - {c})
        for i, a in enumerate(rest):
            for b in rest[i + 1:]:
                if (a in adj[c]) + (b in adj[c]) + (b in adj[a]) == 2:
                    bad += 1
        for u in {c} | (adj[c] & unc):
            labels[u] = c
            unc.discard(u)
    assert not unc, "the centers left vertices unclustered"
    return np.array(labels, dtype=np.int32), bad


def _active_sets(r, order, n):
    """The active set of every round, from the trace's r_i and the round in
    which each vertex was clustered."""
    out, prev = [], -1
    for i in range(r.rounds):
        seg = order[prev + 1:int(r.trace["r_i"][i]) + 1]
        out.append([int(v) for v in seg if r.round_of[v] >= i])
        prev = int(r.trace["r_i"][i])
    return out


@pytest.mark.parametrize("eps", [0.5, 2.0, 8.0])
@pytest.mark.parametrize("seed", range(6))
def test_cw_is_kwikcluster_peeling_of_the_graph_without_active_edges(seed, eps):
    """The paper bounds ClusterWild!'s cost by treating the edges between two
    vertices active in the same round as deleted: on that graph G', CW is a
    greedy peeling that takes the centers round by round in pi order, and
    any greedy peeling costs exactly the bad triangles at each center among
    the vertices still unclustered (section Approximation ratio, the two
    lemmas on the cost of greedy peelings and of CW).  On G the deleted
    edges are cut as well.  So, exactly: CW's labels are that peeling's, and
    cost_G = bad triangles of G' at the centers + deleted edges."""
    g = graphgen.erdos_renyi(28, 4.0 + seed, seed=300 + seed)
    order = graphgen.permutation(g.n, 400 + seed)
    rank = np.empty(g.n, dtype=np.int64)
    rank[order] = np.arange(g.n)
    adj = [set(g.col[g.off[v]:g.off[v + 1]].tolist()) for v in range(g.n)]
    r = oracle.bsp(oracle.CW, g.off, g.col, order, eps, with_round_of=True)
    acts = _active_sets(r, order, g.n)
    gp = [set(s) for s in adj]
    deleted = 0
    for a in acts:
        sa = set(a)
        for v in a:
            for u in adj[v] & sa:
                if u > v:
                    deleted += 1
                gp[v].discard(u)
    centers = [v for a in acts for v in sorted(a, key=lambda x: rank[x])]
    labels, bad = _peel(g.n, gp, centers)
    assert np.array_equal(labels, r.labels)
    assert oracle.cost(g.off, g.col, r.labels) == bad + deleted
    if eps >= 2.0:
        assert deleted > 0  # the larger batches put adjacent vertices in one active set


@pytest.mark.parametrize("seed", range(4))
def test_kwikcluster_cost_is_its_bad_triangles(seed):
    """The same lemma for KwikCluster (nothing deleted): the cost equals the
    bad triangles at the centers, taken in pi order."""
    g = graphgen.erdos_renyi(30, 5.0, seed=500 + seed)
    order = graphgen.permutation(g.n, 600 + seed)
    adj = [set(g.col[g.off[v]:g.off[v + 1]].tolist()) for v in range(g.n)]
    kc = oracle.kwikcluster(g.off, g.col, order)
    centers = [int(v) for v in order if kc[v] == v]
    labels, bad = _peel(g.n, adj, centers)
    assert np.array_equal(labels, kc)
    assert oracle.cost(g.off, g.col, kc) == bad
