"""Pins of the oracle's practical schedule (Implementation Details:
"Estimating but not computing Delta" and "Binomial sampling instead of
fixed-size batches"): the Binomial sampler against the exact distribution,
the halving period against its formula, and the position-batch round loop
against KwikCluster (C4 is serializable) and against each trace field's
definition.
"""
import math

import numpy as np
import pytest
from scipy import stats

import graphgen
import oracle


def _pmf(n, p):
    """Exact Binomial(n, p) probabilities from the binomial coefficients."""
    lp = [math.lgamma(n + 1) - math.lgamma(k + 1) - math.lgamma(n - k + 1) + k * math.log(p) +
          (n - k) * math.log1p(-p) for k in range(n + 1)]
    return np.exp(np.array(lp))


def _chi2_pvalue(samples, n, p):
    pmf = _pmf(n, p)
    counts = np.bincount(samples, minlength=n + 1).astype(float)
    expect = pmf * len(samples)
    # merge the tails until every bin expects at least 5 draws
    keep = expect >= 5
    lo, hi = np.argmax(keep), len(keep) - np.argmax(keep[::-1])
    obs = np.concatenate([[counts[:lo + 1].sum()], counts[lo + 1:hi - 1], [counts[hi - 1:].sum()]])
    exp = np.concatenate([[expect[:lo + 1].sum()], expect[lo + 1:hi - 1], [expect[hi - 1:].sum()]])
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    return stats.chi2.sf(chi2, len(obs) - 1)


# (n, p): inversion (n p < 10), the transformed rejection (n p >= 10) near the
# mode and in the tails, and both through the symmetry for p > 1/2
CASES = [(25, 0.2), (7, 0.5), (40, 0.3), (120, 0.45), (2000, 0.4), (60, 0.85), (500, 0.7), (100000, 0.01)]


@pytest.mark.parametrize("n,p", CASES)
def test_binomial_matches_the_exact_distribution(n, p):
    draws = np.array([oracle.binomial(1234, i, n, p) for i in range(60_000)])
    assert draws.min() >= 0 and draws.max() <= n
    assert _chi2_pvalue(draws, n, p) > 1e-5
    mean, var = n * p, n * p * (1 - p)
    assert abs(draws.mean() - mean) < 6 * math.sqrt(var / len(draws))


def test_binomial_large_mean_moments():
    n, p = 10**8, 1e-5  # mean 1000
    draws = np.array([oracle.binomial(99, i, n, p) for i in range(20_000)], dtype=float)
    mean, var = n * p, n * p * (1 - p)
    assert abs(draws.mean() - mean) < 6 * math.sqrt(var / len(draws))
    assert abs(draws.var() / var - 1) < 0.05


def test_binomial_special_cases():
    for i in range(20):
        assert oracle.binomial(3, i, 0, 0.4) == 0
        assert oracle.binomial(3, i, 17, 0.0) == 0
        assert oracle.binomial(3, i, 17, 1.0) == 17
        assert oracle.binomial(3, i, 1, 0.5) in (0, 1)
    # deterministic in (seed, stream)
    assert [oracle.binomial(8, i, 10**6, 0.3) for i in range(5)] == \
           [oracle.binomial(8, i, 10**6, 0.3) for i in range(5)]


def test_halving_period_formula():
    # K = ceil((2/eps) ln(n log2(Delta_0) / delta))
    for n, d0, eps, delta in ((67_108_864, 300_000, 0.5, 0.1), (20_000, 25, 0.9, 0.1), (1000, 1, 0.1, 0.01)):
        lg = max(math.log2(d0), 1.0) if d0 > 1 else 1.0
        want = max(1, math.ceil(2 / eps * math.log(n * lg / delta)))
        assert oracle.halving_period(n, d0, eps, delta) == want


@pytest.mark.parametrize("n,d0,eps", [(10_000, 40, 0.5), (5_000_000, 9000, 0.9), (300, 0, 0.5), (1, 5, 0.1)])
def test_schedule_takes_every_position(n, d0, eps):
    sched = oracle.binomial_schedule(n, d0, eps, seed=5)
    assert sched.sum() == n and (sched >= 0).all()
    K = oracle.halving_period(n, d0, eps)
    left = n
    for i, b in enumerate(sched):
        p = 1.0 if d0 == 0 else min(1.0, eps * 2 ** (i // K) / d0)
        if p == 1.0:
            assert b == left  # once p reaches 1 the round takes everything left
        left -= b
    # the positions left shrink by about the sampled fraction
    if d0 > 0 and n > 10**6:
        assert abs(sched[0] - n * eps / d0) < 6 * math.sqrt(n * eps / d0)


def _replay_binomial(g, order, algo, eps, seed):
    r = oracle.bsp_binomial(algo, g.off, g.col, order, eps, seed=seed, with_round_of=True)
    n, lab, ro, tr = g.n, r.labels, r.round_of, r.trace
    d0 = int(g.degrees().max()) if n else 0
    K = oracle.halving_period(n, d0, eps)
    sched = oracle.binomial_schedule(n, d0, eps, seed)
    assert np.array_equal(tr["b_i"], sched[:r.rounds])
    rank = np.empty(n, dtype=np.int64)
    rank[order] = np.arange(n)
    src = np.repeat(np.arange(n), np.diff(g.off))
    is_center = lab == np.arange(n)
    cur = 0
    for i in range(r.rounds):
        unc = ro >= i
        assert tr["n_i"][i] == np.count_nonzero(unc)
        h = i // K
        assert tr["delta_i"][i] == (d0 >> h if h < 63 else 0)
        b = int(tr["b_i"][i])
        assert tr["r_i"][i] == cur + b - 1
        assert not unc[order[:cur]].any()  # every position passed is settled
        act = np.zeros(n, dtype=bool)
        seg = order[cur:cur + b]
        act[seg[unc[seg]]] = True
        e = act[src] & act[g.col] & (rank[g.col] < rank[src])
        assert tr["conflicts"][i] == np.unique(src[e]).size
        done = ro == i
        assert tr["centers"][i] == np.count_nonzero(done & is_center)
        assert tr["claimed"][i] == np.count_nonzero(done & ~is_center)
        assert not (done & ~unc).any() and (ro[lab[done]] == i).all()
        if algo == oracle.CW:
            assert is_center[act].all()
        cur += b
    assert (ro >= 0).all()
    return r


@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
@pytest.mark.parametrize("eps", [0.1, 0.5, 0.9])
def test_binomial_rounds_from_definitions(algo, eps):
    g = graphgen.chung_lu(4000, 2.1, 14.0, seed=61)
    order = graphgen.permutation(g.n, 61)
    r = _replay_binomial(g, order, algo, eps, seed=17)
    if algo == oracle.C4:  # serializable: the schedule cannot change C4's labels
        assert np.array_equal(r.labels, oracle.kwikcluster(g.off, g.col, order))


@pytest.mark.parametrize("seed", range(4))
def test_binomial_c4_is_kwikcluster(seed):
    g = graphgen.rmat(12, 16, 0.57, 0.19, 0.19, seed=70 + seed)
    order = graphgen.permutation(g.n, 70 + seed)
    kc = oracle.kwikcluster(g.off, g.col, order)
    for eps in (0.05, 0.5, 2.0):
        r = oracle.bsp_binomial(oracle.C4, g.off, g.col, order, eps, seed=seed)
        assert np.array_equal(r.labels, kc)
        assert int(r.trace["centers"].sum() + r.trace["claimed"].sum()) == g.n


def test_binomial_degenerate_graphs():
    for n, edges in ((1, []), (37, []), (2, [(0, 1)]), (6, [(i, j) for i in range(6) for j in range(i + 1, 6)])):
        g = graphgen.from_edges(n, edges)
        order = graphgen.permutation(n, 3)
        for algo in (oracle.C4, oracle.CW):
            r = _replay_binomial(g, order, algo, 0.5, seed=2)
            assert ((r.labels >= 0) & (r.labels < n)).all()
            if not edges:
                assert r.rounds == 1 and r.labels.tolist() == list(range(n))


@pytest.mark.parametrize("seed", range(3))
def test_position_batches_reduce_to_kwikcluster(seed):
    """Rounds of fixed position batches: one position a round is KwikCluster
    for both algorithms; C4 is KwikCluster for any batch size."""
    g = graphgen.chung_lu(3000, 2.1, 10.0, seed=80 + seed)
    order = graphgen.permutation(g.n, 80 + seed)
    kc = oracle.kwikcluster(g.off, g.col, order)
    ones = np.ones(g.n, dtype=np.int64)
    for algo in (oracle.C4, oracle.CW):
        assert np.array_equal(oracle.bsp_positions(algo, g.off, g.col, order, ones).labels, kc)
    for b in (2, 64, 1000):
        sched = np.full(-(-g.n // b), b, dtype=np.int64)
        assert np.array_equal(oracle.bsp_positions(oracle.C4, g.off, g.col, order, sched).labels, kc)
    with pytest.raises(ValueError):
        oracle.bsp_positions(oracle.CW, g.off, g.col, order, np.array([g.n - 1], np.int64))
