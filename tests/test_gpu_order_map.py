"""GPU parity of the bucketed mapping of pi into internal ids.

Graphs with more than 2^22 vertices map pi through position and id buckets
of 2^15 (count, scan, scatter, gather from an LDS slice of the renumbering,
place).  These tests run sizes just above the threshold, with ragged last
buckets, against the oracle, and feed the check every kind of input that is
not a permutation: a repeated id whose bucket counts still balance (only the
per-bucket bitmap can see it), a repeat across buckets, ids out of range on
either side, the last id repeated, and pi all zero.  A failed check must
leave a device label buffer untouched and the handle usable.  The
asynchronous variants take the same mapping, which also writes each
vertex's rank.
"""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_common import assert_labels_equal, check_against_oracle, torch_cuda, upload

pytestmark = pytest.mark.gpu

BUCKET = 1 << 15


@pytest.fixture(scope="module")
def cc():
    torch_cuda()
    import paper_1507_05086_amd as cc
    cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
    return cc


@pytest.fixture(scope="module")
def er4m(cc):
    g = graphgen.erdos_renyi((1 << 22) + 1, 2.0, seed=41)  # 129 position buckets, the last one entry long
    return g, upload(g)


@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
def test_bucketed_parity(cc, er4m, algo):
    g, gh = er4m
    order = graphgen.permutation(g.n, 41)
    lab, _, _ = check_against_oracle(algo, g, gh, order, 0.5)
    if algo == oracle.C4:
        assert_labels_equal(lab, oracle.kwikcluster(g.off, g.col, order), "C4 vs KwikCluster")


def test_bucketed_host_buffers(cc):
    g = graphgen.erdos_renyi(5_000_000, 1.5, seed=42)
    gh = upload(g, device=False)
    order = graphgen.permutation(g.n, 42)
    check_against_oracle(oracle.C4, g, gh, order, 0.9, device=False)


def _bad_orders(n, seed):
    good = graphgen.permutation(n, seed)
    pos = np.empty(n, np.int64)
    pos[good] = np.arange(n)
    cases = {}
    o = good.copy()
    o[pos[101]] = 100  # 100 twice, 101 missing: same id bucket, counts balance
    cases["repeat_same_bucket"] = o
    o = good.copy()
    o[pos[3 * BUCKET + 7]] = 100  # bucket 0 one over, bucket 3 one under
    cases["repeat_across_buckets"] = o
    o = good.copy()
    o[pos[0]] = n - 1  # the last id, in the one-entry last bucket, twice
    cases["repeat_last_id"] = o
    o = good.copy()
    o[pos[5]] = n + 5
    cases["above_range"] = o
    o = good.copy()
    o[pos[n - 1]] = -1
    cases["negative"] = o
    cases["all_zero"] = np.zeros(n, np.int32)
    return good, cases


def test_bucketed_async(cc, er4m):
    g, gh = er4m
    order = graphgen.permutation(g.n, 44)
    torch = torch_cuda()
    lab, _ = cc.cc_c4_async(gh, torch.from_numpy(order).cuda())
    torch.cuda.synchronize()
    assert_labels_equal(lab.cpu().numpy(), oracle.kwikcluster(g.off, g.col, order), "async C4")
    # one wave: positions in order, 64 at a time, so ClusterWild! is the BSP
    # oracle with batches of 64 positions
    lab, _ = cc.cc_clusterwild_async(gh, torch.from_numpy(order).cuda(), waves=1)
    torch.cuda.synchronize()
    sched = np.full((g.n + 63) // 64, 64, dtype=np.int64)
    ref = oracle.bsp_positions(oracle.CW, g.off, g.col, order, sched)
    assert_labels_equal(lab.cpu().numpy(), ref.labels, "async ClusterWild!, one wave")


def test_bucketed_rejects_non_permutations(cc, er4m):
    torch = torch_cuda()
    g, gh = er4m
    good, cases = _bad_orders(g.n, 43)
    out = torch.full((g.n,), -7, dtype=torch.int32, device="cuda")
    calls = (lambda o: cc.cc_c4(gh, o, 0.5, labels=out), lambda o: cc.cc_clusterwild(gh, o, 0.5, labels=out),
             lambda o: cc.cc_c4_async(gh, o, labels=out), lambda o: cc.cc_clusterwild_async(gh, o, labels=out))
    for name, bad in cases.items():
        for fn in calls:
            with pytest.raises(cc.CCError) as ei:
                fn(torch.from_numpy(np.ascontiguousarray(bad, dtype=np.int32)).cuda())
            assert ei.value.code == cc.CC_ERR_NOT_PERMUTATION, name
            torch.cuda.synchronize()
            assert bool((out == -7).all()), name
    lab, st = cc.cc_c4(gh, torch.from_numpy(good).cuda(), 0.5, labels=out)
    torch.cuda.synchronize()
    assert_labels_equal(out.cpu().numpy(), oracle.kwikcluster(g.off, g.col, good), "after the rejected calls")
