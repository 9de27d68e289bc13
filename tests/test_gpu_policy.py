"""The trained eps policy against the fixed rule it replaces.

C4's labels cannot depend on the batch schedule (Section 3: serializability),
so the learned policy must give labels identical to the fixed rule's and to
KwikCluster's, in fewer rounds and less time.  The graph is an R-MAT of the
training family with a seed no training run used.
"""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_common import assert_labels_equal, torch_cuda, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cc():
    torch_cuda()
    import paper_1507_05086_amd as cc
    return cc


def timed_runs(cc, gh, order, reps):
    times, out = [], None
    for _ in range(reps):
        lab, st = cc.cc_c4(gh, order, 0.5)
        times.append(st.loop_ms)
        out = (lab, st)
    return float(np.median(times)), out[0], out[1]


def test_learned_policy_beats_fixed_eps(cc):
    from paper_1507_05086_amd import policy
    torch = torch_cuda()
    w, eps_min, eps_max = policy.load()
    g = graphgen.rmat(21, 16, 0.57, 0.19, 0.19, seed=321)
    gh = upload(g, validate=False)
    order = torch.from_numpy(graphgen.permutation(g.n, 31)).cuda()
    try:
        cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
        cc.cc_c4(gh, order, 0.5)  # warm-up
        t_fixed, lab_fixed, st_fixed = timed_runs(cc, gh, order, 3)
        cc.cc_set_eps_policy(cc.CC_EPS_LEARNED, w, eps_min, eps_max)
        t_learned, lab_learned, st_learned = timed_runs(cc, gh, order, 3)
    finally:
        cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
    assert st_learned.policy_fallback == 0
    a, b = lab_fixed.cpu().numpy(), lab_learned.cpu().numpy()
    assert_labels_equal(b, a, "learned vs fixed")
    assert_labels_equal(b, oracle.kwikcluster(g.off, g.col, order.cpu().numpy()), "learned vs KwikCluster")
    assert st_learned.rounds < st_fixed.rounds
    print(f"fixed eps=0.5: {t_fixed:.2f} ms, {st_fixed.rounds} rounds; "
          f"learned: {t_learned:.2f} ms, {st_learned.rounds} rounds")
    assert t_learned < 0.8 * t_fixed
