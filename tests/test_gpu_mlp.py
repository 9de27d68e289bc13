"""GPU checks of the learned eps policy: the training and inference kernels
against the float64 reference (oracle/mlp.py), and the policy inside the
round loop.

Tolerances: forward within 1e-5 relative and gradients within 1e-4 relative
(float32 arithmetic against float64, sums over up to a few thousand
samples).  Labels stay integer-exact: C4 must equal KwikCluster whatever the
policy chooses, and ClusterWild! must equal the oracle replaying the batch
sizes the policy realised.
"""
import math

import numpy as np
import pytest

import graphgen
import oracle
from gpu_common import assert_labels_equal, torch_cuda, upload
from oracle import mlp

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


def dev(a):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def feature_like(rng, n):
    """Inputs spread like real round features."""
    return np.stack([rng.uniform(0, 18, n), rng.uniform(0, 14, n), rng.uniform(0, 1, n),
                     rng.uniform(0, 1, n), np.exp(rng.uniform(-3, 3, n)), rng.integers(0, 800, n)], axis=1)


def params_f32(rng, scale):
    return rng.normal(0, scale, mlp.NPARAM).astype(np.float32).astype(np.float64)


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


@pytest.mark.parametrize("n", [1, 63, 1000, 4099])
def test_forward(cc, n):
    rng = np.random.default_rng(n)
    p = params_f32(rng, 0.2)
    X = feature_like(rng, n).astype(np.float32).astype(np.float64)
    y = cc.cc_mlp_forward(dev(p), dev(X)).cpu().numpy()
    ref, _ = mlp.forward(p, X)
    assert rel_err(y, ref) < 1e-5


@pytest.mark.parametrize("n", [1, 37, 1000, 5000])
def test_gradient(cc, n):
    torch = torch_cuda()
    rng = np.random.default_rng(100 + n)
    p = params_f32(rng, 0.2)
    X = np.float32(rng.normal(0, 1, (n, 6))).astype(np.float64)
    t = np.float32(rng.normal(0, 1, n)).astype(np.float64)
    g = torch.zeros(mlp.NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    pd = dev(p)
    cc.cc_mlp_train_step(pd, None, None, dev(X), dev(t), 0, 0.0, grad=g, loss=loss)
    L, gref = mlp.loss_and_grad(p, X, t)
    assert rel_err(g.cpu().numpy(), gref) < 1e-4
    assert math.isclose(float(loss.item()), L, rel_tol=1e-4)
    assert np.array_equal(pd.cpu().numpy(), np.float32(p))  # lr == 0 leaves params alone


def test_gradient_of_empty_batch(cc):
    torch = torch_cuda()
    g = torch.full((mlp.NPARAM,), 7.0, dtype=torch.float32, device="cuda")
    p = dev(np.ones(mlp.NPARAM))
    x = torch.zeros((0, 6), dtype=torch.float32, device="cuda")
    t = torch.zeros(0, dtype=torch.float32, device="cuda")
    cc.cc_mlp_train_step(p, None, None, x, t, 0, 0.0, grad=g)
    assert not g.cpu().numpy().any()


def test_adam_steps(cc):
    torch = torch_cuda()
    rng = np.random.default_rng(9)
    p = params_f32(rng, 0.3)
    X = np.float32(rng.normal(0, 1, (500, 6))).astype(np.float64)
    t = np.float32(rng.normal(0, 1, 500)).astype(np.float64)
    pd, md, vd = dev(p), torch.zeros(mlp.NPARAM, device="cuda"), torch.zeros(mlp.NPARAM, device="cuda")
    pr, mr, vr = p.copy(), np.zeros(mlp.NPARAM), np.zeros(mlp.NPARAM)
    for step in range(1, 6):
        cc.cc_mlp_train_step(pd, md, vd, dev(X), dev(t), step, 1e-3)
        _, g = mlp.loss_and_grad(pr, X, t)
        pr, mr, vr = mlp.adam_step(pr, mr, vr, g, step, 1e-3)
    # the updates differ by float32 rounding of the gradient (Adam divides by |g|)
    assert np.max(np.abs(pd.cpu().numpy() - pr)) < 5e-6 * 5 + 1e-6
    assert rel_err(md.cpu().numpy(), mr) < 1e-4


def test_training_on_gpu_recovers_a_teacher(cc):
    torch = torch_cuda()
    rng = np.random.default_rng(5)
    teacher = rng.normal(0, 0.4, mlp.NPARAM)
    X = rng.normal(0, 1, (256, 6))
    t, _ = mlp.forward(teacher, X)
    p = dev(np.random.default_rng(6).normal(0, 0.4, mlp.NPARAM))
    m = torch.zeros(mlp.NPARAM, device="cuda")
    v = torch.zeros(mlp.NPARAM, device="cuda")
    loss = torch.zeros(1, device="cuda")
    xd, td = dev(X), dev(t)
    cc.cc_mlp_train_step(p, m, v, xd, td, 0, 0.0, loss=loss)
    l0 = float(loss.item())
    for s in range(1, 1501):
        cc.cc_mlp_train_step(p, m, v, xd, td, s, 3e-3, loss=loss)
    assert float(loss.item()) < 0.02 * l0


# ------------------------------------------------ the policy in the loop

def trace_features(trace, eps_call):
    rows = []
    for i in range(len(trace)):
        if i == 0:
            rows.append(mlp.features(trace["n_i"][0], trace["delta_i"][0], 0, 0, 0, 0, eps_call, 0))
        else:
            pr = trace[i - 1]
            rows.append(mlp.features(trace["n_i"][i], trace["delta_i"][i], pr["conflicts"], pr["b_i"],
                                     pr["claimed"], pr["n_i"], float(pr["eps_used"]), i))
    return np.array(rows)


def fixed_b(eps, n, delta):
    q = int(eps * 1e6 + 0.5)
    if delta <= 0:
        return n
    return min(max((q * n + 1_000_000 * delta - 1) // (1_000_000 * delta), 1), n)


def small_policy(seed):
    """Weights whose eps moves with the features (so rounds differ from fixed)."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, 0.05, (64, 6))
    b1 = rng.normal(0, 0.2, 64)
    w2 = rng.normal(0, 0.1, 64)
    return mlp.pack(W1, b1, w2, 0.7).astype(np.float32)


@pytest.mark.parametrize("algo", [oracle.C4, oracle.CW])
def test_learned_policy_in_loop(cc, algo):
    g = graphgen.chung_lu(60_000, 2.1, 14.0, seed=12)
    gh = upload(g)
    order = graphgen.permutation(g.n, 12)
    w = small_policy(3)
    eps_min, eps_max = 1 / 16, 16.0
    cc.cc_set_eps_policy(cc.CC_EPS_LEARNED, w, eps_min, eps_max)
    fn = cc.cc_c4 if algo == oracle.C4 else cc.cc_clusterwild
    lab, st = fn(gh, order, 0.5)
    assert st.policy_fallback == 0 and not st.truncated
    tr = st.trace
    X = trace_features(tr, 0.5)
    for i in range(len(tr)):
        e_ref = mlp.policy_eps(w.astype(np.float64), X[i], eps_min, eps_max)
        assert math.isclose(tr["eps_used"][i], e_ref, rel_tol=2e-5), i
        assert tr["b_i"][i] == fixed_b(float(tr["eps_used"][i]), int(tr["n_i"][i]), int(tr["delta_i"][i])), i
    if algo == oracle.C4:
        assert_labels_equal(lab, oracle.kwikcluster(g.off, g.col, order), "C4 (learned) vs KwikCluster")
    else:
        ref = oracle.bsp(oracle.CW, g.off, g.col, order, 0.5, sched=np.asarray(tr["b_i"], np.int64))
        assert_labels_equal(lab, ref.labels, "CW (learned) vs oracle replay")
        assert ref.rounds == st.rounds


def test_non_finite_weights_fall_back(cc):
    g = graphgen.erdos_renyi(20_000, 10.0, seed=1)
    gh = upload(g)
    order = graphgen.permutation(g.n, 4)
    w = np.zeros(mlp.NPARAM, np.float32)
    w[-1] = np.nan
    cc.cc_set_eps_policy(cc.CC_EPS_LEARNED, w)
    lab, st = cc.cc_clusterwild(gh, order, 0.5)
    assert st.policy_fallback == 1
    ref = oracle.bsp(oracle.CW, g.off, g.col, order, 0.5)
    assert_labels_equal(lab, ref.labels, "fallback = fixed rule")
    assert np.array_equal(st.trace["b_i"], ref.trace["b_i"])
