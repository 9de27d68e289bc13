"""The allocation-free training step (cc_mlp_train_step_noalloc) against the
ordinary one (cc_mlp_train_step): same gradient, loss and Adam update, on two
calls in a row, the second with a smaller batch, through the C ABI."""
import numpy as np
import pytest

from gpu_common import torch_cuda

pytestmark = pytest.mark.gpu


def _case(torch, n, seed):
    rng = np.random.default_rng(seed)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    p = dev(rng.normal(0, 0.3, 513))
    x = dev(rng.normal(0, 2.0, (n, 6)))
    t = dev(rng.normal(0, 1.0, n))
    return p, x, t


def _step(cc, fn, torch, p0, x, t, step, lr):
    p = p0.clone()
    m = torch.zeros(513, device="cuda") + 0.01
    v = torch.zeros(513, device="cuda") + 0.02
    g = torch.full((513,), float("nan"), device="cuda")
    loss = torch.full((1,), float("nan"), device="cuda")
    fn(p, m, v, x, t, step, lr, grad=g, loss=loss)
    torch.cuda.synchronize()
    return [a.cpu().numpy() for a in (p, m, v, g, loss)]


def test_noalloc_matches_the_allocating_step():
    torch = torch_cuda()
    import paper_1507_05086_amd as cc
    # a large batch (all 1024 partial rows in use), then a smaller one: the
    # second call must not see the first call's rows
    for n, seed, step, lr in ((200_000, 1, 3, 1e-3), (1000, 2, 1, 3e-3), (5, 3, 2, 0.0)):
        p0, x, t = _case(torch, n, seed)
        ref = _step(cc, cc.cc_mlp_train_step, torch, p0, x, t, step, lr)
        got = _step(cc, cc.cc_mlp_train_step_noalloc, torch, p0, x, t, step, lr)
        for a, b, name in zip(got, ref, ("params", "adam_m", "adam_v", "grad", "loss")):
            assert np.isfinite(a).all(), name
            # same kernels, same launch shape, same summation order: identical
            assert np.array_equal(a, b), (n, name, float(np.abs(a - b).max()))


def test_noalloc_checks_arguments():
    torch = torch_cuda()
    import paper_1507_05086_amd as cc
    p0, x, t = _case(torch, 10, 4)
    m = torch.zeros(513, device="cuda")
    with pytest.raises(cc.CCError) as ei:
        cc.cc_mlp_train_step_noalloc(p0, m, m, x, t, 0, 1e-3)  # Adam needs step >= 1
    assert ei.value.code == cc.CC_ERR_INVALID_ARG
