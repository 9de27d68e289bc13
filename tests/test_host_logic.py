"""CPU checks of host-side logic: the policy trainer's helpers and the
benchmark's counter summary."""
import csv
import json
import math
import os

import numpy as np

import graphgen
import oracle
from oracle import mlp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_trainer_features_match_the_reference():
    from paper_1507_05086_amd import policy
    dt = np.dtype([(f, np.float64 if f == "eps_used" else np.int64) for f in
                   ("n_i", "delta_i", "b_i", "r_i", "centers", "claimed", "conflicts", "eps_used", "t_ns")])
    tr = np.zeros(3, dt)
    tr["n_i"] = [1000, 900, 500]
    tr["delta_i"] = [40, 0, 7]
    tr["b_i"] = [13, 20, 30]
    tr["claimed"] = [80, 380, 0]
    tr["conflicts"] = [1, 4, 0]
    tr["eps_used"] = [0.5, 1.5, 2.0]
    X = policy.trace_features(tr, 0.5)
    for i in range(3):
        ref = mlp.features(tr["n_i"][i], tr["delta_i"][i], tr["conflicts"][i - 1] if i else 0,
                           tr["b_i"][i - 1] if i else 0, tr["claimed"][i - 1] if i else 0,
                           tr["n_i"][i - 1] if i else 0, tr["eps_used"][i - 1] if i else 0.5, i)
        assert np.allclose(X[i], ref)


def test_round_picking():
    from paper_1507_05086_amd import policy
    rng = np.random.default_rng(0)
    for rounds in (3, 40, 300):
        pick = policy.pick_rounds(rounds, 16, rng)
        assert pick == sorted(set(pick)) and len(pick) <= 16
        assert all(0 <= r < rounds - 1 for r in pick)
    assert policy.pick_rounds(5, 16, rng) == [0, 1, 2, 3]


def test_standardization_folds_into_the_first_layer():
    from paper_1507_05086_amd import policy
    rng = np.random.default_rng(2)
    w = rng.normal(0, 0.3, mlp.NPARAM)
    X = rng.normal(3, 5, (50, 6))
    mu, sd = X.mean(axis=0), X.std(axis=0)
    y_std, _ = mlp.forward(w, (X - mu) / sd)
    y_raw, _ = mlp.forward(policy.fold_standardization(w, mu, sd), X)
    assert np.allclose(y_std, y_raw, atol=1e-9)


def test_counter_summary(tmp_path, monkeypatch):
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: "test")
    os.makedirs(tmp_path / "profiles")
    # a calibration copy of 1 MiB read as half its size, then two calls
    # (the first call starts with the bucketed mapping of pi, the second with the direct one)
    seq = [("neg_kernel", 512.0), ("ccd::(anonymous namespace)::k_om_count(ccd::OrderMap, int const*, long)", 10.0),
           ("ccd::k_select(ccd::Ws)", 20.0), ("ccd::k_finalize(ccd::Ws, int*)", 5.0),
           ("ccd::k_check_order(ccd::Ws)", 1.0), ("ccd::k_finalize(ccd::Ws, int*)", 2.0)]
    for name, counter, scale in (("f.csv", "FETCH_SIZE", 1.0), ("w.csv", "WRITE_SIZE", 2.0)):
        with open(tmp_path / name, "w", newline="") as f:
            wr = csv.writer(f)
            wr.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
            for d, (k, kib) in enumerate(seq):
                wr.writerow([d + 1, k, counter, kib * scale])
    bench.summarize_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "toy", 1)
    out = json.load(open(tmp_path / "profiles" / "traffic_toy.json"))
    assert math.isclose(out["fetch_copy_factor"], 0.5) and math.isclose(out["write_copy_factor"], 1.0)
    c4, cw = out["calls"]["cc_c4"], out["calls"]["cc_clusterwild"]
    assert c4["dispatches"] == 3 and cw["dispatches"] == 2
    assert math.isclose(c4["fetch_bytes"], 35 * 1024 / 0.5) and math.isclose(cw["write_bytes"], 3 * 2048 / 1.0)


def test_library_draws_the_oracles_practical_schedule():
    """The library's host-side Binomial schedule is the oracle's, draw for
    draw (both follow the same published steps in IEEE double arithmetic)."""
    import paper_1507_05086_amd as cc
    cases = [(20_000, 25, 0.5, 11), (2_000_000, 9000, 0.1, 21), (2_000_000, 9000, 0.9, 22),
             (67_108_864, 300_000, 0.5, 31), (5000, 1, 0.5, 3), (5000, 0, 0.5, 3), (1, 7, 2.0, 1),
             (1000, 999, 40.0, 9), (10**9, 10**6, 0.05, 5)]
    rng = np.random.default_rng(4)
    for _ in range(40):
        cases.append((int(rng.integers(1, 10**7)), int(rng.integers(0, 10**5)),
                      float(np.exp(rng.uniform(np.log(0.02), np.log(20.0)))), int(rng.integers(0, 2**63))))
    for n, d0, eps, seed in cases:
        for delta in (0.1, 0.01):
            lib, period = cc.cc_binomial_schedule(n, d0, eps, seed, delta)
            ref = oracle.binomial_schedule(n, d0, eps, seed, delta)
            assert period == oracle.halving_period(n, d0, eps, delta)
            assert np.array_equal(lib, ref), (n, d0, eps, seed, delta)


def test_practical_schedule_argument_checks():
    import pytest
    import paper_1507_05086_amd as cc
    for args in ((-1, 5, 0.5, 1, 0.1), (10, -1, 0.5, 1, 0.1), (10, 5, 0.0, 1, 0.1), (10, 5, 0.5, 1, 1.0)):
        with pytest.raises(cc.CCError) as ei:
            cc.cc_binomial_schedule(*args)
        assert ei.value.code == cc.CC_ERR_INVALID_ARG
    with pytest.raises(cc.CCError) as ei:
        cc.cc_set_eps_policy(cc.CC_EPS_BINOMIAL, (1, 0.0))
    assert ei.value.code == cc.CC_ERR_POLICY
    cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
