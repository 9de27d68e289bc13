"""Training of the learned eps policy (an addition to the paper's fixed rule).

Algorithm 2 sizes round i's active set as B_i = ceil(eps n_i / Delta_i) with
one eps for the whole run.  The learned policy predicts eps_i per round from
six features of the run so far (see ``cc_set_eps_policy`` in include/cc.h).
C4's labels do not depend on the schedule (Section 3: C4 is serializable), so
the policy can only change the number of rounds and the time.

Labels (rollout from a replayed state).  A state is the loop just before
round i of a recorded run.  It is rebuilt exactly by replaying the recorded
batch sizes B_0..B_{i-1} through the TRACE policy; the rest of the run then
uses the fixed rule with each candidate eps_k in {2^(k/2) / 16 : k = 0..16}, and
the candidate whose whole run is fastest is the target eps* (the replayed
prefix is the same for every candidate, so comparing whole runs compares the
remainders).  Regression target: ln eps*.

States come from runs of the fixed rule at several eps and, in later passes,
from runs of the policy being trained (so it also learns the states it visits
itself).  Training minimises the mean squared error with the library's own
GPU kernels (``cc_mlp_train_step``); the features are standardised for
training and the standardisation is folded into the first layer afterwards,
so the exported weights take the raw features the round loop computes.

Run ``python -m paper_1507_05086_amd.policy train`` on a GPU to rebuild
``policy_weights.json``.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "policy_weights.json")
CANDIDATES = [2.0 ** (k / 2.0) / 16.0 for k in range(17)]  # 1/16 .. 16 in half octaves
EPS_MIN, EPS_MAX = 1.0 / 16.0, 16.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def trace_features(trace, eps_call: float) -> np.ndarray:
    """Feature rows of every recorded round, as the round loop forms them."""
    n = len(trace)
    X = np.zeros((n, 6), np.float64)
    for i in range(n):
        X[i, 0] = math.log(trace["n_i"][i])
        X[i, 1] = math.log(max(int(trace["delta_i"][i]), 1))
        if i == 0:
            X[i, 4] = eps_call
        else:
            b, np_ = int(trace["b_i"][i - 1]), int(trace["n_i"][i - 1])
            X[i, 2] = trace["conflicts"][i - 1] / b if b > 0 else 0.0
            X[i, 3] = trace["claimed"][i - 1] / np_ if np_ > 0 else 0.0
            X[i, 4] = float(trace["eps_used"][i - 1])
            X[i, 5] = float(i)
    return X


def pick_rounds(rounds: int, count: int, rng) -> list:
    """States to label: rounds before the last one (a rollout times a whole
    remaining run, so no round is special to the host's grouping of rounds)."""
    pool = list(range(rounds - 1))
    if len(pool) <= count:
        return pool
    # half spread evenly in log(i + 1), half uniform
    logs = np.unique(np.round(np.expm1(np.linspace(0, math.log(rounds), count // 2))).astype(int))
    pick = {min(pool, key=lambda r: abs(r - x)) for x in logs}
    rest = [r for r in pool if r not in pick]
    pick.update(rng.choice(rest, size=min(len(rest), count - len(pick)), replace=False).tolist())
    return sorted(pick)


def rollout(cc, gh, order, trace, i: int, repeats: int = 2):
    """ln eps* of the state before round i of `trace`: the candidate whose
    remaining run (fixed rule from round i on) is fastest."""
    prefix = np.asarray(trace["b_i"][:i], np.int64)
    best, best_t = None, float("inf")
    for e in CANDIDATES:
        cc.cc_set_eps_policy(cc.CC_EPS_TRACE, prefix)
        t = float("inf")
        for _ in range(repeats):
            _, st = cc.cc_c4(gh, order, e, labels=_scratch_labels(order), trace_capacity=0)
            t = min(t, st.loop_ms)
        if t < best_t:
            best_t, best = t, e
    cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
    return math.log(best)


_lab_cache = {}


def _scratch_labels(order):
    import torch
    key = (order.numel(), order.device)
    if key not in _lab_cache:
        _lab_cache.clear()
        _lab_cache[key] = torch.empty(order.numel(), dtype=torch.int32, device=order.device)
    return _lab_cache[key]


def collect(cc, gh, order, eps_bases, per_run: int, rng, weights=None):
    """(X, t) samples from runs of the fixed rule at each eps in eps_bases
    and, if `weights` is given, of that policy."""
    Xs, ts = [], []
    runs = [("fixed", e) for e in eps_bases] + ([("learned", 0.5)] if weights is not None else [])
    for kind, e in runs:
        if kind == "learned":
            cc.cc_set_eps_policy(cc.CC_EPS_LEARNED, weights, EPS_MIN, EPS_MAX)
        else:
            cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
        _, st = cc.cc_c4(gh, order, e, labels=_scratch_labels(order), trace_capacity=1 << 16)
        cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
        tr = st.trace
        X = trace_features(tr, e)
        for i in pick_rounds(st.rounds, per_run, rng):
            Xs.append(X[i])
            ts.append(rollout(cc, gh, order, tr, i))
            log(f"  {kind} eps={e}: round {i}/{st.rounds} -> eps* {math.exp(ts[-1]):.3g}")
    return np.array(Xs), np.array(ts)


def fold_standardization(w, mu, sd):
    """Weights for raw features from weights trained on (x - mu) / sd:
    W1' = W1 / sd (per input), b1' = b1 - W1' mu; the second layer is unchanged."""
    w = np.asarray(w, np.float64)
    W1 = w[:384].reshape(64, 6)
    W1r = W1 / sd
    b1r = w[384:448] - W1r @ mu
    return np.concatenate([W1r.ravel(), b1r, w[448:512], w[512:513]])


def train_mlp(cc, X, t, steps: int, lr: float, seed: int):
    """Adam on the GPU kernels; returns raw-feature weights (float32[513])."""
    import torch
    mu, sd = X.mean(axis=0), X.std(axis=0)
    sd[sd < 1e-6] = 1.0
    Xn = (X - mu) / sd
    rng = np.random.default_rng(seed)
    p0 = np.concatenate([rng.normal(0, 1 / math.sqrt(6), 384), np.full(64, 0.1),
                         rng.normal(0, 1 / 8, 64), [float(np.mean(t))]]).astype(np.float32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    p, m, v = dev(p0), torch.zeros(513, device="cuda"), torch.zeros(513, device="cuda")
    xd, td, loss = dev(Xn), dev(t), torch.zeros(1, device="cuda")
    for s in range(1, steps + 1):
        cc.cc_mlp_train_step(p, m, v, xd, td, s, lr, loss=loss)
    final = float(loss.item())
    return fold_standardization(p.cpu().numpy(), mu, sd).astype(np.float32), final


def save(weights, meta, path=WEIGHTS):
    with open(path, "w") as f:
        json.dump({"params": [float(x) for x in weights], "eps_min": EPS_MIN, "eps_max": EPS_MAX, **meta}, f)


def load(path=WEIGHTS):
    """(float32[513] weights, eps_min, eps_max) of a saved policy."""
    with open(path) as f:
        d = json.load(f)
    w = np.asarray(d["params"], dtype=np.float32)
    if w.shape != (513,):
        raise ValueError(f"{path}: expected 513 parameters")
    return w, float(d["eps_min"]), float(d["eps_max"])


def training_graphs(scales):
    """R-MAT graphs (a, b, c) = (0.57, 0.19, 0.19), edge factor 16, two seeds per scale."""
    import graphgen
    for s in scales:
        for seed in (100 + s, 200 + s):
            yield f"rmat{s}/seed{seed}", (lambda s=s, seed=seed: graphgen.rmat(s, 16, 0.57, 0.19, 0.19, seed=seed))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--scales", default="18,19,20,21,22,23,24")
    tr.add_argument("--per-run", type=int, default=24)
    tr.add_argument("--bases", default="0.5,2,8")
    tr.add_argument("--passes", type=int, default=3)
    tr.add_argument("--steps", type=int, default=4000)
    tr.add_argument("--lr", type=float, default=3e-3)
    tr.add_argument("--seed", type=int, default=7)
    tr.add_argument("--out", default=WEIGHTS)
    args = ap.parse_args()

    import torch
    import graphgen
    import paper_1507_05086_amd as cc
    scales = [int(x) for x in args.scales.split(",")]
    bases = [float(x) for x in args.bases.split(",")]
    rng = np.random.default_rng(args.seed)
    graphs = []
    for name, make in training_graphs(scales):
        t0 = time.perf_counter()
        g = make()
        off = torch.from_numpy(g.off).cuda()
        col = torch.from_numpy(g.col).cuda()
        gh = cc.cc_graph_from_csr(off, col, borrow=True)
        order = torch.from_numpy(graphgen.permutation(g.n, 1000 + len(graphs))).cuda()
        graphs.append((name, gh, order, (off, col)))
        log(f"{name}: n={g.n} m={g.m} ready in {time.perf_counter() - t0:.1f} s")
        del g
    X_all, t_all = np.zeros((0, 6)), np.zeros(0)
    weights, loss = None, float("nan")
    for ps in range(args.passes):
        for name, gh, order, _ in graphs:
            t0 = time.perf_counter()
            X, t = collect(cc, gh, order, bases if ps == 0 else [], args.per_run, rng, weights)
            X_all = np.concatenate([X_all, X])
            t_all = np.concatenate([t_all, t])
            log(f"pass {ps} {name}: {len(t)} labelled states in {time.perf_counter() - t0:.1f} s "
                f"(eps* mean {np.exp(t).mean():.2f})")
        weights, loss = train_mlp(cc, X_all, t_all, args.steps, args.lr, args.seed + ps)
        log(f"pass {ps}: trained on {len(t_all)} states, final mse {loss:.4f}")
    save(weights, {"trained_on": [n for n, *_ in graphs], "samples": int(len(t_all)), "mse": loss,
                   "label": "rollout: fastest fixed eps for the rest of the run",
                   "candidates": CANDIDATES}, path=args.out)
    log(f"wrote {args.out}")


if __name__ == "__main__":
    main()
