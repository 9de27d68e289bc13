#!/usr/bin/env python3
"""Throughput of the C4 + ClusterWild! round loop on one MI355X.

A step is one cc_c4 call plus one cc_clusterwild call (fixed eps rule) on the
same resident graph and order: every step of the hot path (delta, active-set
selection, election, claims, peeling, labels) runs once per algorithm.
`value` is positive edges clustered per second over the step:
2 * m / step_time.  Inputs (CSR, order, output buffers) are in HBM before the
timed region starts.  Each call is also bracketed by HIP events on the
stream its kernels run on (whole call: order check, rounds, labels).

Default workload: R-MAT scale 26, edge factor 16, (a,b,c,d) = (0.57, 0.19,
0.19, 0.05), symmetrised and deduplicated (~1.05e9 undirected positive
edges), seeded order, eps = 0.5.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_graph(name):
    import graphgen
    return graphgen.workload(name)


def algorithmic_bytes(st, n, nnz, deg, labels, c4):
    """Bytes the method must move in one call, counted per unit:
      8 B per adjacency entry (a 4 B column and a 4 B neighbour word) of
        E_peel = every entry once (each row is walked when its vertex is
                 clustered, to take it out of its neighbours' degrees),
        E_claim = the rows of all centers,
        E_elect = the rows of all active vertices (C4 only);
      8 B per atomic read-modify-write; 32 B per vertex (offsets, order, rank,
      initial state, final label).
    E_claim comes from the labels (a center is its own label); E_elect adds to
    it the rows of the active vertices that were not centers, which the
    library's counters give (listed active rows minus listed center rows).
    Returns (these bytes, the bytes of the entries the implementation actually
    read: lazy deletion skips rows with no unclustered neighbour left)."""
    import numpy as np
    centers = labels == np.arange(n, dtype=labels.dtype)
    e_claim = int(deg[centers].sum())
    e_elect = int(st.scanned_elect) + e_claim - int(st.scanned_claim) if c4 else 0
    alg = 8 * (nnz + e_claim + e_elect) + 8 * st.atomics + 32 * n
    read = st.scanned_elect + st.scanned_claim + st.scanned_delta + st.scanned_peel
    return alg, 8 * read + 8 * st.atomics + 32 * n, {"E_peel": nnz, "E_claim": e_claim, "E_elect": e_elect}


def source_hash():
    """Hash of the HIP sources: counter-based traffic is reported only for the
    kernels it was measured on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1507_05086_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per call from the committed rocprofv3 counter summary, or None
    when it is missing or was taken on other kernels."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash():
        return None
    return d


# a call's first kernel: the bucketed mapping of pi (large graphs) or the direct one
CALL_FIRST, CALL_LAST = ("k_om_count", "k_check_order"), "k_finalize"


def kernel_short_name(name):
    """'ccd::(anonymous namespace)::k_om_count(ccd::OrderMap, ...)' -> 'k_om_count'."""
    return name.replace("(anonymous namespace)::", "").split("(")[0].split("::")[-1]


def summarize_counters(fetch_csv, write_csv, workload, copy_mb):
    """HBM traffic per round-loop call from two rocprofv3 --pmc runs of
    `bench.py --steps 1 --warmup 0 --no-extras --copy-calibration-mb M`
    (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch).  Dispatches are split into
    calls at the loop's first and last kernels (the C4 call comes first), and
    both counters are scaled by what they read for the calibration copy
    (M MiB read, M MiB written)."""
    import csv

    def per_dispatch(path, counter):
        rows = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                d = int(r["Dispatch_Id"])
                name = r["Kernel_Name"]
                rows.setdefault(d, [name, 0.0])[1] += float(r["Counter_Value"]) * 1024.0
        return [rows[d] for d in sorted(rows)]

    out = {"source_hash": source_hash(), "workload": workload, "copy_mb": copy_mb, "calls": {}}
    for counter, path, key in (("FETCH_SIZE", fetch_csv, "fetch"), ("WRITE_SIZE", write_csv, "write")):
        seq = per_dispatch(path, counter)
        copy = [b for name, b in seq if "neg" in name.lower()]
        if not copy:
            raise SystemExit(f"{path}: no calibration copy kernel found")
        factor = copy[0] / (copy_mb * 2 ** 20)
        out[f"{key}_copy_factor"] = round(factor, 4)
        calls, cur = [], None
        for name, b in seq:
            short = kernel_short_name(name)
            if short.startswith(CALL_FIRST):
                cur = [0.0, 0]
            if cur is not None:
                cur[0] += b
                cur[1] += 1
            if cur is not None and short.startswith(CALL_LAST):
                calls.append(cur)
                cur = None
        for nm, c in zip(("cc_c4", "cc_clusterwild"), calls):
            e = out["calls"].setdefault(nm, {})
            e[f"{key}_bytes"] = c[0] / factor
            e["dispatches"] = c[1]
    for e in out["calls"].values():
        e["hbm_bytes"] = e.get("fetch_bytes", 0.0) + e.get("write_bytes", 0.0)
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def bench_batched(cc, torch, steps):
    """The batched workload: 4096 planted-block graphs in one persistent launch."""
    import numpy as np
    import graphgen
    g = graphgen.workload("sbm4096")
    dev = torch.device("cuda:0")
    off = torch.from_numpy(g.off).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    gh = cc.cc_graph_from_csr(off, col, vtx_ptr=g.vtx_ptr)
    order = torch.from_numpy(graphgen.batch_permutations(g.vtx_ptr, 4096)).to(dev)
    labs = {"c4": torch.empty(g.n, dtype=torch.int32, device=dev),
            "clusterwild": torch.empty(g.n, dtype=torch.int32, device=dev)}
    out = {"workload": "sbm4096", "graphs": g.ngraphs, "n": g.n, "m": g.m}
    for name, algo, fn in (("c4", cc.CC_ALGO_C4, cc.cc_c4), ("clusterwild", cc.CC_ALGO_CLUSTERWILD, cc.cc_clusterwild)):
        lab = labs[name]
        t0 = time.perf_counter()
        best = cc.cc_batch_autotune(gh, order, algo, 0.5)
        tune_s = time.perf_counter() - t0
        fn(gh, order, 0.5, labels=lab)
        torch.cuda.synchronize()
        ks, t0 = [], time.perf_counter()
        for _ in range(steps):
            _, st = fn(gh, order, 0.5, labels=lab)
            ks.append(st.loop_ms)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        out[name] = {"launch_ms": round(float(np.median(ks)), 3), "call_ms": round(wall * 1e3, 3),
                     "edges_per_s": g.m / (float(np.median(ks)) / 1e3), "max_rounds": st.rounds,
                     "shape": {"block": best.block, "wave_max_n": best.wave_max_n, "quad_max_n": best.quad_max_n}, "autotune_s": round(tune_s, 2)}
    # ablation: the same graphs one call each (every 16th graph, scaled by 16)
    sample = list(range(0, g.ngraphs, 16))
    handles = []
    for i in sample:
        a, b = int(g.vtx_ptr[i]), int(g.vtx_ptr[i + 1])
        o = g.off[a:b + 1]
        gi = cc.cc_graph_from_csr(torch.from_numpy(o - o[0]).to(dev), torch.from_numpy(g.col[o[0]:o[-1]]).to(dev))
        handles.append((gi, order[a:b].contiguous(), torch.empty(b - a, dtype=torch.int32, device=dev)))
    for gi, oi, li in handles:  # workspaces allocated outside the timing
        cc.cc_c4(gi, oi, 0.5, labels=li)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for gi, oi, li in handles:
        cc.cc_c4(gi, oi, 0.5, labels=li)
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - t0) * 1e3 * g.ngraphs / len(sample)
    out["sequential_c4_ms_estimate"] = round(seq_ms, 1)
    out["speedup_vs_sequential"] = round(seq_ms / out["c4"]["call_ms"], 1)
    # the timed launch's labels against the single-graph path on the sampled graphs
    same = all(torch.equal(labs["c4"][int(g.vtx_ptr[i]):int(g.vtx_ptr[i + 1])], li)
               for i, (_, _, li) in zip(sample, handles))
    out["c4_labels_equal_single_graph_calls"] = {"graphs_checked": len(sample), "equal": bool(same)}
    return out


def timed_call(cc, torch, fn, gh, order, eps, lab):
    """One call bracketed by HIP events on the stream its kernels run on."""
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    _, st = fn(gh, order, eps, labels=lab)
    e1.record(s)
    e1.synchronize()
    return st, e0.elapsed_time(e1)


def bench_learned(cc, torch, gh, order, lab_ref, eps_fixed, reps, other_seeds=(32, 33)):
    """The learned eps policy against the fixed rule on the same graph and
    order: eps = 0.5 and every half-octave candidate eps of the trainer (the
    best fixed eps in hindsight), for C4 and ClusterWild!; then, for C4 on the
    other evaluation orders, against eps = 0.5 with the labels compared."""
    import numpy as np
    from paper_1507_05086_amd import policy
    w, lo, hi = policy.load()
    lab = torch.empty_like(lab_ref)
    out = {"fixed_eps": eps_fixed, "candidates": len(policy.CANDIDATES)}
    for name, fn in (("c4", cc.cc_c4), ("clusterwild", cc.cc_clusterwild)):
        cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
        sweep = {}
        for e in sorted(set(policy.CANDIDATES) | {eps_fixed}):
            ts = [timed_call(cc, torch, fn, gh, order, e, lab) for _ in range(reps)]
            sweep[e] = (min(t for _, t in ts), ts[-1][0].rounds)
        best = min(sweep, key=lambda e: sweep[e][0])
        cc.cc_set_eps_policy(cc.CC_EPS_LEARNED, w, lo, hi)
        try:
            ts = [timed_call(cc, torch, fn, gh, order, 0.5, lab) for _ in range(reps)]
        finally:
            cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
        torch.cuda.synchronize()
        st = ts[-1][0]
        learned_ms = min(t for _, t in ts)
        r = {"fixed_ms": round(sweep[eps_fixed][0], 3), "fixed_rounds": sweep[eps_fixed][1],
             "best_fixed_eps": round(best, 4), "best_fixed_ms": round(sweep[best][0], 3),
             "best_fixed_rounds": sweep[best][1],
             "learned_ms": round(learned_ms, 3), "learned_rounds": st.rounds,
             "speedup_vs_fixed": round(sweep[eps_fixed][0] / learned_ms, 3),
             "speedup_vs_best_fixed": round(sweep[best][0] / learned_ms, 3),
             "policy_fallback": st.policy_fallback,
             "sweep_ms": {f"{e:.4g}": round(t, 3) for e, (t, _) in sorted(sweep.items())}}
        if name == "c4":
            r["labels_identical"] = bool(torch.equal(lab, lab_ref))
        out[name] = r
    # the other evaluation orders: C4 under the policy against the fixed rule
    import graphgen
    others = {}
    for seed in other_seeds:
        o = torch.from_numpy(graphgen.permutation(order.numel(), seed)).to(order.device)
        ref = torch.empty_like(lab_ref)
        cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
        tf = [timed_call(cc, torch, cc.cc_c4, gh, o, eps_fixed, ref) for _ in range(reps)]
        cc.cc_set_eps_policy(cc.CC_EPS_LEARNED, w, lo, hi)
        try:
            tl = [timed_call(cc, torch, cc.cc_c4, gh, o, 0.5, lab) for _ in range(reps)]
        finally:
            cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
        torch.cuda.synchronize()
        fixed_ms, learned_ms = min(t for _, t in tf), min(t for _, t in tl)
        others[str(seed)] = {"fixed_ms": round(fixed_ms, 3), "fixed_rounds": tf[-1][0].rounds,
                             "learned_ms": round(learned_ms, 3), "learned_rounds": tl[-1][0].rounds,
                             "speedup_vs_fixed": round(fixed_ms / learned_ms, 3),
                             "labels_identical": bool(torch.equal(lab, ref))}
    out["c4_other_orders"] = others
    return out


def bench_practical(cc, torch, gh, order, lab_ref, eps, reps, seed=31, delta=0.1):
    """The paper's practical schedule (Delta-hat halving, Binomial batches over
    pi positions) on the same graph and order as the fixed rule."""
    lab = torch.empty_like(lab_ref)
    out = {"seed": seed, "delta": delta, "eps": eps}
    cc.cc_set_eps_policy(cc.CC_EPS_BINOMIAL, (seed, delta))
    try:
        for name, fn in (("c4", cc.cc_c4), ("clusterwild", cc.cc_clusterwild)):
            ts = [timed_call(cc, torch, fn, gh, order, eps, lab) for _ in range(reps)]
            st = ts[-1][0]
            out[name] = {"call_ms": round(min(t for _, t in ts), 3), "loop_ms": round(st.loop_ms, 3),
                         "rounds": st.rounds, "empty_rounds": int((st.trace["b_i"] == 0).sum())}
            if name == "c4":
                out[name]["labels_identical_to_fixed_rule"] = bool(torch.equal(lab, lab_ref))
    finally:
        cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
    return out


def bench_async(cc, torch, gh, order, lab_ref, n, nnz, deg, reps):
    """Asynchronous C4 and ClusterWild! (Algorithm 3, no rounds) on the same
    graph and order: whole-call time, C4's labels against the round loop's,
    ClusterWild!'s objective against KwikCluster's (C4's)."""
    import numpy as np
    lab = torch.empty_like(lab_ref)
    out = {}
    kc_cost = int(cc.cc_cost(gh, lab_ref)[0])
    for name, fn in (("c4", cc.cc_c4_async), ("clusterwild", cc.cc_clusterwild_async)):
        ts = []
        for _ in range(reps):
            s = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            _, st = fn(gh, order, labels=lab)
            e1.record(s)
            e1.synchronize()
            ts.append((st, e0.elapsed_time(e1)))
        st, call = ts[-1][0], min(t for _, t in ts)
        labels = lab.cpu().numpy()
        centers = labels == np.arange(n, dtype=labels.dtype)
        e_claim = int(deg[centers].sum())
        # per unit as for the round loop; no peel: nothing keeps degrees
        alg = 8 * (e_claim + (int(st.scanned_elect) if name == "c4" else 0)) + 8 * st.atomics + 32 * n
        r = {"call_ms": round(call, 3), "kernel_ms": round(st.loop_ms, 3), "edges_per_s": (nnz // 2) / (call / 1e3),
             "scanned": {"is_center": st.scanned_elect, "claim": st.scanned_claim}, "atomics": st.atomics,
             "alg_bytes_no_peel": alg, "achieved_gbs": alg / (call / 1e3) / 1e9}
        if name == "c4":
            r["labels_identical_to_round_loop"] = bool(torch.equal(lab, lab_ref))
        else:
            cw = int(cc.cc_cost(gh, lab)[0])
            r["cost_over_kwikcluster"] = round(cw / kc_cost, 5) if kc_cost else None
        out[name] = r
    return out


def experiments(cc, torch, graphs, orders, eps_list):
    """The paper's experiment types (Experiments: synchronisation rounds,
    blocked vertices, objective value) on synthetic stand-ins: for each graph,
    `orders` seeded orders, C4 and ClusterWild! at each eps under the fixed
    rule (exact Delta) and under the practical schedule: rounds, the share
    of vertices C4 blocks, and ClusterWild!'s objective relative to
    KwikCluster's (C4's labels are KwikCluster's)."""
    import numpy as np
    import graphgen
    dev = torch.device("cuda:0")
    out = {}
    for name in graphs:
        t = time.perf_counter()
        g = graphgen.workload(name)
        off = torch.from_numpy(np.ascontiguousarray(g.off)).to(dev)
        col = torch.from_numpy(np.ascontiguousarray(g.col)).to(dev)
        gh = cc.cc_graph_from_csr(off, col, borrow=True)
        lab4 = torch.empty(g.n, dtype=torch.int32, device=dev)
        labw = torch.empty(g.n, dtype=torch.int32, device=dev)
        log(f"experiments: {name} n={g.n} m={g.m} ready in {time.perf_counter() - t:.1f} s")
        res = {"n": g.n, "m": g.m, "orders": orders}
        for sched in ("fixed", "practical"):
            for eps in eps_list:
                rows = []
                for k in range(orders):
                    seed = 1000 + k
                    order = torch.from_numpy(graphgen.permutation(g.n, seed)).to(dev)
                    if sched == "practical":
                        cc.cc_set_eps_policy(cc.CC_EPS_BINOMIAL, (seed, 0.1))
                    try:
                        _, s4 = cc.cc_c4(gh, order, eps, labels=lab4, trace_capacity=0)
                        _, sw = cc.cc_clusterwild(gh, order, eps, labels=labw, trace_capacity=0)
                    finally:
                        cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
                    kc = int(cc.cc_cost(gh, lab4)[0])
                    cw = int(cc.cc_cost(gh, labw)[0])
                    rows.append((s4.rounds, sw.rounds, s4.blocked / g.n, cw / kc if kc else 1.0, s4.loop_ms, sw.loop_ms))
                a = np.array(rows, dtype=float)
                res[f"{sched}/eps={eps}"] = {
                    "c4_rounds_mean": round(a[:, 0].mean(), 1), "cw_rounds_mean": round(a[:, 1].mean(), 1),
                    "c4_blocked_pct_mean": round(100 * a[:, 2].mean(), 4), "c4_blocked_pct_max": round(100 * a[:, 2].max(), 4),
                    "cw_over_kc_cost_median": round(float(np.median(a[:, 3])), 5),
                    "cw_over_kc_cost_max": round(a[:, 3].max(), 5),
                    "c4_loop_ms_median": round(float(np.median(a[:, 4])), 3),
                    "cw_loop_ms_median": round(float(np.median(a[:, 5])), 3)}
                log(f"  {name} {sched} eps={eps}: {res[f'{sched}/eps={eps}']}")
        out[name] = res
        del gh, off, col, g
        torch.cuda.empty_cache()
    return out


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(g, order, eps, gpu_labels):
    """The oracle as it stands (serial C, one thread) on the benchmarked graph
    itself: C4's round loop once (ClusterWild! would double the time and
    says nothing more about the CPU)."""
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    ref = oracle.c4(g.off, g.col, order, eps)
    t = time.perf_counter() - t0
    model, ncpu = host_cpu()
    return {"value": g.m / t, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"the benchmarked graph itself (n={g.n}, m={g.m}), one C4 call of the BSP oracle, eps={eps}, "
                      f"one thread: {t:.2f} s, {ref.rounds} rounds",
            "host_cpu": model, "host_nproc": ncpu,
            "labels_match_gpu": bool(np.array_equal(ref.labels, gpu_labels))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat26")
    ap.add_argument("--eps", type=float, default=0.5)
    ap.add_argument("--seed", type=int, default=31)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched and learned-policy lines")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="run one element-wise copy of this many MiB first (counter calibration)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_<workload>.json from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--experiments", default="",
                    help="comma-separated workloads: print the experiment tables (rounds, blocked share, "
                         "ClusterWild!/KwikCluster objective over seeded orders) instead of the benchmark line")
    ap.add_argument("--orders", type=int, default=10, help="orders per graph and eps for --experiments")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, args.workload, args.copy_calibration_mb)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the round loop runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import graphgen
    import paper_1507_05086_amd as cc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.experiments:
        tables = experiments(cc, torch, args.experiments.split(","), args.orders, (0.1, 0.5, 0.9))
        print(json.dumps({"experiments": tables}), flush=True)
        return
    if args.copy_calibration_mb:
        src = torch.ones(args.copy_calibration_mb * 2 ** 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    t = time.perf_counter()
    g = make_graph(args.workload)
    deg = g.degrees()
    log(f"graph {args.workload}: n={g.n} m={g.m} max_deg={int(deg.max())} "
        f"generated in {time.perf_counter() - t:.1f} s")
    off = torch.from_numpy(np.ascontiguousarray(g.off)).to(dev)
    col = torch.from_numpy(np.ascontiguousarray(g.col)).to(dev)
    n, m, nnz = g.n, g.m, g.nnz
    torch.cuda.synchronize()
    t = time.perf_counter()
    gh = cc.cc_graph_from_csr(off, col, borrow=True)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t) * 1e3
    order_h = graphgen.permutation(n, args.seed)
    order = torch.from_numpy(order_h).to(dev)
    lab_c4 = torch.empty(n, dtype=torch.int32, device=dev)
    lab_cw = torch.empty(n, dtype=torch.int32, device=dev)
    cc.cc_set_eps_policy(cc.CC_EPS_FIXED)

    def step():
        s4 = timed_call(cc, torch, cc.cc_c4, gh, order, args.eps, lab_c4)
        sw = timed_call(cc, torch, cc.cc_clusterwild, gh, order, args.eps, lab_cw)
        return s4, sw

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats.append(step())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    value = 2 * m / (ms_per_step / 1e3)

    def summary(runs, labels, c4):
        st = runs[-1][0]
        call = float(np.median([t for _, t in runs]))
        loop = float(np.median([r.loop_ms for r, _ in runs]))
        alg, read, units = algorithmic_bytes(st, n, nnz, deg, labels, c4)
        return {"call_ms": round(call, 3), "loop_ms": round(loop, 3), "rounds": st.rounds,
                "edges_per_s": m / (call / 1e3), "alg_bytes": alg, "achieved_gbs": alg / (call / 1e3) / 1e9,
                "units": units, "read_bytes": read, "read_gbs": read / (call / 1e3) / 1e9,
                "atomics": st.atomics, "blocked": st.blocked,
                "scanned": {"elect": st.scanned_elect, "claim": st.scanned_claim,
                            "delta": st.scanned_delta, "peel": st.scanned_peel}}

    lab4_h, labw_h = lab_c4.cpu().numpy(), lab_cw.cpu().numpy()
    s4 = summary([x[0] for x in stats], lab4_h, True)
    sw = summary([x[1] for x in stats], labw_h, False)
    dom_name, dom = ("cc_c4", s4) if s4["call_ms"] >= sw["call_ms"] else ("cc_clusterwild", sw)
    tr = measured_traffic(args.workload)
    traffic = None
    if tr is not None and dom_name in tr.get("calls", {}):
        traffic = tr["calls"][dom_name]["hbm_bytes"]
    roof = {"bound": "hbm", "achieved": round(dom["achieved_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(dom["achieved_gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": f"one whole {dom_name} call (order check, every round's kernels, labels): "
                      f"algorithmic bytes / call time by HIP events on its stream",
            "read_frac": round(dom["read_gbs"] / HBM_PEAK_GBS, 4)}
    line = {
        "metric": "edges/sec and rounds, C4 & ClusterWild on 1B-edge R-MAT; learned-\u03b5 vs fixed-\u03b5 time",
        "value": value, "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "eps": args.eps, "order_seed": args.seed,
                   "step": "cc_c4 + cc_clusterwild"},
        "setup_ms": round(setup_ms, 1),
        "c4": s4, "clusterwild": sw,
        "roofline": roof,
    }
    if not args.no_extras:
        log("asynchronous variants ...")
        line["async"] = bench_async(cc, torch, gh, order, lab_c4, n, nnz, deg, 3)
        log("practical schedule ...")
        line["practical_schedule"] = bench_practical(cc, torch, gh, order, lab_c4, args.eps, 3)
        log("learned eps policy vs fixed ...")
        line["learned_eps"] = bench_learned(cc, torch, gh, order, lab_c4, args.eps, 2)
        log("batched workload ...")
        line["batched"] = bench_batched(cc, torch, 5)
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        line["cpu_baseline"] = cpu_baseline(g, order_h, args.eps, lab4_h)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
