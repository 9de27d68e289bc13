#!/usr/bin/env python3
"""Throughput of the C4 + ClusterWild! round loop on one MI355X.

A step is one cc_c4 call plus one cc_clusterwild call (fixed eps rule) on the
same resident graph and order: every step of the hot path (delta, active-set
selection, election, claims, peeling, labels) runs once per algorithm.
`value` is positive edges clustered per second over the step:
2 * m / step_time.  Inputs (CSR, order, output buffers) are in HBM before the
timed region starts.

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


def algorithmic_bytes(st, n):
    """Bytes the method itself must move in one call (see the design notes):
    8 B per adjacency item scanned (4 B column + 4 B neighbour word) in the
    election, claim, degree-refresh and peel passes, 8 B per atomic
    read-modify-write, and 32 B per vertex (offsets, order, rank, initial
    state, final label)."""
    scanned = st.scanned_elect + st.scanned_claim + st.scanned_delta + st.scanned_peel
    return 8 * scanned + 8 * st.atomics + 32 * n


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


CALL_FIRST, CALL_LAST = "k_check_order", "k_finalize"


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
            short = name.split("(")[0].split("::")[-1]
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
    lab = torch.empty(g.n, dtype=torch.int32, device=dev)
    out = {"workload": "sbm4096", "graphs": g.ngraphs, "n": g.n, "m": g.m}
    for name, algo, fn in (("c4", cc.CC_ALGO_C4, cc.cc_c4), ("clusterwild", cc.CC_ALGO_CLUSTERWILD, cc.cc_clusterwild)):
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
    return out


def bench_learned(cc, torch, gh, order, lab_ref, fixed_stats, reps):
    """Learned eps policy against the fixed rule (eps = 0.5) on the same graph."""
    import numpy as np
    from paper_1507_05086_amd import policy
    w, lo, hi = policy.load()
    lab = torch.empty_like(lab_ref)
    cc.cc_set_eps_policy(cc.CC_EPS_LEARNED, w, lo, hi)
    try:
        ks = []
        for _ in range(reps):
            _, st = cc.cc_c4(gh, order, 0.5, labels=lab)
            ks.append(st.loop_ms)
    finally:
        cc.cc_set_eps_policy(cc.CC_EPS_FIXED)
    torch.cuda.synchronize()
    same = bool(torch.equal(lab, lab_ref))
    fixed_ms = float(np.median([s.loop_ms for s in fixed_stats]))
    learned_ms = float(np.median(ks))
    return {"fixed_eps": 0.5, "fixed_ms": round(fixed_ms, 3), "fixed_rounds": fixed_stats[-1].rounds,
            "learned_ms": round(learned_ms, 3), "learned_rounds": st.rounds,
            "speedup": round(fixed_ms / learned_ms, 3), "labels_identical": same,
            "policy_fallback": st.policy_fallback}


def cpu_baseline(sample):
    """The oracle, as it stands, on a bounded sample of the same graph family."""
    import graphgen
    import oracle
    g = graphgen.workload(sample)
    order = graphgen.permutation(g.n, 31)
    t0 = time.perf_counter()
    oracle.c4(g.off, g.col, order, 0.5)
    t1 = time.perf_counter()
    oracle.clusterwild(g.off, g.col, order, 0.5)
    t2 = time.perf_counter()
    return {"value": 2 * g.m / (t2 - t0), "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample} (n={g.n}, m={g.m}), C4 + ClusterWild! BSP oracle, eps=0.5, one thread: "
                      f"C4 {t1 - t0:.2f} s, ClusterWild! {t2 - t1:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat26")
    ap.add_argument("--eps", type=float, default=0.5)
    ap.add_argument("--seed", type=int, default=31)
    ap.add_argument("--cpu-sample", default="rmat23")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched and learned-policy lines")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="run one element-wise copy of this many MiB first (counter calibration)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_<workload>.json from two rocprofv3 --pmc runs and exit")
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
    if args.copy_calibration_mb:
        src = torch.ones(args.copy_calibration_mb * 2 ** 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    t = time.perf_counter()
    g = make_graph(args.workload)
    log(f"graph {args.workload}: n={g.n} m={g.m} max_deg={int(g.degrees().max())} "
        f"generated in {time.perf_counter() - t:.1f} s")
    off = torch.from_numpy(np.ascontiguousarray(g.off)).to(dev)
    col = torch.from_numpy(np.ascontiguousarray(g.col)).to(dev)
    n, m = g.n, g.m
    del g
    gh = cc.cc_graph_from_csr(off, col, borrow=True)
    order = torch.from_numpy(graphgen.permutation(n, args.seed)).to(dev)
    lab_c4 = torch.empty(n, dtype=torch.int32, device=dev)
    lab_cw = torch.empty(n, dtype=torch.int32, device=dev)
    cc.cc_set_eps_policy(cc.CC_EPS_FIXED)

    def step():
        _, s4 = cc.cc_c4(gh, order, args.eps, labels=lab_c4)
        _, sw = cc.cc_clusterwild(gh, order, args.eps, labels=lab_cw)
        return s4, sw

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        stats.append(step())
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    value = 2 * m / (ms_per_step / 1e3)

    c4 = [s[0] for s in stats]
    cw = [s[1] for s in stats]

    def summary(runs):
        loop = float(np.mean([r.loop_ms for r in runs]))
        nbytes = algorithmic_bytes(runs[-1], n)
        return {"loop_ms": round(loop, 3), "rounds": runs[-1].rounds, "edges_per_s": m / (loop / 1e3),
                "alg_bytes": nbytes, "achieved_gbs": nbytes / (loop / 1e3) / 1e9,
                "atomics": runs[-1].atomics,
                "scanned": {"elect": runs[-1].scanned_elect, "claim": runs[-1].scanned_claim,
                            "delta": runs[-1].scanned_delta, "peel": runs[-1].scanned_peel}}

    s4, sw = summary(c4), summary(cw)
    dom = s4 if s4["loop_ms"] >= sw["loop_ms"] else sw
    dom_name = "cc_c4" if dom is s4 else "cc_clusterwild"
    tr = measured_traffic(args.workload)
    traffic = None
    if tr is not None and dom_name in tr.get("calls", {}):
        traffic = tr["calls"][dom_name]["hbm_bytes"]
    roof = {"bound": "hbm", "achieved": round(dom["achieved_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(dom["achieved_gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "round loop of " + dom_name + " (all kernels of one call)"}
    line = {
        "metric": "edges/sec (C4 + ClusterWild! round loop, fixed eps)",
        "value": value, "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "eps": args.eps, "order_seed": args.seed,
                   "step": "cc_c4 + cc_clusterwild"},
        "c4": s4, "clusterwild": sw,
        "roofline": roof,
    }
    if not args.no_extras:
        log("learned eps policy vs fixed ...")
        line["learned_eps"] = bench_learned(cc, torch, gh, order, lab_c4, c4, 3)
        log("batched workload ...")
        line["batched"] = bench_batched(cc, torch, 5)
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        line["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
