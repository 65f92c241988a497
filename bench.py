"""Benchmark: exact butterfly counting (global + per-vertex + per-edge) on one GPU.

One step = the whole counting path over one resident graph: validate the CSR
and build the V side (pb_graph_create), degree ordering (pb_rank), relabel,
plan, wedge retrieval + aggregation, butterfly credit and output combine
(pb_count with all three outputs).  Inputs are synthetic and already resident
in HBM when the timed region starts.

Default workload: Chung-Lu power-law bipartite graph, |U| = 2M, |V| = 500k,
m = 50M, exponent 2.1 on both sides, max weight 50k, seed 2; degree order.

Prints ONE JSON line (rank 0).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic bytes per wedge of the dense-window kernel: the wedge's x2 is
# read once per pass (4 B); per-vertex output needs the second pass (8 B);
# per-edge output adds one int64 read-modify-write of the credited slot (16 B)
BYTES_PER_WEDGE = {"global": 4, "vertex": 8, "edge": 24, "all": 24}
HBM_PEAK_GBS = 8000.0
INT8_MFMA_PEAK_TOPS = 5000.0  # dense int8 matrix-core peak of the MI355X
PROFILES = os.path.join(ROOT, "profiles")


# The files the counting kernels (and so every profiled kernel) are built from.
KERNEL_SOURCES = ("pb_count.hip", "pb_hub.hip", "pb_internal.h")


def code_only(text):
    """C++ source with its comments and empty lines removed and each run of
    blanks outside string and character literals (kept as written) reduced
    to one space, so only a change of code changes it."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in " \t":
            if out and out[-1] not in " \n":
                out.append(" ")
            i += 1
        elif c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            while i < n and text[i] != "\n":
                i += 1
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return "\n".join(l.strip() for l in "".join(out).split("\n") if l.strip())


def kernel_source_hash():
    """sha256 over the code of the counting kernels' sources, comments left
    out (a measured HBM traffic figure is only quoted for the code it was
    measured on)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1907_08607_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name), encoding="utf-8") as f:
            h.update(name.encode() + b"\0" + code_only(f.read()).encode())
    return h.hexdigest()


def measured_traffic(kernel, workload, outputs):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy calibration), or None
    when there is none for these sources, workload and outputs."""
    path = os.path.join(PROFILES, f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith((" ", "#")):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("source_sha256") != kernel_source_hash() or fields.get("outputs") != outputs:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="powerlaw_50m",
                    choices=["powerlaw_50m", "hub_100m", "er_1k", "batch", "serve", "copy", "approx", "choose", "tip",
                             "wing", "cpu_full"])
    ap.add_argument("--p", type=float, default=0.1, help="approx: sampling rate")
    ap.add_argument("--tip-scale", type=float, default=0.05, help="tip: size of the power-law graph")
    ap.add_argument("--wing-scale", type=float, default=0.003, help="wing: size of the power-law graph")
    ap.add_argument("--graphs", type=int, default=4096, help="batch: graphs in the batch")
    ap.add_argument("--pool-small", type=int, default=10_000, help="serve: resident small graphs")
    ap.add_argument("--pool-big", type=int, default=50, help="serve: resident 5M-edge graphs")
    ap.add_argument("--rate", type=float, default=2000.0, help="serve: Poisson arrivals per second")
    ap.add_argument("--duration", type=float, default=60.0, help="serve: seconds of arrivals")
    ap.add_argument("--slots", type=int, default=4, help="serve: concurrent batches")
    ap.add_argument("--max-batch", type=int, default=64, help="serve: requests per batch")
    ap.add_argument("--seq-requests", type=int, default=20_000,
                    help="serve: first requests of the trace replayed by the sequential baseline")
    ap.add_argument("--tune", action="store_true", help="batch: autotune the per-bucket table first")
    ap.add_argument("--scale", type=float, default=1.0, help="shrink the workload (tests only)")
    ap.add_argument("--rank", default=None, help="ordering (default: the workload's own)")
    ap.add_argument("--agg", default="auto", choices=["auto", "hash", "dense", "sort"])
    ap.add_argument("--hub", default="auto", choices=["auto", "off", "force"], help="hub tile mode")
    ap.add_argument("--outputs", default="all", choices=["all", "global", "vertex", "edge"])
    ap.add_argument("--cache-opt", action="store_true",
                    help="retrieve wedges from their lower-ranked endpoint (same counts)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-target-s", type=float, default=15.0, help="CPU-baseline sample budget")
    return ap.parse_args()


def make_graph(args):
    from paper_1907_08607_amd import graphgen as gg
    if args.workload == "powerlaw_50m":
        g = gg.workload_powerlaw_50m(seed=2, scale=args.scale)
        desc = {"workload": "chung_lu_powerlaw", "n_u": g.n_u, "n_v": g.n_v, "m": g.m, "exponent": 2.1,
                "max_weight": 50_000 * args.scale if args.scale != 1.0 else 50_000, "seed": 2}
        rank = "degree"
    elif args.workload == "hub_100m":
        g = gg.workload_hub_100m(seed=3, scale=args.scale)
        desc = {"workload": "hub_skewed", "n_u": g.n_u, "n_v": g.n_v, "m": g.m, "v_exponent": 1.8,
                "u_geometric_mean": 5, "seed": 3}
        rank = "approx_codeg"
    else:
        g = gg.workload_er_1k(seed=1)
        desc = {"workload": "erdos_renyi", "n_u": g.n_u, "n_v": g.n_v, "m": g.m, "seed": 1}
        rank = "side_auto"
    rank = args.rank or rank
    desc["rank"] = rank
    desc["outputs"] = "global+vertex+edge" if args.outputs == "all" else args.outputs
    return g, desc, rank


def host_info():
    """The host the oracle was timed on: the cores this process may use (what
    `nproc` prints) and the CPU model."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"host_nproc": len(os.sched_getaffinity(0)), "host_cpu": model}


def cpu_baseline(g, wedges, target_s):
    """The oracle (single thread) on every k-th endpoint of its endpoint side,
    scaled to the full run by work.  The oracle's time is a fixed part (input
    checks, the V-side CSR, zeroed output buffers), timed on a sample of one
    endpoint, plus a part proportional to its 2-hop walk, w(t) = sum of deg(s)
    over s in N(t); only the latter is scaled, by (sum of w over all endpoints)
    / (sum of w over the sampled ones).  Scaling the whole sample time by k
    counts the fixed part k times and over-weights whatever heavy endpoints
    the sample happens to hold."""
    import numpy as np

    import oracle
    deg_u = np.diff(g.u_off).astype(np.float64)
    deg_v = np.bincount(g.u_adj, minlength=g.n_v).astype(np.float64)
    # the oracle's side rule: centres on U when its squared-degree sum is smaller
    centers_u = float((deg_u ** 2).sum()) <= float((deg_v ** 2).sum())
    u_of_edge = np.repeat(np.arange(g.n_u), np.diff(g.u_off))
    if centers_u:
        w = np.bincount(g.u_adj, weights=deg_u[u_of_edge], minlength=g.n_v)
    else:
        w = np.bincount(u_of_edge, weights=deg_v[g.u_adj], minlength=g.n_u)
    total_work = float(w.sum())
    n_t = len(w)
    # the run's fixed part (CSR check, V-side build, zeroed buffers): a sample of endpoint 0 alone
    fixed = oracle.count_sample(g, max(1, n_t))
    stride = max(1, int(2.0 * total_work / 2e8))
    t = oracle.count_sample(g, stride)
    # re-aim the stride until the sample's scaled part takes between half and twice the target
    for _ in range(3):
        if stride == 1 or 0.5 * target_s <= t - fixed <= 2.0 * target_s:
            break
        stride = max(1, int(round(max(t - fixed, 1e-3) * stride / target_s)))
        t = oracle.count_sample(g, stride)
    sample_work = float(w[::stride].sum())
    scaled = max(t - fixed, 0.0)
    est = fixed + (scaled * total_work / sample_work if sample_work > 0 else scaled * stride)
    return {"value": wedges / est, "unit": "wedges/s", "cores": 1, "kind": "oracle", **host_info(),
            "sample": f"oracle dense 2-hop counter (global+vertex+edge) on every {stride}-th endpoint "
                      f"of its endpoint side: {t:.1f} s measured, of which {fixed:.1f} s is the run's fixed part; "
                      f"the rest covers {100 * sample_work / total_work:.2f}% of the 2-hop work, so "
                      f"{est:.1f} s estimated full run; wedges = the GPU ordering's wedge count",
            "est_full_s": est}


def run_cpu_full(args):
    """Checks the sampled CPU baseline once (host only, no GPU): the oracle's
    full single-threaded run on the power-law workload next to the estimate
    the cpu_baseline leg makes from its sample."""
    import oracle
    from paper_1907_08607_amd import graphgen as gg
    g = gg.workload_powerlaw_50m(seed=2, scale=args.scale)
    print("[bench] full single-threaded oracle run", file=sys.stderr, flush=True)
    t = time.perf_counter()
    oracle.count(g)
    full = time.perf_counter() - t
    est = cpu_baseline(g, 1, args.cpu_target_s)
    print(json.dumps({"metric": "oracle seconds, full run vs sampled estimate", "workload": "chung_lu_powerlaw",
                      "m": g.m, "full_s": full, "estimate_s": est["est_full_s"],
                      "full_over_estimate": full / est["est_full_s"], "sample": est["sample"], "cores": 1,
                      **host_info()}), flush=True)


def run_copy(args):
    """Copy calibration: a plain device-to-device copy of known size, the
    reference that rocprofv3's FETCH_SIZE / WRITE_SIZE counters are scaled by."""
    import torch
    n = 1 << 26  # 256 MiB of int32
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(args.steps):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.steps
    nbytes = 4 * n
    print(json.dumps({"metric": "copy GB/s", "value": 2 * nbytes / (ms * 1e-3) / 1e9, "unit": "GB/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
                      "config": {"workload": "copy", "bytes_read_per_launch": nbytes,
                                 "bytes_written_per_launch": nbytes}}), flush=True)


def run_approx(args):
    """Approximate total counts by sparsification (Section 4.6): on the
    powerlaw_50m graph, edge and colorful sparsification at rate --p, each
    estimate = sparsify + exact count of the kept graph (graph set-up, degree
    order, global count).  `value` is input edges per second of one edge
    sparsification estimate; the roofline is that of the sparsify pass (keep
    flags, scan, compaction), timed on its own."""
    import argparse as _ap
    import numpy as np
    import torch

    import paper_1907_08607_amd as pb
    g, desc, _ = make_graph(_ap.Namespace(**{**vars(args), "workload": "powerlaw_50m", "rank": "degree"}))
    desc["outputs"] = "global"
    print(f"[bench] graph {desc}", file=sys.stderr, flush=True)
    G = pb.Graph.from_csr(g)
    rank = pb.pb_rank(G, "degree")
    exact = int(pb.pb_count_global(G, rank).cpu()[0])
    res = {}
    for kind in ("edge", "color"):
        for i in range(args.warmup):
            pb.pb_count_approx(G, kind, args.p, 1000 + i)
        ests, times = [], []
        for i in range(args.steps):
            t0 = time.perf_counter()
            c, est, kept = pb.pb_count_approx(G, kind, args.p, 2000 + i)
            times.append(time.perf_counter() - t0)
            ests.append(est)
        # the sparsify pass alone
        for i in range(args.warmup):
            pb.pb_sparsify(G, kind, args.p, 1000 + i)
        torch.cuda.synchronize()
        ts = []
        for i in range(args.steps):
            t0 = time.perf_counter()
            _, adj = pb.pb_sparsify(G, kind, args.p, 2000 + i)
            ts.append(time.perf_counter() - t0)
        res[kind] = {"ms_per_estimate": 1e3 * float(np.mean(times)), "ms_sparsify": 1e3 * float(np.mean(ts)),
                     "kept_edges": int(kept), "estimates": ests,
                     "rel_err_mean": float(np.mean(ests)) / exact - 1.0,
                     "rel_err_rms": float(np.sqrt(np.mean((np.array(ests) / exact - 1.0) ** 2)))}
        print(f"[bench] {kind}: {res[kind]['ms_per_estimate']:.1f} ms per estimate", file=sys.stderr, flush=True)
    G.close()
    e = res["edge"]
    m, kept = g.m, e["kept_edges"]
    # sparsify pass, edge kind: flags written (4 B), scanned (read 4, write 4),
    # compacted (flag, position and id read, 12 B), kept ids written (4 B
    # each), row offsets (u_off 8 B and a position 4 B read, 8 B written)
    nbytes = 24 * m + 4 * kept + 20 * (g.n_u + 1)
    ach = nbytes / (e["ms_sparsify"] * 1e-3) / 1e9
    line = {"metric": "edges/s", "value": m / (e["ms_per_estimate"] * 1e-3), "unit": "edges/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": e["ms_per_estimate"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
            "data": "synthetic",
            "config": {"workload": "approx_powerlaw_50m", "graph": desc, "p": args.p, "exact": exact,
                       "edge": res["edge"], "color": res["color"],
                       "note": "one estimate = sparsify + graph set-up + degree order + exact global count "
                               "of the kept graph; estimates use seeds 2000.."},
            "roofline": {"bound": "hbm", "kernel": "pb_sparsify (edge)", "achieved": ach, "peak": 8000.0,
                         "unit": "GB/s", "frac": ach / 8000.0, "traffic": None, "bytes_per_call": nbytes,
                         "call_ms": e["ms_sparsify"], "note": "host-timed call, includes its launches and "
                                                             "one stream synchronisation"}}
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        oracle.count_approx(g, "edge", args.p, 2000)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": m / dt, "unit": "edges/s", "cores": 1, "kind": "oracle", **host_info(),
                                "sample": f"one edge-sparsification estimate at p={args.p} "
                                          f"(sparsify + dense 2-hop count of the kept graph): {dt:.1f} s"}
    print(json.dumps(line), flush=True)


def run_choose(args):
    """The ranking chooser of Section 6.2 on both single-graph workloads: W
    under side order and under each degree-like order, the metric f, the
    choice, and the time of one choice (ranking both ways + two wedge counts);
    also the time of the exact and approximate complement-coreness orders.
    `value` is input edges per second of the wedge count (pb_wedges) on the
    powerlaw_50m graph under degree order."""
    import argparse as _ap
    import torch

    import paper_1907_08607_amd as pb
    out, wedge_rate = {}, None
    for w in ("powerlaw_50m", "hub_100m"):
        g, desc, _ = make_graph(_ap.Namespace(**{**vars(args), "workload": w, "rank": None}))
        G = pb.Graph.from_csr(g)
        res = {}
        for other in ("approx_degree", "degree", "approx_codeg", "codeg"):
            pb.pb_rank_choose(G, other)
            t0 = time.perf_counter()
            for _ in range(args.steps):
                _, chosen, ws, wr = pb.pb_rank_choose(G, other)
            ms = 1e3 * (time.perf_counter() - t0) / args.steps
            res[other] = {"chosen": chosen, "w_side": ws, "w_other": wr, "f": (ws - wr) / ws if ws else 0.0,
                          "ms_choose": ms}
        for kind in ("codeg", "approx_codeg"):  # the two complement-coreness orders alone
            pb.pb_rank(G, kind)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                pb.pb_rank(G, kind)
            torch.cuda.synchronize()
            res[f"ms_rank_{kind}"] = 1e3 * (time.perf_counter() - t0) / args.steps
        rk = pb.pb_rank(G, "degree")
        torch.cuda.synchronize()
        pb.pb_wedges(G, rk)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            pb.pb_wedges(G, rk)
        ms_w = 1e3 * (time.perf_counter() - t0) / args.steps
        res["ms_wedges_degree"] = ms_w
        if w == "powerlaw_50m":
            wedge_rate = (g.m / (ms_w * 1e-3), ms_w)
        out[w] = res
        G.close()
        print(f"[bench] {w}: {res}", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "edges/s", "value": wedge_rate[0], "unit": "edges/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": 1, "ms_per_step": wedge_rate[1], "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
                      "config": {"workload": "rank_choose", "results": out,
                                 "note": "value: pb_wedges on powerlaw_50m under degree order (host-timed, "
                                         "includes its one synchronisation)"}}), flush=True)


def run_tip(args):
    """Tip decomposition (vertex peeling, Section 3.2 and Algorithm 5) of the
    power-law generator at --tip-scale of the powerlaw_50m size, side chosen
    as the one with the fewest endpoint wedges.  One step = the whole
    decomposition (initial per-vertex count + every peeling round).  `value`
    is input edges per second of one decomposition."""
    import argparse as _ap
    import numpy as np
    import torch

    import paper_1907_08607_amd as pb
    g, desc, _ = make_graph(_ap.Namespace(**{**vars(args), "workload": "powerlaw_50m", "scale": args.tip_scale,
                                               "rank": "degree"}))
    desc["outputs"] = "tip numbers"
    print(f"[bench] graph {desc}", file=sys.stderr, flush=True)
    G = pb.Graph.from_csr(g)
    for _ in range(args.warmup):
        tip, side, rounds = pb.pb_tip_decompose(G)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        tip, side, rounds = pb.pb_tip_decompose(G)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    t = tip.cpu().numpy()
    peeled = t[t >= 0]
    G.close()
    line = {"metric": "edges/s", "value": g.m / (ms * 1e-3), "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "int64", "data": "synthetic",
            "config": {"workload": "tip_decomposition", "graph": desc, "side": side, "rounds": rounds,
                       "ms_per_round": ms / rounds if rounds else None, "peeled_vertices": int(peeled.size),
                       "max_tip": int(peeled.max()) if peeled.size else 0,
                       "note": "one step = initial per-vertex count + all peeling rounds (queued in "
                               "batches of 64, one host synchronisation per batch)"}}
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        want, want_rounds = oracle.tip(g, side)
        dt = time.perf_counter() - t0
        line["config"]["same_as_oracle"] = bool(np.array_equal(want, t)) and want_rounds == rounds
        line["cpu_baseline"] = {"value": g.m / dt, "unit": "edges/s", "cores": 1, "kind": "oracle", **host_info(),
                                "sample": f"the whole decomposition of the same graph: {dt:.1f} s"}
    print(json.dumps(line), flush=True)


def run_wing(args):
    """Wing decomposition (edge peeling, Section 3.2 and Algorithm 6) of the
    power-law generator at --wing-scale of the powerlaw_50m size.  One step =
    the whole decomposition (initial per-edge count + every peeling round).
    `value` is input edges per second of one decomposition."""
    import argparse as _ap
    import numpy as np
    import torch

    import paper_1907_08607_amd as pb
    g, desc, _ = make_graph(_ap.Namespace(**{**vars(args), "workload": "powerlaw_50m", "scale": args.wing_scale,
                                               "rank": "degree"}))
    desc["outputs"] = "wing numbers"
    print(f"[bench] graph {desc}", file=sys.stderr, flush=True)
    G = pb.Graph.from_csr(g)
    for _ in range(args.warmup):
        wing, rounds = pb.pb_wing_decompose(G)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        wing, rounds = pb.pb_wing_decompose(G)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    w = wing.cpu().numpy()
    G.close()
    line = {"metric": "edges/s", "value": g.m / (ms * 1e-3), "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "int64", "data": "synthetic",
            "config": {"workload": "wing_decomposition", "graph": desc, "rounds": rounds,
                       "ms_per_round": ms / rounds if rounds else None, "max_wing": int(w.max()) if w.size else 0,
                       "note": "one step = initial per-edge count + all peeling rounds (queued in batches of 64, "
                               "one host synchronisation per batch)"}}
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        want, want_rounds = oracle.wing(g)
        dt = time.perf_counter() - t0
        line["config"]["same_as_oracle"] = bool(np.array_equal(want, w)) and want_rounds == rounds
        line["cpu_baseline"] = {"value": g.m / dt, "unit": "edges/s", "cores": 1, "kind": "oracle", **host_info(),
                                "sample": f"the whole decomposition of the same graph: {dt:.1f} s"}
    print(json.dumps(line), flush=True)


def upload(graphs, pb):
    return [pb.Graph.from_csr(g) for g in graphs]


def run_batch(args):
    """Batched workload: many uneven graphs counted in one pass vs one launch per graph."""
    import numpy as np
    import torch

    import paper_1907_08607_amd as pb
    from paper_1907_08607_amd import graphgen as gg

    t0 = time.time()
    graphs = gg.workload_batch(args.graphs, seed=4)
    print(f"[bench] {len(graphs)} graphs generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    Gs = upload(graphs, pb)
    ranks = [pb.pb_rank(G, "degree") for G in Gs]
    outs = (None, None, [torch.empty(max(G.m, 1), dtype=torch.int64, device="cuda") for G in Gs])
    tuning = None
    if args.tune:
        sample = list(range(0, len(Gs), max(1, len(Gs) // 256)))
        tuning = pb.pb_autotune([Gs[i] for i in sample], [ranks[i] for i in sample], repeats=3)
        print(f"[bench] autotuned table {tuning.as_dict()}", file=sys.stderr, flush=True)
    stats = pb.pb_stats()
    for _ in range(args.warmup):
        pb.pb_count_batched(Gs, ranks, False, False, True, agg=args.agg, tuning=tuning, outs=outs, stats=stats)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        pb.pb_count_batched(Gs, ranks, False, False, True, agg=args.agg, tuning=tuning, outs=outs, stats=stats)
    torch.cuda.synchronize()
    batched = (time.perf_counter() - t) / args.steps
    # the same work, one graph per launch
    single_outs = [torch.empty(max(G.m, 1), dtype=torch.int64, device="cuda") for G in Gs]
    torch.cuda.synchronize()
    t = time.perf_counter()
    for G, r, o in zip(Gs, ranks, single_outs):
        pb.pb_count(G, r, False, False, True, agg=args.agg, tuning=tuning, outs=(None, None, o))
    torch.cuda.synchronize()
    single = time.perf_counter() - t
    same = all(torch.equal(a[:G.m], b[:G.m]) for a, b, G in zip(outs[2], single_outs, Gs))
    m_total = sum(G.m for G in Gs)
    record = {
        "metric": "graphs/s", "value": len(Gs) / batched, "unit": "graphs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": batched * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "batched_chung_lu", "graphs": len(Gs), "edges_total": m_total,
                   "sizes": "|U|,|V| log-uniform [64, 20k], m log-uniform [256, 5e5] clamped to |U||V|/4, exp 2.1",
                   "rank": "degree", "outputs": "edge", "wedges": stats.wedges,
                   "wedges_per_s": stats.wedges / batched,
                   "tuning": tuning.as_dict() if tuning is not None else "built-in",
                   "one_graph_per_launch_graphs_per_s": len(Gs) / single,
                   "speedup_vs_one_graph_per_launch": single / batched,
                   "same_results_as_one_graph_per_launch": same},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        # the oracle on the batch's graphs in order, for about the target time
        import oracle
        print("[bench] timing the oracle on the host", file=sys.stderr, flush=True)
        done, t_cpu = 0, 0.0
        for g in graphs:
            t1 = time.perf_counter()
            oracle.count(g, want_vertex=False, want_edge=True)
            t_cpu += time.perf_counter() - t1
            done += 1
            if t_cpu >= args.cpu_target_s:
                break
        record["cpu_baseline"] = {"value": done / t_cpu, "unit": "graphs/s", "cores": 1, "kind": "oracle", **host_info(),
                                  "sample": f"oracle dense 2-hop counter (per-edge) on the first {done} of the "
                                            f"{len(graphs)} graphs, one after another: {t_cpu:.1f} s"}
        # the same oracle on every usable core: one thread per core, each
        # taking the next graph (the oracle's C calls release the GIL)
        from concurrent.futures import ThreadPoolExecutor
        cores = host_info()["host_nproc"]
        sample = graphs[:min(len(graphs), done * cores)]
        t1 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=cores) as ex:
            list(ex.map(lambda g: oracle.count(g, want_vertex=False, want_edge=True), sample))
        t_par = time.perf_counter() - t1
        record["cpu_baseline_all_cores"] = {
            "value": len(sample) / t_par, "unit": "graphs/s", "cores": cores, "kind": f"oracle x {cores} threads",
            **host_info(), "sample": f"the first {len(sample)} graphs over {cores} threads: {t_par:.1f} s"}
    print(json.dumps(record), flush=True)


def check_serve_outputs(args, Gs, outs, which, kinds, pb):
    """Compares what the served requests wrote with the oracle's values for
    the pool (tests/golden/serve_pool.json, made by the oracle alone): the
    total of every graph queried for it and the per-vertex / per-edge array
    digests of every graph queried for those.  Every output starts at -1, so
    a graph's output that no request wrote cannot pass."""
    import hashlib

    import numpy as np
    import torch
    path = os.path.join(ROOT, "tests", "golden", "serve_pool.json")
    if args.pool_small != 10_000 or args.pool_big > 50 or not os.path.exists(path):
        return None
    with open(path) as f:
        want = json.load(f)
    print("[bench] checking the served outputs against the oracle's values", file=sys.stderr, flush=True)
    asked = {}
    for gi, k in zip(which.tolist(), kinds.tolist()):
        asked[gi] = asked.get(gi, 0) | int(k)
    torch.cuda.synchronize()
    bad, outputs = [], 0
    for gi, mask in sorted(asked.items()):
        G, (go, vo, eo) = Gs[gi], outs[gi]
        j = gi if gi < args.pool_small else 10_000 + (gi - args.pool_small)
        d16 = lambda t, k: hashlib.sha256(np.ascontiguousarray(t.cpu().numpy()[:k], dtype="<i8").tobytes()
                                          ).hexdigest()[:16]
        if mask & pb.WANT["global"]:
            outputs += 1
            if int(go.cpu()[0]) != want["global"][j]:
                bad.append((gi, "global"))
        if mask & pb.WANT["vertex"]:
            outputs += 1
            if d16(vo, G.n) != want["vertex_sha256_16"][j]:
                bad.append((gi, "vertex"))
        if mask & pb.WANT["edge"]:
            outputs += 1
            if d16(eo, G.m) != want["edge_sha256_16"][j]:
                bad.append((gi, "edge"))
    return {"graphs": len(asked), "outputs": outputs, "all_equal": not bad, "differing": bad[:10]}


def run_serve(args):
    """Serving workload: Poisson arrivals of count queries over a resident pool."""
    import numpy as np
    import torch

    import paper_1907_08607_amd as pb
    from paper_1907_08607_amd import graphgen as gg

    t0 = time.time()
    graphs = gg.workload_serve_pool(args.pool_small, args.pool_big)
    print(f"[bench] pool of {len(graphs)} graphs generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    Gs = upload(graphs, pb)
    ranks = [pb.pb_rank(G, "degree") for G in Gs]
    print(f"[bench] pool resident and ranked ({sum(G.m for G in Gs)} edges)", file=sys.stderr, flush=True)
    # one output set per graph (every request on a graph writes the same values)
    outs = [(torch.full((1,), -1, dtype=torch.int64, device="cuda"),
             torch.full((G.n,), -1, dtype=torch.int64, device="cuda"),
             torch.full((max(G.m, 1),), -1, dtype=torch.int64, device="cuda")) for G in Gs]
    rng = np.random.default_rng(55)
    n_req = int(args.rate * args.duration)
    arrivals = np.cumsum(rng.exponential(1.0 / args.rate, n_req))
    which = rng.integers(0, len(Gs), n_req)
    kinds = rng.choice([pb.WANT["global"], pb.WANT["vertex"], pb.WANT["edge"]], n_req)
    torch.cuda.synchronize()

    def lat_stats(lat):
        lat = np.sort(np.asarray(lat)) * 1e3
        return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))

    # continuous batching server
    srv = pb.Server(hbm_budget=0, slots=args.slots, max_batch=args.max_batch, agg=args.agg)
    gids = [srv.add_graph(G, r) for G, r in zip(Gs, ranks)]
    t_base = time.perf_counter()
    for i in range(n_req):
        if i and i % 20000 == 0:
            print(f"[bench] served {i} of {n_req} arrivals", file=sys.stderr, flush=True)
        wait = arrivals[i] - (time.perf_counter() - t_base)
        if wait > 0:
            time.sleep(wait)
        o = outs[which[i]]
        srv.submit(gids[which[i]], int(kinds[i]), o[0], o[1], o[2])
    srv.drain()
    comps = srv.poll(n_req + 16)
    srv.close()
    assert len(comps) == n_req and all(c.status == 0 for c in comps)
    checked = check_serve_outputs(args, Gs, outs, which, kinds, pb)
    lat = [c.done_s - c.submit_s for c in comps]
    span = max(c.done_s for c in comps) - min(c.submit_s for c in comps)
    p50, p99 = lat_stats(lat)
    batch_sizes = [c.batch for c in comps]
    # sequential one-graph-per-launch serving of the same trace
    seq_lat = []
    t_base = time.perf_counter()
    names = {pb.WANT["global"]: (True, False, False), pb.WANT["vertex"]: (False, True, False),
             pb.WANT["edge"]: (False, False, True)}
    n_seq = min(n_req, args.seq_requests)
    print("[bench] sequential replay", file=sys.stderr, flush=True)
    for i in range(n_seq):
        if i and i % 5000 == 0:
            print(f"[bench] sequential {i} of {n_seq}", file=sys.stderr, flush=True)
        now = time.perf_counter() - t_base
        if arrivals[i] > now:
            time.sleep(arrivals[i] - now)
        wg, wv, we = names[int(kinds[i])]
        o = outs[which[i]]
        pb.pb_count(Gs[which[i]], ranks[which[i]], wg, wv, we, agg=args.agg,
                    outs=(o[0] if wg else None, o[1] if wv else None, o[2] if we else None))
        seq_lat.append(time.perf_counter() - t_base - arrivals[i])
    seq_span = time.perf_counter() - t_base
    s50, s99 = lat_stats(seq_lat)
    record = {
        "metric": "requests/s", "value": n_req / span, "unit": "requests/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": span * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": "serving", "pool_small": args.pool_small, "pool_big": args.pool_big,
                   "rate_per_s": args.rate, "duration_s": args.duration, "requests": n_req, "slots": args.slots,
                   "max_batch": args.max_batch, "p50_ms": p50, "p99_ms": p99,
                   "mean_batch": float(np.mean(batch_sizes)),
                   "sequential_requests": n_seq, "sequential_requests_per_s": n_seq / seq_span, "sequential_p50_ms": s50,
                   "sequential_p99_ms": s99, "oracle_check": checked},
    }
    print(json.dumps(record), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: the counting path "
              "runs on a single device, with no collectives", file=sys.stderr)
        sys.exit(2)
    if args.workload == "cpu_full":
        return run_cpu_full(args)
    import numpy as np
    import torch

    import paper_1907_08607_amd as pb

    pb.load_library()
    torch.cuda.set_device(0)
    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "serve":
        return run_serve(args)
    if args.workload == "copy":
        return run_copy(args)
    if args.workload == "approx":
        return run_approx(args)
    if args.workload == "choose":
        return run_choose(args)
    if args.workload == "tip":
        return run_tip(args)
    if args.workload == "wing":
        return run_wing(args)
    t0 = time.time()
    g, desc, rank_kind = make_graph(args)
    print(f"[bench] graph {desc} built in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    off = torch.from_numpy(g.u_off).cuda()
    adj = torch.from_numpy(g.u_adj.view(np.int32)).cuda()
    outs = (torch.empty(1, dtype=torch.int64, device="cuda"),
            torch.empty(g.n, dtype=torch.int64, device="cuda"),
            torch.empty(g.m, dtype=torch.int64, device="cuda"))
    stream = torch.cuda.current_stream()

    want = {"all": (0, 1, 2), "global": (0,), "vertex": (1,), "edge": (2,)}[args.outputs]
    step_outs = tuple(o if i in want else None for i, o in enumerate(outs))

    def step(stats):
        G = pb.Graph(g.n_u, g.n_v, off, adj, stream)
        r = pb.pb_rank(G, rank_kind, stream=stream)
        pb.pb_count(G, r, agg=args.agg, hub=args.hub, stats=stats, outs=step_outs, stream=stream, timing=True,
                    cache_opt=args.cache_opt)
        G.close()

    for i in range(args.warmup):
        st = pb.pb_stats()
        step(st)
        print(f"[bench] warmup {i} done: {st.wedges} wedges", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    stats = []
    t_start = time.perf_counter()
    for i in range(args.steps):
        st = pb.pb_stats()
        step(st)
        stats.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    print(f"[bench] {args.steps} steps in {elapsed:.3f}s", file=sys.stderr, flush=True)

    wedges = stats[0].wedges
    ms_step = elapsed / args.steps * 1e3
    value = wedges * args.steps / elapsed
    mean = lambda k: sum(getattr(s, k) for s in stats) / len(stats)
    heavy_ms = mean("ms_heavy")
    w_heavy = stats[0].wedges_heavy
    global_ms = mean("ms_global")
    w_global = stats[0].wedges_global
    bpw = BYTES_PER_WEDGE[args.outputs]
    # the roofline is quoted for the counting kernel that takes the most time:
    # the heavy dense-window kernel, or the giant sources' global-histogram
    # path (its walk passes, endpoint step and histogram clear)
    # the committed counter summaries were taken with the default options
    profiled = not args.cache_opt and args.hub == "auto"
    if global_ms > heavy_ms:
        rk, rw, rms = "k_gh_walk (passes 1, 2) + k_gh_endpoint", w_global, global_ms
        parts = [measured_traffic(k, args.workload, args.outputs) if profiled else None
                 for k in ("k_gh_walk_pass1", "k_gh_walk_pass2")]
        traffic = sum(parts) if all(x is not None for x in parts) else None
        traffic_note = "measured traffic of the two walk passes (the endpoint step's is not included)"
    else:
        rk, rw, rms = "k_count_heavy", w_heavy, heavy_ms
        traffic = measured_traffic("k_count_heavy", args.workload, args.outputs) if profiled else None
        traffic_note = None
    achieved = (rw * bpw / (rms * 1e-3)) / 1e9 if rms > 0 else 0.0
    # the unit figure above prices the per-edge credit as an int64
    # read-modify-write; where every slot credit fits 32 bits the library keeps
    # 4-byte counters, so the kernel's own floor is lower: quoted beside it
    sb = stats[0].slot_credit_bytes
    kbpw = bpw if args.outputs in ("global", "vertex") or not sb else 8 + 2 * sb
    achieved_k = (rw * kbpw / (rms * 1e-3)) / 1e9 if rms > 0 else 0.0
    phases = {k: round(mean(k), 3) for k in ("ms_prepare", "ms_heavy", "ms_global", "ms_dense", "ms_hash",
                                              "ms_sort", "ms_hub_gemm", "ms_hub_pass", "ms_output")}
    st0 = stats[0]
    gemm_ms = mean("ms_hub_gemm")
    hub = {"mode": args.hub, "rows": st0.hub_rows, "cols": st0.hub_cols, "wedges_hub": st0.wedges_hub,
           "mfma_int8_ops": st0.hub_mfma_ops,
           "mfma_tops": st0.hub_mfma_ops / (gemm_ms * 1e-3) / 1e12 if gemm_ms > 0 else None}
    hub["mfma_frac"] = hub["mfma_tops"] / INT8_MFMA_PEAK_TOPS if hub["mfma_tops"] else None
    record = {
        "metric": "wedges/s", "value": value, "unit": "wedges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": dict(desc, wedges=wedges, butterflies=int(outs[0].cpu()[0]) if 0 in want else None, phases_ms=phases,
                       wedges_heavy=w_heavy, wedges_global=w_global, wedges_dense=st0.wedges_dense,
                       wedges_hash=st0.wedges_hash,
                       wedges_sort=st0.wedges_sort, window_items=st0.window_items, hub=hub),
        "roofline": {"bound": "hbm", "kernel": rk, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "bytes_per_wedge": bpw, "wedges_per_launch": rw, "launch_ms": rms,
                     "slot_credit_bytes": sb, "kernel_bytes_per_wedge": kbpw,
                     "frac_at_kernel_bytes": achieved_k / HBM_PEAK_GBS},
        "cpu_baseline": None,
    }
    if traffic_note:
        record["roofline"]["traffic_note"] = traffic_note
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle sample on the host", file=sys.stderr, flush=True)
        cb = cpu_baseline(g, wedges, args.cpu_target_s)
        record["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample", "host_nproc", "host_cpu")}
    print(json.dumps(record), flush=True)


if __name__ == "__main__":
    main()
