"""Writes the expected values for the full-size parity tests.

Calls only the CPU oracle (oracle/) and the seeded input generators; no value
here comes from the GPU library.  For each workload it records the CSR hash
(so a test can confirm it regenerated the same graph), the butterfly total,
SHA-256 digests of the per-vertex and per-edge int64 arrays (little endian),
the wedge count of the workload's ordering, and a sample of single values.
With --codeg it records instead the digest of the exact complement-coreness
ordering of each workload's graph (codeg_<name>.json).

The many-graph workloads are recorded per graph: ``batch`` (the 4096
batched graphs, per-edge counts) writes batch_4096.json and ``serve`` (the
10,050-graph serving pool, all three outputs) writes serve_pool.json, each
graph's total and the first 16 hex digits of its arrays' SHA-256 digests.
Their oracle calls run on every host core (one graph per thread).

    python tests/golden/make_golden.py powerlaw_50m hub_100m
    python tests/golden/make_golden.py --codeg powerlaw_50m hub_100m
    python tests/golden/make_golden.py batch serve
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1907_08607_amd import graphgen as gg  # noqa: E402

WORKLOADS = {
    "powerlaw_50m": (lambda: gg.workload_powerlaw_50m(seed=2), "degree",
                     "Chung-Lu power law, |U|=2M, |V|=500k, m=50M, exponent 2.1, max weight 50k, seed 2"),
    "hub_100m": (lambda: gg.workload_hub_100m(seed=3), "approx_codeg",
                 "hub-skewed, |U|=20M, |V|=100k, m=100M, V power law 1.8 up to 1M, U geometric mean 5, seed 3"),
}


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


def make(name: str) -> dict:
    make_graph, rank_kind, desc = WORKLOADS[name]
    t = time.time()
    g = make_graph()
    print(f"{name}: generated in {time.time() - t:.1f}s", flush=True)
    t = time.time()
    glob, vert, edge = oracle.count(g)
    print(f"{name}: oracle counts in {time.time() - t:.1f}s", flush=True)
    t = time.time()
    rank = oracle.rank(g, rank_kind)
    wedges = oracle.wedges(g, rank)
    print(f"{name}: ranking + wedges in {time.time() - t:.1f}s", flush=True)
    rng = np.random.default_rng(12345)
    vs = sorted(set(rng.integers(0, g.n, 64).tolist()) | {int(np.argmax(vert))})
    es = sorted(set(rng.integers(0, g.m, 64).tolist()) | {int(np.argmax(edge))})
    return {
        "workload": name, "description": desc, "csr_sha256": g.sha256(),
        "n_u": g.n_u, "n_v": g.n_v, "m": g.m, "rank": rank_kind, "rank_sha256": digest(rank.astype(np.int64)),
        "wedges": wedges, "global": glob, "vertex_sha256": digest(vert), "edge_sha256": digest(edge),
        "vertex_sum": int(vert.sum()), "edge_sum": int(edge.sum()),
        "vertex_samples": {str(x): int(vert[x]) for x in vs},
        "edge_samples": {str(e): int(edge[e]) for e in es},
        "made_by": "tests/golden/make_golden.py (oracle/orc_count, orc_rank, orc_wedges)",
    }


def make_codeg(name: str) -> dict:
    make_graph, _, desc = WORKLOADS[name]
    g = make_graph()
    t = time.time()
    rank = oracle.rank(g, "codeg")
    print(f"{name}: complement coreness in {time.time() - t:.1f}s", flush=True)
    return {
        "workload": name, "description": desc, "csr_sha256": g.sha256(), "rank": "codeg",
        "rank_sha256": digest(rank.astype(np.int64)),
        "made_by": "tests/golden/make_golden.py --codeg (oracle/orc_rank)",
    }


def short(a: np.ndarray) -> str:
    return digest(a)[:16]


def oracle_all(graphs, want_vertex: bool):
    """oracle.count of every graph, one graph per thread (the C calls run
    without the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=os.cpu_count() or 1) as ex:
        return list(ex.map(lambda g: oracle.count(g, want_vertex=want_vertex, want_edge=True), graphs))


def graphs_digest(graphs) -> str:
    h = hashlib.sha256()
    for g in graphs:
        h.update(g.sha256().encode())
    return h.hexdigest()


def make_batch() -> dict:
    t = time.time()
    gs = gg.workload_batch(4096, seed=4)
    print(f"batch: generated in {time.time() - t:.1f}s", flush=True)
    t = time.time()
    res = oracle_all(gs, want_vertex=False)
    print(f"batch: oracle counts in {time.time() - t:.1f}s", flush=True)
    return {
        "workload": "batch", "description": "4096 Chung-Lu graphs, |U|,|V| log-uniform [64, 20k], m log-uniform "
        "[256, 5e5] clamped to |U||V|/4, exponent 2.1, seed 4",
        "count": len(gs), "graphs_sha256": graphs_digest(gs), "edges_total": int(sum(g.m for g in gs)),
        "global": [r[0] for r in res], "edge_sha256_16": [short(r[2]) for r in res],
        "made_by": "tests/golden/make_golden.py batch (oracle/orc_count)",
    }


def make_serve() -> dict:
    t = time.time()
    gs = gg.workload_serve_pool()
    print(f"serve: generated in {time.time() - t:.1f}s", flush=True)
    t = time.time()
    res = oracle_all(gs, want_vertex=True)
    print(f"serve: oracle counts in {time.time() - t:.1f}s", flush=True)
    return {
        "workload": "serve", "description": "serving pool: 10,000 graphs shaped as the batch (seed 5) and 50 "
        "Chung-Lu graphs with |U|=200k, |V|=50k, m=5M, exponent 2.1",
        "count": len(gs), "graphs_sha256": graphs_digest(gs), "edges_total": int(sum(g.m for g in gs)),
        "global": [r[0] for r in res], "vertex_sha256_16": [short(r[1]) for r in res],
        "edge_sha256_16": [short(r[2]) for r in res],
        "made_by": "tests/golden/make_golden.py serve (oracle/orc_count)",
    }


MANY = {"batch": ("batch_4096.json", make_batch), "serve": ("serve_pool.json", make_serve)}


if __name__ == "__main__":
    if sys.argv[1:] and all(a in MANY for a in sys.argv[1:]):
        for name in sys.argv[1:]:
            fname, fn = MANY[name]
            d = fn()
            with open(os.path.join(HERE, fname), "w") as f:
                json.dump(d, f, separators=(",", ":"))
            print(json.dumps({k: d[k] for k in ("workload", "count", "edges_total")}), flush=True)
        sys.exit(0)
    if sys.argv[1:2] == ["--codeg"]:
        for name in sys.argv[2:] or list(WORKLOADS):
            d = make_codeg(name)
            with open(os.path.join(HERE, f"codeg_{name}.json"), "w") as f:
                json.dump(d, f, indent=1)
            print(json.dumps({k: d[k] for k in ("workload", "rank_sha256")}), flush=True)
        sys.exit(0)
    for name in sys.argv[1:] or list(WORKLOADS):
        d = make(name)
        with open(os.path.join(HERE, f"{name}.json"), "w") as f:
            json.dump(d, f, indent=1)
        print(json.dumps({k: d[k] for k in ("workload", "global", "wedges", "m")}), flush=True)
