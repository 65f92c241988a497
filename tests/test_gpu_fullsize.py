"""GPU parity at the full workload sizes, against values the oracle wrote
(tests/golden/*.json, made by tests/golden/make_golden.py): the regenerated
graph's hash, the ordering, the wedge count, the total, and SHA-256 digests of
the whole per-vertex and per-edge arrays (so every element is compared)."""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_1907_08607_amd import graphgen as gg

torch = pytest.importorskip("torch")
pb = pytest.importorskip("paper_1907_08607_amd")

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MAKERS = {
    "powerlaw_50m": lambda: gg.workload_powerlaw_50m(seed=2),
    "hub_100m": lambda: gg.workload_hub_100m(seed=3),
}


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pb.load_library()


@pytest.mark.parametrize("name", sorted(MAKERS))
def test_full_size_workload(name):
    path = os.path.join(GOLDEN, f"{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{name}.json not generated")
    with open(path) as f:
        want = json.load(f)
    g = MAKERS[name]()
    assert g.sha256() == want["csr_sha256"], "generator produced a different graph"
    G = pb.Graph.from_csr(g)
    rank = pb.pb_rank(G, want["rank"])
    r = rank.cpu().numpy().view(np.uint32)
    assert digest(r.astype(np.int64)) == want["rank_sha256"], "ordering differs from the reference"
    stats = pb.pb_stats()
    gl, ve, ed = pb.pb_count(G, rank, stats=stats)
    torch.cuda.synchronize()
    assert stats.wedges == want["wedges"]
    assert int(gl.cpu()[0]) == want["global"]
    v = ve.cpu().numpy()
    e = ed.cpu().numpy()
    for x, c in want["vertex_samples"].items():
        assert v[int(x)] == c, f"vertex {x}"
    for k, c in want["edge_samples"].items():
        assert e[int(k)] == c, f"edge {k}"
    assert int(v.sum()) == want["vertex_sum"] and int(e.sum()) == want["edge_sum"]
    assert digest(v) == want["vertex_sha256"]
    assert digest(e) == want["edge_sha256"]
    G.close()


@pytest.mark.parametrize("name", sorted(MAKERS))
def test_full_size_codeg_rank(name):
    """The exact complement-coreness ordering of the full graph (thousands of
    rounds) against the oracle's digest of it."""
    path = os.path.join(GOLDEN, f"codeg_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"codeg_{name}.json not generated")
    with open(path) as f:
        want = json.load(f)
    g = MAKERS[name]()
    assert g.sha256() == want["csr_sha256"], "generator produced a different graph"
    G = pb.Graph.from_csr(g)
    rank = pb.pb_rank(G, "codeg")
    torch.cuda.synchronize()
    r = rank.cpu().numpy().view(np.uint32)
    assert digest(r.astype(np.int64)) == want["rank_sha256"], "ordering differs from the reference"
    G.close()
