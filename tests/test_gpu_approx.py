"""GPU parity of approximate counting by sparsification (Section 4.6
"Approximate counting"): the kept graph must equal the oracle's edge for edge
(both draw from the same counter-based generator, SplitMix64), its exact count
must equal the oracle's, and the scaled estimate must be the same double."""
import hashlib

import numpy as np
import pytest

import oracle
from paper_1907_08607_amd import graphgen as gg

torch = pytest.importorskip("torch")
pb = pytest.importorskip("paper_1907_08607_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pb.load_library()


def kept_on_gpu(g, kind, p, seed):
    G = pb.Graph.from_csr(g)
    off, adj = pb.pb_sparsify(G, kind, p, seed)
    torch.cuda.synchronize()
    out = off.cpu().numpy(), adj.cpu().numpy().view(np.uint32)
    G.close()
    return out


GRAPHS = {
    "er_1k": lambda: gg.workload_er_1k(1),
    "er_planted": lambda: gg.workload_er_1k_planted(1),
    "powerlaw_small": lambda: gg.chung_lu(20_000, 8_000, 200_000, 2.1, 2000, 800, 5),
    "tiny": lambda: gg.random_small(9, 7, 0.5, 3),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("kind,p,seed", [("edge", 0.5, 1), ("edge", 0.1, 2), ("edge", 0.999, 3),
                                         ("color", 0.5, 4), ("color", 0.2, 5), ("color", 0.34, 6)])
def test_kept_graph_matches_oracle(name, kind, p, seed):
    g = GRAPHS[name]()
    want = oracle.sparsify(g, kind, p, seed)
    off, adj = kept_on_gpu(g, kind, p, seed)
    assert np.array_equal(off, want.u_off)
    assert np.array_equal(adj, want.u_adj)


@pytest.mark.parametrize("kind", ["edge", "color"])
def test_p_one_is_the_input(kind):
    g = GRAPHS["er_planted"]()
    off, adj = kept_on_gpu(g, kind, 1.0, 9)
    assert np.array_equal(off, g.u_off) and np.array_equal(adj, g.u_adj)


def test_nothing_kept_and_empty_graph():
    g = GRAPHS["er_1k"]()
    off, adj = kept_on_gpu(g, "edge", 1e-12, 1)  # threshold ~2^24.1: no edge of 10^4 survives
    assert adj.size == 0 and not off.any()
    G = pb.Graph.from_csr(g)
    c, est, kept = pb.pb_count_approx(G, "edge", 1e-12, 1)
    assert (c, est, kept) == (0, 0.0, 0)
    G.close()
    e = gg.from_edges(5, 4, np.zeros(0, np.int64), np.zeros(0, np.int64))
    G = pb.Graph.from_csr(e)
    for kind in ("edge", "color"):
        assert pb.pb_count_approx(G, kind, 0.5, 3) == (0, 0.0, 0)
    G.close()


@pytest.mark.parametrize("name", ["er_planted", "powerlaw_small"])
@pytest.mark.parametrize("kind,p,seed", [("edge", 0.5, 11), ("color", 0.5, 12), ("color", 0.25, 13),
                                         ("edge", 1.0, 14)])
@pytest.mark.parametrize("rank", ["degree", "side_auto"])
def test_count_approx_matches_oracle(name, kind, p, seed, rank):
    g = GRAPHS[name]()
    c_want, est_want, kept_want = oracle.count_approx(g, kind, p, seed)
    G = pb.Graph.from_csr(g)
    c, est, kept = pb.pb_count_approx(G, kind, p, seed, rank=rank)
    G.close()
    assert (c, kept) == (c_want, kept_want)
    assert est == est_want  # the same double expression on both sides


def test_rejects_bad_p():
    G = pb.Graph.from_csr(GRAPHS["tiny"]())
    for kind, bad in (("edge", 0.0), ("edge", 1.5), ("color", float("nan")), ("color", 1e-12)):
        with pytest.raises(pb.PBError):
            pb.pb_sparsify(G, kind, bad, 1)
    G.close()


def test_full_size_kept_graph_digest():
    """The powerlaw_50m graph (|U|=2M, |V|=500k, m=50M) at p = 0.1, both
    kinds: the kept CSR's SHA-256 equals the oracle's (every kept edge)."""
    g = gg.workload_powerlaw_50m(seed=2)
    for kind, seed in (("edge", 21), ("color", 22)):
        want = oracle.sparsify(g, kind, 0.1, seed)
        off, adj = kept_on_gpu(g, kind, 0.1, seed)
        h = lambda a, b: hashlib.sha256(np.ascontiguousarray(a, "<i8").tobytes() +
                                        np.ascontiguousarray(b, "<u4").tobytes()).hexdigest()
        assert adj.size == want.m
        assert h(off, adj) == h(want.u_off, want.u_adj)
