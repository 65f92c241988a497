"""GPU parity of the wedge count W(rank) (Algorithm 2's retrieved wedges) and
of the ranking chooser of Section 6.2 (side order when f = (w_s - w_r)/w_s
< 0.1).  W must equal the oracle's wedge walk for every ordering kind, and the
chooser must take the same decision as one made from the oracle's counts."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1907_08607_amd import graphgen as gg

torch = pytest.importorskip("torch")
pb = pytest.importorskip("paper_1907_08607_amd")

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pb.load_library()


GRAPHS = {
    "er_planted": lambda: gg.workload_er_1k_planted(1),
    "powerlaw_small": lambda: gg.chung_lu(20_000, 8_000, 200_000, 2.1, 2000, 800, 5),
    "hub_small": lambda: gg.hub_skewed(40_000, 400, 200_000, 1.8, 20_000, 5.0, 3),
    "tiny": lambda: gg.random_small(9, 7, 0.5, 3),
    "empty": lambda: gg.from_edges(4, 3, np.zeros(0, np.int64), np.zeros(0, np.int64)),
}


def rank_tensor(r):
    return torch.from_numpy(np.asarray(r, dtype=np.uint32).view(np.int32)).cuda()


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("kind", sorted(oracle.RANK_KINDS))
def test_wedges_match_oracle(name, kind):
    g = GRAPHS[name]()
    r = oracle.rank(g, kind)
    G = pb.Graph.from_csr(g)
    assert pb.pb_wedges(G, rank_tensor(r)) == oracle.wedges(g, r)
    G.close()


@pytest.mark.parametrize("name", ["er_planted", "powerlaw_small", "hub_small", "empty"])
@pytest.mark.parametrize("other", ["approx_degree", "degree", "approx_codeg"])
def test_chooser_matches_oracle_decision(name, other):
    g = GRAPHS[name]()
    ws = oracle.wedges(g, oracle.rank(g, "side_auto"))
    wr = oracle.wedges(g, oracle.rank(g, other))
    want = "side_auto" if (wr >= ws or 10 * (ws - wr) < ws) else other
    G = pb.Graph.from_csr(g)
    r, chosen, w_side, w_other = pb.pb_rank_choose(G, other)
    torch.cuda.synchronize()
    assert (chosen, w_side, w_other) == (want, ws, wr)
    assert np.array_equal(r.cpu().numpy().view(np.uint32), oracle.rank(g, want))
    G.close()


def test_chooser_takes_both_branches():
    # a uniform graph favours side order, a skewed one the degree-like order
    decisions = set()
    for name in ("er_planted", "powerlaw_small"):
        G = pb.Graph.from_csr(GRAPHS[name]())
        decisions.add(pb.pb_rank_choose(G, "approx_degree")[1])
        G.close()
    assert decisions == {"side_auto", "approx_degree"}


@pytest.mark.parametrize("name,maker", [("powerlaw_50m", lambda: gg.workload_powerlaw_50m(seed=2)),
                                        ("hub_100m", lambda: gg.workload_hub_100m(seed=3))])
def test_full_size_wedges(name, maker):
    path = os.path.join(GOLDEN, f"{name}.json")
    if not os.path.exists(path):
        pytest.skip("golden values not generated")
    want = json.load(open(path))
    G = pb.Graph.from_csr(maker())
    rank = pb.pb_rank(G, want["rank"])
    assert pb.pb_wedges(G, rank) == want["wedges"]
    G.close()
