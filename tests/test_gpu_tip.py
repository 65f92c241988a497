"""GPU parity of tip decomposition (vertex peeling, Section 3.2 and
Algorithm 5): the tip numbers and the number of rounds must equal the
oracle's on every graph and side."""
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


GRAPHS = {
    "tiny": lambda: gg.random_small(9, 8, 0.5, 3),
    "complete": lambda: gg.complete(7, 5),
    "er_planted": lambda: gg.workload_er_1k_planted(1),
    "powerlaw_small": lambda: gg.chung_lu(20_000, 8_000, 200_000, 2.1, 2000, 800, 5),
    "hub_small": lambda: gg.hub_skewed(40_000, 400, 200_000, 1.8, 20_000, 5.0, 3),
    "empty": lambda: gg.from_edges(4, 3, np.zeros(0, np.int64), np.zeros(0, np.int64)),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("side", ["auto", "u", "v"])
def test_tips_match_oracle(name, side):
    g = GRAPHS[name]()
    want, want_rounds = oracle.tip(g, side)
    G = pb.Graph.from_csr(g)
    tip, peeled, rounds = pb.pb_tip_decompose(G, side)
    torch.cuda.synchronize()
    got = tip.cpu().numpy()
    G.close()
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"differs at {bad[:10]}: {got[bad[:10]]} vs {want[bad[:10]]}"
    if g.n_u + g.n_v:
        assert rounds == want_rounds
    if side != "auto":
        assert peeled == side


def test_disjoint_union_and_transpose():
    g = gg.disjoint_union(gg.random_small(10, 9, 0.5, 4), gg.complete(5, 6))
    G = pb.Graph.from_csr(g)
    tip, _, _ = pb.pb_tip_decompose(G, "u")
    assert np.array_equal(tip.cpu().numpy(), oracle.tip(g, "u")[0])
    G.close()
    t = gg.transpose(g)
    T = pb.Graph.from_csr(t)
    tt, _, _ = pb.pb_tip_decompose(T, "v")
    # peeling V of the transpose is peeling U of the original
    assert np.array_equal(tt.cpu().numpy()[t.n_u:], tip.cpu().numpy()[:g.n_u])
    T.close()
