"""GPU parity of wing decomposition (edge peeling, Section 3.2 and
Algorithm 6): the wing numbers and the number of rounds must equal the
oracle's."""
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
    "powerlaw_small": lambda: gg.chung_lu(4_000, 2_000, 30_000, 2.1, 400, 200, 5),
    "hub_small": lambda: gg.hub_skewed(8_000, 100, 30_000, 1.8, 3_000, 5.0, 3),
    "union": lambda: gg.disjoint_union(gg.random_small(10, 9, 0.5, 4), gg.complete(5, 6)),
    "empty": lambda: gg.from_edges(4, 3, np.zeros(0, np.int64), np.zeros(0, np.int64)),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_wings_match_oracle(name):
    g = GRAPHS[name]()
    want, want_rounds = oracle.wing(g)
    G = pb.Graph.from_csr(g)
    wing, rounds = pb.pb_wing_decompose(G)
    torch.cuda.synchronize()
    got = wing.cpu().numpy()
    G.close()
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"differs at {bad[:10]}: {got[bad[:10]]} vs {want[bad[:10]]}"
    assert rounds == want_rounds
