"""GPU parity of the exact complement-coreness ordering (Section 3.1.1) against
the oracle's round-by-round definition: each round removes every remaining
vertex whose number of remaining neighbours is the largest, and those vertices
take the next ranks in id order.

The GPU path works in key windows: the live vertices whose keys lie in the top
run of keys holding at most 4096 vertices.  One workgroup runs the rounds
inside a window; a round whose removed vertices have more than 16384
neighbours to visit, and a window that is one key of more than 4096 vertices,
run on all workgroups.  The graphs below reach each of these cases:
  * the power law at 1/50 size: several windows, the last one key 1 of more
    than 4096 vertices;
  * three giant V vertices of degree 40000: rounds handed to all workgroups;
  * the hub-skewed generator at 1/200 size: 500 V vertices over 100k U ones;
  * all of them with U and V swapped, and graphs with isolated vertices."""
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
    "powerlaw_1_50": lambda: gg.workload_powerlaw_50m(scale=0.02),
    "giant_hubs": lambda: gg.giant_hubs(60_000, 3_000, 3, 40_000, 2, 5),
    "hub_1_200": lambda: gg.workload_hub_100m(scale=0.005),
    # 5000 isolated U vertices after a small random part: key 0 alone is a
    # window of more than 4096 vertices
    "isolated": lambda: gg.from_edges(5300, 200, *np.nonzero(np.random.default_rng(9).random((300, 200)) < 0.05)),
    "empty_edges": lambda: gg.from_edges(3000, 1000, [], []),
}


def gpu_rank(g, kind="codeg"):
    G = pb.Graph.from_csr(g)
    r = pb.pb_rank(G, kind)
    torch.cuda.synchronize()
    out = r.cpu().numpy().view(np.uint32).copy()
    G.close()
    return out


@pytest.mark.parametrize("transposed", [False, True])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_codeg_matches_oracle(name, transposed):
    g = GRAPHS[name]()
    if transposed:
        g = gg.transpose(g)
    want = np.asarray(oracle.rank(g, "codeg"), dtype=np.uint32)
    got = gpu_rank(g)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{name}: rank differs at {bad[:10]} got {got[bad[:10]]} want {want[bad[:10]]}"


def test_codeg_repeatable_and_counts():
    """Two calls give the same permutation, and counting under it gives the
    oracle's counts (the ordering changes only the work, never the result)."""
    g = GRAPHS["giant_hubs"]()
    a, b = gpu_rank(g), gpu_rank(g)
    assert np.array_equal(a, b)
    assert np.array_equal(np.sort(a), np.arange(g.n, dtype=np.uint32))
    G = pb.Graph.from_csr(g)
    r = torch.from_numpy(a.view(np.int32)).cuda()
    gl, ve, ed = pb.pb_count(G, r)
    torch.cuda.synchronize()
    want = oracle.count(g)
    assert int(gl.cpu()[0]) == want[0]
    assert np.array_equal(ve.cpu().numpy(), want[1])
    assert np.array_equal(ed.cpu().numpy(), want[2])
    G.close()
