"""GPU parity at the limits of the heavy kernel's narrow window counters.

Above the last vertex of its side with degree >= 16, a heavy source counts its
candidates in 4-bit counters; above the last one with degree >= 256, in 8-bit
counters.  Both rest on R(x1, x2) <= deg(x2) (Section 3.1.2's wedge count of a
pair cannot exceed the degree of either endpoint).  These graphs put
candidates exactly at each limit: a source x1 adjacent to centres 0..big-1, and
groups of same-side vertices adjacent to centres 0..d-1 for d = 15, 16, 255,
256, so R(x1, x2) = deg(x2) = d.  A counter one bit too narrow, or a threshold
one vertex off, wraps a count and fails the comparison.  Filler vertices of
degree 1 to 3 stretch the candidate range past the whole-range dense kernel's
4096 ids, so the sources take the windowed heavy kernel."""
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


def bound_graph(big, groups, filler, seed):
    """U0 is adjacent to V 0..big-1; each group (count, d) adds `count` U
    vertices adjacent to V 0..d-1; then `filler` U vertices of degree 1..3."""
    rng = np.random.default_rng(seed)
    u, v = [0] * big, list(range(big))
    nxt = 1
    for count, d in groups:
        for _ in range(count):
            u += [nxt] * d
            v += list(range(d))
            nxt += 1
    for _ in range(filler):
        k = int(rng.integers(1, 4))
        cols = rng.choice(big, size=k, replace=False)
        u += [nxt] * k
        v += cols.tolist()
        nxt += 1
    return gg.from_edges(nxt, big, u, v)


CASES = {
    # x1 has 300 up-slots: the wave path with its run state in registers
    "wave": dict(big=300, groups=[(40, 15), (40, 16), (5, 255), (5, 256)], filler=6000, seed=11),
    # x1 and the 70 vertices of degree 1400 have more than 1024 up-slots and
    # long runs: the block-wide path; R = 1400 lands in the 16-bit windows
    "block": dict(big=1500, groups=[(70, 1400), (40, 15), (40, 16), (5, 255), (5, 256)], filler=6000, seed=12),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    c = CASES[request.param]
    g = bound_graph(**c)
    deg_u = np.diff(np.asarray(g.u_off))
    # the construction's premise: every centre ranks below x1 under degree
    # order, so R(x1, x2) = deg(x2) for each group vertex
    deg_v = np.bincount(np.asarray(g.u_adj), minlength=g.n_v)
    assert deg_v.max() < c["big"] == deg_u[0]
    return request.param, g, oracle.count(g)


def run(g, agg, hub):
    G = pb.Graph.from_csr(g)
    r = torch.from_numpy(np.asarray(oracle.rank(g, "degree"), dtype=np.uint32).view(np.int32)).cuda()
    st = pb.pb_stats()
    gl, ve, ed = pb.pb_count(G, r, agg=agg, hub=hub, stats=st)
    torch.cuda.synchronize()
    out = (int(gl.cpu()[0]), ve.cpu().numpy(), ed.cpu().numpy())
    G.close()
    return out, st


def assert_same(got, want, what):
    assert got[0] == want[0], f"{what}: global {got[0]} != {want[0]}"
    bad = np.nonzero(got[1] != want[1])[0]
    assert bad.size == 0, f"{what}: per-vertex differs at {bad[:10]} got {got[1][bad[:10]]} want {want[1][bad[:10]]}"
    bad = np.nonzero(got[2] != want[2])[0]
    assert bad.size == 0, f"{what}: per-edge differs at {bad[:10]} got {got[2][bad[:10]]} want {want[2][bad[:10]]}"


@pytest.mark.parametrize("hub", ["off", "auto"])
@pytest.mark.parametrize("agg", ["dense", "auto"])
def test_counter_limits(case, agg, hub):
    name, g, want = case
    got, st = run(g, agg, hub)
    assert_same(got, want, f"{name} agg={agg} hub={hub}")
    if agg == "dense" and hub == "off":
        assert st.wedges_heavy > 0


@pytest.mark.parametrize("agg", ["dense", "auto"])
def test_counter_limits_other_side(case, agg):
    """The same graph with U and V swapped: the sources and candidates sit on
    the V side, whose thresholds are kept apart from the U side's."""
    name, g, _ = case
    t = gg.transpose(g)
    want = oracle.count(t)
    got, st = run(t, agg, "off")
    assert_same(got, want, f"{name} transposed agg={agg}")
    if agg == "dense":
        assert st.wedges_heavy > 0
