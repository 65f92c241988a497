"""GPU: the allocation-free entry point (pb_count_noalloc, scratch from the
library's fixed per-device array) against pb_count, through the C ABI: equal
outputs on two calls in a row, the second on a smaller graph; refusal of a
graph whose scratch cannot fit; no device memory taken by the call."""
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


def outs_for(G, fill=-1):
    return (torch.full((1,), fill, dtype=torch.int64, device="cuda"),
            torch.full((G.n,), fill, dtype=torch.int64, device="cuda"),
            torch.full((max(G.m, 1),), fill, dtype=torch.int64, device="cuda"))


def both(G, r, agg="auto", cache_opt=False):
    want = pb.pb_count(G, r, agg=agg, cache_opt=cache_opt)
    got = outs_for(G)
    torch.cuda.synchronize()  # the fills are done before the call writes
    st = pb.pb_stats()
    pb.pb_count_noalloc(G, r, got, agg=agg, stats=st, cache_opt=cache_opt)
    torch.cuda.synchronize()
    return [t.cpu() for t in want], [t.cpu() for t in got], st


@pytest.mark.parametrize("agg", ["auto", "hash", "dense", "sort"])
def test_noalloc_equals_pb_count_then_a_smaller_graph(agg):
    big = gg.batch_graph(15_000, 12_000, 300_000, 71)      # a batched-workload graph near its upper sizes
    small = gg.workload_er_1k_planted(1)
    for g in (big, small):                                  # two calls in a row, the second smaller
        G = pb.Graph.from_csr(g)
        r = pb.pb_rank(G, "degree")
        want, got, st = both(G, r, agg)
        assert int(got[0][0]) == int(want[0][0])
        assert torch.equal(got[1], want[1])
        assert torch.equal(got[2][:g.m], want[2][:g.m])
        wo = oracle.count(g)
        assert int(got[0][0]) == wo[0] and (got[2][:g.m].numpy() == wo[2]).all()
        assert st.wedges == oracle.wedges(g, r.cpu().numpy().view(np.uint32))
        G.close()


def test_noalloc_single_outputs_and_cache_opt():
    g = gg.chung_lu(20_000, 8_000, 200_000, 2.1, 2000, 800, 5)
    G = pb.Graph.from_csr(g)
    r = pb.pb_rank(G, "approx_codeg")
    want = pb.pb_count(G, r)
    for k in range(3):
        o = [None, None, None]
        o[k] = outs_for(G)[k]
        torch.cuda.synchronize()
        pb.pb_count_noalloc(G, r, tuple(o))
        torch.cuda.synchronize()
        assert torch.equal(o[k].cpu()[:want[k].numel()], want[k].cpu())
    _, got, _ = both(G, r, cache_opt=True)
    assert torch.equal(got[2][:g.m], want[2].cpu())
    G.close()


def test_noalloc_refuses_a_graph_too_large_for_its_array():
    g = gg.workload_powerlaw_50m(scale=0.05)  # 2.5M edges: more scratch than the array holds
    G = pb.Graph.from_csr(g)
    r = pb.pb_rank(G, "degree")
    o = outs_for(G)
    torch.cuda.synchronize()
    with pytest.raises(pb.PBError) as e:
        pb.pb_count_noalloc(G, r, o)
    assert e.value.status == -5
    assert int(o[0].cpu()[0]) == -1  # nothing was written
    G.close()


def test_noalloc_takes_no_device_memory():
    g = gg.batch_graph(10_000, 10_000, 200_000, 72)
    G = pb.Graph.from_csr(g)
    r = pb.pb_rank(G, "degree")
    o = outs_for(G)
    torch.cuda.synchronize()
    pb.pb_count_noalloc(G, r, o)  # first call: the library's code and array are resident
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        pb.pb_count_noalloc(G, r, o)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    want = pb.pb_count(G, r)
    assert torch.equal(o[2].cpu()[:g.m], want[2].cpu())
    G.close()
