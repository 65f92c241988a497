"""GPU parity of the batched workload at its full size: the 4096 Chung-Lu
graphs (|U|, |V| log-uniform in [64, 20k], m log-uniform in [256, 5e5]
clamped to |U||V|/4, exponent 2.1, seed 4) counted in one batched pass, each
graph's per-edge counts compared with the oracle's (the totals and array
digests in tests/golden/batch_4096.json, written by make_golden.py from the
oracle alone).  Run under the built-in per-bucket table and under one chosen
by the autotuner."""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_1907_08607_amd import graphgen as gg

torch = pytest.importorskip("torch")
pb = pytest.importorskip("paper_1907_08607_amd")

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "batch_4096.json")


@pytest.fixture(scope="module")
def batch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pb.load_library()
    with open(GOLDEN) as f:
        want = json.load(f)
    gs = gg.workload_batch(want["count"], seed=4)
    h = hashlib.sha256()
    for g in gs:
        h.update(g.sha256().encode())
    assert h.hexdigest() == want["graphs_sha256"], "the generator no longer draws the recorded graphs"
    Gs = [pb.Graph.from_csr(g) for g in gs]
    ranks = [pb.pb_rank(G, "degree") for G in Gs]
    yield gs, Gs, ranks, want
    for G in Gs:
        G.close()


def check(gs, gl, ed, want):
    torch.cuda.synchronize()
    glob = torch.cat([t[:1] for t in gl]).cpu().numpy()
    assert glob.tolist() == want["global"]
    flat = torch.cat([t[:g.m] for t, g in zip(ed, gs)]).cpu().numpy()
    off = 0
    bad = []
    for i, g in enumerate(gs):
        d = hashlib.sha256(np.ascontiguousarray(flat[off:off + g.m], dtype="<i8").tobytes()).hexdigest()[:16]
        off += g.m
        if d != want["edge_sha256_16"][i]:
            bad.append(i)
    assert not bad, f"per-edge counts differ from the oracle on graphs {bad[:10]} ({len(bad)} in all)"


def test_full_batch_builtin_table(batch):
    gs, Gs, ranks, want = batch
    st = pb.pb_stats()
    gl, _, ed = pb.pb_count_batched(Gs, ranks, True, False, True, stats=st)
    check(gs, gl, ed, want)
    assert st.wedges_heavy > 0 and st.wedges_hash > 0


def test_full_batch_autotuned_table(batch):
    gs, Gs, ranks, want = batch
    sample = list(range(0, len(Gs), 16))
    t = pb.pb_autotune([Gs[i] for i in sample], [ranks[i] for i in sample], repeats=1)
    gl, _, ed = pb.pb_count_batched(Gs, ranks, True, False, True, tuning=t)
    check(gs, gl, ed, want)
