"""The C ABI without a GPU: every declared symbol is exported, and the host-side
argument checks answer before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "parbutterfly.h")


@pytest.fixture(scope="module")
def lib():
    import paper_1907_08607_amd as pb
    if not os.path.exists(pb.LIB_PATH):
        from paper_1907_08607_amd import build
        build.build()
    return pb.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pb_[a-z_]+)\s*\(", text)))


def test_header_declares_the_calls():
    names = declared_functions()
    for want in ("pb_graph_create", "pb_graph_destroy", "pb_rank", "pb_count", "pb_count_global",
                 "pb_count_vertex", "pb_count_edge", "pb_count_batched", "pb_autotune", "pb_status_str",
                 "pb_opts_default", "pb_sparsify", "pb_count_approx", "pb_wedges", "pb_rank_choose",
                 "pb_tip_decompose", "pb_wing_decompose"):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def declared_statuses():
    """(name, value) of every pb_status constant the header declares."""
    with open(os.path.join(ROOT, "include", "parbutterfly.h")) as f:
        text = f.read()
    body = re.search(r"typedef enum \{(.*?)\} pb_status;", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    return [(k, int(v)) for k, v in re.findall(r"(PB_\w+)\s*=\s*(-?\d+)", body)]


def test_status_strings(lib):
    import paper_1907_08607_amd as pb
    decl = declared_statuses()
    assert {v: k for k, v in decl} == pb.STATUS
    strs = set()
    for code in pb.STATUS:
        assert pb.status_str(code)
        strs.add(pb.status_str(code))
    assert len(strs) == len(pb.STATUS)  # every code has its own text
    assert pb.status_str(-4).startswith("rank")
    assert "never returned" in pb.status_str(-6)


def test_opts_default(lib):
    import paper_1907_08607_amd as pb
    o = pb.make_opts()
    assert o.agg == 0 and o.hub == 0 and o.workspace_cap_bytes == 0 and o.flags == 0
    assert not o.stats and not o.tuning


def test_host_side_argument_checks(lib):
    import paper_1907_08607_amd as pb
    h = ctypes.c_void_p()
    assert lib.pb_graph_create(None, None, ctypes.byref(h)) == -1
    csr = pb.pb_csr(3, 3, 9, None, None)
    assert lib.pb_graph_create(ctypes.byref(csr), None, ctypes.byref(h)) == -1  # null offsets
    csr = pb.pb_csr(3, 3, 1 << 31, 8, 8)
    assert lib.pb_graph_create(ctypes.byref(csr), None, ctypes.byref(h)) == -1  # m too large
    csr = pb.pb_csr(2, 2, 5, 8, 8)
    assert lib.pb_graph_create(ctypes.byref(csr), None, ctypes.byref(h)) == -2  # m > |U||V|
    assert lib.pb_rank(None, 3, None, None) == -1
    assert lib.pb_count(None, None, None, None, None, None, None) == -1
    for name in ("pb_count_global", "pb_count_vertex", "pb_count_edge"):
        assert getattr(lib, name)(None, None, None, None, None) == -1
    assert lib.pb_count_batched(None, None, 0, None, None, None, None, None) == -1
    assert lib.pb_autotune(None, None, 0, None, 1, None, None) == -1
    lib.pb_graph_destroy(None)


def test_bad_opts_rejected(lib):
    import paper_1907_08607_amd as pb
    fake = ctypes.c_void_p(8)  # never dereferenced: the options are checked first
    bad = pb.make_opts()
    bad.agg = 9
    assert lib.pb_count(fake, fake, ctypes.byref(bad), fake, None, None, None) == -1
    t = pb.pb_tuning(4096, 512, 1, 1, 2)  # light_max above the light kernel's capacity
    o = pb.make_opts(tuning=t)
    assert lib.pb_count(fake, fake, ctypes.byref(o), fake, None, None, None) == -1


def test_server_argument_checks(lib):
    import paper_1907_08607_amd as pb
    lib = pb._load_server_api()
    h = ctypes.c_void_p()
    assert lib.pb_server_create(None, ctypes.byref(h)) == -1
    cfg = pb.pb_server_config(0, 0, 8, 0, None)  # no slots
    assert lib.pb_server_create(ctypes.byref(cfg), ctypes.byref(h)) == -1
    cfg = pb.pb_server_config(0, 2, 0, 0, None)  # empty batches
    assert lib.pb_server_create(ctypes.byref(cfg), ctypes.byref(h)) == -1
    cfg = pb.pb_server_config(0, 2, 8, 7, None)  # unknown aggregator
    assert lib.pb_server_create(ctypes.byref(cfg), ctypes.byref(h)) == -1
    rid = ctypes.c_uint64()
    assert lib.pb_server_submit(None, 0, 1, None, None, None, ctypes.byref(rid)) == -1
    n = ctypes.c_uint32()
    assert lib.pb_server_poll(None, None, 0, ctypes.byref(n)) == -1
    assert lib.pb_server_drain(None) == -1
    lib.pb_server_destroy(None)


def test_sparsify_argument_checks(lib):
    k = ctypes.c_uint64()
    c, e = ctypes.c_int64(), ctypes.c_double()
    # no graph: rejected before any device work
    assert lib.pb_sparsify(None, 0, ctypes.c_double(0.5), ctypes.c_uint64(1), None, None, ctypes.byref(k), None) == -1
    assert lib.pb_count_approx(None, 1, ctypes.c_double(0.5), ctypes.c_uint64(1), 3, None, ctypes.byref(c),
                               ctypes.byref(e), None, None) == -1


def test_wedges_and_chooser_argument_checks(lib):
    w = ctypes.c_uint64()
    chosen = ctypes.c_int()
    assert lib.pb_wedges(None, None, ctypes.byref(w), None) == -1
    assert lib.pb_rank_choose(None, 4, None, ctypes.byref(chosen), None, None, None) == -1


def test_tip_decompose_argument_checks(lib):
    side = ctypes.c_int()
    assert lib.pb_tip_decompose(None, 0, None, None, ctypes.byref(side), None, None) == -1


def test_wing_decompose_argument_checks(lib):
    assert lib.pb_wing_decompose(None, None, None, None, None) == -1
