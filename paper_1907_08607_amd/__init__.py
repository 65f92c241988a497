"""Python binding of libparbutterfly (exact butterfly counting on MI355X).

Argument marshalling only: every step of the computation runs in the HIP
library's kernels.  Device memory and streams come from PyTorch.  The
function names mirror the C ABI in include/parbutterfly.h.

    import torch, paper_1907_08607_amd as pb
    g = pb.Graph(n_u, n_v, u_off_cuda_int64, u_adj_cuda_uint32)
    rank = pb.pb_rank(g, "degree")
    total, per_vertex, per_edge = pb.pb_count(g, rank)
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libparbutterfly.so")

PB_OK = 0
STATUS = {
    0: "PB_OK", -1: "PB_ERR_INVALID_ARG", -2: "PB_ERR_NOT_SIMPLE", -3: "PB_ERR_ID_RANGE",
    -4: "PB_ERR_BAD_RANK", -5: "PB_ERR_NO_MEMORY", -6: "PB_ERR_OVERFLOW", -7: "PB_ERR_HIP",
    -8: "PB_ERR_INTERNAL",
}
RANK_KINDS = {
    "side_auto": 0, "side_u": 1, "side_v": 2, "degree": 3, "approx_degree": 4,
    "codeg": 5, "approx_codeg": 6,
}
AGGS = {"auto": 0, "hash": 1, "dense": 2, "sort": 3}
HUBS = {"auto": 0, "off": 1, "force": 2}


class PBError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)} ({status_str(status)})")


class pb_csr(ctypes.Structure):
    _fields_ = [("n_u", ctypes.c_uint32), ("n_v", ctypes.c_uint32), ("m", ctypes.c_uint64),
                ("u_off", ctypes.c_void_p), ("u_adj", ctypes.c_void_p)]


PB_FLAG_TIMING = 1
PB_FLAG_CACHE_OPT = 2


class pb_stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in (
        "wedges", "sources", "sources_hash", "sources_dense", "sources_sort", "window_items",
        "wedges_hash", "wedges_dense", "wedges_sort", "wedges_hub", "workspace_bytes")] + [
        (name, ctypes.c_double) for name in ("ms_prepare", "ms_dense", "ms_hash", "ms_sort", "ms_output")] + [
        ("wedges_heavy", ctypes.c_uint64), ("ms_heavy", ctypes.c_double)] + [
        (name, ctypes.c_uint64) for name in ("hub_rows", "hub_cols", "hub_mfma_ops")] + [
        (name, ctypes.c_double) for name in ("ms_hub_gemm", "ms_hub_pass")] + [
        ("wedges_global", ctypes.c_uint64), ("ms_global", ctypes.c_double),
        ("slot_credit_bytes", ctypes.c_uint64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class pb_tuning(ctypes.Structure):
    _fields_ = [("light_max", ctypes.c_uint32), ("medium_max", ctypes.c_uint32), ("light_agg", ctypes.c_int),
                ("medium_agg", ctypes.c_int), ("heavy_agg", ctypes.c_int), ("light_wg", ctypes.c_uint32),
                ("medium_wg", ctypes.c_uint32), ("light_width", ctypes.c_uint32), ("medium_width", ctypes.c_uint32),
                ("heavy_width", ctypes.c_uint32)]

    def as_dict(self):
        names = {v: k for k, v in AGGS.items()}
        return {"light_max": self.light_max, "medium_max": self.medium_max, "light_agg": names[self.light_agg],
                "medium_agg": names[self.medium_agg], "heavy_agg": names[self.heavy_agg],
                "light_wg": self.light_wg or 64, "medium_wg": self.medium_wg or 256,
                "light_width": self.light_width, "medium_width": self.medium_width,
                "heavy_width": self.heavy_width}


class pb_opts(ctypes.Structure):
    _fields_ = [("agg", ctypes.c_int), ("hub", ctypes.c_int), ("workspace_cap_bytes", ctypes.c_uint64),
                ("wg_size", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("stats", ctypes.POINTER(pb_stats)), ("tuning", ctypes.POINTER(pb_tuning))]


_lib = None


def load_library():
    """Load libparbutterfly.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1907_08607_amd.build` "
                          "or __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.pb_opts_default.argtypes = [ctypes.POINTER(pb_opts)]
    lib.pb_opts_default.restype = None
    lib.pb_status_str.argtypes = [ctypes.c_int]
    lib.pb_status_str.restype = ctypes.c_char_p
    lib.pb_graph_create.argtypes = [ctypes.POINTER(pb_csr), P, ctypes.POINTER(P)]
    lib.pb_graph_create.restype = ctypes.c_int
    lib.pb_graph_destroy.argtypes = [P]
    lib.pb_graph_destroy.restype = None
    lib.pb_rank.argtypes = [P, ctypes.c_int, P, P]
    lib.pb_rank.restype = ctypes.c_int
    lib.pb_count.argtypes = [P, P, ctypes.POINTER(pb_opts), P, P, P, P]
    lib.pb_count.restype = ctypes.c_int
    lib.pb_count_noalloc.argtypes = [P, P, ctypes.POINTER(pb_opts), P, P, P, P]
    lib.pb_count_noalloc.restype = ctypes.c_int
    for name in ("pb_count_global", "pb_count_vertex", "pb_count_edge"):
        fn = getattr(lib, name)
        fn.argtypes = [P, P, ctypes.POINTER(pb_opts), P, P]
        fn.restype = ctypes.c_int
    PP = ctypes.POINTER(ctypes.c_void_p)
    lib.pb_count_batched.argtypes = [PP, PP, ctypes.c_uint32, ctypes.POINTER(pb_opts), PP, PP, PP, P]
    lib.pb_count_batched.restype = ctypes.c_int
    lib.pb_autotune.argtypes = [PP, PP, ctypes.c_uint32, ctypes.POINTER(pb_opts), ctypes.c_uint32,
                                ctypes.POINTER(pb_tuning), P]
    lib.pb_autotune.restype = ctypes.c_int
    lib.pb_wedges.argtypes = [P, P, ctypes.POINTER(ctypes.c_uint64), P]
    lib.pb_wedges.restype = ctypes.c_int
    lib.pb_rank_choose.argtypes = [P, ctypes.c_int, P, ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64), P]
    lib.pb_rank_choose.restype = ctypes.c_int
    lib.pb_tip_decompose.argtypes = [P, ctypes.c_int, ctypes.POINTER(pb_opts), P, ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_uint64), P]
    lib.pb_tip_decompose.restype = ctypes.c_int
    lib.pb_wing_decompose.argtypes = [P, ctypes.POINTER(pb_opts), P, ctypes.POINTER(ctypes.c_uint64), P]
    lib.pb_wing_decompose.restype = ctypes.c_int
    lib.pb_sparsify.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_uint64, P, P,
                                ctypes.POINTER(ctypes.c_uint64), P]
    lib.pb_sparsify.restype = ctypes.c_int
    lib.pb_count_approx.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_uint64, ctypes.c_int,
                                    ctypes.POINTER(pb_opts), ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint64), P]
    lib.pb_count_approx.restype = ctypes.c_int
    _lib = lib
    return lib


def status_str(status: int) -> str:
    return load_library().pb_status_str(int(status)).decode()


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check(status: int, what: str):
    if status != PB_OK:
        raise PBError(status, what)


def _dev_ptr(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    return ctypes.c_void_p(t.data_ptr())


class Graph:
    """A validated bipartite graph on the device (owns the derived V-side CSR).

    u_off: int64 CUDA tensor [n_u + 1]; u_adj: int32/uint32 CUDA tensor [m] of
    V ids, each row strictly increasing.  The tensors are kept alive here."""

    def __init__(self, n_u: int, n_v: int, u_off, u_adj, stream=None):
        torch = _torch()
        lib = load_library()
        if u_adj.device.type != "cuda" or u_adj.dtype not in (torch.int32, getattr(torch, "uint32", torch.int32)):
            raise TypeError("u_adj must be a 32-bit CUDA (HIP) tensor")
        self.n_u, self.n_v, self.m = int(n_u), int(n_v), int(u_adj.numel())
        self.u_off, self.u_adj = u_off, u_adj
        csr = pb_csr(self.n_u, self.n_v, self.m, _dev_ptr(u_off, torch.int64, "u_off"),
                     ctypes.c_void_p(u_adj.data_ptr()) if self.m else None)
        if u_off.numel() != self.n_u + 1:
            raise ValueError("u_off must have n_u + 1 entries")
        handle = ctypes.c_void_p()
        _check(lib.pb_graph_create(ctypes.byref(csr), _stream(stream), ctypes.byref(handle)), "pb_graph_create")
        self._h = handle

    @property
    def n(self) -> int:
        return self.n_u + self.n_v

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("graph destroyed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            load_library().pb_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @classmethod
    def from_csr(cls, csr, device="cuda", stream=None):
        """From an object with n_u, n_v, u_off (numpy int64), u_adj (numpy uint32)."""
        torch = _torch()
        import numpy as np
        off = torch.from_numpy(np.ascontiguousarray(csr.u_off, dtype=np.int64)).to(device)
        adj = torch.from_numpy(np.ascontiguousarray(csr.u_adj, dtype=np.uint32).view(np.int32)).to(device)
        return cls(csr.n_u, csr.n_v, off, adj, stream)


def make_opts(agg="auto", hub="auto", workspace_cap=0, stats=None, timing=False, tuning=None,
              cache_opt=False, wg_size=0) -> pb_opts:
    o = pb_opts()
    load_library().pb_opts_default(ctypes.byref(o))
    o.wg_size = int(wg_size)
    if timing:
        o.flags |= PB_FLAG_TIMING
    if cache_opt:
        o.flags |= PB_FLAG_CACHE_OPT
    if tuning is not None:
        o.tuning = ctypes.pointer(tuning)
    o.agg = AGGS[agg] if isinstance(agg, str) else int(agg)
    o.hub = HUBS[hub] if isinstance(hub, str) else int(hub)
    o.workspace_cap_bytes = int(workspace_cap)
    if stats is not None:
        o.stats = ctypes.pointer(stats)
    return o


def pb_rank(g: Graph, kind="degree", out=None, stream=None):
    """Vertex ordering (int32 CUDA tensor holding uint32 ranks, n entries)."""
    torch = _torch()
    k = RANK_KINDS[kind] if isinstance(kind, str) else int(kind)
    if out is None:
        out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    _check(load_library().pb_rank(g.handle, k, _dev_ptr(out, torch.int32, "rank"), _stream(stream)), "pb_rank")
    return out


def pb_count(g: Graph, rank, want_global=True, want_vertex=True, want_edge=True, agg="auto", hub="auto",
             workspace_cap=0, stats: pb_stats | None = None, outs=None, stream=None, timing=False, tuning=None,
             cache_opt=False):
    """(global int64 tensor[1] or None, per-vertex int64[n] or None, per-edge int64[m] or None)."""
    torch = _torch()
    if outs is None:
        outs = (torch.empty(1, dtype=torch.int64, device="cuda") if want_global else None,
                torch.empty(g.n, dtype=torch.int64, device="cuda") if want_vertex else None,
                torch.empty(g.m, dtype=torch.int64, device="cuda") if want_edge else None)
    gout, vout, eout = outs
    opts = make_opts(agg, hub, workspace_cap, stats, timing, tuning, cache_opt)
    ptr = lambda t, name: None if t is None else _dev_ptr(t, torch.int64, name)
    _check(load_library().pb_count(g.handle, _dev_ptr(rank, torch.int32, "rank"), ctypes.byref(opts),
                                   ptr(gout, "global_out"), ptr(vout, "vertex_out"), ptr(eout, "edge_out"),
                                   _stream(stream)), "pb_count")
    return gout, vout, eout


def pb_count_noalloc(g: Graph, rank, outs, agg="auto", stats: pb_stats | None = None, stream=None,
                     cache_opt=False):
    """pb_count with every scratch block taken from the library's fixed
    per-device array: `outs` = (global int64[1] or None, per-vertex int64[n] or
    None, per-edge int64[m] or None), caller-allocated."""
    torch = _torch()
    gout, vout, eout = outs
    opts = make_opts(agg, "off", 0, stats, False, None, cache_opt)
    ptr = lambda t, name: None if t is None else _dev_ptr(t, torch.int64, name)
    _check(load_library().pb_count_noalloc(g.handle, _dev_ptr(rank, torch.int32, "rank"), ctypes.byref(opts),
                                           ptr(gout, "global_out"), ptr(vout, "vertex_out"),
                                           ptr(eout, "edge_out"), _stream(stream)), "pb_count_noalloc")
    return outs


def _single(name, g, rank, n_out, agg, hub, workspace_cap, stats, stream):
    torch = _torch()
    out = torch.empty(n_out, dtype=torch.int64, device="cuda")
    opts = make_opts(agg, hub, workspace_cap, stats)
    _check(getattr(load_library(), name)(g.handle, _dev_ptr(rank, torch.int32, "rank"), ctypes.byref(opts),
                                         _dev_ptr(out, torch.int64, "out"), _stream(stream)), name)
    return out


def pb_count_global(g, rank, agg="auto", hub="auto", workspace_cap=0, stats=None, stream=None):
    return _single("pb_count_global", g, rank, 1, agg, hub, workspace_cap, stats, stream)


def pb_count_vertex(g, rank, agg="auto", hub="auto", workspace_cap=0, stats=None, stream=None):
    return _single("pb_count_vertex", g, rank, g.n, agg, hub, workspace_cap, stats, stream)


def pb_count_edge(g, rank, agg="auto", hub="auto", workspace_cap=0, stats=None, stream=None):
    return _single("pb_count_edge", g, rank, g.m, agg, hub, workspace_cap, stats, stream)


def pb_wedges(g: Graph, rank, stream=None) -> int:
    """W(rank): the wedges the framework retrieves under `rank`."""
    torch = _torch()
    w = ctypes.c_uint64()
    _check(load_library().pb_wedges(g.handle, _dev_ptr(rank, torch.int32, "rank"), ctypes.byref(w),
                                    _stream(stream)), "pb_wedges")
    return w.value


def pb_rank_choose(g: Graph, other="approx_degree", out=None, stream=None):
    """Section 6.2's chooser: (rank tensor, chosen kind name, w_side, w_other)."""
    torch = _torch()
    k = RANK_KINDS[other] if isinstance(other, str) else int(other)
    if out is None:
        out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    chosen, ws, wr = ctypes.c_int(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(load_library().pb_rank_choose(g.handle, k, _dev_ptr(out, torch.int32, "rank"), ctypes.byref(chosen),
                                         ctypes.byref(ws), ctypes.byref(wr), _stream(stream)), "pb_rank_choose")
    name = {v: n for n, v in RANK_KINDS.items()}[chosen.value]
    return out, name, ws.value, wr.value


PEEL_SIDES = {"auto": 0, "u": 1, "v": 2}


def pb_tip_decompose(g: Graph, side="auto", agg="auto", hub="auto", out=None, stream=None):
    """Tip numbers by vertex peeling: (int64 CUDA tensor [n], -1 on the side
    not peeled; the side peeled, "u" or "v"; rounds)."""
    torch = _torch()
    if out is None:
        out = torch.empty(g.n, dtype=torch.int64, device="cuda")
    opts = make_opts(agg, hub)
    s_out, rounds = ctypes.c_int(), ctypes.c_uint64()
    _check(load_library().pb_tip_decompose(g.handle, PEEL_SIDES[side], ctypes.byref(opts),
                                           _dev_ptr(out, torch.int64, "tip_out"), ctypes.byref(s_out),
                                           ctypes.byref(rounds), _stream(stream)), "pb_tip_decompose")
    return out, {1: "u", 2: "v"}.get(s_out.value, "u"), rounds.value


def pb_wing_decompose(g: Graph, agg="auto", hub="auto", out=None, stream=None):
    """Wing numbers by edge peeling: (int64 CUDA tensor [m] by u_adj position, rounds)."""
    torch = _torch()
    if out is None:
        out = torch.empty(max(g.m, 1), dtype=torch.int64, device="cuda")
    opts = make_opts(agg, hub)
    rounds = ctypes.c_uint64()
    _check(load_library().pb_wing_decompose(g.handle, ctypes.byref(opts), _dev_ptr(out, torch.int64, "wing_out"),
                                            ctypes.byref(rounds), _stream(stream)), "pb_wing_decompose")
    return out[:g.m], rounds.value


SPARSIFY_KINDS = {"edge": 0, "color": 1}


def pb_sparsify(g: Graph, kind="edge", p=0.5, seed=0, stream=None):
    """The kept graph of edge or colorful sparsification: (u_off int64 CUDA
    tensor [n_u + 1], u_adj int32 CUDA tensor [kept])."""
    torch = _torch()
    off = torch.empty(g.n_u + 1, dtype=torch.int64, device="cuda")
    adj = torch.empty(max(g.m, 1), dtype=torch.int32, device="cuda")
    kept = ctypes.c_uint64()
    _check(load_library().pb_sparsify(g.handle, SPARSIFY_KINDS[kind], float(p), int(seed) & (2**64 - 1),
                                      _dev_ptr(off, torch.int64, "out_u_off"),
                                      ctypes.c_void_p(adj.data_ptr()) if g.m else None, ctypes.byref(kept),
                                      _stream(stream)), "pb_sparsify")
    return off, adj[:kept.value]


def pb_count_approx(g: Graph, kind="edge", p=0.5, seed=0, rank="degree", agg="auto", hub="auto",
                    stats=None, stream=None):
    """(kept graph's exact count, scaled estimate of the total, kept edges)."""
    opts = make_opts(agg, hub, 0, stats)
    count, est, kept = ctypes.c_int64(), ctypes.c_double(), ctypes.c_uint64()
    k = RANK_KINDS[rank] if isinstance(rank, str) else int(rank)
    _check(load_library().pb_count_approx(g.handle, SPARSIFY_KINDS[kind], float(p), int(seed) & (2**64 - 1), k,
                                          ctypes.byref(opts), ctypes.byref(count), ctypes.byref(est),
                                          ctypes.byref(kept), _stream(stream)), "pb_count_approx")
    return count.value, est.value, kept.value


def _ptr_array(items):
    arr = (ctypes.c_void_p * len(items))()
    for i, x in enumerate(items):
        arr[i] = x
    return arr


def pb_count_batched(graphs, ranks, want_global=True, want_vertex=False, want_edge=True, agg="auto", hub="auto",
                     stats: pb_stats | None = None, tuning=None, outs=None, stream=None, timing=False, wg_size=0):
    """outs, if given: (global list or None, vertex list or None, edge list or None)."""
    """Counts a batch of graphs in one pass; returns per-graph (global, vertex, edge) lists."""
    torch = _torch()
    k = len(graphs)
    if k != len(ranks) or k == 0:
        raise ValueError("graphs and ranks must be non-empty and of equal length")
    if outs is None:
        outs = ([torch.empty(1, dtype=torch.int64, device="cuda") for _ in graphs] if want_global else None,
                [torch.empty(g.n, dtype=torch.int64, device="cuda") for g in graphs] if want_vertex else None,
                [torch.empty(max(g.m, 1), dtype=torch.int64, device="cuda") for g in graphs] if want_edge else None)
    arrs = [None if o is None else _ptr_array([t.data_ptr() for t in o]) for o in outs]
    gp = _ptr_array([g.handle.value for g in graphs])
    rp = _ptr_array([_dev_ptr(r, torch.int32, "rank").value for r in ranks])
    opts = make_opts(agg, hub, 0, stats, timing, tuning, wg_size=wg_size)
    cast = lambda a: None if a is None else ctypes.cast(a, ctypes.POINTER(ctypes.c_void_p))
    _check(load_library().pb_count_batched(cast(gp), cast(rp), k, ctypes.byref(opts), cast(arrs[0]), cast(arrs[1]),
                                           cast(arrs[2]), _stream(stream)), "pb_count_batched")
    return outs


def pb_autotune(graphs, ranks, repeats=3, agg="auto", stream=None) -> pb_tuning:
    """Per-bucket aggregator table for the AUTO policy, timed on these graphs."""
    torch = _torch()
    gp = _ptr_array([g.handle.value for g in graphs])
    rp = _ptr_array([_dev_ptr(r, torch.int32, "rank").value for r in ranks])
    out = pb_tuning()
    opts = make_opts(agg)
    cast = lambda a: ctypes.cast(a, ctypes.POINTER(ctypes.c_void_p))
    _check(load_library().pb_autotune(cast(gp), cast(rp), len(graphs), ctypes.byref(opts), int(repeats),
                                      ctypes.byref(out), _stream(stream)), "pb_autotune")
    return out


# ---------------------------------------------------------------- serving

WANT = {"global": 1, "vertex": 2, "edge": 4}


class pb_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("slots", ctypes.c_uint32), ("max_batch", ctypes.c_uint32),
                ("agg", ctypes.c_int), ("tuning", ctypes.POINTER(pb_tuning))]


class pb_completion(ctypes.Structure):
    _fields_ = [("request_id", ctypes.c_uint64), ("status", ctypes.c_int32), ("batch", ctypes.c_uint32),
                ("submit_s", ctypes.c_double), ("start_s", ctypes.c_double), ("done_s", ctypes.c_double)]


def _load_server_api():
    lib = load_library()
    if getattr(lib, "_server_api", False):
        return lib
    P = ctypes.c_void_p
    lib.pb_server_create.argtypes = [ctypes.POINTER(pb_server_config), ctypes.POINTER(P)]
    lib.pb_server_create.restype = ctypes.c_int
    lib.pb_server_add_graph.argtypes = [P, P, P, ctypes.POINTER(ctypes.c_uint32)]
    lib.pb_server_add_graph.restype = ctypes.c_int
    lib.pb_server_submit.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, P, P, P, ctypes.POINTER(ctypes.c_uint64)]
    lib.pb_server_submit.restype = ctypes.c_int
    lib.pb_server_poll.argtypes = [P, ctypes.POINTER(pb_completion), ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]
    lib.pb_server_poll.restype = ctypes.c_int
    lib.pb_server_drain.argtypes = [P]
    lib.pb_server_drain.restype = ctypes.c_int
    lib.pb_server_destroy.argtypes = [P]
    lib.pb_server_destroy.restype = None
    lib._server_api = True
    return lib


class Server:
    """Resident-graph counting server (continuous batching over worker slots)."""

    def __init__(self, hbm_budget=0, slots=2, max_batch=64, agg="auto", tuning=None):
        lib = _load_server_api()
        self._tuning = tuning
        cfg = pb_server_config(int(hbm_budget), int(slots), int(max_batch), AGGS[agg] if isinstance(agg, str) else agg,
                               ctypes.pointer(tuning) if tuning is not None else None)
        h = ctypes.c_void_p()
        _check(lib.pb_server_create(ctypes.byref(cfg), ctypes.byref(h)), "pb_server_create")
        self._h = h
        self._keep = []  # graphs, ranks and output tensors the server references

    def add_graph(self, g: Graph, rank) -> int:
        torch = _torch()
        gid = ctypes.c_uint32()
        _check(_load_server_api().pb_server_add_graph(self._h, g.handle, _dev_ptr(rank, torch.int32, "rank"),
                                                      ctypes.byref(gid)), "pb_server_add_graph")
        self._keep.append((g, rank))
        return gid.value

    def submit(self, graph_id: int, want: int, gout=None, vout=None, eout=None) -> int:
        rid = ctypes.c_uint64()
        p = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
        _check(_load_server_api().pb_server_submit(self._h, int(graph_id), int(want), p(gout), p(vout), p(eout),
                                                   ctypes.byref(rid)), "pb_server_submit")
        self._keep.append((gout, vout, eout))
        return rid.value

    def poll(self, max_items=4096):
        buf = (pb_completion * max_items)()
        n = ctypes.c_uint32()
        _check(_load_server_api().pb_server_poll(self._h, buf, max_items, ctypes.byref(n)), "pb_server_poll")
        return [buf[i] for i in range(n.value)]

    def drain(self):
        _check(_load_server_api().pb_server_drain(self._h), "pb_server_drain")

    def close(self):
        if getattr(self, "_h", None) is not None:
            _load_server_api().pb_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
