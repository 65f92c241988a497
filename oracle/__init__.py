"""Butterfly-counting oracle: TEST INFRASTRUCTURE ONLY.

A ctypes front end to ``oracle.c`` (plain single-threaded C, computed from
the definitions in the paper's Preliminaries and Lemma lem-count).  Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may
import this package; the counting library never does.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB, build

SIDE_AUTO, SIDE_U, SIDE_V, DEGREE, APPROX_DEGREE, CODEG, APPROX_CODEG = range(7)
RANK_KINDS = {
    "side_auto": SIDE_AUTO, "side_u": SIDE_U, "side_v": SIDE_V, "degree": DEGREE,
    "approx_degree": APPROX_DEGREE, "codeg": CODEG, "approx_codeg": APPROX_CODEG,
}

_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int64


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        for name in ("orc_bf4", "orc_pairs", "orc_count"):
            getattr(lib, name).argtypes = [_I, _I, _P, _P, _P, _P, _P]
        lib.orc_vside.argtypes = [_I, _I, _P, _P, _P, _P]
        lib.orc_count_sample.argtypes = [_I, _I, _P, _P, _I, _P]
        lib.orc_vertex_one.argtypes = [_I, _I, _P, _P, _P, _P, _I, _P]
        lib.orc_edge_one.argtypes = [_I, _I, _P, _P, _P, _P, _I, _P]
        lib.orc_wedges.argtypes = [_I, _I, _P, _P, _P, _P, _P]
        lib.orc_rank.argtypes = [_I, _I, _P, _P, ctypes.c_int, _P]
        lib.orc_splitmix.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.orc_splitmix.restype = ctypes.c_uint64
        lib.orc_sparsify.argtypes = [_I, _I, _P, _P, ctypes.c_int, ctypes.c_double, ctypes.c_uint64, _P, _P, _P]
        lib.orc_tip.argtypes = [_I, _I, _P, _P, ctypes.c_int, _P, _P]
        lib.orc_wing.argtypes = [_I, _I, _P, _P, _P, _P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _csr(g):
    return (np.ascontiguousarray(g.u_off, dtype=np.int64),
            np.ascontiguousarray(g.u_adj, dtype=np.uint32))


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"{what}: oracle error {rc}")


def _counts(fn, g, want_vertex=True, want_edge=True):
    off, adj = _csr(g)
    glob = np.zeros(1, dtype=np.int64)
    vert = np.zeros(g.n_u + g.n_v, dtype=np.int64) if want_vertex else None
    edge = np.zeros(g.m, dtype=np.int64) if want_edge else None
    _check(fn(g.n_u, g.n_v, _ptr(off), _ptr(adj), _ptr(glob), _ptr(vert), _ptr(edge)), fn.__name__)
    return int(glob[0]), vert, edge


def count_bf4(g, want_vertex=True, want_edge=True):
    """4-tuple brute force: (global, per-vertex, per-edge)."""
    return _counts(_load().orc_bf4, g, want_vertex, want_edge)


def count_pairs(g, want_vertex=True, want_edge=True):
    """Vertex-pair brute force (the Lemma over all pairs)."""
    return _counts(_load().orc_pairs, g, want_vertex, want_edge)


def count(g, want_vertex=True, want_edge=True):
    """The oracle proper: (global, per-vertex int64[n], per-edge int64[m])."""
    return _counts(_load().orc_count, g, want_vertex, want_edge)


def count_sample(g, stride: int) -> float:
    """Seconds the oracle proper takes on every stride-th endpoint (one thread);
    times stride estimates its full run (a bounded CPU-baseline sample)."""
    import time
    off, adj = _csr(g)
    glob = np.zeros(1, dtype=np.int64)
    lib = _load()
    t0 = time.perf_counter()
    _check(lib.orc_count_sample(g.n_u, g.n_v, _ptr(off), _ptr(adj), int(stride), _ptr(glob)), "orc_count_sample")
    return time.perf_counter() - t0


class Sampler:
    """Single per-vertex / per-edge counts computed alone, for sampled checks."""

    def __init__(self, g):
        self.g = g
        self.off, self.adj = _csr(g)
        self.v_off = np.zeros(g.n_v + 1, dtype=np.int64)
        self.v_adj = np.zeros(max(g.m, 1), dtype=np.uint32)
        _check(_load().orc_vside(g.n_u, g.n_v, _ptr(self.off), _ptr(self.adj),
                                 _ptr(self.v_off), _ptr(self.v_adj)), "orc_vside")

    def vertex(self, x: int) -> int:
        out = np.zeros(1, dtype=np.int64)
        _check(_load().orc_vertex_one(self.g.n_u, self.g.n_v, _ptr(self.off), _ptr(self.adj),
                                      _ptr(self.v_off), _ptr(self.v_adj), int(x), _ptr(out)),
               "orc_vertex_one")
        return int(out[0])

    def edge(self, e: int) -> int:
        out = np.zeros(1, dtype=np.int64)
        _check(_load().orc_edge_one(self.g.n_u, self.g.n_v, _ptr(self.off), _ptr(self.adj),
                                    _ptr(self.v_off), _ptr(self.v_adj), int(e), _ptr(out)),
               "orc_edge_one")
        return int(out[0])


def wedges(g, rank: np.ndarray, per_source: bool = False):
    """Wedges retrieved under ``rank`` (total, and per source if asked)."""
    off, adj = _csr(g)
    rank = np.ascontiguousarray(rank, dtype=np.uint32)
    if rank.shape != (g.n_u + g.n_v,):
        raise ValueError("rank must have n entries")
    total = np.zeros(1, dtype=np.int64)
    per = np.zeros(g.n_u + g.n_v, dtype=np.int64) if per_source else None
    _check(_load().orc_wedges(g.n_u, g.n_v, _ptr(off), _ptr(adj), _ptr(rank), _ptr(total), _ptr(per)),
           "orc_wedges")
    return (int(total[0]), per) if per_source else int(total[0])


def rank(g, kind: str) -> np.ndarray:
    """Reference ordering: rank[x] for every unified id x."""
    off, adj = _csr(g)
    out = np.zeros(g.n_u + g.n_v, dtype=np.uint32)
    _check(_load().orc_rank(g.n_u, g.n_v, _ptr(off), _ptr(adj), RANK_KINDS[kind], _ptr(out)),
           "orc_rank")
    return out


SPARSIFY_KINDS = {"edge": 0, "color": 1}


class Kept:
    """The graph a sparsification keeps (U-side CSR, same fields as the inputs)."""

    def __init__(self, n_u: int, n_v: int, u_off: np.ndarray, u_adj: np.ndarray):
        self.n_u, self.n_v = n_u, n_v
        self.u_off, self.u_adj = u_off, u_adj
        self.m = int(u_off[-1]) if len(u_off) else 0


def splitmix(seed: int, i: int) -> int:
    """SplitMix64 output number i + 1 from state ``seed``."""
    return int(_load().orc_splitmix(seed & (2**64 - 1), i & (2**64 - 1)))


def sparsify(g, kind: str, p: float, seed: int) -> Kept:
    """Edge (keep each edge with probability p) or colorful (ceil(1/p) colours,
    keep same-coloured edges) sparsification, Section 4.6."""
    off, adj = _csr(g)
    out_off = np.zeros(g.n_u + 1, dtype=np.int64)
    out_adj = np.zeros(max(g.m, 1), dtype=np.uint32)
    kept = np.zeros(1, dtype=np.int64)
    _check(_load().orc_sparsify(g.n_u, g.n_v, _ptr(off), _ptr(adj), SPARSIFY_KINDS[kind], float(p),
                                seed & (2**64 - 1), _ptr(out_off), _ptr(out_adj), _ptr(kept)), "orc_sparsify")
    return Kept(g.n_u, g.n_v, out_off, out_adj[:int(kept[0])].copy())


def scale(kind: str, p: float) -> float:
    """Factor that makes the kept graph's count an unbiased estimate: 1/p^4 for
    edge sparsification; c^3 with c = ceil(1/p) colours for colorful (a
    butterfly survives when its other three vertices take the first one's
    colour, probability (1/c)^3)."""
    import math
    if p >= 1.0:
        return 1.0
    if kind == "edge":
        return 1.0 / (p * p * p * p)
    c = float(math.ceil(1.0 / p))
    return c * c * c


def count_approx(g, kind: str, p: float, seed: int):
    """(exact count of the kept graph, scaled estimate, kept edges)."""
    k = sparsify(g, kind, p, seed)
    c = count(k, want_vertex=False, want_edge=False)[0]
    return c, c * scale(kind, p), k.m


PEEL_SIDES = {"auto": 0, "u": 1, "v": 2}


def tip(g, side: str = "auto"):
    """Tip numbers by vertex peeling (Section 3.2, Algorithm 5): (tip int64[n]
    with -1 on the side not peeled, rounds)."""
    off, adj = _csr(g)
    out = np.zeros(g.n_u + g.n_v, dtype=np.int64)
    rounds = np.zeros(1, dtype=np.int64)
    _check(_load().orc_tip(g.n_u, g.n_v, _ptr(off), _ptr(adj), PEEL_SIDES[side], _ptr(out), _ptr(rounds)), "orc_tip")
    return out, int(rounds[0])


def wing(g):
    """Wing numbers by edge peeling (Section 3.2, Algorithm 6): (wing int64[m]
    by u_adj position, rounds)."""
    off, adj = _csr(g)
    out = np.zeros(max(g.m, 1), dtype=np.int64)
    rounds = np.zeros(1, dtype=np.int64)
    _check(_load().orc_wing(g.n_u, g.n_v, _ptr(off), _ptr(adj), _ptr(out), _ptr(rounds)), "orc_wing")
    return out[:g.m], int(rounds[0])
