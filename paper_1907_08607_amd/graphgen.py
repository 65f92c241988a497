"""Seeded synthetic bipartite graphs (input making only).

This module draws the graphs that both the counting library and the CPU
oracle consume.  It holds none of the counting method's arithmetic: it only
samples edge sets and lays them out as a U-side CSR (row offsets int64,
column ids uint32, every row strictly increasing), the input format the
paper assumes (Preliminaries, graph notation: CSR with separate offset and
edge arrays; graphs simple and undirected).

Workload shapes stand in for the paper's KONECT graphs (Table 1), which are
not available here:

* ``er``          Erdos-Renyi: m distinct (u, v) pairs drawn uniformly.
* ``chung_lu``    power-law expected degrees on both sides (balanced
                  KONECT graphs such as livejournal / orkut).
* ``hub_skewed``  power-law V side with exponent 1.8, geometric U side
                  (the |U| >> |V| KONECT graphs such as delicious).
* ``complete``    K_{a,b}, and ``plant_complete`` adds a disjoint K_{a,b}.

Every generator is deterministic in its seed (numpy PCG64).
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np


@dataclasses.dataclass
class BipartiteCSR:
    n_u: int
    n_v: int
    u_off: np.ndarray  # int64[n_u + 1]
    u_adj: np.ndarray  # uint32[m], each row strictly increasing

    @property
    def m(self) -> int:
        return int(self.u_adj.shape[0])

    @property
    def n(self) -> int:
        return self.n_u + self.n_v

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.asarray([self.n_u, self.n_v, self.m], dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.u_off, dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.u_adj, dtype=np.uint32).tobytes())
        return h.hexdigest()

    def edges(self) -> tuple[np.ndarray, np.ndarray]:
        """(u, v) arrays in CSR order (the per-edge output order)."""
        deg = np.diff(self.u_off)
        u = np.repeat(np.arange(self.n_u, dtype=np.int64), deg)
        return u, self.u_adj.astype(np.int64)


def from_edges(n_u: int, n_v: int, u: np.ndarray, v: np.ndarray) -> BipartiteCSR:
    """Build a CSR from an edge list with distinct (u, v) pairs."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    if u.size:
        if u.min() < 0 or u.max() >= n_u or v.min() < 0 or v.max() >= n_v:
            raise ValueError("edge endpoint out of range")
    key = u * np.int64(n_v) + v
    key = np.unique(key)
    if key.size != u.size:
        raise ValueError("duplicate edges")
    uu = key // np.int64(max(n_v, 1))
    vv = (key - uu * np.int64(n_v)).astype(np.uint32)
    off = np.zeros(n_u + 1, dtype=np.int64)
    np.cumsum(np.bincount(uu, minlength=n_u), out=off[1:])
    return BipartiteCSR(n_u, n_v, off, vv)


def _mix64(x: np.ndarray, seed: int) -> np.ndarray:
    """splitmix64 finaliser: a fixed pseudo-random priority per key."""
    z = x.astype(np.uint64) + np.uint64((0x9E3779B97F4A7C15 * (seed + 1)) & 0xFFFFFFFFFFFFFFFF)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def _pair_until(m: int, n_v: int, draw, rng, seed: int, max_rounds: int = 64) -> np.ndarray:
    """Draw (u, v) pairs in batches until at least m distinct ones exist, then keep
    the m distinct pairs of smallest seeded priority (so the result does not depend
    on how the draws were batched beyond the seed)."""
    keys = np.empty(0, dtype=np.int64)
    drawn = 0
    batch = int(m * 1.05) + 64
    for _ in range(max_rounds):
        u, v = draw(batch, rng)
        drawn += batch
        keys = np.unique(np.concatenate([keys, u.astype(np.int64) * np.int64(n_v) + v.astype(np.int64)]))
        if keys.size >= m:
            break
        hit = max(keys.size / drawn, 1e-3)
        batch = int(2 * (m - keys.size) / hit) + 64
    else:
        raise RuntimeError("could not draw enough distinct pairs")
    if keys.size > m:
        pri = _mix64(keys, seed)
        keep = np.argpartition(pri, m - 1)[:m]
        keys = keys[keep]
    return keys


def _csr_from_keys(n_u: int, n_v: int, keys: np.ndarray) -> BipartiteCSR:
    keys = np.sort(keys)
    u = keys // np.int64(n_v)
    v = (keys - u * np.int64(n_v)).astype(np.uint32)
    off = np.zeros(n_u + 1, dtype=np.int64)
    np.cumsum(np.bincount(u, minlength=n_u), out=off[1:])
    return BipartiteCSR(n_u, n_v, off, v)


def er(n_u: int, n_v: int, m: int, seed: int) -> BipartiteCSR:
    """m distinct pairs drawn uniformly from U x V."""
    if m > n_u * n_v:
        raise ValueError("m exceeds |U||V|")
    rng = np.random.Generator(np.random.PCG64(seed))

    def draw(k, r):
        return r.integers(0, n_u, size=k), r.integers(0, n_v, size=k)

    return _csr_from_keys(n_u, n_v, _pair_until(m, n_v, draw, rng, seed))


def powerlaw_mean(gamma: float, dmin: float, dmax: float) -> float:
    """Mean of the continuous density proportional to d^-gamma on [dmin, dmax]."""
    def integral(k):  # int_dmin^dmax d^(k - gamma) dd
        e = k + 1.0 - gamma
        if abs(e) < 1e-12:
            return np.log(dmax / dmin)
        return (dmax ** e - dmin ** e) / e
    return integral(1.0) / integral(0.0)


def solve_dmin(gamma: float, mean: float, dmax: float) -> float:
    """dmin such that the truncated power law on [dmin, dmax] has this mean."""
    lo, hi = 1e-9, dmax
    for _ in range(200):
        mid = np.sqrt(lo * hi)
        if powerlaw_mean(gamma, mid, dmax) < mean:
            lo = mid
        else:
            hi = mid
    return float(np.sqrt(lo * hi))


def powerlaw_weights(count: int, gamma: float, dmin: float, dmax: float, rng) -> np.ndarray:
    """Inverse-CDF samples of the truncated power law d^-gamma on [dmin, dmax]."""
    r = rng.random(count)
    a = 1.0 - gamma
    return (dmin ** a + r * (dmax ** a - dmin ** a)) ** (1.0 / a)


def _weighted_draw(w_u: np.ndarray, w_v: np.ndarray):
    """Endpoints proportional to weight: the per-vertex draw counts are one
    multinomial sample per side; the V draws are then randomly permuted so the
    (u, v) pairing is uniform, which makes the pairs i.i.d. in distribution."""
    p_u = w_u / w_u.sum()
    p_v = w_v / w_v.sum()

    def draw(k, r):
        u = np.repeat(np.arange(p_u.size, dtype=np.int64), r.multinomial(k, p_u))
        v = np.repeat(np.arange(p_v.size, dtype=np.int64), r.multinomial(k, p_v))
        return u, r.permutation(v)

    return draw


def chung_lu_weights(w_u: np.ndarray, w_v: np.ndarray, m: int, seed: int) -> BipartiteCSR:
    """Chung-Lu pairing: endpoints drawn proportional to weight until m distinct pairs."""
    n_u, n_v = int(w_u.size), int(w_v.size)
    if m > n_u * n_v:
        raise ValueError("m exceeds |U||V|")
    rng = np.random.Generator(np.random.PCG64([seed, 1]))
    return _csr_from_keys(n_u, n_v, _pair_until(m, n_v, _weighted_draw(w_u, w_v), rng, seed))


def chung_lu(n_u: int, n_v: int, m: int, gamma: float, dmax_u: float, dmax_v: float,
             seed: int) -> BipartiteCSR:
    """Power-law expected degrees on both sides, means m/|U| and m/|V|."""
    rng = np.random.Generator(np.random.PCG64([seed, 0]))
    w_u = powerlaw_weights(n_u, gamma, solve_dmin(gamma, m / n_u, dmax_u), dmax_u, rng)
    w_v = powerlaw_weights(n_v, gamma, solve_dmin(gamma, m / n_v, dmax_v), dmax_v, rng)
    return chung_lu_weights(w_u, w_v, m, seed)


def hub_skewed(n_u: int, n_v: int, m: int, gamma_v: float, dmax_v: float, mean_u: float,
               seed: int) -> BipartiteCSR:
    """Power-law V weights (mean m/|V|), geometric U weights with the given mean."""
    rng = np.random.Generator(np.random.PCG64([seed, 0]))
    w_v = powerlaw_weights(n_v, gamma_v, solve_dmin(gamma_v, m / n_v, dmax_v), dmax_v, rng)
    w_u = rng.geometric(1.0 / mean_u, size=n_u).astype(np.float64)
    return chung_lu_weights(w_u, w_v, m, seed)


def complete(a: int, b: int) -> BipartiteCSR:
    """K_{a,b}."""
    u = np.repeat(np.arange(a), b)
    v = np.tile(np.arange(b), a)
    return from_edges(a, b, u, v)


def disjoint_union(g: BipartiteCSR, h: BipartiteCSR) -> BipartiteCSR:
    """g then h, with h's U ids shifted by |U_g| and V ids by |V_g|."""
    gu, gv = g.edges()
    hu, hv = h.edges()
    return from_edges(g.n_u + h.n_u, g.n_v + h.n_v,
                      np.concatenate([gu, hu + g.n_u]), np.concatenate([gv, hv + g.n_v]))


def plant_complete(g: BipartiteCSR, a: int, b: int) -> BipartiteCSR:
    """g plus a disjoint K_{a,b} on new ids (U ids after g's, V ids after g's)."""
    return disjoint_union(g, complete(a, b))


def relabel(g: BipartiteCSR, perm_u: np.ndarray, perm_v: np.ndarray) -> BipartiteCSR:
    """Rename u -> perm_u[u], v -> perm_v[v] (an isomorphic copy)."""
    u, v = g.edges()
    return from_edges(g.n_u, g.n_v, np.asarray(perm_u)[u], np.asarray(perm_v)[v])


def transpose(g: BipartiteCSR) -> BipartiteCSR:
    """Swap the roles of U and V."""
    u, v = g.edges()
    return from_edges(g.n_v, g.n_u, v, u)


def random_small(n_u: int, n_v: int, p: float, seed: int) -> BipartiteCSR:
    """Each of the |U||V| pairs present independently with probability p."""
    rng = np.random.Generator(np.random.PCG64([seed, 7]))
    mask = rng.random((n_u, n_v)) < p
    u, v = np.nonzero(mask)
    return from_edges(n_u, n_v, u, v)


def giant_hubs(n_u: int, n_v: int, hubs: int, hub_deg: int, per_u: int, seed: int) -> BipartiteCSR:
    """A few giant V vertices on a sparse background: V ids 0..hubs-1 each take
    hub_deg distinct random U neighbours, and every U vertex takes per_u random
    V neighbours (duplicates dropped).  The hubs are sources with far more
    up-slots than any other, the shape of the heaviest sources of a hub-skewed
    graph, at a size the oracle finishes quickly."""
    rng = np.random.Generator(np.random.PCG64([seed, 11]))
    hu = np.concatenate([rng.choice(n_u, size=hub_deg, replace=False) for _ in range(hubs)])
    hv = np.repeat(np.arange(hubs), hub_deg)
    bu = np.repeat(np.arange(n_u), per_u)
    bv = rng.integers(0, n_v, size=bu.size)
    keys = np.unique(np.concatenate([hu * np.int64(n_v) + hv, bu * np.int64(n_v) + bv]))
    return _csr_from_keys(n_u, n_v, keys)


# --------------------------------------------------------------------------
# The named workloads.

def workload_er_1k(seed: int = 1) -> BipartiteCSR:
    """ER: |U|=1000, |V|=800, m=10,000."""
    return er(1000, 800, 10_000, seed)


def workload_er_1k_planted(seed: int = 1) -> BipartiteCSR:
    """The ER graph plus a disjoint K_{20,15}."""
    return plant_complete(workload_er_1k(seed), 20, 15)


def workload_powerlaw_50m(seed: int = 2, scale: float = 1.0) -> BipartiteCSR:
    """Chung-Lu, exponent 2.1 both sides, |U|=2M, |V|=500k, m=50M, max weight 50k.

    ``scale`` shrinks every size (vertex counts, m, max weight) for small tests.
    """
    n_u, n_v, m = int(2_000_000 * scale), int(500_000 * scale), int(50_000_000 * scale)
    dmax = max(50_000.0 * scale, 8.0)
    return chung_lu(n_u, n_v, m, 2.1, min(dmax, n_v), min(dmax, n_u), seed)


def workload_hub_100m(seed: int = 3, scale: float = 1.0) -> BipartiteCSR:
    """|U|=20M, |V|=100k, m=100M; V power law exponent 1.8 up to 1M, U geometric mean 5."""
    n_u, n_v, m = int(20_000_000 * scale), int(100_000 * scale), int(100_000_000 * scale)
    dmax = max(1_000_000.0 * scale, 8.0)
    return hub_skewed(n_u, n_v, m, 1.8, min(dmax, n_u), 5.0, seed)


def batch_shapes(count: int, seed: int) -> list[tuple[int, int, int]]:
    """(|U|, |V|, m) per graph: sizes log-uniform, m clamped to |U||V|/4."""
    rng = np.random.Generator(np.random.PCG64([seed, 3]))
    out = []
    for _ in range(count):
        n_u = int(round(np.exp(rng.uniform(np.log(64), np.log(20_000)))))
        n_v = int(round(np.exp(rng.uniform(np.log(64), np.log(20_000)))))
        m = int(round(np.exp(rng.uniform(np.log(256), np.log(500_000)))))
        m = min(m, (n_u * n_v) // 4)
        out.append((n_u, n_v, m))
    return out


def batch_graph(n_u: int, n_v: int, m: int, seed: int) -> BipartiteCSR:
    """One graph of the batched workload: Chung-Lu, exponent 2.1, weights capped
    at the opposite side's size."""
    return chung_lu(n_u, n_v, m, 2.1, float(n_v), float(n_u), seed)


def workload_batch(count: int = 4096, seed: int = 4) -> list[BipartiteCSR]:
    return [batch_graph(nu, nv, m, seed * 1_000_003 + i)
            for i, (nu, nv, m) in enumerate(batch_shapes(count, seed))]


def serve_big_graph(i: int) -> BipartiteCSR:
    """One of the serving pool's large graphs: Chung-Lu, |U|=200k, |V|=50k,
    m=5M, exponent 2.1."""
    return chung_lu(200_000, 50_000, 5_000_000, 2.1, 50_000.0, 200_000.0, 5_000 + i)


def workload_serve_pool(pool_small: int = 10_000, pool_big: int = 50) -> list[BipartiteCSR]:
    """The serving pool: graphs shaped as the batched workload (seed 5), then
    the large graphs."""
    return workload_batch(pool_small, seed=5) + [serve_big_graph(i) for i in range(pool_big)]
