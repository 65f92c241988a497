"""Pure-Python brute force for tiny graphs (no shared code with oracle/ or the
library): butterflies from the four-edge definition, wedges from the
framework's path definition, and the orderings simulated step by step."""
from itertools import combinations


def edge_set(g):
    u, v = g.edges()
    return {(int(a), int(b)): k for k, (a, b) in enumerate(zip(u, v))}


def butterflies(g):
    """Every butterfly as (u1, u2, v1, v2) with u1 < u2, v1 < v2 (Preliminaries)."""
    es = edge_set(g)
    out = []
    for u1, u2 in combinations(range(g.n_u), 2):
        for v1, v2 in combinations(range(g.n_v), 2):
            if all((a, b) in es for a in (u1, u2) for b in (v1, v2)):
                out.append((u1, u2, v1, v2))
    return out


def counts(g):
    es = edge_set(g)
    vert = [0] * (g.n_u + g.n_v)
    edge = [0] * g.m
    bfs = butterflies(g)
    for u1, u2, v1, v2 in bfs:
        for x in (u1, u2):
            vert[x] += 1
        for y in (v1, v2):
            vert[g.n_u + y] += 1
        for a in (u1, u2):
            for b in (v1, v2):
                edge[es[(a, b)]] += 1
    return len(bfs), vert, edge


def neighbours(g):
    """Adjacency over unified ids."""
    nb = [set() for _ in range(g.n_u + g.n_v)]
    for a, b in edge_set(g):
        nb[a].add(g.n_u + b)
        nb[g.n_u + b].add(a)
    return nb


def wedges(g, rank):
    """Framework step 2: paths x - y - z, x != z, rank y > rank x, rank z > rank x."""
    nb = neighbours(g)
    out = []
    for x in range(g.n_u + g.n_v):
        for y in nb[x]:
            if rank[y] <= rank[x]:
                continue
            for z in nb[y]:
                if z != x and rank[z] > rank[x]:
                    out.append((x, y, z))
    return out


def level(d):
    return d.bit_length() - 1 if d > 0 else -1


def order(g, kind):
    """rank[x] for the orderings of Section 3.1.1, ties by smaller unified id."""
    nb = neighbours(g)
    n = g.n_u + g.n_v
    deg = [len(s) for s in nb]
    if kind in ("side_u", "side_v", "side_auto"):
        u_first = kind == "side_u"
        if kind == "side_auto":
            wu = sum(d * (d - 1) // 2 for d in deg[g.n_u:])
            wv = sum(d * (d - 1) // 2 for d in deg[:g.n_u])
            u_first = wu <= wv
        seq = list(range(n)) if u_first else list(range(g.n_u, n)) + list(range(g.n_u))
    elif kind == "degree":
        seq = sorted(range(n), key=lambda x: (-deg[x], x))
    elif kind == "approx_degree":
        seq = sorted(range(n), key=lambda x: (-level(deg[x]), x))
    elif kind in ("codeg", "approx_codeg"):
        key = (lambda d: d) if kind == "codeg" else level
        alive = set(range(n))
        seq = []
        while alive:
            cur = {x: len(nb[x] & alive) for x in alive}
            top = max(key(cur[x]) for x in alive)
            front = sorted(x for x in alive if key(cur[x]) == top)
            seq.extend(front)
            alive -= set(front)
    else:
        raise ValueError(kind)
    rank = [0] * n
    for i, x in enumerate(seq):
        rank[x] = i
    return rank
