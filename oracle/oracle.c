/*
 * Butterfly-counting oracle: TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded C that computes what the counting library
 * computes, straight from the definitions, so that the library can be checked
 * against it.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load this code; the library never does, and the two
 * share no source.
 *
 * Definitions (paper, Section 2 "Preliminaries", graph notation):
 *   a butterfly is {u1, u2 in U, v1, v2 in V} with all four edges present;
 *   b(x) = number of butterflies containing vertex x;
 *   b(e) = number of butterflies containing edge e;
 *   B    = number of butterflies.
 * Lemma "lem-count" (Section 4.4, equations eq-vert and eq-edge):
 *   b(u)   = sum over u' != u of C(|N(u) & N(u')|, 2)
 *   b(u,v) = sum over u' in N(v), u' != u, of (|N(u) & N(u')| - 1)
 *
 * Input format (every function): a U-side CSR, u_off[n_u + 1] (int64) and
 * u_adj[m] (uint32, V-local ids), rows strictly increasing.  Unified vertex
 * ids are U = [0, n_u) then V = [n_u, n_u + n_v).  Per-vertex outputs are in
 * unified-id order, per-edge outputs in u_adj position order.
 *
 * Tiers:
 *   orc_bf4    4-tuple brute force from the butterfly definition (tiny graphs)
 *   orc_pairs  vertex-pair brute force: the Lemma summed over all pairs
 *   orc_count  the oracle proper: dense 2-hop counts per endpoint, O(sum deg^2)
 *   orc_wedges number of wedges the ranked framework retrieves for a ranking
 *   orc_rank   the reference vertex orderings (Section 3.1.1)
 *   orc_sparsify  the kept graph of edge or colorful sparsification (Section
 *              4.6 "Approximate counting")
 *   orc_tip    tip numbers by vertex peeling (Section 3.2, Algorithm 5)
 *   orc_wing   wing numbers by edge peeling (Section 3.2, Algorithm 6)
 * Every function returns 0 on success and a negative value on bad input or
 * allocation failure.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static int64_t choose2(int64_t c) { return c * (c - 1) / 2; }

/* ------------------------------------------------------------------------- */
/* Input checks shared by the entry points of this file.                      */

static int check_csr(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj) {
    if (n_u < 0 || n_v < 0 || !u_off) return -1;
    if (u_off[0] != 0) return -1;
    for (int64_t u = 0; u < n_u; ++u) {
        if (u_off[u + 1] < u_off[u]) return -1;
        for (int64_t k = u_off[u]; k < u_off[u + 1]; ++k) {
            if ((int64_t)u_adj[k] >= n_v) return -2;
            if (k > u_off[u] && u_adj[k] <= u_adj[k - 1]) return -3;
        }
    }
    return 0;
}

/* V-side adjacency built by plain counting: v_off[n_v+1], v_adj[m] = u ids in
 * increasing order, v_eid[m] = position of that edge in u_adj. */
typedef struct {
    int64_t *off;
    uint32_t *adj;
    int64_t *eid;
} vside;

static int build_vside(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj,
                       vside *out) {
    int64_t m = u_off[n_u];
    out->off = (int64_t *)calloc((size_t)n_v + 1, sizeof(int64_t));
    out->adj = (uint32_t *)malloc((size_t)(m ? m : 1) * sizeof(uint32_t));
    out->eid = (int64_t *)malloc((size_t)(m ? m : 1) * sizeof(int64_t));
    int64_t *fill = (int64_t *)calloc((size_t)n_v + 1, sizeof(int64_t));
    if (!out->off || !out->adj || !out->eid || !fill) {
        free(out->off); free(out->adj); free(out->eid); free(fill);
        return -4;
    }
    for (int64_t k = 0; k < m; ++k) out->off[u_adj[k] + 1]++;
    for (int64_t v = 0; v < n_v; ++v) out->off[v + 1] += out->off[v];
    for (int64_t u = 0; u < n_u; ++u)
        for (int64_t k = u_off[u]; k < u_off[u + 1]; ++k) {
            int64_t v = u_adj[k];
            int64_t p = out->off[v] + fill[v]++;
            out->adj[p] = (uint32_t)u;
            out->eid[p] = k;
        }
    free(fill);
    return 0;
}

static void free_vside(vside *s) { free(s->off); free(s->adj); free(s->eid); }

static void zero_outputs(int64_t n, int64_t m, int64_t *glob, int64_t *vert, int64_t *edge) {
    if (glob) *glob = 0;
    if (vert) memset(vert, 0, (size_t)n * sizeof(int64_t));
    if (edge) memset(edge, 0, (size_t)m * sizeof(int64_t));
}

/* ------------------------------------------------------------------------- */
/* T0: enumerate every {u1 < u2} x {v1 < v2} and test the four edges. */

int orc_bf4(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj,
            int64_t *glob, int64_t *vert, int64_t *edge) {
    int rc = check_csr(n_u, n_v, u_off, u_adj);
    if (rc) return rc;
    int64_t m = u_off[n_u];
    /* eidx[u * n_v + v] = edge position + 1, or 0 when absent */
    int64_t cells = n_u * n_v;
    int64_t *eidx = (int64_t *)calloc((size_t)(cells > 0 ? cells : 1), sizeof(int64_t));
    if (!eidx) return -4;
    for (int64_t u = 0; u < n_u; ++u)
        for (int64_t k = u_off[u]; k < u_off[u + 1]; ++k) eidx[u * n_v + u_adj[k]] = k + 1;
    zero_outputs(n_u + n_v, m, glob, vert, edge);
    for (int64_t u1 = 0; u1 < n_u; ++u1)
        for (int64_t u2 = u1 + 1; u2 < n_u; ++u2)
            for (int64_t v1 = 0; v1 < n_v; ++v1)
                for (int64_t v2 = v1 + 1; v2 < n_v; ++v2) {
                    int64_t a = eidx[u1 * n_v + v1], b = eidx[u1 * n_v + v2];
                    int64_t c = eidx[u2 * n_v + v1], d = eidx[u2 * n_v + v2];
                    if (!a || !b || !c || !d) continue;
                    if (glob) *glob += 1;
                    if (vert) {
                        vert[u1]++; vert[u2]++;
                        vert[n_u + v1]++; vert[n_u + v2]++;
                    }
                    if (edge) { edge[a - 1]++; edge[b - 1]++; edge[c - 1]++; edge[d - 1]++; }
                }
    free(eidx);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* T1: the Lemma applied to every pair of same-side vertices, with
 * |N(t) & N(t')| from a sorted merge. */

static int64_t merge_count(const uint32_t *a, int64_t na, const uint32_t *b, int64_t nb) {
    int64_t i = 0, j = 0, c = 0;
    while (i < na && j < nb) {
        if (a[i] < b[j]) ++i;
        else if (a[i] > b[j]) ++j;
        else { ++c; ++i; ++j; }
    }
    return c;
}

int orc_pairs(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj,
              int64_t *glob, int64_t *vert, int64_t *edge) {
    int rc = check_csr(n_u, n_v, u_off, u_adj);
    if (rc) return rc;
    int64_t m = u_off[n_u];
    vside vs;
    if (build_vside(n_u, n_v, u_off, u_adj, &vs)) return -4;
    zero_outputs(n_u + n_v, m, glob, vert, edge);
    /* U pairs: global, b(u) by eq-vert */
    int64_t total = 0;
    for (int64_t a = 0; a < n_u; ++a)
        for (int64_t b = a + 1; b < n_u; ++b) {
            int64_t c = merge_count(u_adj + u_off[a], u_off[a + 1] - u_off[a],
                                    u_adj + u_off[b], u_off[b + 1] - u_off[b]);
            int64_t bf = choose2(c);
            total += bf;
            if (vert) { vert[a] += bf; vert[b] += bf; }
        }
    if (glob) *glob = total;
    /* V pairs: b(v) by eq-vert applied with the sides swapped */
    if (vert)
        for (int64_t a = 0; a < n_v; ++a)
            for (int64_t b = a + 1; b < n_v; ++b) {
                int64_t c = merge_count(vs.adj + vs.off[a], vs.off[a + 1] - vs.off[a],
                                        vs.adj + vs.off[b], vs.off[b + 1] - vs.off[b]);
                int64_t bf = choose2(c);
                vert[n_u + a] += bf;
                vert[n_u + b] += bf;
            }
    /* edges: eq-edge, b(u,v) = sum_{u' in N(v), u' != u} (|N(u) & N(u')| - 1) */
    if (edge)
        for (int64_t u = 0; u < n_u; ++u)
            for (int64_t k = u_off[u]; k < u_off[u + 1]; ++k) {
                int64_t v = u_adj[k], s = 0;
                for (int64_t q = vs.off[v]; q < vs.off[v + 1]; ++q) {
                    int64_t u2 = vs.adj[q];
                    if (u2 == u) continue;
                    s += merge_count(u_adj + u_off[u], u_off[u + 1] - u_off[u],
                                     u_adj + u_off[u2], u_off[u2 + 1] - u_off[u2]) - 1;
                }
                edge[k] = s;
            }
    free_vside(&vs);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* T2, the oracle proper.  Centers S are the side with the smaller sum of
 * squared degrees, endpoints T the other side.  For each endpoint t the dense
 * array c[t'] = |N(t) & N(t')| is built by walking t -> s -> t'; then
 *   b(t)   = sum_{t'} C(c[t'], 2)                         (eq-vert)
 *   b(t,s) = sum_{t' in N(s), t' != t} (c[t'] - 1)        (eq-edge)
 *   b(s)   = (1/2) sum_{t in N(s)} b(t,s)  (a butterfly holds two edges at s)
 *   B      = (1/2) sum_t b(t)              (a butterfly holds two T vertices)
 */
static int count_t2(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj,
                    int64_t t_stride, int64_t *glob, int64_t *vert, int64_t *edge);

int orc_count(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj,
              int64_t *glob, int64_t *vert, int64_t *edge) {
    return count_t2(n_u, n_v, u_off, u_adj, 1, glob, vert, edge);
}

/* The same computation restricted to every t_stride-th endpoint (outputs are
 * partial sums): lets a caller time a bounded sample of the full oracle run. */
int orc_count_sample(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj,
                     int64_t t_stride, int64_t *glob) {
    if (t_stride < 1) return -1;
    int64_t m = u_off[n_u];
    int64_t *vert = (int64_t *)malloc((size_t)(n_u + n_v > 0 ? n_u + n_v : 1) * sizeof(int64_t));
    int64_t *edge = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    int rc = (vert && edge) ? count_t2(n_u, n_v, u_off, u_adj, t_stride, glob, vert, edge) : -4;
    free(vert);
    free(edge);
    return rc;
}

static int count_t2(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj,
                    int64_t t_stride, int64_t *glob, int64_t *vert, int64_t *edge) {
    int rc = check_csr(n_u, n_v, u_off, u_adj);
    if (rc) return rc;
    int64_t m = u_off[n_u];
    vside vs;
    if (build_vside(n_u, n_v, u_off, u_adj, &vs)) return -4;

    double sq_u = 0.0, sq_v = 0.0; /* only decides the side */
    for (int64_t u = 0; u < n_u; ++u) { double d = (double)(u_off[u + 1] - u_off[u]); sq_u += d * d; }
    for (int64_t v = 0; v < n_v; ++v) { double d = (double)(vs.off[v + 1] - vs.off[v]); sq_v += d * d; }
    int centers_u = sq_u <= sq_v; /* S = U when its squared-degree sum is smaller */

    /* endpoint side T adjacency (t -> s) and center side S adjacency (s -> t) */
    int64_t n_t = centers_u ? n_v : n_u;
    const int64_t *t_off = centers_u ? vs.off : u_off;
    const uint32_t *t_adj = centers_u ? vs.adj : u_adj;
    const int64_t *s_off = centers_u ? u_off : vs.off;
    const uint32_t *s_adj = centers_u ? u_adj : vs.adj;
    int64_t t_base = centers_u ? n_u : 0; /* unified id of t = t_base + t */
    int64_t s_base = centers_u ? 0 : n_u;

    int64_t *cnt = (int64_t *)calloc((size_t)(n_t ? n_t : 1), sizeof(int64_t));
    int64_t *touched = (int64_t *)malloc((size_t)(n_t ? n_t : 1) * sizeof(int64_t));
    int64_t *bedge = (int64_t *)calloc((size_t)(m ? m : 1), sizeof(int64_t)); /* in u_adj order */
    if (!cnt || !touched || !bedge) {
        free(cnt); free(touched); free(bedge); free_vside(&vs);
        return -4;
    }
    zero_outputs(n_u + n_v, m, glob, vert, edge);
    int64_t twice_total = 0;
    for (int64_t t = 0; t < n_t; t += t_stride) {
        int64_t nt = 0;
        for (int64_t a = t_off[t]; a < t_off[t + 1]; ++a) {
            int64_t s = t_adj[a];
            for (int64_t b = s_off[s]; b < s_off[s + 1]; ++b) {
                int64_t t2 = s_adj[b];
                if (t2 == t) continue;
                if (cnt[t2]++ == 0) touched[nt++] = t2;
            }
        }
        int64_t bt = 0;
        for (int64_t i = 0; i < nt; ++i) bt += choose2(cnt[touched[i]]);
        twice_total += bt;
        if (vert) vert[t_base + t] = bt;
        for (int64_t a = t_off[t]; a < t_off[t + 1]; ++a) {
            int64_t s = t_adj[a];
            int64_t sum = 0;
            for (int64_t b = s_off[s]; b < s_off[s + 1]; ++b) {
                int64_t t2 = s_adj[b];
                if (t2 == t) continue;
                sum += cnt[t2] - 1;
            }
            /* the edge (t, s) in u_adj order */
            int64_t k = centers_u ? vs.eid[a] : a;
            bedge[k] = sum;
            if (vert) vert[s_base + s] += sum;
        }
        for (int64_t i = 0; i < nt; ++i) cnt[touched[i]] = 0;
    }
    if (vert)
        for (int64_t s = 0; s < (centers_u ? n_u : n_v); ++s) vert[s_base + s] /= 2;
    if (glob) *glob = twice_total / 2;
    if (edge) memcpy(edge, bedge, (size_t)m * sizeof(int64_t));
    free(cnt); free(touched); free(bedge); free_vside(&vs);
    return 0;
}

/* Single outputs, computed alone (for sampled checks on large graphs). */

/* b(x) for one unified id x, by eq-vert with a dense 2-hop count. */
int orc_vertex_one(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj,
                   const int64_t *v_off, const uint32_t *v_adj, int64_t x, int64_t *out) {
    if (x < 0 || x >= n_u + n_v) return -1;
    int is_u = x < n_u;
    int64_t t = is_u ? x : x - n_u;
    int64_t n_t = is_u ? n_u : n_v;
    const int64_t *t_off = is_u ? u_off : v_off;
    const uint32_t *t_adj = is_u ? u_adj : v_adj;
    const int64_t *s_off = is_u ? v_off : u_off;
    const uint32_t *s_adj = is_u ? v_adj : u_adj;
    int64_t *cnt = (int64_t *)calloc((size_t)(n_t ? n_t : 1), sizeof(int64_t));
    if (!cnt) return -4;
    int64_t r = 0;
    for (int64_t a = t_off[t]; a < t_off[t + 1]; ++a) {
        int64_t s = t_adj[a];
        for (int64_t b = s_off[s]; b < s_off[s + 1]; ++b) {
            int64_t t2 = s_adj[b];
            if (t2 == t) continue;
            r += cnt[t2]++; /* adds C(c+1,2) - C(c,2) = c */
        }
    }
    free(cnt);
    *out = r;
    return 0;
}

/* b(e) for the edge at u_adj position e, by eq-edge with a marker array over N(u). */
int orc_edge_one(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj,
                 const int64_t *v_off, const uint32_t *v_adj, int64_t e, int64_t *out) {
    int64_t m = u_off[n_u];
    if (e < 0 || e >= m) return -1;
    int64_t lo = 0, hi = n_u; /* u = the row holding position e */
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) / 2;
        if (u_off[mid] <= e) lo = mid; else hi = mid;
    }
    int64_t u = lo, v = u_adj[e];
    unsigned char *mark = (unsigned char *)calloc((size_t)(n_v ? n_v : 1), 1);
    if (!mark) return -4;
    for (int64_t k = u_off[u]; k < u_off[u + 1]; ++k) mark[u_adj[k]] = 1;
    int64_t s = 0;
    for (int64_t q = v_off[v]; q < v_off[v + 1]; ++q) {
        int64_t u2 = v_adj[q];
        if (u2 == u) continue;
        int64_t c = 0;
        for (int64_t k = u_off[u2]; k < u_off[u2 + 1]; ++k) c += mark[u_adj[k]];
        s += c - 1;
    }
    free(mark);
    *out = s;
    return 0;
}

/* V-side CSR for callers of the single-output functions. */
int orc_vside(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj,
              int64_t *v_off, uint32_t *v_adj) {
    int rc = check_csr(n_u, n_v, u_off, u_adj);
    if (rc) return rc;
    vside vs;
    if (build_vside(n_u, n_v, u_off, u_adj, &vs)) return -4;
    memcpy(v_off, vs.off, (size_t)(n_v + 1) * sizeof(int64_t));
    memcpy(v_adj, vs.adj, (size_t)u_off[n_u] * sizeof(uint32_t));
    free_vside(&vs);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Wedges retrieved under a ranking (framework step 2, Section 3.1): every
 * path x - y - z with x != z, rank(y) > rank(x) and rank(z) > rank(x).  For
 * each edge, x is its lower-ranked endpoint and y the other one, and the
 * count is |{z in N(y) : rank z > rank x}|, found by binary search in the
 * rank-sorted copy of N(y).  per_source[x] (optional, unified ids) receives
 * the wedges rooted at x. */

static int cmp_u32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

int orc_wedges(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj,
               const uint32_t *rank, int64_t *total, int64_t *per_source) {
    int rc = check_csr(n_u, n_v, u_off, u_adj);
    if (rc) return rc;
    int64_t n = n_u + n_v, m = u_off[n_u];
    vside vs;
    if (build_vside(n_u, n_v, u_off, u_adj, &vs)) return -4;
    /* rank-sorted neighbour ranks of every vertex */
    uint32_t *ru = (uint32_t *)malloc((size_t)(m ? m : 1) * sizeof(uint32_t));
    uint32_t *rv = (uint32_t *)malloc((size_t)(m ? m : 1) * sizeof(uint32_t));
    if (!ru || !rv) { free(ru); free(rv); free_vside(&vs); return -4; }
    for (int64_t k = 0; k < m; ++k) ru[k] = rank[n_u + u_adj[k]];
    for (int64_t k = 0; k < m; ++k) rv[k] = rank[vs.adj[k]];
    for (int64_t u = 0; u < n_u; ++u)
        qsort(ru + u_off[u], (size_t)(u_off[u + 1] - u_off[u]), sizeof(uint32_t), cmp_u32);
    for (int64_t v = 0; v < n_v; ++v)
        qsort(rv + vs.off[v], (size_t)(vs.off[v + 1] - vs.off[v]), sizeof(uint32_t), cmp_u32);
    if (per_source) memset(per_source, 0, (size_t)n * sizeof(int64_t));
    int64_t w = 0;
    for (int64_t u = 0; u < n_u; ++u)
        for (int64_t k = u_off[u]; k < u_off[u + 1]; ++k) {
            int64_t v = u_adj[k];
            uint32_t r_u = rank[u], r_v = rank[n_u + v];
            const uint32_t *list; int64_t len; uint32_t rx; int64_t x;
            if (r_u < r_v) { list = rv + vs.off[v]; len = vs.off[v + 1] - vs.off[v]; rx = r_u; x = u; }
            else { list = ru + u_off[u]; len = u_off[u + 1] - u_off[u]; rx = r_v; x = n_u + v; }
            int64_t lo = 0, hi = len; /* first index with list[i] > rx */
            while (lo < hi) {
                int64_t mid = (lo + hi) / 2;
                if (list[mid] <= rx) lo = mid + 1; else hi = mid;
            }
            w += len - lo;
            if (per_source) per_source[x] += len - lo;
        }
    *total = w;
    free(ru); free(rv); free_vside(&vs);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Reference orderings (Section 3.1.1 "Ranking").  rank[x] = index of unified
 * id x in the order.  Ties always go to the smaller unified id.
 *   ORC_SIDE_U / ORC_SIDE_V: one whole side first, ids ascending in each side
 *   ORC_SIDE_AUTO: the side whose choice retrieves fewer wedges; U first iff
 *       sum_{v in V} C(deg v, 2) <= sum_{u in U} C(deg u, 2)
 *   ORC_DEGREE: decreasing degree
 *   ORC_APPROX_DEGREE: decreasing floor(log2 degree) (degree 0 last)
 *   ORC_CODEG / ORC_APPROX_CODEG: complement degeneracy and its approximation:
 *       rounds; each round removes every remaining vertex whose key equals the
 *       largest key among remaining vertices, key = current degree (number of
 *       remaining neighbours) or its floor(log2) (0 -> -1); the removed
 *       vertices take the next ranks in id order. */

static int level_of(int64_t d) {
    if (d <= 0) return -1;
    int l = 0;
    while (d > 1) { d >>= 1; ++l; }
    return l;
}

typedef struct { int64_t key; int64_t id; } keyed;

static int cmp_keyed(const void *a, const void *b) {
    const keyed *x = (const keyed *)a, *y = (const keyed *)b;
    if (x->key != y->key) return x->key > y->key ? -1 : 1; /* key descending */
    return (x->id > y->id) - (x->id < y->id);               /* id ascending */
}

int orc_rank(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj, int kind,
             uint32_t *rank) {
    int rc = check_csr(n_u, n_v, u_off, u_adj);
    if (rc) return rc;
    int64_t n = n_u + n_v;
    vside vs;
    if (build_vside(n_u, n_v, u_off, u_adj, &vs)) return -4;
    int64_t *deg = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
    if (!deg) { free_vside(&vs); return -4; }
    for (int64_t u = 0; u < n_u; ++u) deg[u] = u_off[u + 1] - u_off[u];
    for (int64_t v = 0; v < n_v; ++v) deg[n_u + v] = vs.off[v + 1] - vs.off[v];
    rc = 0;
    if (kind == ORC_SIDE_U || kind == ORC_SIDE_V || kind == ORC_SIDE_AUTO) {
        int u_first = kind == ORC_SIDE_U;
        if (kind == ORC_SIDE_AUTO) {
            int64_t wu = 0, wv = 0; /* wedges with endpoints in U / in V */
            for (int64_t v = 0; v < n_v; ++v) wu += choose2(deg[n_u + v]);
            for (int64_t u = 0; u < n_u; ++u) wv += choose2(deg[u]);
            u_first = wu <= wv;
        }
        for (int64_t x = 0; x < n; ++x) {
            int is_u = x < n_u;
            if (u_first) rank[x] = (uint32_t)x;
            else rank[x] = (uint32_t)(is_u ? n_v + x : x - n_u);
        }
    } else if (kind == ORC_DEGREE || kind == ORC_APPROX_DEGREE) {
        keyed *ks = (keyed *)malloc((size_t)(n ? n : 1) * sizeof(keyed));
        if (!ks) { rc = -4; goto done; }
        for (int64_t x = 0; x < n; ++x) {
            ks[x].id = x;
            ks[x].key = kind == ORC_DEGREE ? deg[x] : level_of(deg[x]);
        }
        qsort(ks, (size_t)n, sizeof(keyed), cmp_keyed);
        for (int64_t i = 0; i < n; ++i) rank[ks[i].id] = (uint32_t)i;
        free(ks);
    } else if (kind == ORC_CODEG || kind == ORC_APPROX_CODEG) {
        int64_t *cur = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
        unsigned char *gone = (unsigned char *)calloc((size_t)(n ? n : 1), 1);
        unsigned char *front = (unsigned char *)calloc((size_t)(n ? n : 1), 1);
        if (!cur || !gone || !front) { free(cur); free(gone); free(front); rc = -4; goto done; }
        memcpy(cur, deg, (size_t)n * sizeof(int64_t));
        int64_t next = 0;
        while (next < n) {
            int64_t best = INT64_MIN;
            for (int64_t x = 0; x < n; ++x)
                if (!gone[x]) {
                    int64_t k = kind == ORC_CODEG ? cur[x] : level_of(cur[x]);
                    if (k > best) best = k;
                }
            for (int64_t x = 0; x < n; ++x) {
                front[x] = 0;
                if (gone[x]) continue;
                int64_t k = kind == ORC_CODEG ? cur[x] : level_of(cur[x]);
                if (k == best) { front[x] = 1; rank[x] = (uint32_t)next++; }
            }
            for (int64_t x = 0; x < n; ++x) {
                if (!front[x]) continue;
                gone[x] = 1;
                if (x < n_u) {
                    for (int64_t k = u_off[x]; k < u_off[x + 1]; ++k) cur[n_u + u_adj[k]]--;
                } else {
                    int64_t v = x - n_u;
                    for (int64_t k = vs.off[v]; k < vs.off[v + 1]; ++k) cur[vs.adj[k]]--;
                }
            }
        }
        free(cur); free(gone); free(front);
    } else {
        rc = -1;
    }
done:
    free(deg);
    free_vside(&vs);
    return rc;
}

/*
 * Sparsification (Section 4.6 "Approximate counting").  Edge sparsification
 * keeps each edge independently with probability p; colorful sparsification
 * gives every vertex one of c = ceil(1/p) colours and keeps the edges whose
 * two endpoints have the same colour.  The kept graph is then counted exactly.
 *
 * Random numbers: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) from state `seed`: its output
 * number i + 1 is x(i) = mix(seed + (i + 1) * 0x9E3779B97F4A7C15), mix being
 * its 64-bit finaliser.  Edge e (its position in u_adj) is kept when x(e) <
 * floor(p * 2^64) (every edge when p >= 1).  Vertex i (unified id) has colour
 * floor(x(i) * c / 2^64).
 */
uint64_t orc_splitmix(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* high 64 bits of the 128-bit product x * c, from 32-bit halves */
static uint64_t mul_hi(uint64_t x, uint64_t c) {
    const uint64_t x0 = x & 0xFFFFFFFFull, x1 = x >> 32, c0 = c & 0xFFFFFFFFull, c1 = c >> 32;
    const uint64_t p00 = x0 * c0, p01 = x0 * c1, p10 = x1 * c0, p11 = x1 * c1;
    const uint64_t mid = (p00 >> 32) + (p01 & 0xFFFFFFFFull) + (p10 & 0xFFFFFFFFull);
    return p11 + (p01 >> 32) + (p10 >> 32) + (mid >> 32);
}

/* kind 0: edge sparsification, 1: colorful.  Writes the kept edges in input
 * order as a U-side CSR (out_off[n_u + 1], out_adj[m] capacity) and their
 * number in *kept. */
int orc_sparsify(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj, int kind, double p,
                 uint64_t seed, int64_t *out_off, uint32_t *out_adj, int64_t *kept) {
    if (check_csr(n_u, n_v, u_off, u_adj) != 0 || !(p > 0.0) || kind < 0 || kind > 1) return -1;
    const int all = p >= 1.0;
    const uint64_t thr = all ? 0 : (uint64_t)ldexp(p, 64);
    const uint64_t c = all ? 1 : (uint64_t)ceil(1.0 / p);
    int64_t k = 0;
    out_off[0] = 0;
    for (int64_t u = 0; u < n_u; ++u) {
        const uint64_t cu = mul_hi(orc_splitmix(seed, (uint64_t)u), c);
        for (int64_t e = u_off[u]; e < u_off[u + 1]; ++e) {
            int keep;
            if (kind == 0) {
                keep = all || orc_splitmix(seed, (uint64_t)e) < thr;
            } else {
                const uint64_t cv = mul_hi(orc_splitmix(seed, (uint64_t)(n_u + u_adj[e])), c);
                keep = cu == cv;
            }
            if (keep) out_adj[k++] = u_adj[e];
        }
        out_off[u + 1] = k;
    }
    *kept = k;
    return 0;
}

/*
 * Tip decomposition by vertex peeling (Section 3.2 "Peeling Framework" and
 * Algorithm 5, PEEL-V / UPDATE-V).  One side X is peeled (side 1 = U, 2 = V,
 * 0 = the side whose vertices, as wedge endpoints, give the fewest wedges:
 * U when sum over V of C(deg, 2) <= sum over U of C(deg, 2)).  B starts as
 * the per-vertex butterfly counts.  Each round sets k = max(k, smallest B
 * among the remaining X vertices), peels every remaining X vertex with B <= k
 * (its tip number is k), and for every peeled u1 and every remaining u2 of X
 * lowers B(u2) by C(c, 2), c = the number of common neighbours of u1 and u2
 * (the butterflies the peeled vertices take with them).  tip[x] is written for
 * every unified id; the other side gets -1.  *rounds_out counts the rounds.
 */
int orc_tip(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj, int side, int64_t *tip,
            int64_t *rounds_out) {
    if (check_csr(n_u, n_v, u_off, u_adj) != 0 || side < 0 || side > 2) return -1;
    const int64_t n = n_u + n_v, m = n_u ? u_off[n_u] : 0;
    vside vs;
    if (build_vside(n_u, n_v, u_off, u_adj, &vs) != 0) return -2;
    int64_t *glob = malloc(sizeof(int64_t)), *vert = calloc((size_t)(n ? n : 1), sizeof(int64_t));
    int64_t *edge = calloc((size_t)(m ? m : 1), sizeof(int64_t));
    if (!glob || !vert || !edge || orc_count(n_u, n_v, u_off, u_adj, glob, vert, edge) != 0) {
        free(glob); free(vert); free(edge); free_vside(&vs);
        return -2;
    }
    if (side == 0) {
        int64_t su = 0, sv = 0;  /* wedges with U endpoints (V centres), with V endpoints */
        for (int64_t v = 0; v < n_v; ++v) su += choose2(vs.off[v + 1] - vs.off[v]);
        for (int64_t u = 0; u < n_u; ++u) sv += choose2(u_off[u + 1] - u_off[u]);
        side = su <= sv ? 1 : 2;
    }
    /* X = peeled side: its vertices' lists (off/adj into the other side) and
     * the other side's lists back into X; ids local to each side */
    const int64_t nx = side == 1 ? n_u : n_v, base = side == 1 ? 0 : n_u;
    const int64_t *xoff = side == 1 ? u_off : vs.off, *yoff = side == 1 ? vs.off : u_off;
    const uint32_t *xadj = side == 1 ? u_adj : vs.adj, *yadj = side == 1 ? vs.adj : u_adj;
    int64_t *b = malloc(sizeof(int64_t) * (size_t)(nx ? nx : 1));
    int64_t *c = calloc((size_t)(nx ? nx : 1), sizeof(int64_t));
    char *gone = calloc((size_t)(nx ? nx : 1), 1);
    int64_t *front = malloc(sizeof(int64_t) * (size_t)(nx ? nx : 1));
    if (!b || !c || !gone || !front) {
        free(b); free(c); free(gone); free(front); free(glob); free(vert); free(edge); free_vside(&vs);
        return -2;
    }
    for (int64_t x = 0; x < n; ++x) tip[x] = -1;
    for (int64_t x = 0; x < nx; ++x) b[x] = vert[base + x];
    int64_t left = nx, k = 0, rounds = 0;
    while (left > 0) {
        int64_t mn = -1;
        for (int64_t x = 0; x < nx; ++x)
            if (!gone[x] && (mn < 0 || b[x] < mn)) mn = b[x];
        if (mn > k) k = mn;
        int64_t nf = 0;
        for (int64_t x = 0; x < nx; ++x)
            if (!gone[x] && b[x] <= k) front[nf++] = x;
        for (int64_t i = 0; i < nf; ++i) {
            gone[front[i]] = 1;
            tip[base + front[i]] = k;
        }
        /* UPDATE-V: 2-hop counts from each peeled vertex to the remaining ones */
        for (int64_t i = 0; i < nf; ++i) {
            const int64_t u1 = front[i];
            for (int64_t p = xoff[u1]; p < xoff[u1 + 1]; ++p) {
                const uint32_t y = xadj[p];
                for (int64_t q = yoff[y]; q < yoff[y + 1]; ++q)
                    if (!gone[yadj[q]]) c[yadj[q]]++;
            }
            for (int64_t p = xoff[u1]; p < xoff[u1 + 1]; ++p) {
                const uint32_t y = xadj[p];
                for (int64_t q = yoff[y]; q < yoff[y + 1]; ++q) {
                    const uint32_t u2 = yadj[q];
                    if (c[u2]) {
                        b[u2] -= choose2(c[u2]);
                        c[u2] = 0;
                    }
                }
            }
        }
        left -= nf;
        ++rounds;
    }
    *rounds_out = rounds;
    free(b); free(c); free(gone); free(front); free(glob); free(vert); free(edge); free_vside(&vs);
    return 0;
}

/*
 * Wing decomposition by edge peeling (Section 3.2 "Peeling Framework" and
 * Algorithm 6, PEEL-E / UPDATE-E).  B starts as the per-edge butterfly
 * counts.  Each round sets k = max(k, smallest B among the remaining edges)
 * and peels every remaining edge with B <= k (its wing number is k).  Every
 * butterfly that loses an edge this round and had lost none before is
 * destroyed once: the peeled edge of smallest id among its edges peeled this
 * round enumerates it, and each of its edges that remains loses 1.  The
 * butterflies of edge (u1, v1) are (u1, v1, u2, v2) for u2 in N(v1), u2 !=
 * u1, and v2 in N(u1) & N(u2), v2 != v1.  wing[e] is indexed by u_adj
 * position; *rounds_out counts the rounds.
 */
static int64_t find_edge(const int64_t *u_off, const uint32_t *u_adj, int64_t u, uint32_t v) {
    int64_t lo = u_off[u], hi = u_off[u + 1];
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (u_adj[mid] < v) lo = mid + 1; else hi = mid;
    }
    return (lo < u_off[u + 1] && u_adj[lo] == v) ? lo : -1;
}

int orc_wing(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj, int64_t *wing,
             int64_t *rounds_out) {
    if (check_csr(n_u, n_v, u_off, u_adj) != 0) return -1;
    const int64_t n = n_u + n_v, m = n_u ? u_off[n_u] : 0;
    vside vs;
    if (build_vside(n_u, n_v, u_off, u_adj, &vs) != 0) return -2;
    int64_t *glob = malloc(sizeof(int64_t)), *vert = calloc((size_t)(n ? n : 1), sizeof(int64_t));
    int64_t *b = calloc((size_t)(m ? m : 1), sizeof(int64_t));
    int64_t *eu = malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
    int64_t *state = calloc((size_t)(m ? m : 1), sizeof(int64_t));  /* round peeled in, 0 = remaining */
    int64_t *front = malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
    if (!glob || !vert || !b || !eu || !state || !front || orc_count(n_u, n_v, u_off, u_adj, glob, vert, b) != 0) {
        free(glob); free(vert); free(b); free(eu); free(state); free(front); free_vside(&vs);
        return -2;
    }
    for (int64_t u = 0; u < n_u; ++u)
        for (int64_t e = u_off[u]; e < u_off[u + 1]; ++e) eu[e] = u;
    int64_t left = m, k = 0, rounds = 0;
    while (left > 0) {
        const int64_t r = rounds + 1;
        int64_t mn = -1;
        for (int64_t e = 0; e < m; ++e)
            if (!state[e] && (mn < 0 || b[e] < mn)) mn = b[e];
        if (mn > k) k = mn;
        int64_t nf = 0;
        for (int64_t e = 0; e < m; ++e)
            if (!state[e] && b[e] <= k) front[nf++] = e;
        for (int64_t i = 0; i < nf; ++i) {
            state[front[i]] = r;
            wing[front[i]] = k;
        }
        for (int64_t i = 0; i < nf; ++i) {
            const int64_t e = front[i], u1 = eu[e];
            const uint32_t v1 = u_adj[e];
            for (int64_t p = vs.off[v1]; p < vs.off[v1 + 1]; ++p) {
                const int64_t u2 = vs.adj[p], e2 = vs.eid[p];  /* edge (u2, v1) */
                if (u2 == u1) continue;
                for (int64_t a = u_off[u1]; a < u_off[u1 + 1]; ++a) {
                    const uint32_t v2 = u_adj[a];
                    if (v2 == v1) continue;
                    const int64_t e3 = find_edge(u_off, u_adj, u2, v2);  /* edge (u2, v2) */
                    if (e3 < 0) continue;
                    const int64_t e1 = a;                                /* edge (u1, v2) */
                    const int64_t other[3] = {e1, e2, e3};
                    int skip = 0;
                    for (int j = 0; j < 3; ++j) {
                        const int64_t s2 = state[other[j]];
                        if ((s2 && s2 < r) || (s2 == r && other[j] < e)) skip = 1;
                    }
                    if (skip) continue;
                    for (int j = 0; j < 3; ++j)
                        if (!state[other[j]]) b[other[j]] -= 1;
                }
            }
        }
        left -= nf;
        rounds = r;
    }
    *rounds_out = rounds;
    free(glob); free(vert); free(b); free(eu); free(state); free(front); free_vside(&vs);
    return 0;
}
