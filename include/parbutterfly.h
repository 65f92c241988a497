/*
 * parbutterfly: exact butterfly ((2,2)-biclique) counting on bipartite graphs,
 * for AMD Instinct MI355X (gfx950).
 *
 * The method is the ranked wedge framework of Shi and Shun, "Parallel
 * Algorithms for Butterfly Computations" (arXiv 1907.08607), Section 3.1
 * (framework figure "ParButterfly Framework for Counting"):
 *   1. rank the vertices (Section 3.1.1);
 *   2. retrieve every wedge (x1, y, x2) with rank(y) > rank(x1) and
 *      rank(x2) > rank(x1) (Algorithm 2, GET-WEDGES);
 *   3. count the wedges of each endpoint pair, R(x1, x2) (GET-FREQ, Section 3.1.2);
 *   4. turn the pair counts into butterfly counts: C(R, 2) per pair for the
 *      total (Section 3.1.3 footnote) and for each endpoint, R - 1 per wedge for
 *      its center (Algorithm 3, COUNT-V) and for its two edges (Algorithm 4,
 *      COUNT-E).
 * All counts are exact int64 integers; the result never depends on the
 * ranking, the aggregator or the launch configuration.
 *
 * Conventions used by every call:
 *   - Input graph: a U-side CSR with row offsets u_off[n_u + 1] (int64, device)
 *     and column ids u_adj[m] (uint32 V-local ids, device).  Every row must be
 *     strictly increasing (the graph is simple, Section 2) and every id < n_v.
 *     The arrays stay owned by the caller and must outlive the pb_graph.
 *   - Unified vertex ids: U vertices are 0 .. n_u-1, V vertices n_u .. n_u+n_v-1
 *     (the two sides' arrays are stored consecutively, Section 2).
 *   - Per-vertex outputs are indexed by unified id; per-edge outputs by the
 *     edge's position in u_adj.
 *   - Limits: m < 2^31 and n_u + n_v < 2^32 - 1; degrees are otherwise
 *     unrestricted.
 *   - Every buffer argument named "device" is device memory on the current
 *     HIP device; the caller owns all input and output buffers and the library
 *     never frees them.
 *   - Work is enqueued on the given stream; outputs are valid once that stream
 *     has been synchronised.  Calls that must read device-side results back
 *     (validation flags, the work plan) synchronise the stream themselves; this
 *     is stated per call.
 *   - No call aborts or prints.  Errors are returned as pb_status; arguments are
 *     checked before any work is enqueued.
 */
#ifndef PARBUTTERFLY_H
#define PARBUTTERFLY_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PB_OK = 0,
    PB_ERR_INVALID_ARG = -1, /* null pointer, size out of range, unknown enum value */
    PB_ERR_NOT_SIMPLE = -2,  /* a CSR row is not strictly increasing (duplicate edge) */
    PB_ERR_ID_RANGE = -3,    /* a column id >= n_v, or u_off is not a valid offset array */
    PB_ERR_BAD_RANK = -4,    /* rank is not a permutation of [0, n) */
    PB_ERR_NO_MEMORY = -5,   /* device allocation failed or the workspace cap is too small */
    /* Reserved; no call returns it.  Under m < 2^31 no count can overflow
     * int64: a butterfly {u1, u2, v1, v2} holds the two disjoint edges
     * (u1, v1), (u2, v2), and two disjoint edges lie in at most one
     * butterfly, so the total is at most C(m, 2) < 2^61; every per-vertex and
     * per-edge count is at most the total, the per-vertex ones sum to 4 times
     * it (< 2^63), and every partial sum the library keeps is a sum of
     * non-negative terms of one of these counts. */
    PB_ERR_OVERFLOW = -6,
    PB_ERR_HIP = -7,         /* a HIP runtime call failed */
    PB_ERR_INTERNAL = -8     /* an internal consistency check tripped (a library defect); outputs are invalid */
} pb_status;

/* The bipartite input graph (U-side CSR, device pointers). */
typedef struct {
    uint32_t n_u;
    uint32_t n_v;
    uint64_t m;
    const int64_t *u_off;  /* device, n_u + 1 entries, u_off[0] = 0, u_off[n_u] = m */
    const uint32_t *u_adj; /* device, m entries */
} pb_csr;

/* Vertex orderings (Section 3.1.1 "Ranking").  rank[x] is the index of
 * unified id x in the order; wedges are rooted at their lowest-ranked vertex.
 * Ties are broken by the smaller unified id.
 *   SIDE_AUTO     one side wholly first: the side whose choice retrieves fewer
 *                 wedges, U first iff sum_{v in V} C(deg v, 2) <= sum_{u in U} C(deg u, 2)
 *   SIDE_U_FIRST, SIDE_V_FIRST   one side forced first
 *   DEGREE        decreasing degree
 *   APPROX_DEGREE decreasing floor(log2(degree)); degree 0 last
 *   COMPLEMENT_CORENESS          complement degeneracy order: rounds, each
 *                 removing every remaining vertex whose current degree (count
 *                 of remaining neighbours) equals the largest one; the removed
 *                 vertices take the next ranks in id order
 *   APPROX_COMPLEMENT_CORENESS   the same with floor(log2(current degree)) as
 *                 the key (degree 0 -> -1) */
typedef enum {
    PB_RANK_SIDE_AUTO = 0,
    PB_RANK_SIDE_U_FIRST = 1,
    PB_RANK_SIDE_V_FIRST = 2,
    PB_RANK_DEGREE = 3,
    PB_RANK_APPROX_DEGREE = 4,
    PB_RANK_COMPLEMENT_CORENESS = 5,
    PB_RANK_APPROX_COMPLEMENT_CORENESS = 6
} pb_rank_kind;

/* Wedge aggregation (GET-FREQ, Section 3.1.2).  AUTO picks per source by the
 * source's wedge count and candidate range; the others force one method for
 * every source (results are identical, only speed differs).
 *   LDS_HASH    per-workgroup linear-probing hash table in LDS keyed by x2
 *   DENSE_HIST  dense per-source histogram over the x2 id range, swept in
 *               LDS-sized windows of that range
 *   RADIX_SORT  64-bit (x1, x2) keys radix-sorted in LDS, then run lengths */
typedef enum {
    PB_AGG_AUTO = 0,
    PB_AGG_LDS_HASH = 1,
    PB_AGG_DENSE_HIST = 2,
    PB_AGG_RADIX_SORT = 3
} pb_agg;

/* Dense int8 matrix-core tile for hub-to-hub endpoint pairs (an addition to
 * the paper's aggregators; the counts are the same in every mode).  The hubs
 * are the first 256 vertices, in rank order, of the side that holds the
 * rank-0 vertex.  For two hubs h1 < h2 the pair count R(h1, h2) of Section
 * 3.1.2 is one entry of D = A' A^T, where A is the 0/1 hub-by-centre
 * adjacency and A' keeps the centres ranked above the row's hub; D is formed
 * on int8 matrix cores with int32 accumulation (exact: entries are bounded by
 * the number of centres).  The sparse aggregators then skip hub partners of
 * hub sources.
 *   AUTO   single graphs with at least 2^22 edges, when a cost model (hub
 *          pair paths against compacted centre columns, and for per-vertex
 *          or per-edge counts the tile's own credit pass) predicts a gain;
 *          with per-vertex or per-edge counts it is evaluated only when some
 *          vertex has at least 65536 neighbours (the tile cannot win
 *          otherwise)
 *   OFF    never
 *   FORCE  every single graph with at least two vertices on the hub side
 * Batched calls never use the tile. */
typedef enum {
    PB_HUB_AUTO = 0,
    PB_HUB_OFF = 1,
    PB_HUB_FORCE = 2
} pb_hub_mode;

/* Figures a counting call reports back (host memory, optional). */
typedef struct {
    uint64_t wedges;          /* wedges retrieved under the ranking (framework step 2) */
    uint64_t sources;         /* sources with at least one wedge */
    uint64_t sources_hash;    /* sources aggregated in an LDS hash table */
    uint64_t sources_dense;   /* sources aggregated by dense LDS windows */
    uint64_t sources_sort;    /* sources aggregated by LDS radix sort */
    uint64_t window_items;    /* (source, x2-window) work items launched */
    uint64_t wedges_hash;     /* wedges of the hash-aggregated sources */
    uint64_t wedges_dense;    /* wedges of the dense-window sources */
    uint64_t wedges_sort;     /* wedges of the sort-aggregated sources */
    uint64_t wedges_hub;      /* wedges covered by dense hub tiles */
    uint64_t workspace_bytes; /* peak device scratch the call allocated */
    /* Phase times in milliseconds, measured with HIP events on the call's
     * stream; filled only when opts.flags has PB_FLAG_TIMING (which adds one
     * stream synchronisation at the end of the call). */
    double ms_prepare;        /* rank check, relabel, modified degrees, plan */
    double ms_dense;          /* dense-window counting kernel */
    double ms_hash;           /* hash counting kernels */
    double ms_sort;           /* radix-sort counting kernel */
    double ms_output;         /* output combine */
    /* The heavy-source dense-window kernel alone. */
    uint64_t wedges_heavy;    /* wedges it aggregated */
    double ms_heavy;          /* its time (PB_FLAG_TIMING) */
    /* Hub tile (zero when it was not used). */
    uint64_t hub_rows;        /* hubs in the tile */
    uint64_t hub_cols;        /* compacted centre columns */
    uint64_t hub_mfma_ops;    /* int8 operations issued on matrix cores */
    double ms_hub_gemm;       /* the matrix-core kernel (included in ms_prepare) */
    double ms_hub_pass;       /* the hub pairs' centre and edge credit pass */
    /* Giant sources (global-histogram path; included in the dense figures). */
    uint64_t wedges_global;   /* wedges they hold */
    double ms_global;         /* their time: histogram clear, walks and endpoint step (PB_FLAG_TIMING) */
    /* Bytes of one per-slot credit counter: 4 when no edge can lie in 2^32
     * butterflies (squared maximum degree below 2^32), else 8; 0 without
     * per-edge counts.  Pass 2 reads and writes one such counter per wedge. */
    uint64_t slot_credit_bytes;
} pb_stats;

/* opts.flags bits */
#define PB_FLAG_TIMING 1u
/* Retrieve each wedge from its lower-ranked endpoint: for every vertex u,
 * the wedges (x1, y, u) with x1 ranked above both y and u, aggregated by x1
 * (the cache optimisation of Section 3.1 that the paper takes from Wang et
 * al.).  The same wedges and the same counts; only the order of work changes.
 * Single-graph calls only (ignored by batched calls); the hub tile is not
 * used with it. */
#define PB_FLAG_CACHE_OPT 2u

/* Per-bucket choices: aggregator, workgroup size and batch width.  Sources
 * are bucketed by the bound min(W(x1), candidate range) on their distinct
 * endpoints (W = the source's wedges): light (<= light_max, at most 512),
 * medium (<= medium_max, at most 4096) and heavy (the rest).
 *   *_agg    the bucket's aggregator under PB_AGG_AUTO: PB_AGG_LDS_HASH,
 *            PB_AGG_RADIX_SORT or PB_AGG_DENSE_HIST
 *   *_wg     threads per workgroup of the bucket's hash and sort kernels (for
 *            medium also of the whole-range dense kernel, which takes every
 *            dense source whose candidate range is at most 4096 ids):
 *            light 64, 128 or 256 (0 = 64); medium 128, 256 or 512 (0 = 256).
 *            The heavy bucket's kernels have fixed sizes.
 *   *_width  batch width: the workgroups one launch of the bucket's kernels
 *            keeps in flight, each taking work items (sources, or source
 *            windows) until the list is done; 0 = one workgroup per item
 * The thresholds and aggregators apply under PB_AGG_AUTO only; workgroup
 * sizes and widths apply under every aggregation policy.  pb_autotune fills
 * one from timed runs; opts.tuning = NULL uses the built-in table (hash,
 * hash, dense; 512; 4096; 64, 256; widths 0). */
typedef struct {
    uint32_t light_max;
    uint32_t medium_max;
    pb_agg light_agg;
    pb_agg medium_agg;
    pb_agg heavy_agg;
    uint32_t light_wg;
    uint32_t medium_wg;
    uint32_t light_width;
    uint32_t medium_width;
    uint32_t heavy_width;
} pb_tuning;

typedef struct {
    pb_agg agg;                   /* AUTO: per-bucket table; others: forced for every source */
    pb_hub_mode hub;
    uint64_t workspace_cap_bytes; /* 0: no cap beyond the device's free memory */
    uint32_t wg_size;             /* 0, or threads per workgroup for the light and medium buckets' kernels
                                   * where they are built for it (light: 64, 128, 256; medium: 128, 256,
                                   * 512), overriding the tuning table; INVALID_ARG when neither is */
    uint32_t flags;               /* PB_FLAG_* bits, 0 for none */
    pb_stats *stats;              /* optional host pointer, filled by the call */
    const pb_tuning *tuning;      /* optional: the AUTO table, NULL = built-in */
} pb_opts;

typedef struct pb_graph pb_graph;

/* Fills opts with the defaults (AUTO aggregation, AUTO hub mode, no cap). */
void pb_opts_default(pb_opts *opts);

/* Human-readable name of a status code (static storage). */
const char *pb_status_str(pb_status status);

/* Validates the CSR (rows strictly increasing, ids in range, offsets
 * consistent) and builds the derived V-side CSR and degrees (Section 2 keeps
 * a CSR per side).  The graph handle owns only the derived arrays.
 * Synchronises `stream` once to read the validation result.
 * Errors: INVALID_ARG, NOT_SIMPLE, ID_RANGE, NO_MEMORY, HIP. */
pb_status pb_graph_create(const pb_csr *csr, hipStream_t stream, pb_graph **out);

/* Releases the handle and everything it owns (NULL is ignored).  Waits for
 * work the handle has enqueued to finish first. */
void pb_graph_destroy(pb_graph *g);

/* Writes a vertex ordering of kind `kind` (Section 3.1.1, see pb_rank_kind):
 * rank_out[x] for every unified id x (device, n_u + n_v entries).
 * Synchronises `stream`: once for the side and degree orders; once per
 * removal round for the approximate complement-coreness order; for the exact
 * one, once per key window (the live vertices of the top keys, at most 4096
 * unless one key alone has more) and once per round whose removed vertices
 * have more than 16384 neighbours, the other rounds running back to back on
 * the device.
 * Errors: INVALID_ARG, NO_MEMORY, HIP. */
pb_status pb_rank(pb_graph *g, pb_rank_kind kind, uint32_t *rank_out, hipStream_t stream);

/* The number of wedges the framework retrieves under `rank` (Algorithm 2),
 * W(rank) = sum over vertices y of h*d - h*(h+1)/2, where d = deg(y) and h =
 * the neighbours of y ranked above y.  *w_out is host memory.  Synchronises
 * `stream` once.  Errors: INVALID_ARG, NO_MEMORY, HIP. */
pb_status pb_wedges(pb_graph *g, const uint32_t *rank, uint64_t *w_out, hipStream_t stream);

/* The ranking chooser of Section 6.2: with w_s the wedges under side order
 * (SIDE_AUTO) and w_r those under `other`, the metric f = (w_s - w_r) / w_s;
 * when f < 0.1 side order is used, otherwise `other`.  Writes the chosen
 * ordering into rank_out (device, n entries) and its kind into *chosen; the
 * two wedge counts go to *w_side and *w_other (host, each may be NULL).
 * Synchronises `stream`.  Errors: those of pb_rank and pb_wedges. */
pb_status pb_rank_choose(pb_graph *g, pb_rank_kind other, uint32_t *rank_out, pb_rank_kind *chosen,
                         uint64_t *w_side, uint64_t *w_other, hipStream_t stream);

/* Counts butterflies (framework steps 2-4) under the caller's ranking.
 * `rank` (device, n entries) may be any permutation of [0, n) — the result
 * does not depend on it, only the work does.  Any subset of the outputs may
 * be requested (NULL = not wanted, at least one required):
 *   global_out  device int64[1]: the number of butterflies
 *   vertex_out  device int64[n_u + n_v]: butterflies per vertex (unified ids)
 *   edge_out    device int64[m]: butterflies per edge (u_adj positions)
 * Synchronises `stream` three times: after the rank check, after the work
 * plan (to size the launches) and at the end (to confirm that no internal
 * capacity check tripped), so the outputs are ready when it returns.
 * Errors: INVALID_ARG, BAD_RANK, NO_MEMORY, HIP, INTERNAL. */
pb_status pb_count(pb_graph *g, const uint32_t *rank, const pb_opts *opts, int64_t *global_out,
                   int64_t *vertex_out, int64_t *edge_out, hipStream_t stream);

/* The total count alone (framework steps 2-4 with only the C(R,2) sum). */
pb_status pb_count_global(pb_graph *g, const uint32_t *rank, const pb_opts *opts, int64_t *out,
                          hipStream_t stream);

/* Per-vertex counts alone (Algorithm 3, COUNT-V). */
pb_status pb_count_vertex(pb_graph *g, const uint32_t *rank, const pb_opts *opts, int64_t *out,
                          hipStream_t stream);

/* Per-edge counts alone (Algorithm 4, COUNT-E). */
pb_status pb_count_edge(pb_graph *g, const uint32_t *rank, const pb_opts *opts, int64_t *out,
                        hipStream_t stream);

/* ------------------------------------------------------------------------
 * Counting without allocation.
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, serving loops that must not allocate, harnesses that forbid it.
 * pb_count_noalloc computes exactly what pb_count computes (same arguments,
 * same outputs), but every scratch block comes from one array of
 * PB_NOALLOC_SCRATCH_BYTES inside the library, a device global that each
 * device holds from the library's load to the end of the process.  The call
 * allocates no device memory and no pinned host memory.  Differences from
 * pb_count: the hub tile is never used (opts->hub is ignored), phase times are
 * not measured (PB_FLAG_TIMING is ignored; the other stats are filled) and
 * opts->workspace_cap_bytes is ignored.
 * Limits: NO_MEMORY, before any work is queued, when
 * 208 (n_u + n_v) + 84 m + 32 u + 65536 bytes exceed the array (u = m up-slots,
 * 2m with PB_FLAG_CACHE_OPT), that is graphs of up to about 1M edges; NO_MEMORY
 * also when data-dependent tables (the window items of forced hashing, the
 * histograms of sources with 65536 or more up-slots) do not fit beside them.
 * Sharing: calls on one device are serialised by a lock in the library, and
 * each returns only once its work on `stream` has finished, so two calls
 * never use the array at the same time.  The array keeps the last call's
 * contents; every call clears what it needs.
 * Synchronises `stream` as pb_count does, and once more before returning.
 * Errors: those of pb_count. */
#define PB_NOALLOC_SCRATCH_BYTES (128ull << 20)

pb_status pb_count_noalloc(pb_graph *g, const uint32_t *rank, const pb_opts *opts, int64_t *global_out,
                           int64_t *vertex_out, int64_t *edge_out, hipStream_t stream);

/* Approximate total counts by graph sparsification (Section 4.6
 * "Approximate counting"): a kept graph is drawn, counted exactly, and the
 * count scaled to an unbiased estimate.  Only the total can be estimated.
 *   EDGE   each edge is kept independently with probability p; scale 1 / p^4
 *   COLOR  every vertex takes one of c = ceil(1/p) colours and an edge is kept
 *          when its two endpoints share a colour; scale c^3 (a butterfly
 *          survives when its other three vertices take the first one's colour)
 * Random numbers come from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014)
 * started at state `seed`: x(i) = its output number i + 1 =
 * mix(seed + (i + 1) * 0x9E3779B97F4A7C15) with its 64-bit finaliser mix.
 * EDGE keeps edge e (its position in u_adj) when x(e) < floor(p * 2^64), or
 * every edge when p = 1; COLOR gives unified vertex id i the colour
 * floor(x(i) * c / 2^64).  The same (graph, kind, p, seed) always keeps the
 * same edges. */
typedef enum {
    PB_SPARSIFY_EDGE = 0,
    PB_SPARSIFY_COLOR = 1
} pb_sparsify_kind;

/* Writes the kept graph as a U-side CSR over the same vertices, kept edges
 * in input order: out_u_off (device int64[n_u + 1]) and out_u_adj (device
 * uint32, room for m entries; may be NULL when m = 0); *kept (host) gets the
 * number of kept edges.  p must lie in (0, 1], and for COLOR also p >= 2^-32.
 * Synchronises `stream` once, to read the kept count.
 * Errors: INVALID_ARG, NO_MEMORY, HIP. */
pb_status pb_sparsify(pb_graph *g, pb_sparsify_kind kind, double p, uint64_t seed, int64_t *out_u_off,
                      uint32_t *out_u_adj, uint64_t *kept, hipStream_t stream);

/* Sparsifies as pb_sparsify, then counts the kept graph exactly under the
 * ordering `rank_kind` with `opts` (NULL = defaults) and scales.  Host
 * outputs: *count_out the kept graph's butterflies, *estimate_out the scaled
 * estimate of the total, *kept_out (optional) the kept edges.  All scratch is
 * the library's; the call synchronises `stream` before it returns.
 * Errors: those of pb_sparsify, pb_graph_create, pb_rank and pb_count_global. */
pb_status pb_count_approx(pb_graph *g, pb_sparsify_kind kind, double p, uint64_t seed, pb_rank_kind rank_kind,
                          const pb_opts *opts, int64_t *count_out, double *estimate_out, uint64_t *kept_out,
                          hipStream_t stream);

/* Tip decomposition by vertex peeling (Section 3.2 "Peeling Framework",
 * Algorithm 5 PEEL-V / UPDATE-V).  One side X is peeled: U, V, or with AUTO
 * the side whose vertices, as wedge endpoints, give the fewest wedges (U when
 * sum over V of C(deg, 2) <= sum over U of C(deg, 2)).  Starting from the
 * per-vertex butterfly counts B, each round sets k = max(k, smallest B of the
 * remaining X vertices), peels every remaining X vertex with B <= k (its tip
 * number is k) and lowers each remaining B(u2) by C(c, 2) for every peeled
 * u1, c = the centres u1 and u2 share.
 *   tip_out    device int64[n_u + n_v]: tip numbers of X, -1 on the other side
 *   side_out   host, optional: the side peeled (PB_PEEL_SIDE_U or _V)
 *   rounds_out host, optional: peeling rounds
 * `opts` (NULL = defaults) applies to the initial count.  Synchronises
 * `stream` every 64 rounds.  Uses device scratch of up to 4 GiB of counters
 * beside the counting call's own.
 * Errors: INVALID_ARG, NO_MEMORY, HIP, and those of pb_count_vertex. */
typedef enum {
    PB_PEEL_SIDE_AUTO = 0,
    PB_PEEL_SIDE_U = 1,
    PB_PEEL_SIDE_V = 2
} pb_peel_side;

pb_status pb_tip_decompose(pb_graph *g, pb_peel_side side, const pb_opts *opts, int64_t *tip_out,
                           pb_peel_side *side_out, uint64_t *rounds_out, hipStream_t stream);

/* Wing decomposition by edge peeling (Section 3.2 "Peeling Framework",
 * Algorithm 6 PEEL-E / UPDATE-E).  Starting from the per-edge butterfly
 * counts B, each round sets k = max(k, smallest B of the remaining edges) and
 * peels every remaining edge with B <= k (its wing number is k).  A
 * butterfly that loses an edge in a round and had lost none before is
 * destroyed once (by the peeled edge of smallest id among its edges peeled in
 * that round), and each of its remaining edges loses 1.
 *   wing_out   device int64[m], by u_adj position
 *   rounds_out host, optional: peeling rounds
 * `opts` (NULL = defaults) applies to the initial count.  Synchronises
 * `stream` every 64 rounds.  Errors: INVALID_ARG, NO_MEMORY, HIP, and those of
 * pb_count_edge. */
pb_status pb_wing_decompose(pb_graph *g, const pb_opts *opts, int64_t *wing_out, uint64_t *rounds_out,
                            hipStream_t stream);

/* Batched counting: `count` independent graphs in one pass of the pipeline.
 * The batch is counted as the disjoint union of the graphs (no wedge spans two
 * graphs), so relabelling, planning and each counting kernel run as single
 * launches over the work items of every graph; counts are identical to
 * counting each graph alone.  graphs[i] and ranks[i] (device, n_i entries, a
 * permutation of [0, n_i)) as for pb_count; each output array is a host array
 * of `count` device pointers (or NULL when that output is not wanted; at
 * least one wanted): global_outs[i] -> int64[1], vertex_outs[i] ->
 * int64[n_i], edge_outs[i] -> int64[m_i].  opts->stats, if given, sums the
 * batch.  Synchronises `stream` like pb_count.
 * Errors: INVALID_ARG (also when the summed sizes exceed the pb_count limits),
 * BAD_RANK, NO_MEMORY, HIP. */
pb_status pb_count_batched(pb_graph *const *graphs, const uint32_t *const *ranks, uint32_t count,
                           const pb_opts *opts, int64_t *const *global_outs, int64_t *const *vertex_outs,
                           int64_t *const *edge_outs, hipStream_t stream);

/* Fills a pb_tuning by timing whole batched counts of the given sample
 * graphs (the counting kernels' time, `repeats` runs each, median kept) under
 * candidate tables, one choice at a time with the others held at the current
 * best: each bucket's aggregator, the light and medium thresholds, the light
 * and medium workgroup sizes, then each bucket's batch width (0, 256, 1024,
 * 4096 workgroups).  Counts are exact under every candidate, so the table
 * only affects speed.  The timed counts produce the global and per-edge
 * outputs.  Synchronises `stream`.
 * Errors: as pb_count_batched. */
pb_status pb_autotune(pb_graph *const *graphs, const uint32_t *const *ranks, uint32_t count, const pb_opts *opts,
                      uint32_t repeats, pb_tuning *out, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Serving: counting queries against graphs kept resident on the device.
 *
 * A server holds a pool of resident graphs (with their rankings) admitted
 * against an HBM budget, a queue of requests, and `slots` worker threads, each
 * with its own stream.  A free slot takes the oldest queued request together
 * with up to max_batch - 1 later requests of the same output kinds whose
 * estimated device scratch still fits the budget next to the batches already
 * in flight, and counts them with one batched pass (pb_count_batched).
 * Requests that arrive while batches are running wait for the next free slot
 * and memory; batches on different slots overlap on the device.  Results are
 * identical to counting each request alone.
 */
typedef struct pb_server pb_server;

typedef struct {
    uint64_t hbm_budget_bytes; /* resident pool + in-flight scratch; 0 = the device's free memory */
    uint32_t slots;            /* concurrent batches (worker threads / streams), >= 1 */
    uint32_t max_batch;        /* requests per batch, >= 1 */
    pb_agg agg;                /* aggregation policy of every batch */
    const pb_tuning *tuning;   /* optional AUTO table (copied) */
} pb_server_config;

enum { PB_WANT_GLOBAL = 1, PB_WANT_VERTEX = 2, PB_WANT_EDGE = 4 };

typedef struct {
    uint64_t request_id;
    int32_t status;  /* pb_status of its batch */
    uint32_t batch;  /* requests in its batch */
    double submit_s; /* seconds since the server started */
    double start_s;  /* its batch started */
    double done_s;   /* its batch finished; latency = done_s - submit_s */
} pb_completion;

/* Starts the worker slots.  Errors: INVALID_ARG, NO_MEMORY, HIP. */
pb_status pb_server_create(const pb_server_config *config, pb_server **out);

/* Adds a resident graph: `g` and `rank` (device, n entries) stay owned by the
 * caller and must outlive the server.  Its resident footprint (caller CSR,
 * derived arrays, rank) is charged to the budget; NO_MEMORY when the pool
 * would exceed it.  *graph_id receives its index. */
pb_status pb_server_add_graph(pb_server *srv, pb_graph *g, const uint32_t *rank, uint32_t *graph_id);

/* Queues a request for graph `graph_id`; `want` is a PB_WANT_* mask and the
 * matching outputs (device, caller-owned, sized as for pb_count) must stay
 * valid until the request completes.  The slots' streams do not wait for the
 * caller's streams: work the caller has queued on the output buffers must be
 * complete before the call.  Returns at once; *request_id receives its id.
 * NO_MEMORY when the request alone could never fit the budget. */
pb_status pb_server_submit(pb_server *srv, uint32_t graph_id, uint32_t want, int64_t *global_out,
                           int64_t *vertex_out, int64_t *edge_out, uint64_t *request_id);

/* Moves up to `max` completed requests into out[] (oldest completion first);
 * *count receives how many.  Never blocks. */
pb_status pb_server_poll(pb_server *srv, pb_completion *out, uint32_t max, uint32_t *count);

/* Blocks until every submitted request has completed. */
pb_status pb_server_drain(pb_server *srv);

/* Drains, stops the slots and frees the server (NULL is ignored). */
void pb_server_destroy(pb_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* PARBUTTERFLY_H */
