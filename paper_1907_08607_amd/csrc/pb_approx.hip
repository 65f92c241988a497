// Approximate total counts by graph sparsification (Section 4.6
// "Approximate counting"): one filter pass over the edges draws the kept
// graph, a scan and a compaction lay it out as a U-side CSR, and the exact
// pipeline counts it.  The estimate is the kept graph's count times 1/p^4
// (edge sparsification) or c^3 (colorful sparsification with c colours).
#include "pb_internal.h"

#include <cmath>

using namespace pb;

namespace {

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output number i + 1 of the
// generator started at state `seed`, i.e. its finaliser applied to
// seed + (i + 1) * gamma.  A counter-based draw: any element's number is
// computed on its own.
__device__ inline uint64_t splitmix(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct Keep {
    uint64_t seed;
    uint64_t thr;      // edge sparsification: keep edge e when x(e) < thr
    uint64_t colours;  // colorful: c
    uint32_t n_u;
    int kind;
    bool all;  // p = 1: every edge
};

// flag[e] = 1 when edge e is kept
__global__ void k_keep(Keep K, const uint32_t *eu, const uint32_t *u_adj, uint64_t m, uint32_t *flag) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x) {
        bool keep;
        if (K.all) {
            keep = true;
        } else if (K.kind == PB_SPARSIFY_EDGE) {
            keep = splitmix(K.seed, e) < K.thr;
        } else {
            // colour of unified id i: floor(x(i) * c / 2^64)
            const uint64_t cu = __umul64hi(splitmix(K.seed, eu[e]), K.colours);
            const uint64_t cv = __umul64hi(splitmix(K.seed, (uint64_t)K.n_u + u_adj[e]), K.colours);
            keep = cu == cv;
        }
        flag[e] = keep ? 1u : 0u;
    }
}

// kept edge e goes to position pos[e] (exclusive scan of the flags)
__global__ void k_kept_adj(const uint32_t *u_adj, const uint32_t *flag, const uint32_t *pos, uint64_t m,
                           uint32_t *out_adj) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x)
        if (flag[e]) out_adj[pos[e]] = u_adj[e];
}

// row u of the kept graph starts where the kept edges before u_off[u] end
__global__ void k_kept_off(const int64_t *u_off, const uint32_t *pos, uint64_t rows, int64_t *out_off) {
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < rows; u += (uint64_t)gridDim.x * blockDim.x)
        out_off[u] = pos[u_off[u]];
}

uint32_t grid_of(uint64_t n) {
    const uint64_t g = (n + 255) / 256;
    return (uint32_t)(g == 0 ? 1 : g > 65536 ? 65536 : g);
}

pb_status check_args(const pb_graph *g, pb_sparsify_kind kind, double p) {
    if (!g) return PB_ERR_INVALID_ARG;
    if (kind != PB_SPARSIFY_EDGE && kind != PB_SPARSIFY_COLOR) return PB_ERR_INVALID_ARG;
    if (!(p > 0.0) || !(p <= 1.0)) return PB_ERR_INVALID_ARG;  // also NaN
    if (kind == PB_SPARSIFY_COLOR && p < std::ldexp(1.0, -32)) return PB_ERR_INVALID_ARG;
    return PB_OK;
}

pb_status sparsify_impl(pb_graph *g, pb_sparsify_kind kind, double p, uint64_t seed, int64_t *out_off,
                        uint32_t *out_adj, uint64_t *kept, hipStream_t s) {
    PB_TRY(check_args(g, kind, p));
    if (!out_off || !kept || (g->m && !out_adj)) return PB_ERR_INVALID_ARG;
    const bool all = p >= 1.0;
    const Keep K{seed, all ? 0ull : (uint64_t)std::ldexp(p, 64), all ? 1ull : (uint64_t)std::ceil(1.0 / p), g->n_u,
                 (int)kind, all};
    const uint64_t m = g->m;
    Workspace ws(s, 0);
    uint32_t *flag = ws.alloc<uint32_t>(m);
    uint32_t *pos = ws.alloc<uint32_t>(m + 1);
    if (ws.failed) return PB_ERR_NO_MEMORY;
    if (m) {
        hipLaunchKernelGGL(k_keep, dim3(grid_of(m)), dim3(256), 0, s, K, (const uint32_t *)g->eu, g->u_adj, m, flag);
        PB_TRY_HIP(hipGetLastError());
        PB_TRY((scan_exclusive<uint32_t, uint32_t>(flag, pos, m, pos + m, ws)));
        hipLaunchKernelGGL(k_kept_adj, dim3(grid_of(m)), dim3(256), 0, s, g->u_adj, (const uint32_t *)flag,
                           (const uint32_t *)pos, m, out_adj);
        PB_TRY_HIP(hipGetLastError());
    } else {
        PB_TRY(fill<uint32_t>(pos, 0u, 1, s));
    }
    hipLaunchKernelGGL(k_kept_off, dim3(grid_of((uint64_t)g->n_u + 1)), dim3(256), 0, s, g->u_off,
                       (const uint32_t *)pos, (uint64_t)g->n_u + 1, out_off);
    PB_TRY_HIP(hipGetLastError());
    uint32_t k = 0;
    PB_TRY_HIP(hipMemcpyAsync(&k, pos + m, sizeof(k), hipMemcpyDeviceToHost, s));
    PB_TRY_HIP(hipStreamSynchronize(s));
    *kept = k;
    return PB_OK;
}

struct GraphHolder {
    pb_graph *h = nullptr;
    ~GraphHolder() { pb_graph_destroy(h); }
};

}  // namespace

extern "C" {

pb_status pb_sparsify(pb_graph *g, pb_sparsify_kind kind, double p, uint64_t seed, int64_t *out_u_off,
                      uint32_t *out_u_adj, uint64_t *kept, hipStream_t stream) {
    return sparsify_impl(g, kind, p, seed, out_u_off, out_u_adj, kept, stream);
}

pb_status pb_count_approx(pb_graph *g, pb_sparsify_kind kind, double p, uint64_t seed, pb_rank_kind rank_kind,
                          const pb_opts *opts, int64_t *count_out, double *estimate_out, uint64_t *kept_out,
                          hipStream_t stream) {
    PB_TRY(check_args(g, kind, p));
    if (!count_out || !estimate_out) return PB_ERR_INVALID_ARG;
    const uint64_t n = (uint64_t)g->n_u + g->n_v;
    pb_status st = PB_OK;
    int64_t count = 0;
    uint64_t kept = 0;
    {
        Workspace ws(stream, 0);
        int64_t *off = ws.alloc<int64_t>((uint64_t)g->n_u + 1);
        uint32_t *adj = ws.alloc<uint32_t>(g->m);
        uint32_t *rank = ws.alloc<uint32_t>(n);
        int64_t *gout = ws.alloc<int64_t>(1);
        if (ws.failed) return PB_ERR_NO_MEMORY;
        PB_TRY(sparsify_impl(g, kind, p, seed, off, adj, &kept, stream));
        GraphHolder kg;
        const pb_csr csr{g->n_u, g->n_v, kept, off, kept ? adj : nullptr};
        PB_TRY(pb_graph_create(&csr, stream, &kg.h));
        PB_TRY(pb_rank(kg.h, rank_kind, rank, stream));
        st = pb_count_global(kg.h, rank, opts, gout, stream);
        if (st != PB_OK) return st;
        PB_TRY_HIP(hipMemcpyAsync(&count, gout, sizeof(count), hipMemcpyDeviceToHost, stream));
        PB_TRY_HIP(hipStreamSynchronize(stream));
    }
    double scale = 1.0;
    if (p < 1.0) {
        if (kind == PB_SPARSIFY_EDGE) {
            scale = 1.0 / (p * p * p * p);
        } else {
            const double c = std::ceil(1.0 / p);
            scale = c * c * c;
        }
    }
    *count_out = count;
    *estimate_out = (double)count * scale;
    if (kept_out) *kept_out = kept;
    return PB_OK;
}

}  // extern "C"
