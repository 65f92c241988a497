// Tip decomposition by vertex peeling (Section 3.2 "Peeling Framework",
// Algorithm 5 PEEL-V / UPDATE-V), level-synchronous on the device.
//
// One side X is peeled.  B starts as the per-vertex butterfly counts (the
// counting path).  Each round sets k = max(k, the smallest B among the
// remaining X vertices), peels every remaining X vertex with B <= k (tip
// number k) and runs UPDATE-V: for each peeled u1 and each remaining u2 the
// two share c centres, and the C(c, 2) butterflies through u1 leave B(u2).
//
// UPDATE-V gives each peeled vertex to one workgroup, which walks its 2-hop
// neighbourhood twice over a private dense counter slice of |X| words.  The
// 2-hop entries are taken as one flat sequence, 1024 neighbour lists at a
// time (a block scan of their lengths, then each thread finds its list by
// binary search), so a vertex with long lists spreads over all the threads.
// The first walk counts c(u1, u2) with atomic adds, the second takes each
// count with an atomic exchange (which also clears the slice for the next
// vertex) and subtracts C(c, 2) from B(u2) once per u2.  Most rounds peel one
// or a few vertices, which would leave all but a few workgroups idle; a round
// of at most PEEL_FEW vertices is instead spread over the whole GPU, one
// neighbour list of the 2-hop walk per wave, its two walks in two launches.
//
// The round state (k, the round's minimum, vertices left, rounds) stays on
// the device, so rounds are queued in batches with one host synchronisation
// per batch; a round with no vertex left does nothing.
#include "pb_internal.h"

using namespace pb;

namespace {

constexpr uint32_t PEEL_T = 1024;                      // threads per workgroup in the update
constexpr uint32_t PEEL_MAX_GRID = 256;                // update workgroups (counter slices) at most
constexpr uint64_t PEEL_SCRATCH = uint64_t(1) << 32;  // bytes of counter slices at most
constexpr uint32_t PEEL_BATCH = 64;                    // rounds queued per host synchronisation
constexpr uint32_t PEEL_FEW = 8;                       // rounds of at most this many vertices spread over the GPU
constexpr uint32_t SPREAD_GRID = 2048;                 // workgroups of the spread update (256 threads each)

struct PeelState {
    int64_t k;                 // the level reached by the previous rounds
    unsigned long long mn;     // this round's smallest B (~0: none left)
    unsigned long long left;   // vertices (or edges) not yet peeled
    unsigned long long rounds; // rounds that peeled something
    unsigned long long rid;    // edge peeling: id of the current round (1, 2, ...)
};

struct Side {
    // X vertices are unified ids base .. base + nx - 1.  Their lists (ids on
    // the other side, local) and the other side's lists (local X ids).
    const int64_t *xoff64;  // U-CSR row offsets when X = U
    const uint32_t *xoff32; // V-CSR row offsets when X = V
    const uint32_t *xadj;
    const int64_t *yoff64;
    const uint32_t *yoff32;
    const uint32_t *yadj;
    uint32_t base, nx;
    __device__ uint64_t xb(uint32_t x) const { return xoff64 ? (uint64_t)xoff64[x] : xoff32[x]; }
    __device__ uint64_t yb(uint32_t y) const { return yoff64 ? (uint64_t)yoff64[y] : yoff32[y]; }
};

// smallest B among remaining X vertices into *best (which starts at ~0: none left)
__global__ __launch_bounds__(256) void k_peel_min(const int64_t *b, const uint32_t *gone, uint32_t nx,
                                                  unsigned long long *best) {
    __shared__ unsigned long long tmp[256 / WAVE];
    unsigned long long mn = ~0ull;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < nx; x += gridDim.x * blockDim.x)
        if (!gone[x]) {
            const unsigned long long v = (unsigned long long)b[x];
            mn = v < mn ? v : mn;
        }
    for (int s = WAVE / 2; s >= 1; s >>= 1) {
        const unsigned long long o = __shfl_xor(mn, s, WAVE);
        mn = o < mn ? o : mn;
    }
    if ((threadIdx.x & (WAVE - 1)) == 0) tmp[threadIdx.x / WAVE] = mn;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 256 / WAVE; ++i) mn = tmp[i] < mn ? tmp[i] : mn;
        if (mn != ~0ull) atomicMin(best, mn);
    }
}

// this round's level: max(k, the round's minimum)
__device__ inline int64_t round_k(const PeelState *st) {
    const unsigned long long mn = st->mn;
    return mn != ~0ull && (int64_t)mn > st->k ? (int64_t)mn : st->k;
}

// the round's peeled vertices (B <= k among the remaining ones): tip number
// k, and appended to front[] (in no particular order; the update does not
// depend on it) with one counter atomic per wave
__global__ void k_peel_take(const int64_t *b, uint32_t nx, uint32_t base, const PeelState *st, uint32_t *gone,
                            uint32_t *front, uint32_t *nfront, int64_t *tip) {
    const int64_t k = round_k(st);
    const uint32_t lane = threadIdx.x & (WAVE - 1);
    for (uint32_t x0 = blockIdx.x * blockDim.x; x0 < nx; x0 += gridDim.x * blockDim.x) {
        const uint32_t x = x0 + threadIdx.x;
        const bool take = x < nx && !gone[x] && b[x] <= k;
        const uint64_t mask = __ballot(take);
        if (mask == 0) continue;
        const uint32_t leader = (uint32_t)__ffsll((unsigned long long)mask) - 1;
        uint32_t at = 0;
        if (lane == leader) at = atomicAdd(nfront, (uint32_t)__popcll(mask));
        at = __shfl(at, (int)leader, WAVE);
        if (take) {
            front[at + (uint32_t)__popcll(mask & lanemask_lt())] = x;
            gone[x] = 1;
            tip[base + x] = k;
        }
    }
}

// closes a round (one thread): k advances, the peeled vertices leave `left`,
// and the next round's minimum starts empty
__global__ void k_peel_close(uint32_t *nfront, PeelState *st) {
    const uint32_t nf = *nfront;
    st->k = round_k(st);
    st->left -= nf;
    st->rounds += nf ? 1 : 0;
    st->mn = ~0ull;
    *nfront = 0;
}

// UPDATE-V: one workgroup per peeled vertex (see the file comment).  `cnt`
// holds gridDim.x slices of nx words, all zero on entry and on exit.
__global__ __launch_bounds__(PEEL_T) void k_peel_update(Side S, const uint32_t *front, const uint32_t *nfront,
                                                        const uint32_t *gone, uint32_t few, uint32_t *cnt, int64_t *b) {
    __shared__ uint32_t s_off[PEEL_T];  // flat start of each list of the chunk
    __shared__ uint32_t s_y0[PEEL_T];   // first entry of each list
    __shared__ uint32_t s_tmp[PEEL_T / WAVE + 1];
    const uint32_t t = threadIdx.x;
    uint32_t *c = cnt + (uint64_t)blockIdx.x * S.nx;
    const uint32_t nf = *nfront;
    if (nf <= few) return;  // k_peel_spread takes the round
    for (uint32_t i = blockIdx.x; i < nf; i += gridDim.x) {
        const uint32_t u1 = front[i];
        const uint64_t p0 = S.xb(u1), p1 = S.xb(u1 + 1);
        for (int pass = 1; pass <= 2; ++pass) {
            for (uint64_t pc = p0; pc < p1; pc += PEEL_T) {
                const uint64_t p = pc + t;
                uint32_t len = 0, y0 = 0;
                if (p < p1) {
                    const uint32_t y = S.xadj[p];
                    y0 = (uint32_t)S.yb(y);
                    len = (uint32_t)(S.yb(y + 1) - y0);
                }
                uint32_t total;
                const uint32_t off = block_exclusive_sum<PEEL_T>(len, s_tmp, &total);
                s_off[t] = off;
                s_y0[t] = y0;
                __syncthreads();
                const uint32_t nl = p1 - pc < PEEL_T ? (uint32_t)(p1 - pc) : PEEL_T;
                for (uint32_t f = t; f < total; f += PEEL_T) {
                    uint32_t lo = 0, hi = nl;  // largest j < nl with s_off[j] <= f
                    while (hi - lo > 1) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (s_off[mid] <= f) lo = mid; else hi = mid;
                    }
                    const uint32_t u2 = S.yadj[s_y0[lo] + (f - s_off[lo])];
                    if (gone[u2]) continue;
                    if (pass == 1) {
                        atomicAdd(&c[u2], 1u);
                    } else {
                        const uint32_t cc = atomicExch(&c[u2], 0u);
                        if (cc >= 2) {
                            const unsigned long long tt = (unsigned long long)cc * (cc - 1) / 2;
                            atomicAdd(reinterpret_cast<unsigned long long *>(&b[u2]), 0ull - tt);
                        }
                    }
                }
                __syncthreads();  // s_off / s_y0 are refilled by the next chunk; pass 2 follows pass 1
            }
        }
    }
}

// UPDATE-V for a round of at most `few` peeled vertices, spread over the
// whole GPU: peeled vertex i keeps its own counter slice, and every wave takes
// one neighbour y of a peeled vertex at a time and walks N(y) with its lanes.
// PASS 1 counts c(u1, u2); PASS 2 (a launch of its own, after all of PASS 1)
// takes each count with an atomic exchange and subtracts C(c, 2) from B(u2).
template <int PASS>
__global__ __launch_bounds__(256) void k_peel_spread(Side S, const uint32_t *front, const uint32_t *nfront,
                                                     const uint32_t *gone, uint32_t few, uint32_t *cnt, int64_t *b) {
    const uint32_t nf = *nfront;
    if (nf == 0 || nf > few) return;
    // first-level entries of the peeled vertices, laid end to end
    uint64_t start[PEEL_FEW], end[PEEL_FEW], first[PEEL_FEW + 1];
    first[0] = 0;
#pragma unroll
    for (uint32_t i = 0; i < PEEL_FEW; ++i) {
        start[i] = i < nf ? S.xb(front[i]) : 0;
        end[i] = i < nf ? S.xb(front[i] + 1) : 0;
        first[i + 1] = first[i] + (end[i] - start[i]);
    }
    const uint64_t items = first[PEEL_FEW];
    const uint32_t lane = threadIdx.x & (WAVE - 1);
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / WAVE);
    for (uint64_t t = (uint64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; t < items; t += waves) {
        uint32_t i = 0;
#pragma unroll
        for (uint32_t j = 1; j < PEEL_FEW; ++j)
            if (first[j] <= t) i = j;
        uint32_t *c = cnt + (uint64_t)i * S.nx;
        const uint32_t y = S.xadj[start[i] + (t - first[i])];
        const uint64_t y0 = S.yb(y), y1 = S.yb(y + 1);
        for (uint64_t q = y0 + lane; q < y1; q += WAVE) {
            const uint32_t u2 = S.yadj[q];
            if (gone[u2]) continue;
            if (PASS == 1) {
                atomicAdd(&c[u2], 1u);
            } else {
                const uint32_t cc = atomicExch(&c[u2], 0u);
                if (cc >= 2) {
                    const unsigned long long tt = (unsigned long long)cc * (cc - 1) / 2;
                    atomicAdd(reinterpret_cast<unsigned long long *>(&b[u2]), 0ull - tt);
                }
            }
        }
    }
}

// tip = -1 everywhere; B = the X side's per-vertex counts
__global__ void k_peel_init(const int64_t *vcount, uint32_t base, uint32_t nx, uint64_t n, int64_t *tip,
                            int64_t *b) {
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (uint64_t)gridDim.x * blockDim.x) {
        tip[x] = -1;
        if (x >= base && x - base < nx) b[x - base] = vcount[x];
    }
}

// wedges with endpoints on U (centres on V) and with endpoints on V
__global__ __launch_bounds__(256) void k_side_wedges(const uint32_t *deg, uint32_t n_u, uint64_t n,
                                                     unsigned long long *sums) {
    __shared__ unsigned long long tmp[256 / WAVE];
    unsigned long long su = 0, sv = 0;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (uint64_t)gridDim.x * blockDim.x) {
        const unsigned long long d = deg[x], w = d * (d - (d ? 1 : 0)) / 2;
        if (x < n_u) sv += w; else su += w;
    }
    su = block_sum<256>(su, tmp);
    sv = block_sum<256>(sv, tmp);
    if (threadIdx.x == 0) {
        if (su) atomicAdd(&sums[0], su);
        if (sv) atomicAdd(&sums[1], sv);
    }
}

uint32_t grid_of(uint64_t n, uint32_t cap) {
    const uint64_t g = (n + 255) / 256;
    return (uint32_t)(g == 0 ? 1 : g > cap ? cap : g);
}

struct HostBuf {
    void *p = nullptr;
    ~HostBuf() { if (p) (void)hipHostFree(p); }
};

pb_status peel_impl(pb_graph *g, pb_peel_side side, const pb_opts *opts, int64_t *tip, pb_peel_side *side_out,
                    uint64_t *rounds_out, hipStream_t s) {
    if (!g || !tip) return PB_ERR_INVALID_ARG;
    if ((int)side < PB_PEEL_SIDE_AUTO || (int)side > PB_PEEL_SIDE_V) return PB_ERR_INVALID_ARG;
    const uint64_t n = (uint64_t)g->n_u + g->n_v;
    if (n == 0) {
        if (side_out) *side_out = side == PB_PEEL_SIDE_V ? PB_PEEL_SIDE_V : PB_PEEL_SIDE_U;
        if (rounds_out) *rounds_out = 0;
        return PB_OK;
    }
    Workspace ws(s, 0);
    HostBuf hb;
    PB_TRY_HIP(hipHostMalloc(&hb.p, 64, hipHostMallocDefault));
    unsigned long long *h = static_cast<unsigned long long *>(hb.p);
    unsigned long long *dsum = ws.alloc<unsigned long long>(4);
    if (ws.failed) return PB_ERR_NO_MEMORY;
    if (side == PB_PEEL_SIDE_AUTO) {
        PB_TRY(fill<uint64_t>((uint64_t *)dsum, 0ull, 2, s));
        hipLaunchKernelGGL(k_side_wedges, dim3(grid_of(n, 1024)), dim3(256), 0, s, (const uint32_t *)g->deg, g->n_u, n,
                           dsum);
        PB_TRY_HIP(hipGetLastError());
        PB_TRY_HIP(hipMemcpyAsync(h, dsum, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        PB_TRY_HIP(hipStreamSynchronize(s));
        side = h[0] <= h[1] ? PB_PEEL_SIDE_U : PB_PEEL_SIDE_V;
    }
    const bool on_u = side == PB_PEEL_SIDE_U;
    Side S{};
    S.base = on_u ? 0u : g->n_u;
    S.nx = on_u ? g->n_u : g->n_v;
    if (on_u) {
        S.xoff64 = g->u_off; S.xadj = g->u_adj; S.yoff32 = g->v_off; S.yadj = g->v_adj;
    } else {
        S.xoff32 = g->v_off; S.xadj = g->v_adj; S.yoff64 = g->u_off; S.yadj = g->u_adj;
    }
    // per-vertex butterfly counts under degree order (the counts do not depend on it)
    uint32_t *rank = ws.alloc<uint32_t>(n);
    int64_t *vcount = ws.alloc<int64_t>(n);
    if (ws.failed) return PB_ERR_NO_MEMORY;
    PB_TRY(pb_rank(g, PB_RANK_DEGREE, rank, s));
    PB_TRY(pb_count_vertex(g, rank, opts, vcount, s));
    ws.release(rank);
    const uint32_t nx = S.nx;
    int64_t *b = ws.alloc<int64_t>(nx);
    uint32_t *gone = ws.alloc<uint32_t>(nx), *nfront = ws.alloc<uint32_t>(1);
    uint32_t *front = ws.alloc<uint32_t>(nx);
    if (ws.failed) return PB_ERR_NO_MEMORY;
    hipLaunchKernelGGL(k_peel_init, dim3(grid_of(n, 65536)), dim3(256), 0, s, (const int64_t *)vcount, S.base, nx, n,
                       tip, b);
    PB_TRY_HIP(hipGetLastError());
    ws.release(vcount);
    uint64_t rounds = 0;
    if (nx) {
        // counter slices: one per update workgroup, as many as fit the scratch bound
        const uint64_t slice = (uint64_t)nx * sizeof(uint32_t);
        uint64_t grid = PEEL_SCRATCH / slice;
        grid = grid > PEEL_MAX_GRID ? PEEL_MAX_GRID : grid < 1 ? 1 : grid;
        const uint32_t ugrid = (uint32_t)grid;
        const uint32_t few = ugrid < PEEL_FEW ? ugrid : PEEL_FEW;  // spread rounds need one slice per vertex
        uint32_t *cnt = ws.alloc<uint32_t>((uint64_t)ugrid * nx);
        PeelState *st = ws.alloc<PeelState>(1);
        if (ws.failed) return PB_ERR_NO_MEMORY;
        PB_TRY(fill<uint32_t>(cnt, 0u, (uint64_t)ugrid * nx, s));
        PB_TRY(fill<uint32_t>(gone, 0u, nx, s));
        PB_TRY(fill<uint32_t>(nfront, 0u, 1, s));
        const PeelState st0{0, ~0ull, nx, 0, 1};
        PB_TRY_HIP(hipMemcpyAsync(st, &st0, sizeof(st0), hipMemcpyHostToDevice, s));
        PeelState *hst = static_cast<PeelState *>(hb.p);
        for (;;) {
            for (uint32_t r = 0; r < PEEL_BATCH; ++r) {
                hipLaunchKernelGGL(k_peel_min, dim3(grid_of(nx, 1024)), dim3(256), 0, s, (const int64_t *)b,
                                   (const uint32_t *)gone, nx, &st->mn);
                hipLaunchKernelGGL(k_peel_take, dim3(grid_of(nx, 65536)), dim3(256), 0, s, (const int64_t *)b, nx,
                                   S.base, (const PeelState *)st, gone, front, nfront, tip);
                hipLaunchKernelGGL(k_peel_update, dim3(ugrid), dim3(PEEL_T), 0, s, S, (const uint32_t *)front,
                                   (const uint32_t *)nfront, (const uint32_t *)gone, few, cnt, b);
                hipLaunchKernelGGL(k_peel_spread<1>, dim3(SPREAD_GRID), dim3(256), 0, s, S, (const uint32_t *)front,
                                   (const uint32_t *)nfront, (const uint32_t *)gone, few, cnt, b);
                hipLaunchKernelGGL(k_peel_spread<2>, dim3(SPREAD_GRID), dim3(256), 0, s, S, (const uint32_t *)front,
                                   (const uint32_t *)nfront, (const uint32_t *)gone, few, cnt, b);
                hipLaunchKernelGGL(k_peel_close, dim3(1), dim3(1), 0, s, nfront, st);
                PB_TRY_HIP(hipGetLastError());
            }
            PB_TRY_HIP(hipMemcpyAsync(hst, st, sizeof(PeelState), hipMemcpyDeviceToHost, s));
            PB_TRY_HIP(hipStreamSynchronize(s));
            if (hst->left == 0) break;
            if (hst->left > nx) return PB_ERR_INTERNAL;  // cannot happen: each round takes at most what is left
        }
        rounds = hst->rounds;
    }
    PB_TRY_HIP(hipStreamSynchronize(s));
    if (side_out) *side_out = side;
    if (rounds_out) *rounds_out = rounds;
    return PB_OK;
}

// ---------------------------------------------------------------- edge peeling

// Wing decomposition (Section 3.2, Algorithm 6 PEEL-E / UPDATE-E), rounds as
// for vertices.  state[e] is the round that peeled edge e (0: remaining).
// A butterfly that loses edges in round r and had lost none before is
// destroyed once: by the peeled edge of smallest id among its edges peeled in
// r, which lowers each of its remaining edges by 1.

__global__ __launch_bounds__(256) void k_wing_min(const int64_t *b, const uint32_t *state, uint64_t m,
                                                  unsigned long long *best) {
    __shared__ unsigned long long tmp[256 / WAVE];
    unsigned long long mn = ~0ull;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x)
        if (!state[e]) {
            const unsigned long long v = (unsigned long long)b[e];
            mn = v < mn ? v : mn;
        }
    for (int d = WAVE / 2; d >= 1; d >>= 1) {
        const unsigned long long o = __shfl_xor(mn, d, WAVE);
        mn = o < mn ? o : mn;
    }
    if ((threadIdx.x & (WAVE - 1)) == 0) tmp[threadIdx.x / WAVE] = mn;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 256 / WAVE; ++i) mn = tmp[i] < mn ? tmp[i] : mn;
        if (mn != ~0ull) atomicMin(best, mn);
    }
}

// the round's peeled edges (B <= k among the remaining ones): wing number k,
// state = this round, appended to front[] in no particular order (the update
// decides by edge id, not by position) with one counter atomic per wave
__global__ void k_wing_take(const int64_t *b, uint64_t m, const PeelState *st, uint32_t *state, uint32_t *front,
                            uint32_t *nfront, int64_t *wing) {
    const int64_t k = round_k(st);
    const uint32_t rid = (uint32_t)st->rid;
    const uint32_t lane = threadIdx.x & (WAVE - 1);
    for (uint64_t e0 = (uint64_t)blockIdx.x * blockDim.x; e0 < m; e0 += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t e = e0 + threadIdx.x;
        const bool take = e < m && !state[e] && b[e] <= k;
        const uint64_t mask = __ballot(take);
        if (mask == 0) continue;
        const uint32_t leader = (uint32_t)__ffsll((unsigned long long)mask) - 1;
        uint32_t at = 0;
        if (lane == leader) at = atomicAdd(nfront, (uint32_t)__popcll(mask));
        at = __shfl(at, (int)leader, WAVE);
        if (take) {
            front[at + (uint32_t)__popcll(mask & lanemask_lt())] = (uint32_t)e;
            state[e] = rid;
            wing[e] = k;
        }
    }
}

struct WingGraph {
    const int64_t *u_off;
    const uint32_t *u_adj, *eu, *v_off, *v_adj, *v_eid;
};

// UPDATE-E: one workgroup per peeled edge (u1, v1); each thread takes one u2
// in N(v1) and merges the sorted rows N(u1) and N(u2) for the v2 they share.
__global__ __launch_bounds__(256) void k_wing_update(WingGraph W, const uint32_t *front, const uint32_t *nfront,
                                                     const PeelState *st, const uint32_t *state, int64_t *b) {
    const uint32_t nf = *nfront;
    const uint32_t rid = (uint32_t)st->rid;
    for (uint32_t i = blockIdx.x; i < nf; i += gridDim.x) {
        const uint32_t e = front[i];
        const uint32_t u1 = W.eu[e], v1 = W.u_adj[e];
        const int64_t a0 = W.u_off[u1], a1 = W.u_off[u1 + 1];
        for (uint32_t p = W.v_off[v1] + threadIdx.x; p < W.v_off[v1 + 1]; p += blockDim.x) {
            const uint32_t u2 = W.v_adj[p], e2 = W.v_eid[p];  // edge (u2, v1)
            if (u2 == u1) continue;
            const uint32_t s2 = state[e2];
            if ((s2 && s2 < rid) || (s2 == rid && e2 < e)) continue;
            int64_t a = a0, c = W.u_off[u2];
            const int64_t c1 = W.u_off[u2 + 1];
            while (a < a1 && c < c1) {
                const uint32_t va = W.u_adj[a], vc = W.u_adj[c];
                if (va < vc) { ++a; continue; }
                if (vc < va) { ++c; continue; }
                if (va != v1) {
                    const uint32_t e1 = (uint32_t)a, e3 = (uint32_t)c;  // edges (u1, v2), (u2, v2)
                    const uint32_t s1 = state[e1], s3 = state[e3];
                    const bool skip = (s1 && s1 < rid) || (s3 && s3 < rid) || (s1 == rid && e1 < e) ||
                                      (s3 == rid && e3 < e);
                    if (!skip) {
                        if (!s1) atomicAdd(reinterpret_cast<unsigned long long *>(&b[e1]), ~0ull);
                        if (!s2) atomicAdd(reinterpret_cast<unsigned long long *>(&b[e2]), ~0ull);
                        if (!s3) atomicAdd(reinterpret_cast<unsigned long long *>(&b[e3]), ~0ull);
                    }
                }
                ++a;
                ++c;
            }
        }
    }
}

__global__ void k_wing_close(uint32_t *nfront, PeelState *st) {
    const uint32_t nf = *nfront;
    st->k = round_k(st);
    st->left -= nf;
    st->rounds += nf ? 1 : 0;
    st->rid += 1;
    st->mn = ~0ull;
    *nfront = 0;
}

pb_status wing_impl(pb_graph *g, const pb_opts *opts, int64_t *wing, uint64_t *rounds_out, hipStream_t s) {
    if (!g || (g->m && !wing)) return PB_ERR_INVALID_ARG;
    const uint64_t n = (uint64_t)g->n_u + g->n_v, m = g->m;
    if (m == 0) {
        if (rounds_out) *rounds_out = 0;
        return PB_OK;
    }
    Workspace ws(s, 0);
    HostBuf hb;
    PB_TRY_HIP(hipHostMalloc(&hb.p, 64, hipHostMallocDefault));
    uint32_t *rank = ws.alloc<uint32_t>(n);
    int64_t *b = ws.alloc<int64_t>(m);
    if (ws.failed) return PB_ERR_NO_MEMORY;
    PB_TRY(pb_rank(g, PB_RANK_DEGREE, rank, s));
    PB_TRY(pb_count_edge(g, rank, opts, b, s));
    ws.release(rank);
    uint32_t *state = ws.alloc<uint32_t>(m), *nfront = ws.alloc<uint32_t>(1);
    uint32_t *front = ws.alloc<uint32_t>(m);
    PeelState *st = ws.alloc<PeelState>(1);
    if (ws.failed) return PB_ERR_NO_MEMORY;
    PB_TRY(fill<uint32_t>(state, 0u, m, s));
    PB_TRY(fill<uint32_t>(nfront, 0u, 1, s));
    const PeelState st0{0, ~0ull, m, 0, 1};
    PB_TRY_HIP(hipMemcpyAsync(st, &st0, sizeof(st0), hipMemcpyHostToDevice, s));
    const WingGraph W{g->u_off, g->u_adj, g->eu, g->v_off, g->v_adj, g->v_eid};
    PeelState *hst = static_cast<PeelState *>(hb.p);
    for (;;) {
        for (uint32_t r = 0; r < PEEL_BATCH; ++r) {
            hipLaunchKernelGGL(k_wing_min, dim3(grid_of(m, 1024)), dim3(256), 0, s, (const int64_t *)b,
                               (const uint32_t *)state, m, &st->mn);
            hipLaunchKernelGGL(k_wing_take, dim3(grid_of(m, 65536)), dim3(256), 0, s, (const int64_t *)b, m,
                               (const PeelState *)st, state, front, nfront, wing);
            hipLaunchKernelGGL(k_wing_update, dim3(1024), dim3(256), 0, s, W, (const uint32_t *)front,
                               (const uint32_t *)nfront, (const PeelState *)st, (const uint32_t *)state, b);
            hipLaunchKernelGGL(k_wing_close, dim3(1), dim3(1), 0, s, nfront, st);
            PB_TRY_HIP(hipGetLastError());
        }
        PB_TRY_HIP(hipMemcpyAsync(hst, st, sizeof(PeelState), hipMemcpyDeviceToHost, s));
        PB_TRY_HIP(hipStreamSynchronize(s));
        if (hst->left == 0) break;
        if (hst->left > m) return PB_ERR_INTERNAL;  // cannot happen: each round takes at most what is left
    }
    if (rounds_out) *rounds_out = hst->rounds;
    return PB_OK;
}

}  // namespace

extern "C" pb_status pb_tip_decompose(pb_graph *g, pb_peel_side side, const pb_opts *opts, int64_t *tip_out,
                                      pb_peel_side *side_out, uint64_t *rounds_out, hipStream_t stream) {
    return peel_impl(g, side, opts, tip_out, side_out, rounds_out, stream);
}

extern "C" pb_status pb_wing_decompose(pb_graph *g, const pb_opts *opts, int64_t *wing_out, uint64_t *rounds_out,
                                       hipStream_t stream) {
    return wing_impl(g, opts, wing_out, rounds_out, stream);
}
