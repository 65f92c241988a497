// Graph handle (input validation, V-side CSR) and vertex orderings.
//
// Section 2 keeps one CSR per side; the caller supplies the U side and the
// handle derives the V side by a stable sort of the edges by V id.
// Section 3.1.1 defines the orderings built by pb_rank.
#include "pb_internal.h"

#include <cstring>
#include <new>

using namespace pb;

namespace {

enum : uint32_t { BAD_OFFSETS = 1u, BAD_ID = 2u, NOT_INCREASING = 4u };

constexpr int EDGE_BLOCK = 256;
constexpr int EDGES_PER_BLOCK = 1024;

__global__ void k_check_offsets(const int64_t *u_off, uint32_t n_u, uint64_t m, uint32_t *flags) {
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u <= n_u;
         u += (uint64_t)gridDim.x * blockDim.x) {
        const int64_t o = u_off[u];
        bool bad = o < 0 || (uint64_t)o > m;
        if (u == 0 && o != 0) bad = true;
        if (u == n_u && (uint64_t)o != m) bad = true;
        if (u > 0 && u_off[u - 1] > o) bad = true;
        if (bad) atomicOr(flags, (uint32_t)BAD_OFFSETS);
    }
}

// Largest r in [lo, hi) with u_off[r] <= e (rows are [u_off[r], u_off[r+1])).
__device__ inline uint32_t row_of(const int64_t *u_off, uint32_t lo, uint32_t hi, uint64_t e) {
    while (hi - lo > 1) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if ((uint64_t)u_off[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// eu[e] = the U row holding edge e; checks ids and strict increase.  Each
// block first finds the row range covering its edges, then each thread
// searches that (short) range.
__global__ __launch_bounds__(EDGE_BLOCK) void k_edge_rows(const int64_t *u_off, const uint32_t *u_adj,
                                                          uint32_t n_u, uint32_t n_v, uint64_t m,
                                                          uint32_t *eu, uint32_t *flags) {
    __shared__ uint32_t s_lo, s_hi;
    const uint64_t e0 = (uint64_t)blockIdx.x * EDGES_PER_BLOCK;
    const uint64_t e1 = e0 + EDGES_PER_BLOCK < m ? e0 + EDGES_PER_BLOCK : m;
    if (threadIdx.x == 0) {
        s_lo = row_of(u_off, 0, n_u, e0);
        s_hi = row_of(u_off, 0, n_u, e1 - 1) + 1;
    }
    __syncthreads();
    const uint32_t lo = s_lo, hi = s_hi > lo ? s_hi : lo + 1;
    uint32_t bad = 0;
    for (uint64_t e = e0 + threadIdx.x; e < e1; e += EDGE_BLOCK) {
        uint32_t r = row_of(u_off, lo, hi, e);
        if (r >= n_u) r = n_u - 1;
        eu[e] = r;
        const uint32_t v = u_adj[e];
        if (v >= n_v) bad |= BAD_ID;
        if ((int64_t)e > u_off[r] && e > 0 && u_adj[e - 1] >= v) bad |= NOT_INCREASING;
    }
    if (bad) atomicOr(flags, bad);
}

// Sort keys of the V-side CSR: the V id in the high word, the edge's U
// endpoint riding along in the low word (the sort reads the high word only),
// so the sorted keys give v_adj without a gather through the edge ids.
__global__ void k_iota_keys(const uint32_t *u_adj, const uint32_t *eu, uint64_t m, uint64_t *keys, uint32_t *vals) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (uint64_t)gridDim.x * blockDim.x) {
        keys[e] = ((uint64_t)u_adj[e] << 32) | eu[e];
        vals[e] = (uint32_t)e;
    }
}

// V-side row offsets from the edges sorted by V id: position p starts the
// rows of every id in (key[p-1], key[p]].  Skipped when an id was out of
// range (the keys are then not a valid order and the call fails anyway).
__global__ void k_voff_from_sorted(const uint64_t *key, uint64_t m, uint32_t n_v, const uint32_t *flags,
                                   uint32_t *v_off) {
    if (flags[0] & BAD_ID) return;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p <= m;
         p += (uint64_t)gridDim.x * blockDim.x) {
        const int64_t prev = p == 0 ? -1 : (int64_t)(key[p - 1] >> 32);
        const int64_t cur = p == m ? (int64_t)n_v : (int64_t)(key[p] >> 32);
        for (int64_t v = prev + 1; v <= cur; ++v) v_off[v] = (uint32_t)p;
    }
}

__global__ void k_split_sorted(const uint64_t *keys, const uint32_t *eids, uint64_t m, uint32_t *v_adj,
                               uint32_t *v_eid) {
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m;
         p += (uint64_t)gridDim.x * blockDim.x) {
        v_adj[p] = (uint32_t)keys[p];
        v_eid[p] = eids[p];
    }
}

constexpr uint32_t DEG_GRID = 1024;
__global__ __launch_bounds__(256) void k_degrees(const int64_t *u_off, const uint32_t *v_off, uint32_t n_u,
                                                 uint32_t n_v, uint32_t *deg, uint32_t *max_deg) {
    __shared__ uint32_t wmax[256 / WAVE];
    uint32_t best = 0;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < (uint64_t)n_u + n_v;
         x += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t d;
        if (x < n_u) d = (uint32_t)(u_off[x + 1] - u_off[x]);
        else d = v_off[x - n_u + 1] - v_off[x - n_u];
        deg[x] = d;
        best = d > best ? d : best;
    }
    for (int s = WAVE / 2; s >= 1; s >>= 1) {
        const uint32_t o = __shfl_xor(best, s, WAVE);
        best = o > best ? o : best;
    }
    if ((threadIdx.x & (WAVE - 1)) == 0) wmax[threadIdx.x / WAVE] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 256 / WAVE; ++i) best = wmax[i] > best ? wmax[i] : best;
        atomicMax(max_deg, best);
    }
}

inline uint32_t grid_for(uint64_t n, uint32_t block = 256, uint32_t cap = 65536) {
    uint64_t g = (n + block - 1) / block;
    if (g == 0) g = 1;
    return (uint32_t)(g > cap ? cap : g);
}

// ---------------------------------------------------------------- orderings

// sums[0] = sum_{v in V} C(deg v, 2) (wedges with U endpoints, U first)
// sums[1] = sum_{u in U} C(deg u, 2) (wedges with V endpoints, V first)
__global__ void k_side_sums(const uint32_t *deg, uint32_t n_u, uint32_t n_v, unsigned long long *sums) {
    unsigned long long su = 0, sv = 0;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < (uint64_t)n_u + n_v;
         x += (uint64_t)gridDim.x * blockDim.x) {
        const unsigned long long d = deg[x];
        const unsigned long long c = d * (d - (d > 0)) / 2;
        if (x < n_u) sv += c; else su += c;
    }
    su = wave_sum(su);
    sv = wave_sum(sv);
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        atomicAdd(&sums[0], su);
        atomicAdd(&sums[1], sv);
    }
}

// mode 0: U first, 1: V first, 2: decide from sums.
__global__ void k_side_rank(uint32_t n_u, uint32_t n_v, int mode, const unsigned long long *sums,
                            uint32_t *rank) {
    bool u_first = mode == 0;
    if (mode == 2) u_first = sums[0] <= sums[1];
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < (uint64_t)n_u + n_v;
         x += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t r;
        if (u_first) r = (uint32_t)x;
        else r = x < n_u ? (uint32_t)(n_v + x) : (uint32_t)(x - n_u);
        rank[x] = r;
    }
}

__device__ inline uint32_t level_key(uint32_t d) {  // floor(log2 d) + 1, 0 for d = 0
    return d ? 32u - (uint32_t)__clz(d) : 0u;
}

// key = (descending primary key) << idbits | id
__global__ void k_order_keys(const uint32_t *deg, uint64_t n, int approx, uint32_t max_key, int idbits,
                             uint64_t *keys, uint32_t *vals) {
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t k = approx ? level_key(deg[x]) : deg[x];
        keys[x] = ((uint64_t)(max_key - k) << idbits) | x;
        vals[x] = (uint32_t)x;
    }
}

__global__ void k_scatter_rank(const uint32_t *ids, uint64_t n, uint32_t *rank) {
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (uint64_t)gridDim.x * blockDim.x)
        rank[ids[p]] = (uint32_t)p;
}

// Complement-coreness rounds.
// The largest key among the remaining vertices (+1, so 0 means none left):
// reduced in the block first, one atomic per block.
constexpr uint32_t CODEG_MAX_GRID = 1024;
__global__ __launch_bounds__(256) void k_codeg_max(const uint32_t *cur, const uint32_t *alive, uint64_t n, int approx,
                                                   uint32_t *best) {
    __shared__ uint32_t wmax[256 / WAVE];
    uint32_t b = 0;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (uint64_t)gridDim.x * blockDim.x)
        if (alive[x]) {
            const uint32_t k = (approx ? level_key(cur[x]) : cur[x]) + 1;  // +1: alive marker
            b = k > b ? k : b;
        }
    for (int s = WAVE / 2; s >= 1; s >>= 1) {
        const uint32_t o = __shfl_xor(b, s, WAVE);
        b = o > b ? o : b;
    }
    if ((threadIdx.x & (WAVE - 1)) == 0) wmax[threadIdx.x / WAVE] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 256 / WAVE; ++i) b = wmax[i] > b ? wmax[i] : b;
        if (b) atomicMax(best, b);
    }
}

// One round's removal: the live vertices whose key equals the largest
// (`best`, +1) are ranked next in increasing id, without a flag array or a
// scan over all vertices.  A tile of CR_TILE ids is 4 waves of 16 steps of
// 64 consecutive ids; k_codeg_count counts the tile's picks, the tile counts
// are scanned, and k_codeg_take recounts them by ballots and ranks them.
constexpr uint32_t CR_T = 256;
constexpr uint32_t CR_STEPS = 16;
constexpr uint32_t CR_WAVE_SPAN = WAVE * CR_STEPS;            // 1024 ids per wave
constexpr uint32_t CR_TILE = CR_T / WAVE * CR_WAVE_SPAN;      // 4096 ids per workgroup

__device__ inline bool codeg_pick(const uint32_t *cur, const uint32_t *alive, uint64_t x, uint64_t n, int approx,
                                  uint32_t top) {
    return x < n && alive[x] && (approx ? level_key(cur[x]) : cur[x]) + 1 == top;
}

__global__ __launch_bounds__(CR_T) void k_codeg_count(const uint32_t *cur, const uint32_t *alive, uint64_t n,
                                                      int approx, const uint32_t *best, uint32_t *tcnt) {
    __shared__ uint32_t wc[CR_T / WAVE];
    const uint32_t top = *best, lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const uint64_t x0 = (uint64_t)blockIdx.x * CR_TILE + (uint64_t)w * CR_WAVE_SPAN + lane;
    uint32_t c = 0;
#pragma unroll 4
    for (uint32_t j = 0; j < CR_STEPS; ++j) c += (uint32_t)__popcll(__ballot(codeg_pick(cur, alive, x0 + j * WAVE, n, approx, top)));
    if (lane == 0) wc[w] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (uint32_t i = 0; i < CR_T / WAVE; ++i) t += wc[i];
        tcnt[blockIdx.x] = t;
    }
}

// toff: exclusive scan of the tile counts.  Ranks next + (picks before x)
// in increasing id, fills front in that order and retires the picks.
__global__ __launch_bounds__(CR_T) void k_codeg_take(const uint32_t *cur, uint32_t *alive, uint64_t n, int approx,
                                                     const uint32_t *best, const uint32_t *toff, uint32_t next,
                                                     uint32_t *rank, uint32_t *front) {
    __shared__ uint32_t wc[CR_T / WAVE];
    const uint32_t top = *best, lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const uint64_t x0 = (uint64_t)blockIdx.x * CR_TILE + (uint64_t)w * CR_WAVE_SPAN + lane;
    uint64_t bal[CR_STEPS];
    uint32_t c = 0;
#pragma unroll
    for (uint32_t j = 0; j < CR_STEPS; ++j) {
        bal[j] = __ballot(codeg_pick(cur, alive, x0 + j * WAVE, n, approx, top));
        c += (uint32_t)__popcll(bal[j]);
    }
    if (lane == 0) wc[w] = c;
    __syncthreads();
    uint32_t p = toff[blockIdx.x];
    for (uint32_t i = 0; i < w; ++i) p += wc[i];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (uint32_t j = 0; j < CR_STEPS; ++j) {
        if ((bal[j] >> lane) & 1) {
            const uint64_t x = x0 + j * WAVE;
            const uint32_t q = p + (uint32_t)__popcll(bal[j] & lt);
            rank[x] = next + q;
            front[q] = (uint32_t)x;
            alive[x] = 0;
        }
        p += (uint32_t)__popcll(bal[j]);
    }
}

// A removed vertex of degree at most DEC_SMALL is handled by one thread;
// a larger one is visited in items of DEC_CHUNK neighbours, one workgroup
// each, so one huge vertex spreads over many workgroups instead of forming
// one serial chain.
constexpr uint32_t DEC_SMALL = 64;
constexpr uint32_t DEC_CHUNK = 2048;
constexpr uint32_t DEC_GRID = 4096;

__device__ inline void codeg_drop(uint32_t y, const uint32_t *alive, uint32_t *cur) {
    if (alive[y]) atomicSub(&cur[y], 1u);  // a neighbour removed earlier keeps its key
}

// Small front vertices (one thread each); chunk counts of the large ones.
__global__ void k_codeg_small(const uint32_t *front, uint32_t nfront, const uint32_t *deg, const int64_t *u_off,
                              const uint32_t *u_adj, const uint32_t *v_off, const uint32_t *v_adj, uint32_t n_u,
                              const uint32_t *alive, uint32_t *cur, uint32_t *cnt) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nfront;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t x = front[i], d = deg[x];
        if (d > DEC_SMALL) {
            cnt[i] = (d + DEC_CHUNK - 1) / DEC_CHUNK;
            continue;
        }
        cnt[i] = 0;
        if (x < n_u) {
            for (int64_t k = u_off[x]; k < u_off[x + 1]; ++k) codeg_drop(n_u + u_adj[k], alive, cur);
        } else {
            for (uint32_t k = v_off[x - n_u]; k < v_off[x - n_u + 1]; ++k) codeg_drop(v_adj[k], alive, cur);
        }
    }
}

// Large front vertices: every live neighbour loses one remaining neighbour.
// Item `it` belongs to the front vertex i with coff[i] <= it < coff[i + 1];
// each workgroup takes a contiguous share of the items.
__global__ void k_codeg_decrement(const uint32_t *front, const uint32_t *coff, uint32_t nfront,
                                  const int64_t *u_off, const uint32_t *u_adj, const uint32_t *v_off,
                                  const uint32_t *v_adj, uint32_t n_u, const uint32_t *alive, uint32_t *cur) {
    uint32_t i0, i1;  // a contiguous share of the items per workgroup
    item_share(coff[nfront], blockIdx.x, gridDim.x, &i0, &i1);
    rows_of_items(coff, nfront, i0, i1, [&](uint32_t i, uint32_t it) {
        const uint32_t x = front[i];
        const uint64_t skip = (uint64_t)(it - coff[i]) * DEC_CHUNK;
        if (x < n_u) {
            const int64_t b = u_off[x] + (int64_t)skip, e = u_off[x + 1];
            const int64_t end = b + DEC_CHUNK < e ? b + DEC_CHUNK : e;
            for (int64_t k = b + threadIdx.x; k < end; k += blockDim.x) codeg_drop(n_u + u_adj[k], alive, cur);
        } else {
            const uint32_t v = x - n_u;
            const uint64_t b = v_off[v] + skip, e = v_off[v + 1];
            const uint64_t end = b + DEC_CHUNK < e ? b + DEC_CHUNK : e;
            for (uint64_t k = b + threadIdx.x; k < end; k += blockDim.x) codeg_drop(v_adj[k], alive, cur);
        }
    });
}

// Exact complement coreness over key windows.  A window holds every live
// vertex whose key lies in [L, H], H the largest live key, with L chosen so
// that at most CW_CAP vertices qualify (or exactly the vertices of key H when
// they alone are more).  Keys only fall, so until every window vertex is
// removed or drops below L, each round's largest key and its vertices are
// found inside the window: one workgroup runs those rounds back to back,
// reading only the window's vertices, and hands a round back to the host
// only when its removed vertices have more than CW_DMAX neighbours to visit.
constexpr uint32_t CW_CAP = 4096;    // window vertices run by one workgroup
constexpr uint32_t CW_BINS = 4096;   // keys H, H-1, ... histogrammed to choose L
constexpr uint32_t CW_DMAX = 16384;  // neighbour visits one in-kernel round may make
constexpr uint32_t CW_T = 1024;
constexpr uint32_t CW_U = 4;        // neighbour loads in flight per thread

enum : uint32_t { CW_EXHAUSTED = 0, CW_BIG = 1 };

struct CodegState {
    uint32_t status;  // CW_EXHAUSTED or CW_BIG
    uint32_t next;    // next rank to hand out
    uint32_t key;     // CW_BIG: the round's key
    uint32_t nf;      // CW_BIG: vertices the round removed (ranked, in front[0, nf))
};

// hist[d] = live vertices of key H - d (d < CW_BINS), H = *best - 1.  Counts
// are taken in LDS and added once per block.
__global__ __launch_bounds__(256) void k_codeg_hist(const uint32_t *cur, const uint32_t *alive, uint64_t n,
                                                    const uint32_t *best, uint32_t *hist) {
    __shared__ uint32_t h[CW_BINS];
    for (uint32_t i = threadIdx.x; i < CW_BINS; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const uint32_t top = *best - 1;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (uint64_t)gridDim.x * blockDim.x)
        if (alive[x]) {
            const uint32_t d = top - cur[x];
            if (d < CW_BINS) atomicAdd(&h[d], 1u);
        }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < CW_BINS; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

// lim[0] = L: the keys H, H-1, ..., L are the longest run from the top whose
// vertices number at most CW_CAP, or key H alone when it has more.
__global__ __launch_bounds__(CW_T) void k_codeg_cut(const uint32_t *hist, const uint32_t *best, uint32_t *lim) {
    constexpr uint32_t PER = CW_BINS / CW_T;
    __shared__ uint32_t tmp[CW_T / WAVE + 1];
    __shared__ uint32_t first_over;
    const uint32_t top = *best - 1;
    if (threadIdx.x == 0) first_over = CW_BINS;
    uint32_t v[PER], sum = 0;
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) {
        v[j] = hist[threadIdx.x * PER + j];
        sum += v[j];
    }
    uint32_t total;
    uint32_t pre = block_exclusive_sum<CW_T, uint32_t>(sum, tmp, &total);
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) {
        pre += v[j];
        if (pre > CW_CAP) atomicMin(&first_over, threadIdx.x * PER + j);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t bins = first_over ? first_over : 1u;  // bins 0 .. bins-1 are taken
        if (bins > top + 1) bins = top + 1;
        lim[0] = top + 1 - bins;
    }
}

__global__ void k_codeg_inwin(const uint32_t *cur, const uint32_t *alive, uint64_t n, const uint32_t *lim,
                              uint32_t *flag) {
    const uint32_t lo = lim[0];
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (uint64_t)gridDim.x * blockDim.x)
        flag[x] = alive[x] && cur[x] >= lo;
}

__global__ void k_codeg_gather(const uint32_t *flag, const uint32_t *pos, uint64_t n, uint32_t *win) {
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (uint64_t)gridDim.x * blockDim.x)
        if (flag[x]) win[pos[x]] = (uint32_t)x;
}

// A window of one key (more vertices than one workgroup takes): every
// window vertex is removed, ranked in window order (= id order).
__global__ void k_codeg_wtake(const uint32_t *win, uint32_t nw, uint32_t next, uint32_t *alive, uint32_t *rank,
                              uint32_t *front) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += gridDim.x * blockDim.x) {
        const uint32_t x = win[i];
        rank[x] = next + i;
        front[i] = x;
        alive[x] = 0;
    }
}

// The rounds of one window (at most CW_CAP vertices, ids increasing).  Each
// round: the largest live key M among the window's vertices; if M < L the
// window is exhausted.  Its vertices take the next ranks in id order, and
// every neighbour of theirs loses one.  A removed vertex's key is never read
// again, so its neighbours are dropped without a liveness test.
//
// The whole window lives on one CU, so the waves only need each other's
// writes to have reached L2 (a full wait before the barrier) and read keys
// and liveness from L2 (relaxed atomic loads, which miss L1); no device-wide
// fence is needed between rounds.
__device__ inline uint32_t l2_load(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(CW_T) void k_codeg_window(const uint32_t *win, uint32_t nw, uint32_t lo, uint32_t next,
                                                       const uint32_t *deg, const int64_t *u_off,
                                                       const uint32_t *u_adj, const uint32_t *v_off,
                                                       const uint32_t *v_adj, uint32_t n_u, uint32_t *cur,
                                                       uint32_t *alive, uint32_t *rank, uint32_t *front,
                                                       CodegState *st) {
    constexpr uint32_t PER = CW_CAP / CW_T;
    __shared__ uint32_t fv[CW_CAP];                   // the round's vertices
    __shared__ uint32_t foff[CW_CAP + 1];             // their offsets in the flat neighbour sequence
    __shared__ unsigned long long fadj[CW_CAP];       // where their neighbour lists start
    __shared__ uint32_t tmp32[CW_T / WAVE + 1];
    __shared__ unsigned long long tmp64[CW_T / WAVE + 1];
    __shared__ uint32_t wmax[CW_T / WAVE];
    const uint32_t tid = threadIdx.x, lane = tid & (WAVE - 1);
    uint32_t ids[PER], dg[PER];
    unsigned long long at0[PER];
    bool slot[PER];
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) {
        const uint32_t i = tid * PER + j;
        slot[j] = i < nw;
        ids[j] = slot[j] ? win[i] : win[0];  // a valid id, never used as a window vertex
        dg[j] = slot[j] ? deg[ids[j]] : 0u;
        at0[j] = ids[j] < n_u ? (unsigned long long)u_off[ids[j]] : (unsigned long long)v_off[ids[j] - n_u];
    }
    for (;;) {
        uint32_t av[PER], cv[PER], key[PER], best = 0;  // key + 1, 0 = removed or not a window slot
#pragma unroll
        for (uint32_t j = 0; j < PER; ++j) {
            av[j] = l2_load(&alive[ids[j]]);
            cv[j] = l2_load(&cur[ids[j]]);
        }
#pragma unroll
        for (uint32_t j = 0; j < PER; ++j) {
            key[j] = slot[j] && av[j] ? cv[j] + 1 : 0u;
            best = key[j] > best ? key[j] : best;
        }
        for (int d = WAVE / 2; d >= 1; d >>= 1) {
            const uint32_t o = __shfl_xor(best, d, WAVE);
            best = o > best ? o : best;
        }
        if (lane == 0) wmax[tid / WAVE] = best;
        __syncthreads();
        best = 0;
        for (uint32_t w = 0; w < CW_T / WAVE; ++w) best = wmax[w] > best ? wmax[w] : best;
        if (best == 0 || best - 1 < lo) {
            if (tid == 0) {
                st->status = CW_EXHAUSTED;
                st->next = next;
            }
            return;
        }
        uint32_t f = 0;
        unsigned long long sd = 0;
#pragma unroll
        for (uint32_t j = 0; j < PER; ++j)
            if (key[j] == best) {
                ++f;
                sd += dg[j];
            }
        uint32_t nf;
        unsigned long long sum;
        uint32_t fp = block_exclusive_sum<CW_T, uint32_t>(f, tmp32, &nf);
        unsigned long long sp = block_exclusive_sum<CW_T, unsigned long long>(sd, tmp64, &sum);
        if (sum > CW_DMAX) {
            // ranked here; the neighbours are dropped by all workgroups
#pragma unroll
            for (uint32_t j = 0; j < PER; ++j)
                if (key[j] == best) {
                    rank[ids[j]] = next + fp;
                    alive[ids[j]] = 0;
                    front[fp] = ids[j];
                    ++fp;
                }
            if (tid == 0) {
                st->status = CW_BIG;
                st->next = next + nf;
                st->key = best - 1;
                st->nf = nf;
            }
            return;
        }
#pragma unroll
        for (uint32_t j = 0; j < PER; ++j)
            if (key[j] == best) {
                rank[ids[j]] = next + fp;
                alive[ids[j]] = 0;
                fv[fp] = ids[j];
                foff[fp] = (uint32_t)sp;
                fadj[fp] = at0[j];
                ++fp;
                sp += dg[j];
            }
        if (tid == 0) foff[nf] = (uint32_t)sum;
        __syncthreads();
        // visit q of the flat neighbour sequence: front vertex p, the largest
        // with foff[p] <= q, found by a fixed number of halving steps so that
        // a thread's CW_U searches and loads proceed side by side
        const uint32_t total = (uint32_t)sum;
        uint32_t lg = 0;
        while ((1u << lg) < nf) ++lg;
        for (uint32_t q0 = tid; q0 < total; q0 += CW_U * CW_T) {
            uint32_t q[CW_U], pa[CW_U], y[CW_U];
#pragma unroll
            for (uint32_t u = 0; u < CW_U; ++u) {
                const uint32_t qq = q0 + u * CW_T;
                q[u] = qq < total ? qq : total - 1;
                pa[u] = 0;
            }
            for (uint32_t sh = lg; sh-- > 0;) {
#pragma unroll
                for (uint32_t u = 0; u < CW_U; ++u) {
                    const uint32_t c = pa[u] + (1u << sh);
                    if (c < nf && foff[c] <= q[u]) pa[u] = c;
                }
            }
#pragma unroll
            for (uint32_t u = 0; u < CW_U; ++u) {
                const bool us = fv[pa[u]] < n_u;
                const unsigned long long at = fadj[pa[u]] + (q[u] - foff[pa[u]]);
                const uint32_t *src = us ? u_adj + at : v_adj + at;
                y[u] = *src + (us ? n_u : 0u);
            }
#pragma unroll
            for (uint32_t u = 0; u < CW_U; ++u)
                if (q0 + u * CW_T < total) atomicSub(&cur[y[u]], 1u);
        }
        __builtin_amdgcn_s_waitcnt(0);  // this wave's removals and decrements have reached L2
        __syncthreads();
        next += nf;
    }
}

pb_status rank_codeg_exact(pb_graph *g, uint32_t *rank, hipStream_t s) {
    const uint64_t n = (uint64_t)g->n_u + g->n_v;
    Workspace ws(s, 0);
    uint32_t *cur = ws.alloc<uint32_t>(n), *alive = ws.alloc<uint32_t>(n);
    uint32_t *flag = ws.alloc<uint32_t>(n), *pos = ws.alloc<uint32_t>(n + 1);
    uint32_t *win = ws.alloc<uint32_t>(n), *front = ws.alloc<uint32_t>(n);
    uint32_t *ccnt = ws.alloc<uint32_t>(n + 1), *coff = ws.alloc<uint32_t>(n + 1);
    uint32_t *best = ws.alloc<uint32_t>(2), *hist = ws.alloc<uint32_t>(CW_BINS);
    CodegState *st = ws.alloc<CodegState>(1);
    uint32_t *lim = best + 1;
    if (ws.failed) return PB_ERR_NO_MEMORY;
    uint32_t *host = nullptr;  // [0] = window size, [1..4] = state
    PB_TRY_HIP(hipHostMalloc((void **)&host, 8 * sizeof(uint32_t), hipHostMallocDefault));
    pb_status rc = PB_OK;
    const auto sync_read = [&](void *dst, const void *src, size_t bytes) {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s) == hipSuccess &&
               hipStreamSynchronize(s) == hipSuccess;
    };
    // removes the `nf` vertices in front[0, nf): their live neighbours lose one
    const auto drop_front = [&](uint32_t nf) -> pb_status {
        hipLaunchKernelGGL(k_codeg_small, dim3(grid_for(nf)), dim3(256), 0, s, (const uint32_t *)front, nf,
                           (const uint32_t *)g->deg, g->u_off, g->u_adj, g->v_off, g->v_adj, g->n_u,
                           (const uint32_t *)alive, cur, ccnt);
        PB_TRY((scan_exclusive<uint32_t, uint32_t>(ccnt, coff, nf, coff + nf, ws)));
        hipLaunchKernelGGL(k_codeg_decrement, dim3(DEC_GRID), dim3(256), 0, s, (const uint32_t *)front,
                           (const uint32_t *)coff, nf, g->u_off, g->u_adj, g->v_off, g->v_adj, g->n_u,
                           (const uint32_t *)alive, cur);
        PB_TRY_HIP(hipGetLastError());
        return PB_OK;
    };
    do {
        if (hipMemcpyAsync(cur, g->deg, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s) != hipSuccess) {
            rc = PB_ERR_HIP;
            break;
        }
        if ((rc = fill<uint32_t>(alive, 1u, n, s)) != PB_OK) break;
        uint32_t next = 0;
        while (next < n && rc == PB_OK) {
            // the window: largest live key H, cut L, live vertices of key >= L
            if ((rc = fill<uint32_t>(best, 0u, 1, s)) != PB_OK) break;
            if ((rc = fill<uint32_t>(hist, 0u, CW_BINS, s)) != PB_OK) break;
            hipLaunchKernelGGL(k_codeg_max, dim3(grid_for(n, 256, CODEG_MAX_GRID)), dim3(256), 0, s, cur, alive, n,
                               0, best);
            hipLaunchKernelGGL(k_codeg_hist, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, cur, alive, n,
                               (const uint32_t *)best, hist);
            hipLaunchKernelGGL(k_codeg_cut, dim3(1), dim3(CW_T), 0, s, (const uint32_t *)hist,
                               (const uint32_t *)best, lim);
            hipLaunchKernelGGL(k_codeg_inwin, dim3(grid_for(n)), dim3(256), 0, s, cur, alive, n,
                               (const uint32_t *)lim, flag);
            if ((rc = scan_exclusive<uint32_t, uint32_t>(flag, pos, n, pos + n, ws)) != PB_OK) break;
            hipLaunchKernelGGL(k_codeg_gather, dim3(grid_for(n)), dim3(256), 0, s, (const uint32_t *)flag,
                               (const uint32_t *)pos, n, win);
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(host + 1, lim, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
                !sync_read(host, pos + n, sizeof(uint32_t))) {
                rc = PB_ERR_HIP;
                break;
            }
            const uint32_t nw = host[0], lo = host[1];
            if (nw == 0) { rc = PB_ERR_INTERNAL; break; }  // cannot happen while vertices remain
            if (nw > CW_CAP) {
                // only key H's vertices: one round removes them all
                hipLaunchKernelGGL(k_codeg_wtake, dim3(grid_for(nw)), dim3(256), 0, s, (const uint32_t *)win, nw,
                                   next, alive, rank, front);
                if ((rc = drop_front(nw)) != PB_OK) break;
                next += nw;
                continue;
            }
            for (;;) {
                hipLaunchKernelGGL(k_codeg_window, dim3(1), dim3(CW_T), 0, s, (const uint32_t *)win, nw, lo, next,
                                   (const uint32_t *)g->deg, g->u_off, g->u_adj, g->v_off, g->v_adj, g->n_u, cur,
                                   alive, rank, front, st);
                if (hipGetLastError() != hipSuccess || !sync_read(host + 4, st, sizeof(CodegState))) {
                    rc = PB_ERR_HIP;
                    break;
                }
                CodegState h;
                memcpy(&h, host + 4, sizeof(h));
                next = h.next;
                if (h.status == CW_EXHAUSTED) break;
                if (h.status != CW_BIG || h.nf == 0) { rc = PB_ERR_INTERNAL; break; }  // a round removes someone
                // a round with many neighbours to visit: ranked by the window
                // kernel, its neighbours dropped by all workgroups
                if ((rc = drop_front(h.nf)) != PB_OK) break;
            }
        }
    } while (0);
    (void)hipStreamSynchronize(s);
    (void)hipHostFree(host);
    return rc;
}

pb_status rank_codeg(pb_graph *g, bool approx, uint32_t *rank, hipStream_t s) {
    const uint64_t n = (uint64_t)g->n_u + g->n_v;
    const uint32_t nt = ceil_div(n, CR_TILE);
    Workspace ws(s, 0);
    uint32_t *cur = ws.alloc<uint32_t>(n), *alive = ws.alloc<uint32_t>(n);
    uint32_t *tcnt = ws.alloc<uint32_t>(nt + 1), *toff = ws.alloc<uint32_t>(nt + 1);
    uint32_t *front = ws.alloc<uint32_t>(n), *best = ws.alloc<uint32_t>(1);
    uint32_t *ccnt = ws.alloc<uint32_t>(n + 1), *coff = ws.alloc<uint32_t>(n + 1);
    uint32_t *host = nullptr;
    if (ws.failed) return PB_ERR_NO_MEMORY;
    PB_TRY_HIP(hipHostMalloc((void **)&host, sizeof(uint32_t), hipHostMallocDefault));
    pb_status st = PB_OK;
    do {
        if (hipMemcpyAsync(cur, g->deg, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s) != hipSuccess) {
            st = PB_ERR_HIP;
            break;
        }
        if ((st = fill<uint32_t>(alive, 1u, n, s)) != PB_OK) break;
        uint32_t next = 0;
        while (next < n) {
            if ((st = fill<uint32_t>(best, 0u, 1, s)) != PB_OK) break;
            hipLaunchKernelGGL(k_codeg_max, dim3(grid_for(n, 256, CODEG_MAX_GRID)), dim3(256), 0, s, cur, alive, n,
                               (int)approx, best);
            hipLaunchKernelGGL(k_codeg_count, dim3(nt), dim3(CR_T), 0, s, (const uint32_t *)cur,
                               (const uint32_t *)alive, n, (int)approx, (const uint32_t *)best, tcnt);
            if ((st = scan_exclusive<uint32_t, uint32_t>(tcnt, toff, nt, toff + nt, ws)) != PB_OK) break;
            hipLaunchKernelGGL(k_codeg_take, dim3(nt), dim3(CR_T), 0, s, (const uint32_t *)cur, alive, n,
                               (int)approx, (const uint32_t *)best, (const uint32_t *)toff, next, rank, front);
            if (hipMemcpyAsync(host, toff + nt, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                st = PB_ERR_HIP;
                break;
            }
            const uint32_t nf = *host;
            if (nf == 0) { st = PB_ERR_INTERNAL; break; }  // cannot happen while vertices remain
            hipLaunchKernelGGL(k_codeg_small, dim3(grid_for(nf)), dim3(256), 0, s, (const uint32_t *)front, nf,
                               (const uint32_t *)g->deg, g->u_off, g->u_adj, g->v_off, g->v_adj, g->n_u,
                               (const uint32_t *)alive, cur, ccnt);
            if ((st = scan_exclusive<uint32_t, uint32_t>(ccnt, coff, nf, coff + nf, ws)) != PB_OK) break;
            hipLaunchKernelGGL(k_codeg_decrement, dim3(DEC_GRID), dim3(256), 0, s, (const uint32_t *)front,
                               (const uint32_t *)coff, nf, g->u_off, g->u_adj, g->v_off, g->v_adj, g->n_u,
                               (const uint32_t *)alive, cur);
            if (hipGetLastError() != hipSuccess) { st = PB_ERR_HIP; break; }
            next += nf;
        }
    } while (0);
    (void)hipStreamSynchronize(s);
    (void)hipHostFree(host);
    return st;
}

}  // namespace

extern "C" {

void pb_opts_default(pb_opts *opts) {
    if (!opts) return;
    opts->agg = PB_AGG_AUTO;
    opts->hub = PB_HUB_AUTO;
    opts->workspace_cap_bytes = 0;
    opts->wg_size = 0;
    opts->flags = 0;
    opts->stats = nullptr;
    opts->tuning = nullptr;
}

const char *pb_status_str(pb_status s) {
    switch (s) {
        case PB_OK: return "ok";
        case PB_ERR_INVALID_ARG: return "invalid argument";
        case PB_ERR_NOT_SIMPLE: return "graph not simple (a CSR row is not strictly increasing)";
        case PB_ERR_ID_RANGE: return "vertex id or offset out of range";
        case PB_ERR_BAD_RANK: return "rank is not a permutation of [0, n)";
        case PB_ERR_NO_MEMORY: return "out of device memory or workspace cap";
        case PB_ERR_OVERFLOW: return "count overflows int64 (reserved, never returned)";
        case PB_ERR_HIP: return "HIP runtime error";
        case PB_ERR_INTERNAL: return "internal consistency check failed";
    }
    return "unknown status";
}

pb_status pb_graph_create(const pb_csr *csr, hipStream_t s, pb_graph **out) {
    if (!csr || !out) return PB_ERR_INVALID_ARG;
    *out = nullptr;
    if (!csr->u_off) return PB_ERR_INVALID_ARG;
    if (csr->m > 0 && !csr->u_adj) return PB_ERR_INVALID_ARG;
    if (csr->m >= (uint64_t(1) << 31)) return PB_ERR_INVALID_ARG;
    if ((uint64_t)csr->n_u + csr->n_v >= 0xFFFFFFFFull) return PB_ERR_INVALID_ARG;
    if (csr->m > (uint64_t)csr->n_u * csr->n_v) return PB_ERR_NOT_SIMPLE;

    pb_graph *g = new (std::nothrow) pb_graph();
    if (!g) return PB_ERR_NO_MEMORY;
    g->n_u = csr->n_u;
    g->n_v = csr->n_v;
    g->m = csr->m;
    g->u_off = csr->u_off;
    g->u_adj = csr->u_adj;
    g->last_stream = s;
    (void)hipGetDevice(&g->device);
    const uint64_t n = (uint64_t)g->n_u + g->n_v, m = g->m;

    pb_status st = PB_OK;
    uint32_t *hflags = nullptr;
    {
        Workspace ws(s, 0);
        uint32_t *flags = ws.alloc<uint32_t>(2);  // [0] flags, [1] max degree
        bool ok = flags && (g->eu = (uint32_t *)scratch_get(s, (m ? m : 1) * sizeof(uint32_t))) != nullptr &&
                  (g->v_off = (uint32_t *)scratch_get(s, (g->n_v + 1) * sizeof(uint32_t))) != nullptr &&
                  (g->v_adj = (uint32_t *)scratch_get(s, (m ? m : 1) * sizeof(uint32_t))) != nullptr &&
                  (g->v_eid = (uint32_t *)scratch_get(s, (m ? m : 1) * sizeof(uint32_t))) != nullptr &&
                  (g->deg = (uint32_t *)scratch_get(s, (n ? n : 1) * sizeof(uint32_t))) != nullptr &&
                  hipHostMalloc((void **)&hflags, 2 * sizeof(uint32_t), hipHostMallocDefault) == hipSuccess;
        if (!ok) st = PB_ERR_NO_MEMORY;
        do {
            if (st != PB_OK) break;
            if ((st = fill<uint32_t>(flags, 0u, 2, s)) != PB_OK) break;
            hipLaunchKernelGGL(k_check_offsets, dim3(grid_for(g->n_u + 1ull)), dim3(256), 0, s, g->u_off, g->n_u, m,
                               flags);
            if (m > 0 && g->n_u > 0) {
                hipLaunchKernelGGL(k_edge_rows, dim3(ceil_div(m, EDGES_PER_BLOCK)), dim3(EDGE_BLOCK), 0, s, g->u_off,
                                   g->u_adj, g->n_u, g->n_v, m, g->eu, flags);
            }
            if (hipGetLastError() != hipSuccess) { st = PB_ERR_HIP; break; }
            // V-side CSR: a stable sort of edge ids by V id gives the rows, and
            // the sorted ids give the offsets.
            if (m == 0 && (st = fill<uint32_t>(g->v_off, 0u, g->n_v + 1ull, s)) != PB_OK) break;
            if (m > 0) {
                uint64_t *k0 = ws.alloc<uint64_t>(m), *k1 = ws.alloc<uint64_t>(m);
                uint32_t *v0 = ws.alloc<uint32_t>(m), *v1 = ws.alloc<uint32_t>(m);
                if (ws.failed) { st = PB_ERR_NO_MEMORY; break; }
                hipLaunchKernelGGL(k_iota_keys, dim3(grid_for(m)), dim3(256), 0, s, g->u_adj, g->eu, m, k0, v0);
                uint64_t *kr;
                uint32_t *vr;
                if ((st = radix_sort_pairs_bits(k0, v0, k1, v1, m, 32, 32 + bits_for(g->n_v ? g->n_v - 1 : 0), ws,
                                                &kr, &vr)) != PB_OK)
                    break;
                hipLaunchKernelGGL(k_split_sorted, dim3(grid_for(m)), dim3(256), 0, s, (const uint64_t *)kr,
                                   (const uint32_t *)vr, m, g->v_adj, g->v_eid);
                hipLaunchKernelGGL(k_voff_from_sorted, dim3(grid_for(m + 1)), dim3(256), 0, s, (const uint64_t *)kr, m,
                                   g->n_v, (const uint32_t *)flags, g->v_off);
            }
            hipLaunchKernelGGL(k_degrees, dim3(grid_for(n, 256, DEG_GRID)), dim3(256), 0, s, g->u_off, g->v_off,
                               g->n_u, g->n_v, g->deg, flags + 1);
            if (hipGetLastError() != hipSuccess) { st = PB_ERR_HIP; break; }
            if (hipMemcpyAsync(hflags, flags, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                st = PB_ERR_HIP;
                break;
            }
            if (hflags[0] & BAD_OFFSETS) st = PB_ERR_ID_RANGE;
            else if (hflags[0] & BAD_ID) st = PB_ERR_ID_RANGE;
            else if (hflags[0] & NOT_INCREASING) st = PB_ERR_NOT_SIMPLE;
            g->max_deg = hflags[1];
        } while (0);
    }
    if (hflags) (void)hipHostFree(hflags);
    if (st != PB_OK) {
        (void)hipStreamSynchronize(s);
        pb_graph_destroy(g);
        return st;
    }
    *out = g;
    return PB_OK;
}

void pb_graph_destroy(pb_graph *g) {
    if (!g) return;
    (void)hipDeviceSynchronize();
    // after the device-wide wait nothing uses the arrays: back to the
    // library's scratch cache of the device they came from
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != g->device) (void)hipSetDevice(g->device);
    for (uint32_t *p : {g->eu, g->v_off, g->v_adj, g->v_eid, g->deg}) scratch_put(nullptr, p);
    if (cur != g->device) (void)hipSetDevice(cur);
    delete g;
}

pb_status pb_rank(pb_graph *g, pb_rank_kind kind, uint32_t *rank, hipStream_t s) {
    if (!g || !rank) return PB_ERR_INVALID_ARG;
    const uint64_t n = (uint64_t)g->n_u + g->n_v;
    if (n == 0) return PB_OK;
    switch (kind) {
        case PB_RANK_SIDE_AUTO:
        case PB_RANK_SIDE_U_FIRST:
        case PB_RANK_SIDE_V_FIRST: {
            Workspace ws(s, 0);
            unsigned long long *sums = ws.alloc<unsigned long long>(2);
            if (!sums) return PB_ERR_NO_MEMORY;
            PB_TRY(fill<uint64_t>((uint64_t *)sums, 0ull, 2, s));
            if (kind == PB_RANK_SIDE_AUTO)
                hipLaunchKernelGGL(k_side_sums, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, g->deg, g->n_u, g->n_v, sums);
            const int mode = kind == PB_RANK_SIDE_U_FIRST ? 0 : kind == PB_RANK_SIDE_V_FIRST ? 1 : 2;
            hipLaunchKernelGGL(k_side_rank, dim3(grid_for(n)), dim3(256), 0, s, g->n_u, g->n_v, mode, sums, rank);
            PB_TRY_HIP(hipGetLastError());
            return PB_OK;
        }
        case PB_RANK_DEGREE:
        case PB_RANK_APPROX_DEGREE: {
            const bool approx = kind == PB_RANK_APPROX_DEGREE;
            const uint32_t max_key = approx ? 32u : g->max_deg;
            const int idbits = bits_for(n - 1);
            const int nbits = idbits + bits_for(max_key);
            Workspace ws(s, 0);
            uint64_t *k0 = ws.alloc<uint64_t>(n), *k1 = ws.alloc<uint64_t>(n);
            uint32_t *v0 = ws.alloc<uint32_t>(n), *v1 = ws.alloc<uint32_t>(n);
            if (ws.failed) return PB_ERR_NO_MEMORY;
            hipLaunchKernelGGL(k_order_keys, dim3(grid_for(n)), dim3(256), 0, s, g->deg, n, (int)approx, max_key,
                               idbits, k0, v0);
            PB_TRY_HIP(hipGetLastError());
            uint64_t *kr;
            uint32_t *vr;
            PB_TRY(radix_sort_pairs(k0, v0, k1, v1, n, nbits, ws, &kr, &vr));
            hipLaunchKernelGGL(k_scatter_rank, dim3(grid_for(n)), dim3(256), 0, s, vr, n, rank);
            PB_TRY_HIP(hipGetLastError());
            return PB_OK;
        }
        case PB_RANK_COMPLEMENT_CORENESS:
            return rank_codeg_exact(g, rank, s);
        case PB_RANK_APPROX_COMPLEMENT_CORENESS:
            return rank_codeg(g, true, rank, s);
    }
    return PB_ERR_INVALID_ARG;
}

}  // extern "C"
