// Butterfly counting: relabel by rank, plan, wedge retrieval + aggregation,
// butterfly credit, output combine.
//
// Paper map (arXiv 1907.08607):
//   relabel + modified degrees   Algorithm 1 (PREPROCESS), Section 4.3
//   wedge retrieval              Algorithm 2 (GET-WEDGES), Section 4.4.1
//   wedge aggregation            GET-FREQ, Sections 3.1.2 and 4.2.1
//   butterfly credit             Section 3.1.3, Algorithms 3 (COUNT-V) and 4 (COUNT-E)
//
// Layout after relabelling.  Vertices are renamed to their rank r.  N(r) is
// stored at nbr[roff[r] .. roff[r+1]) sorted by decreasing rank, so the
// neighbours ranked above r form the prefix of length hideg[r] (the modified
// degree deg_r(r) of Section 4.3).  A neighbour is stored by its side-major id
// (smid): U vertices in rank order take 0..n_u-1, V vertices n_u..n-1; within
// one side smid increases with rank, so every list is also sorted by
// decreasing smid and an smid range of candidate endpoints is a contiguous
// part of each list.
//   For each "up-slot" (r -> y, rank y > r) the run N(y)[0 .. pos) with
// pos = position of r in N(y) = deg_r(y) holds exactly the second endpoints
// x2 with rank x2 > r (Algorithm 2 inner loop).  Up-slots of r are numbered
// upoff[r] .. upoff[r+1]; uprun[k] = roff[y], uplen[k] = pos.
#include "pb_internal.h"

#include <algorithm>
#include <mutex>

using namespace pb;

namespace {

enum : int { MODE_GLOBAL = 1, MODE_VERTEX = 2, MODE_EDGE = 4 };
enum : uint32_t { FLAG_BAD_RANK = 1u, FLAG_INTERNAL = 2u };

constexpr uint32_t EMPTY = 0xFFFFFFFFu;

inline uint32_t grid_for(uint64_t n, uint32_t block = 256, uint32_t cap = 65536) {
    uint64_t g = (n + block - 1) / block;
    if (g == 0) g = 1;
    return (uint32_t)(g > cap ? cap : g);
}

#define GRID_STRIDE(i, n)                                                           \
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
         i += (uint64_t)gridDim.x * blockDim.x)

// ---------------------------------------------------------------- relabel

__global__ void k_rank_check(const uint32_t *rank, uint64_t n, uint32_t *order, uint32_t *seen,
                             uint32_t *flags, uint32_t *top) {
    GRID_STRIDE(x, n) {
        const uint32_t r = rank[x];
        if (r >= n) { atomicOr(flags, FLAG_BAD_RANK); continue; }
        if (atomicAdd(&seen[r], 1u) != 0) atomicOr(flags, FLAG_BAD_RANK);
        order[r] = (uint32_t)x;
        if (r == 0) *top = (uint32_t)x;
    }
}

__global__ void k_rank_side(const uint32_t *order, const uint32_t *deg, uint64_t n, uint32_t n_u,
                            uint32_t *isv, uint32_t *rdeg) {
    GRID_STRIDE(r, n) {
        const uint32_t x = order[r];
        isv[r] = x >= n_u;
        rdeg[r] = deg[x];
    }
}

__global__ void k_smid(const uint32_t *isv, const uint32_t *vbefore, uint64_t n, uint32_t n_u,
                       uint32_t *smid) {
    GRID_STRIDE(r, n) smid[r] = isv[r] ? n_u + vbefore[r] : (uint32_t)r - vbefore[r];
}

// Two directed slots per edge e: value 2e (U -> V) and 2e+1 (V -> U).  Key =
// source rank in the high bits, complemented destination rank in the low bits,
// so ascending keys give rows in rank order with neighbours by decreasing rank.
__global__ void k_slot_keys(const uint32_t *eu, const uint32_t *u_adj, const uint32_t *rank, uint64_t m,
                            uint32_t n_u, int b, uint64_t *keys, uint32_t *vals) {
    const uint64_t mask = (uint64_t(1) << b) - 1;
    GRID_STRIDE(e, m) {
        const uint64_t ru = rank[eu[e]], rv = rank[n_u + u_adj[e]];
        keys[2 * e] = (ru << b) | (mask - rv);
        keys[2 * e + 1] = (rv << b) | (mask - ru);
        vals[2 * e] = (uint32_t)(2 * e);
        vals[2 * e + 1] = (uint32_t)(2 * e + 1);
    }
}

// Destination-major slot keys for one graph: destinations in decreasing rank
// order, each followed by its slots (x -> y) for every neighbour x, taken
// from y's row of its own side's CSR.  Row of destination rank d starts at
// 2m - roff[d + 1].  A stable sort of these keys on the source-rank bits alone
// then leaves every row in decreasing neighbour rank, as the full key
// (source rank, complemented destination rank) requires.
struct DestRows {
    const uint32_t *order, *roff, *rank;
    const int64_t *u_off;
    const uint32_t *u_adj, *v_off, *v_adj, *v_eid;
    uint32_t n_u;
    uint64_t ns;
    int b;
};
constexpr uint32_t DEST_SMALL = 64;    // rows up to this long: one thread each
constexpr uint32_t DEST_CHUNK = 2048;  // longer rows: items of this many entries
constexpr uint32_t DEST_GRID = 4096;

__device__ inline void dest_entries(const DestRows &D, uint32_t d, uint64_t j0, uint64_t j1, uint64_t *keys,
                                    uint32_t *vals, uint32_t stride) {
    const uint64_t mask = (uint64_t(1) << D.b) - 1;
    const uint32_t y = D.order[d];
    const uint64_t q0 = D.ns - D.roff[d + 1];
    const uint64_t low = mask - d;
    if (y < D.n_u) {
        const int64_t e0 = D.u_off[y];
        for (uint64_t j = j0; j < j1; j += stride) {
            const uint64_t e = (uint64_t)e0 + j;
            keys[q0 + j] = ((uint64_t)D.rank[D.n_u + D.u_adj[e]] << D.b) | low;
            vals[q0 + j] = (uint32_t)(2 * e + 1);  // slot (v -> u)
        }
    } else {
        const uint32_t p0 = D.v_off[y - D.n_u];
        for (uint64_t j = j0; j < j1; j += stride) {
            const uint32_t p = p0 + (uint32_t)j;
            keys[q0 + j] = ((uint64_t)D.rank[D.v_adj[p]] << D.b) | low;
            vals[q0 + j] = 2 * D.v_eid[p];  // slot (u -> v)
        }
    }
}

// Short rows: a wave takes 64 consecutive destination ranks, lays their
// entries end to end and deals them to its lanes in order, so every store
// covers consecutive positions (a thread per row would leave most lanes idle
// behind the longest row and scatter each store).  cnt = items of the long
// rows, which this kernel leaves to k_dest_long.  Slot ids, positions and
// row offsets are below 2m < 2^32.
__global__ __launch_bounds__(256) void k_dest_small(DestRows D, uint64_t n, uint64_t *keys, uint32_t *vals,
                                                    uint32_t *cnt) {
    const uint32_t lane = threadIdx.x & (WAVE - 1);
    const uint64_t mask = (uint64_t(1) << D.b) - 1;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w0 = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(WAVE - 1)); w0 < n; w0 += stride) {
        const uint64_t d = w0 + lane;
        uint32_t len = 0, y = 0, q0 = 0, src = 0;  // row length, vertex, first position, first CSR entry
        if (d < n) {
            len = D.roff[d + 1] - D.roff[d];
            cnt[d] = len > DEST_SMALL ? (len + DEST_CHUNK - 1) / DEST_CHUNK : 0u;
            if (len > DEST_SMALL) len = 0;
            y = D.order[d];
            q0 = (uint32_t)(D.ns - D.roff[d + 1]);
            src = y < D.n_u ? (uint32_t)D.u_off[y] : D.v_off[y - D.n_u];
        }
        const uint32_t incl = wave_inclusive_sum(len);
        const uint32_t total = __builtin_amdgcn_readfirstlane(__shfl(incl, WAVE - 1, WAVE));
        for (uint32_t t = 0; t < total; t += WAVE) {
            const uint32_t f = t + lane;
            // the row holding flat entry f: the first lane whose inclusive sum exceeds f
            uint32_t i = 0;
#pragma unroll
            for (uint32_t step = WAVE / 2; step; step >>= 1)
                if (__shfl(incl, (int)(i + step - 1), WAVE) <= f) i += step;
            const uint32_t ii = i < WAVE ? i : WAVE - 1;
            const uint32_t j = f - (__shfl(incl, (int)ii, WAVE) - __shfl(len, (int)ii, WAVE));
            const uint32_t yi = __shfl(y, (int)ii, WAVE);
            const uint32_t q = __shfl(q0, (int)ii, WAVE) + j;
            const uint32_t e = __shfl(src, (int)ii, WAVE) + j;
            const uint64_t low = mask - (w0 + ii);
            if (f < total) {
                if (yi < D.n_u) {
                    keys[q] = ((uint64_t)D.rank[D.n_u + D.u_adj[e]] << D.b) | low;
                    vals[q] = 2 * e + 1;  // slot (v -> u)
                } else {
                    keys[q] = ((uint64_t)D.rank[D.v_adj[e]] << D.b) | low;
                    vals[q] = 2 * D.v_eid[e];  // slot (u -> v)
                }
            }
        }
    }
}

// Long rows: item `it` belongs to destination rank d with coff[d] <= it < coff[d + 1];
// each workgroup takes a contiguous share of the items.
__global__ void k_dest_long(DestRows D, uint64_t n, const uint32_t *coff, uint64_t *keys, uint32_t *vals) {
    uint32_t i0, i1;
    item_share(coff[n], blockIdx.x, gridDim.x, &i0, &i1);
    rows_of_items(coff, n, i0, i1, [&](uint32_t d, uint32_t it) {
        const uint64_t len = D.roff[d + 1] - D.roff[d];
        const uint64_t j0 = (uint64_t)(it - coff[d]) * DEST_CHUNK;
        const uint64_t j1 = j0 + DEST_CHUNK < len ? j0 + DEST_CHUNK : len;
        dest_entries(D, d, j0 + threadIdx.x, j1, keys, vals, blockDim.x);
    });
}

// Position of each slot in the ranked CSR: slot 2e (u -> v of edge e) at
// eslot[e], slot 2e + 1 (v -> u) at eslot[m + e], so a U row's edges, which
// are consecutive input edges, write and read consecutive words.
__device__ inline uint64_t eslot_at(uint32_t slot, uint64_t m) { return (slot & 1u) * m + (slot >> 1); }

__global__ void k_slots(const uint64_t *keys, const uint32_t *vals, uint64_t ns, int b, const uint32_t *smid,
                        const uint32_t *roff, uint32_t *nbr, uint32_t *eslot, uint32_t *hideg) {
    const uint64_t mask = (uint64_t(1) << b) - 1;
    GRID_STRIDE(p, ns) {
        const uint64_t key = keys[p];
        const uint32_t r = (uint32_t)(key >> b);
        const uint32_t d = (uint32_t)(mask - (key & mask));
        nbr[p] = smid[d];
        eslot[eslot_at(vals[p], ns >> 1)] = (uint32_t)p;
        if (d > r) {
            bool last_up = p + 1 == ns;
            if (!last_up) {
                const uint64_t k2 = keys[p + 1];
                const uint32_t r2 = (uint32_t)(k2 >> b);
                const uint32_t d2 = (uint32_t)(mask - (k2 & mask));
                last_up = r2 != r || d2 < r;
            }
            if (last_up) hideg[r] = (uint32_t)(p + 1 - roff[r]);
        }
    }
}

__global__ void k_upslots(const uint64_t *keys, const uint32_t *vals, uint64_t ns, int b, const uint32_t *roff,
                          const uint32_t *upoff, const uint32_t *eslot, uint32_t *uprun, uint32_t *uplen) {
    const uint64_t mask = (uint64_t(1) << b) - 1;
    GRID_STRIDE(p, ns) {
        const uint64_t key = keys[p];
        const uint32_t r = (uint32_t)(key >> b);
        const uint32_t d = (uint32_t)(mask - (key & mask));
        if (d > r && p - roff[r] < upoff[r + 1] - upoff[r]) {
            const uint32_t k = upoff[r] + (uint32_t)(p - roff[r]);
            const uint32_t rev = eslot[eslot_at(vals[p] ^ 1u, ns >> 1)];  // slot (d -> r)
            uprun[k] = roff[d];
            uplen[k] = rev - roff[d];
        }
    }
}

// Up-slots of the cache-optimised order: every slot (u -> y) is an up-slot
// (so up-slot k is slot k), and its run is the suffix of N(y) holding the
// neighbours ranked before both y and u (N(y) is by decreasing rank, so
// those come last): q = min(deg y - hideg y, deg y - pos - 1) entries, pos =
// the position of u in N(y).
__global__ void k_upslots_copt(const uint64_t *keys, const uint32_t *vals, uint64_t ns, int b, const uint32_t *roff,
                               const uint32_t *hideg, const uint32_t *eslot, uint32_t *uprun, uint32_t *uplen) {
    const uint64_t mask = (uint64_t(1) << b) - 1;
    GRID_STRIDE(p, ns) {
        const uint64_t key = keys[p];
        const uint32_t d = (uint32_t)(mask - (key & mask));
        const uint32_t pos = eslot[eslot_at(vals[p] ^ 1u, ns >> 1)] - roff[d];  // slot (d -> u) within N(d)
        const uint32_t degy = roff[d + 1] - roff[d];
        const uint32_t before_y = degy - hideg[d], before_u = degy - pos - 1;
        const uint32_t q = before_y < before_u ? before_y : before_u;
        uprun[p] = roff[d] + degy - q;
        uplen[p] = q;
    }
}

// cache-optimised order: the candidates of source r are the smids before its own
__global__ void k_cend_copt(const uint32_t *smid, uint64_t n, uint32_t *cend) {
    GRID_STRIDE(r, n) cend[r] = smid[r];
}

// Narrow windows: R(x1, x2) <= deg(x2), so above the largest id of a side
// with degree >= 256 every count fits 8 bits, and above the largest with
// degree >= 16, 4 bits.  from[0] / from[1] (U / V side, 8-bit) and from[2] /
// from[3] (4-bit), holding the side's first id on entry, become one past those
// ids.
// One atomic per workgroup and threshold: the maxima are reduced in the
// workgroup first.
__global__ __launch_bounds__(256) void k_byte_from(const uint32_t *rank, const uint32_t *smid, const uint32_t *deg,
                                                   uint64_t n, uint32_t n_u, uint32_t *from) {
    __shared__ uint32_t tmp[4][256 / WAVE];
    uint32_t mx[4] = {0u, 0u, 0u, 0u};  // 8-bit U, 8-bit V, 4-bit U, 4-bit V
    GRID_STRIDE(x, n) {
        const uint32_t d = deg[x];
        if (d >= 16) {
            const uint32_t sm = smid[rank[x]];
            const uint32_t side = sm < n_u ? 0 : 1;
            if (sm + 1 > mx[2 + side]) mx[2 + side] = sm + 1;
            if (d >= 256 && sm + 1 > mx[side]) mx[side] = sm + 1;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t v = mx[q];
        for (int dd = WAVE / 2; dd >= 1; dd >>= 1) {
            const uint32_t o = __shfl_xor(v, dd, WAVE);
            v = o > v ? o : v;
        }
        if ((threadIdx.x & (WAVE - 1)) == 0) tmp[q][threadIdx.x / WAVE] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        uint32_t v = 0;
        for (int i = 0; i < 256 / WAVE; ++i) v = tmp[threadIdx.x][i] > v ? tmp[threadIdx.x][i] : v;
        if (v) atomicMax(&from[threadIdx.x], v);
    }
}

// ---------------------------------------------------------------- plan

// Work lists: every source with wedges goes to exactly one.
enum : int {
    L_HASH_LIGHT = 0,  // 1-wave LDS hash, distinct bound <= 512
    L_HASH_MEDIUM,     // 256-thread LDS hash, distinct bound <= 4096
    L_HASH_WIN,        // 256-thread LDS hash over candidate windows of HASH_WIN ids
    L_SORT_LIGHT,      // 1-wave LDS radix sort, <= 512 wedges
    L_SORT_MEDIUM,     // 256-thread LDS radix sort, <= 2048 wedges
    L_SORT_HEAVY,      // 256-thread LDS radix sort over candidate windows
    L_DENSE_HEAVY,     // 1024-thread dense LDS windows swept with cursors
    L_DENSE_SMALL,     // 256-thread dense counters, candidate range <= 4096
    L_DENSE_GLOBAL,    // giant sources: dense histogram in global scratch, split over workgroups
    L_HASH_PACKED,     // 1024-thread packed LDS hash: few wedges over a wide candidate range
    NLISTS
};
constexpr int NSORTED = 5;  // lists dispatched most-wedges-first
__host__ __device__ inline int sorted_slot(int list) {
    return list == L_HASH_WIN ? 0 : list == L_SORT_HEAVY ? 1 : list == L_DENSE_HEAVY ? 2
                                  : list == L_DENSE_GLOBAL ? 3 : list == L_HASH_PACKED ? 4 : -1;
}

constexpr uint32_t LIGHT_D = 512;       // 1-wave hash: 1024 slots
constexpr uint32_t MEDIUM_D = 4096;     // 256-thread hash: 8192 slots
constexpr uint32_t SMALL_WIN = 4096;    // dense range of the 256-thread whole-range dense kernel
constexpr uint32_t WIN_WORDS = 32704;   // about 128 KB of LDS counters in the heavy dense kernel
constexpr uint32_t HASH_WIN = 4096;     // candidate window of a hash item over a heavy source
constexpr uint32_t SORT_LIGHT_W = 512;  // wedges sorted by the 1-wave sort kernel
constexpr uint32_t SORT_W = 2048;       // wedges sorted by the 256-thread sort kernels
// A dense-aggregated source with this many up-slots would be one long serial
// chain in a single workgroup; it gets a histogram in global scratch instead,
// with its up-slots split into items of GH_CHUNK over many workgroups.
constexpr uint32_t GH_MIN_UPS = 65536;
constexpr uint32_t GH_CHUNK = 8192;
constexpr uint32_t GH_SEG = 65536;      // histogram entries per endpoint-step item
constexpr uint32_t NXCD = 8;            // accelerator complex dies; workgroup b runs on die b % NXCD
constexpr uint32_t GH_WG_PER_XCD = 256;  // of 256 threads (the walk: that many threads per die)
constexpr int GH_T = 256;               // workgroup size of the giant-source walk

// Aggregator per bucket of the distinct-endpoint bound (light, medium, heavy),
// the workgroup size of the light and medium buckets' kernels (hash, sort,
// and for medium also the whole-range dense kernel) and each bucket's batch
// width: the workgroups one launch keeps in flight, each taking items until
// the list is done (0 = one workgroup per item).
struct Policy {
    uint32_t light_max, medium_max;
    int agg[3];
    bool packed;  // AUTO: heavy-bucket sources with few wedges may take the packed hash
    uint32_t wg[2] = {64, 256};
    uint32_t width[3] = {0, 0, 0};
};

// Workgroup sizes each bucket's kernels are built for.
__host__ __device__ inline bool light_wg_ok(uint32_t t) { return t == 64 || t == 128 || t == 256; }
__host__ __device__ inline bool medium_wg_ok(uint32_t t) { return t == 128 || t == 256 || t == 512; }

constexpr uint32_t PH_T = 1024;                   // threads of a packed-hash workgroup
constexpr uint32_t PH_SLOTS = 32768;              // packed hash: 128 KB of LDS
constexpr uint32_t PH_FULL = PH_SLOTS / 4 * 3;    // keys at which a window is refused and narrowed
constexpr uint32_t PH_TARGET = PH_SLOTS / 8 * 3;  // keys a window is sized for
// Sources with at most PH_ONE_WINDOW wedges, or sparser than PH_DENSITY
// wedges per candidate, take packed-hash windows sized to their wedges
// instead of dense windows sized to the LDS.
constexpr uint32_t PH_ONE_WINDOW = 16384;
constexpr double PH_DENSITY = 0.05;

__host__ __device__ inline uint32_t bit_width(uint32_t x) {
    uint32_t b = 0;
    while (b < 32 && (x >> b)) ++b;
    return b;
}

struct PlanCounts {
    uint32_t list[NLISTS];
    uint32_t items;  // hash (source, window) items
    uint32_t flags;
    uint32_t top;    // unified id of the rank-0 vertex
    uint32_t hub_items;  // (hub, up-slot chunk) items of the hub credit pass
    unsigned long long sources;
    unsigned long long wedges[NLISTS];
    HubCounters hub;
};

// First candidate endpoint id of a source with side-major id s: s + 1, or the
// end of the hub range for a hub (its hub partners are counted by the tile).
__host__ __device__ inline uint32_t cand_lo(uint32_t s, uint32_t hub_base, uint32_t hub_end) {
    return (s >= hub_base && s < hub_end) ? hub_end : s + 1;
}

// Hub sources lose the wedges of their hub partners (counted by the tile).
// List slots and totals are reserved per block (LDS atomics, then one global
// atomic per list per block), so no global counter sees one atomic per source.
constexpr uint32_t PLAN_GRID = 2048;
__global__ __launch_bounds__(256) void k_plan(const uint32_t *upoff, const uint64_t *wscan, const uint32_t *smid,
                                              const uint32_t *cend, uint64_t n, Policy pol, uint32_t hub_base,
                                              uint32_t hub_end, const unsigned long long *roww, uint32_t *lists,
                                              uint32_t *nwin, uint64_t *wl, PlanCounts *pc, uint32_t copt_nu) {
    __shared__ uint32_t cnt[NLISTS], base[NLISTS], s_items;
    __shared__ unsigned long long wsum[NLISTS], s_sources;
    if (!pc->hub.on) hub_end = hub_base;
    const uint32_t tid = threadIdx.x;
    for (uint64_t b0 = (uint64_t)blockIdx.x * 256; b0 < n; b0 += (uint64_t)gridDim.x * 256) {
        if (tid < NLISTS) {
            cnt[tid] = 0;
            wsum[tid] = 0;
        }
        if (tid == 0) {
            s_items = 0;
            s_sources = 0;
        }
        __syncthreads();
        const uint64_t r = b0 + tid;
        int which = -1;
        uint32_t local = 0, nw = 1, range = 0;
        uint64_t w = 0;
        if (r < n) {
            const uint32_t sm = smid[r];
            w = wscan[upoff[r + 1]] - wscan[upoff[r]];
            if (sm >= hub_base && sm < hub_end) w -= roww[sm - hub_base];
            const uint32_t lo = copt_nu ? (sm < copt_nu - 1 ? 0u : copt_nu - 1) : cand_lo(sm, hub_base, hub_end);
            if (w != 0 && lo < cend[r]) {
                range = cend[r] - lo;
                const uint64_t dist = w < range ? w : range;
                const int bucket = dist <= pol.light_max ? 0 : dist <= pol.medium_max ? 1 : 2;
                switch (pol.agg[bucket]) {
                    case PB_AGG_LDS_HASH:  // the policy keeps light_max <= 512 and medium_max <= 4096
                        which = bucket == 0 ? L_HASH_LIGHT : bucket == 1 ? L_HASH_MEDIUM : L_HASH_WIN;
                        break;
                    case PB_AGG_RADIX_SORT:
                        which = w <= SORT_LIGHT_W ? L_SORT_LIGHT : w <= SORT_W ? L_SORT_MEDIUM : L_SORT_HEAVY;
                        break;
                    default: {
                        const uint32_t ups = upoff[r + 1] - upoff[r];
                        which = range <= SMALL_WIN    ? L_DENSE_SMALL
                                : ups >= GH_MIN_UPS ? L_DENSE_GLOBAL
                                                    : L_DENSE_HEAVY;
                        // few wedges over a wide range: packed-hash windows
                        // sized to the wedges instead of many dense windows
                        if (which == L_DENSE_HEAVY && pol.packed &&
                            (w <= PH_ONE_WINDOW || (double)w < PH_DENSITY * range) &&
                            bit_width(range) + bit_width(ups) <= 32)
                            which = L_HASH_PACKED;
                        break;
                    }
                }
                local = atomicAdd(&cnt[which], 1u);
                atomicAdd(&wsum[which], (unsigned long long)w);
                atomicAdd(&s_sources, 1ull);
                if (which == L_HASH_WIN) {
                    nw = (range + HASH_WIN - 1) / HASH_WIN;
                    atomicAdd(&s_items, nw);
                }
            }
        }
        __syncthreads();
        if (tid < NLISTS && cnt[tid]) {
            base[tid] = atomicAdd(&pc->list[tid], cnt[tid]);
            atomicAdd(&pc->wedges[tid], wsum[tid]);
        }
        if (tid == 0) {
            if (s_sources) atomicAdd(&pc->sources, s_sources);
            if (s_items) atomicAdd(&pc->items, s_items);
        }
        __syncthreads();
        if (which >= 0) {
            const uint32_t slot = base[which] + local;
            lists[(uint64_t)which * n + slot] = (uint32_t)r;
            const int sk = sorted_slot(which);
            if (sk >= 0) {
                nwin[(uint64_t)sk * n + slot] = nw;
                wl[(uint64_t)sk * n + slot] = w;
            }
        }
        __syncthreads();  // cnt and base are reset by the next round
    }
}

// Sort key: most wedges per item first (longest items are dispatched first).
__global__ void k_heavy_keys(const uint32_t *nwin, const uint64_t *w, uint32_t nh, uint64_t *keys, uint32_t *vals) {
    GRID_STRIDE(i, (uint64_t)nh) {
        uint64_t per = w[i] / nwin[i];
        if (per > 0xFFFFFFFFull) per = 0xFFFFFFFFull;
        keys[i] = 0xFFFFFFFFull - per;
        vals[i] = (uint32_t)i;
    }
}

__global__ void k_heavy_gather(const uint32_t *perm, const uint32_t *heavy, const uint32_t *nwin, const uint64_t *w,
                               uint32_t nh, uint32_t *src_sorted, uint32_t *nwin_sorted, uint64_t *w_sorted) {
    GRID_STRIDE(i, (uint64_t)nh) {
        src_sorted[i] = heavy[perm[i]];
        nwin_sorted[i] = nwin[perm[i]];
        w_sorted[i] = w[perm[i]];
    }
}

// hash items: x = source rank, y = window index
__global__ void k_heavy_expand(const uint32_t *src_sorted, const uint32_t *nwin_sorted, const uint32_t *ioff,
                               uint32_t nh, uint2 *items) {
    GRID_STRIDE(i, (uint64_t)nh) {
        const uint32_t o = ioff[i];
        for (uint32_t j = 0; j < nwin_sorted[i]; ++j) items[o + j] = make_uint2(src_sorted[i], j);
    }
}

// Largest j < ng with base[j] <= x (base non-decreasing, base[0] <= x).
template <class T>
__device__ inline uint32_t graph_of(const T *base, uint32_t ng, T x) {
    uint32_t lo = 0, hi = ng;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (base[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// Candidate range end of each rank (its own side of its own graph) and, for a
// batch, the graph of each rank.  Ranks are graph-blocked in a batch, so a
// graph's U (V) vertices hold a contiguous block of side-major ids.
__global__ void k_cend(const uint32_t *isv, uint64_t n, uint32_t n_u, uint32_t ng, const uint32_t *rbase,
                       const uint32_t *ubase, const uint32_t *vbase, uint32_t *cend, uint32_t *gid) {
    GRID_STRIDE(r, n) {
        if (ng <= 1) {
            cend[r] = isv[r] ? (uint32_t)n : n_u;
        } else {
            const uint32_t j = graph_of<uint32_t>(rbase, ng, (uint32_t)r);
            gid[r] = j;
            cend[r] = isv[r] ? n_u + vbase[j + 1] : ubase[j + 1];
        }
    }
}

// ---------------------------------------------------------------- counting

struct Ranked {
    const uint32_t *roff, *nbr, *upoff, *uprun, *uplen, *smid;
    const uint32_t *cend;  // per rank: end of its candidate id range (its side of its graph)
    const uint32_t *gid;   // per rank: its graph in a batch (null: one graph)
    uint32_t n_u, n;
    uint32_t hub_base, hub_end;  // side-major ids of the hub tile's vertices (empty: no tile)
    bool copt;                   // cache-optimised order: candidates are the smids before the source's
    // first candidate endpoint id of source r
    __device__ uint32_t lo(uint32_t r) const {
        if (copt) return smid[r] < n_u ? 0u : n_u;
        return cand_lo(smid[r], hub_base, hub_end);
    }
};

struct Acc {
    unsigned long long *g;  // one per graph
    unsigned long long *v;  // n, by smid
    unsigned long long *s;  // 2m, by slot (64-bit slot credits)
    uint32_t *s32;          // 2m, by slot, when every slot's credit fits 32 bits
    uint32_t *err;          // internal-consistency flag
    int mode;
    __device__ int passes() const { return (mode & (MODE_VERTEX | MODE_EDGE)) ? 2 : 1; }
    __device__ void slot_add(uint32_t p, unsigned long long d) const {
        if (s32) atomicAdd(&s32[p], (uint32_t)d);
        else atomicAdd(&s[p], d);
    }
};

// Smallest i in [lo, len] with p[i] < v (p strictly decreasing, p[j] >= v for j < lo).
__device__ inline uint32_t first_below(const uint32_t *p, uint32_t lo, uint32_t len, uint32_t v) {
    uint32_t hi = len;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (p[mid] < v) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// Entries of zero padding after the ranked lists: vector reads of up to 20
// entries from any list position stay inside the allocation.
constexpr uint32_t NBR_PAD = 64;

// Smallest e in (s, len] with p[e] < v, where p = nbr + start is strictly
// decreasing, s < len and p[s] >= v; *pe = p[e] (0 when e == len).  The 16
// entries after s come in one round trip of aligned 16-byte loads: that
// settles every part of at most 16 entries.  A longer part reads the run's
// last entry (a part that runs to the end of the run is then settled), then
// gallops and narrows with two independent probes per round trip.  Every
// window repeats this for every run it meets, and the lines a probe reads
// past e are not the walk's, so probes are kept few: two per round took
// the heavy kernel's reads on the 50M-edge power-law graph from 236 GB to
// 213 GB and its time down by 4% against eight per round.
constexpr uint32_t PROBE_DIRECT = 81;  // remaining entries narrowed without galloping first
__device__ inline uint32_t probe_below(const uint32_t *nbr, uint32_t start, uint32_t s, uint32_t len, uint32_t v,
                                       uint32_t *pe) {
    const uint32_t a = start + s + 1;  // absolute index of p[s + 1]
    const uint32_t b = a & ~3u;
    uint32_t w[20];
    const uint4 *q = reinterpret_cast<const uint4 *>(nbr + b);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const uint4 c = q[i];
        w[4 * i] = c.x;
        w[4 * i + 1] = c.y;
        w[4 * i + 2] = c.z;
        w[4 * i + 3] = c.w;
    }
    const uint32_t lim = len - s - 1 < 16 ? len - s - 1 : 16u;  // entries after s that exist, up to 16
    uint32_t cnt = 0;
#pragma unroll
    for (int i = 0; i < 20; ++i) {
        const uint32_t rel = b + i - a;  // wraps to a huge value before p[s + 1]
        if (rel < lim && w[i] >= v) ++cnt;
    }
    if (cnt < lim) {
        uint32_t val = 0;
#pragma unroll
        for (int i = 0; i < 20; ++i)
            if (b + i - a == cnt) val = w[i];
        *pe = val;
        return s + 1 + cnt;
    }
    if (lim < 16) {  // the run ends within the 16: every entry after s is >= v
        *pe = 0;
        return len;
    }
    const uint32_t last = nbr[start + len - 1];  // the run's smallest entry
    if (last >= v) {
        *pe = 0;
        return len;
    }
    // answer in (x, y]; p[x] >= v; p[y] = yv < v
    uint32_t x = s + 16, y = len - 1, yv = last;
    if (y - x > PROBE_DIRECT)
        for (uint64_t scale = 16;; scale <<= 2) {  // x + 16, 32; then 64, 128; ...
            uint32_t qi[2], qv[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const uint64_t d = x + (scale << j);
                qi[j] = d < y ? (uint32_t)d : y;
                qv[j] = qi[j] < y ? nbr[start + qi[j]] : 0u;
            }
            bool found = false;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if (found) continue;
                if (qi[j] >= y || qv[j] < v) {
                    found = true;
                    if (qi[j] < y) {
                        y = qi[j];
                        yv = qv[j];
                    }
                } else {
                    x = qi[j];
                }
            }
            if (found) break;
        }
    while (y - x > 1) {  // two probes split the candidates x+1 .. y-1 in three
        const uint32_t wdt = y - x - 1;
        uint32_t nx = x, ny = y, nyv = yv;
#pragma unroll
        for (int j = 1; j <= 2; ++j) {
            const uint32_t qi = x + 1 + (uint32_t)(((uint64_t)wdt * j) / 3);
            const uint32_t qv = nbr[start + qi];
            if (qv >= v) {
                if (qi > nx) nx = qi;
            } else if (qi < ny) {
                ny = qi;
                nyv = qv;
            }
        }
        x = nx;
        y = ny;
        yv = nyv;
    }
    *pe = y < len ? yv : 0u;
    return y;
}

// Dense counters for the candidate window [lo, lo + size), 2^cs of them to a
// 32-bit word: 32-bit (cs 0), 16-bit (`half`, cs 1), 8-bit (`byte`, cs 2) or
// 4-bit (`nib`, cs 3).  A narrow width is used only where every count fits it.
template <int T>
struct DenseAgg {
    uint32_t *w;
    uint32_t lo, size;
    bool half;
    uint32_t *err;
    bool byte = false, nib = false;
    __device__ uint32_t cs() const { return nib ? 3u : byte ? 2u : half ? 1u : 0u; }
    __device__ void init() const {
        const uint32_t c = cs(), words = (size + (1u << c) - 1) >> c;
        for (uint32_t i = threadIdx.x; i < words; i += T) w[i] = 0;
    }
    __device__ void insert(uint32_t x) const {
        const uint32_t d = x - lo;
        if (d >= size) { atomicOr(err, FLAG_INTERNAL); return; }
        const uint32_t c = cs();
        atomicAdd(&w[d >> c], 1u << ((d & ((1u << c) - 1)) << (5 - c)));
    }
    __device__ bool finalize() const { return true; }
    __device__ uint32_t count(uint32_t x) const {
        const uint32_t d = x - lo;
        if (d >= size) return 1u;
        const uint32_t c = cs();
        const uint32_t v = w[d >> c] >> ((d & ((1u << c) - 1)) << (5 - c));
        return c ? v & ((1u << (32 >> c)) - 1) : v;
    }
    // Every non-zero counter, four words a thread per step: the four LDS
    // reads are issued before any is tested, so a window that is mostly
    // empty costs a quarter of the round trips.
    template <class F>
    __device__ void for_each(F f) const {
        const uint32_t c = cs(), per = 1u << c, bits = 32 >> c;
        const uint32_t mask = c ? (1u << bits) - 1 : 0xFFFFFFFFu;
        const uint32_t words = (size + per - 1) >> c;
        for (uint32_t i0 = threadIdx.x; i0 < words; i0 += 4 * T) {
            uint32_t v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = i0 + k * T < words ? w[i0 + k * T] : 0u;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (!v[k]) continue;
                const uint32_t i = i0 + k * T;
                for (uint32_t j = 0; j < per; ++j) {
                    const uint32_t cc = (v[k] >> (j * bits)) & mask;
                    if (cc) f(lo + i * per + j, cc);
                }
            }
        }
    }
};

// Linear-probing hash table keyed by x2 (capacity a power of two).
template <int T, int CAP>
struct HashAgg {
    uint32_t *keys, *cnts;
    uint32_t *err;
    __device__ static uint32_t slot(uint32_t x) { return (x * 2654435769u) >> (32 - __builtin_ctz(CAP)); }
    __device__ void init() const {
        for (uint32_t i = threadIdx.x; i < CAP; i += T) { keys[i] = EMPTY; cnts[i] = 0; }
    }
    // The planner sizes CAP to at least twice the distinct keys; a full table
    // (which the plan rules out) is reported instead of probed forever.
    __device__ void insert(uint32_t x) const {
        uint32_t h = slot(x);
        for (int probe = 0; probe < CAP; ++probe) {
            // one compare-and-swap both claims an empty slot and reads a taken one
            const uint32_t k = atomicCAS(&keys[h], EMPTY, x);
            if (k == EMPTY || k == x) { atomicAdd(&cnts[h], 1u); return; }
            h = (h + 1) & (CAP - 1);
        }
        atomicOr(err, FLAG_INTERNAL);
    }
    __device__ bool finalize() const { return true; }
    __device__ uint32_t count(uint32_t x) const {
        uint32_t h = slot(x);
        for (int probe = 0; probe < CAP; ++probe) {
            if (keys[h] == x) return cnts[h];
            h = (h + 1) & (CAP - 1);
        }
        return 1u;
    }
    // every key and its count, four slots a thread per step with the reads
    // issued before any is tested
    template <class F>
    __device__ void for_each(F f) const {
        for (uint32_t i0 = threadIdx.x; i0 < CAP; i0 += 4 * T) {
            uint32_t k[4], c[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool in = i0 + q * T < CAP;
                k[q] = in ? keys[i0 + q * T] : EMPTY;
                c[q] = in ? cnts[i0 + q * T] : 0u;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (k[q] != EMPTY) f(k[q], c[q]);
        }
    }
};

// Linear-probing hash of (candidate, count) packed into one word,
// (key + 1) << cbits | count with key = x2 - lo, 0 = empty.  Valid when
// bits(range) + cbits <= 32 and cbits = bits(up-slots): a count never
// exceeds the source's up-slots, since R(x1, x2) <= deg_x1(x1).
template <int T, int CAP, int FULL>
struct PackedHashAgg {
    uint32_t *w;
    uint32_t *keys;  // shared: keys inserted so far
    uint32_t lo, cbits;
    uint32_t *err;
    __device__ static uint32_t slot(uint32_t key) { return (key * 2654435769u) >> (32 - __builtin_ctz(CAP)); }
    __device__ void init() const {
        for (uint32_t i = threadIdx.x; i < CAP; i += T) w[i] = 0;
        if (threadIdx.x == 0) *keys = 0;
    }
    // A new key claims an empty slot by compare-and-swap (which also reads a
    // taken slot), and each call's new keys are counted with one atomic per
    // wave.  The walk skips a wave's inserts once FULL keys are in
    // (saturated(), read once per U x 64 wedges of the wave), so fewer than
    // FULL + T * U keys are ever in: with FULL + T * U <= CAP probing always
    // ends, and finalize() refuses a window that reached FULL, which the
    // caller narrows.
    __device__ void insert(uint32_t x) const {
        const uint32_t key = x - lo, tag = key + 1;
        uint32_t h = slot(key);
        bool fresh = false;
        int probe = 0;
        for (; probe < CAP; ++probe) {
            const uint32_t e = atomicCAS(&w[h], 0u, (tag << cbits) | 1u);
            if (e == 0) {
                fresh = true;
                break;
            }
            if ((e >> cbits) == tag) {
                atomicAdd(&w[h], 1u);
                break;
            }
            h = (h + 1) & (CAP - 1);
        }
        if (probe == CAP) atomicOr(err, FLAG_INTERNAL);
        const uint64_t nb = __ballot(fresh);
        if (nb && __lane_id() == (uint32_t)__ffsll((unsigned long long)__ballot(1)) - 1)
            atomicAdd(keys, (uint32_t)__popcll(nb));
    }
    __device__ bool saturated() const {
        return __builtin_amdgcn_readfirstlane(
                   __hip_atomic_load(keys, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) >= FULL;
    }
    // The inserts of U sub-tiles at once: the first probes of all of them are
    // issued back to back, so their LDS round trips overlap; a probe that meets
    // another key continues alone.  Call with the whole wave.
    template <int U>
    __device__ void insert_all(const uint32_t *x, const bool *ok) const {
        uint32_t h[U], v[U], e[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t key = x[u] - lo;
            h[u] = slot(key);
            v[u] = ((key + 1) << cbits) | 1u;
            e[u] = ok[u] ? atomicCAS(&w[h[u]], 0u, v[u]) : 0u;
        }
        uint32_t fresh = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!ok[u]) continue;
            if (e[u] == 0) {
                ++fresh;
                continue;
            }
            const uint32_t tag = v[u] >> cbits;
            uint32_t hh = h[u], ee = e[u];
            int probe = 1;
            while ((ee >> cbits) != tag && probe < CAP) {
                hh = (hh + 1) & (CAP - 1);
                ee = atomicCAS(&w[hh], 0u, v[u]);
                ++probe;
                if (ee == 0) break;
            }
            if (ee == 0) ++fresh;
            else if ((ee >> cbits) == tag) atomicAdd(&w[hh], 1u);
            else atomicOr(err, FLAG_INTERNAL);
        }
        const uint32_t total = wave_sum(fresh);
        if (total && __lane_id() == 0) atomicAdd(keys, total);
    }
    // count() of U sub-tiles, first probes issued back to back.
    template <int U>
    __device__ void count_all(const uint32_t *x, const bool *ok, uint32_t *c) const {
        uint32_t h[U], e[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            h[u] = slot(x[u] - lo);
            e[u] = ok[u] ? w[h[u]] : 0u;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c[u] = 1u;
            if (!ok[u]) continue;
            const uint32_t tag = x[u] - lo + 1;
            uint32_t hh = h[u], ee = e[u];
            for (int probe = 1; (ee >> cbits) != tag && ee != 0 && probe < CAP; ++probe) {
                hh = (hh + 1) & (CAP - 1);
                ee = w[hh];
            }
            if ((ee >> cbits) == tag) c[u] = ee & ((1u << cbits) - 1);
        }
    }
    __device__ bool finalize() const {
        __syncthreads();
        const bool ok = *keys < FULL;
        __syncthreads();  // everyone has read the count before anyone re-inits
        return ok;
    }
    __device__ uint32_t count(uint32_t x) const {
        const uint32_t key = x - lo, tag = key + 1;
        uint32_t h = slot(key);
        for (int probe = 0; probe < CAP; ++probe) {
            const uint32_t e = w[h];
            if ((e >> cbits) == tag) return e & ((1u << cbits) - 1);
            if (e == 0) break;
            h = (h + 1) & (CAP - 1);
        }
        return 1u;
    }
    template <class F>
    __device__ void for_each(F f) const {
        for (uint32_t i0 = threadIdx.x; i0 < CAP; i0 += 4 * T) {
            uint32_t e[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) e[q] = i0 + q * T < CAP ? w[i0 + q * T] : 0u;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (e[q]) f(lo + (e[q] >> cbits) - 1, e[q] & ((1u << cbits) - 1));
        }
    }
};

// Whether the walk should skip a wave's inserts: only a packed hash refuses
// keys.
template <class Agg>
__device__ inline bool saturated(const Agg &) { return false; }
template <int T, int CAP, int FULL>
__device__ inline bool saturated(const PackedHashAgg<T, CAP, FULL> &a) { return a.saturated(); }

// The inserts and count reads of a walk's U sub-tiles (ok[u]: lane holds a
// wedge of sub-tile u); the packed hash overlaps their first probes.
template <int U, class Agg>
__device__ inline void insert_all(const Agg &agg, const uint32_t *x, const bool *ok) {
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (ok[u]) agg.insert(x[u]);
}
template <int U, int T, int CAP, int FULL>
__device__ inline void insert_all(const PackedHashAgg<T, CAP, FULL> &agg, const uint32_t *x, const bool *ok) {
    agg.template insert_all<U>(x, ok);
}
template <int U, class Agg>
__device__ inline void count_all(const Agg &agg, const uint32_t *x, const bool *ok, uint32_t *c) {
#pragma unroll
    for (int u = 0; u < U; ++u) c[u] = ok[u] ? agg.count(x[u]) : 1u;
}
template <int U, int T, int CAP, int FULL>
__device__ inline void count_all(const PackedHashAgg<T, CAP, FULL> &agg, const uint32_t *x, const bool *ok,
                                 uint32_t *c) {
    agg.template count_all<U>(x, ok, c);
}

// Block-wide stable LSD radix sort of n 64-bit keys in LDS, 4 bits a pass
// over bits [0, nbits) (nbits a multiple of 8, so the result ends in `a`).
// Thread t owns the contiguous keys [t*S, (t+1)*S); its per-digit counts live
// in column t of cnt[16][T]; one block scan over cnt (digit-major) turns them
// into stable destinations.  Needs 16*T counters and T/WAVE+1 scan words.
template <int T>
__device__ void block_radix_sort(uint64_t *a, uint64_t *b, uint32_t n, int nbits, uint32_t *cnt, uint32_t *tmp) {
    const uint32_t tid = threadIdx.x;
    const uint32_t S = (n + T - 1) / T;
    const uint32_t beg = tid * S < n ? tid * S : n, end = beg + S < n ? beg + S : n;
    for (int shift = 0; shift < nbits; shift += 4) {
#pragma unroll
        for (int d = 0; d < 16; ++d) cnt[d * T + tid] = 0;
        __syncthreads();
        for (uint32_t i = beg; i < end; ++i) cnt[((a[i] >> shift) & 15u) * T + tid] += 1;
        __syncthreads();
        uint32_t v[16], sum = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            v[j] = cnt[16 * tid + j];
            sum += v[j];
        }
        uint32_t total;
        uint32_t run = block_exclusive_sum<T>(sum, tmp, &total);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            cnt[16 * tid + j] = run;
            run += v[j];
        }
        __syncthreads();
        for (uint32_t i = beg; i < end; ++i) {
            const uint64_t key = a[i];
            const uint32_t slot = ((key >> shift) & 15u) * T + tid;
            b[cnt[slot]] = key;
            cnt[slot] += 1;
        }
        __syncthreads();
        uint64_t *t = a;
        a = b;
        b = t;
    }
}

// Sort-based aggregation (GET-FREQ by sorting, Section 3.1.2): the wedges'
// keys x2 - lo are appended to an LDS buffer, radix-sorted, and each run of
// equal keys gives one endpoint pair and its count R.  A window of width 1
// needs no keys (every wedge has the same x2).  Over CAP keys the item is
// refused (finalize() returns false) and the caller narrows the window.
template <int T, int CAP>
struct SortAgg {
    uint64_t *a, *b;   // CAP keys each; after finalize b holds the distinct keys
    uint32_t *cnt;     // 16*T >= CAP: sort counters, then the count of each distinct key
    uint32_t *start;   // CAP: first sorted position of each distinct key
    uint32_t *meta;    // [0] keys appended, [1] distinct keys
    uint32_t *tmp;     // T/WAVE + 1
    uint32_t lo, width;
    __device__ void init() const {
        if (threadIdx.x == 0) { meta[0] = 0; meta[1] = 0; }
    }
    __device__ void insert(uint32_t x) const {
        const uint64_t act = __ballot(1);
        const uint32_t lane = threadIdx.x & (WAVE - 1);
        const uint32_t leader = __ffsll((unsigned long long)act) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&meta[0], (uint32_t)__popcll(act));
        base = __shfl(base, leader, WAVE);
        const uint32_t idx = base + (uint32_t)__popcll(act & lanemask_lt());
        if (width > 1 && idx < CAP) a[idx] = x - lo;
    }
    __device__ bool finalize() const {
        __syncthreads();
        const uint32_t n = meta[0];
        __syncthreads();  // everyone has n before anyone may return and re-init
        if (width == 1) {  // one candidate: R = number of wedges
            if (threadIdx.x == 0 && n) { b[0] = 0; cnt[0] = n; meta[1] = 1; }
            __syncthreads();
            return true;
        }
        if (n > CAP) return false;  // every thread read the same n
        int bits = 0;
        while (bits < 32 && ((width - 1) >> bits)) ++bits;
        bits = (bits + 7) & ~7;
        block_radix_sort<T>(a, b, n, bits, cnt, tmp);
        // distinct keys: thread-contiguous segments, flags scanned
        const uint32_t tid = threadIdx.x, S = (n + T - 1) / T;
        const uint32_t beg = tid * S < n ? tid * S : n, end = beg + S < n ? beg + S : n;
        uint32_t heads = 0;
        for (uint32_t i = beg; i < end; ++i) heads += (i == 0 || a[i] != a[i - 1]);
        uint32_t nu;
        uint32_t u = block_exclusive_sum<T>(heads, tmp, &nu);
        for (uint32_t i = beg; i < end; ++i)
            if (i == 0 || a[i] != a[i - 1]) { b[u] = a[i]; start[u] = i; ++u; }
        __syncthreads();
        for (uint32_t j = tid; j < nu; j += T) cnt[j] = (j + 1 < nu ? start[j + 1] : n) - start[j];
        if (tid == 0) meta[1] = nu;
        __syncthreads();
        return true;
    }
    __device__ uint32_t count(uint32_t x) const {
        const uint64_t key = width > 1 ? (uint64_t)(x - lo) : 0;
        uint32_t l = 0, h = meta[1];
        while (h - l > 1) {
            const uint32_t mid = (l + h) >> 1;
            if (b[mid] <= key) l = mid; else h = mid;
        }
        return cnt[l];
    }
    template <class F>
    __device__ void for_each(F f) const {
        const uint32_t nu = meta[1];
        for (uint32_t j = threadIdx.x; j < nu; j += T) f(lo + (uint32_t)b[j], cnt[j]);
    }
};

// Which part [a, a + cnt) of run k (up-slot k, run N(y)[0, pos) at nbr[start])
// an item covers, in each pass.
// The whole run, cut below `lo` for a hub source (whose hub partners sit at
// the end of each run).
struct FullRange {
    uint32_t lo;
    bool cut;
    __device__ void operator()(const Ranked &G, int, uint32_t, uint32_t start, uint32_t pos, uint32_t &a,
                               uint32_t &cnt) const {
        a = 0;
        cnt = cut ? first_below(G.nbr + start, 0, pos, lo) : pos;
    }
    __device__ void commit(uint32_t) const {}
};
__device__ inline FullRange full_range(const Ranked &G, uint32_t r) {
    const uint32_t lo = G.lo(r);
    return FullRange{lo, lo != G.smid[r] + 1};
}

// Candidate window [lo, hi): both ends by binary search.
struct SearchRange {
    uint32_t lo, hi;
    __device__ void operator()(const Ranked &G, int, uint32_t, uint32_t start, uint32_t pos, uint32_t &a,
                               uint32_t &cnt) const {
        a = first_below(G.nbr + start, 0, pos, hi);
        cnt = first_below(G.nbr + start, a, pos, lo) - a;
    }
    __device__ void commit(uint32_t) const {}
};

// Windows of one source taken from the highest ids down: each run's part in
// the window starts where its part in the previous window ended (cursor `cur`,
// one per up-slot) and ends at the first entry below lo.  The value at the
// cursor is kept beside it (`cval`, 0 once the run is used up), so a run with
// nothing in the window is recognised without reading the run; otherwise the
// end is found by galloping from the cursor.  Pass 1 stores the new cursor and
// its value in nxt/nval; pass 2 (or pass 1 when there is no pass 2) commits
// them, so a refused window leaves the cursors as they were.
struct CursorRange {
    uint32_t *cur, *nxt, *cval, *nval;
    uint32_t lo;
    bool first, two_pass;
    __device__ void operator()(const Ranked &G, int pass, uint32_t k, uint32_t start, uint32_t pos, uint32_t &a,
                               uint32_t &cnt) const {
        const uint32_t *p = G.nbr + start;
        uint32_t s, v;
        if (first) {
            s = 0;
            v = pos ? p[0] : 0u;
        } else {
            s = cur[k];
            v = cval[k];
        }
        uint32_t e;
        if (pass == 1) {
            e = s;
            uint32_t ev = v;
            if (s < pos && v >= lo) e = probe_below(G.nbr, start, s, pos, lo, &ev);
            if (two_pass) {
                nxt[k] = e;
                nval[k] = ev;
            } else {
                cur[k] = e;
                cval[k] = ev;
            }
        } else {
            e = nxt[k];
            cur[k] = e;
            cval[k] = nval[k];
        }
        a = s;
        cnt = e - s;
    }
    // pass 2 skipped: the cursor moves on as pass 2 would have moved it
    __device__ void commit(uint32_t k) const {
        if (two_pass) {
            cur[k] = nxt[k];
            cval[k] = nval[k];
        }
    }
};

template <int T>
struct RunShared {
    uint32_t off[T];    // flat start of each non-empty run part (compacted)
    uint32_t begin[T];  // slot of its first wedge
    uint32_t kidx[T];   // its up-slot index
    unsigned long long sum[T];
    unsigned long long tmp64[T / WAVE + 1];
    uint8_t mark[4 * T];  // per wave: 4 byte strips, run starts inside each of 4 64-wedge tiles
    uint32_t keys;      // packed hash: keys inserted in the current window
};

// The run table of the heavy dense kernel: chunks of 2T up-slots, two per
// thread, so a source's window takes half the chunk phases.  It fits beside
// the 128 KB window by narrower fields: run sums in 32 bits (a run part's sum
// of R - 1 over distinct endpoints x2 is below m) and up-slot indices
// relative to the source's first (a heavy source has fewer than 65536).
template <int T>
struct HeavyRuns {
    static constexpr int N = 2 * T;
    unsigned long long tmp64[T / WAVE + 1];
    uint32_t sum[N];
    uint32_t off[N];
    uint32_t begin[N];
    uint16_t kidx[N];
    uint8_t mark[4 * T];
    uint32_t keys;
};

// Largest i in [lo, n) with off[i] <= f (off strictly increasing, off[lo] <= f).
__device__ inline uint32_t last_le(const uint32_t *off, uint32_t lo, uint32_t n, uint32_t f) {
    uint32_t hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (off[mid] <= f) lo = mid; else hi = mid;
    }
    return lo;
}

// One work item: source r and the part of each of its runs that `range`
// selects.  Pass 1 retrieves the wedges (Algorithm 2) into the aggregator
// (GET-FREQ); the endpoint step adds C(R,2) per pair (total, and both
// endpoints for per-vertex); pass 2 walks the wedges again and adds R-1 to
// each center / both edges (Algorithms 3, 4).
//
// Up-slots are taken T at a time; the non-empty run parts are compacted and
// laid end to end (block scan).  Each wave walks that flat sequence U*64
// wedges at a time with lane-consecutive wedges, so the reads of x2 and the
// per-edge credit atomics are coalesced.  For each 64 wedges the wave keeps the
// (at most 64) runs they touch one per lane, and a lane finds its run with a
// 6-step shuffle search.
// Lays the non-empty run parts of this thread's run (a, cnt at slot start)
// end to end over the block: sh.off/begin/kidx get the compacted table;
// returns (total wedges, parts).  Zeroes the parts' run sums.
template <int T>
__device__ inline void compact_runs(uint32_t k, uint32_t start, uint32_t a, uint32_t cnt, RunShared<T> &sh,
                                    uint32_t *total, uint32_t *nne) {
    // one scan gives both the flat offset (low 32 bits) and the compacted
    // index (high 32 bits) of every non-empty part
    const unsigned long long packed = ((unsigned long long)(cnt > 0) << 32) | cnt;
    unsigned long long tot64;
    const unsigned long long pre = block_exclusive_sum<T>(packed, sh.tmp64, &tot64);
    *total = (uint32_t)tot64;
    *nne = (uint32_t)(tot64 >> 32);
    if (cnt > 0) {
        const uint32_t ci = (uint32_t)(pre >> 32);
        sh.off[ci] = (uint32_t)pre;
        sh.begin[ci] = start + a;
        sh.kidx[ci] = k;
        sh.sum[ci] = 0;
    }
    __syncthreads();
}

// Adds each lane's d to the run it belongs to: one prefix sum over the wave,
// then the last lane of every run segment adds the segment's total.  `first`
// is the lane where the lane's segment starts in this tile (0 if the run
// began in an earlier tile).  Needs 64 * max d < 2^32.
__device__ inline void segment_add(uint32_t d, bool ok, uint32_t first, bool last, unsigned long long *dst,
                                   uint32_t lane) {
    const uint32_t incl = wave_inclusive_sum(ok ? d : 0u);
    const uint32_t before = __shfl(incl, first ? first - 1 : 0, WAVE);
    const uint32_t seg = incl - (first ? before : 0u);
    if (ok && last && seg)
        __hip_atomic_fetch_add(dst, (unsigned long long)seg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ inline void segment_add(uint32_t d, bool ok, uint32_t first, bool last, uint32_t *dst, uint32_t lane) {
    const uint32_t incl = wave_inclusive_sum(ok ? d : 0u);
    const uint32_t before = __shfl(incl, first ? first - 1 : 0, WAVE);
    const uint32_t seg = incl - (first ? before : 0u);
    if (ok && last && seg) __hip_atomic_fetch_add(dst, seg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Adds the wave's d to one run's sum (every lane's wedge is in that run).
__device__ inline void run_add(unsigned long long *dst, uint32_t d, uint32_t lane) {
    const uint32_t tot = __builtin_amdgcn_readlane(wave_inclusive_sum(d), WAVE - 1);
    if (tot && lane == 0)
        __hip_atomic_fetch_add(dst, (unsigned long long)tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline void run_add(uint32_t *dst, uint32_t d, uint32_t lane) {
    const uint32_t tot = __builtin_amdgcn_readlane(wave_inclusive_sum(d), WAVE - 1);
    if (tot && lane == 0) __hip_atomic_fetch_add(dst, tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Walks the compacted wedge sequence of one chunk (see count_item): pass 1
// inserts each x2 into the aggregator; pass 2 credits R-1 to the slot
// (y -> x2) and sums it per run into sh.sum.
//
// A wave holds 64 consecutive runs, one per lane (flat start o and slot
// offset dlt = slot - flat index).  For a tile of 64 consecutive wedges, the
// runs starting inside the tile are marked in a 64-byte LDS strip and
// gathered with one ballot; a lane's run is then the run holding the tile's
// first wedge plus the number of marked starts up to its own position.
template <int T, int U, int PASS, class Agg, class SH>
__device__ inline void walk_runs(const Ranked &G, const Acc &A, const Agg &agg, SH &sh, uint32_t total,
                                 uint32_t nne) {
    static_assert(U <= 4, "one byte strip per sub-tile");
    const uint32_t tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
    const bool edge = A.mode & MODE_EDGE;
    // Lanes exchange data through these strips within one wave: relaxed
    // wavefront-scope atomic accesses, so each store and load is issued as
    // written (LDS runs one wave's operations in order).
    uint8_t *strip = sh.mark + wv * (4 * WAVE);
    const uint64_t le = lanemask_lt() | (1ull << lane);
    // each wave walks one contiguous share of whole 64-wedge tiles, so the
    // held runs move forward with a ballot instead of a search
    constexpr uint32_t NW = T / WAVE;
    total = __builtin_amdgcn_readfirstlane(total);
    nne = __builtin_amdgcn_readfirstlane(nne);
    const uint32_t tiles = (total + WAVE - 1) / WAVE, per = (tiles + NW - 1) / NW;
    const uint32_t t0 = wv * per < tiles ? wv * per : tiles, t1 = t0 + per < tiles ? t0 + per : tiles;
    const uint32_t f1 = t1 * WAVE < total ? t1 * WAVE : total;
    // runs i0 .. i0+63 held one per lane
    uint32_t i0 = 0, o = 0xFFFFFFFFu, dlt = 0, o_end = 0;
    for (uint32_t wb = t0 * WAVE; wb < f1; wb += U * WAVE) {
        uint32_t pidx[U], rel[U], xs[U] = {};  // xs of lanes past the end stay 0
        uint64_t st[U];
        bool ok[U];
        const uint32_t span_last = wb + U * WAVE - 1 < f1 ? wb + U * WAVE - 1 : f1 - 1;
        if (span_last < o_end && __ballot(o > wb && o <= span_last) == 0) {
            // no held run starts inside the span: one run (the last held
            // one starting at or before wb) covers all of it
            const uint32_t j0 = (uint32_t)__popcll(__ballot(o <= wb)) - 1;
            const uint32_t d0 = __builtin_amdgcn_readlane(dlt, j0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t base = wb + u * WAVE;
                ok[u] = base + lane < f1;
                st[u] = 0;
                rel[u] = i0 + j0;
                pidx[u] = d0 + base + lane;
            }
        } else if (span_last < o_end) {
            // every sub-tile lies inside the held runs: the strips of all
            // sub-tiles are cleared, marked and read back to back, so their
            // LDS round trips overlap
            uint32_t before[U], mk[U], jj[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t base = wb + u * WAVE;
                ok[u] = base + lane < f1;
                before[u] = (uint32_t)__popcll(__ballot(o <= base));
                __hip_atomic_store(&strip[u * WAVE + lane], (uint8_t)0, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WAVEFRONT);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t base = wb + u * WAVE;
                if (base < f1 && o > base && o - base < WAVE)
                    __hip_atomic_store(&strip[u * WAVE + (o - base)], (uint8_t)1, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WAVEFRONT);
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                mk[u] = __hip_atomic_load(&strip[u * WAVE + lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t starts = __ballot(mk[u] != 0);
                jj[u] = before[u] - 1 + (uint32_t)__popcll(starts & le);
                st[u] = starts;
                rel[u] = i0 + jj[u];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) pidx[u] = __shfl(dlt, jj[u], WAVE) + wb + u * WAVE + lane;
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t base = wb + u * WAVE;
                st[u] = 0;
                ok[u] = base + lane < f1;
                rel[u] = 0;
                pidx[u] = 0;
                if (base < f1) {  // wave-uniform
                    const uint32_t last = base + WAVE - 1 < f1 ? base + WAVE - 1 : f1 - 1;
                    if (last >= o_end) {
                        // reload: the 64 runs from the one holding `base` always
                        // cover [base, base + 64); that run is found among the
                        // held ones when it is there
                        const uint32_t c = (uint32_t)__popcll(__ballot(o <= base));
                        uint32_t ni;
                        if (c == 0) ni = last_le(sh.off, 0, nne, base);
                        else if (c < WAVE) ni = i0 + c - 1;
                        else ni = last_le(sh.off, i0 + WAVE - 1, nne, base);
                        i0 = __builtin_amdgcn_readfirstlane(ni);
                        const uint32_t kk = i0 + lane;
                        o = kk < nne ? sh.off[kk] : 0xFFFFFFFFu;
                        dlt = kk < nne ? sh.begin[kk] - o : 0u;
                        o_end = __builtin_amdgcn_readfirstlane(i0 + WAVE < nne ? sh.off[i0 + WAVE] : total);
                    }
                    const uint32_t f = base + lane;
                    const uint32_t before = (uint32_t)__popcll(__ballot(o <= base));  // held runs starting <= base
                    __hip_atomic_store(&strip[lane], (uint8_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                    if (o > base && o - base < WAVE)
                        __hip_atomic_store(&strip[o - base], (uint8_t)1, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WAVEFRONT);
                    const uint64_t starts = __ballot(
                        __hip_atomic_load(&strip[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT) != 0);
                    const uint32_t j = before - 1 + (uint32_t)__popcll(starts & le);
                    pidx[u] = __shfl(dlt, j, WAVE) + f;
                    rel[u] = i0 + j;
                    st[u] = starts;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (ok[u]) xs[u] = G.nbr[pidx[u]];
        if (PASS == 1) {
            if (!saturated(agg)) insert_all<U>(agg, xs, ok);
        } else {
            uint32_t cs[U];
            count_all<U>(agg, xs, ok, cs);
            // sub-tiles past the end credit nothing (ok false, d = 0); no early
            // exit, so the four sub-tiles' credit chains can interleave
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t d = ok[u] ? cs[u] - 1 : 0u;
                if (d && edge) A.slot_add(pidx[u], d);
                if (st[u] == 0) {
                    // (uniform) no run starts in the sub-tile: all its wedges
                    // belong to run rel[u]
                    run_add(&sh.sum[rel[u]], d, lane);
                } else {
                    const uint64_t sm = st[u] & le;
                    const uint32_t first = sm ? 63u - (uint32_t)__clzll(sm) : 0u;
                    const bool last =
                        lane == WAVE - 1 || ((st[u] >> (lane + 1)) & 1) || !(wb + u * WAVE + lane + 1 < f1);
                    segment_add(d, ok[u], first, last, &sh.sum[rel[u]], lane);
                }
            }
        }
    }
    __syncthreads();
}

// Pass-2 run sums of one chunk: the center credit (per-vertex) and the credit
// of the slot (r -> y) (per-edge).
template <int T>
__device__ inline void flush_runs(const Ranked &G, const Acc &A, uint32_t r, uint32_t k0, RunShared<T> &sh,
                                  uint32_t nne) {
    const uint32_t tid = threadIdx.x;
    if (tid < nne) {
        const unsigned long long sm = sh.sum[tid];
        if (sm) {
            const uint32_t up = G.roff[r] + (sh.kidx[tid] - k0);  // slot (r -> y)
            if (A.mode & MODE_VERTEX) atomicAdd(&A.v[G.nbr[up]], sm);
            if (A.mode & MODE_EDGE) A.slot_add(up, sm);
        }
    }
    __syncthreads();
}

// The endpoint step after pass 1: C(R,2) per pair into the total and, for
// per-vertex counts, into both endpoints.
template <int T, class Agg, class SH>
__device__ inline unsigned long long endpoint_credit(const Ranked &G, const Acc &A, uint32_t r, const Agg &agg,
                                                    SH &sh) {
    unsigned long long local = 0;
    const bool vert = A.mode & MODE_VERTEX;
    agg.for_each([&](uint32_t key, uint32_t cc) {
        if (cc >= 2) {
            const unsigned long long t = (unsigned long long)cc * (cc - 1) / 2;
            local += t;
            if (vert) atomicAdd(&A.v[key], t);
        }
    });
    const unsigned long long tot = block_sum<T>(local, sh.tmp64);
    if (threadIdx.x == 0 && tot) {
        if (A.mode & MODE_GLOBAL) atomicAdd(&A.g[G.gid ? G.gid[r] : 0u], tot);
        if (vert) atomicAdd(&A.v[G.smid[r]], tot);
    }
    __syncthreads();
    return tot;  // the same in every thread
}

// One work item: source r and the part of each of its runs that `range`
// selects.  Pass 1 retrieves the wedges (Algorithm 2) into the aggregator
// (GET-FREQ); the endpoint step adds C(R,2) per pair (total, and both
// endpoints for per-vertex); pass 2 walks the wedges again and adds R-1 to
// each center / both edges (Algorithms 3, 4).
//
// Up-slots are taken T at a time; the non-empty run parts are compacted and
// laid end to end (block scan).  Each wave walks that flat sequence U*64
// wedges at a time with lane-consecutive wedges, so the reads of x2 and the
// per-edge credit atomics are coalesced.  For each 64 wedges the wave keeps the
// (at most 64) runs they touch one per lane, and a lane finds its run with a
// 6-step shuffle search.
template <int T, int U, class Agg, class Range>
__device__ bool count_item(const Ranked &G, const Acc &A, uint32_t r, const Agg &agg, const Range &range,
                           RunShared<T> &sh, int passes) {
    const uint32_t tid = threadIdx.x;
    const uint32_t k0 = G.upoff[r], k1 = G.upoff[r + 1];
    agg.init();
    __syncthreads();
    const bool credit = A.mode & (MODE_VERTEX | MODE_EDGE);
    const uint32_t c_last = k1 > k0 ? k0 + (k1 - k0 - 1) / T * T : k0;
    bool pairs = true;
    for (int pass = 1; pass <= passes; ++pass) {
        if (pass == 2 && !pairs) {
            // no pair has R >= 2: every pass-2 credit is zero
            for (uint32_t k = k0 + tid; k < k1; k += T) range.commit(k);
            break;
        }
        // pass 2 takes the chunks in reverse (the runs pass 1 read last are
        // still in the L2)
        for (uint32_t i = 0, c = pass == 1 ? k0 : c_last; c < k1 && i <= (c_last - k0) / T;
             ++i, c = pass == 1 ? c + T : c - T) {
            const uint32_t k = c + tid;
            uint32_t a = 0, cnt = 0, start = 0;
            if (k < k1) {
                start = G.uprun[k];
                range(G, pass, k, start, G.uplen[k], a, cnt);
            }
            uint32_t total, nne;
            compact_runs<T>(k, start, a, cnt, sh, &total, &nne);
            if (pass == 1) walk_runs<T, U, 1>(G, A, agg, sh, total, nne);
            else if (credit) walk_runs<T, U, 2>(G, A, agg, sh, total, nne);
            if (pass == 2) flush_runs<T>(G, A, r, k0, sh, nne);
        }
        if (pass == 1) {
            if (!agg.finalize()) return false;  // (uniform) capacity exceeded: caller retries
            pairs = endpoint_credit<T>(G, A, r, agg, sh) != 0;
        }
    }
    __syncthreads();
    return true;
}

template <int T, int U, int CAP>
__global__ __launch_bounds__(T) void k_count_hash(Ranked G, Acc A, const uint32_t *list, uint32_t count) {
    __shared__ uint32_t keys[CAP];
    __shared__ uint32_t cnts[CAP];
    __shared__ RunShared<T> sh;
    HashAgg<T, CAP> agg{keys, cnts, A.err};
    for (uint32_t i = blockIdx.x; i < count; i += gridDim.x)
        count_item<T, U>(G, A, list[i], agg, full_range(G, list[i]), sh, A.passes());
}

// Hash over a candidate window of at most CAP/2 ids (forced hash on heavy
// sources); the window's part of each run is found by binary search.
template <int T, int U, int CAP>
__global__ __launch_bounds__(T) void k_count_hash_win(Ranked G, Acc A, const uint2 *items, uint32_t count) {
    __shared__ uint32_t keys[CAP];
    __shared__ uint32_t cnts[CAP];
    __shared__ RunShared<T> sh;
    HashAgg<T, CAP> agg{keys, cnts, A.err};
    for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {
        const uint2 it = items[i];
        const uint32_t r = it.x, w = it.y;
        const uint32_t side_end = G.cend[r];
        const uint32_t lo = G.lo(r) + w * HASH_WIN;
        const uint32_t hi = side_end - lo > HASH_WIN ? lo + HASH_WIN : side_end;
        count_item<T, U>(G, A, r, agg, SearchRange{lo, hi}, sh, A.passes());
    }
}

// compact_runs for a HeavyRuns table, one run per thread, up-slot indices
// relative to k0.
template <int T>
__device__ inline void compact_rel(uint32_t k, uint32_t k0, uint32_t start, uint32_t a, uint32_t cnt,
                                   HeavyRuns<T> &sh, uint32_t *total, uint32_t *nne) {
    const unsigned long long packed = ((unsigned long long)(cnt > 0) << 32) | cnt;
    unsigned long long tot64;
    const unsigned long long pre = block_exclusive_sum<T>(packed, sh.tmp64, &tot64);
    *total = (uint32_t)tot64;
    *nne = (uint32_t)(tot64 >> 32);
    if (cnt > 0) {
        const uint32_t ci = (uint32_t)(pre >> 32);
        sh.off[ci] = (uint32_t)pre;
        sh.begin[ci] = start + a;
        sh.kidx[ci] = (uint16_t)(k - k0);
        sh.sum[ci] = 0;
    }
    __syncthreads();
}

// The same with two runs per thread (entries j = 0, 1 in thread order).
template <int T>
__device__ inline void compact_two(const uint32_t *k, uint32_t k0, const uint32_t *start, const uint32_t *a,
                                   const uint32_t *cnt, HeavyRuns<T> &sh, uint32_t *total, uint32_t *nne) {
    const unsigned long long packed = ((unsigned long long)((cnt[0] > 0) + (cnt[1] > 0)) << 32) | (cnt[0] + cnt[1]);
    unsigned long long tot64;
    const unsigned long long pre = block_exclusive_sum<T>(packed, sh.tmp64, &tot64);
    *total = (uint32_t)tot64;
    *nne = (uint32_t)(tot64 >> 32);
    uint32_t ci = (uint32_t)(pre >> 32), off = (uint32_t)pre;
#pragma unroll
    for (int j = 0; j < 2; ++j)
        if (cnt[j] > 0) {
            sh.off[ci] = off;
            sh.begin[ci] = start[j] + a[j];
            sh.kidx[ci] = (uint16_t)(k[j] - k0);
            sh.sum[ci] = 0;
            ++ci;
            off += cnt[j];
        }
    __syncthreads();
}

template <int T>
__device__ inline void flush_rel(const Ranked &G, const Acc &A, uint32_t r, HeavyRuns<T> &sh, uint32_t nne) {
    for (uint32_t i = threadIdx.x; i < nne; i += T) {
        const uint32_t sm = sh.sum[i];
        if (sm) {
            const uint32_t up = G.roff[r] + sh.kidx[i];  // slot (r -> y)
            if (A.mode & MODE_VERTEX) atomicAdd(&A.v[G.nbr[up]], (unsigned long long)sm);
            if (A.mode & MODE_EDGE) A.slot_add(up, sm);
        }
    }
    __syncthreads();
}

// count_item over chunks of 2T up-slots (thread t takes c + t and c + T + t).
template <int T, int U, class Agg, class Range>
__device__ void count_item_two(const Ranked &G, const Acc &A, uint32_t r, const Agg &agg, const Range &range,
                               HeavyRuns<T> &sh, int passes) {
    const uint32_t tid = threadIdx.x;
    const uint32_t k0 = G.upoff[r], k1 = G.upoff[r + 1];
    agg.init();
    __syncthreads();
    const bool credit = A.mode & (MODE_VERTEX | MODE_EDGE);
    const uint32_t c_last = k1 > k0 ? k0 + (k1 - k0 - 1) / (2 * T) * (2 * T) : k0;
    bool pairs = true;
    for (int pass = 1; pass <= passes; ++pass) {
        if (pass == 2 && !pairs) {
            // no endpoint pair of the window has R >= 2, so every pass-2
            // credit (R - 1 per wedge) is zero: only the cursors move on
            for (uint32_t c = k0; c < k1; c += 2 * T)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    if (c + j * T + tid < k1) range.commit(c + j * T + tid);
            break;
        }
        // pass 2 takes the chunks in reverse, so it starts on the runs pass 1
        // read last, while they are still in the L2
        for (uint32_t i = 0, c = pass == 1 ? k0 : c_last; c < k1 && i <= (c_last - k0) / (2 * T);
             ++i, c = pass == 1 ? c + 2 * T : c - 2 * T) {
            uint32_t k[2], a[2] = {0, 0}, cnt[2] = {0, 0}, start[2] = {0, 0};
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                k[j] = c + j * T + tid;
                if (k[j] < k1) {
                    start[j] = G.uprun[k[j]];
                    range(G, pass, k[j], start[j], G.uplen[k[j]], a[j], cnt[j]);
                }
            }
            uint32_t total, nne;
            compact_two<T>(k, k0, start, a, cnt, sh, &total, &nne);
            if (pass == 1) walk_runs<T, U, 1>(G, A, agg, sh, total, nne);
            else if (credit) walk_runs<T, U, 2>(G, A, agg, sh, total, nne);
            if (pass == 2) flush_rel<T>(G, A, r, sh, nne);
        }
        if (pass == 1) {
            agg.finalize();  // dense windows are never refused
            pairs = endpoint_credit<T>(G, A, r, agg, sh) != 0;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------- wave-independent heavy sweep

// Per-wave scratch of the wave-independent sweep.
struct WaveRuns {
    uint8_t mark[4 * WAVE];          // run starts inside each of 4 64-wedge tiles
    unsigned long long sum[WAVE];    // pass-2 credit of each run
};

// Wave-level compaction of one chunk of 64 up-slots (lane = up-slot): the
// non-empty run parts are laid end to end; lane i then holds the i-th one's
// flat start `o`, slot offset `dlt` (slot = dlt + flat index) and up-slot
// `kc`.  Lanes past the last part get o = ~0.
__device__ inline void wave_compact(uint32_t cnt, uint32_t first_slot, uint32_t k, uint32_t lane, uint32_t &o,
                                    uint32_t &dlt, uint32_t &kc, uint32_t &nne, uint32_t &total) {
    const uint32_t incl = wave_inclusive_sum(cnt);
    total = __builtin_amdgcn_readfirstlane(__shfl(incl, WAVE - 1, WAVE));
    const uint32_t excl = incl - cnt;
    const uint64_t ne = __ballot(cnt > 0);
    nne = (uint32_t)__popcll(ne);
    const uint32_t below = (uint32_t)__popcll(ne & lanemask_lt());
    // a full permutation: parts to lanes 0 .. nne-1 in order, empty lanes after
    const int tgt = (int)(4 * (cnt > 0 ? below : nne + (lane - below)));
    o = (uint32_t)__builtin_amdgcn_ds_permute(tgt, (int)excl);
    dlt = (uint32_t)__builtin_amdgcn_ds_permute(tgt, (int)(first_slot - excl));
    kc = (uint32_t)__builtin_amdgcn_ds_permute(tgt, (int)k);
    if (lane >= nne) o = 0xFFFFFFFFu;
}

// Walks the wedges of one compacted chunk (wave_compact) with no block
// synchronisation: the same tile scheme as walk_runs, with every run held in
// the wave from the start.
template <int U, int PASS, class Agg>
__device__ inline void wave_walk(const Ranked &G, const Acc &A, const Agg &agg, WaveRuns &wr, uint32_t o,
                                 uint32_t dlt, uint32_t total, uint32_t lane) {
    static_assert(U <= 4, "one byte strip per sub-tile");
    const bool edge = A.mode & MODE_EDGE;
    const uint64_t le = lanemask_lt() | (1ull << lane);
    if (PASS == 2) __hip_atomic_store(&wr.sum[lane], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    for (uint32_t wb = 0; wb < total; wb += U * WAVE) {
        uint32_t pidx[U], rel[U], xs[U], before[U], mk[U];
        bool ok[U];
        // the strips of all sub-tiles are cleared, marked and read back to
        // back, so their LDS round trips overlap
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t base = wb + u * WAVE;
            ok[u] = base + lane < total;
            before[u] = (uint32_t)__popcll(__ballot(o <= base));
            __hip_atomic_store(&wr.mark[u * WAVE + lane], (uint8_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t base = wb + u * WAVE;
            if (base < total && o > base && o - base < WAVE)
                __hip_atomic_store(&wr.mark[u * WAVE + (o - base)], (uint8_t)1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            mk[u] = __hip_atomic_load(&wr.mark[u * WAVE + lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t starts = __ballot(mk[u] != 0);
            rel[u] = before[u] - 1 + (uint32_t)__popcll(starts & le);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) pidx[u] = __shfl(dlt, rel[u], WAVE) + wb + u * WAVE + lane;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (ok[u]) xs[u] = G.nbr[pidx[u]];
        if (PASS == 1) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (ok[u]) agg.insert(xs[u]);
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (!ok[u]) continue;
                const uint32_t d = agg.count(xs[u]) - 1;
                if (d) {
                    if (edge) A.slot_add(pidx[u], d);
                    __hip_atomic_fetch_add(&wr.sum[rel[u]], (unsigned long long)d, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WAVEFRONT);
                }
            }
        }
    }
}

// Pass-2 run sums of one wave chunk: centre credit and slot (r -> y).
__device__ inline void wave_flush(const Ranked &G, const Acc &A, uint32_t r, uint32_t k0, WaveRuns &wr, uint32_t kc,
                                  uint32_t nne, uint32_t lane) {
    if (lane < nne) {
        const unsigned long long sm =
            __hip_atomic_load(&wr.sum[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        if (sm) {
            const uint32_t up = G.roff[r] + (kc - k0);  // slot (r -> y)
            if (A.mode & MODE_VERTEX) atomicAdd(&A.v[G.nbr[up]], sm);
            if (A.mode & MODE_EDGE) A.slot_add(up, sm);
        }
    }
}

// Endpoint step of one window, every wave on its own share of the counters.
template <int T>
__device__ inline bool wave_endpoint(const Ranked &G, const Acc &A, uint32_t r, const DenseAgg<T> &agg,
                                     uint32_t lane) {
    unsigned long long local = 0;
    const bool vert = A.mode & MODE_VERTEX;
    agg.for_each([&](uint32_t key, uint32_t cc) {
        if (cc >= 2) {
            const unsigned long long t = (unsigned long long)cc * (cc - 1) / 2;
            local += t;
            if (vert) atomicAdd(&A.v[key], t);
        }
    });
    local = wave_sum(local);
    if (lane == 0 && local) {
        if (A.mode & MODE_GLOBAL) atomicAdd(&A.g[G.gid ? G.gid[r] : 0u], local);
        if (vert) atomicAdd(&A.v[G.smid[r]], local);
    }
    return local != 0;  // the same in every lane
}

// Heavy sources: one workgroup per source sweeps the source's candidate range
// from the top in windows that fit about 128 KB of LDS counters (65408 ids
// with 16-bit counters when the source has fewer than 65536 up-neighbours,
// since R(x1, x2) <= deg_x1(x1); else 32704 ids).  Within a window the up-slots are
// walked in one of three ways:
//   * sources with at most T up-slots: each thread keeps its up-slot's run and
//     cursor in registers for the whole sweep; per window the run parts are
//     laid end to end over the workgroup once (compact_runs) and both passes
//     walk that one table, every wave on an equal share;
//   * wave-independent (wave_compact / wave_walk) for larger sources whose
//     runs are short (fewer than SHORT_RUN wedges per up-slot): every wave
//     takes its own chunks of 64 up-slots and the workgroup synchronises only
//     between the window's passes, since per-chunk block synchronisation
//     would dominate;
//   * block-wide chunks of 2T up-slots, two per thread (count_item_two), for
//     the other sources, which keeps whole chunks' wedges in one balanced
//     flat walk.
constexpr uint64_t SHORT_RUN = 64;

template <int T, int U>
__global__ __launch_bounds__(T) void k_count_heavy(Ranked G, Acc A, const uint32_t *list, const uint64_t *wsrc,
                                                   uint32_t *cur, uint32_t *nxt, uint32_t *cval, uint32_t *nval,
                                                   const uint32_t *byte_from, uint32_t count) {
    constexpr uint32_t NW = T / WAVE;
    static_assert(sizeof(WaveRuns) * NW <= sizeof(HeavyRuns<T>), "wave scratch shares the run table's LDS");
    __shared__ uint32_t words[WIN_WORDS];
    __shared__ HeavyRuns<T> sh;
    const uint32_t tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
    WaveRuns &wr = reinterpret_cast<WaveRuns *>(&sh)[wv];
    const bool two_pass = A.mode & (MODE_VERTEX | MODE_EDGE);
    for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {
        const uint32_t r = list[i];
        const uint32_t k0 = G.upoff[r], k1 = G.upoff[r + 1], ups = k1 - k0;
        const bool half = ups <= 0xFFFFu;
        const uint32_t wsz = half ? 2 * WIN_WORDS : WIN_WORDS;
        const bool small = ups <= (uint32_t)T;
        const bool waves = small || wsrc[i] < SHORT_RUN * ups;
        // small sources: lane state for up-slot k0 + tid
        const uint32_t ks = k0 + tid;
        const bool have = small && ks < k1;
        const uint32_t s_start = have ? G.uprun[ks] : 0u, s_pos = have ? G.uplen[ks] : 0u;
        uint32_t s_cur = 0, s_val = s_pos ? G.nbr[s_start] : 0u;
        const uint32_t lo_min = G.lo(r);
        // ids from bfrom up take 8-bit counters (4 * WIN_WORDS in a window),
        // from nfrom up 4-bit ones (8 * WIN_WORDS).  R(x1, x2) <= deg_x1(x1)
        // = ups as well, so a source with fewer than 256 (16) up-slots takes
        // 8-bit (4-bit) counters over its whole range.
        const uint32_t side = G.smid[r] < G.n_u ? 0 : 1;
        const uint32_t bfrom = byte_from[side], nfrom = byte_from[2 + side];
        const bool nib_all = ups < 16, byte_all = ups < 256;
        uint32_t hi = G.cend[r];
        bool first = true;
        __syncthreads();  // the previous source is done with the shared tables
        while (hi > lo_min) {
            const bool nib = nib_all || hi > nfrom, byte = !nib && (byte_all || hi > bfrom);
            const uint32_t width = nib ? 8 * WIN_WORDS : byte ? 4 * WIN_WORDS : wsz;
            uint32_t lo = hi - lo_min > width ? hi - width : lo_min;
            // a window narrowed by the id thresholds alone stops at its threshold
            if (nib && !nib_all && lo < nfrom) lo = nfrom;
            if (byte && !byte_all && lo < bfrom) lo = bfrom;
            const DenseAgg<T> agg{words, lo, hi - lo, half, A.err, byte, nib};
            const CursorRange rng{cur, nxt, cval, nval, lo, first, two_pass};
            if (!waves) {
                count_item_two<T, U>(G, A, r, agg, rng, sh, A.passes());
            } else {
                {
                    const uint32_t c = agg.cs(), nwords = (hi - lo + (1u << c) - 1) >> c;
                    for (uint32_t w = tid; w < nwords; w += T) words[w] = 0;
                }
                __syncthreads();
                if (small) {
                    // the window's run parts of all up-slots laid end to end
                    // over the workgroup, so every wave takes an equal share
                    uint32_t e = s_cur, ev = s_val;
                    if (s_cur < s_pos && s_val >= lo) e = probe_below(G.nbr, s_start, s_cur, s_pos, lo, &ev);
                    uint32_t total, nne;
                    compact_rel<T>(ks, k0, s_start, s_cur, e - s_cur, sh, &total, &nne);
                    walk_runs<T, U, 1>(G, A, agg, sh, total, nne);
                    // (walk_runs ends on a barrier) the endpoint step, then
                    // pass 2 only if some pair has R >= 2
                    if (block_sum<T>((unsigned long long)wave_endpoint<T>(G, A, r, agg, lane), sh.tmp64) && two_pass) {
                        walk_runs<T, U, 2>(G, A, agg, sh, total, nne);
                        flush_rel<T>(G, A, r, sh, nne);
                    }
                    s_cur = e;
                    s_val = ev;
                } else {
                    for (uint32_t c = k0 + wv * WAVE; c < k1; c += NW * WAVE) {
                        const uint32_t k = c + lane;
                        uint32_t a = 0, cnt = 0, start = 0;
                        if (k < k1) {
                            start = G.uprun[k];
                            rng(G, 1, k, start, G.uplen[k], a, cnt);
                        }
                        uint32_t o, dlt, kc, nne, total;
                        wave_compact(cnt, start + a, k, lane, o, dlt, kc, nne, total);
                        wave_walk<U, 1>(G, A, agg, wr, o, dlt, total, lane);
                    }
                    __syncthreads();
                    // (tmp64 overlaps wave 0's strips, free between the passes; block_sum ends on a barrier)
                    const bool pairs = block_sum<T>((unsigned long long)wave_endpoint<T>(G, A, r, agg, lane), sh.tmp64);
                    if (two_pass && !pairs) {
                        for (uint32_t k = k0 + tid; k < k1; k += T) rng.commit(k);  // no credit to give
                    } else if (two_pass) {
                        for (uint32_t c = k0 + wv * WAVE; c < k1; c += NW * WAVE) {
                            const uint32_t k = c + lane;
                            uint32_t a = 0, cnt = 0, start = 0;
                            if (k < k1) {
                                start = G.uprun[k];
                                rng(G, 2, k, start, G.uplen[k], a, cnt);
                            }
                            uint32_t o, dlt, kc, nne, total;
                            wave_compact(cnt, start + a, k, lane, o, dlt, kc, nne, total);
                            wave_walk<U, 2>(G, A, agg, wr, o, dlt, total, lane);
                            wave_flush(G, A, r, k0, wr, kc, nne, lane);
                        }
                    }
                }
                __syncthreads();
            }
            hi = lo;
            first = false;
        }
    }
}

template <int T, int CAP>
struct SortShared {
    uint64_t a[CAP], b[CAP];
    uint32_t cnt[16 * T];
    uint32_t start[CAP];
    uint32_t meta[2];
    uint32_t tmp[T / WAVE + 1];
};

// Sort aggregation of whole sources with at most CAP wedges.
template <int T, int U, int CAP>
__global__ __launch_bounds__(T) void k_count_sort(Ranked G, Acc A, const uint32_t *list, uint32_t count) {
    static_assert(16 * T >= CAP, "count array too small");
    __shared__ SortShared<T, CAP> ss;
    __shared__ RunShared<T> sh;
    for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {
        const uint32_t r = list[i];
        const uint32_t lo = G.lo(r), side_end = G.cend[r];
        SortAgg<T, CAP> agg{ss.a, ss.b, ss.cnt, ss.start, ss.meta, ss.tmp, lo, side_end - lo};
        if (!count_item<T, U>(G, A, r, agg, full_range(G, r), sh, A.passes())) atomicOr(A.err, FLAG_INTERNAL);
    }
}

// Sort aggregation of larger sources: windows of the candidate range from the
// top, each first tried at a width that should hold about CAP/2 wedges and
// halved while its wedges exceed CAP.  The cursors only advance once a window
// has been counted (two passes always, so a refused window leaves them as
// they were).
template <int T, int U, int CAP>
__global__ __launch_bounds__(T) void k_count_sort_heavy(Ranked G, Acc A, const uint32_t *list, const uint64_t *wsrc,
                                                        uint32_t *cur, uint32_t *nxt, uint32_t *cval, uint32_t *nval,
                                                        uint32_t count) {
    static_assert(16 * T >= CAP, "count array too small");
    __shared__ SortShared<T, CAP> ss;
    __shared__ RunShared<T> sh;
    for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {
        const uint32_t r = list[i];
        const uint32_t lo_min = G.lo(r);
        uint32_t hi = G.cend[r];
        const uint64_t w = wsrc[i] ? wsrc[i] : 1;
        uint64_t guess = (uint64_t)(hi - lo_min) * (CAP / 2) / w;
        uint32_t width = guess < 1 ? 1u : guess > hi - lo_min ? hi - lo_min : (uint32_t)guess;
        bool first = true;
        while (hi > lo_min) {
            const uint32_t lo = hi - lo_min > width ? hi - width : lo_min;
            SortAgg<T, CAP> agg{ss.a, ss.b, ss.cnt, ss.start, ss.meta, ss.tmp, lo, hi - lo};
            if (!count_item<T, U>(G, A, r, agg, CursorRange{cur, nxt, cval, nval, lo, first, true}, sh, 2)) {
                width = (hi - lo) / 2 ? (hi - lo) / 2 : 1u;
                continue;
            }
            hi = lo;
            first = false;
            width = width < 0x40000000u ? 2 * width : width;  // try wider again
        }
    }
}

// Sources with few wedges over a wide candidate range: packed-LDS-hash windows
// from the top of the range, each first tried at a width that should hold
// about PH_TARGET distinct endpoints and halved while it overflows (the
// cursors advance only once a window has been counted, so always two passes).
template <int T, int U>
__global__ __launch_bounds__(T) void k_count_phash(Ranked G, Acc A, const uint32_t *list, const uint64_t *wsrc,
                                                   uint32_t *cur, uint32_t *nxt, uint32_t *cval, uint32_t *nval,
                                                   uint32_t count) {
    static_assert(PH_FULL + T * U <= PH_SLOTS, "keys inserted after the walk's last check must still fit");
    __shared__ uint32_t words[PH_SLOTS];
    __shared__ RunShared<T> sh;
    for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {
        const uint32_t r = list[i];
        const uint32_t k0 = G.upoff[r], k1 = G.upoff[r + 1];
        const uint32_t cbits = bit_width(k1 - k0);
        const uint32_t lo_min = G.lo(r);
        uint32_t hi = G.cend[r];
        const uint64_t w = wsrc[i] ? wsrc[i] : 1;
        const uint64_t guess = (uint64_t)(hi - lo_min) * PH_TARGET / w;
        uint32_t width = guess < 1 ? 1u : guess > hi - lo_min ? hi - lo_min : (uint32_t)guess;
        if (k1 - k0 <= (uint32_t)T) {
            // one up-slot per thread, its cursor in registers (committed once
            // a window has been counted); one compaction serves both passes
            const uint32_t k = k0 + threadIdx.x;
            const bool have = k < k1;
            const uint32_t start = have ? G.uprun[k] : 0u, pos = have ? G.uplen[k] : 0u;
            uint32_t sc = 0, sv = pos ? G.nbr[start] : 0u;
            while (hi > lo_min) {
                const uint32_t lo = hi - lo_min > width ? hi - width : lo_min;
                const PackedHashAgg<T, PH_SLOTS, PH_FULL> agg{words, &sh.keys, lo, cbits, A.err};
                agg.init();
                uint32_t e = sc, ev = sv;
                if (sc < pos && sv >= lo) e = probe_below(G.nbr, start, sc, pos, lo, &ev);
                uint32_t total, nne;
                compact_runs<T>(k, start, sc, e - sc, sh, &total, &nne);
                walk_runs<T, U, 1>(G, A, agg, sh, total, nne);
                if (!agg.finalize()) {  // (uniform) the window overflowed: narrow it
                    width = (hi - lo) / 2 ? (hi - lo) / 2 : 1u;
                    continue;
                }
                // pass 2 only when some pair has R >= 2 (else every credit is zero)
                if (endpoint_credit<T>(G, A, r, agg, sh) && (A.mode & (MODE_VERTEX | MODE_EDGE))) {
                    walk_runs<T, U, 2>(G, A, agg, sh, total, nne);
                    flush_runs<T>(G, A, r, k0, sh, nne);
                }
                sc = e;
                sv = ev;
                hi = lo;
            }
            continue;
        }
        bool first = true;
        while (hi > lo_min) {
            const uint32_t lo = hi - lo_min > width ? hi - width : lo_min;
            const PackedHashAgg<T, PH_SLOTS, PH_FULL> agg{words, &sh.keys, lo, cbits, A.err};
            if (!count_item<T, U>(G, A, r, agg, CursorRange{cur, nxt, cval, nval, lo, first, true}, sh, 2)) {
                width = (hi - lo) / 2 ? (hi - lo) / 2 : 1u;
                continue;
            }
            hi = lo;
            first = false;
        }
    }
}

// Whole-range dense counting for sources whose candidate range fits WINSZ.
template <int T, int U, int WINSZ>
__global__ __launch_bounds__(T) void k_count_dense_src(Ranked G, Acc A, const uint32_t *list, uint32_t count) {
    __shared__ uint32_t words[WINSZ];
    __shared__ RunShared<T> sh;
    for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {
        const uint32_t r = list[i];
        const uint32_t side_end = G.cend[r];
        const uint32_t lo = G.lo(r);
        DenseAgg<T> agg{words, lo, side_end - lo, false, A.err};
        count_item<T, U>(G, A, r, agg, full_range(G, r), sh, A.passes());
    }
}

// ---------------------------------------------------------------- giant sources

// Dense per-source histogram in global scratch (GET-FREQ by histogramming,
// Section 3.1.2, one counter per candidate endpoint): pass 1 adds one per
// wedge, the endpoint step reads every counter once, pass 2 reads R back.
// Counters stay in the L2 of one die: all items of a source run on
// workgroups of the same die.
//
// Pass 1 does not send every wedge to the histogram: a wedge's endpoint
// among the first GH_HOT candidates of the source (the highest ranked ones,
// which take most of a giant source's wedges) is counted in a window of
// 16-bit LDS counters instead, and the window is added to the histogram, one
// atomic per non-zero counter, when the workgroup moves to another source or
// has walked GH_HOT_UPS up-slots into it.  A run holds an endpoint at most
// once, so a counter never exceeds the up-slots walked since the last flush
// and cannot wrap.  Global atomics on random histogram lines are what limits
// the walk; the window takes most of them off the L2.
constexpr uint32_t GH_HOT = 14336;      // ids in the window: 28 KB, 4 walk workgroups per CU
constexpr uint32_t GH_HOT_UPS = 65535;  // up-slots walked into one window between flushes

struct GlobalAgg {
    uint32_t *h;
    uint32_t lo;
    uint32_t *hot;         // pass 1: GH_HOT / 2 LDS words, two 16-bit counters each
    const uint32_t *drow;  // pass 2 of a hub source: its row of the hub tile, for partners below lo
    uint32_t hub_base;
    __device__ void insert(uint32_t x) const {
        const uint32_t i = x - lo;
        if (i < GH_HOT) atomicAdd(&hot[i >> 1], 1u << ((i & 1u) * 16));
        else atomicAdd(&h[i], 1u);
    }
    // pass 2: the first GH_HOT / 2 counts were copied to `hot`; a hub
    // partner's count is the tile's
    __device__ uint32_t count(uint32_t x) const {
        if (x < lo) return drow[x - hub_base];
        const uint32_t i = x - lo;
        return i < GH_HOT / 2 ? hot[i] : h[i];
    }
};

// Adds the LDS window to the histogram `h` and clears it.  Call from all
// threads.
template <int T>
__device__ inline void gh_flush(uint32_t *hot, uint32_t *h) {
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < GH_HOT / 2; i += T) {
        const uint32_t w = hot[i];
        if (w) {
            hot[i] = 0;
            // only inserted endpoints, which are inside the source's range, are non-zero
            if (w & 0xFFFFu) atomicAdd(&h[2 * i], w & 0xFFFFu);
            if (w >> 16) atomicAdd(&h[2 * i + 1], w >> 16);
        }
    }
    __syncthreads();
}

struct GhSrc {
    uint32_t r, lo, ups, range;  // source rank, first candidate id, up-slots, candidate range
    uint64_t hoff;               // its counters: hist[hoff .. hoff + range)
};

// Also marks, in gh_hub (HUB_T flags, zeroed by the caller), the tile's hubs
// that are giant sources: their pass 2 credits the hub partners too.
__global__ void k_gh_info(Ranked G, const uint32_t *src, uint32_t c, uint32_t *info, uint32_t *gh_hub) {
    GRID_STRIDE(i, (uint64_t)c) {
        const uint32_t r = src[i];
        const uint32_t lo = G.lo(r);
        info[4 * i] = r;
        info[4 * i + 1] = lo;
        info[4 * i + 2] = G.upoff[r + 1] - G.upoff[r];
        info[4 * i + 3] = G.cend[r] - lo;
        const uint32_t sm = G.smid[r];
        if (sm >= G.hub_base && sm < G.hub_end) gh_hub[sm - G.hub_base] = 1u;
    }
}

// Walks items (source s, up-slot chunk j) of this workgroup's die: pass 1
// inserts every wedge into the source's counters, pass 2 credits R - 1.  A
// workgroup takes a contiguous share of its die's list (sources in order,
// each source's chunks in order), so its items mostly belong to one source:
// the LDS window of pass 1 is flushed rarely, and pass 2 copies the counts of
// a source's first GH_HOT / 2 candidates to LDS once.
//
// A giant source that is one of the tile's hubs skips its hub partners in
// pass 1 (the tile counts those pairs).  With `D` (the tile) its pass 2 walks
// the whole run and takes a hub partner's R from the tile, which does the hub
// credit pass's work for that source in the same walk.
template <int T, int U, int PASS>
__global__ __launch_bounds__(T) void k_gh_walk(Ranked G, Acc A, const GhSrc *src, const uint2 *items,
                                               const uint32_t *xoff, uint32_t *hist, const uint32_t *D) {
    __shared__ RunShared<T> sh;
    __shared__ uint32_t hot[GH_HOT / 2];
    const uint32_t x = blockIdx.x % NXCD, per = gridDim.x / NXCD, b = blockIdx.x / NXCD;
    const uint64_t nx = xoff[x + 1] - xoff[x];
    const uint32_t j0 = xoff[x] + (uint32_t)(nx * b / per), j1 = xoff[x] + (uint32_t)(nx * (b + 1) / per);
    uint32_t held = 0xFFFFFFFFu, acc = 0;  // source the window holds, up-slots walked into it
    if (PASS == 1) {
        for (uint32_t i = threadIdx.x; i < GH_HOT / 2; i += T) hot[i] = 0;
        __syncthreads();
    }
    for (uint32_t j = j0; j < j1; ++j) {
        const uint2 it = items[j];
        const GhSrc sr = src[it.x];
        const uint32_t k0 = G.upoff[sr.r], k1 = G.upoff[sr.r + 1];
        const uint32_t kb = k0 + it.y * GH_CHUNK;
        const uint32_t ke = kb + GH_CHUNK < k1 ? kb + GH_CHUNK : k1;
        if (PASS == 1) {
            if (held != it.x || acc + (ke - kb) > GH_HOT_UPS) {
                if (held != 0xFFFFFFFFu) gh_flush<T>(hot, hist + src[held].hoff);
                held = it.x;
                acc = 0;
            }
            acc += ke - kb;
        } else if (held != it.x) {
            // pass 2 reads the counts of the first GH_HOT / 2 candidates from LDS
            __syncthreads();
            const uint32_t lim = sr.range < GH_HOT / 2 ? sr.range : GH_HOT / 2;
            for (uint32_t i = threadIdx.x; i < lim; i += T) hot[i] = hist[sr.hoff + i];
            __syncthreads();
            held = it.x;
        }
        const uint32_t sm = G.smid[sr.r];
        const bool cut = sr.lo != sm + 1;  // a hub source: its run ends in hub partners
        const uint32_t *drow = PASS == 2 && cut && D ? D + (uint64_t)(sm - G.hub_base) * HUB_T : nullptr;
        const GlobalAgg agg{hist + sr.hoff, sr.lo, hot, drow, G.hub_base};
        for (uint32_t c = kb; c < ke; c += T) {
            const uint32_t k = c + threadIdx.x;
            uint32_t cnt = 0, start = 0;
            if (k < ke) {
                start = G.uprun[k];
                const uint32_t pos = G.uplen[k];
                // the whole run is ranked after the source; the hub partners come last
                cnt = cut && !drow ? first_below(G.nbr + start, 0, pos, sr.lo) : pos;
            }
            uint32_t total, nne;
            compact_runs<T>(k, start, 0u, cnt, sh, &total, &nne);
            walk_runs<T, U, PASS>(G, A, agg, sh, total, nne);
            if (PASS == 2) flush_runs<T>(G, A, sr.r, k0, sh, nne);
        }
    }
    if (PASS == 1 && held != 0xFFFFFFFFu) gh_flush<T>(hot, hist + src[held].hoff);
}

// Endpoint step over the counters: C(R,2) per candidate into the total and,
// for per-vertex counts, into both endpoints.  Items (source, segment of
// GH_SEG counters), grouped by die like the walk.
template <int T>
__global__ __launch_bounds__(T) void k_gh_endpoint(Ranked G, Acc A, const GhSrc *src, const uint2 *items,
                                                   const uint32_t *xoff, const uint32_t *hist) {
    __shared__ unsigned long long tmp[T / WAVE + 1];
    const bool vert = A.mode & MODE_VERTEX;
    const uint32_t x = blockIdx.x % NXCD, per = gridDim.x / NXCD;
    for (uint32_t j = xoff[x] + blockIdx.x / NXCD; j < xoff[x + 1]; j += per) {
        const uint2 it = items[j];
        const GhSrc sr = src[it.x];
        const uint32_t b = it.y * GH_SEG, e = b + GH_SEG < sr.range ? b + GH_SEG : sr.range;
        const uint32_t *h = hist + sr.hoff;
        unsigned long long local = 0;
        for (uint32_t i = b + threadIdx.x; i < e; i += T) {
            const uint32_t cc = h[i];
            if (cc >= 2) {
                const unsigned long long t = (unsigned long long)cc * (cc - 1) / 2;
                local += t;
                if (vert) atomicAdd(&A.v[sr.lo + i], t);
            }
        }
        const unsigned long long tot = block_sum<T>(local, tmp);
        if (threadIdx.x == 0 && tot) {
            if (A.mode & MODE_GLOBAL) atomicAdd(&A.g[G.gid ? G.gid[sr.r] : 0u], tot);
            if (vert) atomicAdd(&A.v[G.smid[sr.r]], tot);
        }
    }
}

// ---------------------------------------------------------------- hub credit pass

constexpr uint32_t HUB_CHUNK = 4096;          // up-slots per item of the hub credit pass
constexpr uint64_t HUB_AUTO_MIN_M = 1u << 22;  // AUTO considers the tile from this many edges
constexpr uint32_t HUB_PASS_GRID = 4096;

// R of hub pairs, read from the tile (the credit pass needs count() only).
struct HubAgg {
    const uint32_t *row;  // D row of the lower endpoint
    uint32_t base;
    __device__ void insert(uint32_t) const {}
    __device__ uint32_t count(uint32_t x) const { return row[x - base]; }
};

// Items of the hub credit pass: hub i owns ceil(up-slots / HUB_CHUNK)
// consecutive items starting at hoff[i]; hoff[HUB_T] is the total.
__global__ __launch_bounds__(HUB_T) void k_hub_items(const uint32_t *upoff, const uint32_t *hub_rank, uint32_t H,
                                                     uint32_t *hoff, PlanCounts *pc) {
    __shared__ uint32_t tmp[HUB_T / WAVE + 1];
    const uint32_t i = threadIdx.x;
    uint32_t c = 0;
    if (i < H && pc->hub.on) {
        const uint32_t r = hub_rank[i];
        c = (upoff[r + 1] - upoff[r] + HUB_CHUNK - 1) / HUB_CHUNK;
    }
    uint32_t total;
    const uint32_t o = block_exclusive_sum<HUB_T>(c, tmp, &total);
    hoff[i] = o;
    if (i == 0) {
        hoff[HUB_T] = total;
        pc->hub_items = total;
    }
}

// Pass 2 for the hub pairs (Algorithms 3, 4 with R from the tile): for each
// up-slot (h1 -> y) of a hub, the part of N(y) inside (h1, hub end) holds its
// hub partners; each gets R - 1 on the slot (y -> h2) and the run's sum goes
// to the centre y and the slot (h1 -> y).  A hub's up-slots are split into
// items of HUB_CHUNK, so one giant hub spreads over many workgroups.
// Hubs flagged in `skip` (giant sources whose histogram walk credits their
// hub partners) are left out.
template <int T, int U>
__global__ __launch_bounds__(T) void k_count_hub_pass(Ranked G, Acc A, const uint32_t *hub_rank, const uint32_t *hoff,
                                                      const uint32_t *D, const uint32_t *skip) {
    __shared__ RunShared<T> sh;
    const uint32_t count = hoff[HUB_T];
    for (uint32_t it = blockIdx.x; it < count; it += gridDim.x) {
        uint32_t lo = 0, hi = HUB_T;  // hoff[lo] <= it < hoff[hi]
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (hoff[mid] <= it) lo = mid; else hi = mid;
        }
        if (skip[lo]) continue;  // (uniform)
        const uint32_t r = hub_rank[lo];
        const uint32_t k0 = G.upoff[r], k1 = G.upoff[r + 1];
        const uint32_t kb = k0 + (it - hoff[lo]) * HUB_CHUNK;
        const uint32_t ke = kb + HUB_CHUNK < k1 ? kb + HUB_CHUNK : k1;
        const HubAgg agg{D + (uint64_t)lo * HUB_T, G.hub_base};
        const uint32_t s_lo = G.smid[r] + 1;
        for (uint32_t c = kb; c < ke; c += T) {
            const uint32_t k = c + threadIdx.x;
            uint32_t a = 0, cnt = 0, start = 0;
            if (k < ke) {
                start = G.uprun[k];
                const uint32_t pos = G.uplen[k];
                const uint32_t *p = G.nbr + start;
                a = first_below(p, 0, pos, G.hub_end);
                cnt = first_below(p, a, pos, s_lo) - a;
            }
            uint32_t total, nne;
            compact_runs<T>(k, start, a, cnt, sh, &total, &nne);
            walk_runs<T, U, 2>(G, A, agg, sh, total, nne);
            flush_runs<T>(G, A, r, k0, sh, nne);
        }
    }
}

// ---------------------------------------------------------------- outputs

struct CoreOut {
    int64_t *gout, *vout, *eout;                          // one graph
    int64_t *const *gouts, *const *vouts, *const *eouts;  // a batch: device arrays of per-graph pointers
};

// Batch layout (device arrays of ng + 1 entries): graph j owns U ids
// [ubase[j], ubase[j+1]), V-local ids [vbase[j], vbase[j+1]), edges
// [ebase[j], ebase[j+1]) and ranks [rbase[j], rbase[j+1]).
struct BatchLayout {
    uint32_t ng;
    const uint32_t *ubase, *vbase, *rbase;
    const uint64_t *ebase;
};

__global__ void k_out_global(const unsigned long long *g, uint32_t ng, CoreOut out) {
    GRID_STRIDE(j, (uint64_t)ng) {
        if (out.gouts) out.gouts[j][0] = (int64_t)g[j];
        else out.gout[0] = (int64_t)g[0];
    }
}

__global__ void k_out_vertex(const uint32_t *rank, const uint32_t *smid, const unsigned long long *v, uint64_t n,
                             uint32_t n_u, BatchLayout bl, CoreOut out) {
    GRID_STRIDE(x, n) {
        const int64_t val = v ? (int64_t)v[smid[rank[x]]] : 0;
        if (!out.vouts) {
            out.vout[x] = val;
        } else if (x < n_u) {
            const uint32_t j = graph_of<uint32_t>(bl.ubase, bl.ng, (uint32_t)x);
            out.vouts[j][x - bl.ubase[j]] = val;
        } else {
            const uint32_t xv = (uint32_t)(x - n_u);
            const uint32_t j = graph_of<uint32_t>(bl.vbase, bl.ng, xv);
            out.vouts[j][(bl.ubase[j + 1] - bl.ubase[j]) + (xv - bl.vbase[j])] = val;
        }
    }
}

__global__ void k_out_edge(const uint32_t *eslot, const unsigned long long *s, const uint32_t *s32, uint64_t m,
                           BatchLayout bl, CoreOut out) {
    GRID_STRIDE(e, m) {
        const int64_t val = s32 ? (int64_t)s32[eslot[e]] + (int64_t)s32[eslot[m + e]]
                                : (int64_t)(s[eslot[e]] + s[eslot[m + e]]);
        if (!out.eouts) {
            out.eout[e] = val;
        } else {
            const uint32_t j = graph_of<uint64_t>(bl.ebase, bl.ng, e);
            out.eouts[j][e - bl.ebase[j]] = val;
        }
    }
}

// Per-vertex counts from per-edge counts of one graph: each butterfly at x
// holds exactly two of x's edges, so b(x) = (sum of b(e) over the edges e at
// x) / 2 (the definitions of Section 2).  U rows are contiguous in the
// per-edge output; V rows reach it through the V-side CSR's edge ids.  A row
// of at most VTX_SHORT entries is summed by one thread; a longer one is split
// into items of VTX_CHUNK entries, each summed by a wave and added to the
// row's total (cnt[x] = its items, scanned into coff), then halved.
constexpr uint32_t VTX_SHORT = 64;
constexpr uint32_t VTX_CHUNK = 2048;

__device__ inline void vertex_row(const int64_t *u_off, const uint32_t *v_off, uint32_t n_u, uint64_t x,
                                  uint64_t *b, uint64_t *e) {
    if (x < n_u) {
        *b = (uint64_t)u_off[x];
        *e = (uint64_t)u_off[x + 1];
    } else {
        *b = v_off[x - n_u];
        *e = v_off[x - n_u + 1];
    }
}

__global__ void k_vtx_short(const int64_t *u_off, const uint32_t *v_off, const uint32_t *v_eid, uint32_t n_u,
                            uint64_t n, const int64_t *eout, int64_t *vout, uint32_t *cnt) {
    GRID_STRIDE(x, n) {
        uint64_t b, e;
        vertex_row(u_off, v_off, n_u, x, &b, &e);
        int64_t sum = 0;
        uint32_t items = 0;
        if (e - b <= VTX_SHORT) {
            for (uint64_t i = b; i < e; ++i) sum += eout[x < n_u ? i : v_eid[i]];
            sum /= 2;
        } else {
            items = (uint32_t)((e - b + VTX_CHUNK - 1) / VTX_CHUNK);
        }
        vout[x] = sum;  // long rows: 0, the items add to it
        cnt[x] = items;
    }
}

// Item `it` belongs to vertex x with coff[x] <= it < coff[x + 1]; each wave
// takes a contiguous share of the items and adds one total per row.
__global__ __launch_bounds__(256) void k_vtx_long(const int64_t *u_off, const uint32_t *v_off, const uint32_t *v_eid,
                                                  uint32_t n_u, uint64_t n, const uint32_t *coff, const int64_t *eout,
                                                  int64_t *vout) {
    const uint32_t lane = threadIdx.x & (WAVE - 1);
    uint32_t i0, i1;  // a contiguous share of the items per wave
    item_share(coff[n], blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE, gridDim.x * (blockDim.x / WAVE), &i0,
               &i1);
    uint32_t held = 0xFFFFFFFFu;  // the row whose items the wave is summing
    int64_t acc = 0;
    rows_of_items(coff, n, i0, i1, [&](uint32_t x, uint32_t it) {
        if (x != held) {
            if (lane == 0 && acc) atomicAdd((unsigned long long *)&vout[held], (unsigned long long)acc);
            held = x;
            acc = 0;
        }
        uint64_t b, e;
        vertex_row(u_off, v_off, n_u, x, &b, &e);
        const uint64_t cb = b + (uint64_t)(it - coff[x]) * VTX_CHUNK;
        const uint64_t ce = cb + VTX_CHUNK < e ? cb + VTX_CHUNK : e;
        int64_t sum = 0;
        for (uint64_t i = cb + lane; i < ce; i += WAVE) sum += eout[x < n_u ? i : v_eid[i]];
        acc += wave_sum(sum);
    });
    if (lane == 0 && acc) atomicAdd((unsigned long long *)&vout[held], (unsigned long long)acc);
}

__global__ void k_vtx_halve(const uint32_t *cnt, uint64_t n, int64_t *vout) {
    GRID_STRIDE(x, n)
        if (cnt[x]) vout[x] /= 2;
}

constexpr uint32_t MAX_ITEM_GRID = 1u << 20;

// `width` caps the workgroups in flight (0: one per item, up to MAX_ITEM_GRID);
// the kernels loop over their items with a grid stride.
template <class K, class... Args>
void launch_items(K kernel, uint32_t count, uint32_t threads, uint32_t width, hipStream_t s, Args... args) {
    const uint32_t cap = width ? std::min(width, MAX_ITEM_GRID) : MAX_ITEM_GRID;
    const uint32_t grid = std::min(count, cap);
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(threads), 0, s, args..., count);
}

// ---------------------------------------------------------------- the counting pipeline

// Everything the pipeline reads, in unified-id space (one graph, or the
// disjoint union of a batch).
struct CoreIn {
    uint64_t n;
    uint32_t n_u;
    uint64_t m;
    const uint32_t *eu;    // m: U endpoint (unified id) of each edge
    const uint32_t *ev;    // m: V endpoint (V-local id)
    const uint32_t *deg;   // n
    const uint32_t *rank;  // n
    uint32_t max_deg;
    BatchLayout bl;        // ng = 1 for one graph
    // one graph: both sides' CSRs (null for a batch)
    const int64_t *u_off;
    const uint32_t *u_adj, *v_off, *v_adj, *v_eid;
};

bool policy_from(const pb_opts &o, Policy *p) {
    *p = Policy{LIGHT_D, MEDIUM_D, {PB_AGG_LDS_HASH, PB_AGG_LDS_HASH, PB_AGG_DENSE_HIST}, true};
    if (o.tuning) {
        // the table's launch shapes apply under every aggregation policy, its
        // aggregators and thresholds under AUTO only
        const pb_tuning &t = *o.tuning;
        const uint32_t lw = t.light_wg ? t.light_wg : 64u, mw = t.medium_wg ? t.medium_wg : 256u;
        if (!light_wg_ok(lw) || !medium_wg_ok(mw)) return false;
        p->wg[0] = lw;
        p->wg[1] = mw;
        p->width[0] = t.light_width;
        p->width[1] = t.medium_width;
        p->width[2] = t.heavy_width;
        if (o.agg == PB_AGG_AUTO) {
            const pb_agg a[3] = {t.light_agg, t.medium_agg, t.heavy_agg};
            for (int i = 0; i < 3; ++i)
                if (a[i] != PB_AGG_LDS_HASH && a[i] != PB_AGG_DENSE_HIST && a[i] != PB_AGG_RADIX_SORT) return false;
            if (t.light_max > LIGHT_D || t.medium_max > MEDIUM_D || t.light_max > t.medium_max) return false;
            p->light_max = t.light_max;
            p->medium_max = t.medium_max;
            for (int i = 0; i < 3; ++i) p->agg[i] = a[i];
        }
    }
    if (o.wg_size) {
        // one size for the light and medium buckets, where their kernels have it
        const bool l = light_wg_ok(o.wg_size), m = medium_wg_ok(o.wg_size);
        if (!l && !m) return false;
        if (l) p->wg[0] = o.wg_size;
        if (m) p->wg[1] = o.wg_size;
    }
    if (o.agg == PB_AGG_AUTO) return true;
    if (o.agg != PB_AGG_LDS_HASH && o.agg != PB_AGG_DENSE_HIST && o.agg != PB_AGG_RADIX_SORT) return false;
    p->agg[0] = p->agg[1] = p->agg[2] = o.agg;
    p->packed = false;  // a forced aggregator serves every source
    return true;
}

// Runs framework steps 2-4 (Section 3.1) on `in`.  `list_ms`, if given,
// receives the time of each work list's kernel (NLISTS entries).  With
// `region` (device memory of `region_bytes`) every scratch block comes from
// that region and the call allocates nothing, device or pinned host memory:
// no phase timing (events) and no hub tile then.
pb_status count_core(const CoreIn &in, const CoreOut &out, int mode, const pb_opts &opts, const Policy &pol,
                     hipStream_t s, float *list_ms, void *region = nullptr, uint64_t region_bytes = 0) {
    const uint64_t n = in.n, m = in.m, ns = 2 * m;
    const uint32_t ng = in.bl.ng;
    // Chunk and segment sums are 32-bit.  Every chunk holds up-slots of one
    // source x1, whose centres y are distinct vertices of one side, so its
    // wedges number at most the sum of their degrees <= m < 2^31; a run
    // segment's credits sum R(x1, x2) - 1 over distinct x2 of one side, each
    // R <= deg(x2), so they too stay below m.  No degree limit is needed.
    if (opts.stats) *opts.stats = pb_stats{};

    const bool timing = !region && (((opts.flags & PB_FLAG_TIMING) && opts.stats) || list_ms);
    const bool copt = (opts.flags & PB_FLAG_CACHE_OPT) && in.bl.ng <= 1;
    const uint64_t nups = copt ? 2 * in.m : in.m;  // up-slots: every slot, or one per edge
    // events: [0] start, [1] plan done, [2 + i] after list i, [2 + NLISTS] end,
    // then the hub tile's matrix-core kernel and the hub credit pass
    constexpr int NEV = NLISTS + 3;
    constexpr int E_HG0 = NEV, E_HG1 = NEV + 1, E_HP0 = NEV + 2, E_HP1 = NEV + 3;
    struct Events {
        hipEvent_t e[NEV + 4] = {};
        bool ok = false;
        ~Events() {
            for (auto &x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } ev;
    if (timing) {
        ev.ok = true;
        for (auto &x : ev.e) ev.ok = ev.ok && hipEventCreate(&x) == hipSuccess;
        if (ev.ok) ev.ok = hipEventRecord(ev.e[0], s) == hipSuccess;
    }
    auto mark = [&](int i) {
        if (ev.ok) ev.ok = hipEventRecord(ev.e[i], s) == hipSuccess;
    };

    Workspace ws = region ? Workspace(s, region, region_bytes) : Workspace(s, opts.workspace_cap_bytes);
    // plan read-backs: pinned host memory, or a pageable local without a region
    // (the stream is synchronised after each copy either way)
    PlanCounts local_pc{}, *hpc = &local_pc;
    if (!region) PB_TRY_HIP(hipHostMalloc((void **)&hpc, sizeof(PlanCounts), hipHostMallocDefault));
    struct HostFree {
        PlanCounts *p;
        bool pinned;
        ~HostFree() {
            if (pinned) (void)hipHostFree(p);
        }
    } host_free{hpc, !region};

    // With per-edge counts of one graph at hand, per-vertex counts are summed
    // from them at the end (k_vertex_from_edges) and the counting kernels run
    // without per-vertex credits (kmode): no scattered vertex atomics.
    const bool derive_vertex = (mode & MODE_VERTEX) && (mode & MODE_EDGE) && in.v_off && ng == 1;
    const int kmode = derive_vertex ? mode & ~MODE_VERTEX : mode;
    // Accumulators first so an empty graph still writes zeros.
    unsigned long long *gacc = ws.alloc<unsigned long long>(ng);
    unsigned long long *vacc = (kmode & MODE_VERTEX) ? ws.alloc<unsigned long long>(n) : nullptr;
    // A slot's credit is at most b(e) <= (deg(y) - 1)(deg(x2) - 1), so 32-bit
    // slot counters are exact when max_deg^2 < 2^32.
    const bool slot32 = (uint64_t)in.max_deg * in.max_deg < (uint64_t(1) << 32);
    unsigned long long *sacc = (mode & MODE_EDGE) && !slot32 ? ws.alloc<unsigned long long>(ns) : nullptr;
    uint32_t *sacc32 = (mode & MODE_EDGE) && slot32 ? ws.alloc<uint32_t>(ns) : nullptr;
    PlanCounts *pc = ws.alloc<PlanCounts>(1);
    uint32_t *order = ws.alloc<uint32_t>(n), *seen = ws.alloc<uint32_t>(n);
    if (ws.failed) return PB_ERR_NO_MEMORY;
    PB_TRY(fill<uint64_t>((uint64_t *)gacc, 0, ng, s));
    if (vacc) PB_TRY(fill<uint64_t>((uint64_t *)vacc, 0, n, s));
    if (sacc) PB_TRY(fill<uint64_t>((uint64_t *)sacc, 0, ns, s));
    if (sacc32) PB_TRY(fill<uint32_t>(sacc32, 0u, ns, s));
    PB_TRY(fill<uint32_t>((uint32_t *)pc, 0u, sizeof(PlanCounts) / 4, s));

    // 1. rank check (one sync) -------------------------------------------------
    if (n > 0) {
        PB_TRY(fill<uint32_t>(seen, 0u, n, s));
        PB_TRY(fill<uint32_t>(order, 0u, n, s));
        hipLaunchKernelGGL(k_rank_check, dim3(grid_for(n)), dim3(256), 0, s, in.rank, n, order, seen, &pc->flags,
                           &pc->top);
        PB_TRY_HIP(hipGetLastError());
        PB_TRY_HIP(hipMemcpyAsync(hpc, pc, sizeof(PlanCounts), hipMemcpyDeviceToHost, s));
        PB_TRY_HIP(hipStreamSynchronize(s));
        if (hpc->flags & FLAG_BAD_RANK) return PB_ERR_BAD_RANK;
    }
    ws.release(seen);

    // Hub tile candidates (one graph only): the first HUB_T vertices in rank
    // order of the rank-0 vertex's side.
    uint32_t hub_base = 0, hub_end = 0;
    // AUTO: with a credit pass and no source that could take the giant-source
    // path, the tile costs more per hub-pair path than the sparse path (its
    // cost model could not choose it), so it is not even evaluated
    const bool hub_auto_ok = m >= HUB_AUTO_MIN_M && (!(kmode & (MODE_VERTEX | MODE_EDGE)) || in.max_deg >= GH_MIN_UPS);
    if (m > 0 && ng == 1 && !copt && !region && opts.hub != PB_HUB_OFF &&
        (opts.hub == PB_HUB_FORCE || hub_auto_ok)) {
        const bool hub_v = hpc->top >= in.n_u;
        const uint64_t side = hub_v ? n - in.n_u : in.n_u;
        const uint32_t H = (uint32_t)std::min<uint64_t>(HUB_T, side);
        if (H >= 2) {
            hub_base = hub_v ? in.n_u : 0u;
            hub_end = hub_base + H;
        }
    }
    uint32_t *byte_from = nullptr;
    uint32_t *hub_rank = nullptr, *hub_d = nullptr, *hub_off = nullptr;
    unsigned long long *hub_roww = nullptr;
    uint32_t hub_grid = 0;

    uint64_t wtotal = 0;
    PlanCounts plan{};
    bool hub_pass_ran = false;
    // host tables of the giant-source items (alive until the call's last synchronisation)
    std::vector<uint32_t> gh_info;
    std::vector<GhSrc> gh_src;
    std::vector<uint2> gh_items, gh_eitems;
    uint32_t gh_xoff[NXCD + 1] = {}, gh_exoff[NXCD + 1] = {};
    uint32_t *smid = nullptr, *eslot = nullptr;
    if (m > 0) {
        // 2. relabel (Algorithm 1) ---------------------------------------------
        uint32_t *isv = ws.alloc<uint32_t>(n), *vbefore = ws.alloc<uint32_t>(n + 1);
        uint32_t *rdeg = ws.alloc<uint32_t>(n), *roff = ws.alloc<uint32_t>(n + 1);
        uint32_t *cend = ws.alloc<uint32_t>(n), *gid = ng > 1 ? ws.alloc<uint32_t>(n) : nullptr;
        smid = ws.alloc<uint32_t>(n);
        if (ws.failed) return PB_ERR_NO_MEMORY;
        hipLaunchKernelGGL(k_rank_side, dim3(grid_for(n)), dim3(256), 0, s, order, in.deg, n, in.n_u, isv, rdeg);
        PB_TRY((scan_exclusive<uint32_t, uint32_t>(isv, vbefore, n, vbefore + n, ws)));
        hipLaunchKernelGGL(k_smid, dim3(grid_for(n)), dim3(256), 0, s, isv, vbefore, n, in.n_u, smid);
        PB_TRY((scan_exclusive<uint32_t, uint32_t>(rdeg, roff, n, roff + n, ws)));
        hipLaunchKernelGGL(k_cend, dim3(grid_for(n)), dim3(256), 0, s, isv, n, in.n_u, ng, in.bl.rbase, in.bl.ubase,
                           in.bl.vbase, cend, gid);
        if (copt) hipLaunchKernelGGL(k_cend_copt, dim3(grid_for(n)), dim3(256), 0, s, (const uint32_t *)smid, n, cend);
        // byte windows (one graph): each side from one past its last id of degree >= 256
        byte_from = ws.alloc<uint32_t>(4);
        if (ws.failed) return PB_ERR_NO_MEMORY;
        {
            for (int t = 0; t < 2; ++t) {
                PB_TRY(fill<uint32_t>(byte_from + 2 * t, ng <= 1 ? 0u : (uint32_t)n, 1, s));
                PB_TRY(fill<uint32_t>(byte_from + 2 * t + 1, ng <= 1 ? in.n_u : (uint32_t)n, 1, s));
            }
            if (ng <= 1)
                hipLaunchKernelGGL(k_byte_from, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, in.rank,
                                   (const uint32_t *)smid, in.deg, n, in.n_u, byte_from);
            PB_TRY_HIP(hipGetLastError());
        }
        ws.release(vbefore);
        ws.release(rdeg);

        const int b = bits_for(n - 1);
        uint64_t *k0 = ws.alloc<uint64_t>(ns), *k1 = ws.alloc<uint64_t>(ns);
        uint32_t *v0 = ws.alloc<uint32_t>(ns), *v1 = ws.alloc<uint32_t>(ns);
        if (ws.failed) return PB_ERR_NO_MEMORY;
        uint64_t *ks;
        uint32_t *vs;
        if (in.v_off) {
            // one graph: destination-major keys, then a sort on the source bits only
            uint32_t *dcnt = ws.alloc<uint32_t>(n + 1), *dcoff = ws.alloc<uint32_t>(n + 1);
            if (ws.failed) return PB_ERR_NO_MEMORY;
            const DestRows D{order, roff, in.rank, in.u_off, in.u_adj, in.v_off, in.v_adj, in.v_eid, in.n_u, ns, b};
            hipLaunchKernelGGL(k_dest_small, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, D, n, k0, v0, dcnt);
            PB_TRY((scan_exclusive<uint32_t, uint32_t>(dcnt, dcoff, n, dcoff + n, ws)));
            hipLaunchKernelGGL(k_dest_long, dim3(DEST_GRID), dim3(256), 0, s, D, n, (const uint32_t *)dcoff, k0, v0);
            PB_TRY_HIP(hipGetLastError());
            ws.release(dcoff);
            ws.release(dcnt);
            PB_TRY(radix_sort_pairs_bits(k0, v0, k1, v1, ns, b, 2 * b, ws, &ks, &vs));
        } else {
            hipLaunchKernelGGL(k_slot_keys, dim3(grid_for(m)), dim3(256), 0, s, in.eu, in.ev, in.rank, m, in.n_u, b,
                               k0, v0);
            PB_TRY_HIP(hipGetLastError());
            PB_TRY(radix_sort_pairs(k0, v0, k1, v1, ns, 2 * b, ws, &ks, &vs));
        }

        uint32_t *nbr = ws.alloc<uint32_t>(ns + NBR_PAD);
        eslot = ws.alloc<uint32_t>(ns);
        uint32_t *hideg = ws.alloc<uint32_t>(n + 1), *upoff = ws.alloc<uint32_t>(n + 1);
        if (ws.failed) return PB_ERR_NO_MEMORY;
        PB_TRY(fill<uint32_t>(hideg, 0u, n + 1, s));
        PB_TRY(fill<uint32_t>(nbr + ns, 0u, NBR_PAD, s));
        hipLaunchKernelGGL(k_slots, dim3(grid_for(ns)), dim3(256), 0, s, ks, vs, ns, b, smid, roff, nbr, eslot,
                           hideg);
        uint32_t *uprun = ws.alloc<uint32_t>(nups), *uplen = ws.alloc<uint32_t>(nups);
        if (ws.failed) return PB_ERR_NO_MEMORY;
        if (copt) {
            // every slot is an up-slot: upoff is roff
            PB_TRY_HIP(hipMemcpyAsync(upoff, roff, (n + 1) * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
            hipLaunchKernelGGL(k_upslots_copt, dim3(grid_for(ns)), dim3(256), 0, s, ks, vs, ns, b, roff,
                               (const uint32_t *)hideg, eslot, uprun, uplen);
        } else {
            PB_TRY((scan_exclusive<uint32_t, uint32_t>(hideg, upoff, n, upoff + n, ws)));
            hipLaunchKernelGGL(k_upslots, dim3(grid_for(ns)), dim3(256), 0, s, ks, vs, ns, b, roff, upoff, eslot,
                               uprun, uplen);
        }
        PB_TRY_HIP(hipGetLastError());
        ws.release(k0);
        ws.release(k1);
        ws.release(v0);
        ws.release(v1);
        ws.release(hideg);
        ws.release(isv);

        // 3a. hub tile: R of hub pairs on matrix cores, C(R,2) credits ------------
        if (hub_end > hub_base) {
            hub_rank = ws.alloc<uint32_t>(HUB_T);
            hub_d = ws.alloc<uint32_t>((uint64_t)HUB_T * HUB_T);
            hub_roww = ws.alloc<unsigned long long>(HUB_T);
            hub_off = ws.alloc<uint32_t>(HUB_T + 1);
            if (ws.failed) return PB_ERR_NO_MEMORY;
            const HubIn hin{n,       in.n_u,  smid,
                            roff,    upoff,   nbr,
                            hub_base, hub_end, opts.hub == PB_HUB_FORCE,
                            (kmode & (MODE_VERTEX | MODE_EDGE)) != 0, gacc, vacc};
            PB_TRY(hub_tile(hin, &pc->hub, HubOut{hub_rank, hub_d, hub_roww}, ws, s, ev.ok ? ev.e[E_HG0] : nullptr,
                            ev.ok ? ev.e[E_HG1] : nullptr, &hub_grid, &hpc->hub.on));
            if (kmode & (MODE_VERTEX | MODE_EDGE))
                hipLaunchKernelGGL(k_hub_items, dim3(1), dim3(HUB_T), 0, s, (const uint32_t *)upoff,
                                   (const uint32_t *)hub_rank, hub_end - hub_base, hub_off, pc);
            PB_TRY_HIP(hipGetLastError());
        }

        // 3. plan: wedges per source, bucket by distinct-endpoint bound -------
        uint64_t *wscan = ws.alloc<uint64_t>(nups + 1);
        uint32_t *lists = ws.alloc<uint32_t>((uint64_t)NLISTS * n);
        uint32_t *nwin = ws.alloc<uint32_t>((uint64_t)NSORTED * n);
        uint64_t *wl = ws.alloc<uint64_t>((uint64_t)NSORTED * n);
        if (ws.failed) return PB_ERR_NO_MEMORY;
        PB_TRY((scan_exclusive<uint32_t, uint64_t>(uplen, wscan, nups, wscan + nups, ws)));
        hipLaunchKernelGGL(k_plan, dim3(grid_for(n, 256, PLAN_GRID)), dim3(256), 0, s, upoff, wscan, smid, cend, n,
                           pol, hub_base, hub_end, (const unsigned long long *)hub_roww, lists, nwin, wl, pc,
                           copt ? in.n_u + 1 : 0u);
        PB_TRY_HIP(hipGetLastError());
        PB_TRY_HIP(hipMemcpyAsync(hpc, pc, sizeof(PlanCounts), hipMemcpyDeviceToHost, s));
        PB_TRY_HIP(hipMemcpyAsync(&wtotal, wscan + nups, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        PB_TRY_HIP(hipStreamSynchronize(s));
        plan = *hpc;
        ws.release(wscan);
        auto list_of = [&](int l) { return (const uint32_t *)(lists + (uint64_t)l * n); };

        // most-wedges-first order for the window lists
        const uint32_t *sorted_src[NSORTED] = {};
        const uint64_t *sorted_w[NSORTED] = {};
        uint2 *items = nullptr;
        uint32_t *cur = nullptr, *nxt = nullptr, *cval = nullptr, *nval = nullptr;
        for (int l = 0; l < NLISTS; ++l) {
            const int sk = sorted_slot(l);
            const uint32_t nh = plan.list[l];
            if (sk < 0 || nh == 0) continue;
            uint64_t *hk0 = ws.alloc<uint64_t>(nh), *hk1 = ws.alloc<uint64_t>(nh);
            uint32_t *hv0 = ws.alloc<uint32_t>(nh), *hv1 = ws.alloc<uint32_t>(nh);
            uint32_t *hnw = ws.alloc<uint32_t>(nh), *hsrc = ws.alloc<uint32_t>(nh);
            uint64_t *hw = ws.alloc<uint64_t>(nh);
            if (ws.failed) return PB_ERR_NO_MEMORY;
            const uint32_t *nw = nwin + (uint64_t)sk * n;
            const uint64_t *w = wl + (uint64_t)sk * n;
            hipLaunchKernelGGL(k_heavy_keys, dim3(grid_for(nh)), dim3(256), 0, s, nw, w, nh, hk0, hv0);
            uint64_t *hks;
            uint32_t *hvs;
            PB_TRY(radix_sort_pairs(hk0, hv0, hk1, hv1, nh, 32, ws, &hks, &hvs));
            hipLaunchKernelGGL(k_heavy_gather, dim3(grid_for(nh)), dim3(256), 0, s, hvs, list_of(l), nw, w, nh, hsrc,
                               hnw, hw);
            if (l == L_HASH_WIN) {
                uint32_t *hoff = ws.alloc<uint32_t>(nh + 1);
                items = ws.alloc<uint2>(plan.items);
                if (ws.failed) return PB_ERR_NO_MEMORY;
                PB_TRY((scan_exclusive<uint32_t, uint32_t>(hnw, hoff, nh, hoff + nh, ws)));
                hipLaunchKernelGGL(k_heavy_expand, dim3(grid_for(nh)), dim3(256), 0, s, hsrc, hnw, hoff, nh, items);
            } else if (!cur && (l == L_DENSE_HEAVY || l == L_SORT_HEAVY || l == L_HASH_PACKED)) {
                cur = ws.alloc<uint32_t>(nups);
                nxt = ws.alloc<uint32_t>(nups);
                cval = ws.alloc<uint32_t>(nups);
                nval = ws.alloc<uint32_t>(nups);
                if (ws.failed) return PB_ERR_NO_MEMORY;
            }
            PB_TRY_HIP(hipGetLastError());
            sorted_src[sk] = hsrc;
            sorted_w[sk] = hw;
        }

        // 4. count ---------------------------------------------------------------
        const bool hub_on = plan.hub.on && hub_end > hub_base;
        Ranked G{roff, nbr, upoff, uprun, uplen, smid, cend, gid, in.n_u, (uint32_t)n,
                 hub_on ? hub_base : 0u, hub_on ? hub_end : 0u, copt};
        Acc A{gacc, vacc, sacc, sacc32, &pc->flags, kmode};

        // giant sources: per-die item lists, built on the host (one extra
        // synchronisation, only when there are such sources)
        GhSrc *d_gh_src = nullptr;
        uint2 *d_gh_items = nullptr, *d_gh_eitems = nullptr;
        uint32_t *d_gh_xoff = nullptr, *d_gh_exoff = nullptr, *gh_hist = nullptr;
        uint64_t gh_total = 0;
        // hubs whose pass 2 the giant-source walk does (read by the hub credit pass)
        uint32_t *gh_hub = ws.alloc<uint32_t>(HUB_T);
        if (ws.failed) return PB_ERR_NO_MEMORY;
        PB_TRY(fill<uint32_t>(gh_hub, 0u, HUB_T, s));
        if (const uint32_t c = plan.list[L_DENSE_GLOBAL]) {
            uint32_t *d_info = ws.alloc<uint32_t>(4ull * c);
            if (ws.failed) return PB_ERR_NO_MEMORY;
            hipLaunchKernelGGL(k_gh_info, dim3(grid_for(c)), dim3(256), 0, s, G, sorted_src[sorted_slot(L_DENSE_GLOBAL)],
                               c, d_info, gh_hub);
            PB_TRY_HIP(hipGetLastError());
            gh_info.resize(4ull * c);
            PB_TRY_HIP(hipMemcpyAsync(gh_info.data(), d_info, 16ull * c, hipMemcpyDeviceToHost, s));
            PB_TRY_HIP(hipStreamSynchronize(s));
            // sources are in most-wedges-first order: deal them round-robin to the dies
            std::vector<uint2> per_w[NXCD], per_e[NXCD];
            gh_src.resize(c);
            for (uint32_t i = 0; i < c; ++i) {
                const uint32_t *f = &gh_info[4ull * i];
                gh_src[i] = GhSrc{f[0], f[1], f[2], f[3], gh_total};
                gh_total += f[3];
                for (uint32_t j = 0; j < ceil_div(f[2], GH_CHUNK); ++j) per_w[i % NXCD].push_back(make_uint2(i, j));
                for (uint32_t j = 0; j < ceil_div(f[3], GH_SEG); ++j) per_e[i % NXCD].push_back(make_uint2(i, j));
            }
            for (uint32_t x = 0; x < NXCD; ++x) {
                gh_xoff[x] = (uint32_t)gh_items.size();
                gh_exoff[x] = (uint32_t)gh_eitems.size();
                gh_items.insert(gh_items.end(), per_w[x].begin(), per_w[x].end());
                gh_eitems.insert(gh_eitems.end(), per_e[x].begin(), per_e[x].end());
            }
            gh_xoff[NXCD] = (uint32_t)gh_items.size();
            gh_exoff[NXCD] = (uint32_t)gh_eitems.size();
            d_gh_src = ws.alloc<GhSrc>(c);
            d_gh_items = ws.alloc<uint2>(gh_items.size());
            d_gh_eitems = ws.alloc<uint2>(gh_eitems.size());
            d_gh_xoff = ws.alloc<uint32_t>(2 * (NXCD + 1));
            gh_hist = ws.alloc<uint32_t>(gh_total);
            if (ws.failed) return PB_ERR_NO_MEMORY;
            d_gh_exoff = d_gh_xoff + NXCD + 1;
            PB_TRY_HIP(hipMemcpyAsync(d_gh_src, gh_src.data(), sizeof(GhSrc) * c, hipMemcpyHostToDevice, s));
            PB_TRY_HIP(hipMemcpyAsync(d_gh_items, gh_items.data(), sizeof(uint2) * gh_items.size(),
                                      hipMemcpyHostToDevice, s));
            PB_TRY_HIP(hipMemcpyAsync(d_gh_eitems, gh_eitems.data(), sizeof(uint2) * gh_eitems.size(),
                                      hipMemcpyHostToDevice, s));
            PB_TRY_HIP(hipMemcpyAsync(d_gh_xoff, gh_xoff, sizeof(gh_xoff), hipMemcpyHostToDevice, s));
            PB_TRY_HIP(hipMemcpyAsync(d_gh_exoff, gh_exoff, sizeof(gh_exoff), hipMemcpyHostToDevice, s));
        }
        mark(1);
        for (int l = 0; l < NLISTS; ++l) {
            const uint32_t c = plan.list[l];
            if (c) {
                switch (l) {
                    case L_DENSE_HEAVY:
                        launch_items(k_count_heavy<1024, 4>, c, 1024, pol.width[2], s, G, A, sorted_src[2], sorted_w[2],
                                     cur, nxt, cval, nval, (const uint32_t *)byte_from);
                        break;
                    case L_SORT_HEAVY:
                        launch_items(k_count_sort_heavy<256, 4, SORT_W>, c, 256, pol.width[2], s, G, A, sorted_src[1],
                                     sorted_w[1], cur, nxt, cval, nval);
                        break;
                    case L_HASH_WIN:
                        launch_items(k_count_hash_win<256, 4, 2 * HASH_WIN>, plan.items, 256, pol.width[2], s, G, A,
                                     (const uint2 *)items);
                        break;
                    case L_HASH_MEDIUM: {
                        const uint32_t t = pol.wg[1], w = pol.width[1];
                        if (t == 128) launch_items(k_count_hash<128, 4, 2 * MEDIUM_D>, c, t, w, s, G, A, list_of(l));
                        else if (t == 512) launch_items(k_count_hash<512, 4, 2 * MEDIUM_D>, c, t, w, s, G, A, list_of(l));
                        else launch_items(k_count_hash<256, 4, 2 * MEDIUM_D>, c, 256, w, s, G, A, list_of(l));
                        break;
                    }
                    case L_HASH_LIGHT: {
                        const uint32_t t = pol.wg[0], w = pol.width[0];
                        if (t == 128) launch_items(k_count_hash<128, 4, 2 * LIGHT_D>, c, t, w, s, G, A, list_of(l));
                        else if (t == 256) launch_items(k_count_hash<256, 4, 2 * LIGHT_D>, c, t, w, s, G, A, list_of(l));
                        else launch_items(k_count_hash<64, 4, 2 * LIGHT_D>, c, 64, w, s, G, A, list_of(l));
                        break;
                    }
                    case L_SORT_MEDIUM: {
                        const uint32_t t = pol.wg[1], w = pol.width[1];
                        if (t == 128) launch_items(k_count_sort<128, 4, SORT_W>, c, t, w, s, G, A, list_of(l));
                        else if (t == 512) launch_items(k_count_sort<512, 4, SORT_W>, c, t, w, s, G, A, list_of(l));
                        else launch_items(k_count_sort<256, 4, SORT_W>, c, 256, w, s, G, A, list_of(l));
                        break;
                    }
                    case L_SORT_LIGHT: {
                        const uint32_t t = pol.wg[0], w = pol.width[0];
                        if (t == 128) launch_items(k_count_sort<128, 4, SORT_LIGHT_W>, c, t, w, s, G, A, list_of(l));
                        else if (t == 256) launch_items(k_count_sort<256, 4, SORT_LIGHT_W>, c, t, w, s, G, A, list_of(l));
                        else launch_items(k_count_sort<64, 4, SORT_LIGHT_W>, c, 64, w, s, G, A, list_of(l));
                        break;
                    }
                    case L_DENSE_SMALL: {
                        const uint32_t t = pol.wg[1], w = pol.width[1];
                        if (t == 128) launch_items(k_count_dense_src<128, 4, SMALL_WIN>, c, t, w, s, G, A, list_of(l));
                        else if (t == 512) launch_items(k_count_dense_src<512, 4, SMALL_WIN>, c, t, w, s, G, A, list_of(l));
                        else launch_items(k_count_dense_src<256, 4, SMALL_WIN>, c, 256, w, s, G, A, list_of(l));
                        break;
                    }
                    case L_HASH_PACKED:
                        launch_items(k_count_phash<PH_T, 4>, c, PH_T, pol.width[2], s, G, A, sorted_src[sorted_slot(l)],
                                     sorted_w[sorted_slot(l)], cur, nxt, cval, nval);
                        break;
                    case L_DENSE_GLOBAL: {
                        const dim3 grid(NXCD * GH_WG_PER_XCD);
                        PB_TRY(fill<uint32_t>(gh_hist, 0u, gh_total, s));
                        const dim3 walk_grid(NXCD * GH_WG_PER_XCD * 256 / GH_T);
                        k_gh_walk<GH_T, 4, 1><<<walk_grid, GH_T, 0, s>>>(G, A, d_gh_src, d_gh_items, d_gh_xoff,
                                                                         gh_hist, nullptr);
                        k_gh_endpoint<256><<<grid, 256, 0, s>>>(G, A, d_gh_src, d_gh_eitems, d_gh_exoff, gh_hist);
                        if (kmode & (MODE_VERTEX | MODE_EDGE))
                            k_gh_walk<GH_T, 4, 2><<<walk_grid, GH_T, 0, s>>>(
                                G, A, d_gh_src, d_gh_items, d_gh_xoff, gh_hist, hub_on ? (const uint32_t *)hub_d : nullptr);
                        break;
                    }
                }
                PB_TRY_HIP(hipGetLastError());
            }
            mark(2 + l);
        }
        if (hub_on && (kmode & (MODE_VERTEX | MODE_EDGE)) && plan.hub_items) {
            hub_pass_ran = true;
            if (ev.ok) ev.ok = hipEventRecord(ev.e[E_HP0], s) == hipSuccess;
            k_count_hub_pass<256, 4><<<dim3(std::min(plan.hub_items, HUB_PASS_GRID)), dim3(256), 0, s>>>(
                G, A, hub_rank, hub_off, hub_d, gh_hub);
            PB_TRY_HIP(hipGetLastError());
            if (ev.ok) ev.ok = hipEventRecord(ev.e[E_HP1], s) == hipSuccess;
        }
    } else {
        for (int l = 0; l < NLISTS; ++l) mark(1 + l);
        mark(1 + NLISTS);
    }

    // 5. outputs -------------------------------------------------------------------
    if ((mode & MODE_EDGE) && m)
        hipLaunchKernelGGL(k_out_edge, dim3(grid_for(m)), dim3(256), 0, s, eslot, sacc, sacc32, m, in.bl, out);
    if (derive_vertex) {
        uint32_t *vcnt = ws.alloc<uint32_t>(n + 1), *vcoff = ws.alloc<uint32_t>(n + 1);
        if (ws.failed) return PB_ERR_NO_MEMORY;
        const int64_t *eo = out.eout;
        hipLaunchKernelGGL(k_vtx_short, dim3(grid_for(n)), dim3(256), 0, s, in.u_off, in.v_off, in.v_eid, in.n_u, n,
                           eo, out.vout, vcnt);
        PB_TRY((scan_exclusive<uint32_t, uint32_t>(vcnt, vcoff, n, vcoff + n, ws)));
        hipLaunchKernelGGL(k_vtx_long, dim3(4096), dim3(256), 0, s, in.u_off, in.v_off, in.v_eid, in.n_u, n,
                           (const uint32_t *)vcoff, eo, out.vout);
        hipLaunchKernelGGL(k_vtx_halve, dim3(grid_for(n)), dim3(256), 0, s, (const uint32_t *)vcnt, n, out.vout);
    } else if (mode & MODE_VERTEX)
        hipLaunchKernelGGL(k_out_vertex, dim3(grid_for(n)), dim3(256), 0, s, in.rank, smid, m ? vacc : nullptr, n,
                           in.n_u, in.bl, out);
    if (mode & MODE_GLOBAL) hipLaunchKernelGGL(k_out_global, dim3(grid_for(ng)), dim3(256), 0, s, gacc, ng, out);
    PB_TRY_HIP(hipGetLastError());
    mark(2 + NLISTS);
    PB_TRY_HIP(hipMemcpyAsync(hpc, pc, sizeof(PlanCounts), hipMemcpyDeviceToHost, s));
    PB_TRY_HIP(hipStreamSynchronize(s));
    if (hpc->flags & FLAG_INTERNAL) return PB_ERR_INTERNAL;

    // t[0] prepare, t[1 + l] list l, t[1 + NLISTS] output; hub kernels apart
    float t[NEV - 1] = {}, t_gemm = 0, t_hub_pass = 0;
    if (timing && ev.ok) {
        for (int i = 0; i + 1 < NEV; ++i) (void)hipEventElapsedTime(&t[i], ev.e[i], ev.e[i + 1]);
        if (hub_pass_ran) {
            (void)hipEventElapsedTime(&t_hub_pass, ev.e[E_HP0], ev.e[E_HP1]);
            (void)hipEventElapsedTime(&t[1 + NLISTS], ev.e[E_HP1], ev.e[2 + NLISTS]);
        }
        if (hub_grid && plan.hub.on) (void)hipEventElapsedTime(&t_gemm, ev.e[E_HG0], ev.e[E_HG1]);
    }
    if (list_ms)
        for (int l = 0; l < NLISTS; ++l) list_ms[l] = t[1 + l];
    if (opts.stats) {
        pb_stats &st = *opts.stats;
        st.wedges = wtotal;
        st.sources = plan.sources;
        st.sources_hash =
            plan.list[L_HASH_LIGHT] + plan.list[L_HASH_MEDIUM] + plan.list[L_HASH_WIN] + plan.list[L_HASH_PACKED];
        st.sources_dense = plan.list[L_DENSE_HEAVY] + plan.list[L_DENSE_SMALL] + plan.list[L_DENSE_GLOBAL];
        st.sources_sort = plan.list[L_SORT_LIGHT] + plan.list[L_SORT_MEDIUM] + plan.list[L_SORT_HEAVY];
        st.window_items = plan.items + plan.list[L_DENSE_HEAVY] + plan.list[L_SORT_HEAVY];
        st.wedges_hash = plan.wedges[L_HASH_LIGHT] + plan.wedges[L_HASH_MEDIUM] + plan.wedges[L_HASH_WIN] +
                         plan.wedges[L_HASH_PACKED];
        st.wedges_dense = plan.wedges[L_DENSE_HEAVY] + plan.wedges[L_DENSE_SMALL] + plan.wedges[L_DENSE_GLOBAL];
        st.wedges_sort = plan.wedges[L_SORT_LIGHT] + plan.wedges[L_SORT_MEDIUM] + plan.wedges[L_SORT_HEAVY];
        st.workspace_bytes = ws.peak;
        st.wedges_heavy = plan.wedges[L_DENSE_HEAVY];
        st.wedges_global = plan.wedges[L_DENSE_GLOBAL];
        st.slot_credit_bytes = sacc32 ? 4u : sacc ? 8u : 0u;
        if (hub_grid && plan.hub.on) {
            st.wedges_hub = plan.hub.wedges;
            st.hub_rows = hub_end - hub_base;
            st.hub_cols = plan.hub.cols;
            st.hub_mfma_ops = hub_gemm_ops(plan.hub.cols);
        }
        if (timing && ev.ok) {
            st.ms_heavy = t[1 + L_DENSE_HEAVY];
            st.ms_global = t[1 + L_DENSE_GLOBAL];
            st.ms_hub_gemm = t_gemm;
            st.ms_hub_pass = t_hub_pass;
            st.ms_prepare = t[0];
            st.ms_hash = t[1 + L_HASH_LIGHT] + t[1 + L_HASH_MEDIUM] + t[1 + L_HASH_WIN] + t[1 + L_HASH_PACKED];
            st.ms_dense = t[1 + L_DENSE_HEAVY] + t[1 + L_DENSE_SMALL] + t[1 + L_DENSE_GLOBAL];
            st.ms_sort = t[1 + L_SORT_LIGHT] + t[1 + L_SORT_MEDIUM] + t[1 + L_SORT_HEAVY];
            st.ms_output = t[1 + NLISTS];
        }
    }
    return PB_OK;
}

pb_status check_opts(const pb_opts *opts_in, pb_opts *opts, Policy *pol) {
    pb_opts_default(opts);
    if (opts_in) *opts = *opts_in;
    if ((int)opts->agg < PB_AGG_AUTO || (int)opts->agg > PB_AGG_RADIX_SORT) return PB_ERR_INVALID_ARG;
    if ((int)opts->hub < PB_HUB_AUTO || (int)opts->hub > PB_HUB_FORCE) return PB_ERR_INVALID_ARG;
    if (!policy_from(*opts, pol)) return PB_ERR_INVALID_ARG;
    return PB_OK;
}

pb_status count_impl(pb_graph *g, const uint32_t *rank, const pb_opts *opts_in, int64_t *gout, int64_t *vout,
                     int64_t *eout, hipStream_t s) {
    if (!g || !rank) return PB_ERR_INVALID_ARG;
    if (!gout && !vout && !eout) return PB_ERR_INVALID_ARG;
    pb_opts opts;
    Policy pol;
    PB_TRY(check_opts(opts_in, &opts, &pol));
    const int mode = (gout ? MODE_GLOBAL : 0) | (vout ? MODE_VERTEX : 0) | (eout ? MODE_EDGE : 0);
    CoreIn in{(uint64_t)g->n_u + g->n_v, g->n_u, g->m, g->eu, g->u_adj, g->deg, rank, g->max_deg,
              BatchLayout{1, nullptr, nullptr, nullptr, nullptr}, g->u_off, g->u_adj, g->v_off, g->v_adj, g->v_eid};
    CoreOut out{gout, vout, eout, nullptr, nullptr, nullptr};
    return count_core(in, out, mode, opts, pol, s, nullptr);
}

// ---------------------------------------------------------------- batches

struct GraphDesc {
    const uint32_t *eu, *uadj, *deg, *rank;
    uint32_t n_u, n_v;
    uint64_t m;
    uint32_t ubase, vbase, rbase;
    uint64_t ebase;
};

__global__ void k_union_edges(const GraphDesc *gd, const uint64_t *ebase, uint32_t ng, uint64_t m, uint32_t *eu,
                              uint32_t *ev) {
    GRID_STRIDE(e, m) {
        const uint32_t j = graph_of<uint64_t>(ebase, ng, e);
        const GraphDesc &d = gd[j];
        const uint64_t le = e - d.ebase;
        eu[e] = d.ubase + d.eu[le];
        ev[e] = d.vbase + d.uadj[le];
    }
}

// deg and rank of the union; rank of graph j's vertex = rbase[j] + its rank in j
__global__ void k_union_vertices(const GraphDesc *gd, const uint32_t *ubase, const uint32_t *vbase, uint32_t ng,
                                 uint64_t n, uint32_t n_u, uint32_t *deg, uint32_t *rank, uint32_t *flags) {
    GRID_STRIDE(x, n) {
        uint32_t j, local;
        if (x < n_u) {
            j = graph_of<uint32_t>(ubase, ng, (uint32_t)x);
            local = (uint32_t)x - ubase[j];
        } else {
            const uint32_t xv = (uint32_t)(x - n_u);
            j = graph_of<uint32_t>(vbase, ng, xv);
            local = gd[j].n_u + (xv - vbase[j]);
        }
        const GraphDesc &d = gd[j];
        deg[x] = d.deg[local];
        const uint32_t r = d.rank[local];
        if (r >= d.n_u + d.n_v) atomicOr(flags, FLAG_BAD_RANK);
        rank[x] = d.rbase + (r < d.n_u + d.n_v ? r : 0u);
    }
}

struct BatchBuild {
    CoreIn in;
    CoreOut out;
    int mode;
};

// Lays out the batch as one disjoint union (device arrays in `ws`).
pb_status build_batch(pb_graph *const *gs, const uint32_t *const *ranks, uint32_t count, int64_t *const *gouts,
                      int64_t *const *vouts, int64_t *const *eouts, Workspace &ws, hipStream_t s, BatchBuild *bb) {
    if (!gs || !ranks || count == 0) return PB_ERR_INVALID_ARG;
    if (!gouts && !vouts && !eouts) return PB_ERR_INVALID_ARG;
    std::vector<GraphDesc> gd(count);
    std::vector<uint32_t> ub(count + 1), vb(count + 1), rb(count + 1);
    std::vector<uint64_t> eb(count + 1);
    uint64_t U = 0, V = 0, M = 0, N = 0;
    uint32_t max_deg = 0;
    for (uint32_t j = 0; j < count; ++j) {
        const pb_graph *g = gs[j];
        if (!g || !ranks[j]) return PB_ERR_INVALID_ARG;
        if ((gouts && !gouts[j]) || (vouts && !vouts[j]) || (eouts && !eouts[j] && g->m)) return PB_ERR_INVALID_ARG;
        ub[j] = (uint32_t)U;
        vb[j] = (uint32_t)V;
        rb[j] = (uint32_t)N;
        eb[j] = M;
        gd[j] = GraphDesc{g->eu, g->u_adj, g->deg, ranks[j], g->n_u, g->n_v, g->m, (uint32_t)U, (uint32_t)V,
                          (uint32_t)N, M};
        U += g->n_u;
        V += g->n_v;
        M += g->m;
        N += (uint64_t)g->n_u + g->n_v;
        max_deg = std::max(max_deg, g->max_deg);
        if (N >= 0xFFFFFFFFull || M >= (uint64_t(1) << 31)) return PB_ERR_INVALID_ARG;
    }
    ub[count] = (uint32_t)U;
    vb[count] = (uint32_t)V;
    rb[count] = (uint32_t)N;
    eb[count] = M;

    GraphDesc *d_gd = ws.alloc<GraphDesc>(count);
    uint32_t *d_ub = ws.alloc<uint32_t>(count + 1), *d_vb = ws.alloc<uint32_t>(count + 1);
    uint32_t *d_rb = ws.alloc<uint32_t>(count + 1);
    uint64_t *d_eb = ws.alloc<uint64_t>(count + 1);
    int64_t **d_outs[3] = {nullptr, nullptr, nullptr};
    int64_t *const *h_outs[3] = {gouts, vouts, eouts};
    for (int k = 0; k < 3; ++k)
        if (h_outs[k]) d_outs[k] = ws.alloc<int64_t *>(count);
    uint32_t *eu = ws.alloc<uint32_t>(M), *ev = ws.alloc<uint32_t>(M);
    uint32_t *deg = ws.alloc<uint32_t>(N), *rank = ws.alloc<uint32_t>(N), *flags = ws.alloc<uint32_t>(1);
    if (ws.failed) return PB_ERR_NO_MEMORY;
    // host -> device copies of the layout (pageable sources: the copy completes
    // before the call returns)
    PB_TRY_HIP(hipMemcpyAsync(d_gd, gd.data(), count * sizeof(GraphDesc), hipMemcpyHostToDevice, s));
    PB_TRY_HIP(hipMemcpyAsync(d_ub, ub.data(), (count + 1) * 4, hipMemcpyHostToDevice, s));
    PB_TRY_HIP(hipMemcpyAsync(d_vb, vb.data(), (count + 1) * 4, hipMemcpyHostToDevice, s));
    PB_TRY_HIP(hipMemcpyAsync(d_rb, rb.data(), (count + 1) * 4, hipMemcpyHostToDevice, s));
    PB_TRY_HIP(hipMemcpyAsync(d_eb, eb.data(), (count + 1) * 8, hipMemcpyHostToDevice, s));
    for (int k = 0; k < 3; ++k)
        if (h_outs[k])
            PB_TRY_HIP(hipMemcpyAsync(d_outs[k], h_outs[k], count * sizeof(int64_t *), hipMemcpyHostToDevice, s));
    PB_TRY(fill<uint32_t>(flags, 0u, 1, s));
    if (M) hipLaunchKernelGGL(k_union_edges, dim3(grid_for(M)), dim3(256), 0, s, d_gd, d_eb, count, M, eu, ev);
    if (N)
        hipLaunchKernelGGL(k_union_vertices, dim3(grid_for(N)), dim3(256), 0, s, d_gd, d_ub, d_vb, count, N,
                           (uint32_t)U, deg, rank, flags);
    PB_TRY_HIP(hipGetLastError());
    uint32_t hflag = 0;
    PB_TRY_HIP(hipMemcpyAsync(&hflag, flags, 4, hipMemcpyDeviceToHost, s));
    PB_TRY_HIP(hipStreamSynchronize(s));
    if (hflag & FLAG_BAD_RANK) return PB_ERR_BAD_RANK;
    bb->mode = (gouts ? MODE_GLOBAL : 0) | (vouts ? MODE_VERTEX : 0) | (eouts ? MODE_EDGE : 0);
    bb->in = CoreIn{N, (uint32_t)U, M, eu, ev, deg, rank, max_deg, BatchLayout{count, d_ub, d_vb, d_rb, d_eb},
                    nullptr, nullptr, nullptr, nullptr, nullptr};
    bb->out = CoreOut{nullptr, nullptr, nullptr, d_outs[0], d_outs[1], d_outs[2]};
    return PB_OK;
}

// ---------------------------------------------------------------- allocation-free counting

// Device scratch of pb_count_noalloc: one array per device, held for the life
// of the process.  Host code reaches it only through the address
// hipGetSymbolAddress gives on each device.
static __device__ __align__(256) unsigned char scratch[PB_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
struct NoallocDevice {
    std::mutex mu;
    void *ptr = nullptr;  // the array's address on this device, once looked up
};
NoallocDevice noalloc_devices[NOALLOC_MAX_DEVICES];

// An upper bound on the scratch one counting call carves from the array for
// a graph of n vertices and m edges, before the data-dependent tables (window
// items of forced hashing, giant-source histograms), which are checked when
// they are sized.  Per vertex: 4-byte rank, side, offset and degree tables,
// the 8-byte vertex credits, the work lists and the per-vertex derivation's
// item counts (204 bytes in all).  Per
// up-slot: run start and length, four cursors and the wedge scan (32 bytes;
// m up-slots, 2m with the cache-optimised order).  Per edge: sort keys and
// values in two buffers (48 bytes), the ranked lists and slot table (16),
// slot credits (16) and the sort histograms; plus block rounding.
inline uint64_t noalloc_need(uint64_t n, uint64_t m, bool copt) {
    const uint64_t ups = copt ? 2 * m : m;
    return 208 * n + 84 * m + 32 * ups + (uint64_t(1) << 16);
}

}  // namespace

extern "C" {

pb_status pb_count(pb_graph *g, const uint32_t *rank, const pb_opts *opts, int64_t *global_out, int64_t *vertex_out,
                   int64_t *edge_out, hipStream_t stream) {
    return count_impl(g, rank, opts, global_out, vertex_out, edge_out, stream);
}

pb_status pb_count_global(pb_graph *g, const uint32_t *rank, const pb_opts *opts, int64_t *out, hipStream_t stream) {
    if (!out) return PB_ERR_INVALID_ARG;
    return count_impl(g, rank, opts, out, nullptr, nullptr, stream);
}

pb_status pb_count_vertex(pb_graph *g, const uint32_t *rank, const pb_opts *opts, int64_t *out, hipStream_t stream) {
    if (!out) return PB_ERR_INVALID_ARG;
    return count_impl(g, rank, opts, nullptr, out, nullptr, stream);
}

pb_status pb_count_edge(pb_graph *g, const uint32_t *rank, const pb_opts *opts, int64_t *out, hipStream_t stream) {
    if (!out) return PB_ERR_INVALID_ARG;
    return count_impl(g, rank, opts, nullptr, nullptr, out, stream);
}

pb_status pb_count_noalloc(pb_graph *g, const uint32_t *rank, const pb_opts *opts_in, int64_t *global_out,
                           int64_t *vertex_out, int64_t *edge_out, hipStream_t stream) {
    if (!g || !rank) return PB_ERR_INVALID_ARG;
    if (!global_out && !vertex_out && !edge_out) return PB_ERR_INVALID_ARG;
    pb_opts opts;
    Policy pol;
    PB_TRY(check_opts(opts_in, &opts, &pol));
    const int mode = (global_out ? MODE_GLOBAL : 0) | (vertex_out ? MODE_VERTEX : 0) | (edge_out ? MODE_EDGE : 0);
    const uint64_t n = (uint64_t)g->n_u + g->n_v;
    if (noalloc_need(n, g->m, (opts.flags & PB_FLAG_CACHE_OPT) != 0) > PB_NOALLOC_SCRATCH_BYTES)
        return PB_ERR_NO_MEMORY;
    int dev = 0;
    PB_TRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return PB_ERR_INVALID_ARG;
    NoallocDevice &d = noalloc_devices[dev];
    std::lock_guard<std::mutex> lk(d.mu);  // one call at a time uses this device's array
    if (!d.ptr) {
        // the array's device address on this device (the symbol's name is a
        // host-side stand-in, never a device pointer)
        void *p = nullptr;
        PB_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return PB_ERR_HIP;
        d.ptr = p;
    }
    CoreIn in{n, g->n_u, g->m, g->eu, g->u_adj, g->deg, rank, g->max_deg,
              BatchLayout{1, nullptr, nullptr, nullptr, nullptr}, g->u_off, g->u_adj, g->v_off, g->v_adj, g->v_eid};
    CoreOut out{global_out, vertex_out, edge_out, nullptr, nullptr, nullptr};
    const pb_status st = count_core(in, out, mode, opts, pol, stream, nullptr, d.ptr, PB_NOALLOC_SCRATCH_BYTES);
    // the array is free for the next call only once this call's work is done
    // (an error return may leave work queued)
    if (hipStreamSynchronize(stream) != hipSuccess && st == PB_OK) return PB_ERR_HIP;
    return st;
}

pb_status pb_count_batched(pb_graph *const *graphs, const uint32_t *const *ranks, uint32_t count, const pb_opts *opts_in,
                           int64_t *const *global_outs, int64_t *const *vertex_outs, int64_t *const *edge_outs,
                           hipStream_t stream) {
    if (!graphs || !ranks || count == 0) return PB_ERR_INVALID_ARG;
    pb_opts opts;
    Policy pol;
    PB_TRY(check_opts(opts_in, &opts, &pol));
    Workspace ws(stream, 0);
    BatchBuild bb;
    PB_TRY(build_batch(graphs, ranks, count, global_outs, vertex_outs, edge_outs, ws, stream, &bb));
    return count_core(bb.in, bb.out, bb.mode, opts, pol, stream, nullptr);
}

pb_status pb_autotune(pb_graph *const *graphs, const uint32_t *const *ranks, uint32_t count, const pb_opts *opts_in,
                      uint32_t repeats, pb_tuning *out, hipStream_t stream) {
    if (!out || !graphs || !ranks || count == 0) return PB_ERR_INVALID_ARG;
    pb_opts opts;
    Policy pol;
    PB_TRY(check_opts(opts_in, &opts, &pol));
    opts.agg = PB_AGG_AUTO;
    opts.stats = nullptr;
    if (repeats == 0) repeats = 1;
    // scratch outputs for the timed counts: global and per-edge of every graph
    Workspace ws(stream, 0);
    uint64_t mtot = 0;
    for (uint32_t j = 0; j < count; ++j) {
        if (!graphs || !graphs[j]) return PB_ERR_INVALID_ARG;
        mtot += graphs[j]->m;
    }
    int64_t *gbuf = ws.alloc<int64_t>(count), *ebuf = ws.alloc<int64_t>(mtot ? mtot : 1);
    if (ws.failed) return PB_ERR_NO_MEMORY;
    std::vector<int64_t *> gp(count), ep(count);
    uint64_t off = 0;
    for (uint32_t j = 0; j < count; ++j) {
        gp[j] = gbuf + j;
        ep[j] = ebuf + off;
        off += graphs[j]->m;
    }
    BatchBuild bb;
    PB_TRY(build_batch(graphs, ranks, count, gp.data(), nullptr, ep.data(), ws, stream, &bb));

    Policy best = Policy{LIGHT_D, MEDIUM_D, {PB_AGG_LDS_HASH, PB_AGG_LDS_HASH, PB_AGG_DENSE_HIST}, true};
    auto time_policy = [&](const Policy &p, float *ms) -> pb_status {
        std::vector<float> runs;
        for (uint32_t rep = 0; rep < repeats; ++rep) {
            float lm[NLISTS];
            PB_TRY(count_core(bb.in, bb.out, bb.mode, opts, p, stream, lm));
            float tot = 0;
            for (float x : lm) tot += x;
            runs.push_back(tot);
        }
        std::sort(runs.begin(), runs.end());
        *ms = runs[runs.size() / 2];
        return PB_OK;
    };
    float best_ms;
    PB_TRY(time_policy(best, &best_ms));
    // one bucket at a time: its aggregator, then its threshold
    const int choices[3][3] = {{PB_AGG_LDS_HASH, PB_AGG_RADIX_SORT, PB_AGG_DENSE_HIST},
                               {PB_AGG_LDS_HASH, PB_AGG_RADIX_SORT, PB_AGG_DENSE_HIST},
                               {PB_AGG_DENSE_HIST, PB_AGG_LDS_HASH, PB_AGG_RADIX_SORT}};
    for (int bkt = 0; bkt < 3; ++bkt)
        for (int c : choices[bkt]) {
            if (c == best.agg[bkt]) continue;
            Policy p = best;
            p.agg[bkt] = c;
            float ms;
            PB_TRY(time_policy(p, &ms));
            if (ms < best_ms) { best = p; best_ms = ms; }
        }
    const uint32_t light_opts[] = {64, 128, 256, 512};
    for (uint32_t lm : light_opts) {
        if (lm == best.light_max) continue;
        Policy p = best;
        p.light_max = lm;
        float ms;
        PB_TRY(time_policy(p, &ms));
        if (ms < best_ms) { best = p; best_ms = ms; }
    }
    const uint32_t medium_opts[] = {1024, 2048, 4096};
    for (uint32_t mm : medium_opts) {
        if (mm == best.medium_max || mm < best.light_max) continue;
        Policy p = best;
        p.medium_max = mm;
        float ms;
        PB_TRY(time_policy(p, &ms));
        if (ms < best_ms) { best = p; best_ms = ms; }
    }
    // workgroup sizes of the light and medium buckets' kernels
    const uint32_t wg_opts[2][3] = {{64, 128, 256}, {128, 256, 512}};
    for (int bkt = 0; bkt < 2; ++bkt)
        for (uint32_t t : wg_opts[bkt]) {
            if (t == best.wg[bkt]) continue;
            Policy p = best;
            p.wg[bkt] = t;
            float ms;
            PB_TRY(time_policy(p, &ms));
            if (ms < best_ms) { best = p; best_ms = ms; }
        }
    // batch width of each bucket's launches
    const uint32_t width_opts[] = {0, 256, 1024, 4096};
    for (int bkt = 0; bkt < 3; ++bkt)
        for (uint32_t wdt : width_opts) {
            if (wdt == best.width[bkt]) continue;
            Policy p = best;
            p.width[bkt] = wdt;
            float ms;
            PB_TRY(time_policy(p, &ms));
            if (ms < best_ms) { best = p; best_ms = ms; }
        }
    *out = pb_tuning{best.light_max, best.medium_max, (pb_agg)best.agg[0], (pb_agg)best.agg[1], (pb_agg)best.agg[2],
                     best.wg[0],      best.wg[1],      best.width[0],      best.width[1],      best.width[2]};
    return PB_OK;
}

}  // extern "C"
