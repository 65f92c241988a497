// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/parbutterfly.h"

namespace pb {

constexpr int WAVE = 64;

#define PB_TRY_HIP(expr)                                  \
    do {                                                  \
        hipError_t pb_e_ = (expr);                        \
        if (pb_e_ != hipSuccess) return PB_ERR_HIP;       \
    } while (0)

#define PB_TRY(expr)                                      \
    do {                                                  \
        pb_status pb_s_ = (expr);                         \
        if (pb_s_ != PB_OK) return pb_s_;                 \
    } while (0)

// Device scratch cache.  Blocks handed back by a Workspace stay with the
// library for the life of the process and are reused by later calls on any
// stream: each cached block carries an event recorded on the stream that
// released it, and a stream that takes the block waits for that event first
// (stream-ordered, no host wait).  A new block is allocated only when no
// cached block of the current device fits.  Thread safe.
void *scratch_get(hipStream_t s, uint64_t bytes);
void scratch_put(hipStream_t s, void *p);

// Stream-ordered scratch for one library call.  Every allocation goes back to
// the cache when the Workspace goes out of scope.  `cap` bounds the total
// bytes (0 = unbounded).
//
// With a fixed region instead (`region`, `region_bytes`: device memory the
// caller owns), blocks are carved from it as a stack and nothing is ever
// allocated: a block is placed after the highest live one, so releasing the
// top block (and any freed blocks below it) makes room again.  A request the
// region cannot hold fails like an exhausted cap.
struct Workspace {
    hipStream_t stream;
    uint64_t cap;
    uint64_t used = 0;
    uint64_t peak = 0;
    bool failed = false;
    std::vector<std::pair<void *, uint64_t>> ptrs;
    char *region = nullptr;
    uint64_t region_bytes = 0;

    Workspace(hipStream_t s, uint64_t cap_bytes) : stream(s), cap(cap_bytes) {}
    Workspace(hipStream_t s, void *fixed, uint64_t fixed_bytes)
        : stream(s), cap(0), region(static_cast<char *>(fixed)), region_bytes(fixed_bytes) {}
    Workspace(const Workspace &) = delete;
    Workspace &operator=(const Workspace &) = delete;
    ~Workspace() { release_all(); }

    // End offset of the highest live block of the fixed region.
    uint64_t region_top() const {
        uint64_t top = 0;
        for (auto &p : ptrs) {
            const uint64_t end = (uint64_t)(static_cast<char *>(p.first) - region) + p.second;
            if (end > top) top = end;
        }
        return top;
    }

    void *alloc_bytes(uint64_t bytes) {
        if (bytes == 0) bytes = 256;
        bytes = (bytes + 255) & ~uint64_t(255);
        if (cap && used + bytes > cap) { failed = true; return nullptr; }
        void *p;
        if (region) {
            const uint64_t top = region_top();
            if (bytes > region_bytes - top) {
                failed = true;
                return nullptr;
            }
            p = region + top;
        } else {
            p = scratch_get(stream, bytes);
        }
        if (!p) {
            failed = true;
            return nullptr;
        }
        ptrs.push_back({p, bytes});
        used += bytes;
        if (used > peak) peak = used;
        return p;
    }
    template <class T>
    T *alloc(uint64_t count) { return static_cast<T *>(alloc_bytes(count * sizeof(T))); }

    // Hands one allocation back early (stream-ordered).
    void release(void *p) {
        for (size_t i = 0; i < ptrs.size(); ++i)
            if (ptrs[i].first == p) {
                if (!region) scratch_put(stream, p);
                used -= ptrs[i].second;
                ptrs.erase(ptrs.begin() + i);
                return;
            }
    }
    void release_all() {
        if (!region)
            for (auto &p : ptrs) scratch_put(stream, p.first);
        ptrs.clear();
        used = 0;
    }
};

// ---------------------------------------------------------------- primitives

// out[i] = sum_{j < i} in[j] for i < n; if total != nullptr, *total (device) =
// sum of all n.  `out` may alias `in`.
template <class Tin, class Tout>
pb_status scan_exclusive(const Tin *in, Tout *out, uint64_t n, Tout *total, Workspace &ws);

// Stable LSD radix sort of (keys, vals) by key bits [0, nbits), 8 bits a pass.
// Ping-pongs between (k0, v0) and (k1, v1); on return *kres / *vres point at
// whichever pair holds the sorted result.  n < 2^32.
pb_status radix_sort_pairs(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, uint64_t n,
                           int nbits, Workspace &ws, uint64_t **kres, uint32_t **vres);
// The same over key bits [lo_bit, hi_bit) only (a stable sort, so pairs
// equal in those bits keep their input order).
pb_status radix_sort_pairs_bits(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, uint64_t n, int lo_bit,
                                int hi_bit, Workspace &ws, uint64_t **kres, uint32_t **vres);

template <class T>
pb_status fill(T *p, T value, uint64_t n, hipStream_t s);

// Number of bits needed to represent values 0..x.
inline int bits_for(uint64_t x) {
    int b = 0;
    while (b < 64 && (x >> b) != 0) ++b;
    return b;
}

inline uint32_t ceil_div(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// ---------------------------------------------------------------- device helpers

__device__ inline uint64_t lanemask_lt() { return __lanemask_lt(); }

template <class T>
__device__ inline T wave_inclusive_sum(T v) {
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        T t = __shfl_up(v, d, WAVE);
        if (lane >= d) v += t;
    }
    return v;
}

// 32-bit lanes: the same scan in registers with DPP row shifts and row
// broadcasts (wave64 on gfx9), no LDS round trips.  Every lane of the wave
// must be active.
template <>
__device__ inline uint32_t wave_inclusive_sum<uint32_t>(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15 -> rows 1, 3
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31 -> rows 2, 3
    return v;
}

template <class T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int d = WAVE / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, WAVE);
    return v;
}

// Block-wide exclusive sum.  `s_tmp` needs THREADS / WAVE + 1 entries of
// shared memory.  Returns the thread's exclusive prefix; *total gets the block
// sum in every thread.  Contains __syncthreads(); call from all threads.
template <int THREADS, class T>
__device__ inline T block_exclusive_sum(T v, T *s_tmp, T *total) {
    constexpr int NW = THREADS / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    T inc = wave_inclusive_sum(v);
    if (lane == WAVE - 1) s_tmp[w] = inc;
    __syncthreads();
    if (w == 0) {
        T x = lane < NW ? s_tmp[lane] : T(0);
        T xi = wave_inclusive_sum(x);
        if (lane < NW) s_tmp[lane] = xi - x;
        if (lane == NW - 1) s_tmp[NW] = xi;
    }
    __syncthreads();
    T r = s_tmp[w] + inc - v;
    *total = s_tmp[NW];
    __syncthreads();
    return r;
}

template <int THREADS, class T>
__device__ inline T block_sum(T v, T *s_tmp) {
    constexpr int NW = THREADS / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    T s = wave_sum(v);
    if (lane == 0) s_tmp[w] = s;
    __syncthreads();
    T r = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) r += s_tmp[i];
    __syncthreads();
    return r;
}


// Calls f(row, item) for the items [i0, i1) of a scanned item count (coff
// over n rows: row d owns items coff[d] .. coff[d + 1] - 1, coff[n] in all),
// in order.  The first item's row comes from a binary search; leaving a row,
// the next is found by galloping forward from it (rows without items can lie
// between, millions of them in a skewed graph), so a caller that takes a
// contiguous share of the items searches once per row instead of once per
// item, and never walks rows one by one.
template <class F>
__device__ inline void rows_of_items(const uint32_t *coff, uint64_t n, uint32_t i0, uint32_t i1, F f) {
    if (i0 >= i1) return;
    uint64_t d = 0;
    for (uint32_t it = i0; it < i1; ++it) {
        if (it == i0 || coff[d + 1] <= it) {
            // the last row r with coff[r] <= it (rows after the one holding it start above it)
            uint64_t lo = it == i0 ? 0 : d + 1, hi;
            if (it == i0) {
                hi = n;
            } else {
                uint64_t step = 1;
                hi = lo + 1;
                while (hi < n && coff[hi] <= it) {
                    lo = hi;
                    step <<= 1;
                    hi = lo + step;
                }
                if (hi > n) hi = n;
            }
            while (hi - lo > 1) {  // coff[lo] <= it < coff[hi] (coff[n] = all items > it)
                const uint64_t mid = (lo + hi) >> 1;
                if (coff[mid] <= it) lo = mid; else hi = mid;
            }
            d = lo;
        }
        f((uint32_t)d, it);
    }
}

// The share [*i0, *i1) of `items` that part `part` of `parts` takes.
__device__ inline void item_share(uint32_t items, uint32_t part, uint32_t parts, uint32_t *i0, uint32_t *i1) {
    const uint32_t q = (uint32_t)(((uint64_t)items + parts - 1) / parts);
    const uint64_t a = (uint64_t)part * q, b = a + q;
    *i0 = a < items ? (uint32_t)a : items;
    *i1 = b < items ? (uint32_t)b : items;
}

// ---------------------------------------------------------------- hub tile

// Dense hub-to-hub pairs on int8 matrix cores.  The hubs are the first HUB_T
// (or fewer) vertices in rank order of one side; their side-major ids form
// [base, end).  For hub pairs h1 < h2 (rank order) and centres y on the other
// side, A[h][y] = 1 when y is a neighbour of h and A'[h][y] additionally needs
// rank y > rank h.  D = A' A^T then holds R(h1, h2) = |{y in N(h1) & N(h2) :
// rank y > rank h1}| above the diagonal (Section 3.1.2's wedge counts of the
// pair), as an exact int32 sum of 0/1 products.
constexpr uint32_t HUB_T = 256;

struct HubCounters {
    uint32_t on;                // tile in use (set on device; AUTO may decline)
    uint32_t cols;              // compacted centre columns
    unsigned long long paths;   // sum over kept columns of C(k, 2), k = hub neighbours
    unsigned long long wedges;  // wedges of hub pairs: sum of R over h1 < h2
};

struct HubIn {
    uint64_t n;
    uint32_t n_u;
    const uint32_t *smid, *roff, *upoff, *nbr;  // ranked CSR (rank-indexed)
    uint32_t base, end;                         // hub side-major ids
    bool force;                                 // skip the cost model
    bool two_pass;                              // per-vertex or per-edge counts: the hub pairs need a credit pass
    unsigned long long *g;                      // global accumulator (one graph)
    unsigned long long *v;                      // per-vertex accumulator by smid, or null
};

struct HubOut {
    uint32_t *hub_rank;         // HUB_T: rank of hub i
    uint32_t *D;                // HUB_T * HUB_T: R(hub i, hub j) for i < j, else 0
    unsigned long long *roww;   // HUB_T: wedges of hub i as the lower endpoint
};

// Builds the tile and credits C(R,2) per hub pair to the global count and both
// endpoints.  Without in.force the AUTO cost model decides from a sample of
// the columns; the decision goes to `host_on` (pinned host memory) and a
// declined tile returns at once (hc->on = 0).  `ev0`/`ev1`, if not null, are
// recorded around the matrix-core kernel; *gemm_grid is 0 when it did not run.
pb_status hub_tile(const HubIn &in, HubCounters *hc, const HubOut &out, Workspace &ws, hipStream_t s,
                   hipEvent_t ev0, hipEvent_t ev1, uint32_t *gemm_grid, uint32_t *host_on);

// int8 operations the matrix-core kernel issues for `cols` compacted columns.
uint64_t hub_gemm_ops(uint32_t cols);

}  // namespace pb

// ---------------------------------------------------------------- the graph handle

struct pb_graph {
    uint32_t n_u = 0, n_v = 0;
    uint64_t m = 0;
    int device = 0;
    const int64_t *u_off = nullptr;  // caller-owned
    const uint32_t *u_adj = nullptr; // caller-owned
    uint32_t *eu = nullptr;          // m: U endpoint of each edge
    uint32_t *v_off = nullptr;       // n_v + 1: V-side row offsets
    uint32_t *v_adj = nullptr;       // m: U ids, increasing within a row
    uint32_t *v_eid = nullptr;       // m: edge id (position in u_adj) of each V-side entry
    uint32_t *deg = nullptr;         // n: degree per unified id
    uint32_t max_deg = 0;
    hipStream_t last_stream = nullptr;
};
