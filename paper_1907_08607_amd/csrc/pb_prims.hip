// Device-wide primitives: exclusive scan, stable LSD radix sort, fill.
// (The paper's prefix sum and integer sort, Section 2 "Parallel primitives".)
#include "pb_internal.h"

#include <map>
#include <mutex>
#include <unordered_map>

namespace pb {

// ---------------------------------------------------------------- scan

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

template <class Tin, class Tout>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const Tin *in, uint64_t n,
                                                              Tout *partial) {
    __shared__ Tout s_tmp[SCAN_THREADS / WAVE + 1];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    Tout s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        uint64_t idx = base + (uint64_t)i * SCAN_THREADS + threadIdx.x;
        if (idx < n) s += (Tout)in[idx];
    }
    s = block_sum<SCAN_THREADS>(s, s_tmp);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Each thread owns SCAN_ITEMS consecutive elements.
template <class Tin, class Tout>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_down(const Tin *in, Tout *out, uint64_t n,
                                                            const Tout *partial, Tout *total) {
    __shared__ Tout s_tmp[SCAN_THREADS / WAVE + 1];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    Tout v[SCAN_ITEMS];
    Tout s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        uint64_t idx = base + i;
        v[i] = idx < n ? (Tout)in[idx] : Tout(0);
        s += v[i];
    }
    Tout blk_total;
    Tout pre = block_exclusive_sum<SCAN_THREADS>(s, s_tmp, &blk_total);
    Tout off = (partial ? partial[blockIdx.x] : Tout(0)) + pre;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        uint64_t idx = base + i;
        if (idx < n) out[idx] = off;
        off += v[i];
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
        *total = (partial ? partial[blockIdx.x] : Tout(0)) + blk_total;
}

template <class Tin, class Tout>
pb_status scan_exclusive(const Tin *in, Tout *out, uint64_t n, Tout *total, Workspace &ws) {
    if (n == 0) {
        if (total) return fill<Tout>(total, Tout(0), 1, ws.stream);
        return PB_OK;
    }
    const uint64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    Tout *partial = nullptr;
    if (nb > 1) {
        partial = ws.alloc<Tout>(nb);
        if (!partial) return PB_ERR_NO_MEMORY;
        hipLaunchKernelGGL((k_scan_reduce<Tin, Tout>), dim3((uint32_t)nb), dim3(SCAN_THREADS), 0,
                           ws.stream, in, n, partial);
        PB_TRY_HIP(hipGetLastError());
        PB_TRY((scan_exclusive<Tout, Tout>(partial, partial, nb, nullptr, ws)));
    }
    hipLaunchKernelGGL((k_scan_down<Tin, Tout>), dim3((uint32_t)nb), dim3(SCAN_THREADS), 0, ws.stream,
                       in, out, n, partial, total);
    PB_TRY_HIP(hipGetLastError());
    if (partial) ws.release(partial);
    return PB_OK;
}

template pb_status scan_exclusive<uint32_t, uint32_t>(const uint32_t *, uint32_t *, uint64_t,
                                                      uint32_t *, Workspace &);
template pb_status scan_exclusive<uint32_t, uint64_t>(const uint32_t *, uint64_t *, uint64_t,
                                                      uint64_t *, Workspace &);
template pb_status scan_exclusive<uint64_t, uint64_t>(const uint64_t *, uint64_t *, uint64_t,
                                                      uint64_t *, Workspace &);

// ---------------------------------------------------------------- fill

template <class T>
__global__ void k_fill(T *p, T value, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

template <class T>
pb_status fill(T *p, T value, uint64_t n, hipStream_t s) {
    if (n == 0) return PB_OK;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL((k_fill<T>), dim3((uint32_t)blocks), dim3(256), 0, s, p, value, n);
    PB_TRY_HIP(hipGetLastError());
    return PB_OK;
}

template pb_status fill<uint32_t>(uint32_t *, uint32_t, uint64_t, hipStream_t);
template pb_status fill<uint64_t>(uint64_t *, uint64_t, uint64_t, hipStream_t);
template pb_status fill<int64_t>(int64_t *, int64_t, uint64_t, hipStream_t);

// ---------------------------------------------------------------- radix sort

constexpr int RS_THREADS = 256;  // histogram kernel: one thread per digit
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;
constexpr int RSS_THREADS = 1024;  // scatter kernel
constexpr int RSS_ITEMS = RS_TILE / RSS_THREADS;
constexpr int RSS_WAVES = RSS_THREADS / WAVE;

// Lanes of this wave whose (valid) digit equals this lane's digit.
template <int BITS>
__device__ inline uint64_t match_digit(uint32_t d, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const bool bit = (d >> b) & 1;
        const uint64_t bal = __ballot(valid && bit);
        m &= bit ? bal : ~bal;
    }
    return m;
}

// Digits of BITS bits (8, or 9 where that saves a pass): 2^BITS buckets.
template <int BITS>
__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint64_t *keys, uint64_t n, int shift,
                                                        uint32_t *hist, uint32_t nb) {
    constexpr uint32_t DIG = 1u << BITS;
    __shared__ uint32_t cnt[DIG];
    for (uint32_t d = threadIdx.x; d < DIG; d += RS_THREADS) cnt[d] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
    for (int it = 0; it < RS_ITEMS; ++it) {
        const uint64_t idx = base + (uint64_t)it * RS_THREADS + threadIdx.x;
        const bool valid = idx < n;
        const uint32_t d = valid ? (uint32_t)(keys[idx] >> shift) & (DIG - 1) : 0u;
        const uint64_t m = match_digit<BITS>(d, valid);
        if (valid && (m & lanemask_lt()) == 0) atomicAdd(&cnt[d], (uint32_t)__popcll(m));
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < DIG; d += RS_THREADS) hist[(uint64_t)d * nb + blockIdx.x] = cnt[d];
}

// Stable scatter of one tile of RS_TILE keys.  `hist` holds the exclusive
// scan over (digit, tile) of the per-tile digit counts, with the total at
// hist[2^BITS * nb], so this tile's count of digit d is the difference of two
// neighbouring entries.  The tile is first ordered by digit in LDS (each key at
// its digit's tile-local start plus the number of equal digits before it in
// the tile), then written out run by run, so consecutive lanes store to
// consecutive addresses of one bucket.  Per-wave digit counts and offsets are
// below RS_TILE, so they are kept in 16 bits.
template <int BITS>
__global__ __launch_bounds__(RSS_THREADS) void k_rs_scatter(const uint64_t *kin, const uint32_t *vin,
                                                            uint64_t n, int shift,
                                                            const uint32_t *hist, uint32_t nb,
                                                            uint64_t *kout, uint32_t *vout) {
    constexpr uint32_t DIG = 1u << BITS;
    static_assert(DIG <= RSS_THREADS && RS_TILE < 65536, "one thread per digit; 16-bit offsets");
    __shared__ uint64_t s_key[RS_TILE];
    __shared__ uint32_t s_val[RS_TILE];
    __shared__ uint32_t s_gbase[DIG];  // global start of this tile's part of bucket d
    __shared__ uint32_t s_lbase[DIG];  // tile-local start of digit d
    __shared__ uint32_t s_run[DIG];    // next tile-local slot of digit d
    __shared__ uint16_t s_w[RSS_WAVES][DIG];
    __shared__ uint32_t s_tmp[RSS_WAVES + 1];
    const int tid = threadIdx.x;
    const int w = tid / WAVE;
    const bool dig = tid < (int)DIG;  // the first DIG threads own one digit each
    uint32_t g0 = 0, cnt = 0;
    if (dig) {
        const uint64_t hb = (uint64_t)tid * nb + blockIdx.x;
        g0 = hist[hb];
        cnt = hist[hb + 1] - g0;
    }
    uint32_t tile_n;
    const uint32_t l0 = block_exclusive_sum<RSS_THREADS>(cnt, s_tmp, &tile_n);
    if (dig) {
        s_gbase[tid] = g0;
        s_lbase[tid] = l0;
        s_run[tid] = l0;
    }
    const uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
    for (int it = 0; it < RSS_ITEMS; ++it) {
        const uint64_t idx = base + (uint64_t)it * RSS_THREADS + tid;
        const bool valid = idx < n;
        const uint64_t k = valid ? kin[idx] : 0;
        const uint32_t v = valid ? vin[idx] : 0;
        const uint32_t d = (uint32_t)(k >> shift) & (DIG - 1);
        if (dig) {
#pragma unroll
            for (int q = 0; q < RSS_WAVES; ++q) s_w[q][tid] = 0;
        }
        __syncthreads();
        const uint64_t m = match_digit<BITS>(d, valid);
        const uint32_t rank_in_wave = (uint32_t)__popcll(m & lanemask_lt());
        if (valid && rank_in_wave == 0) s_w[w][d] = (uint16_t)__popcll(m);
        __syncthreads();
        if (dig) {
            uint32_t run = s_run[tid];
#pragma unroll
            for (int q = 0; q < RSS_WAVES; ++q) {
                const uint32_t c = s_w[q][tid];
                s_w[q][tid] = (uint16_t)run;
                run += c;
            }
            s_run[tid] = run;
        }
        __syncthreads();
        if (valid) {
            const uint32_t lp = s_w[w][d] + rank_in_wave;
            s_key[lp] = k;
            s_val[lp] = v;
        }
        __syncthreads();  // s_w is cleared again by the next round
    }
    for (uint32_t i = tid; i < tile_n; i += RSS_THREADS) {
        const uint64_t k = s_key[i];
        const uint32_t d = (uint32_t)(k >> shift) & (DIG - 1);
        const uint32_t dst = s_gbase[d] + (i - s_lbase[d]);
        kout[dst] = k;
        vout[dst] = s_val[i];
    }
}

// ---------------------------------------------------------------- scratch cache

namespace {

struct Block {
    uint64_t bytes;
    int dev;
    hipEvent_t ev;  // recorded on the stream that handed the block back
};

struct Cache {
    std::mutex mu;
    std::multimap<uint64_t, std::pair<void *, Block>> idle;  // by size
    std::unordered_map<void *, Block> busy;
};

Cache &cache() {
    static Cache *c = new Cache;  // lives to the end of the process
    return *c;
}

// Size classes: powers of two up to 1 MiB, then multiples of 2 MiB.
uint64_t size_class(uint64_t b) {
    if (b <= (uint64_t(1) << 20)) {
        uint64_t r = 256;
        while (r < b) r <<= 1;
        return r;
    }
    const uint64_t g = uint64_t(2) << 20;
    return (b + g - 1) / g * g;
}

}  // namespace

void *scratch_get(hipStream_t s, uint64_t bytes) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    const uint64_t want = size_class(bytes);
    Cache &c = cache();
    {
        std::lock_guard<std::mutex> lk(c.mu);
        // the smallest idle block of this device that is not wastefully large
        for (auto it = c.idle.lower_bound(want); it != c.idle.end() && it->first <= 2 * want; ++it) {
            if (it->second.second.dev != dev) continue;
            void *p = it->second.first;
            const Block b = it->second.second;
            c.idle.erase(it);
            if (hipStreamWaitEvent(s, b.ev, 0) != hipSuccess) {
                (void)hipGetLastError();
                (void)hipEventSynchronize(b.ev);
            }
            c.busy[p] = b;
            return p;
        }
    }
    void *p = nullptr;
    if (hipMallocAsync(&p, want, s) != hipSuccess || !p) {
        (void)hipGetLastError();
        // out of memory: give this device's idle blocks back, then retry once
        std::vector<std::pair<void *, Block>> drop;
        {
            std::lock_guard<std::mutex> lk(c.mu);
            for (auto it = c.idle.begin(); it != c.idle.end();) {
                if (it->second.second.dev == dev) {
                    drop.push_back(it->second);
                    it = c.idle.erase(it);
                } else {
                    ++it;
                }
            }
        }
        for (auto &d : drop) {
            (void)hipStreamWaitEvent(s, d.second.ev, 0);
            (void)hipFreeAsync(d.first, s);
            (void)hipEventDestroy(d.second.ev);
        }
        p = nullptr;
        if (hipMallocAsync(&p, want, s) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFreeAsync(p, s);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(c.mu);
    c.busy[p] = Block{want, dev, ev};
    return p;
}

void scratch_put(hipStream_t s, void *p) {
    if (!p) return;
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.busy.find(p);
    if (it == c.busy.end()) return;
    const Block b = it->second;
    c.busy.erase(it);
    if (hipEventRecord(b.ev, s) != hipSuccess) (void)hipGetLastError();
    c.idle.emplace(b.bytes, std::make_pair(p, b));
}

pb_status radix_sort_pairs(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, uint64_t n,
                           int nbits, Workspace &ws, uint64_t **kres, uint32_t **vres) {
    return radix_sort_pairs_bits(k0, v0, k1, v1, n, 0, nbits, ws, kres, vres);
}

pb_status radix_sort_pairs_bits(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, uint64_t n, int lo_bit,
                                int hi_bit, Workspace &ws, uint64_t **kres, uint32_t **vres) {
    *kres = k0;
    *vres = v0;
    if (n <= 1 || hi_bit <= lo_bit) return PB_OK;
    if (n >= (uint64_t(1) << 32)) return PB_ERR_INVALID_ARG;
    // 9-bit digits where they take one pass fewer than 8-bit ones (a 25-bit
    // key in 3 passes instead of 4, a 17-bit one in 2 instead of 3)
    const int bits = hi_bit - lo_bit;
    const int dbits = (bits + 8) / 9 < (bits + 7) / 8 ? 9 : 8;
    const uint32_t nb = ceil_div(n, RS_TILE);
    const uint64_t nh = (uint64_t)nb << dbits;
    uint32_t *hist = ws.alloc<uint32_t>(nh + 1);
    if (!hist) return PB_ERR_NO_MEMORY;
    uint64_t *ks = k0, *kd = k1;
    uint32_t *vs = v0, *vd = v1;
    for (int shift = lo_bit; shift < hi_bit; shift += dbits) {
        if (dbits == 9)
            hipLaunchKernelGGL(k_rs_hist<9>, dim3(nb), dim3(RS_THREADS), 0, ws.stream, ks, n, shift, hist, nb);
        else
            hipLaunchKernelGGL(k_rs_hist<8>, dim3(nb), dim3(RS_THREADS), 0, ws.stream, ks, n, shift, hist, nb);
        PB_TRY_HIP(hipGetLastError());
        PB_TRY((scan_exclusive<uint32_t, uint32_t>(hist, hist, nh, hist + nh, ws)));
        if (dbits == 9)
            hipLaunchKernelGGL(k_rs_scatter<9>, dim3(nb), dim3(RSS_THREADS), 0, ws.stream, ks, vs, n, shift, hist,
                               nb, kd, vd);
        else
            hipLaunchKernelGGL(k_rs_scatter<8>, dim3(nb), dim3(RSS_THREADS), 0, ws.stream, ks, vs, n, shift, hist,
                               nb, kd, vd);
        PB_TRY_HIP(hipGetLastError());
        uint64_t *tk = ks; ks = kd; kd = tk;
        uint32_t *tv = vs; vs = vd; vd = tv;
    }
    ws.release(hist);
    *kres = ks;
    *vres = vs;
    return PB_OK;
}

}  // namespace pb
