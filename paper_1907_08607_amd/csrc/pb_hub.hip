// Hub-to-hub tile: the pair counts R of the highest-priority vertices of one
// side as a dense 0/1 product D = A' A^T on int8 matrix cores (gfx950
// v_mfma_i32_32x32x32_i8, int32 accumulation), instead of one hash or counter
// update per wedge.  The products are 0/1, so every sum is an exact integer no
// larger than the number of centres.
//
// Pipeline (on the device; AUTO reads its decision back once, and a declined
// tile launches nothing more):
//   k_hub_rank    rank of each hub
//   k_hub_mark    keep the centres with >= 2 hub neighbours, at least one of
//                 them ranked below the centre; sum C(k,2) over kept centres
//                 (AUTO first runs it on a 1/16 sample to decide)
//   k_hub_decide  cost model (or forced on)
//   k_hub_fill    compacted column table: slot range of the hub neighbours
//                 (the tail of N(y), since hubs have the smallest side-major
//                 ids) and where A' starts inside it
//   k_hub_gemm    split-K over column chunks: each workgroup scatters 128
//                 columns into two LDS byte tiles and accumulates the upper
//                 64x64 blocks of D in registers (loading the next chunks'
//                 columns meanwhile), then writes its partial D
//   k_hub_reduce  sums the partials; per pair: C(R,2) into the total and both
//                 endpoints (Section 3.1.3); per hub: its wedges as the lower
//                 endpoint (the plan subtracts them)
#include "pb_internal.h"

#include <algorithm>

using namespace pb;

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr uint32_t KC = 128;               // centre columns per LDS tile
constexpr uint32_t ROWB = KC + 16;         // bytes per tile row; the pad spreads 16-byte reads over all banks
constexpr uint32_t GEMM_THREADS = 1024;    // 16 waves: one 64x64 block of D each (upper ones compute)
constexpr uint32_t GEMM_MAX_GRID = 256;    // one workgroup per compute unit

// AUTO cost model, nanoseconds, fitted to on/off runs of the tile on both
// single-graph workloads (all three outputs):
//   sparse path, per hub-pair path (a wedge the tile would take over), both
//   passes: NS_SPARSE in LDS windows, NS_SPARSE_GIANT when a hub source has
//   at least GIANT_UPS up-slots (its wedges go to the global histogram, where
//   a source's highest-ranked candidates, the hubs among them, are counted
//   in LDS: the 9.7e7 hub paths of the 100M-edge hub graph cost the walk
//   nothing measurable); one pass (total only) costs half;
//   tile: NS_FIXED + NS_FIXED_VERTEX per vertex (column marking and
//   compaction) + NS_PER_COL per compacted column (the matrix-core product),
//   plus NS_HUB_PASS per path for the hub pairs' credit pass when per-vertex
//   or per-edge counts are wanted and no hub source is giant (a giant hub's
//   credits ride in the histogram walk's pass 2).
constexpr double NS_SPARSE = 0.0075;
constexpr double NS_SPARSE_GIANT = 0.005;
constexpr double NS_FIXED = 100000.0;
constexpr double NS_FIXED_VERTEX = 0.035;
constexpr double NS_PER_COL = 0.1;
constexpr double NS_HUB_PASS = 0.04;
constexpr uint32_t GIANT_UPS = 65536;  // the planner's global-histogram threshold
constexpr uint32_t HUB_SAMPLE = 16;     // AUTO estimates paths and columns from every 16th vertex

#define HUB_GRID_STRIDE(i, n)                                                       \
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
         i += (uint64_t)gridDim.x * blockDim.x)

inline uint32_t grid_for(uint64_t n, uint32_t block = 256, uint32_t cap = 65536) {
    uint64_t g = (n + block - 1) / block;
    if (g == 0) g = 1;
    return (uint32_t)(g > cap ? cap : g);
}

// Smallest i in [lo, len] with p[i] < v (p strictly decreasing).
__device__ inline uint32_t tail_start(const uint32_t *p, uint32_t lo, uint32_t len, uint32_t v) {
    uint32_t hi = len;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (p[mid] < v) hi = mid; else lo = mid + 1;
    }
    return lo;
}

__device__ inline bool other_side(const HubIn &in, uint32_t s) { return (s >= in.n_u) != (in.base >= in.n_u); }

__global__ void k_hub_rank(const uint32_t *smid, uint64_t n, uint32_t base, uint32_t end, uint32_t *hub_rank) {
    HUB_GRID_STRIDE(r, n) {
        const uint32_t s = smid[r];
        if (s >= base && s < end) hub_rank[s - base] = (uint32_t)r;
    }
}

// Marks the kept centre columns (keep[r]) and adds their hub-pair paths and
// their number to hc.  With stride > 1 (keep null) it visits one vertex in
// `stride`, as runs of 64 consecutive ranks every 64 * stride (whole cache
// lines of the rank-indexed tables): a sample for the AUTO estimate.
__global__ void k_hub_mark(HubIn in, uint32_t *keep, HubCounters *hc, uint32_t stride) {
    unsigned long long paths = 0;
    uint32_t cols = 0;
    const uint64_t runs = (in.n + 64ull * stride - 1) / (64ull * stride);
    HUB_GRID_STRIDE(i, stride == 1 ? in.n : runs * 64) {
        const uint64_t r = stride == 1 ? i : (i >> 6) * 64 * stride + (i & 63);
        if (r >= in.n) continue;
        uint32_t flag = 0;
        if (other_side(in, in.smid[r])) {
            const uint32_t o = in.roff[r], deg = in.roff[r + 1] - o;
            const uint32_t hi = in.upoff[r + 1] - in.upoff[r];  // neighbours ranked above y
            const uint32_t k = deg - tail_start(in.nbr + o, 0, deg, in.end);
            if (k >= 2 && hi < deg) {
                flag = 1;
                paths += (unsigned long long)k * (k - 1) / 2;
            }
        }
        if (keep) keep[r] = flag;
        cols += flag;
    }
    // one atomic per wave for the whole kernel
    paths = wave_sum(paths);
    cols = wave_sum(cols);
    if ((threadIdx.x & (WAVE - 1)) == 0 && paths) atomicAdd(&hc->paths, paths);
    if ((threadIdx.x & (WAVE - 1)) == 0 && cols) atomicAdd(&hc->cols, cols);
}

// Clears the sample's sums before the exact marking.
__global__ void k_hub_reset(HubCounters *hc) {
    hc->paths = 0;
    hc->cols = 0;
}

// The AUTO decision from k_hub_mark's sums over every stride-th vertex.
__global__ void k_hub_decide(const uint32_t *hub_rank, HubIn in, HubCounters *hc, uint32_t stride) {
    const double c = (double)hc->cols * stride;
    bool giant = false;
    for (uint32_t i = 0; i < in.end - in.base; ++i) {
        const uint32_t r = hub_rank[i];
        giant = giant || in.upoff[r + 1] - in.upoff[r] >= GIANT_UPS;
    }
    const double paths = (double)hc->paths * stride;
    const double dense = NS_FIXED + NS_FIXED_VERTEX * (double)in.n + NS_PER_COL * c +
                         (in.two_pass && !giant ? NS_HUB_PASS * paths : 0.0);
    const double sparse = (giant ? NS_SPARSE_GIANT : NS_SPARSE) * paths * (in.two_pass ? 1.0 : 0.5);
    hc->on = (in.force || sparse > dense) ? 1u : 0u;
    if (!hc->on) {  // a declined tile reports no columns
        hc->cols = 0;
        hc->paths = 0;
    }
}

__global__ void k_hub_fill(HubIn in, const uint32_t *keep, const uint32_t *coff, const HubCounters *hc,
                           uint32_t *cstart, uint32_t *clen, uint32_t *ca) {
    if (!hc->on) return;
    HUB_GRID_STRIDE(r, in.n) {
        if (!keep[r]) continue;
        const uint32_t c = coff[r];
        const uint32_t o = in.roff[r], deg = in.roff[r + 1] - o;
        const uint32_t hi = in.upoff[r + 1] - in.upoff[r];
        const uint32_t t0 = tail_start(in.nbr + o, 0, deg, in.end);
        cstart[c] = o + t0;
        clen[c] = deg - t0;
        // tail entries from position hi on are ranked below y: those are A'
        ca[c] = hi > t0 ? hi - t0 : 0u;
    }
}

// Split-K product.  The upper triangle of D in 64x64 blocks is 6 blocks off
// the diagonal (2x2 tiles of 32x32 each) and 4 on it (3 tiles: the lower-left
// one lies below the diagonal).  Waves are placed on SIMD w % 4, so the blocks
// go to waves 0-7, 10 and 11: each SIMD issues 8 or 10 tile products per K
// step (one wave per block on waves 0-9 would put 16 on one SIMD).  Every
// tile is a chain of 32x32x32 int8 MFMAs over the chunk.  Both operands are
// read from LDS with the same lane/byte pattern, so the K order inside an
// instruction does not matter.  Output layout of a 32x32 tile: lane l,
// register q holds row 8(q/4) + 4(l/32) + q%4, column l%32.
//
// Column work: 8 threads per column.  While the matrix cores run on chunk c,
// the threads load the neighbours of chunk c+1 (whose column table arrived
// during chunk c-1) and the column table of chunk c+2, so the product, not
// the two dependent global loads, sets the pace.  A thread keeps its first
// two neighbours of a chunk in registers for setting and clearing the tile
// bytes; longer columns read the rest again.  A column's bytes are set and
// cleared only by its own 8 threads, which sit in one wave, and a wave's LDS
// stores take effect in order, so clearing chunk c and setting chunk c+1
// need no barrier between them.
// block (4 bi + bj) of wave w in bits 4w..4w+3; GEMM_ACTIVE: the waves that compute
constexpr uint64_t GEMM_BLOCKS = 0x1ull | 0x3ull << 4 | 0x7ull << 8 | 0xbull << 12 | 0x2ull << 16 | 0x6ull << 20 |
                                 0x0ull << 24 | 0xaull << 28 | 0x5ull << 40 | 0xfull << 44;
constexpr uint32_t GEMM_ACTIVE = 0x0cff;

struct HubCol {
    uint32_t st, len, a0;
};

__device__ inline HubCol hub_col(const uint32_t *cstart, const uint32_t *clen, const uint32_t *ca, uint64_t c,
                                 uint32_t C) {
    if (c >= C) return HubCol{0u, 0u, 0u};
    return HubCol{cstart[c], clen[c], ca[c]};
}

// The thread's neighbours at positions sub and sub + 8 of the column, read
// unconditionally (position st stands in for an absent one; the hub tile
// only runs on a graph with edges), so that nothing waits for them before
// they are used; hub_idx turns them into hub indices.
__device__ inline void hub_first(const uint32_t *nbr, const HubCol &k, uint32_t sub, uint32_t &r0, uint32_t &r1) {
    r0 = nbr[sub < k.len ? k.st + sub : k.st];
    r1 = nbr[sub + 8 < k.len ? k.st + sub + 8 : k.st];
}

// hub index of the neighbour at position j of the column, HUB_T when absent
__device__ inline uint32_t hub_idx(uint32_t raw, uint32_t j, const HubCol &k, uint32_t base) {
    return j < k.len ? raw - base : HUB_T;
}

__device__ inline void hub_put(uint8_t *tA, uint8_t *tB, uint32_t h, uint32_t j, uint32_t a0, uint32_t col,
                               uint8_t v) {
    if (h < HUB_T) {
        tB[h * ROWB + col] = v;
        if (j >= a0) tA[h * ROWB + col] = v;
    }
}

__global__ __launch_bounds__(GEMM_THREADS) void k_hub_gemm(const uint32_t *cstart, const uint32_t *clen,
                                                           const uint32_t *ca, const uint32_t *nbr, uint32_t base,
                                                           const HubCounters *hc, uint32_t *part) {
    __shared__ __attribute__((aligned(16))) uint8_t tA[HUB_T * ROWB];  // A' (lower endpoint h1)
    __shared__ __attribute__((aligned(16))) uint8_t tB[HUB_T * ROWB];  // A (upper endpoint h2)
    if (!hc->on) return;
    const uint32_t C = hc->cols;
    const uint32_t tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
    const uint32_t blk = (uint32_t)(GEMM_BLOCKS >> (4 * w)) & 15u;
    const bool active = (GEMM_ACTIVE >> w) & 1u;
    const uint32_t bi = blk >> 2, bj = blk & 3;
    const bool diag = bi == bj;
    v16i acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[a][b][q] = 0;

    // the tiles are cleared once; after each chunk every thread clears the
    // bytes it set, so a chunk costs its neighbours, not 73 KB of stores
    {
        uint4 *za = reinterpret_cast<uint4 *>(tA), *zb = reinterpret_cast<uint4 *>(tB);
        for (uint32_t i = tid; i < HUB_T * ROWB / 16; i += GEMM_THREADS) {
            za[i] = make_uint4(0, 0, 0, 0);
            zb[i] = make_uint4(0, 0, 0, 0);
        }
    }
    const uint32_t col = tid >> 3, sub = tid & 7;
    const uint32_t step = gridDim.x * KC;
    uint64_t c0 = (uint64_t)blockIdx.x * KC;
    HubCol k0 = hub_col(cstart, clen, ca, c0 + col, C);
    uint32_t r0, r1;
    hub_first(nbr, k0, sub, r0, r1);
    HubCol k1 = hub_col(cstart, clen, ca, c0 + step + col, C);
    __syncthreads();
    for (; c0 < C; c0 += step) {
        const uint32_t h0 = hub_idx(r0, sub, k0, base), h1 = hub_idx(r1, sub + 8, k0, base);
        hub_put(tA, tB, h0, sub, k0.a0, col, 1);
        hub_put(tA, tB, h1, sub + 8, k0.a0, col, 1);
        for (uint32_t j = sub + 16; j < k0.len; j += 8) hub_put(tA, tB, nbr[k0.st + j] - base, j, k0.a0, col, 1);
        __syncthreads();
        // next chunk's neighbours and the column table after it, in flight during the product
        uint32_t g0, g1;
        hub_first(nbr, k1, sub, g0, g1);
        const HubCol k2 = hub_col(cstart, clen, ca, c0 + 2ull * step + col, C);
        if (active) {
#pragma unroll
            for (uint32_t ks = 0; ks < KC; ks += 32) {
                const uint32_t kb = ks + 16 * (lane >> 5);
                v4i a[2], b[2];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    a[t] = *reinterpret_cast<const v4i *>(&tA[(bi * 64 + t * 32 + (lane & 31)) * ROWB + kb]);
                    b[t] = *reinterpret_cast<const v4i *>(&tB[(bj * 64 + t * 32 + (lane & 31)) * ROWB + kb]);
                }
                acc[0][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[0], b[0], acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[0], b[1], acc[0][1], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[1], b[1], acc[1][1], 0, 0, 0);
                if (!diag) acc[1][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[1], b[0], acc[1][0], 0, 0, 0);
            }
        }
        __syncthreads();
        hub_put(tA, tB, h0, sub, k0.a0, col, 0);
        hub_put(tA, tB, h1, sub + 8, k0.a0, col, 0);
        for (uint32_t j = sub + 16; j < k0.len; j += 8) hub_put(tA, tB, nbr[k0.st + j] - base, j, k0.a0, col, 0);
        k0 = k1;
        k1 = k2;
        r0 = g0;
        r1 = g1;
    }
    if (active) {
        uint32_t *P = part + (uint64_t)blockIdx.x * HUB_T * HUB_T;
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int tj = 0; tj < 2; ++tj) {
                if (diag && ti == 1 && tj == 0) continue;  // below the diagonal: never read
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const uint32_t i = bi * 64 + ti * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                    const uint32_t j = bj * 64 + tj * 32 + (lane & 31);
                    P[i * HUB_T + j] = (uint32_t)acc[ti][tj][q];
                }
            }
    }
}

// One block per row i, one thread per column j.
__global__ __launch_bounds__(HUB_T) void k_hub_reduce(const uint32_t *part, uint32_t nparts, uint32_t H,
                                                      unsigned long long *g, unsigned long long *v, uint32_t base,
                                                      HubCounters *hc, uint32_t *D, unsigned long long *roww) {
    __shared__ unsigned long long tmp[HUB_T / WAVE + 1];
    if (!hc->on) return;
    const uint32_t i = blockIdx.x, j = threadIdx.x;
    uint32_t s = 0;
    if (i < H && j < H && j > i)
        for (uint32_t b = 0; b < nparts; ++b) s += part[((uint64_t)b * HUB_T + i) * HUB_T + j];
    D[i * HUB_T + j] = s;
    const unsigned long long t = s >= 2 ? (unsigned long long)s * (s - 1) / 2 : 0ull;
    if (v && t) {
        atomicAdd(&v[base + i], t);
        atomicAdd(&v[base + j], t);
    }
    const unsigned long long rs = block_sum<HUB_T>((unsigned long long)s, tmp);
    const unsigned long long ts = block_sum<HUB_T>(t, tmp);
    if (j == 0) {
        roww[i] = rs;
        if (rs) atomicAdd(&hc->wedges, rs);
        if (ts) atomicAdd(g, ts);
    }
}

}  // namespace

namespace pb {

uint64_t hub_gemm_ops(uint32_t cols) {
    // per chunk of KC columns: 36 tiles of 32x32 (6 blocks of 4, 4 diagonal
    // blocks of 3), KC/32 MFMAs of 32x32x32 (2 * 32^3 operations) each
    const uint64_t chunks = (cols + KC - 1) / KC;
    return chunks * 36ull * (KC / 32) * 2ull * 32 * 32 * 32;
}

pb_status hub_tile(const HubIn &in, HubCounters *hc, const HubOut &out, Workspace &ws, hipStream_t s,
                   hipEvent_t ev0, hipEvent_t ev1, uint32_t *gemm_grid, uint32_t *host_on) {
    const uint64_t n = in.n;
    const uint32_t H = in.end - in.base;
    if (H < 2 || H > HUB_T) return PB_ERR_INVALID_ARG;
    *gemm_grid = 0;
    hipLaunchKernelGGL(k_hub_rank, dim3(grid_for(n)), dim3(256), 0, s, in.smid, n, in.base, in.end, out.hub_rank);
    if (!in.force) {
        // AUTO decides from every HUB_SAMPLE-th vertex's columns; the host
        // reads the decision, so a declined tile costs the sample and one
        // synchronisation, not the marking, scan and compaction of all columns
        hipLaunchKernelGGL(k_hub_mark, dim3(grid_for((n + HUB_SAMPLE - 1) / HUB_SAMPLE, 256, 1024)), dim3(256), 0, s,
                           in, (uint32_t *)nullptr, hc, HUB_SAMPLE);
        hipLaunchKernelGGL(k_hub_decide, dim3(1), dim3(1), 0, s, (const uint32_t *)out.hub_rank, in, hc, HUB_SAMPLE);
        PB_TRY_HIP(hipGetLastError());
        PB_TRY_HIP(hipMemcpyAsync(host_on, &hc->on, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        PB_TRY_HIP(hipStreamSynchronize(s));
        if (!*host_on) return PB_OK;
        hipLaunchKernelGGL(k_hub_reset, dim3(1), dim3(1), 0, s, hc);
    }
    // centres live on the other side: at most that many columns
    const uint64_t other = in.base >= in.n_u ? in.n_u : n - in.n_u;
    uint32_t *keep = ws.alloc<uint32_t>(n + 1), *coff = ws.alloc<uint32_t>(n + 1);
    uint32_t *cstart = ws.alloc<uint32_t>(other + 1), *clen = ws.alloc<uint32_t>(other + 1);
    uint32_t *ca = ws.alloc<uint32_t>(other + 1);
    const uint32_t grid = std::max<uint32_t>(1u, std::min<uint32_t>(GEMM_MAX_GRID, ceil_div(other, KC)));
    uint32_t *part = ws.alloc<uint32_t>((uint64_t)grid * HUB_T * HUB_T);
    if (ws.failed) return PB_ERR_NO_MEMORY;
    *gemm_grid = grid;
    hipLaunchKernelGGL(k_hub_mark, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, in, keep, hc, 1u);
    PB_TRY_HIP(hipGetLastError());
    PB_TRY((scan_exclusive<uint32_t, uint32_t>(keep, coff, n, coff + n, ws)));
    if (in.force) hipLaunchKernelGGL(k_hub_decide, dim3(1), dim3(1), 0, s, (const uint32_t *)out.hub_rank, in, hc, 1u);
    hipLaunchKernelGGL(k_hub_fill, dim3(grid_for(n)), dim3(256), 0, s, in, keep, coff, hc, cstart, clen, ca);
    PB_TRY_HIP(hipGetLastError());
    if (ev0) PB_TRY_HIP(hipEventRecord(ev0, s));
    hipLaunchKernelGGL(k_hub_gemm, dim3(grid), dim3(GEMM_THREADS), 0, s, cstart, clen, ca, in.nbr, in.base, hc,
                       part);
    PB_TRY_HIP(hipGetLastError());
    if (ev1) PB_TRY_HIP(hipEventRecord(ev1, s));
    hipLaunchKernelGGL(k_hub_reduce, dim3(HUB_T), dim3(HUB_T), 0, s, part, grid, H, in.g, in.v, in.base, hc, out.D,
                       out.roww);
    PB_TRY_HIP(hipGetLastError());
    ws.release(part);
    ws.release(ca);
    ws.release(clen);
    ws.release(cstart);
    ws.release(coff);
    ws.release(keep);
    return PB_OK;
}

}  // namespace pb
