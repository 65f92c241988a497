// Wedge counts of a ranking and the ranking chooser of the experiments'
// ranking results (Section 6.2, metric f and Table 3).
//
// W(rank), the wedges the framework retrieves (Algorithm 2), has a per-vertex
// closed form.  A wedge (x1, y, x2) is retrieved once, from the endpoint x1
// ranked above both others.  Fix the centre y with d = deg(y) and let h(y) be
// the number of its neighbours ranked above y.  Those h neighbours are the
// possible x1; the j-th of them in rank order has d - j neighbours of y ranked
// below it, each a possible x2.  So W = sum over y of h*d - h*(h+1)/2.  h(y)
// is one comparison per edge end, summed per row of each side's CSR.
#include "pb_internal.h"

using namespace pb;

namespace {

constexpr uint32_t NO_KEY = 0xFFFFFFFFu;

// h(y) for the rows of one side.  Entry p of that side's CSR belongs to row
// key(p) (rows are contiguous); it counts when its neighbour is ranked above
// the row's vertex.  Each wave sums the entries of every row segment it holds
// and adds the segment's sum with one atomic.
struct Rows {
    const uint32_t *rank;
    const uint32_t *eu;     // U row of each edge (U-CSR order)
    const uint32_t *u_adj;  // V id of each edge
    const uint32_t *v_adj;  // U id of each V-CSR entry
    const uint32_t *v_eid;  // edge of each V-CSR entry
    uint32_t n_u;
    uint64_t m;
};

__global__ __launch_bounds__(256) void k_above(Rows R, int vside, uint32_t *h) {
    const uint32_t lane = threadIdx.x & (WAVE - 1);
    const uint64_t le = lanemask_lt() | (1ull << lane);
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / WAVE);
    for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE) * WAVE; base < R.m;
         base += waves * WAVE) {
        const uint64_t p = base + lane;
        uint32_t key = NO_KEY, val = 0;
        if (p < R.m) {
            uint32_t self, other;
            if (!vside) {
                self = R.eu[p];
                other = R.n_u + R.u_adj[p];
            } else {
                self = R.n_u + R.u_adj[R.v_eid[p]];
                other = R.v_adj[p];
            }
            key = self;
            val = R.rank[other] < R.rank[self] ? 1u : 0u;
        }
        const uint32_t prev = __shfl(key, lane ? lane - 1 : 0, WAVE);
        const uint64_t heads = __ballot(lane == 0 || prev != key);
        const uint32_t incl = wave_inclusive_sum(val);
        const uint32_t start = 63u - (uint32_t)__clzll(heads & le);
        const uint32_t before = __shfl(incl, start ? start - 1 : 0, WAVE);
        const uint32_t seg = incl - (start ? before : 0u);
        const bool last = lane == WAVE - 1 || ((heads >> (lane + 1)) & 1);
        if (last && seg && key != NO_KEY) atomicAdd(&h[key], seg);
    }
}

// W = sum over y of h*d - h*(h+1)/2
__global__ __launch_bounds__(256) void k_wedge_sum(const uint32_t *h, const uint32_t *deg, uint64_t n,
                                                   unsigned long long *w) {
    __shared__ unsigned long long tmp[256 / WAVE];
    unsigned long long s = 0;
    for (uint64_t y = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; y < n; y += (uint64_t)gridDim.x * blockDim.x) {
        const unsigned long long hh = h[y], d = deg[y];
        s += hh * d - hh * (hh + 1) / 2;
    }
    s = block_sum<256>(s, tmp);
    if (threadIdx.x == 0 && s) atomicAdd(w, s);
}

uint32_t grid_of(uint64_t n, uint32_t cap) {
    const uint64_t g = (n + 255) / 256;
    return (uint32_t)(g == 0 ? 1 : g > cap ? cap : g);
}

pb_status wedges_impl(pb_graph *g, const uint32_t *rank, uint64_t *w_out, hipStream_t s) {
    if (!g || !rank || !w_out) return PB_ERR_INVALID_ARG;
    const uint64_t n = (uint64_t)g->n_u + g->n_v;
    *w_out = 0;
    if (n == 0 || g->m == 0) return PB_OK;
    Workspace ws(s, 0);
    uint32_t *h = ws.alloc<uint32_t>(n);
    unsigned long long *w = ws.alloc<unsigned long long>(1);
    if (ws.failed) return PB_ERR_NO_MEMORY;
    PB_TRY(fill<uint32_t>(h, 0u, n, s));
    PB_TRY(fill<uint64_t>((uint64_t *)w, 0ull, 1, s));
    const Rows R{rank, g->eu, g->u_adj, g->v_adj, g->v_eid, g->n_u, g->m};
    for (int side = 0; side < 2; ++side)
        hipLaunchKernelGGL(k_above, dim3(grid_of(g->m, 4096)), dim3(256), 0, s, R, side, h);
    hipLaunchKernelGGL(k_wedge_sum, dim3(grid_of(n, 1024)), dim3(256), 0, s, (const uint32_t *)h,
                       (const uint32_t *)g->deg, n, w);
    PB_TRY_HIP(hipGetLastError());
    unsigned long long hw = 0;
    PB_TRY_HIP(hipMemcpyAsync(&hw, w, sizeof(hw), hipMemcpyDeviceToHost, s));
    PB_TRY_HIP(hipStreamSynchronize(s));
    *w_out = hw;
    return PB_OK;
}

}  // namespace

extern "C" {

pb_status pb_wedges(pb_graph *g, const uint32_t *rank, uint64_t *w_out, hipStream_t stream) {
    return wedges_impl(g, rank, w_out, stream);
}

pb_status pb_rank_choose(pb_graph *g, pb_rank_kind other, uint32_t *rank_out, pb_rank_kind *chosen,
                         uint64_t *w_side, uint64_t *w_other, hipStream_t stream) {
    if (!g || !rank_out || !chosen) return PB_ERR_INVALID_ARG;
    if ((int)other < PB_RANK_SIDE_AUTO || (int)other > PB_RANK_APPROX_COMPLEMENT_CORENESS) return PB_ERR_INVALID_ARG;
    uint64_t ws_ = 0, wr = 0;
    // the other order first (into rank_out), then side order if it wins
    PB_TRY(pb_rank(g, other, rank_out, stream));
    PB_TRY(wedges_impl(g, rank_out, &wr, stream));
    {
        Workspace ws(stream, 0);
        const uint64_t n = (uint64_t)g->n_u + g->n_v;
        uint32_t *side = ws.alloc<uint32_t>(n);
        if (ws.failed) return PB_ERR_NO_MEMORY;
        PB_TRY(pb_rank(g, PB_RANK_SIDE_AUTO, side, stream));
        PB_TRY(wedges_impl(g, side, &ws_, stream));
        // f = (w_s - w_r) / w_s < 0.1, in integers: w_r >= w_s, or 10 (w_s - w_r) < w_s
        const bool use_side = wr >= ws_ || 10 * (ws_ - wr) < ws_;
        if (use_side && n) PB_TRY_HIP(hipMemcpyAsync(rank_out, side, n * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                                                     stream));
        PB_TRY_HIP(hipStreamSynchronize(stream));
        *chosen = use_side ? PB_RANK_SIDE_AUTO : other;
    }
    if (w_side) *w_side = ws_;
    if (w_other) *w_other = wr;
    return PB_OK;
}

}  // extern "C"
