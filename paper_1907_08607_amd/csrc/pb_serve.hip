// Serving runtime: resident graph pool, request queue, continuous batching
// over worker slots (one thread and one stream each).
#include "pb_internal.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>

namespace {

struct Request {
    uint64_t id;
    uint32_t graph, want;
    int64_t *gout, *vout, *eout;
    uint64_t footprint;
    double submit_s;
};

struct Resident {
    pb_graph *g;
    const uint32_t *rank;
    uint64_t bytes;
};

// Device scratch of counting one graph (the pipeline's peak allocations plus
// its share of a batch's union arrays), a conservative estimate.
uint64_t scratch_bytes(const pb_graph *g) {
    const uint64_t n = (uint64_t)g->n_u + g->n_v, m = g->m;
    return 128 * m + 112 * n + (1u << 16);
}

// What a resident graph occupies: the caller's CSR, the handle's derived
// arrays and the ranking.
uint64_t resident_bytes(const pb_graph *g) {
    const uint64_t n = (uint64_t)g->n_u + g->n_v, m = g->m;
    return 8 * ((uint64_t)g->n_u + 1) + 4 * m      // caller CSR
           + 4 * m + 4 * ((uint64_t)g->n_v + 1) + 8 * m + 4 * n  // eu, v_off, v_adj, v_eid, deg
           + 4 * n;                                // rank
}

}  // namespace

struct pb_server {
    pb_server_config cfg{};
    pb_tuning tuning{};
    bool has_tuning = false;
    uint64_t budget = 0, resident = 0, inflight = 0;
    std::vector<Resident> pool;
    std::deque<Request> queue;
    std::deque<pb_completion> done;
    uint64_t next_id = 0, submitted = 0, completed = 0;
    bool stop = false;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    int device = 0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    // Under the lock: the next batch this slot may run, or empty.
    std::vector<Request> take_batch() {
        std::vector<Request> batch;
        if (queue.empty()) return batch;
        const uint32_t want = queue.front().want;
        uint64_t fp = 0;
        for (auto it = queue.begin(); it != queue.end() && batch.size() < cfg.max_batch;) {
            if (it->want != want) { ++it; continue; }
            if (resident + inflight + fp + it->footprint > budget) {
                if (batch.empty() && inflight == 0) {
                    // alone on an idle device and still too big: cannot happen
                    // (submit refuses such requests); run it to avoid a stall
                } else {
                    break;
                }
            }
            fp += it->footprint;
            batch.push_back(*it);
            it = queue.erase(it);
        }
        inflight += fp;
        return batch;
    }

    void worker(uint32_t slot) {
        (void)hipSetDevice(device);
        hipStream_t s = streams[slot];
        pb_opts opts;
        pb_opts_default(&opts);
        opts.agg = cfg.agg;
        opts.tuning = has_tuning ? &tuning : nullptr;
        std::vector<pb_graph *> gs;
        std::vector<const uint32_t *> rs;
        std::vector<int64_t *> go, vo, eo;
        while (true) {
            std::vector<Request> batch;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] {
                    if (stop && queue.empty()) return true;
                    batch = take_batch();
                    return !batch.empty();
                });
                if (batch.empty()) return;  // stopping
            }
            const double start = now();
            const uint32_t want = batch[0].want;
            gs.clear(); rs.clear(); go.clear(); vo.clear(); eo.clear();
            uint64_t fp = 0;
            for (const Request &r : batch) {
                gs.push_back(pool[r.graph].g);
                rs.push_back(pool[r.graph].rank);
                go.push_back(r.gout);
                vo.push_back(r.vout);
                eo.push_back(r.eout);
                fp += r.footprint;
            }
            const pb_status st = pb_count_batched(gs.data(), rs.data(), (uint32_t)batch.size(), &opts,
                                                  (want & PB_WANT_GLOBAL) ? go.data() : nullptr,
                                                  (want & PB_WANT_VERTEX) ? vo.data() : nullptr,
                                                  (want & PB_WANT_EDGE) ? eo.data() : nullptr, s);
            const double end = now();
            {
                std::lock_guard<std::mutex> lk(mu);
                inflight -= fp;
                for (const Request &r : batch)
                    done.push_back(pb_completion{r.id, (int32_t)st, (uint32_t)batch.size(), r.submit_s, start, end});
                completed += batch.size();
            }
            cv_work.notify_all();  // memory freed: other slots may admit more
            cv_done.notify_all();
        }
    }
};

extern "C" {

pb_status pb_server_create(const pb_server_config *config, pb_server **out) {
    if (!config || !out || config->slots == 0 || config->max_batch == 0) return PB_ERR_INVALID_ARG;
    if ((int)config->agg < PB_AGG_AUTO || (int)config->agg > PB_AGG_RADIX_SORT) return PB_ERR_INVALID_ARG;
    *out = nullptr;
    pb_server *srv = new (std::nothrow) pb_server();
    if (!srv) return PB_ERR_NO_MEMORY;
    srv->cfg = *config;
    if (config->tuning) {
        srv->tuning = *config->tuning;
        srv->has_tuning = true;
    }
    srv->cfg.tuning = nullptr;
    if (hipGetDevice(&srv->device) != hipSuccess) { delete srv; return PB_ERR_HIP; }
    srv->budget = config->hbm_budget_bytes;
    if (srv->budget == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) { delete srv; return PB_ERR_HIP; }
        srv->budget = free_b;
    }
    for (uint32_t i = 0; i < config->slots; ++i) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            pb_server_destroy(srv);
            return PB_ERR_HIP;
        }
        srv->streams.push_back(s);
    }
    for (uint32_t i = 0; i < config->slots; ++i) srv->workers.emplace_back(&pb_server::worker, srv, i);
    *out = srv;
    return PB_OK;
}

pb_status pb_server_add_graph(pb_server *srv, pb_graph *g, const uint32_t *rank, uint32_t *graph_id) {
    if (!srv || !g || !rank || !graph_id) return PB_ERR_INVALID_ARG;
    const uint64_t bytes = resident_bytes(g);
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->resident + bytes > srv->budget) return PB_ERR_NO_MEMORY;
    srv->resident += bytes;
    *graph_id = (uint32_t)srv->pool.size();
    srv->pool.push_back(Resident{g, rank, bytes});
    return PB_OK;
}

pb_status pb_server_submit(pb_server *srv, uint32_t graph_id, uint32_t want, int64_t *global_out,
                           int64_t *vertex_out, int64_t *edge_out, uint64_t *request_id) {
    if (!srv || !request_id) return PB_ERR_INVALID_ARG;
    if (want == 0 || (want & ~7u)) return PB_ERR_INVALID_ARG;
    if (((want & PB_WANT_GLOBAL) && !global_out) || ((want & PB_WANT_VERTEX) && !vertex_out)) return PB_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (graph_id >= srv->pool.size()) return PB_ERR_INVALID_ARG;
        const pb_graph *g = srv->pool[graph_id].g;
        if ((want & PB_WANT_EDGE) && !edge_out && g->m) return PB_ERR_INVALID_ARG;
        const uint64_t fp = scratch_bytes(g);
        if (srv->resident + fp > srv->budget) return PB_ERR_NO_MEMORY;
        Request r{srv->next_id++, graph_id, want, global_out, vertex_out, edge_out, fp, srv->now()};
        *request_id = r.id;
        srv->queue.push_back(r);
        srv->submitted += 1;
    }
    srv->cv_work.notify_one();
    return PB_OK;
}

pb_status pb_server_poll(pb_server *srv, pb_completion *out, uint32_t max, uint32_t *count) {
    if (!srv || !count || (max && !out)) return PB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    uint32_t k = 0;
    while (k < max && !srv->done.empty()) {
        out[k++] = srv->done.front();
        srv->done.pop_front();
    }
    *count = k;
    return PB_OK;
}

pb_status pb_server_drain(pb_server *srv) {
    if (!srv) return PB_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [&] { return srv->completed == srv->submitted; });
    return PB_OK;
}

void pb_server_destroy(pb_server *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    for (auto &t : srv->workers) t.join();
    for (auto s : srv->streams) (void)hipStreamDestroy(s);
    delete srv;
}

}  // extern "C"
