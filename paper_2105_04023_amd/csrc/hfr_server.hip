// Serving engine: influence-maximisation requests over a pool of resident
// graphs, answered by concurrent slots.
//
// Each slot is one host thread with its own HIP stream and its own context,
// so the requests of different slots overlap on the device; a request that
// arrives while others run is queued and admitted as soon as its slot is
// free.  Sketches (the build of Alg. 1 + Alg. 2 for one graph, edge model, R
// and hash seed) stay resident in the slot that built them and are reused by
// later requests with the same key; every request runs its own greedy
// selection (im_select_seeds starts from the build's registers each time).
// Device memory is admitted by budget: the resident graphs and every slot's
// sketches share hbm_budget, each slot holding at most an equal share of what
// the graphs leave; a slot evicts its least recently used idle sketches until
// a new build fits.  A request routes to the slot that holds (or is about to
// build) its sketch, else to the slot with the least queued work.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "hfr_host.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

struct GraphRes {
    int64_t n = 0, m = 0;
    int64_t* xadj = nullptr;
    int32_t* adj = nullptr;
    size_t bytes = 0;
};

// (graph, kind, p bits, R, hash seed, eps_c bits)
using Key = std::tuple<int32_t, int32_t, uint32_t, int32_t, uint32_t, uint64_t>;

struct Request {
    int64_t ticket = 0;
    im_request rq{};
    Key key;
    int32_t* out_seeds = nullptr;
    double work = 0.0;
    Clock::time_point t_submit, t_start, t_end;
    im_response resp{};
    std::string error;
    bool done = false;
};

struct CachedSketch {
    im_sketch* sk = nullptr;
    size_t bytes = 0;
    uint64_t last_use = 0;
};

struct Slot {
    int index = 0;
    hipStream_t stream = nullptr;
    im_ctx* ctx = nullptr;
    std::thread thread;
    std::deque<std::shared_ptr<Request>> queue;
    double queued_work = 0.0;
    std::map<Key, CachedSketch> cache;
};

}  // namespace

struct im_server {
    int device = 0;
    size_t budget = 0;
    size_t graph_bytes = 0;
    size_t slot_budget = 0;
    std::vector<GraphRes> graphs;
    std::vector<std::unique_ptr<Slot>> slots;
    std::map<Key, int> route;  // key -> slot holding or building its sketch
    std::map<int64_t, std::shared_ptr<Request>> requests;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stopping = false;
    bool started = false;  // a request was submitted: the graph pool is fixed
    int64_t next_ticket = 1;
    uint64_t use_clock = 0;
    im_server_stats stats{};
};

namespace {

// Runs one request on its slot (slot thread, server lock not held).
void serve(im_server* sv, Slot* sl, Request* r) {
    const im_request& q = r->rq;
    const GraphRes& g = sv->graphs[q.graph];
    im_status st = IM_OK;
    im_sketch* sk = nullptr;
    bool reused = false;
    double build_ms = 0.0;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sl->cache.find(r->key);
        if (it != sl->cache.end()) {
            sk = it->second.sk;
            it->second.last_use = ++sv->use_clock;
            reused = true;
        }
    }
    if (!sk) {
        im_csr csr{g.n, g.m, g.xadj, g.adj, 1};
        im_probs pr{(im_prob_kind)q.kind, q.p, nullptr};
        im_build_opts bo{};
        bo.eps_c = q.eps_c;
        const auto t0 = Clock::now();
        st = im_build_sketches(sl->ctx, &csr, &pr, q.R, q.hash_seed, &bo, &sk);
        if (st == IM_ERR_OUT_OF_BUDGET) {
            // evict idle sketches of this slot, least recently used first
            while (st == IM_ERR_OUT_OF_BUDGET) {
                im_sketch* victim = nullptr;
                {
                    std::lock_guard<std::mutex> lk(sv->mu);
                    auto best = sl->cache.end();
                    for (auto it = sl->cache.begin(); it != sl->cache.end(); ++it)
                        if (best == sl->cache.end() || it->second.last_use < best->second.last_use) best = it;
                    if (best != sl->cache.end()) {
                        victim = best->second.sk;
                        sv->route.erase(best->first);
                        sl->cache.erase(best);
                        sv->stats.evictions += 1;
                    }
                }
                if (!victim) break;
                im_sketch_free(victim);
                st = im_build_sketches(sl->ctx, &csr, &pr, q.R, q.hash_seed, &bo, &sk);
            }
        }
        build_ms = ms_between(t0, Clock::now());
        if (st == IM_OK) {
            std::lock_guard<std::mutex> lk(sv->mu);
            CachedSketch cs;
            im_sketch_info info{};
            cs.sk = sk;
            if (im_sketch_get_info(sk, &info) == IM_OK) cs.bytes = info.device_bytes;
            cs.last_use = ++sv->use_clock;
            sl->cache[r->key] = cs;
            sv->stats.sketches_built += 1;
        } else {
            r->error = im_last_error();
        }
    }
    int32_t rebuilds = 0;
    double select_ms = 0.0;
    if (st == IM_OK) {
        im_select_opts so{q.eps_g, q.eps_l};
        im_select_stats ss{};
        const auto t0 = Clock::now();
        st = im_select_seeds(sk, q.K, &so, r->out_seeds, nullptr, &ss);
        select_ms = ms_between(t0, Clock::now());
        rebuilds = ss.rebuilds;
        if (st != IM_OK) r->error = im_last_error();
    }
    r->resp.status = st;
    r->resp.slot = sl->index;
    r->resp.sketch_reused = reused ? 1 : 0;
    r->resp.rebuilds = rebuilds;
    r->resp.build_ms = build_ms;
    r->resp.select_ms = select_ms;
}

void slot_main(im_server* sv, Slot* sl) {
    (void)hipSetDevice(sv->device);
    while (true) {
        std::shared_ptr<Request> r;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_work.wait(lk, [&] { return sv->stopping || !sl->queue.empty(); });
            if (sl->queue.empty()) return;  // stopping and drained
            r = sl->queue.front();
            sl->queue.pop_front();
            r->t_start = Clock::now();
        }
        serve(sv, sl, r.get());
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            r->t_end = Clock::now();
            r->resp.queue_ms = ms_between(r->t_submit, r->t_start);
            r->resp.latency_ms = ms_between(r->t_submit, r->t_end);
            r->done = true;
            sl->queued_work -= r->work;
            sv->stats.completed += 1;
            if (r->resp.status != IM_OK) sv->stats.failed += 1;
        }
        sv->cv_done.notify_all();
    }
}

void server_release(im_server* sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stopping = true;
    }
    sv->cv_work.notify_all();
    for (auto& sl : sv->slots)
        if (sl->thread.joinable()) sl->thread.join();
    for (auto& sl : sv->slots) {
        for (auto& kv : sl->cache) im_sketch_free(kv.second.sk);
        if (sl->ctx) im_ctx_free(sl->ctx);
        if (sl->stream) (void)hipStreamDestroy(sl->stream);
    }
    for (auto& g : sv->graphs) {
        if (g.xadj) (void)hipFree(g.xadj);
        if (g.adj) (void)hipFree(g.adj);
    }
    delete sv;
}

}  // namespace

extern "C" {

im_status im_server_create(int32_t device, const im_server_opts* opts, im_server** out) {
    if (!opts || !out) return hfr::fail(IM_ERR_INVALID_ARG, "null argument");
    if (opts->slots < 1 || opts->slots > 64) return hfr::fail(IM_ERR_INVALID_ARG, "slots must be in [1, 64]");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return hfr::fail(IM_ERR_INVALID_ARG, "device %d out of range", device);
    if (hipSetDevice(device) != hipSuccess) return hfr::fail(IM_ERR_DEVICE, "hipSetDevice failed");
    im_server* sv = new im_server;
    sv->device = device;
    sv->budget = opts->hbm_budget;
    for (int i = 0; i < opts->slots; ++i) {
        auto sl = std::make_unique<Slot>();
        sl->index = i;
        if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess) {
            server_release(sv);
            return hfr::fail(IM_ERR_DEVICE, "stream creation failed");
        }
        if (im_ctx_create(device, sl->stream, 0, nullptr, nullptr, nullptr, &sl->ctx) != IM_OK) {
            server_release(sv);
            return IM_ERR_DEVICE;
        }
        sv->slots.push_back(std::move(sl));
    }
    for (auto& sl : sv->slots) sl->thread = std::thread(slot_main, sv, sl.get());
    *out = sv;
    return IM_OK;
}

im_status im_server_add_graph(im_server* sv, const im_csr* graph, int32_t* out_graph) {
    if (!sv || !graph || !out_graph) return hfr::fail(IM_ERR_INVALID_ARG, "null argument");
    const int64_t n = graph->n, m = graph->m;
    if (n < 1 || n >= (1ll << 31) || m < 0 || !graph->xadj || (m > 0 && !graph->adj))
        return hfr::fail(IM_ERR_INVALID_GRAPH, "malformed CSR");
    if (const im_status oc = hfr::csr_offsets_check(graph); oc != IM_OK) return oc;
    if (hipSetDevice(sv->device) != hipSuccess) return hfr::fail(IM_ERR_DEVICE, "hipSetDevice failed");
    GraphRes g;
    g.n = n;
    g.m = m;
    g.bytes = 8 * (size_t)(n + 1) + 4 * (size_t)m;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->started) return hfr::fail(IM_ERR_STATE, "graphs must be added before the first request");
    if (sv->budget && sv->graph_bytes + g.bytes > sv->budget)
        return hfr::fail(IM_ERR_OUT_OF_BUDGET, "the graph pool exceeds the budget");
    const hipMemcpyKind kind = graph->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (hipMalloc(&g.xadj, 8 * (n + 1)) != hipSuccess || (hipMalloc(&g.adj, 4 * (m ? m : 1)) != hipSuccess) ||
        hfr::csr_copy_offsets(graph, g.xadj, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
        (m > 0 && hipMemcpy(g.adj, graph->adj, 4 * m, kind) != hipSuccess)) {
        if (g.xadj) (void)hipFree(g.xadj);
        if (g.adj) (void)hipFree(g.adj);
        return hfr::fail(IM_ERR_DEVICE, "graph upload failed");
    }
    sv->graph_bytes += g.bytes;
    sv->graphs.push_back(g);
    // every slot may hold an equal share of what the graphs leave
    const size_t left = sv->budget ? sv->budget - sv->graph_bytes : 0;
    sv->slot_budget = sv->budget ? std::max<size_t>(left / sv->slots.size(), 1) : 0;
    for (auto& sl : sv->slots) sl->ctx->budget = sv->slot_budget;
    *out_graph = (int32_t)sv->graphs.size() - 1;
    return IM_OK;
}

im_status im_server_submit(im_server* sv, const im_request* rq, int32_t* out_seeds, int64_t* out_ticket) {
    if (!sv || !rq || !out_seeds || !out_ticket) return hfr::fail(IM_ERR_INVALID_ARG, "null argument");
    if (rq->graph < 0 || rq->graph >= (int32_t)sv->graphs.size())
        return hfr::fail(IM_ERR_INVALID_ARG, "unknown graph %d", rq->graph);
    if (rq->kind != IM_PROB_CONSTANT && rq->kind != IM_PROB_WEIGHTED_CASCADE)
        return hfr::fail(IM_ERR_INVALID_ARG, "requests take a constant probability or the weighted cascade");
    if (rq->kind == IM_PROB_CONSTANT && hfr::live_threshold(rq->p) == 0xFFFFFFFFu)
        return hfr::fail(IM_ERR_INVALID_ARG, "probability must be in [0, 1]");
    if (rq->R < 4 || rq->R > 1024 || rq->R % 4) return hfr::fail(IM_ERR_INVALID_ARG, "R must be a multiple of 4 in [4, 1024]");
    const GraphRes& g = sv->graphs[rq->graph];
    if (rq->K < 1 || rq->K > g.n) return hfr::fail(IM_ERR_INVALID_ARG, "K must be in [1, n]");
    if (!(rq->eps_c >= 0.0) || !(rq->eps_g >= 0.0) || !(rq->eps_l >= 0.0))
        return hfr::fail(IM_ERR_INVALID_ARG, "thresholds must be >= 0");
    auto r = std::make_shared<Request>();
    r->rq = *rq;
    uint32_t pbits = 0;
    if (rq->kind == IM_PROB_CONSTANT) memcpy(&pbits, &rq->p, 4);
    uint64_t ebits = 0;
    memcpy(&ebits, &rq->eps_c, 8);
    r->key = Key(rq->graph, rq->kind, pbits, rq->R, rq->hash_seed, ebits);
    r->out_seeds = out_seeds;
    r->work = (double)(g.n + g.m) * (double)rq->R * (1.0 + 0.02 * rq->K);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->started = true;
        r->ticket = sv->next_ticket++;
        r->t_submit = Clock::now();
        int s = -1;
        auto it = sv->route.find(r->key);
        if (it != sv->route.end()) {
            s = it->second;
        } else {
            double best = 0.0;
            for (auto& sl : sv->slots)
                if (s < 0 || sl->queued_work < best) {
                    best = sl->queued_work;
                    s = sl->index;
                }
            sv->route[r->key] = s;
        }
        Slot* sl = sv->slots[s].get();
        sl->queue.push_back(r);
        sl->queued_work += r->work;
        sv->requests[r->ticket] = r;
        sv->stats.submitted += 1;
        *out_ticket = r->ticket;
    }
    sv->cv_work.notify_all();
    return IM_OK;
}

im_status im_server_wait(im_server* sv, int64_t ticket, im_response* out) {
    if (!sv) return hfr::fail(IM_ERR_INVALID_ARG, "null server");
    std::shared_ptr<Request> r;
    {
        std::unique_lock<std::mutex> lk(sv->mu);
        auto it = sv->requests.find(ticket);
        if (it == sv->requests.end()) return hfr::fail(IM_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
        r = it->second;
        sv->cv_done.wait(lk, [&] { return r->done; });
        sv->requests.erase(ticket);
    }
    if (out) *out = r->resp;
    if (r->resp.status != IM_OK) return hfr::fail((im_status)r->resp.status, "%s", r->error.c_str());
    return IM_OK;
}

im_status im_server_get_stats(im_server* sv, im_server_stats* out) {
    if (!sv || !out) return hfr::fail(IM_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->stats;
    size_t used = sv->graph_bytes;
    int64_t resident = 0;
    for (auto& sl : sv->slots) {
        used += im_ctx_bytes_in_use(sl->ctx);
        resident += (int64_t)sl->cache.size();
    }
    out->device_bytes = used;
    out->resident_sketches = resident;
    return IM_OK;
}

void im_server_free(im_server* sv) { server_release(sv); }

}  // extern "C"
