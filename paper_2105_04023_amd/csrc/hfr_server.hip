// Serving engine: influence-maximisation requests over a pool of resident
// graphs, answered by concurrent slots (the scheduling is hfr_sched.h's).
//
// Each slot is one host thread with its own HIP stream and its own context,
// so the requests of different slots overlap on the device.  Requests wait in
// one shared queue and each free slot takes the oldest one it can start now,
// so a request is admitted as soon as any slot and the memory it needs are
// free.  Sketches (the build of Alg. 1 + Alg. 2 for one graph, edge model, p,
// R, hash seed and eps_c) form one pool: a later request with the same key
// reuses an idle copy on whichever slot runs it (the sketch is moved to that
// slot's stream), and a key with every copy busy may get another copy (up to
// max_copies, default 1).
// A request's selection goes through im_select_seeds_resume: a sketch keeps the
// greedy run of its last request, a request with the same thresholds and a K
// no larger is answered from that run and a larger K continues it, so
// repeated and growing K on one key cost only the steps not yet taken.  The
// outputs are those of im_select_seeds, so a served result equals
// im_build_sketches + im_select_seeds run alone.  The resident graphs and all
// sketches share hbm_budget; a build evicts idle sketches least recently used
// first until it fits, and a build that cannot fit even alone is refused.
#include <hip/hip_runtime.h>
#include <string.h>

#include <memory>
#include <mutex>
#include <vector>

#include "hfr_host.h"
#include "hfr_sched.h"

namespace {

struct GraphRes {
    int64_t n = 0, m = 0;
    int64_t* xadj = nullptr;
    int32_t* adj = nullptr;
    size_t bytes = 0;
};

struct Payload {
    im_request rq{};
    GraphRes g;
    int32_t* out_seeds = nullptr;
};

struct SlotRes {
    hipStream_t stream = nullptr;
    im_ctx* ctx = nullptr;
};

// The HIP path behind the scheduler: build and select through the C ABI on the
// slot's context.
struct HipBackend final : hfr::sched::Backend<Payload> {
    int device = 0;
    std::vector<SlotRes> slots;

    im_status build(int slot, const Payload& p, void** handle, size_t* bytes, std::string* err) override {
        (void)hipSetDevice(device);
        const im_request& q = p.rq;
        im_csr csr{p.g.n, p.g.m, p.g.xadj, p.g.adj, 1, 64};
        im_probs pr{(im_prob_kind)q.kind, q.p, nullptr};
        im_build_opts bo{};
        bo.eps_c = q.eps_c;
        im_sketch* sk = nullptr;
        const im_status st = im_build_sketches(slots[slot].ctx, &csr, &pr, q.R, q.hash_seed, &bo, &sk);
        if (st != IM_OK) {
            *err = im_last_error();
            return st;
        }
        im_sketch_info info{};
        *bytes = im_sketch_get_info(sk, &info) == IM_OK ? info.device_bytes : 0;
        *handle = sk;
        return IM_OK;
    }
    void adopt(int slot, void* handle) override {
        (void)hipSetDevice(device);
        hfr::sketch_rebind(static_cast<im_sketch*>(handle), slots[slot].ctx);
    }
    im_status select(int slot, void* handle, const Payload& p, int32_t* rebuilds, std::string* err) override {
        (void)slot;
        (void)hipSetDevice(device);
        im_select_opts so{p.rq.eps_g, p.rq.eps_l};
        im_select_stats ss{};
        const im_status st =
            im_select_seeds_resume(static_cast<im_sketch*>(handle), p.rq.K, &so, p.out_seeds, nullptr, &ss);
        *rebuilds = ss.rebuilds;
        if (st != IM_OK) *err = im_last_error();
        return st;
    }
    void release(void* handle) override {
        (void)hipSetDevice(device);
        im_sketch_free(static_cast<im_sketch*>(handle));
    }
};

}  // namespace

struct im_server {
    int device = 0;
    size_t budget = 0;
    std::mutex mu;                 // guards graphs, graph_bytes, started
    std::vector<GraphRes> graphs;  // fixed once the first request is submitted
    size_t graph_bytes = 0;
    bool started = false;
    HipBackend backend;
    std::unique_ptr<hfr::sched::Scheduler<Payload>> sched;
};

namespace {

void server_release(im_server* sv) {
    if (!sv) return;
    if (sv->sched) sv->sched->stop();  // finishes queued requests, frees every sketch
    sv->sched.reset();
    for (auto& sl : sv->backend.slots) {
        if (sl.ctx) im_ctx_free(sl.ctx);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
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
    if (opts->max_copies < 0 || opts->max_copies > 64)
        return hfr::fail(IM_ERR_INVALID_ARG, "max_copies must be in [0, 64]");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return hfr::fail(IM_ERR_INVALID_ARG, "device %d out of range", device);
    if (hipSetDevice(device) != hipSuccess) return hfr::fail(IM_ERR_DEVICE, "hipSetDevice failed");
    im_server* sv = new im_server;
    sv->device = device;
    sv->budget = opts->hbm_budget;
    sv->backend.device = device;
    for (int i = 0; i < opts->slots; ++i) {
        SlotRes sl;
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) {
            server_release(sv);
            return hfr::fail(IM_ERR_DEVICE, "stream creation failed");
        }
        // no per-context bound: the scheduler admits builds by the server's budget
        if (im_ctx_create(device, sl.stream, 0, nullptr, nullptr, nullptr, &sl.ctx) != IM_OK) {
            (void)hipStreamDestroy(sl.stream);
            server_release(sv);
            return IM_ERR_DEVICE;
        }
        sv->backend.slots.push_back(sl);
    }
    sv->sched = std::make_unique<hfr::sched::Scheduler<Payload>>(opts->slots, opts->hbm_budget, &sv->backend,
                                                                 opts->max_copies ? opts->max_copies : 1);
    sv->sched->start();
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
    sv->sched->set_fixed_bytes(sv->graph_bytes);
    *out_graph = (int32_t)sv->graphs.size() - 1;
    return IM_OK;
}

im_status im_server_submit(im_server* sv, const im_request* rq, int32_t* out_seeds, int64_t* out_ticket) {
    if (!sv || !rq || !out_seeds || !out_ticket) return hfr::fail(IM_ERR_INVALID_ARG, "null argument");
    if (rq->kind != IM_PROB_CONSTANT && rq->kind != IM_PROB_WEIGHTED_CASCADE)
        return hfr::fail(IM_ERR_INVALID_ARG, "requests take a constant probability or the weighted cascade");
    if (rq->kind == IM_PROB_CONSTANT && hfr::live_threshold(rq->p) == 0xFFFFFFFFu)
        return hfr::fail(IM_ERR_INVALID_ARG, "probability must be in [0, 1]");
    if (rq->R < 4 || rq->R > 1024 || rq->R % 4) return hfr::fail(IM_ERR_INVALID_ARG, "R must be a multiple of 4 in [4, 1024]");
    if (!(rq->eps_c >= 0.0) || !(rq->eps_g >= 0.0) || !(rq->eps_l >= 0.0))
        return hfr::fail(IM_ERR_INVALID_ARG, "thresholds must be >= 0");
    Payload p;
    {
        // the graph table is read under the lock that add_graph takes
        std::lock_guard<std::mutex> lk(sv->mu);
        if (rq->graph < 0 || rq->graph >= (int32_t)sv->graphs.size())
            return hfr::fail(IM_ERR_INVALID_ARG, "unknown graph %d", rq->graph);
        p.g = sv->graphs[rq->graph];
        sv->started = true;
    }
    if (rq->K < 1 || rq->K > p.g.n) return hfr::fail(IM_ERR_INVALID_ARG, "K must be in [1, n]");
    p.rq = *rq;
    p.out_seeds = out_seeds;
    uint32_t pbits = 0;
    if (rq->kind == IM_PROB_CONSTANT) memcpy(&pbits, &rq->p, 4);
    uint64_t ebits = 0;
    memcpy(&ebits, &rq->eps_c, 8);
    const hfr::sched::SketchKey key(rq->graph, rq->kind, pbits, rq->R, rq->hash_seed, ebits);
    const size_t need = im_sketch_bytes_needed(p.g.n, p.g.m, rq->R, (im_prob_kind)rq->kind);
    *out_ticket = sv->sched->submit(key, need, p);
    return IM_OK;
}

im_status im_server_cancel(im_server* sv, int64_t ticket) {
    if (!sv) return hfr::fail(IM_ERR_INVALID_ARG, "null server");
    if (sv->sched->cancel(ticket) != IM_OK)
        return hfr::fail(IM_ERR_STATE, "ticket %lld is unknown, running or finished", (long long)ticket);
    return IM_OK;
}

im_status im_server_wait(im_server* sv, int64_t ticket, im_response* out) {
    if (!sv) return hfr::fail(IM_ERR_INVALID_ARG, "null server");
    hfr::sched::Outcome o;
    if (!sv->sched->wait(ticket, &o)) return hfr::fail(IM_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
    if (out) *out = o.resp;
    if (o.resp.status != IM_OK) return hfr::fail((im_status)o.resp.status, "%s", o.error.c_str());
    return IM_OK;
}

im_status im_server_get_stats(im_server* sv, im_server_stats* out) {
    if (!sv || !out) return hfr::fail(IM_ERR_INVALID_ARG, "null argument");
    const hfr::sched::Stats s = sv->sched->stats();
    size_t gb = 0;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        gb = sv->graph_bytes;
    }
    out->submitted = s.submitted;
    out->completed = s.completed;
    out->failed = s.failed;
    out->sketches_built = s.sketches_built;
    out->evictions = s.evictions;
    out->resident_sketches = s.resident_sketches;
    out->device_bytes = gb + s.sketch_bytes;
    return IM_OK;
}

void im_server_free(im_server* sv) { server_release(sv); }

}  // extern "C"
