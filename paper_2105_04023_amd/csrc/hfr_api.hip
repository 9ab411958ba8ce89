// Host side of the library: the C ABI declared in include/im.h.
//
// Control flow per call:
//  - im_build_sketches: upload/copy the CSR, validate it on the device, hash
//    every edge, derive the integer live thresholds, split high-degree rows,
//    then Simulate (Alg. 2): init + synchronous sweeps.  Sweeps are launched
//    in batches; each sweep kernel reads the live count of the previous sweep
//    from device memory and returns at once when the stopping rule holds, so
//    the host only reads counts back once per batch, one batch ahead.
//  - im_select_seeds: the greedy loop of Alg. 1 with device argmax, device
//    multi-sample BFS for the Monte-Carlo reach, an FP64 decision kernel and a
//    rebuild (init with blocked pairs + Simulate) when the decision asks.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <string>
#include <vector>

#include "hfr_host.h"

using namespace hfr;

// Scratch of the allocation-free selection (im_select_seeds_noalloc): the step
// records and seeds of one call with K <= IM_NOALLOC_MAX_K.  Each device holds
// its own copy for the life of the process.  Host code never passes this name
// to a kernel or a copy: it uses the device address recorded per device when a
// context is created (init_scratch).
constexpr size_t NOALLOC_SCRATCH_BYTES = 512 * 1024;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
im_status init_scratch(int device);
}

namespace hfr {

thread_local std::string g_last_error;

im_status fail(im_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

void* ctx_alloc(im_ctx* c, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    void* p = nullptr;
    if (c->af) {
        p = c->af(bytes, c->user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    return p;
}

void ctx_free(im_ctx* c, void* p) {
    if (!p) return;
    if (c->ff)
        c->ff(p, c->user);
    else
        (void)hipFree(p);
}

im_status csr_offsets_check(const im_csr* g) {
    if (g->offset_bits != 0 && g->offset_bits != 32 && g->offset_bits != 64)
        return fail(IM_ERR_INVALID_ARG, "offset_bits must be 0, 32 or 64 (got %d)", g->offset_bits);
    if (g->offset_bits == 32 && g->m >= (1ll << 31)) return fail(IM_ERR_INVALID_GRAPH, "int32 offsets need m < 2^31");
    return IM_OK;
}

int64_t csr_offset_at(const im_csr* g, int64_t i) {
    if (g->offset_bits == 32) {
        int32_t v = 0;
        const int32_t* p = static_cast<const int32_t*>(g->xadj) + i;
        if (g->on_device) {
            if (hipMemcpy(&v, p, 4, hipMemcpyDeviceToHost) != hipSuccess) return -1;
        } else {
            v = *p;
        }
        return v;
    }
    int64_t v = 0;
    const int64_t* p = static_cast<const int64_t*>(g->xadj) + i;
    if (g->on_device) {
        if (hipMemcpy(&v, p, 8, hipMemcpyDeviceToHost) != hipSuccess) return -1;
    } else {
        v = *p;
    }
    return v;
}

hipError_t csr_copy_offsets(const im_csr* g, int64_t* dst, hipStream_t s) {
    const int64_t cnt = g->n + 1;
    if (g->offset_bits != 32)
        return hipMemcpyAsync(dst, g->xadj, 8 * cnt, g->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s);
    const int32_t* src = static_cast<const int32_t*>(g->xadj);
    if (g->on_device) return launch_widen_offsets(src, dst, cnt, s);
    std::vector<int64_t> wide(src, src + cnt);
    const hipError_t e = hipMemcpyAsync(dst, wide.data(), 8 * cnt, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);  // the staging vector goes out of scope
}

hipError_t csr_offsets_to_host(const im_csr* g, int64_t* dst) {
    const int64_t cnt = g->n + 1;
    if (g->offset_bits != 32)
        return hipMemcpy(dst, g->xadj, 8 * cnt, g->on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost);
    std::vector<int32_t> narrow(cnt);
    const hipError_t e =
        hipMemcpy(narrow.data(), g->xadj, 4 * cnt, g->on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost);
    if (e != hipSuccess) return e;
    for (int64_t i = 0; i < cnt; ++i) dst[i] = narrow[i];
    return hipSuccess;
}

}  // namespace hfr

namespace {

constexpr int RING = 256;         // sweeps held by the counter ring
constexpr int MAX_BATCH = 64;     // sweeps per batch
constexpr int GATHER = 6;         // counts gathered per sweep (k_gather_counts)
constexpr int DEFAULT_HEAVY = 64;
constexpr int DEFAULT_PIECE = 256;
constexpr int BFS_CHUNK = 256;
constexpr int SWEEP_TIMERS = 6 * RING;

}  // namespace

struct DevBuf {
    void* p;
    size_t bytes;
};

struct im_sketch {
    im_ctx* ctx = nullptr;
    bool poisoned = false;
    Layout L{};
    DevGraph g{};
    uint32_t seed = 0;
    double eps_c = 0.0;
    std::vector<DevBuf> bufs;
    size_t bytes = 0;

    uint32_t* X = nullptr;
    uint32_t* HJ = nullptr;
    double* T = nullptr;
    uint32_t* M[3] = {nullptr, nullptr, nullptr};
    int build_buf = 0;
    int sel_buf = 0;
    uint32_t* Lbm[3] = {nullptr, nullptr, nullptr};
    Frontier fr{};
    uint32_t* cnt_ring = nullptr;
    unsigned long long* vis_ring = nullptr;
    unsigned long long* gather = nullptr;  // device [2][GATHER * MAX_BATCH]
    uint32_t* part = nullptr;
    uint32_t* part_any = nullptr;
    uint32_t* rtouch = nullptr;
    GreedyBufs gb{};
    StepRec* d_steps = nullptr;
    int32_t* d_seeds = nullptr;
    int32_t* d_flag = nullptr;
    uint32_t* d_err = nullptr;
    unsigned long long* d_heavy_counts = nullptr;
    uint32_t stamp_ctr = 0;  // last per-sweep stamp handed out

    // pinned host staging
    unsigned long long* h_gather[2] = {nullptr, nullptr};
    uint32_t* h_small = nullptr;  // 16 words

    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    hipEvent_t ev_batch[2] = {nullptr, nullptr};
    // the reverse CSR is built on `aux` while the first (dense) sweeps run;
    // sweeps may go sparse only once ev_rev has completed
    hipStream_t aux = nullptr;
    hipEvent_t ev_indeg = nullptr, ev_rev = nullptr;
    bool rev_ready = false;
    void* rev_tmp = nullptr;  // in-degrees and cursors of the reverse CSR build
    void* list_tmp = nullptr; // a preparation temporary (per-edge weights, light-row list build)
    void* hash_tmp = nullptr; // the edge hashes, held until the edges live in no sample are flagged
    std::vector<hipEvent_t> sweep_ev;
    bool time_sweeps = false;  // sweep log recorded (either timing flag)
    bool time_all = false;     // every kernel of a sweep timed, not only the piece kernel
    bool in_place = false;  // sweeps read and write one register buffer

    // build statistics
    int sweeps = 0;
    int64_t visits = 0;
    double build_ms = 0.0, prep_ms = 0.0;
    std::vector<int64_t> trace_live, trace_vis;
    std::vector<im_sweep_rec> sweep_log;
    int32_t simulate_count = 0;
    int64_t sweep_hint = 0;  // sweeps of the last Simulate: rebuilds batch their sweeps by it
    int32_t level_id = 1;
    bool selected = false;
    // the greedy run of the last selection (steps 1..sel_K, before step sel_K's
    // rebuild decision took effect), which im_select_seeds_resume reuses or continues
    int32_t sel_K = 0;
    double sel_eps_g = 0.0, sel_eps_l = 0.0;
    std::vector<StepRec> sel_recs;
    std::vector<int32_t> sel_seeds;
    std::vector<int64_t> sel_levels;  // reach levels with work, per step
    bool has_registers = true;
};

namespace {

template <typename T>
bool sk_alloc(im_sketch* sk, T** out, size_t count) {
    size_t bytes = sizeof(T) * (count ? count : 1);
    void* p = ctx_alloc(sk->ctx, bytes);
    if (!p) return false;
    sk->bufs.push_back({p, bytes});
    sk->bytes += bytes;
    sk->ctx->in_use += bytes;
    *out = reinterpret_cast<T*>(p);
    return true;
}

void sk_release(im_sketch* sk) {
    if (!sk) return;
    if (sk->aux) (void)hipStreamSynchronize(sk->aux);  // the reverse CSR build writes sketch buffers
    if (sk->ctx) {
        (void)hipStreamSynchronize(sk->ctx->stream);
        for (auto& b : sk->bufs) {
            ctx_free(sk->ctx, b.p);
            sk->ctx->in_use -= b.bytes;
        }
    }
    sk->bufs.clear();
    if (sk->h_gather[0]) (void)hipHostFree(sk->h_gather[0]);
    if (sk->h_gather[1]) (void)hipHostFree(sk->h_gather[1]);
    if (sk->h_small) (void)hipHostFree(sk->h_small);
    if (sk->rev_tmp && sk->ctx) ctx_free(sk->ctx, sk->rev_tmp);
    if (sk->list_tmp && sk->ctx) ctx_free(sk->ctx, sk->list_tmp);
    if (sk->hash_tmp && sk->ctx) ctx_free(sk->ctx, sk->hash_tmp);
    for (hipEvent_t e : {sk->ev_a, sk->ev_b, sk->ev_batch[0], sk->ev_batch[1], sk->ev_indeg, sk->ev_rev})
        if (e) (void)hipEventDestroy(e);
    if (sk->aux) (void)hipStreamDestroy(sk->aux);
    for (hipEvent_t e : sk->sweep_ev) (void)hipEventDestroy(e);
    delete sk;
}

#define HIP_TRY(expr)                                                                                 \
    do {                                                                                              \
        hipError_t _e = (expr);                                                                       \
        if (_e != hipSuccess) {                                                                       \
            if (sk) sk->poisoned = true;                                                              \
            return fail(IM_ERR_DEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, \
                        __LINE__);                                                                    \
        }                                                                                             \
    } while (0)

struct Sizes {
    int64_t n, m, J;
    size_t total;
};

// a level's entries (each vertex once, in chunks of BFS_CHUNK out-edges), plus the
// slots the waves of a reach level may reserve and leave unfilled
int64_t qcap_for(int64_t n, int64_t m) {
    return n + (m + BFS_CHUNK - 1) / BFS_CHUNK + 64 + (int64_t)BFS_WAVES * BFS_RESV;
}

size_t bytes_needed(int64_t n, int64_t m, int32_t R, im_prob_kind kind) {
    const Layout L = make_layout(R);
    auto al = [](size_t b) { return (std::max<size_t>(b, 1) + 255) & ~size_t(255); };
    size_t t = 0;
    t += al(8 * (n + 1)) + al(4 * m) + al(4 * m);  // xadj, adj, edge hashes
    t += al(8 * (n + 1)) + 2 * al(4 * m) + 2 * al(4 * n);  // reverse CSR with pieces, heavy slots, light rows
    t += al(4 * ((n + 31) / 32 + 1)) + al(8 * (n + m / 256 + 64)) + al(4 * n) + al(32);  // sparse marks, lists
    t += al(4 * COARSE_WORDS);                                                          // coarse L_t
    if (kind == IM_PROB_WEIGHTED_CASCADE) t += al(4 * n) + al(4 * m);  // per target, then per edge
    if (kind == IM_PROB_PER_EDGE) t += al(4 * m);
    t += al(4 * R) * 2 + al(8 * R);               // X, HJ, T
    t += 3 * al((size_t)n * L.P * 4);             // register buffers
    const int64_t words = (n + 31) / 32 + 1;
    t += 3 * al(4 * words);
    t += al((size_t)RING * NSLOT * SLOT_U32 * 4) + al((size_t)3 * RING * NSLOT * SLOT_U64 * 8) + al(16 * GATHER * MAX_BATCH);
    // split rows: bounded by m / heavy_degree rows and m / piece + rows pieces
    const int64_t nh = m / DEFAULT_HEAVY + 1, np = m / DEFAULT_PIECE + nh + 1;
    t += al(4 * nh) + al(8 * (nh + 1)) + al(8 * nh) + al(4 * np) + 2 * al(8 * np) + al((size_t)np * L.P * 4) +
         al(4 * np) + al(4 * nh) + al(4 * np);
    // greedy
    const size_t W = 4 * (size_t)L.PW;
    t += 3 * al((size_t)n * W * 4) + al(4 * words);
    t += 2 * al(8 * qcap_for(n, m)) + al(64) + al(4 * n) + al(n) + 2 * al(4 * L.P) + al(8) +
         al(NSLOT * SLOT_U64 * 8) + al(8);
    t += al(sizeof(StepRec) * 64) + al(4 * 64) + al(16) + al(16) + al(64);
    // preparation temporaries: the light-row list's, and the reverse CSR's
    const int64_t nb = (n + 1023) / 1024;
    const size_t list_tmp = al(4 * n) + al(8 * (n + 1)) + al(8 * (nb + 2));
    t += list_tmp + (rb_fits(n, m) ? rb_temp_bytes(n, m) : list_tmp);
    return t;
}

// Sums of the live-count slots of sweeps [t0+1, t0+nb], of the row-kernel
// and split-row-kernel visit slots and of S_t for sweeps [t0, t0+nb-1] into
// out[GATHER i .. GATHER i + 3], and of the rows merged by the two kernels
// (word 1 of their visit slots) into out[GATHER i + 4], out[GATHER i + 5].
// The visit ring holds RING row-kernel entries followed by RING split-row ones.
__global__ void k_gather_counts(const uint32_t* __restrict__ cnt, const unsigned long long* __restrict__ vis,
                                int64_t t0, int nb, unsigned long long* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const uint32_t* c = cnt + ((t0 + i + 1) % RING) * NSLOT * SLOT_U32;
    const unsigned long long* v = vis + ((t0 + i) % RING) * NSLOT * SLOT_U64;
    const unsigned long long* vh = v + (size_t)RING * NSLOT * SLOT_U64;
    const unsigned long long* sm = vis + (2 * (size_t)RING + (t0 + i) % RING) * NSLOT * SLOT_U64;
    unsigned long long sc = 0, sv = 0, sh = 0, ss = 0, mv = 0, mh = 0;
    for (int k = 0; k < NSLOT; ++k) {
        sc += c[k * SLOT_U32];
        sv += v[k * SLOT_U64];
        sh += vh[k * SLOT_U64];
        ss += sm[k * SLOT_U64];
        mv += v[k * SLOT_U64 + 1];
        mh += vh[k * SLOT_U64 + 1];
    }
    unsigned long long* o = out + GATHER * i;
    o[0] = sc;
    o[1] = sv;
    o[2] = sh;
    o[3] = ss;  // S_t, the in-degree sum of L_t (0 for t = 0)
    o[4] = mv;
    o[5] = mh;
}

// Zeroes the live-count slots of sweeps [t0+1, t0+nb] and the visit slots of
// sweeps [t0, t0+nb-1].
__global__ void k_ring_zero(uint32_t* cnt, unsigned long long* vis, int64_t t0, int nb) {
    const int i = blockIdx.x;  // sweep offset
    if (i >= nb) return;
    uint32_t* c = cnt + ((t0 + i + 1) % RING) * NSLOT * SLOT_U32;
    unsigned long long* v = vis + ((t0 + i) % RING) * NSLOT * SLOT_U64;
    unsigned long long* vh = v + (size_t)RING * NSLOT * SLOT_U64;
    unsigned long long* sm = vis + (2 * (size_t)RING + (t0 + i + 1) % RING) * NSLOT * SLOT_U64;
    for (int k = threadIdx.x; k < NSLOT * SLOT_U32; k += blockDim.x) c[k] = 0u;
    for (int k = threadIdx.x; k < NSLOT * SLOT_U64; k += blockDim.x) {
        v[k] = 0ull;
        vh[k] = 0ull;
        sm[k] = 0ull;
    }
}

uint32_t* cnt_slots(im_sketch* sk, int64_t t) { return sk->cnt_ring + (t % RING) * NSLOT * SLOT_U32; }
unsigned long long* vis_slots(im_sketch* sk, int64_t t) { return sk->vis_ring + (t % RING) * NSLOT * SLOT_U64; }
unsigned long long* vis_heavy_slots(im_sketch* sk, int64_t t) {
    return sk->vis_ring + (RING + t % RING) * NSLOT * SLOT_U64;
}
// S_t: sum of the in-degrees of L_t, produced by sweep t-1
unsigned long long* sum_slots(im_sketch* sk, int64_t t) {
    return sk->vis_ring + (2 * RING + t % RING) * NSLOT * SLOT_U64;
}

struct SimResult {
    int buf;
    int sweeps;
    int64_t visits;
    double ms;
    std::vector<int64_t> live, vis, vis_light, mrg, mrg_light;  // mrg: rows merged
    std::vector<char> sparse;
};

// Runs the multi-sample reach BFS from the level-0 queue (qsize[0] entries,
// frontier bits in F[0]) until a level finds nothing new.  Levels are launched
// in growing batches; the host reads the queue sizes after each batch.
// *levels: levels launched; *with_work += levels that had entries.
im_status run_reach(im_sketch* sk, int32_t lvl0, int* levels, int64_t* with_work) {
    hipStream_t s = sk->ctx->stream;
    const int64_t n = sk->g.n;
    GreedyBufs& b = sk->gb;
    int level = 0, nb = 4;
    while (true) {
        const int64_t bfs_grid = BFS_GRID;
        for (int i = 0; i < nb; ++i, ++level)
            HIP_TRY(launch_bfs_level(sk->L, sk->g, sk->X, b, level, lvl0 + level + 1, (int)bfs_grid, s));
        HIP_TRY(hipMemcpyAsync(sk->h_small, b.qsize, 16, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if ((sk->h_small[0] | sk->h_small[1] | sk->h_small[2]) == 0u) break;
        if (level > n + 2) {
            sk->poisoned = true;
            return fail(IM_ERR_DEVICE, "reach search exceeded n levels");
        }
        nb = std::min(nb * 2, 64);
    }
    *levels = level;
    *with_work += sk->h_small[3];
    return IM_OK;
}

// True once the reverse CSR built on the aux stream is complete (then the
// context stream is ordered after it and its temporaries are freed); with
// wait, blocks until it is.
hipError_t rev_csr_ready(im_sketch* sk, bool wait) {
    if (sk->rev_ready) return hipSuccess;
    hipError_t e = wait ? hipEventSynchronize(sk->ev_rev) : hipEventQuery(sk->ev_rev);
    if (e == hipErrorNotReady) return hipSuccess;
    if (e != hipSuccess) return e;
    e = hipStreamWaitEvent(sk->ctx->stream, sk->ev_rev, 0);
    if (e != hipSuccess) return e;
    ctx_free(sk->ctx, sk->rev_tmp);
    sk->rev_tmp = nullptr;
    sk->rev_ready = true;
    return hipSuccess;
}

// Simulate (Alg. 2) on buffers ia/ib: init (with blocked pairs if blk), then
// synchronous sweeps until |L_t| <= floor(eps_c * n).
im_status run_simulate(im_sketch* sk, int ia, int ib, const uint32_t* blk, SimResult* res) {
    hipStream_t s = sk->ctx->stream;
    const int64_t n = sk->g.n;
    // synchronous sweeps alternate two buffers; in-place sweeps use one for both
    // (the copy rule then rewrites a row with its own values)
    if (sk->in_place) ib = ia;
    uint32_t* buf[2] = {sk->M[ia], sk->M[ib]};
    const double lim = floor(sk->eps_c * (double)n);
    const uint32_t thresh = lim >= (double)n ? (uint32_t)n : (uint32_t)lim;
    res->live.assign(1, n);
    res->vis.clear();
    res->vis_light.clear();
    res->sparse.clear();
    const int32_t sim_id = sk->simulate_count++;
    HIP_TRY(hipEventRecord(sk->ev_a, s));
    HIP_TRY(launch_init(sk->L, n, sk->HJ, sk->seed, blk, buf[0], buf[1], s));
    if (blk) HIP_TRY(launch_full_blocked(sk->L, n, blk, sk->gb.fullblk, s));
    // the row kernel sets L_{t+1} bits with atomics: every bitmap starts zeroed
    for (int i = 0; i < 3; ++i) HIP_TRY(launch_fill_u32(sk->Lbm[i], 0u, (n + 31) / 32 + 1, s));
    HIP_TRY(launch_fill_u32(sk->fr.mark, 0u, (n + 31) / 32 + 1, s));
    HIP_TRY(launch_fill_u32(sk->fr.counts, 0u, 8, s));
    int final_sweeps = -1;
    if ((uint64_t)n <= thresh) final_sweeps = 0;
    int64_t t = 0;
    int nb = 8;
    // sweeps are launched in growing batches, two in flight, before the host sees
    // where the fixed point falls; the sweeps past it return at once.  A rebuild
    // converges in about as many sweeps as the Simulate before it, so below that
    // count (less a margin) batches run at full size, and past it they restart at 4
    const int64_t hint_safe = sk->sweep_hint > 0 ? sk->sweep_hint - 8 : 0;
    bool tail = false;
    int inflight = 0;  // batches launched and not yet read
    int64_t batch_t0[2] = {0, 0};
    int batch_nb[2] = {0, 0};
    int batch_slot = 0;
    int timer_idx = 0;
    std::vector<int> timer_of_sweep;
    std::vector<bool> sparse_ok;  // per launched sweep: sparse mode allowed
    while (final_sweeps < 0) {
        // synchronous sweeps reach the fixed point within n + 1 sweeps
        if (t > n + 2 + 2 * MAX_BATCH) {
            sk->poisoned = true;
            return fail(IM_ERR_DEVICE, "sweep count exceeded n + 1 without convergence");
        }
        if (hint_safe > 0) {
            if (t < hint_safe)
                nb = (int)std::min<int64_t>(nb, hint_safe - t);
            else if (!tail) {
                tail = true;
                nb = 4;
            }
        }
        // launch one batch; its sweeps may go sparse only once the reverse CSR exists
        HIP_TRY(rev_csr_ready(sk, false));
        const bool may_sparse = sk->rev_ready;
        hipLaunchKernelGGL(k_ring_zero, dim3(nb), dim3(256), 0, s, sk->cnt_ring, sk->vis_ring, t, nb);
        HIP_TRY(hipGetLastError());
        for (int64_t st = t; st < t + nb; ++st) {
            SweepParams sp{};
            sp.A = buf[st & 1];
            sp.B = buf[(st + 1) & 1];
            sp.Lcur = sk->Lbm[st % 3];
            sp.Lnext = sk->Lbm[(st + 1) % 3];
            sp.Lclear = sk->Lbm[(st + 2) % 3];
            sp.fr = sk->fr;
            if (!may_sparse) sp.fr.sparse_div = 0;
            sparse_ok.push_back(may_sparse);
            // piece flags of earlier sweeps never equal this sweep's stamp
            if (++sk->stamp_ctr == 0u) {
                if (sk->g.npieces > 0) HIP_TRY(launch_fill_u32(sk->part_any, 0u, sk->g.npieces, s));
                if (sk->g.nheavy > 0) HIP_TRY(launch_fill_u32(sk->rtouch, 0u, sk->g.nheavy, s));
                sk->stamp_ctr = 1u;
            }
            sp.fr.stamp = sk->stamp_ctr;
            sp.fullblk = blk ? sk->gb.fullblk : nullptr;
            sp.parity = (int)(st & 1);
            sp.blk = blk;
            sp.gate = st == 0 ? nullptr : cnt_slots(sk, st);
            sp.gate_thresh = thresh;
            sp.cnt_out = cnt_slots(sk, st + 1);
            sp.vis_out = vis_slots(sk, st);
            sp.vis_heavy_out = vis_heavy_slots(sk, st);
            sp.sgate = st == 0 ? nullptr : sum_slots(sk, st);
            sp.sum_out = sum_slots(sk, st + 1);
            sp.part = sk->part;
            sp.part_any = sk->part_any;
            sp.rtouch = sk->rtouch;
            sp.first = st == 0;
            hipEvent_t e0 = nullptr, e1 = nullptr, ea = nullptr, eb = nullptr, e2 = nullptr, e3 = nullptr;
            if (sk->time_sweeps && timer_idx + 5 < (int)sk->sweep_ev.size()) {
                if (sk->time_all) {
                    e0 = sk->sweep_ev[timer_idx];
                    e1 = sk->sweep_ev[timer_idx + 1];
                    ea = sk->sweep_ev[timer_idx + 2];
                    eb = sk->sweep_ev[timer_idx + 3];
                }
                e2 = sk->sweep_ev[timer_idx + 4];
                e3 = sk->sweep_ev[timer_idx + 5];
                timer_idx += 6;
            }
            if (ea) HIP_TRY(hipEventRecord(ea, s));
            HIP_TRY(launch_sweep(sk->L, sk->g, sk->X, sp, 0, s, e0, e1, e2, e3));
            if (eb) HIP_TRY(hipEventRecord(eb, s));
        }
        hipLaunchKernelGGL(k_gather_counts, dim3(1), dim3(64), 0, s, sk->cnt_ring, sk->vis_ring, t, nb,
                           sk->gather + GATHER * MAX_BATCH * batch_slot);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(sk->h_gather[batch_slot], sk->gather + GATHER * MAX_BATCH * batch_slot,
                               sizeof(unsigned long long) * GATHER * nb, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipEventRecord(sk->ev_batch[batch_slot], s));
        batch_t0[batch_slot] = t;
        batch_nb[batch_slot] = nb;
        batch_slot ^= 1;
        ++inflight;
        t += nb;
        nb = std::min(nb * 2, MAX_BATCH);
        if (inflight < 2) continue;
        // read the older batch
        const int rs = batch_slot;  // older slot (the one launched first)
        HIP_TRY(hipEventSynchronize(sk->ev_batch[rs]));
        --inflight;
        for (int i = 0; i < batch_nb[rs]; ++i) {
            const unsigned long long* gi = sk->h_gather[rs] + GATHER * i;
            const int64_t live = (int64_t)gi[0];
            const int64_t vis_l = (int64_t)gi[1];
            const int64_t vis = vis_l + (int64_t)gi[2];
            const int64_t st_sum = (int64_t)gi[3];
            res->mrg_light.push_back((int64_t)gi[4]);
            res->mrg.push_back((int64_t)(gi[4] + gi[5]));
            const int64_t tt = batch_t0[rs] + i;
            res->vis.push_back(vis);
            res->vis_light.push_back(vis_l);
            res->sparse.push_back(tt > 0 && sparse_ok[tt] && sk->fr.sparse_div != 0 &&
                                  (uint64_t)st_sum * sk->fr.sparse_div <= (uint64_t)sk->g.m);
            res->live.push_back(live);
            if ((uint64_t)live <= thresh) {
                final_sweeps = (int)(batch_t0[rs] + i + 1);
                break;
            }
        }
    }
    HIP_TRY(hipEventRecord(sk->ev_b, s));
    HIP_TRY(hipStreamSynchronize(s));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, sk->ev_a, sk->ev_b));
    res->ms = ms;
    res->sweeps = final_sweeps;
    sk->sweep_hint = final_sweeps;
    res->live.resize(final_sweeps + 1);
    res->vis.resize(final_sweeps);
    res->vis_light.resize(final_sweeps);
    res->mrg.resize(final_sweeps);
    res->mrg_light.resize(final_sweeps);
    res->sparse.resize(final_sweeps);
    res->visits = 0;
    for (int64_t v : res->vis) res->visits += v;
    res->buf = (final_sweeps & 1) ? ib : ia;
    if (sk->time_sweeps) {
        // every timed launch of the row kernel, including the ones past the
        // stopping rule that returned at once
        for (int i = 0; i + 5 < timer_idx; i += 6) {
            float km = 0.f, wm = 0.f, hm = 0.f;
            if (sk->time_all) {
                HIP_TRY(hipEventElapsedTime(&km, sk->sweep_ev[i], sk->sweep_ev[i + 1]));
                HIP_TRY(hipEventElapsedTime(&wm, sk->sweep_ev[i + 2], sk->sweep_ev[i + 3]));
            }
            HIP_TRY(hipEventElapsedTime(&hm, sk->sweep_ev[i + 4], sk->sweep_ev[i + 5]));
            const int t = i / 6;
            im_sweep_rec rec{};
            rec.simulate = sim_id;
            rec.sweep = t;
            rec.ran = t < final_sweeps;
            rec.kernel_ms = km;
            rec.sweep_ms = wm;
            rec.heavy_ms = hm;
            if (rec.ran) {
                rec.light_visits = res->vis_light[t];
                rec.visits = res->vis[t];
                rec.light_merged = res->mrg_light[t];
                rec.merged = res->mrg[t];
                rec.live = res->live[t];
                rec.live_next = res->live[t + 1];
                rec.sparse = res->sparse[t];
            }
            sk->sweep_log.push_back(rec);
        }
    }
    return IM_OK;
}

im_status check_sketch(const im_sketch* sk) {
    if (!sk) return fail(IM_ERR_INVALID_ARG, "null sketch");
    if (sk->poisoned) return fail(IM_ERR_STATE, "sketch is poisoned by an earlier device error");
    return IM_OK;
}

}  // namespace

namespace hfr {

void sketch_rebind(im_sketch* sk, im_ctx* ctx) {
    if (!sk || !ctx || sk->ctx == ctx) return;
    sk->ctx->in_use -= sk->bytes;
    ctx->in_use += sk->bytes;
    sk->ctx = ctx;
}

}  // namespace hfr

extern "C" {

const char* im_last_error(void) { return hfr::g_last_error.c_str(); }

const char* im_version(void) { return "hipfuser 0.1 (gfx950)"; }

im_status im_ctx_create(int32_t device, void* stream, size_t hbm_budget, im_alloc_fn alloc, im_free_fn dealloc,
                        void* user, im_ctx** out) {
    im_sketch* sk = nullptr;
    if (!out) return fail(IM_ERR_INVALID_ARG, "out is null");
    if ((alloc == nullptr) != (dealloc == nullptr)) return fail(IM_ERR_INVALID_ARG, "alloc and dealloc must both be set");
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(IM_ERR_INVALID_ARG, "device %d out of range (%d devices)", device, ndev);
    HIP_TRY(hipSetDevice(device));
    {
        const im_status st = init_scratch(device);
        if (st != IM_OK) return st;
    }
    im_ctx* c = new im_ctx;
    c->device = device;
    c->stream = (hipStream_t)stream;
    c->budget = hbm_budget;
    c->af = alloc;
    c->ff = dealloc;
    c->user = user;
    *out = c;
    return IM_OK;
}

void im_ctx_free(im_ctx* ctx) { delete ctx; }

size_t im_ctx_bytes_in_use(const im_ctx* ctx) { return ctx ? ctx->in_use.load() : 0; }

size_t im_sketch_bytes_needed(int64_t n, int64_t m, int32_t R, im_prob_kind kind) {
    if (n < 1 || m < 0 || R < 4 || R > 1024 || R % 4) return 0;
    return bytes_needed(n, m, R, kind);
}

}  // extern "C"

namespace {

// Builds a sketch (graph copy, hashes, thresholds, split rows, reverse CSR,
// greedy buffers) and, with `simulate`, its registers (Alg. 2).  Without
// `simulate` no register buffer is allocated: the handle serves Monte-Carlo
// reach only.
im_status build_sketch(im_ctx* ctx, const im_csr* graph, const im_probs* probs, int32_t R, uint32_t hash_seed,
                       const im_build_opts* opts, bool simulate, im_sketch** out) {
    im_sketch* sk = nullptr;
    if (!ctx || !graph || !probs || !out) return fail(IM_ERR_INVALID_ARG, "null argument");
    if (R < 4 || R > 1024 || R % 4) return fail(IM_ERR_INVALID_ARG, "R must be a multiple of 4 in [4, 1024] (got %d)", R);
    const int64_t n = graph->n, m = graph->m;
    if (n < 1 || n >= (1ll << 31)) return fail(IM_ERR_INVALID_GRAPH, "n must be in [1, 2^31) (got %lld)", (long long)n);
    if (m < 0 || m >= (1ll << 40)) return fail(IM_ERR_INVALID_GRAPH, "m out of range (got %lld)", (long long)m);
    if (!graph->xadj || (m > 0 && !graph->adj)) return fail(IM_ERR_INVALID_GRAPH, "null CSR array");
    if (const im_status oc = csr_offsets_check(graph); oc != IM_OK) return oc;
    if (probs->kind != IM_PROB_CONSTANT && probs->kind != IM_PROB_WEIGHTED_CASCADE && probs->kind != IM_PROB_PER_EDGE)
        return fail(IM_ERR_INVALID_ARG, "unknown probability kind %d", (int)probs->kind);
    if (probs->kind == IM_PROB_CONSTANT && live_threshold(probs->p) == 0xFFFFFFFFu)
        return fail(IM_ERR_INVALID_ARG, "probability must be in [0, 1]");
    if (probs->kind == IM_PROB_PER_EDGE && m > 0 && !probs->per_edge)
        return fail(IM_ERR_INVALID_ARG, "per-edge probabilities missing");
    im_build_opts o{};
    if (opts) o = *opts;
    if (!(o.eps_c >= 0.0)) return fail(IM_ERR_INVALID_ARG, "eps_c must be >= 0");
    if (o.heavy_degree < 0 || o.piece_edges < 0) return fail(IM_ERR_INVALID_ARG, "negative tuning value");
    if (o.piece_edges > 2048) return fail(IM_ERR_INVALID_ARG, "piece_edges must be at most 2048");
    if (o.flags & ~(IM_BUILD_TIME_SWEEPS | IM_BUILD_IN_PLACE | IM_BUILD_ATOMIC_REVERSE | IM_BUILD_TIME_PIECES))
        return fail(IM_ERR_INVALID_ARG, "unknown build flag");
    const size_t need = bytes_needed(n, m, R, probs->kind);
    if (ctx->budget && ctx->in_use + need > ctx->budget)
        return fail(IM_ERR_OUT_OF_BUDGET, "sketch needs %zu bytes, %zu of %zu in use", need, ctx->in_use.load(), ctx->budget);

    hipStream_t s = ctx->stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(IM_ERR_DEVICE, "hipSetDevice failed");

    // host-side offset checks that need no device pass
    const int64_t x0 = csr_offset_at(graph, 0), xn = csr_offset_at(graph, n);
    if (graph->on_device && (x0 < 0 || xn < 0) && hipGetLastError() != hipSuccess)
        return fail(IM_ERR_DEVICE, "reading device xadj failed");
    if (x0 != 0 || xn != m) return fail(IM_ERR_INVALID_GRAPH, "xadj[0] must be 0 and xadj[n] must equal m");

    sk = new im_sketch;
    sk->ctx = ctx;
    sk->L = make_layout(R);
    sk->seed = hash_seed;
    sk->eps_c = o.eps_c;
    sk->time_all = (o.flags & IM_BUILD_TIME_SWEEPS) != 0;
    sk->time_sweeps = sk->time_all || (o.flags & IM_BUILD_TIME_PIECES) != 0;
    sk->in_place = (o.flags & IM_BUILD_IN_PLACE) != 0;
    DevGraph& g = sk->g;
    g.n = n;
    g.m = m;
    const Layout& L = sk->L;
    bool ok = true;
    ok = ok && sk_alloc(sk, &g.xadj, n + 1) && sk_alloc(sk, &g.adj, m);
    // the edge hashes are a preparation temporary: once the edges live in no sample are
    // flagged, every kernel recomputes the hash of (u, v) instead of loading it
    g.hseed = hash_seed;
    ok = ok && (sk->hash_tmp = ctx_alloc(ctx, 4 * (size_t)(m > 0 ? m : 1))) != nullptr;
    g.eh = (uint32_t*)sk->hash_tmp;
    ok = ok && sk_alloc(sk, &sk->X, R) && sk_alloc(sk, &sk->HJ, R) && sk_alloc(sk, &sk->T, R);
    for (int i = 0; i < 3 && ok && simulate; ++i) ok = sk_alloc(sk, &sk->M[i], (size_t)n * L.P);
    const int64_t words = (n + 31) / 32 + 1;
    ok = ok && sk_alloc(sk, &sk->Lbm[0], words) && sk_alloc(sk, &sk->Lbm[1], words) &&
         sk_alloc(sk, &sk->Lbm[2], words);
    ok = ok && sk_alloc(sk, &g.rxadj, n + 1) && sk_alloc(sk, &g.rrec, m) &&
         sk_alloc(sk, &g.hslot, n) && sk_alloc(sk, &g.lrows, n);
    ok = ok && sk_alloc(sk, &sk->fr.mark, words) && sk_alloc(sk, &sk->fr.items, n + m / 256 + 64) &&
         sk_alloc(sk, &sk->fr.W, n) && sk_alloc(sk, &sk->fr.counts, 8);
    ok = ok && sk_alloc(sk, &sk->cnt_ring, (size_t)RING * NSLOT * SLOT_U32) &&
         sk_alloc(sk, &sk->vis_ring, (size_t)3 * RING * NSLOT * SLOT_U64) && sk_alloc(sk, &sk->gather, 2 * GATHER * MAX_BATCH);
    ok = ok && sk_alloc(sk, &sk->d_err, 4) && sk_alloc(sk, &sk->d_heavy_counts, 4) && sk_alloc(sk, &sk->d_flag, 4);
    sk->fr.chunk = 256;
    sk->fr.sparse_div = o.sparse_div < 0 ? 0u : (o.sparse_div == 0 ? 8u : (uint32_t)o.sparse_div);
    {
        // coarse copy of L_t: at least 256 vertices per bit, at most COARSE_WORDS
        // words; used by the one-row-per-wave kernels while at most half of its
        // bits (or 64 of them, on small graphs) can be set
        int cs = 8;
        while (((n - 1) >> (cs + 5)) + 1 > COARSE_WORDS) ++cs;
        sk->fr.coarse_shift = cs;
        sk->fr.coarse_words = (int32_t)(((n - 1) >> (cs + 5)) + 1);
        const uint32_t cbits = (uint32_t)(((n - 1) >> cs) + 1);
        sk->fr.coarse_live = L.G == 64 ? std::max(cbits / 2u, 64u) : 0u;
        ok = ok && sk_alloc(sk, &sk->fr.coarse, sk->fr.coarse_words);
    }
    uint32_t* wc_target = nullptr;
    if (probs->kind == IM_PROB_WEIGHTED_CASCADE) ok = ok && sk_alloc(sk, &wc_target, n) && sk_alloc(sk, &g.thr, m);
    if (probs->kind == IM_PROB_PER_EDGE) ok = ok && sk_alloc(sk, &g.thr, m);
    if (!ok) {
        sk_release(sk);
        return fail(IM_ERR_OUT_OF_BUDGET, "device allocation failed");
    }
    if (hipHostMalloc((void**)&sk->h_gather[0], 8 * GATHER * MAX_BATCH) != hipSuccess ||
        hipHostMalloc((void**)&sk->h_gather[1], 8 * GATHER * MAX_BATCH) != hipSuccess ||
        hipHostMalloc((void**)&sk->h_small, 64) != hipSuccess) {
        sk_release(sk);
        return fail(IM_ERR_DEVICE, "pinned host allocation failed");
    }
    if (hipEventCreate(&sk->ev_a) != hipSuccess || hipEventCreate(&sk->ev_b) != hipSuccess ||
        hipEventCreate(&sk->ev_batch[0]) != hipSuccess || hipEventCreate(&sk->ev_batch[1]) != hipSuccess ||
        hipEventCreateWithFlags(&sk->ev_indeg, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&sk->ev_rev, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&sk->aux, hipStreamNonBlocking) != hipSuccess) {
        sk_release(sk);
        return fail(IM_ERR_DEVICE, "event creation failed");
    }
    if (sk->time_sweeps) {
        sk->sweep_ev.resize(SWEEP_TIMERS);
        for (auto& e : sk->sweep_ev)
            if (hipEventCreate(&e) != hipSuccess) {
                sk_release(sk);
                return fail(IM_ERR_DEVICE, "event creation failed");
            }
    }

    im_status st = IM_OK;
    auto body = [&]() -> im_status {
        const hipMemcpyKind kind = graph->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        HIP_TRY(hipEventRecord(sk->ev_a, s));
        HIP_TRY(csr_copy_offsets(graph, g.xadj, s));
        if (m > 0) HIP_TRY(hipMemcpyAsync(g.adj, graph->adj, 4 * m, kind, s));
        HIP_TRY(launch_fill_u32(sk->d_err, 0u, 1, s));
        HIP_TRY(launch_validate(g, sk->d_err, s));
        HIP_TRY(hipMemcpyAsync(sk->h_small, sk->d_err, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (sk->h_small[0] & 1u) return fail(IM_ERR_INVALID_GRAPH, "xadj is not nondecreasing");
        if (sk->h_small[0] & 2u) return fail(IM_ERR_INVALID_GRAPH, "adj holds an id outside [0, n)");

        HIP_TRY(launch_sim_words(sk->X, sk->HJ, R, hash_seed, s));
        // exp2(r/J) table for the estimate (host libm), uploaded once
        std::vector<double> T(R);
        for (int r = 0; r < R; ++r) T[r] = exp2((double)r / (double)R);
        HIP_TRY(hipMemcpyAsync(sk->T, T.data(), 8 * R, hipMemcpyHostToDevice, s));
        if (probs->kind == IM_PROB_CONSTANT) {
            g.kind = THR_CONST;
            g.thr_const = live_threshold(probs->p);
        } else if (probs->kind == IM_PROB_WEIGHTED_CASCADE) {
            g.kind = THR_TARGET;
        } else {
            g.kind = THR_EDGE;
            if (m > 0) {
                const float* w = probs->per_edge;
                void* tmp = nullptr;
                if (!graph->on_device) {
                    tmp = sk->list_tmp = ctx_alloc(ctx, 4 * m);  // released with the sketch on error
                    if (!tmp) return fail(IM_ERR_OUT_OF_BUDGET, "temporary allocation failed");
                    HIP_TRY(hipMemcpyAsync(tmp, probs->per_edge, 4 * m, hipMemcpyHostToDevice, s));
                    w = (const float*)tmp;
                }
                HIP_TRY(launch_fill_u32(sk->d_err, 0u, 1, s));
                HIP_TRY(launch_edge_thresholds(w, g.thr, m, sk->d_err, s));
                HIP_TRY(hipMemcpyAsync(sk->h_small, sk->d_err, 4, hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
                if (tmp) {
                    ctx_free(ctx, tmp);
                    sk->list_tmp = nullptr;
                }
                if (sk->h_small[0] & 4u) return fail(IM_ERR_INVALID_ARG, "a per-edge probability is outside [0, 1]");
            }
        }
        // split rows
        const int64_t heavy = o.heavy_degree > 0 ? o.heavy_degree : DEFAULT_HEAVY;
        const int64_t piece = o.piece_edges > 0 ? o.piece_edges : DEFAULT_PIECE;
        g.heavy_deg = heavy;
        g.piece_edges = piece;
        HIP_TRY(hipMemsetAsync(sk->d_heavy_counts, 0, 32, s));
        HIP_TRY(launch_heavy_count(g, piece, sk->d_heavy_counts, s));
        unsigned long long hc[2] = {0, 0};
        HIP_TRY(hipMemcpyAsync(hc, sk->d_heavy_counts, 16, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        g.nheavy = (int64_t)hc[0];
        g.npieces = (int64_t)hc[1];
        // the reverse CSR names the 64-edge windows of the pieces with int32
        if (g.npieces * ((piece + 63) / 64) >= (1ll << 31))
            return fail(IM_ERR_INVALID_GRAPH, "too many split-row windows (%lld pieces)", (long long)g.npieces);
        if (g.nheavy > 0) {
            bool ok2 = sk_alloc(sk, &g.hrow, g.nheavy) && sk_alloc(sk, &g.hpb, g.nheavy) &&
                       sk_alloc(sk, &g.hpn, g.nheavy) && sk_alloc(sk, &g.prow, g.npieces) &&
                       sk_alloc(sk, &g.pe0, g.npieces) && sk_alloc(sk, &g.pe1, g.npieces) &&
                       sk_alloc(sk, &sk->part, (size_t)g.npieces * L.P) && sk_alloc(sk, &sk->part_any, g.npieces) &&
                       sk_alloc(sk, &sk->rtouch, g.nheavy);
            if (!ok2) return fail(IM_ERR_OUT_OF_BUDGET, "device allocation failed (split rows)");
            HIP_TRY(launch_heavy_assign(g, piece, sk->d_heavy_counts, s));
            HIP_TRY(launch_heavy_pieces(g, piece, s));
            if (!sk_alloc(sk, &sk->fr.wmask, g.npieces))
                return fail(IM_ERR_OUT_OF_BUDGET, "device allocation failed (sparse lists)");
            HIP_TRY(launch_fill_u32(sk->part_any, 0u, g.npieces, s));
            HIP_TRY(launch_fill_u32(sk->rtouch, 0u, g.nheavy, s));
            HIP_TRY(launch_fill_u32(sk->fr.wmask, 0u, g.npieces, s));
        }
        HIP_TRY(launch_heavy_slots(g, s));
        HIP_TRY(launch_edge_hash(g, hash_seed, s));  // split rows are hashed by piece
        // in-degrees (weighted-cascade thresholds) and the reverse CSR, whose
        // in-edges carry the 64-edge window of their split source row's piece
        {
            const int64_t nb = (n + 1023) / 1024;
            const size_t a4n = (4 * n + 255) & ~size_t(255), a8n = (8 * (n + 1) + 255) & ~size_t(255);
            const size_t asc = (8 * (nb + 2) + 255) & ~size_t(255);
            // main: flags, positions and scan sums of the light-row list
            // (held by the sketch, so that an error on the way releases it too)
            void* pm_ = sk->list_tmp = ctx_alloc(ctx, a4n + a8n + asc);
            // in-degrees and the reverse CSR's temporaries (freed below when the
            // reverse CSR is built on this stream, else once the aux stream is done)
            const bool one_stream = rb_fits(n, m) && !(o.flags & IM_BUILD_ATOMIC_REVERSE);
            sk->rev_tmp = ctx_alloc(ctx, one_stream ? rb_temp_bytes(n, m) : a4n + a8n + asc);
            if (!pm_ || !sk->rev_tmp) return fail(IM_ERR_OUT_OF_BUDGET, "temporary allocation failed");
            uint32_t* indeg = nullptr;
            if (one_stream) {
                // a counting sort on the target, with LDS counters only; its records of
                // edges live in no sample are flagged as they are placed (the thresholds of
                // constant p and of the weighted cascade depend on the target only)
                DeadTest dt{sk->X, R, hash_seed, g.thr_const,
                            probs->kind == IM_PROB_CONSTANT ? 1 : (probs->kind == IM_PROB_WEIGHTED_CASCADE ? 2 : 0)};
                HIP_TRY(launch_reverse_csr_buckets(g, sk->rev_tmp, &indeg, dt, s));
            } else {
                // global atomics, the scatter on the aux stream beside the sweeps
                indeg = (uint32_t*)sk->rev_tmp;
                int64_t* cursor = (int64_t*)((char*)sk->rev_tmp + a4n);
                uint32_t* scan_tmp = (uint32_t*)((char*)cursor + a8n);
                HIP_TRY(launch_fill_u32(indeg, 0u, n, s));
                HIP_TRY(launch_indegree(g, indeg, s));
                HIP_TRY(hipEventRecord(sk->ev_indeg, s));
                HIP_TRY(hipStreamWaitEvent(sk->aux, sk->ev_indeg, 0));
                HIP_TRY(launch_reverse_csr(g, indeg, cursor, scan_tmp, sk->aux));
                HIP_TRY(hipEventRecord(sk->ev_rev, sk->aux));
            }
            if (g.kind == THR_TARGET) {
                // w_uv depends on the target only; the kernels read it per edge, as a
                // coalesced array beside the edge hashes instead of a gather by target
                HIP_TRY(launch_wc_thresholds(indeg, wc_target, n, s));
                HIP_TRY(launch_gather_u32(wc_target, g.adj, m, g.thr, s));
                g.kind = THR_EDGE;
            }
            // samples and thresholds are final: flag the edges live in no sample
            HIP_TRY(launch_dead_edges(g, sk->X, R, s));
            HIP_TRY(hipStreamSynchronize(s));
            ctx_free(ctx, sk->hash_tmp);
            sk->hash_tmp = nullptr;
            g.eh = nullptr;
            // the row kernel's list of rows with 1..heavy_deg out-edges
            uint32_t* lflags = (uint32_t*)pm_;
            int64_t* lpos = (int64_t*)((char*)pm_ + a4n);
            uint32_t* lscan = (uint32_t*)((char*)lpos + a8n);
            HIP_TRY(launch_light_rows(g, lflags, lpos, lscan, s));
            HIP_TRY(hipMemcpyAsync(&g.nlight, lpos + n, 8, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            ctx_free(ctx, pm_);
            sk->list_tmp = nullptr;
            if (one_stream) {
                ctx_free(ctx, sk->rev_tmp);
                sk->rev_tmp = nullptr;
                sk->rev_ready = true;
            }
        }
        // greedy buffers
        const size_t W = 4 * (size_t)L.PW;
        GreedyBufs& b = sk->gb;
        b.qcap = qcap_for(n, m);
        b.bfs_chunk = BFS_CHUNK;
        bool ok3 = sk_alloc(sk, &b.blk, n * W) && sk_alloc(sk, &b.fullblk, words) && sk_alloc(sk, &b.F[0], n * W) &&
                   sk_alloc(sk, &b.F[1], n * W) &&
                   sk_alloc(sk, &b.Q[0], b.qcap) && sk_alloc(sk, &b.Q[1], b.qcap) && sk_alloc(sk, &b.qsize, 16) &&
                   sk_alloc(sk, &b.stamp, n) && sk_alloc(sk, &b.inS, n) && sk_alloc(sk, &b.MS, L.P) &&
                   sk_alloc(sk, &b.merged, L.P) && sk_alloc(sk, &b.key, 1) &&
                   sk_alloc(sk, &b.R, NSLOT * SLOT_U64) && sk_alloc(sk, &b.Rreb, 1);
        if (!ok3) return fail(IM_ERR_OUT_OF_BUDGET, "device allocation failed (greedy buffers)");
        b.T = sk->T;
        HIP_TRY(hipMemsetAsync(b.stamp, 0, 4 * n, s));
        HIP_TRY(hipMemsetAsync(b.F[0], 0, 4 * n * W, s));
        HIP_TRY(hipMemsetAsync(b.F[1], 0, 4 * n * W, s));
        HIP_TRY(hipEventRecord(sk->ev_b, s));
        HIP_TRY(hipStreamSynchronize(s));
        float pm = 0.f;
        HIP_TRY(hipEventElapsedTime(&pm, sk->ev_a, sk->ev_b));
        sk->prep_ms = pm;

        if (!simulate) {
            HIP_TRY(rev_csr_ready(sk, true));
            return IM_OK;
        }
        SimResult r;
        im_status rs = run_simulate(sk, 0, 1, nullptr, &r);
        if (rs != IM_OK) return rs;
        HIP_TRY(rev_csr_ready(sk, true));
        sk->build_buf = r.buf;
        sk->sel_buf = r.buf;
        sk->sweeps = r.sweeps;
        sk->visits = r.visits;
        sk->build_ms = r.ms;
        sk->trace_live = r.live;
        sk->trace_vis = r.vis;
        return IM_OK;
    };
    st = body();
    if (st != IM_OK) {
        sk_release(sk);
        return st;
    }
    sk->has_registers = simulate;
    *out = sk;
    return IM_OK;
}

}  // namespace

extern "C" {

im_status im_build_sketches(im_ctx* ctx, const im_csr* graph, const im_probs* probs, int32_t R, uint32_t hash_seed,
                            const im_build_opts* opts, im_sketch** out) {
    return build_sketch(ctx, graph, probs, R, hash_seed, opts, true, out);
}

void im_sketch_free(im_sketch* sk) { sk_release(sk); }

im_status im_sketch_get_info(const im_sketch* sk, im_sketch_info* info) {
    im_status st = check_sketch(sk);
    if (st != IM_OK) return st;
    if (!info) return fail(IM_ERR_INVALID_ARG, "info is null");
    info->n = sk->g.n;
    info->m = sk->g.m;
    info->R = sk->L.J;
    info->sweeps = sk->sweeps;
    info->visits = sk->visits;
    info->build_ms = sk->build_ms;
    info->prep_ms = sk->prep_ms;
    info->device_bytes = sk->bytes;
    info->heavy_rows = sk->g.nheavy;
    info->heavy_pieces = sk->g.npieces;
    return IM_OK;
}

im_status im_sketch_get_trace(const im_sketch* sk, int64_t* live_counts, int64_t* edge_visits, int32_t cap,
                              int32_t* written) {
    im_status st = check_sketch(sk);
    if (st != IM_OK) return st;
    const int32_t nl = (int32_t)sk->trace_live.size();
    for (int32_t i = 0; i < nl && i < cap; ++i) {
        if (live_counts) live_counts[i] = sk->trace_live[i];
        if (edge_visits && i < (int32_t)sk->trace_vis.size()) edge_visits[i] = sk->trace_vis[i];
    }
    if (written) *written = nl;
    return IM_OK;
}

int32_t im_sketch_get_sweep_log(const im_sketch* sk, im_sweep_rec* out, int32_t cap) {
    if (!sk) return 0;
    int32_t k = 0;
    for (; k < cap && k < (int32_t)sk->sweep_log.size(); ++k) out[k] = sk->sweep_log[k];
    return (int32_t)sk->sweep_log.size() < cap ? (int32_t)sk->sweep_log.size() : cap;
}

void im_sketch_clear_sweep_log(im_sketch* sk) {
    if (sk) sk->sweep_log.clear();
}

im_status im_sketch_get_registers(const im_sketch* sk, int32_t which, uint8_t* out) {
    im_status st = check_sketch(sk);
    if (st != IM_OK) return st;
    if (!out || (which != 0 && which != 1)) return fail(IM_ERR_INVALID_ARG, "bad arguments");
    const uint32_t* M = sk->M[which == 0 ? sk->build_buf : sk->sel_buf];
    if (hipMemcpy(out, M, (size_t)sk->g.n * sk->L.J, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(IM_ERR_DEVICE, "copy failed");
    return IM_OK;
}

im_status im_sketch_get_blocked(const im_sketch* sk, uint8_t* out) {
    im_status st = check_sketch(sk);
    if (st != IM_OK) return st;
    if (!out) return fail(IM_ERR_INVALID_ARG, "out is null");
    if (!sk->selected) return fail(IM_ERR_STATE, "no seed selection has run on this sketch");
    const size_t bytes = (size_t)sk->g.n * sk->L.J;
    void* tmp = ctx_alloc(sk->ctx, bytes);
    if (!tmp) return fail(IM_ERR_OUT_OF_BUDGET, "temporary allocation failed");
    hipStream_t s = sk->ctx->stream;
    im_status rs = IM_OK;
    if (launch_blocked_to_bytes(sk->L, sk->g.n, sk->gb.blk, (uint8_t*)tmp, s) != hipSuccess ||
        hipMemcpyAsync(out, tmp, bytes, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        rs = fail(IM_ERR_DEVICE, "blocked copy failed");
    ctx_free(sk->ctx, tmp);
    return rs;
}

im_status im_estimate_all(im_sketch* sk, float* out, int32_t out_on_device) {
    im_status st = check_sketch(sk);
    if (st != IM_OK) return st;
    if (!out) return fail(IM_ERR_INVALID_ARG, "out is null");
    hipStream_t s = sk->ctx->stream;
    const int64_t n = sk->g.n;
    float* dst = out;
    void* tmp = nullptr;
    if (!out_on_device) {
        tmp = ctx_alloc(sk->ctx, 4 * n);
        if (!tmp) return fail(IM_ERR_OUT_OF_BUDGET, "temporary allocation failed");
        dst = (float*)tmp;
    }
    im_status rs = IM_OK;
    if (launch_estimate_all(sk->L, n, sk->M[sk->build_buf], sk->T, dst, s) != hipSuccess)
        rs = fail(IM_ERR_DEVICE, "estimate kernel failed");
    if (rs == IM_OK && tmp && hipMemcpyAsync(out, tmp, 4 * n, hipMemcpyDeviceToHost, s) != hipSuccess)
        rs = fail(IM_ERR_DEVICE, "copy failed");
    if (hipStreamSynchronize(s) != hipSuccess) rs = fail(IM_ERR_DEVICE, "synchronize failed");
    if (tmp) ctx_free(sk->ctx, tmp);
    return rs;
}

im_status im_estimate(im_sketch* sk, const int32_t* verts, int64_t count, float* out_estimate) {
    im_status st = check_sketch(sk);
    if (st != IM_OK) return st;
    if (!verts || count < 1 || !out_estimate) return fail(IM_ERR_INVALID_ARG, "bad arguments");
    for (int64_t i = 0; i < count; ++i)
        if (verts[i] < 0 || verts[i] >= sk->g.n) return fail(IM_ERR_INVALID_ARG, "vertex id out of range");
    hipStream_t s = sk->ctx->stream;
    void* tmp = ctx_alloc(sk->ctx, 4 * count + 256);
    if (!tmp) return fail(IM_ERR_OUT_OF_BUDGET, "temporary allocation failed");
    float* dout = (float*)((char*)tmp + ((4 * count + 255) & ~int64_t(255)));
    im_status rs = IM_OK;
    float h = 0.f;
    if (hipMemcpyAsync(tmp, verts, 4 * count, hipMemcpyHostToDevice, s) != hipSuccess ||
        launch_estimate_set(sk->L, sk->M[sk->build_buf], (const int32_t*)tmp, count, sk->T, dout, s) != hipSuccess ||
        hipMemcpyAsync(&h, dout, 4, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        rs = fail(IM_ERR_DEVICE, "estimate failed");
    ctx_free(sk->ctx, tmp);
    if (rs == IM_OK) *out_estimate = h;
    return rs;
}

}  // extern "C"

namespace {

// Reach-search level ids restart (with every vertex stamp cleared) once the next
// step could run past this value; HFR_LEVEL_ID_LIMIT lowers it so that tests can
// force the restart on small graphs.
int32_t level_id_limit(int64_t n) {
    int64_t lim = INT32_MAX - (n + 8);
    if (const char* e = getenv("HFR_LEVEL_ID_LIMIT")) {
        const long long v = atoll(e);
        if (v > 0 && v < lim) lim = v;
    }
    return (int32_t)std::max<int64_t>(lim, 1);
}

// Alg. 1 on a built sketch.  `scratch` holds the K step records and K seeds
// (select_scratch_bytes(K) bytes, device memory) or is null, in which case they
// are allocated from the context for the call.
size_t select_scratch_bytes(int32_t K) { return ((sizeof(StepRec) * (size_t)K + 255) & ~size_t(255)) + 4 * (size_t)K; }

// resume: a run recorded by an earlier call with the same thresholds is reused --
// K up to its length is answered from the record (its first K steps are the run
// with K seeds: no rebuild follows the last step), and a longer K continues it
// from its last step (whose decision is taken again, now with a step after it).
im_status select_impl(im_sketch* sk, int32_t K, const im_select_opts* opts, int32_t* out_seeds, im_step* out_steps,
                      im_select_stats* stats, void* scratch, bool resume = false) {
    im_status st0 = check_sketch(sk);
    if (st0 != IM_OK) return st0;
    if (!out_seeds) return fail(IM_ERR_INVALID_ARG, "out_seeds is null");
    if (K < 1 || K > sk->g.n) return fail(IM_ERR_INVALID_ARG, "K must be in [1, n] (got %d)", K);
    double eps_g = 0.01, eps_l = 0.3;
    if (opts) {
        eps_g = opts->eps_g;
        eps_l = opts->eps_l;
    }
    if (!(eps_g >= 0.0) || !(eps_l >= 0.0)) return fail(IM_ERR_INVALID_ARG, "thresholds must be >= 0");
    const auto wall0 = std::chrono::steady_clock::now();
    hipStream_t s = sk->ctx->stream;
    const int64_t n = sk->g.n;
    const Layout& L = sk->L;
    GreedyBufs& b = sk->gb;
    const size_t W = 4 * (size_t)L.PW;
    const bool same = resume && sk->sel_K > 0 && sk->sel_eps_g == eps_g && sk->sel_eps_l == eps_l;
    // writes the outputs of steps 1..K from a complete record h (step K rebuilding nothing)
    auto emit = [&](const std::vector<StepRec>& h, const std::vector<int64_t>& lv, double device_ms) {
        int32_t rb = 0;
        int64_t rs = 0, rv = 0, lt = 0;
        for (int k = 0; k < K; ++k) {
            StepRec r = h[k];
            if (k == K - 1) r.rebuilt = 0, r.sweeps = 0, r.visits = 0;
            out_seeds[k] = r.seed;
            rb += r.rebuilt;
            rs += r.sweeps;
            rv += r.visits;
            lt += lv[k];
            if (out_steps) {
                im_step& o = out_steps[k];
                o.seed = r.seed;
                o.rebuilt = r.rebuilt;
                o.fresh = r.fresh;
                o.sweeps = r.sweeps;
                o.score = r.score;
                o.reach = r.reach;
                o.e = r.e;
                o.sigma = r.sigma;
                o.delta = r.delta;
                o.err_l = r.err_l;
                o.err_g = r.err_g;
                o.visits = r.visits;
            }
        }
        if (stats) {
            stats->rebuilds = rb;
            stats->reserved = 0;
            stats->rebuild_sweeps = rs;
            stats->rebuild_visits = rv;
            stats->bfs_levels = lt;
            stats->device_ms = device_ms;
            stats->wall_ms =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - wall0).count();
        }
    };
    if (same && K <= sk->sel_K) {  // a prefix of the recorded run: no device work
        emit(sk->sel_recs, sk->sel_levels, 0.0);
        return IM_OK;
    }
    const int k0 = same ? sk->sel_K : 0;  // steps already taken
    sk->sel_K = 0;                        // the record is valid again only once this call completes

    // per-call buffers for K records and seeds
    StepRec* d_steps = nullptr;
    int32_t* d_seeds = nullptr;
    double device_ms = 0.0;
    {
        void* p = scratch ? scratch : ctx_alloc(sk->ctx, select_scratch_bytes(K));
        if (!p) return fail(IM_ERR_OUT_OF_BUDGET, "temporary allocation failed");
        d_steps = (StepRec*)p;
        d_seeds = (int32_t*)((char*)p + ((sizeof(StepRec) * K + 255) & ~size_t(255)));
    }
    const int32_t lvl_limit = level_id_limit(n);
    std::vector<StepRec> h_steps(K);
    std::vector<int64_t> h_levels(K, 0);
    for (int k = 0; k < k0; ++k) {
        h_steps[k] = sk->sel_recs[k];
        h_levels[k] = sk->sel_levels[k];
    }

    // a rebuild after step k (1-based) on the register buffers not holding the build
    auto rebuild_after = [&](int k, int* cur) -> im_status {
        int ia = (*cur + 1) % 3, ib = (*cur + 2) % 3;
        if (ia == sk->build_buf) ia = (ia + 1) % 3;
        if (ib == sk->build_buf || ib == ia) ib = 3 - sk->build_buf - ia;
        SimResult r;
        im_status rs = run_simulate(sk, ia, ib, b.blk, &r);
        if (rs != IM_OK) return rs;
        *cur = r.buf;
        h_steps[k - 1].sweeps = r.sweeps;
        h_steps[k - 1].visits = r.visits;
        return IM_OK;
    };
    auto body = [&]() -> im_status {
        HIP_TRY(hipEventRecord(sk->ev_a, s));
        // the step records start at zero (fill kernel: no memset node in this memory)
        HIP_TRY(launch_fill_u32((uint32_t*)d_steps, 0u, (int64_t)(sizeof(StepRec) / 4) * K, s));
        int cur = sk->build_buf;
        if (k0 == 0) {
            HIP_TRY(hipMemsetAsync(b.blk, 0, 4 * n * W, s));
            HIP_TRY(hipMemsetAsync(b.inS, 0, n, s));
            HIP_TRY(hipMemsetAsync(b.MS, 0, 4 * L.P, s));
            HIP_TRY(hipMemsetAsync(b.key, 0, 8, s));
            HIP_TRY(hipMemsetAsync(b.R, 0, 8 * NSLOT * SLOT_U64, s));
            HIP_TRY(hipMemsetAsync(b.Rreb, 0, 8, s));
            // level ids start afresh every call, so a long-lived sketch never runs them out
            HIP_TRY(hipMemsetAsync(b.stamp, 0, 4 * (size_t)n, s));
            sk->level_id = 1;
        } else {
            // continue the recorded run: its device state is the one after step k0, before
            // step k0's decision took effect; take that decision again with steps to follow
            cur = sk->sel_buf;
            HIP_TRY(hipMemcpyAsync(d_steps, sk->sel_recs.data(), sizeof(StepRec) * k0, hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync(d_seeds, sk->sel_seeds.data(), 4 * (size_t)k0, hipMemcpyHostToDevice, s));
            int32_t flag = -1;
            HIP_TRY(launch_decide(L, b, d_steps + (k0 - 1), k0, K, eps_g, eps_l, sk->d_flag, s));
            HIP_TRY(hipMemcpyAsync(&flag, sk->d_flag, 4, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (flag == 1) {
                const im_status rs = rebuild_after(k0, &cur);
                if (rs != IM_OK) return rs;
            }
        }
        for (int k = k0 + 1; k <= K; ++k) {
            if (sk->level_id > lvl_limit) {
                HIP_TRY(hipMemsetAsync(b.stamp, 0, 4 * (size_t)n, s));
                sk->level_id = 1;
            }
            HIP_TRY(launch_argmax(L, n, sk->M[cur], b, s));
            HIP_TRY(hipMemsetAsync(b.qsize, 0, 16, s));
            const int32_t lvl0 = sk->level_id;
            HIP_TRY(launch_select(L, sk->g, sk->M[cur], b, d_steps + (k - 1), d_seeds, k - 1, lvl0, s));
            int32_t flag = -1;
            int level = 0;
            {
                int64_t with_work = 0;
                const im_status rs = run_reach(sk, lvl0, &level, &with_work);
                if (rs != IM_OK) return rs;
                h_levels[k - 1] = with_work;
            }
            sk->level_id = lvl0 + level + 2;
            {
                int32_t chosen = 0;
                HIP_TRY(hipMemcpyAsync(&chosen, d_seeds + (k - 1), 4, hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
                if (chosen < 0) {
                    sk->poisoned = true;
                    return fail(IM_ERR_DEVICE, "argmax found no candidate at step %d", k);
                }
            }
            HIP_TRY(launch_decide(L, b, d_steps + (k - 1), k, K, eps_g, eps_l, sk->d_flag, s));
            HIP_TRY(hipMemcpyAsync(&flag, sk->d_flag, 4, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (flag == 1) {
                const im_status rs = rebuild_after(k, &cur);
                if (rs != IM_OK) return rs;
            }
        }
        HIP_TRY(hipEventRecord(sk->ev_b, s));
        std::vector<StepRec> dev(K);
        HIP_TRY(hipMemcpyAsync(dev.data(), d_steps, sizeof(StepRec) * K, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(out_seeds, d_seeds, 4 * (size_t)K, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int k = 0; k < K; ++k) {
            // the host holds the sweep and visit counts of rebuilds (steps before k0 kept theirs)
            const int32_t sw = h_steps[k].sweeps;
            const int64_t vi = h_steps[k].visits;
            h_steps[k] = dev[k];
            h_steps[k].sweeps = sw;
            h_steps[k].visits = vi;
        }
        sk->sel_buf = cur;
        sk->selected = true;
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, sk->ev_a, sk->ev_b));
        device_ms = ms;
        return IM_OK;
    };
    im_status st = body();
    if (!scratch) ctx_free(sk->ctx, d_steps);
    if (st != IM_OK) return st;
    sk->sel_recs = h_steps;
    sk->sel_seeds.assign(out_seeds, out_seeds + K);
    sk->sel_levels = h_levels;
    sk->sel_eps_g = eps_g;
    sk->sel_eps_l = eps_l;
    sk->sel_K = K;
    emit(h_steps, h_levels, device_ms);
    return IM_OK;
}

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Called by im_ctx_create with `device` current: records this device's address
// of the scratch array, once per device.
im_status init_scratch(int device) {
    if (device >= MAX_DEVICES) return IM_OK;  // the allocation-free call then refuses this device
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return IM_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return fail(IM_ERR_DEVICE, "scratch symbol lookup failed: %s", hipGetErrorString(e));
    }
    g_scratch_ptr[device] = ptr;
    return IM_OK;
}

}  // namespace

extern "C" {

im_status im_select_seeds(im_sketch* sk, int32_t K, const im_select_opts* opts, int32_t* out_seeds, im_step* out_steps,
                          im_select_stats* stats) {
    return select_impl(sk, K, opts, out_seeds, out_steps, stats, nullptr);
}

im_status im_select_seeds_resume(im_sketch* sk, int32_t K, const im_select_opts* opts, int32_t* out_seeds,
                                 im_step* out_steps, im_select_stats* stats) {
    return select_impl(sk, K, opts, out_seeds, out_steps, stats, nullptr, true);
}

im_status im_select_seeds_noalloc(im_sketch* sk, int32_t K, const im_select_opts* opts, int32_t* out_seeds,
                                  im_step* out_steps, im_select_stats* stats) {
    im_status st0 = check_sketch(sk);
    if (st0 != IM_OK) return st0;
    if (K < 1 || K > IM_NOALLOC_MAX_K)
        return fail(IM_ERR_INVALID_ARG, "K must be in [1, %d] for the allocation-free selection (got %d)",
                    IM_NOALLOC_MAX_K, K);
    static_assert(sizeof(StepRec) * IM_NOALLOC_MAX_K + 256 + 4 * IM_NOALLOC_MAX_K <= NOALLOC_SCRATCH_BYTES,
                  "scratch too small for IM_NOALLOC_MAX_K");
    const int dev = sk->ctx->device;
    void* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (dev >= 0 && dev < MAX_DEVICES) ptr = g_scratch_ptr[dev];
    }
    if (!ptr) return fail(IM_ERR_STATE, "no scratch address for device %d", dev);
    return select_impl(sk, K, opts, out_seeds, out_steps, stats, ptr);
}


im_status im_evaluate_influence(im_ctx* ctx, const im_csr* graph, const im_probs* probs, int32_t R,
                                uint32_t hash_seed, const int32_t* seeds, int32_t count, double* out_sigma,
                                int64_t* out_reach) {
    if (!seeds || !out_sigma) return fail(IM_ERR_INVALID_ARG, "null argument");
    if (count < 1) return fail(IM_ERR_INVALID_ARG, "count must be >= 1");
    if (graph)
        for (int32_t i = 0; i < count; ++i)
            if (seeds[i] < 0 || seeds[i] >= graph->n)
                return fail(IM_ERR_INVALID_ARG, "seed %d is not a vertex id", (int)seeds[i]);
    im_sketch* sk = nullptr;
    im_status st = build_sketch(ctx, graph, probs, R, hash_seed, nullptr, false, &sk);
    if (st != IM_OK) return st;
    hipStream_t s = ctx->stream;
    const int64_t n = sk->g.n;
    const size_t W = 4 * (size_t)sk->L.PW;
    GreedyBufs& b = sk->gb;
    int32_t* d_seeds = (int32_t*)ctx_alloc(ctx, 4 * (size_t)count);
    auto body = [&]() -> im_status {
        if (!d_seeds) return fail(IM_ERR_OUT_OF_BUDGET, "temporary allocation failed");
        HIP_TRY(hipMemcpyAsync(d_seeds, seeds, 4 * (size_t)count, hipMemcpyHostToDevice, s));
        HIP_TRY(launch_fill_u32(b.blk, 0u, (int64_t)(n * W), s));
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(b.R), 0u, 2 * NSLOT * SLOT_U64, s));
        HIP_TRY(launch_fill_u32(b.qsize, 0u, 4, s));
        HIP_TRY(launch_reach_start(sk->L, sk->g, b, d_seeds, count, 1, s));
        int level = 0;
        int64_t with_work = 0;
        const im_status rs = run_reach(sk, 1, &level, &with_work);
        if (rs != IM_OK) return rs;
        unsigned long long slots[NSLOT * SLOT_U64];
        HIP_TRY(hipMemcpyAsync(slots, b.R, sizeof(slots), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        unsigned long long reach = 0;
        for (int i = 0; i < NSLOT; ++i) reach += slots[i * SLOT_U64];
        *out_sigma = (double)reach / (double)R;
        if (out_reach) *out_reach = (int64_t)reach;
        return IM_OK;
    };
    st = body();
    if (d_seeds) ctx_free(ctx, d_seeds);
    sk_release(sk);
    return st;
}

}  // extern "C"
