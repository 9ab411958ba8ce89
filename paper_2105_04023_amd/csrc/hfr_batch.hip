// Batched solver: many independent influence-maximisation problems (graphs of
// uneven sizes, edge models and R) solved by one persistent kernel launch that
// is captured once in a HIP graph and replayed.
//
// Every job walks the phases of the single-graph path: register init and
// synchronous sweeps to the stopping rule (Alg. 2; rows with many out-edges
// go through pieces and a fix-up), then K greedy steps of argmax, select,
// Monte-Carlo reach level by level and the error-adaptive decision, with a
// rebuild when it asks (Alg. 1).  A phase is cut into tiles.  Waves of the
// persistent grid claim tiles of any job from a per-job counter; the wave
// that completes the last tile of a phase performs the job's serial step
// (stopping rule, select, decision) and publishes the next phase.  No wave
// waits for another: a wave without a tile rescans the jobs, so the grid needs
// no co-residency, and every wave leaves once all jobs are done.  A wave that
// finds no tile for `timeout` ticks of the constant-rate clock raises the
// abort flag and leaves, which makes every other wave leave as well; only a
// broken invariant can cause that, and the run then reports an error.
//
// Memory ordering: a wave releases before it counts a finished tile and
// acquires after it claims one, so every tile of a phase sees all writes of
// the phases before it.  Large jobs are served by every wave of the grid and
// use agent scope (L2 write-back and invalidation across the XCDs).  Small
// jobs, whose long chains of short phases make the per-phase cost dominant,
// are pinned to one XCD at create (balanced by size over the XCDs found on
// the device) and served only by waves on that XCD (hardware register
// XCC_ID): all their data moves through one L2, and since this file is
// compiled in threadgroup-split mode, where workgroup scope spans the CUs
// that share an L2, their release is a wait for stores to reach L2 and their
// acquire an L1 invalidation.  Phase descriptors and control words are
// accessed with agent-scope atomic operations only.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "hfr_device.h"
#include "hfr_host.h"

namespace hfr {
namespace {

constexpr int BFS_CHUNK_B = 256;  // out-edges per BFS queue entry

enum BPhase : uint32_t {
    PH_INIT0 = 1,     // per-run state, edge hashes, WC thresholds, register init
    PH_SWEEP = 2,     // row tiles, then split-row piece tiles, of sweep t
    PH_FIX = 3,       // split rows of sweep t
    PH_ARGMAX = 4,    // greedy scores
    PH_BFS = 5,       // one reach level
    PH_BFSCLEAN = 6,  // clears the frontier bits that level consumed
    PH_INITR = 7,     // register init of a rebuild (blocked pairs are 0)
    PH_DONE = 8,
};

// Phase descriptor of a job, written only by the wave that advances the job.
struct BDesc {
    uint32_t phase;
    int32_t t;           // sweep of the running Simulate
    int32_t a, b;        // register buffers M^t and M^{t+1}
    int32_t cur;         // registers the greedy steps read
    int32_t build_buf;   // registers of the build
    int32_t sim;         // 0: build, > 0: rebuild number
    int32_t k;           // greedy step, 1-based
    int32_t level;       // reach level of the current step
    int32_t level_id;    // queue stamp of level 0 of the current step
    uint32_t qlen;       // queue entries of this level
    uint32_t qlen_next;  // entries queued for the next level
    uint32_t stamp;      // serial of the running sweep (flags of pieces merged in it)
    int32_t pad;
    int64_t sim_visits;  // edge visits of the running Simulate
    double e;            // estimate of the current step
};
static_assert(sizeof(BDesc) % 8 == 0, "BDesc is copied as 32-bit words");

struct BRes {
    unsigned long long Rreb;  // blocked pairs at the last rebuild
    unsigned long long build_visits, rebuild_sweeps, rebuild_visits, bfs_levels;
    uint32_t build_sweeps, rebuilds, sel_buf;
    int32_t status;
};

// Control block of one job: the claim word, the descriptor word, the
// completion counter and the accumulators sit on separate 128-byte lines.
struct BCtl {
    alignas(128) unsigned long long claim;  // seq << 32 | tiles claimed
    alignas(128) unsigned long long dsc;    // seq << 32 | tiles of the phase
    alignas(128) uint32_t done;             // tiles completed
    alignas(128) unsigned long long cnt;    // |L_{t+1}|
    unsigned long long vis;                 // edge visits of sweep t
    unsigned long long key;                 // argmax key
    unsigned long long R;                   // blocked pairs = reach of S times R
    uint32_t qnext;                         // entries queued for the next level
    alignas(128) BDesc d;
    alignas(128) BRes r;
};

// Read-only description of a job: device arrays and tiles.
struct BJob {
    int64_t n, m;
    const int64_t* xadj;
    int32_t* adj;           // the batch's copy; bit 31 (DEAD_EDGE) flags an edge live in no sample
    uint32_t* eh;           // edge hashes, written by PH_INIT0
    uint32_t* thr;          // WC: per target (written by PH_INIT0); per edge: uploaded
    const uint32_t* indeg;  // WC in-degrees
    uint32_t thr_const;
    int32_t kind;
    int32_t J, P, PW, K;
    int32_t pinned;  // served by the waves of one XCD only
    uint32_t seed;
    uint32_t thresh;  // the Simulate stops once |L| <= thresh
    double eps_g, eps_l;
    const double* T;  // exp2(r / J), r < J
    // tiles
    const int32_t* rtile;  // row tile bounds [nrt + 1], multiples of 32 except the last (n)
    int32_t nrt;
    int32_t npt, ppt;  // piece tiles and pieces per tile
    int32_t nht, hpt;  // split-row tiles and rows per tile
    int32_t ept, cpt;  // queue entries per reach tile and per clean-up tile
    int64_t heavy_deg;
    int64_t nheavy, npieces;
    const int32_t* hrow;  // split rows [nheavy]
    const int64_t* hpb;   // first piece of each split row
    const int64_t* hpn;   // pieces of each split row
    const int32_t* prow;  // split-row slot of each piece
    const int64_t* pe0;   // edge range of each piece
    const int64_t* pe1;
    uint32_t* part;      // partial rows of pieces [npieces * P]
    uint32_t* part_any;  // per piece: sweep serial of its last merge with a live edge
    uint32_t* M[3];
    uint32_t* Lb[2];  // L_t bitmaps, by sweep parity
    uint32_t* blk;
    uint32_t* F[2];
    int2* Q[2];
    int32_t* stamp;
    uint8_t* inS;
    uint32_t* MS;
    uint32_t* merged;
    StepRec* steps;
    int32_t* seeds;
    BCtl* ctl;
};

constexpr int MAX_XCC = 16;

struct BGlobal {
    int32_t xbeg[MAX_XCC], xend[MAX_XCC];  // pinned jobs [xbeg[x], xend[x]) run on XCD x (host-written)
    int32_t gbeg, gend;                    // jobs [gbeg, gend) run on every XCD
    alignas(128) uint32_t jobs_done;
    uint32_t xdone[MAX_XCC];      // pinned jobs of XCD x that reached PH_DONE
    uint32_t gdone;               // jobs served by every XCD that reached PH_DONE
    alignas(128) uint32_t abort;  // nonzero: the watchdog fired
    // tiles completed by the waves of XCD x (slot x * 16, one 128-byte line each): the
    // watchdog's evidence that some job, anywhere, is still moving
    alignas(128) unsigned long long xprog[MAX_XCC * 16];
    alignas(128) unsigned long long tiles;
    unsigned long long phases;
};

// ---- atomics ----
#define JOB_SCOPE __HIP_MEMORY_SCOPE_AGENT
DEVI unsigned long long ld64(const unsigned long long* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, JOB_SCOPE); }
DEVI uint32_t ld32(const uint32_t* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, JOB_SCOPE); }
DEVI void st64(unsigned long long* p, unsigned long long v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, JOB_SCOPE); }
DEVI void st32(uint32_t* p, uint32_t v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, JOB_SCOPE); }
DEVI uint32_t ld32_all(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEVI void job_release(bool pinned) {
    if (pinned)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    else
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
}
DEVI void job_acquire(bool pinned) {
    if (pinned)
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    else
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Index of the XCD this wave runs on.
DEVI uint32_t xcc_id() { return __builtin_amdgcn_s_getreg((3 << 11) | 20) & (MAX_XCC - 1); }

DEVI unsigned long long bcast64(unsigned long long v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

DEVI BDesc load_desc(const BDesc* p) {
    BDesc d;
    const uint32_t* s = reinterpret_cast<const uint32_t*>(p);
    uint32_t* o = reinterpret_cast<uint32_t*>(&d);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(BDesc) / 4); ++i) o[i] = __builtin_amdgcn_readfirstlane(ld32(s + i));
    return d;
}

DEVI void store_desc(BDesc* p, const BDesc& d) {
    uint32_t* o = reinterpret_cast<uint32_t*>(p);
    const uint32_t* s = reinterpret_cast<const uint32_t*>(&d);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(BDesc) / 4); ++i) st32(o + i, s[i]);
}

// X_j of Eq. (hash_prob) and hash(j) of the register init, for the dwords of
// this lane (computed in place of a table).
template <int G, int DW>
DEVI void sim_words_of(uint32_t seed, int P, int p, uint32_t (&x)[DW][4]) {
#pragma unroll
    for (int i = 0; i < DW; ++i) {
        const int q = i * G + p;
#pragma unroll
        for (int k = 0; k < 4; ++k) x[i][k] = q < P ? (mm3_key4((uint32_t)(4 * q + k), seed + 2u) & 0x7FFFFFFFu) : 0u;
    }
}

template <int G, int DW>
DEVI void init_words_of(uint32_t seed, int P, int p, uint32_t (&hj)[DW][4]) {
#pragma unroll
    for (int i = 0; i < DW; ++i) {
        const int q = i * G + p;
#pragma unroll
        for (int k = 0; k < 4; ++k) hj[i][k] = q < P ? mm3_key4((uint32_t)(4 * q + k), seed + 3u) : 0u;
    }
}

#define BKIND_DISPATCH(kind, CALL)             \
    do {                                       \
        if ((kind) == THR_CONST) {             \
            constexpr int K_ = THR_CONST;      \
            CALL;                              \
        } else if ((kind) == THR_TARGET) {     \
            constexpr int K_ = THR_TARGET;     \
            CALL;                              \
        } else {                               \
            constexpr int K_ = THR_EDGE;       \
            CALL;                              \
        }                                      \
    } while (0)

// ---- tiles ----

// Register init of rows [r0, r1) (Alg. 1): M_u[j] = clz(hash(u) xor hash(j)),
// 0 for blocked pairs of a rebuild.  The first init of a run also clears the
// run's per-vertex state of those rows, hashes their out-edges (Eq. hash) and
// flags those live in no sample, derives their weighted-cascade thresholds and
// clears a slice of the piece flags.
template <int G, int DW>
DEVI void tile_init(const BJob& jb, const BDesc& d, int tile, bool first_run) {
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63, grp = lane / G, p = lane % G;
    const int64_t r0 = jb.rtile[tile], r1 = jb.rtile[tile + 1];
    const int P = jb.P, PW = jb.PW, W = 4 * PW;
    if (first_run) {
        for (int64_t i = r0 * W + lane; i < r1 * W; i += 64) {
            jb.blk[i] = 0u;
            jb.F[0][i] = 0u;
            jb.F[1][i] = 0u;
        }
        for (int64_t u = r0 + lane; u < r1; u += 64) {
            jb.stamp[u] = 0;
            jb.inS[u] = 0;
            if (jb.kind == THR_TARGET) jb.thr[u] = wc_threshold(jb.indeg[u]);
        }
        for (int64_t base = r0; base < r1; base += RPW) {
            const int64_t u = base + grp;
            if (u < r1) {
                const int64_t eb = jb.xadj[u], ee = jb.xadj[u + 1];
                for (int64_t e = eb + p; e < ee; e += G) {
                    // the id may carry the flag of an earlier run of this batch
                    const int32_t v = adj_target(jb.adj[e]);
                    const uint32_t h = mm3_key8((uint32_t)u, (uint32_t)v, jb.seed) & 0x7FFFFFFFu;
                    jb.eh[e] = h;
                    // an edge live in no sample (min_j (X_j xor h) >= t, Sec. 3.1) is
                    // flagged in its target id: the sweeps and the reach skip it.  X_j
                    // is wave-uniform; a wave stops once all its edges are live somewhere
                    const uint32_t t = jb.kind == THR_CONST    ? jb.thr_const
                                       : jb.kind == THR_TARGET ? wc_threshold(jb.indeg[v])
                                                               : jb.thr[e];
                    uint32_t mn = 0xFFFFFFFFu;
                    for (int j0 = 0; j0 < jb.J; j0 += 16) {
                        if (!__ballot(mn >= t)) break;
                        for (int j = j0; j < j0 + 16 && j < jb.J; ++j)
                            mn = min(mn, (mm3_key4((uint32_t)j, jb.seed + 2u) & 0x7FFFFFFFu) ^ h);
                    }
                    if (mn >= t) jb.adj[e] = (int32_t)((uint32_t)v | DEAD_EDGE);
                }
            }
        }
        if (jb.npieces > 0) {
            const int64_t p0 = (int64_t)tile * jb.npieces / jb.nrt, p1 = (int64_t)(tile + 1) * jb.npieces / jb.nrt;
            for (int64_t i = p0 + lane; i < p1; i += 64) jb.part_any[i] = 0u;
        }
        if (tile == 0)
            for (int q = lane; q < P; q += 64) jb.MS[q] = 0u;
    }
    uint32_t hj[DW][4];
    init_words_of<G, DW>(jb.seed, P, p, hj);
    const uint32_t* blk = first_run ? nullptr : jb.blk;
    uint32_t* A = jb.M[d.a];
    uint32_t* B = jb.M[d.b];
    for (int64_t base = r0; base < r1; base += RPW) {
        const int64_t u = base + grp;
        if (u >= r1) continue;
        const uint32_t hv = mm3_key4((uint32_t)u, jb.seed + 1u);
#pragma unroll
        for (int i = 0; i < DW; ++i) {
            const int q = i * G + p;
            if (q >= P) continue;
            uint32_t w = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) w |= lead_zeros(hv ^ hj[i][k]) << (8 * k);
            if (blk) w &= unblocked_mask(blk, u, q, PW);
            A[u * P + q] = w;
            B[u * P + q] = w;
        }
    }
}

// Sweep t over rows [r0, r1) (whole 32-row words): rows with at most
// heavy_deg out-edges are merged here, the others by pieces and the fix-up.
// Stores every L_{t+1} word of the range.
template <int G, int DW, int KIND>
DEVI void tile_rows(const BJob& jb, BCtl* c, const BDesc& d, int tile) {
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63, grp = lane / G, p = lane % G;
    const int64_t r0 = jb.rtile[tile], r1 = jb.rtile[tile + 1];
    const int first = d.t == 0;
    const uint32_t* A = jb.M[d.a];
    uint32_t* B = jb.M[d.b];
    const uint32_t* Lcur = jb.Lb[d.t & 1];
    uint32_t* Lnext = jb.Lb[(d.t + 1) & 1];
    const uint32_t* blk = d.sim > 0 ? jb.blk : nullptr;
    uint32_t x[DW][4];
    sim_words_of<G, DW>(jb.seed, jb.P, p, x);
    const uint32_t ntv = to_vgpr(0u - jb.thr_const);
    unsigned long long my_vis = 0;
    uint32_t changed_rows = 0;
    for (int64_t w = r0; w < r1; w += 32) {
        const int64_t wend = w + 32 < r1 ? w + 32 : r1;
        uint32_t bits = 0;
        for (int64_t u0 = w; u0 < wend; u0 += RPW) {
            const int64_t u = u0 + grp;
            bool ch = false;
            if (u < wend)
                ch = sweep_row<G, DW, KIND>(u, jb.xadj, jb.adj, EdgeHashes{jb.eh, jb.seed}, jb.thr, ntv, x, A, B, Lcur,
                                            Lnext, blk, nullptr,
                                            jb.heavy_deg, jb.P, jb.PW, first, true, lane, p, my_vis);
            const uint64_t bal = __ballot(ch && p == 0);
#pragma unroll
            for (int gg = 0; gg < RPW; ++gg)
                if ((bal >> (gg * G)) & 1ull) bits |= 1u << (uint32_t)(u0 + gg - w);
        }
        if (lane == 0) Lnext[w >> 5] = bits;
        changed_rows += (uint32_t)__builtin_popcount(bits);
    }
    my_vis = wave_sum(my_vis);
    if (lane == 0) {
        if (changed_rows) atomicAdd(&c->cnt, (unsigned long long)changed_rows);
        if (my_vis) atomicAdd(&c->vis, my_vis);
    }
}

// Sweep t over a range of pieces of split rows: each piece's merged live
// neighbour rows go to its partial row, flagged with the sweep serial.
template <int G, int DW, int KIND>
DEVI void tile_pieces(const BJob& jb, BCtl* c, const BDesc& d, int ptile) {
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63, grp = lane / G, p = lane % G;
    const int64_t p0 = (int64_t)ptile * jb.ppt;
    const int64_t p1 = p0 + jb.ppt < jb.npieces ? p0 + jb.ppt : jb.npieces;
    const int P = jb.P, PW = jb.PW;
    const int first = d.t == 0;
    const uint32_t* A = jb.M[d.a];
    const uint32_t* Lcur = jb.Lb[d.t & 1];
    const uint32_t* blk = d.sim > 0 ? jb.blk : nullptr;
    uint32_t x[DW][4];
    sim_words_of<G, DW>(jb.seed, P, p, x);
    const uint32_t ntv = to_vgpr(0u - jb.thr_const);
    unsigned long long my_vis = 0;
    for (int64_t base = p0; base < p1; base += RPW) {
        const int64_t pc = base + grp;
        if (pc >= p1) continue;
        const int64_t u = jb.hrow[jb.prow[pc]];
        bool skip = false;
        if (blk) {  // a row blocked in every sample neither changes nor counts visits
            bool none = true;
#pragma unroll
            for (int i = 0; i < DW; ++i) {
                const int q = i * G + p;
                if (q < P) none = none && unblocked_mask(blk, u, q, PW) == 0u;
            }
            skip = group_all<G>(none);
        }
        Acc acc[DW];
#pragma unroll
        for (int i = 0; i < DW; ++i) acc[i].e = acc[i].o = 0u;
        uint32_t vis = 0;
        if (!skip)
            vis = merge_edges<G, DW, KIND>(jb.pe0[pc], jb.pe1[pc], (uint32_t)u, jb.adj, EdgeHashes{jb.eh, jb.seed},
                                           jb.thr, ntv, A, Lcur, first, P, lane, p, x, acc);
        if (vis > 0) {
#pragma unroll
            for (int i = 0; i < DW; ++i) {
                const int q = i * G + p;
                if (q < P) jb.part[pc * P + q] = acc[i].e | acc[i].o;
            }
            if (p == 0) jb.part_any[pc] = d.stamp;
        }
        if (p == 0) my_vis += vis;
    }
    my_vis = wave_sum(my_vis);
    if (lane == 0 && my_vis) atomicAdd(&c->vis, my_vis);
}

// Fix-up of split rows [h0, h1) after their pieces (see fix_row).
template <int G, int DW>
DEVI void tile_fix(const BJob& jb, BCtl* c, const BDesc& d, int tile) {
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63, grp = lane / G, p = lane % G;
    const int64_t h0 = (int64_t)tile * jb.hpt;
    const int64_t h1 = h0 + jb.hpt < jb.nheavy ? h0 + jb.hpt : jb.nheavy;
    const int first = d.t == 0;
    const uint32_t* A = jb.M[d.a];
    uint32_t* B = jb.M[d.b];
    const uint32_t* Lcur = jb.Lb[d.t & 1];
    uint32_t* Lnext = jb.Lb[(d.t + 1) & 1];
    const uint32_t* blk = d.sim > 0 ? jb.blk : nullptr;
    uint32_t my_cnt = 0;
    for (int64_t base = h0; base < h1; base += RPW) {
        const int64_t r = base + grp;
        if (r >= h1) continue;
        const int64_t u = jb.hrow[r];
        const bool ch = fix_row<G, DW>(r, u, A, B, Lcur, blk, jb.hpb, jb.hpn, jb.part, jb.part_any, d.stamp, jb.P,
                                       jb.PW, first, lane, p);
        if (ch && p == 0) {
            atomicOr(&Lnext[u >> 5], 1u << (u & 31));
            ++my_cnt;
        }
    }
    my_cnt = wave_sum(my_cnt);
    if (lane == 0 && my_cnt) atomicAdd(&c->cnt, (unsigned long long)my_cnt);
}

template <int G, int DW>
DEVI void tile_argmax(const BJob& jb, BCtl* c, const BDesc& d, int tile) {
    constexpr int RPW = 64 / G;
    const int64_t r0 = jb.rtile[tile], r1 = jb.rtile[tile + 1];
    const unsigned long long best = best_score_rows<G, DW>(r0, r1, RPW, jb.M[d.cur], jb.MS, jb.inS, jb.P);
    if ((threadIdx.x & 63) == 0 && best) atomicMax(&c->key, best);
}

template <int G, int DW, int KIND>
DEVI void tile_bfs(const BJob& jb, BCtl* c, const BDesc& d, int tile) {
    constexpr int RPW = 64 / G;
    const int p = (threadIdx.x & 63) % G;
    const int64_t b0 = (int64_t)tile * jb.ept;
    const int64_t b1 = b0 + jb.ept < (int64_t)d.qlen ? b0 + jb.ept : (int64_t)d.qlen;
    uint32_t x[DW][4];
    sim_words_of<G, DW>(jb.seed, jb.P, p, x);
    const uint32_t ntv = to_vgpr(0u - jb.thr_const);
    const int cur = d.level & 1;
    unsigned long long my_new = bfs_expand_entries<G, DW, KIND>(
        b0, b1, RPW, jb.xadj, jb.adj, EdgeHashes{jb.eh, jb.seed}, jb.thr, ntv, x, jb.F[cur], jb.F[cur ^ 1], jb.Q[cur],
        jb.Q[cur ^ 1],
        &c->qnext, jb.blk, jb.stamp, d.level_id + d.level + 1, BFS_CHUNK_B, jb.P, jb.PW);
    my_new = wave_sum(my_new);
    if ((threadIdx.x & 63) == 0 && my_new) atomicAdd(&c->R, my_new);
}

DEVI void tile_bfsclean(const BJob& jb, const BDesc& d, int tile) {
    const int lane = threadIdx.x & 63;
    const int W = 4 * jb.PW;
    const int cur = d.level & 1;
    const int64_t b0 = (int64_t)tile * jb.cpt;
    const int64_t b1 = b0 + jb.cpt < (int64_t)d.qlen ? b0 + jb.cpt : (int64_t)d.qlen;
    for (int64_t i = b0 * W + lane; i < b1 * W; i += 64) {
        const int2 qe = jb.Q[cur][i / W];
        if (qe.y == 0) jb.F[cur][(int64_t)qe.x * W + (i % W)] = 0u;
    }
}

template <int G, int DW>
DEVI void run_tile(const BJob& jb, BCtl* c, const BDesc& d, int tile) {
    switch (d.phase) {
    case PH_INIT0:
        tile_init<G, DW>(jb, d, tile, true);
        break;
    case PH_INITR:
        tile_init<G, DW>(jb, d, tile, false);
        break;
    case PH_SWEEP:
        if (tile < jb.nrt)
            BKIND_DISPATCH(jb.kind, (tile_rows<G, DW, K_>(jb, c, d, tile)));
        else
            BKIND_DISPATCH(jb.kind, (tile_pieces<G, DW, K_>(jb, c, d, tile - jb.nrt)));
        break;
    case PH_FIX:
        tile_fix<G, DW>(jb, c, d, tile);
        break;
    case PH_ARGMAX:
        tile_argmax<G, DW>(jb, c, d, tile);
        break;
    case PH_BFS:
        BKIND_DISPATCH(jb.kind, (tile_bfs<G, DW, K_>(jb, c, d, tile)));
        break;
    case PH_BFSCLEAN:
        tile_bfsclean(jb, d, tile);
        break;
    default:
        break;
    }
}

// ---- serial steps of a job (one wave, after the last tile of a phase) ----

DEVI uint32_t ceil_div(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

// Runs the job's serial step after phase d.phase and publishes the next phase
// as sequence seq + 1.
DEVI void advance(const BJob& jb, BGlobal* gl, uint32_t seq) {
    BCtl* c = jb.ctl;
    const int lane = threadIdx.x & 63;
    BDesc d = load_desc(&c->d);
    uint32_t phase = PH_DONE, ntiles = 0;
    int32_t status = 0;

    auto begin_sweep = [&]() {
        d.stamp += 1u;
        if (lane == 0) {
            st64(&c->cnt, 0ull);
            st64(&c->vis, 0ull);
        }
        phase = PH_SWEEP;
        ntiles = (uint32_t)(jb.nrt + jb.npt);
    };
    auto start_argmax = [&]() {
        if (lane == 0) st64(&c->key, 0ull);
        phase = PH_ARGMAX;
        ntiles = (uint32_t)jb.nrt;
    };
    // the Simulate ended with its registers in buffer res after d.t sweeps
    auto finish_sim = [&](int32_t res) {
        if (d.sim == 0) {
            if (lane == 0) {
                st32(&c->r.build_sweeps, (uint32_t)d.t);
                st64(&c->r.build_visits, (unsigned long long)d.sim_visits);
            }
            d.build_buf = res;
            d.cur = res;
            d.k = 1;
        } else {
            if (lane == 0) {
                StepRec* rec = jb.steps + (d.k - 1);
                __hip_atomic_store(&rec->sweeps, d.t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&rec->visits, d.sim_visits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                atomicAdd(&c->r.rebuild_sweeps, (unsigned long long)d.t);
                atomicAdd(&c->r.rebuild_visits, (unsigned long long)d.sim_visits);
            }
            d.cur = res;
            d.k += 1;
        }
        start_argmax();
    };
    auto end_sweep = [&]() {
        const unsigned long long cnt = bcast64(ld64(&c->cnt));
        const unsigned long long vis = bcast64(ld64(&c->vis));
        d.sim_visits += (int64_t)vis;
        d.t += 1;
        if (cnt <= jb.thresh) {
            finish_sim(d.b);
        } else if ((int64_t)d.t > jb.n + 2) {
            status = IM_ERR_DEVICE;  // synchronous sweeps reach the fixed point within n + 1 sweeps
        } else {
            const int32_t tmp = d.a;
            d.a = d.b;
            d.b = tmp;
            begin_sweep();
        }
    };
    auto decide = [&]() {
        int fresh = 0, rebuild = 0;
        if (lane == 0) {
            const unsigned long long R = ld64(&c->R);
            const unsigned long long R0 = ld64(&c->r.Rreb);
            rebuild = decide_step(R, R0, jb.J, d.k, jb.K, jb.eps_g, jb.eps_l, d.e, jb.steps + (d.k - 1), &fresh);
            if (rebuild) st64(&c->r.Rreb, R);
        }
        fresh = __builtin_amdgcn_readfirstlane(fresh);
        rebuild = __builtin_amdgcn_readfirstlane(rebuild);
        if (d.k < jb.K)
            for (int q = lane; q < jb.P; q += 64) jb.MS[q] = fresh ? jb.merged[q] : 0u;
        d.level_id += d.level + 2;
        if (rebuild) {
            if (lane == 0) atomicAdd(&c->r.rebuilds, 1u);
            // two buffers other than the build's
            int ia = (d.cur + 1) % 3, ib = (d.cur + 2) % 3;
            if (ia == d.build_buf) ia = (ia + 1) % 3;
            if (ib == d.build_buf || ib == ia) ib = 3 - d.build_buf - ia;
            d.a = ia;
            d.b = ib;
            d.sim += 1;
            d.t = 0;
            d.sim_visits = 0;
            phase = PH_INITR;
            ntiles = (uint32_t)jb.nrt;
        } else if (d.k < jb.K) {
            d.k += 1;
            start_argmax();
        } else {
            if (lane == 0) st32(&c->r.sel_buf, (uint32_t)d.cur);
            phase = PH_DONE;
            ntiles = 0;
        }
    };

    switch (d.phase) {
    case PH_INIT0:
    case PH_INITR:
        d.t = 0;
        d.sim_visits = 0;
        if ((uint64_t)jb.n <= jb.thresh)
            finish_sim(d.a);  // no sweep: the registers stay as initialised
        else
            begin_sweep();
        break;
    case PH_SWEEP:
        if (jb.nheavy > 0) {
            phase = PH_FIX;
            ntiles = (uint32_t)jb.nht;
        } else {
            end_sweep();
        }
        break;
    case PH_FIX:
        end_sweep();
        break;
    case PH_ARGMAX: {
        const unsigned long long key = bcast64(ld64(&c->key));
        uint32_t nch = 0, newcnt = 0;
        double e = 0.0;
        const bool ok = select_seed(key, jb.n, jb.J, jb.P, jb.PW, jb.xadj, jb.M[d.cur], jb.MS, jb.merged, jb.blk,
                                    jb.F[0], jb.Q[0], jb.inS, jb.stamp, d.level_id, BFS_CHUNK_B, jb.T,
                                    jb.steps + (d.k - 1), jb.seeds, d.k - 1, &nch, &newcnt, &e);
        if (!ok) {
            status = IM_ERR_DEVICE;  // no candidate vertex left
            break;
        }
        if (lane == 0) {
            if (newcnt) atomicAdd(&c->R, (unsigned long long)newcnt);
            st32(&c->qnext, 0u);
        }
        d.e = e;
        d.level = 0;
        d.qlen = nch;
        if (nch > 0) {
            phase = PH_BFS;
            ntiles = ceil_div(nch, (uint32_t)jb.ept);
        } else {
            decide();
        }
        break;
    }
    case PH_BFS:
        d.qlen_next = __builtin_amdgcn_readfirstlane(ld32(&c->qnext));
        phase = PH_BFSCLEAN;
        ntiles = ceil_div(d.qlen, (uint32_t)jb.cpt);
        break;
    case PH_BFSCLEAN:
        if (lane == 0) atomicAdd(&c->r.bfs_levels, 1ull);
        d.level += 1;
        if (d.qlen_next == 0) {
            decide();
        } else if ((int64_t)d.level > jb.n + 2) {
            status = IM_ERR_DEVICE;  // a reach search has at most n levels
        } else {
            d.qlen = d.qlen_next;
            if (lane == 0) st32(&c->qnext, 0u);
            phase = PH_BFS;
            ntiles = ceil_div(d.qlen, (uint32_t)jb.ept);
        }
        break;
    default:
        status = IM_ERR_STATE;
        break;
    }
    if (status != 0) {
        phase = PH_DONE;
        ntiles = 0;
        if (lane == 0) st32(reinterpret_cast<uint32_t*>(&c->r.status), (uint32_t)status);
    }
    d.phase = phase;
    if (lane == 0) {
        store_desc(&c->d, d);
        st32(&c->done, 0u);
    }
    job_release(jb.pinned != 0);
    if (lane == 0) {
        st64(&c->dsc, ((unsigned long long)(seq + 1) << 32) | ntiles);
        __hip_atomic_store(&c->claim, (unsigned long long)(seq + 1) << 32, __ATOMIC_RELEASE, JOB_SCOPE);
        atomicAdd(&gl->phases, 1ull);
        if (phase == PH_DONE) {
            // the wave that advances a pinned job runs on that job's XCD
            atomicAdd(jb.pinned ? &gl->xdone[xcc_id()] : &gl->gdone, 1u);
            atomicAdd(&gl->jobs_done, 1u);
        }
    }
}

// The persistent solver.  Every wave loops: claim a tile of a pinned job of
// its XCD or of a job served by all XCDs, run it, count it, and advance the
// job when it completed the phase's last tile.  A wave that finds nothing
// backs off (up to ~28 us) before it scans again.  A wave leaves once every job
// it may serve is done (or all jobs are, or the abort flag is up).  It raises
// the abort flag when, for `timeout` ticks, neither the claim words it scans,
// nor the phase count, nor the tiles completed on any XCD have changed: then
// no wave anywhere is making progress (a broken invariant only).
template <int G, int DW>
__global__ __launch_bounds__(256) void k_batch(const BJob* __restrict__ jobs, int njobs, BGlobal* gl,
                                               unsigned long long timeout_ticks) {
    const int lane = threadIdx.x & 63;
    const uint32_t x = xcc_id();
    const int pb = gl->xbeg[x], n1 = gl->xend[x] - pb;
    const int gb = gl->gbeg, n2 = gl->gend - gb;
    const int nmine = n1 + n2;
    if (nmine <= 0) return;
    int start = (int)(wave_index() % nmine);
    bool idle = false;
    int backoff = 0;
    unsigned long long idle_t0 = 0, last_sig = 0, my_tiles = 0;
    while (true) {
        uint32_t stop = 0;
        if (lane == 0) {
            stop = ld32_all(&gl->abort) | (ld32_all(&gl->jobs_done) >= (uint32_t)njobs ? 1u : 0u);
            // every job this wave may serve is done: other XCDs may still be busy
            if (ld32_all(&gl->xdone[x]) >= (uint32_t)n1 && ld32_all(&gl->gdone) >= (uint32_t)n2) stop = 1u;
        }
        if (__builtin_amdgcn_readfirstlane(stop)) break;
        int jsel = -1;
        unsigned long long claim = 0, dsc = 0, sig = 0;
        for (int i = 0; i < nmine && jsel < 0; ++i) {
            int idx = start + i;
            if (idx >= nmine) idx -= nmine;
            const int j = idx < n1 ? pb + idx : gb + (idx - n1);
            BCtl* c = jobs[j].ctl;
            unsigned long long w = 0, ds = 0;
            if (lane == 0) {
                w = ld64(&c->claim);
                ds = ld64(&c->dsc);
            }
            w = bcast64(w);
            ds = bcast64(ds);
            sig = sig * 0x9E3779B97F4A7C15ull + w;
            if ((w >> 32) != (ds >> 32) || (uint32_t)w >= (uint32_t)ds) continue;
            unsigned long long old = 0, ds2 = 0;
            if (lane == 0) {
                old = __hip_atomic_fetch_add(&c->claim, 1ull, __ATOMIC_ACQUIRE, JOB_SCOPE);
                ds2 = __hip_atomic_load(&c->dsc, __ATOMIC_ACQUIRE, JOB_SCOPE);
            }
            old = bcast64(old);
            ds2 = bcast64(ds2);
            // valid iff the claim belongs to the phase the descriptor word names
            if ((old >> 32) == (ds2 >> 32) && (uint32_t)old < (uint32_t)ds2) {
                jsel = j;
                claim = old;
                dsc = ds2;
                start = idx;
            }
        }
        if (jsel < 0) {
            unsigned long long prog = 0;
            if (lane == 0) {
                prog = ld64(&gl->phases);
                for (int k = 0; k < MAX_XCC; ++k) prog += ld64(&gl->xprog[k * 16]);
            }
            sig = sig * 0x9E3779B97F4A7C15ull + bcast64(prog);
            const unsigned long long now = wall_clock64();
            if (!idle || sig != last_sig) {  // some job moved: not stuck
                idle = true;
                idle_t0 = now;
                last_sig = sig;
            } else if (now - idle_t0 > timeout_ticks) {
                if (lane == 0) atomicOr(&gl->abort, 1u);
                break;
            }
            if (backoff < 10) ++backoff;
            for (int i = 0; i < (1 << backoff); ++i) __builtin_amdgcn_s_sleep(1);
            continue;
        }
        idle = false;
        backoff = 0;
        const BJob& jb = jobs[jsel];
        const bool pinned = jb.pinned != 0;
        job_acquire(pinned);
        BCtl* c = jb.ctl;
        const BDesc d = load_desc(&c->d);
        run_tile<G, DW>(jb, c, d, (int)(uint32_t)claim);
        ++my_tiles;
        if (lane == 0) __hip_atomic_fetch_add(&gl->xprog[x * 16], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        job_release(pinned);
        uint32_t prev = 0;
        if (lane == 0) prev = __hip_atomic_fetch_add(&c->done, 1u, __ATOMIC_ACQ_REL, JOB_SCOPE);
        prev = __builtin_amdgcn_readfirstlane(prev);
        if (prev + 1 == (uint32_t)dsc) {
            job_acquire(pinned);
            advance(jb, gl, (uint32_t)(dsc >> 32));
        }
    }
    if (lane == 0 && my_tiles) atomicAdd(&gl->tiles, my_tiles);
}

// Records the XCD ids that run waves of a large grid (bit x of *mask).
__global__ void k_xcc_probe(uint32_t* mask) {
    if ((threadIdx.x & 63) == 0) atomicOr(mask, 1u << xcc_id());
}

// Arms every job at phase PH_INIT0 (sequence 1) and clears the run counters.
__global__ void k_batch_arm(const BJob* __restrict__ jobs, int njobs, BGlobal* gl) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 0) {  // the job ranges per XCD stay as the host wrote them
        gl->jobs_done = 0;
        for (int k = 0; k < MAX_XCC; ++k) {
            gl->xdone[k] = 0;
            gl->xprog[k * 16] = 0;
        }
        gl->gdone = 0;
        gl->abort = 0;
        gl->tiles = 0;
        gl->phases = 0;
    }
    if (j >= njobs) return;
    BCtl* c = jobs[j].ctl;
    c->claim = 1ull << 32;
    c->dsc = (1ull << 32) | (unsigned long long)(uint32_t)jobs[j].nrt;
    c->done = 0;
    c->cnt = c->vis = c->key = c->R = 0;
    c->qnext = 0;
    BDesc d;
    memset(&d, 0, sizeof(d));
    d.phase = PH_INIT0;
    d.a = 0;
    d.b = 1;
    d.level_id = 1;
    c->d = d;
    BRes r;
    memset(&r, 0, sizeof(r));
    c->r = r;
}

// ---- host side ----

struct BatchCfg {
    int G = 0;
    int tile_edges = 8192;
    int heavy_degree = 512;
    int piece_edges = 512;
    int workgroups = 0;
    int64_t pin_edges = 0;  // jobs with at most this many edges run on one XCD (< 0: none)
};

struct HostJob {
    int32_t index;  // the caller's job index
    int64_t n, m;
    int J, P, PW, K;
    std::vector<int64_t> xadj;
    std::vector<int32_t> adj;
    BJob dj{};
    // split rows (host copies, for the tile tables)
    std::vector<int32_t> hrow, prow;
    std::vector<int64_t> hpb, hpn, pe0, pe1;
    int32_t* d_rtile = nullptr;
    int64_t rtile_cap = 0;
};

}  // namespace
}  // namespace hfr

using namespace hfr;

struct im_batch {
    im_ctx* ctx = nullptr;
    bool poisoned = false;
    std::vector<HostJob> jobs;      // in the caller's order
    std::vector<int32_t> perm;      // device position -> caller's index (see place_jobs)
    std::vector<int> xccs;          // XCD ids that run waves
    std::vector<void*> bufs;
    size_t bytes = 0;
    BJob* d_jobs = nullptr;
    BGlobal* d_gl = nullptr;
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev_in = nullptr, ev0 = nullptr, ev1 = nullptr;
    BatchCfg cfg;
    int cus = 256;
    unsigned long long timeout_ticks = 0;
    int candidates = 0;
    bool ran = false;
    std::vector<BCtl> h_ctl;
    BGlobal h_gl{};
    int32_t xbeg[MAX_XCC] = {}, xend[MAX_XCC] = {};  // job ranges per XCD id
    int32_t gbeg = 0, gend = 0;                        // jobs served by every XCD
    int nxcc = 0;                                      // XCDs found by the probe
    int32_t pin_request = 0;                           // im_batch_opts.pin_edges
    int grid = 0;                                      // workgroups of the captured launch
};

namespace {

void batch_release(im_batch* b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (hipEvent_t e : {b->ev_in, b->ev0, b->ev1})
        if (e) (void)hipEventDestroy(e);
    if (b->ctx) {
        for (void* p : b->bufs) ctx_free(b->ctx, p);
        b->ctx->in_use -= b->bytes;
    }
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

template <typename T>
T* balloc(im_batch* b, size_t count) {
    const size_t bytes = (sizeof(T) * (count ? count : 1) + 255) & ~size_t(255);
    void* p = ctx_alloc(b->ctx, bytes);
    if (!p) return nullptr;
    b->bufs.push_back(p);
    b->bytes += bytes;
    b->ctx->in_use += bytes;
    return reinterpret_cast<T*>(p);
}

#define BHIP(expr)                                                                                             \
    do {                                                                                                       \
        hipError_t _e = (expr);                                                                                \
        if (_e != hipSuccess) {                                                                                \
            b->poisoned = true;                                                                                \
            return fail(IM_ERR_DEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, __LINE__); \
        }                                                                                                      \
    } while (0)

int min_lanes(int Pmax) {
    int G = 4;
    while (G < Pmax) G <<= 1;
    return G;
}

// Tile tables of one job for a decomposition: row tiles of whole 32-row
// words holding about te merged edges (one per row counted too), pieces of
// split rows, and the tile sizes of the other phases.  te is tile_edges, or
// less for small jobs so that a phase still spreads over about MIN_TILES
// tiles: a tile's rows are walked by one wave, one dependent chain of loads
// per row group, so small tiles bound the latency of a phase.
constexpr int64_t MIN_TILES = 512;

void make_tiles(const HostJob& h, const BatchCfg& cfg, std::vector<int32_t>& rtile, BJob& dj) {
    const int RPW = 64 / cfg.G;
    const int64_t n = h.n;
    const int64_t te = std::max<int64_t>(64, std::min<int64_t>(cfg.tile_edges, (h.m + n) / MIN_TILES));
    rtile.clear();
    rtile.push_back(0);
    int64_t acc = 0;
    for (int64_t w = 0; w < n; w += 32) {
        const int64_t we = std::min<int64_t>(w + 32, n);
        for (int64_t u = w; u < we; ++u) {
            const int64_t dgr = h.xadj[u + 1] - h.xadj[u];
            acc += (dgr <= cfg.heavy_degree ? dgr : 0) + 1;
        }
        if (acc >= te || we == n) {
            rtile.push_back((int32_t)we);
            acc = 0;
        }
    }
    dj.nrt = (int32_t)(rtile.size() - 1);
    const int64_t ppt = (int64_t)RPW * std::max<int64_t>(1, te / ((int64_t)cfg.piece_edges * RPW));
    dj.ppt = (int32_t)ppt;
    dj.npt = (int32_t)((h.pe0.size() + ppt - 1) / ppt);
    dj.hpt = RPW * 4;
    dj.nht = (int32_t)((h.hrow.size() + dj.hpt - 1) / dj.hpt);
    dj.ept = std::max(RPW, (int)(te / BFS_CHUNK_B / RPW) * RPW);
    dj.cpt = 1024;
}

void split_rows(HostJob& h, int64_t heavy, int64_t piece) {
    h.hrow.clear();
    h.hpb.clear();
    h.hpn.clear();
    h.prow.clear();
    h.pe0.clear();
    h.pe1.clear();
    for (int64_t u = 0; u < h.n; ++u) {
        const int64_t eb = h.xadj[u], ee = h.xadj[u + 1];
        if (ee - eb <= heavy) continue;
        const int64_t np = (ee - eb + piece - 1) / piece;
        h.hpb.push_back((int64_t)h.pe0.size());
        h.hpn.push_back(np);
        for (int64_t c = 0; c < np; ++c) {
            h.prow.push_back((int32_t)h.hrow.size());
            h.pe0.push_back(eb + c * piece);
            h.pe1.push_back(std::min(ee, eb + (c + 1) * piece));
        }
        h.hrow.push_back((int32_t)u);
    }
}

// Placement for the current decomposition: jobs with at most pin_edges edges
// are pinned to XCDs, largest first onto the least loaded; the others are
// served by every XCD.  Device order: the global jobs (largest first), then
// the pinned jobs of each XCD (largest first), so that within every scan
// range the largest jobs' phases are claimed first.
void place_jobs(im_batch* b) {
    const int count = (int)b->jobs.size();
    std::vector<int32_t> ord(count), home(count, -1);
    for (int i = 0; i < count; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) { return b->jobs[a].m > b->jobs[c].m; });
    std::vector<double> load(b->xccs.size(), 0.0);
    for (int i : ord) {
        if (b->jobs[i].m > b->cfg.pin_edges) continue;
        const size_t x = std::min_element(load.begin(), load.end()) - load.begin();
        home[i] = (int32_t)x;
        load[x] += (double)(b->jobs[i].m + b->jobs[i].n) * (double)b->jobs[i].J;
    }
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) { return home[a] < home[c]; });
    b->perm = ord;
    for (int x = 0; x < MAX_XCC; ++x) b->xbeg[x] = b->xend[x] = 0;
    b->gbeg = b->gend = 0;
    for (int k = 0; k < count; ++k) {
        const int hx = home[ord[k]];
        b->jobs[ord[k]].dj.pinned = hx >= 0;
        if (hx < 0) {
            b->gend = k + 1;
            continue;
        }
        const int x = b->xccs[hx];
        if (b->xend[x] == 0 && b->xbeg[x] == 0) b->xbeg[x] = k;
        b->xend[x] = k + 1;
    }
}

// Places the jobs and uploads the tile tables, the job array and the job
// ranges of the current decomposition.
im_status upload_tiles(im_batch* b) {
    hipStream_t s = b->stream;
    place_jobs(b);
    std::vector<BJob> dj(b->jobs.size());
    for (size_t k = 0; k < b->jobs.size(); ++k) {
        HostJob& h = b->jobs[b->perm[k]];
        std::vector<int32_t> rt;
        make_tiles(h, b->cfg, rt, h.dj);
        if ((int64_t)rt.size() > h.rtile_cap) return fail(IM_ERR_STATE, "row tile table overflow");
        BHIP(hipMemcpyAsync(h.d_rtile, rt.data(), 4 * rt.size(), hipMemcpyHostToDevice, s));
        BHIP(hipStreamSynchronize(s));
        dj[k] = h.dj;
    }
    BHIP(hipMemcpyAsync(b->d_jobs, dj.data(), sizeof(BJob) * dj.size(), hipMemcpyHostToDevice, s));
    BGlobal g0;
    memset(&g0, 0, sizeof(g0));
    memcpy(g0.xbeg, b->xbeg, sizeof(g0.xbeg));
    memcpy(g0.xend, b->xend, sizeof(g0.xend));
    g0.gbeg = b->gbeg;
    g0.gend = b->gend;
    BHIP(hipMemcpyAsync(b->d_gl, &g0, sizeof(g0), hipMemcpyHostToDevice, s));
    BHIP(hipStreamSynchronize(s));
    return IM_OK;
}

im_status capture(im_batch* b) {
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    hipStream_t s = b->stream;
    const int nj = (int)b->jobs.size();
    // workgroups are dispatched round-robin over the XCDs: a multiple of their
    // count gives every XCD the same share of waves
    const int nx = std::max(1, b->nxcc);
    const int grid = (std::max(b->cfg.workgroups, nx) + nx - 1) / nx * nx;
    b->grid = grid;
    BHIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipLaunchKernelGGL(k_batch_arm, dim3((nj + 255) / 256), dim3(256), 0, s, b->d_jobs, nj, b->d_gl);
    switch (b->cfg.G) {
    case 4:
        hipLaunchKernelGGL((k_batch<4, 1>), dim3(grid), dim3(256), 0, s, b->d_jobs, nj, b->d_gl, b->timeout_ticks);
        break;
    case 8:
        hipLaunchKernelGGL((k_batch<8, 1>), dim3(grid), dim3(256), 0, s, b->d_jobs, nj, b->d_gl, b->timeout_ticks);
        break;
    case 16:
        hipLaunchKernelGGL((k_batch<16, 1>), dim3(grid), dim3(256), 0, s, b->d_jobs, nj, b->d_gl, b->timeout_ticks);
        break;
    case 32:
        hipLaunchKernelGGL((k_batch<32, 1>), dim3(grid), dim3(256), 0, s, b->d_jobs, nj, b->d_gl, b->timeout_ticks);
        break;
    default:
        hipLaunchKernelGGL((k_batch<64, 1>), dim3(grid), dim3(256), 0, s, b->d_jobs, nj, b->d_gl, b->timeout_ticks);
        break;
    }
    hipGraph_t g = nullptr;
    const hipError_t e1 = hipStreamEndCapture(s, &g);
    if (e1 != hipSuccess) {
        b->poisoned = true;
        return fail(IM_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e1));
    }
    b->graph = g;
    BHIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return IM_OK;
}

// One replay; reads the control blocks back.  *ms receives the device time.
im_status replay(im_batch* b, float* ms) {
    hipStream_t s = b->stream;
    BHIP(hipEventRecord(b->ev_in, b->ctx->stream));
    BHIP(hipStreamWaitEvent(s, b->ev_in, 0));
    BHIP(hipEventRecord(b->ev0, s));
    BHIP(hipGraphLaunch(b->exec, s));
    BHIP(hipEventRecord(b->ev1, s));
    BHIP(hipEventSynchronize(b->ev1));
    BHIP(hipEventElapsedTime(ms, b->ev0, b->ev1));
    BHIP(hipMemcpyAsync(&b->h_gl, b->d_gl, sizeof(BGlobal), hipMemcpyDeviceToHost, s));
    b->h_ctl.resize(b->jobs.size());
    for (size_t i = 0; i < b->jobs.size(); ++i)
        BHIP(hipMemcpyAsync(&b->h_ctl[i], b->jobs[i].dj.ctl, sizeof(BCtl), hipMemcpyDeviceToHost, s));
    BHIP(hipStreamSynchronize(s));
    if (b->h_gl.abort) {
        b->poisoned = true;
        return fail(IM_ERR_DEVICE, "batched solve stopped: no tile was claimable for the watchdog period");
    }
    if (b->h_gl.jobs_done != (uint32_t)b->jobs.size()) {
        b->poisoned = true;
        return fail(IM_ERR_DEVICE, "batched solve ended with %u of %zu jobs done", b->h_gl.jobs_done, b->jobs.size());
    }
    b->ran = true;
    return IM_OK;
}

// Seeds of every job of the last replay, in batch order (for the autotuner's
// agreement check).
im_status all_seeds(im_batch* b, std::vector<int32_t>& out) {
    out.clear();
    for (auto& h : b->jobs) {
        std::vector<int32_t> s(h.K);
        BHIP(hipMemcpy(s.data(), h.dj.seeds, 4 * (size_t)h.K, hipMemcpyDeviceToHost));
        out.insert(out.end(), s.begin(), s.end());
    }
    return IM_OK;
}

}  // namespace

extern "C" {

im_status im_batch_create(im_ctx* ctx, int32_t count, const im_batch_job* jobs, const im_batch_opts* opts,
                          im_batch** out) {
    if (!ctx || !jobs || !out) return fail(IM_ERR_INVALID_ARG, "null argument");
    if (count < 1) return fail(IM_ERR_INVALID_ARG, "count must be >= 1");
    im_batch_opts o{};
    if (opts) o = *opts;
    if (o.lanes_per_row < 0 || o.tile_edges < 0 || o.heavy_degree < 0 || o.piece_edges < 0 || o.workgroups < 0)
        return fail(IM_ERR_INVALID_ARG, "negative tuning value");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(IM_ERR_DEVICE, "hipSetDevice failed");
    int Pmax = 1;
    for (int i = 0; i < count; ++i) {
        const im_batch_job& j = jobs[i];
        const int64_t n = j.graph.n, m = j.graph.m;
        if (j.R < 4 || j.R > 256 || j.R % 4)
            return fail(IM_ERR_INVALID_ARG, "job %d: R must be a multiple of 4 in [4, 256] (got %d)", i, j.R);
        if (n < 1 || n >= (1ll << 31)) return fail(IM_ERR_INVALID_GRAPH, "job %d: n must be in [1, 2^31)", i);
        if (m < 0 || m >= (1ll << 40)) return fail(IM_ERR_INVALID_GRAPH, "job %d: m out of range", i);
        if (!j.graph.xadj || (m > 0 && !j.graph.adj)) return fail(IM_ERR_INVALID_GRAPH, "job %d: null CSR array", i);
        if (const im_status oc = csr_offsets_check(&j.graph); oc != IM_OK) return oc;
        if (j.K < 1 || j.K > n) return fail(IM_ERR_INVALID_ARG, "job %d: K must be in [1, n]", i);
        const im_prob_kind pk = j.probs.kind;
        if (pk != IM_PROB_CONSTANT && pk != IM_PROB_WEIGHTED_CASCADE && pk != IM_PROB_PER_EDGE)
            return fail(IM_ERR_INVALID_ARG, "job %d: unknown probability kind", i);
        if (pk == IM_PROB_CONSTANT && live_threshold(j.probs.p) == 0xFFFFFFFFu)
            return fail(IM_ERR_INVALID_ARG, "job %d: probability must be in [0, 1]", i);
        if (pk == IM_PROB_PER_EDGE && m > 0 && !j.probs.per_edge)
            return fail(IM_ERR_INVALID_ARG, "job %d: per-edge probabilities missing", i);
        if (!(j.eps_c >= 0.0) || !(j.eps_g >= 0.0) || !(j.eps_l >= 0.0))
            return fail(IM_ERR_INVALID_ARG, "job %d: thresholds must be >= 0", i);
        Pmax = std::max(Pmax, j.R / 4);
    }
    const int Gmin = min_lanes(Pmax);
    if (o.lanes_per_row && (o.lanes_per_row < Gmin || o.lanes_per_row > 64 || (o.lanes_per_row & (o.lanes_per_row - 1))))
        return fail(IM_ERR_INVALID_ARG, "lanes_per_row must be a power of two in [%d, 64]", Gmin);

    im_batch* b = new im_batch;
    b->ctx = ctx;
    int cus = 0, clk_khz = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess ||
        hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess) {
        batch_release(b);
        return fail(IM_ERR_DEVICE, "device attribute query failed");
    }
    b->cus = cus > 0 ? cus : 256;
    // watchdog period: 4 s, or HFR_BATCH_TIMEOUT_MS (tests shorten it)
    unsigned long long timeout_ms = 4000;
    if (const char* e = getenv("HFR_BATCH_TIMEOUT_MS")) {
        const long long v = atoll(e);
        if (v > 0) timeout_ms = (unsigned long long)v;
    }
    b->timeout_ticks = (unsigned long long)(clk_khz > 0 ? clk_khz : 100000) * timeout_ms;
    b->cfg.G = o.lanes_per_row ? o.lanes_per_row : Gmin;
    if (o.tile_edges) b->cfg.tile_edges = o.tile_edges;
    if (o.heavy_degree) b->cfg.heavy_degree = o.heavy_degree;
    if (o.piece_edges) b->cfg.piece_edges = o.piece_edges;
    b->pin_request = o.pin_edges;
    b->cfg.workgroups = o.workgroups ? o.workgroups : 4 * b->cus;

    auto bail = [&](im_status st) {
        batch_release(b);
        return st;
    };
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&b->ev_in) != hipSuccess || hipEventCreate(&b->ev0) != hipSuccess ||
        hipEventCreate(&b->ev1) != hipSuccess)
        return bail(fail(IM_ERR_DEVICE, "stream or event creation failed"));
    hipStream_t s = b->stream;

    // host copies of the graphs (validation and tile tables)
    b->jobs.resize(count);
    for (int i = 0; i < count; ++i) {
        const im_batch_job& j = jobs[i];
        HostJob& h = b->jobs[i];
        h.index = i;
        h.n = j.graph.n;
        h.m = j.graph.m;
        h.J = j.R;
        h.P = j.R / 4;
        h.PW = (h.P + 31) / 32;
        h.K = j.K;
        h.xadj.resize(h.n + 1);
        h.adj.resize(h.m);
        const hipMemcpyKind kind = j.graph.on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
        if (csr_offsets_to_host(&j.graph, h.xadj.data()) != hipSuccess ||
            (h.m > 0 && hipMemcpy(h.adj.data(), j.graph.adj, 4 * h.m, kind) != hipSuccess))
            return bail(fail(IM_ERR_DEVICE, "job %d: reading the CSR failed", i));
        if (h.xadj[0] != 0 || h.xadj[h.n] != h.m)
            return bail(fail(IM_ERR_INVALID_GRAPH, "job %d: xadj[0] must be 0 and xadj[n] must equal m", i));
        for (int64_t u = 0; u < h.n; ++u)
            if (h.xadj[u] > h.xadj[u + 1]) return bail(fail(IM_ERR_INVALID_GRAPH, "job %d: xadj is not nondecreasing", i));
        for (int64_t e = 0; e < h.m; ++e)
            if (h.adj[e] < 0 || h.adj[e] >= h.n) return bail(fail(IM_ERR_INVALID_GRAPH, "job %d: adj holds an id outside [0, n)", i));
    }
    // XCDs that run waves: a probe launch records their ids
    uint32_t xmask = 0;
    {
        uint32_t* dmask = balloc<uint32_t>(b, 1);
        if (!dmask) return bail(fail(IM_ERR_OUT_OF_BUDGET, "device allocation failed"));
        if (hipMemsetAsync(dmask, 0, 4, s) != hipSuccess) return bail(fail(IM_ERR_DEVICE, "memset failed"));
        hipLaunchKernelGGL(k_xcc_probe, dim3(4 * b->cus), dim3(256), 0, s, dmask);
        if (hipGetLastError() != hipSuccess || hipMemcpyAsync(&xmask, dmask, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return bail(fail(IM_ERR_DEVICE, "XCD probe failed"));
    }
    std::vector<int> xccs;
    for (int x = 0; x < MAX_XCC; ++x)
        if (xmask & (1u << x)) xccs.push_back(x);
    if (xccs.empty()) return bail(fail(IM_ERR_DEVICE, "XCD probe found no XCD"));
    b->nxcc = (int)xccs.size();
    b->xccs = xccs;
    {
        // default: a job runs on one XCD unless it holds more than half of an
        // XCD's fair share of the batch's edges
        int64_t mtot = 0;
        for (const HostJob& h : b->jobs) mtot += h.m;
        const int64_t dflt = std::max<int64_t>(1 << 16, mtot / (2 * (int64_t)xccs.size()));
        b->cfg.pin_edges = b->pin_request > 0 ? b->pin_request : (b->pin_request < 0 ? -1 : dflt);
    }

    for (HostJob& h : b->jobs) {
        const im_batch_job& j = jobs[h.index];
        const int64_t n = h.n, m = h.m;
        const int P = h.P, W = 4 * h.PW;
        split_rows(h, b->cfg.heavy_degree, b->cfg.piece_edges);
        BJob& dj = h.dj;
        dj.n = n;
        dj.m = m;
        dj.J = h.J;
        dj.P = P;
        dj.PW = h.PW;
        dj.K = h.K;
        dj.seed = j.hash_seed;
        const double lim = floor(j.eps_c * (double)n);
        dj.thresh = lim >= (double)n ? (uint32_t)n : (uint32_t)lim;
        dj.eps_g = j.eps_g;
        dj.eps_l = j.eps_l;
        dj.heavy_deg = b->cfg.heavy_degree;
        dj.nheavy = (int64_t)h.hrow.size();
        dj.npieces = (int64_t)h.pe0.size();
        const int64_t qcap = n + (m + BFS_CHUNK_B - 1) / BFS_CHUNK_B + 64;
        const int64_t words = (n + 31) / 32 + 1;
        h.rtile_cap = (n + 31) / 32 + 2;
        int64_t* xadj = balloc<int64_t>(b, n + 1);
        int32_t* adj = balloc<int32_t>(b, m);
        dj.eh = balloc<uint32_t>(b, m);
        double* T = balloc<double>(b, h.J);
        h.d_rtile = balloc<int32_t>(b, h.rtile_cap);
        int32_t* hrow = balloc<int32_t>(b, h.hrow.size());
        int64_t* hpb = balloc<int64_t>(b, h.hpb.size());
        int64_t* hpn = balloc<int64_t>(b, h.hpn.size());
        int32_t* prow = balloc<int32_t>(b, h.prow.size());
        int64_t* pe0 = balloc<int64_t>(b, h.pe0.size());
        int64_t* pe1 = balloc<int64_t>(b, h.pe1.size());
        dj.part = balloc<uint32_t>(b, (size_t)dj.npieces * P);
        dj.part_any = balloc<uint32_t>(b, dj.npieces);
        for (int k = 0; k < 3; ++k) dj.M[k] = balloc<uint32_t>(b, (size_t)n * P);
        dj.Lb[0] = balloc<uint32_t>(b, words);
        dj.Lb[1] = balloc<uint32_t>(b, words);
        dj.blk = balloc<uint32_t>(b, (size_t)n * W);
        dj.F[0] = balloc<uint32_t>(b, (size_t)n * W);
        dj.F[1] = balloc<uint32_t>(b, (size_t)n * W);
        dj.Q[0] = balloc<int2>(b, qcap);
        dj.Q[1] = balloc<int2>(b, qcap);
        dj.stamp = balloc<int32_t>(b, n);
        dj.inS = balloc<uint8_t>(b, n);
        dj.MS = balloc<uint32_t>(b, P);
        dj.merged = balloc<uint32_t>(b, P);
        dj.steps = balloc<StepRec>(b, h.K);
        dj.seeds = balloc<int32_t>(b, h.K);
        dj.ctl = balloc<BCtl>(b, 1);
        uint32_t* thr = nullptr;
        uint32_t* indeg = nullptr;
        if (j.probs.kind == IM_PROB_WEIGHTED_CASCADE) {
            thr = balloc<uint32_t>(b, n);
            indeg = balloc<uint32_t>(b, n);
        } else if (j.probs.kind == IM_PROB_PER_EDGE) {
            thr = balloc<uint32_t>(b, m);
        }
        bool ok = xadj && adj && dj.eh && T && h.d_rtile && hrow && hpb && hpn && prow && pe0 && pe1 && dj.part &&
                  dj.part_any && dj.M[0] && dj.M[1] && dj.M[2] && dj.Lb[0] && dj.Lb[1] && dj.blk && dj.F[0] &&
                  dj.F[1] && dj.Q[0] && dj.Q[1] && dj.stamp && dj.inS && dj.MS && dj.merged && dj.steps && dj.seeds &&
                  dj.ctl && (j.probs.kind == IM_PROB_CONSTANT || thr) &&
                  (j.probs.kind != IM_PROB_WEIGHTED_CASCADE || indeg);
        if (!ok || (ctx->budget && ctx->in_use > ctx->budget))
            return bail(fail(IM_ERR_OUT_OF_BUDGET, "batch needs more device memory than the context allows"));
        dj.xadj = xadj;
        dj.adj = adj;
        dj.T = T;
        dj.rtile = h.d_rtile;
        dj.hrow = hrow;
        dj.hpb = hpb;
        dj.hpn = hpn;
        dj.prow = prow;
        dj.pe0 = pe0;
        dj.pe1 = pe1;
        dj.thr = thr;
        dj.indeg = indeg;
        // queue entries always name a vertex, even before they are first written
        if (hipMemsetAsync(dj.Q[0], 0, 8 * qcap, s) != hipSuccess || hipMemsetAsync(dj.Q[1], 0, 8 * qcap, s) != hipSuccess)
            return bail(fail(IM_ERR_DEVICE, "queue initialisation failed"));
        if (hipMemcpyAsync(xadj, h.xadj.data(), 8 * (n + 1), hipMemcpyHostToDevice, s) != hipSuccess ||
            (m > 0 && hipMemcpyAsync(adj, h.adj.data(), 4 * m, hipMemcpyHostToDevice, s) != hipSuccess))
            return bail(fail(IM_ERR_DEVICE, "CSR upload failed"));
        std::vector<double> Th(h.J);
        for (int r = 0; r < h.J; ++r) Th[r] = exp2((double)r / (double)h.J);
        auto up = [&](void* dst, const void* src, size_t bytes) {
            return bytes == 0 || hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
        };
        ok = up(T, Th.data(), 8 * Th.size()) && up(hrow, h.hrow.data(), 4 * h.hrow.size()) &&
             up(hpb, h.hpb.data(), 8 * h.hpb.size()) && up(hpn, h.hpn.data(), 8 * h.hpn.size()) &&
             up(prow, h.prow.data(), 4 * h.prow.size()) && up(pe0, h.pe0.data(), 8 * h.pe0.size()) &&
             up(pe1, h.pe1.data(), 8 * h.pe1.size());
        std::vector<uint32_t> tmp;
        if (j.probs.kind == IM_PROB_CONSTANT) {
            dj.kind = THR_CONST;
            dj.thr_const = live_threshold(j.probs.p);
        } else if (j.probs.kind == IM_PROB_WEIGHTED_CASCADE) {
            dj.kind = THR_TARGET;
            tmp.assign(n, 0u);
            for (int64_t e = 0; e < m; ++e) tmp[h.adj[e]] += 1u;
            ok = ok && up(indeg, tmp.data(), 4 * tmp.size());
        } else {
            dj.kind = THR_EDGE;
            std::vector<float> w(m);
            const hipMemcpyKind kind = j.graph.on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
            if (m > 0 && hipMemcpy(w.data(), j.probs.per_edge, 4 * m, kind) != hipSuccess)
                return bail(fail(IM_ERR_DEVICE, "reading per-edge probabilities failed"));
            tmp.resize(m);
            for (int64_t e = 0; e < m; ++e) {
                tmp[e] = live_threshold(w[e]);
                if (tmp[e] == 0xFFFFFFFFu)
                    return bail(fail(IM_ERR_INVALID_ARG, "job %d: a per-edge probability is outside [0, 1]", h.index));
            }
            ok = ok && up(thr, tmp.data(), 4 * tmp.size());
        }
        if (!ok || hipStreamSynchronize(s) != hipSuccess) return bail(fail(IM_ERR_DEVICE, "upload failed"));
    }
    b->d_jobs = balloc<BJob>(b, count);
    b->d_gl = balloc<BGlobal>(b, 1);
    if (!b->d_jobs || !b->d_gl || (ctx->budget && ctx->in_use > ctx->budget))
        return bail(fail(IM_ERR_OUT_OF_BUDGET, "batch needs more device memory than the context allows"));

    im_status st = IM_OK;
    if (o.autotune) {
        // every candidate decomposition solves the batch once; the fastest is
        // kept and all of them must agree on every seed
        // lanes per row (registers per lane): the smallest power of two covering a
        // row, and twice that (fewer registers per lane, fewer rows per wave)
        std::vector<BatchCfg> cands;
        std::vector<int> lanes = o.lanes_per_row ? std::vector<int>{o.lanes_per_row} : std::vector<int>{Gmin};
        if (!o.lanes_per_row && 2 * Gmin <= 64) lanes.push_back(2 * Gmin);
        std::vector<int> tiles = o.tile_edges ? std::vector<int>{o.tile_edges} : std::vector<int>{4096, 8192};
        std::vector<int64_t> pins = o.pin_edges ? std::vector<int64_t>{b->cfg.pin_edges}
                                                : std::vector<int64_t>{b->cfg.pin_edges, -1};
        std::vector<int> wgs = o.workgroups ? std::vector<int>{o.workgroups} : std::vector<int>{2 * b->cus, 4 * b->cus};
        for (int G : lanes)
            for (int te : tiles)
                for (int64_t pe : pins)
                    for (int wg : wgs) {
                        BatchCfg c = b->cfg;
                        c.G = G;
                        c.tile_edges = te;
                        c.pin_edges = pe;
                        c.workgroups = wg;
                        cands.push_back(c);
                    }
        float best = 1e30f;
        BatchCfg best_cfg = b->cfg;
        std::vector<int32_t> ref, cur;
        for (const BatchCfg& c : cands) {
            b->cfg = c;
            if ((st = upload_tiles(b)) != IM_OK || (st = capture(b)) != IM_OK) return bail(st);
            float ms = 0.f;
            if ((st = replay(b, &ms)) != IM_OK || (st = all_seeds(b, cur)) != IM_OK) return bail(st);
            if (ref.empty())
                ref = cur;
            else if (cur != ref)
                return bail(fail(IM_ERR_DEVICE, "decompositions disagree on the seeds"));
            if (ms < best) {
                best = ms;
                best_cfg = c;
            }
        }
        b->candidates = (int)cands.size();
        b->cfg = best_cfg;
    }
    if ((st = upload_tiles(b)) != IM_OK || (st = capture(b)) != IM_OK) return bail(st);
    b->ran = false;
    *out = b;
    return IM_OK;
}

im_status im_batch_run(im_batch* b, im_batch_stats* stats) {
    if (!b) return fail(IM_ERR_INVALID_ARG, "null batch");
    if (b->poisoned) return fail(IM_ERR_STATE, "batch is poisoned by an earlier device error");
    if (hipSetDevice(b->ctx->device) != hipSuccess) return fail(IM_ERR_DEVICE, "hipSetDevice failed");
    const auto w0 = std::chrono::steady_clock::now();
    float ms = 0.f;
    im_status st = replay(b, &ms);
    if (st != IM_OK) return st;
    if (stats) {
        stats->device_ms = ms;
        stats->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - w0).count();
        stats->tiles = (int64_t)b->h_gl.tiles;
        stats->phases = (int64_t)b->h_gl.phases;
        stats->lanes_per_row = b->cfg.G;
        stats->tile_edges = b->cfg.tile_edges;
        stats->heavy_degree = b->cfg.heavy_degree;
        stats->piece_edges = b->cfg.piece_edges;
        stats->workgroups = b->grid;
        stats->candidates = b->candidates;
    }
    return IM_OK;
}

im_status im_batch_get_result(const im_batch* b, int32_t job, int32_t* out_seeds, im_step* out_steps,
                              im_batch_job_result* res) {
    if (!b) return fail(IM_ERR_INVALID_ARG, "null batch");
    if (job < 0 || job >= (int32_t)b->jobs.size()) return fail(IM_ERR_INVALID_ARG, "job index out of range");
    if (!b->ran) return fail(IM_ERR_STATE, "the batch has not run");
    const HostJob& h = b->jobs[job];
    const BCtl& c = b->h_ctl[job];
    if (res) {
        res->status = c.r.status;
        res->build_sweeps = (int32_t)c.r.build_sweeps;
        res->rebuilds = (int32_t)c.r.rebuilds;
        res->reserved = 0;
        res->build_visits = (int64_t)c.r.build_visits;
        res->rebuild_sweeps = (int64_t)c.r.rebuild_sweeps;
        res->rebuild_visits = (int64_t)c.r.rebuild_visits;
        res->bfs_levels = (int64_t)c.r.bfs_levels;
    }
    if (out_seeds && hipMemcpy(out_seeds, h.dj.seeds, 4 * (size_t)h.K, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(IM_ERR_DEVICE, "copying seeds failed");
    if (out_steps) {
        std::vector<StepRec> rec(h.K);
        if (hipMemcpy(rec.data(), h.dj.steps, sizeof(StepRec) * h.K, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(IM_ERR_DEVICE, "copying steps failed");
        for (int k = 0; k < h.K; ++k) {
            const StepRec& r = rec[k];
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
    return c.r.status == 0 ? IM_OK : fail((im_status)c.r.status, "job %d stopped with a device-side error", job);
}

im_status im_batch_get_registers(const im_batch* b, int32_t job, int32_t which, uint8_t* out) {
    if (!b || !out) return fail(IM_ERR_INVALID_ARG, "null argument");
    if (job < 0 || job >= (int32_t)b->jobs.size()) return fail(IM_ERR_INVALID_ARG, "job index out of range");
    if (which != 0 && which != 1) return fail(IM_ERR_INVALID_ARG, "which must be 0 or 1");
    if (!b->ran) return fail(IM_ERR_STATE, "the batch has not run");
    const HostJob& h = b->jobs[job];
    const BCtl& c = b->h_ctl[job];
    const int buf = which == 0 ? c.d.build_buf : (int)c.r.sel_buf;
    if (buf < 0 || buf > 2) return fail(IM_ERR_STATE, "no registers recorded");
    if (hipMemcpy(out, h.dj.M[buf], (size_t)h.n * h.J, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(IM_ERR_DEVICE, "copying registers failed");
    return IM_OK;
}

size_t im_batch_device_bytes(const im_batch* b) { return b ? b->bytes : 0; }

void im_batch_free(im_batch* b) { batch_release(b); }

}  // extern "C"
