// Internal interface between the host side of the library (hfr_api.hip) and
// its gfx950 kernels (hfr_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hfr {

// Spread counters: atomics from many blocks land on NSLOT distinct 128-byte
// lines instead of one address; readers sum the slots.
constexpr int NSLOT = 32;
constexpr int SLOT_U32 = 32;  // u32 stride between slots (128 B)
constexpr int SLOT_U64 = 16;  // u64 stride between slots (128 B)

// Register layout: a vertex row holds J one-byte registers = P = J/4 dwords.
// A wave serves 64/G rows at once (G lanes per row, DW dwords per lane, lane p
// of a row owns dwords q = i*G + p, i < DW).  The blocked bits of a vertex are
// 4 planes of PW dwords: plane k holds bit q for register 4q+k.
struct Layout {
    int J;
    int P;   // dwords per row
    int PW;  // dwords per blocked-bit plane
    int G;   // lanes per row
    int DW;  // dwords per lane
};

Layout make_layout(int J);

enum ThrKind { THR_CONST = 0, THR_TARGET = 1, THR_EDGE = 2 };

struct DevGraph {
    int64_t n = 0, m = 0;
    int64_t* xadj = nullptr;
    int32_t* adj = nullptr;   // the sketch's copy; DEAD_EDGE may be set once the sweeps' inputs are final
    uint32_t* eh = nullptr;   // 31-bit edge hash per edge, held during preparation only (null: the
                              // kernels recompute the hash of (u, v) from hseed)
    uint32_t hseed = 0;       // hash seed
    uint32_t* thr = nullptr;  // per target vertex (WC) or per edge
    uint32_t thr_const = 0;
    int kind = THR_CONST;
    // rows split across waves
    int64_t heavy_deg = 0;
    int64_t nheavy = 0, npieces = 0;
    int32_t* hrow = nullptr;    // heavy row ids [nheavy]
    int64_t* hpb = nullptr;     // first piece of each heavy row [nheavy]
    int64_t* hpn = nullptr;     // number of pieces of each heavy row [nheavy]
    int32_t* prow = nullptr;    // row of each piece [npieces]
    int64_t* pe0 = nullptr;     // first edge of each piece
    int64_t* pe1 = nullptr;     // one past the last edge of each piece
    // in-edges (reverse CSR), for sweeps that start from the live vertices
    int64_t* rxadj = nullptr;   // [n + 1]
    int2* rrec = nullptr;       // [m] per in-edge: x = source id (DEAD_EDGE set when the edge is live
                                // in no sample), y = for a split source row its 64-edge window,
                                // piece * wpp + window in the piece (wpp = ceil(piece_edges / 64)),
                                // -1 otherwise; one 8-byte record, written once and read together
    int32_t* hslot = nullptr;   // heavy slot of each row, -1 for rows processed whole [n]
    int32_t* lrows = nullptr;   // rows with 1..heavy_deg out-edges, ascending [nlight]
    int64_t nlight = 0;
    int64_t piece_edges = 256;
};

// Flag in bit 31 of an edge's target id (ids are below 2^31): the edge is live in
// none of the J samples (no j with (X_j xor h) < its threshold), so no merge or
// reach step needs the head's row.  Every reader of the id masks it off (adj_target);
// a graph without flags merges as usual.
constexpr uint32_t DEAD_EDGE = 0x80000000u;
__host__ __device__ inline int32_t adj_target(int32_t a) { return a & 0x7FFFFFFF; }
__host__ __device__ inline bool adj_dead(int32_t a) { return a < 0; }

constexpr int COARSE_WORDS = 2048;  // coarse copy of L_t: 8 KiB of LDS per workgroup
// Reach levels: workgroups of 256 per launch, and the queue slots a wave reserves at
// a time (the queue holds up to BFS_WAVES * BFS_RESV slots beyond its entries).
constexpr int BFS_GRID = 2048;
constexpr int BFS_WAVES = BFS_GRID * 4;
constexpr int BFS_RESV = 64;

// Work lists of a sparse sweep.  Counters come in two sets selected by the
// sweep parity; a sweep zeroes the other set for the next sweep.
struct Frontier {
    uint32_t* mark = nullptr;   // n bits: rows to merge in a sparse sweep; zero outside one
    int2* items = nullptr;      // (live vertex, chunk of its in-edges)
    int32_t* W = nullptr;       // the marked rows, listed (split rows among them are skipped)
    uint32_t* counts = nullptr; // [2][4]: items and W of the sweep of each parity (rest unused)
    uint32_t* wmask = nullptr;  // per piece: its 64-edge windows holding an edge into L_t; zero
                                // outside a sparse sweep
    uint32_t* coarse = nullptr; // coarse copy of L_t for dense sweeps with few live vertices: bit c set
                                // iff a vertex of [c << coarse_shift, (c + 1) << coarse_shift) is in L_t
    int32_t coarse_shift = 8;   // so that the copy has at most COARSE_WORDS words
    int32_t coarse_words = 0;
    uint32_t coarse_live = 0;   // largest |L_t| for which the copy is built and used (0: never)
    uint32_t stamp = 0;         // unique per sweep (never 0): piece flags of this sweep
    int32_t chunk = 256;        // in-edges per item
    uint32_t sparse_div = 8;    // sweep t > 0 is sparse iff S_t * sparse_div <= m (0: never)
};

// Per-sweep launch parameters.
struct SweepParams {
    const uint32_t* A;  // registers M^t
    uint32_t* B;        // registers M^{t+1}
    const uint32_t* Lcur;
    uint32_t* Lnext;
    const uint32_t* blk;       // nullptr when no pair is blocked
    const uint32_t* gate;      // live-count slots of L_t (nullptr on the first sweep)
    uint32_t gate_thresh;      // sweep runs iff |L_t| > gate_thresh
    uint32_t* cnt_out;         // slots of |L_{t+1}|
    unsigned long long* vis_out;        // slots: edges with a live head visited by the row kernel
    unsigned long long* vis_heavy_out;  // slots: edges with a live head visited by the split-row kernel
    uint32_t* part;            // partial rows of split-row pieces [npieces * P]
    uint32_t* part_any;        // per piece: 1 if some live edge was merged
    uint32_t* Lclear;          // bitmap of L_{t-1}, zeroed during this sweep for L_{t+2}
    const unsigned long long* sgate;  // slots of S_t = sum of in-degrees over L_t (nullptr on the first sweep)
    unsigned long long* sum_out;      // slots of S_{t+1}
    const uint32_t* fullblk;   // n bits: vertex blocked in every sample (nullptr with blk)
    uint32_t* rtouch;          // per split row: serial of the last sweep that merged one of its pieces
    Frontier fr;
    int parity;                // t & 1
    int first;
};

struct GreedyBufs {
    uint32_t* blk;     // n * 4 * PW
    uint32_t* fullblk; // n bits: blocked in every sample
    uint32_t* F[2];    // frontier bits, same shape as blk
    int2* Q[2];        // queue entries (vertex, chunk)
    uint32_t* qsize;   // 3 ring counters (+ level counter at [3])
    int32_t* stamp;    // last level a vertex was queued for
    uint8_t* inS;      // n
    uint32_t* MS;      // P dwords: M_S'
    uint32_t* merged;  // P dwords: Merge(M_S', M_s)
    unsigned long long* key;   // argmax key
    unsigned long long* R;     // reach slots
    unsigned long long* Rreb;  // reach at the last rebuild
    double* T;         // exp2(r/J), r < J
    int64_t qcap;
    int32_t bfs_chunk;
};

// Device-side record of one greedy step (mirrors im_step).
struct StepRec {
    int32_t seed, rebuilt, fresh, sweeps;
    int64_t score, reach;
    double e, sigma, delta, err_l, err_g;
    int64_t visits;
};

// ---- launchers (hfr_kernels.hip) ----
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t s);
hipError_t launch_validate(const DevGraph& g, uint32_t* err, hipStream_t s);
hipError_t launch_edge_hash(const DevGraph& g, uint32_t seed, hipStream_t s);
hipError_t launch_indegree(const DevGraph& g, uint32_t* indeg, hipStream_t s);
hipError_t launch_wc_thresholds(const uint32_t* indeg, uint32_t* thr, int64_t n, hipStream_t s);
hipError_t launch_gather_u32(const uint32_t* src, const int32_t* idx, int64_t m, uint32_t* out, hipStream_t s);
hipError_t launch_edge_thresholds(const float* w, uint32_t* thr, int64_t m, uint32_t* err, hipStream_t s);
hipError_t launch_sim_words(uint32_t* X, uint32_t* HJ, int J, uint32_t seed, hipStream_t s);
hipError_t launch_widen_offsets(const int32_t* src, int64_t* dst, int64_t count, hipStream_t s);

// Sets DEAD_EDGE in the target id of every edge live in no sample (thresholds final).
hipError_t launch_dead_edges(const DevGraph& g, const uint32_t* X, int J, hipStream_t s);
hipError_t launch_heavy_count(const DevGraph& g, int64_t piece_edges, unsigned long long* counts, hipStream_t s);
hipError_t launch_heavy_assign(const DevGraph& g, int64_t piece_edges, unsigned long long* counts, hipStream_t s);
hipError_t launch_heavy_pieces(const DevGraph& g, int64_t piece_edges, hipStream_t s);
hipError_t launch_init(const Layout& L, int64_t n, const uint32_t* HJ, uint32_t seed, const uint32_t* blk,
                       uint32_t* A, uint32_t* B, hipStream_t s);
hipError_t launch_sweep(const Layout& L, const DevGraph& g, const uint32_t* X, const SweepParams& sp, int grid,
                        hipStream_t s, hipEvent_t ev_light_begin, hipEvent_t ev_light_end,
                        hipEvent_t ev_heavy_begin, hipEvent_t ev_heavy_end);
hipError_t launch_reverse_csr(const DevGraph& g, const uint32_t* indeg, int64_t* cursor, uint32_t* scan_tmp,
                              hipStream_t s);
// Reverse CSR and in-degrees by a counting sort on the target, on one stream
// (graphs with n <= 2^25 and m < 2^31: rb_fits).
bool rb_fits(int64_t n, int64_t m);
size_t rb_temp_bytes(int64_t n, int64_t m);
// Edge-liveness test applied to the reverse CSR's records as they are placed:
// mode 0 none, 1 constant threshold thr_const, 2 weighted cascade (1/indeg(v)).
struct DeadTest {
    const uint32_t* X;  // J sample words
    int J;
    uint32_t seed;
    uint32_t thr_const;
    int mode;
};
hipError_t launch_reverse_csr_buckets(const DevGraph& g, void* tmp, uint32_t** indeg, const DeadTest& dt,
                                      hipStream_t s);
hipError_t launch_heavy_slots(const DevGraph& g, hipStream_t s);
hipError_t launch_light_rows(const DevGraph& g, uint32_t* flags, int64_t* pos, uint32_t* scan_tmp, hipStream_t s);
hipError_t launch_full_blocked(const Layout& L, int64_t n, const uint32_t* blk, uint32_t* fullblk, hipStream_t s);
hipError_t launch_argmax(const Layout& L, int64_t n, const uint32_t* M, const GreedyBufs& b, hipStream_t s);
hipError_t launch_select(const Layout& L, const DevGraph& g, const uint32_t* M, const GreedyBufs& b,
                         StepRec* rec, int32_t* seeds_dev, int k, int32_t level_id, hipStream_t s);
hipError_t launch_bfs_level(const Layout& L, const DevGraph& g, const uint32_t* X, const GreedyBufs& b, int level,
                            int32_t level_id_next, int grid, hipStream_t s);
hipError_t launch_reach_start(const Layout& L, const DevGraph& g, const GreedyBufs& b, const int32_t* verts,
                              int count, int32_t level_id, hipStream_t s);
hipError_t launch_decide(const Layout& L, const GreedyBufs& b, StepRec* rec, int k, int K, double eps_g,
                         double eps_l, int32_t* rebuild_flag, hipStream_t s);
hipError_t launch_estimate_all(const Layout& L, int64_t n, const uint32_t* M, const double* T, float* out,
                               hipStream_t s);
hipError_t launch_estimate_set(const Layout& L, const uint32_t* M, const int32_t* verts, int64_t count,
                               const double* T, float* out, hipStream_t s);
hipError_t launch_blocked_to_bytes(const Layout& L, int64_t n, const uint32_t* blk, uint8_t* out, hipStream_t s);

// Integer live threshold of a binary32 weight: the number of 31-bit integers
// x with x < w * (2^31 - 1); 0xFFFFFFFF when w is not in [0, 1].
__host__ __device__ inline uint32_t live_threshold(float w) {
    if (!(w >= 0.0f && w <= 1.0f)) return 0xFFFFFFFFu;
    uint32_t bits = __builtin_bit_cast(uint32_t, w);
    uint32_t ex = (bits >> 23) & 0xFFu;
    uint64_t mant = bits & 0x7FFFFFu;
    int sh;
    if (ex == 0) {
        sh = 149;
    } else {
        mant |= 1ull << 23;
        sh = 150 - (int)ex;
    }
    if (mant == 0) return 0u;
    uint64_t prod = mant * 2147483647ull;  // < 2^55
    if (sh >= 64) return 1u;
    uint64_t q = prod >> sh;
    return (uint32_t)(q + ((prod & ((1ull << sh) - 1)) != 0));
}

}  // namespace hfr
