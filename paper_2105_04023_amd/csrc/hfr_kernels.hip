// gfx950 kernels of the sketch-based influence-maximisation path
// (Gokturk & Kaya, arXiv 2105.04023).
//
// Registers are one byte per (vertex, simulation), vertex-major, packed four
// to a dword (Sec. 3.3: the registers of one vertex are adjacent).  A row of
// J registers is P = J/4 dwords; G lanes serve one row, so a 64-wide wave
// reads a neighbour's row with coalesced dword loads (J = 256: one row per
// wave, one dword per lane).
//
// The sweep is pull-based (Sec. 4.5): a row u is only written by the wave
// that owns it, so no register needs an atomic.  Sampling is fused (Sec.
// 3.1): an edge's 31-bit hash h is loaded once per visit and every lane tests
// its four simulations with (X_j xor h) < thr, branch-free.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hfr_device.h"
#include "hfr_internal.h"

namespace hfr {

// Edge hashes of a graph for the kernels: its array while it exists (preparation),
// else recomputed from (u, v) and the seed.
static inline EdgeHashes hashes(const DevGraph& g) { return EdgeHashes{g.eh, g.hseed}; }

// ----------------------------------------------------------------------------
// Utilities and graph preparation.
// ----------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, v, count);
    return hipGetLastError();
}

// err bit 1: offsets decrease; bit 2: an id is out of range.
__global__ void k_validate(const int64_t* __restrict__ xadj, const int32_t* __restrict__ adj, int64_t n, int64_t m,
                           uint32_t* err) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    uint32_t bad = 0;
    for (int64_t u = tid; u < n; u += stride)
        if (xadj[u] > xadj[u + 1]) bad |= 1u;
    for (int64_t e = tid; e < m; e += stride) {
        int32_t v = adj[e];
        if (v < 0 || (int64_t)v >= n) bad |= 2u;
    }
    if (bad) atomicOr(err, bad);
}

hipError_t launch_validate(const DevGraph& g, uint32_t* err, hipStream_t s) {
    hipLaunchKernelGGL(k_validate, dim3(4096), dim3(256), 0, s, g.xadj, g.adj, g.n, g.m, err);
    return hipGetLastError();
}

// Calls f(u, e) once for every out-edge e of every row u with at most
// heavy_deg out-edges, on the lane that owns it (lanes diverge around the
// call).  A wave takes 64 consecutive rows at a time and walks their edges as
// one flat range, 64 per window; the row of a flat edge is found by a binary
// search over the rows' starts, held one per lane.
template <class F>
DEVI void for_light_edges(const int64_t* __restrict__ xadj, int64_t n, int64_t heavy_deg, F&& f) {
    const int lane = threadIdx.x & 63;
    for (int64_t u0 = wave_index() * 64; u0 < n; u0 += wave_count() * 64) {
        const int nr = n - u0 < 64 ? (int)(n - u0) : 64;
        const int64_t u = u0 + (lane < nr ? lane : nr - 1);
        const int64_t rb = xadj[u], re = xadj[u + 1];
        const int64_t len = (lane < nr && re - rb <= heavy_deg) ? re - rb : 0;
        // flat offsets of the light edges of the chunk
        int64_t off = len;
#pragma unroll
        for (int k = 1; k < 64; k <<= 1) {
            const int64_t o = __shfl_up(off, k, 64);
            if (lane >= k) off += o;
        }
        const int64_t total = __shfl(off, 63, 64);
        const int64_t start = off - len;  // exclusive prefix
        for (int64_t base = 0; base < total; base += 64) {
            const int64_t f_ = base + lane;
            int lo = 0, hi = nr - 1;  // largest row i with start_i <= f_
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const int mid = (lo + hi + 1) >> 1;
                const int64_t sm = __shfl(start, mid, 64);
                if (lo < hi) {
                    if (sm <= f_)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
            }
            const int64_t e = __shfl(rb, lo, 64) + (f_ - __shfl(start, lo, 64));
            if (f_ < total) f(u0 + lo, e);
        }
    }
}

// Calls f(u, e, pc, b0) once for every edge e of every piece pc (of split row
// u, edges [b0, pe1[pc])); one wave per piece.
template <class F>
DEVI void for_piece_edges(const int32_t* __restrict__ hrow, const int32_t* __restrict__ prow,
                          const int64_t* __restrict__ pe0, const int64_t* __restrict__ pe1, int64_t npieces, F&& f) {
    const int lane = threadIdx.x & 63;
    for (int64_t pc = wave_index(); pc < npieces; pc += wave_count()) {
        const int64_t u = hrow[prow[pc]];
        const int64_t b0 = pe0[pc], e1 = pe1[pc];
        for (int64_t e = b0 + lane; e < e1; e += 64) f(u, e, pc, b0);
    }
}

// Eq. (hash): h(u, v) = Murmur3(LE32(u) || LE32(v)) mod 2^31, in two balanced
// parts: the rows with at most heavy_deg out-edges, then the pieces of the
// split rows.
__global__ void k_edge_hash_light(const int64_t* __restrict__ xadj, const int32_t* __restrict__ adj, uint32_t* eh,
                                  int64_t n, int64_t heavy_deg, uint32_t seed) {
    for_light_edges(xadj, n, heavy_deg, [&](int64_t u, int64_t e) {
        eh[e] = mm3_key8((uint32_t)u, (uint32_t)adj[e], seed) & 0x7FFFFFFFu;
    });
}

__global__ void k_edge_hash_pieces(const int32_t* __restrict__ adj, const int32_t* __restrict__ hrow,
                                   const int32_t* __restrict__ prow, const int64_t* __restrict__ pe0,
                                   const int64_t* __restrict__ pe1, int64_t npieces, uint32_t* eh, uint32_t seed) {
    for_piece_edges(hrow, prow, pe0, pe1, npieces, [&](int64_t u, int64_t e, int64_t, int64_t) {
        eh[e] = mm3_key8((uint32_t)u, (uint32_t)adj[e], seed) & 0x7FFFFFFFu;
    });
}

hipError_t launch_edge_hash(const DevGraph& g, uint32_t seed, hipStream_t s) {
    hipLaunchKernelGGL(k_edge_hash_light, dim3(8192), dim3(256), 0, s, g.xadj, g.adj, g.eh, g.n, g.heavy_deg, seed);
    if (g.npieces > 0)
        hipLaunchKernelGGL(k_edge_hash_pieces, dim3(8192), dim3(256), 0, s, g.adj, g.hrow, g.prow, g.pe0, g.pe1,
                           g.npieces, g.eh, seed);
    return hipGetLastError();
}

// In-degrees.  R-MAT-like graphs put their highest in-degrees on the lowest
// ids, so the counts of ids below HOT_IDS are first gathered per block in LDS.
constexpr int HOT_IDS = 8192;

__global__ __launch_bounds__(256) void k_indegree(const int32_t* __restrict__ adj, int64_t m, int64_t n,
                                                  uint32_t* indeg) {
    __shared__ uint32_t hot[HOT_IDS];
    for (int i = threadIdx.x; i < HOT_IDS; i += blockDim.x) hot[i] = 0u;
    __syncthreads();
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = adj_target(adj[e]);
        if (v < HOT_IDS)
            atomicAdd(&hot[v], 1u);
        else
            atomicAdd(&indeg[v], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < HOT_IDS && i < n; i += blockDim.x)
        if (hot[i]) atomicAdd(&indeg[i], hot[i]);
}

hipError_t launch_indegree(const DevGraph& g, uint32_t* indeg, hipStream_t s) {
    if (g.m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_indegree, dim3(1024), dim3(256), 0, s, g.adj, g.m, g.n, indeg);
    return hipGetLastError();
}

__global__ void k_wc_thresholds(const uint32_t* __restrict__ indeg, uint32_t* thr, int64_t n) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        thr[v] = wc_threshold(indeg[v]);
}

// out[e] = src[idx[e]].
__global__ void k_gather_u32(const uint32_t* __restrict__ src, const int32_t* __restrict__ idx, int64_t m,
                             uint32_t* out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = src[idx[e]];
}

hipError_t launch_gather_u32(const uint32_t* src, const int32_t* idx, int64_t m, uint32_t* out, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_u32, dim3(8192), dim3(256), 0, s, src, idx, m, out);
    return hipGetLastError();
}

hipError_t launch_wc_thresholds(const uint32_t* indeg, uint32_t* thr, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_wc_thresholds, dim3(4096), dim3(256), 0, s, indeg, thr, n);
    return hipGetLastError();
}

__global__ void k_edge_thresholds(const float* __restrict__ w, uint32_t* thr, int64_t m, uint32_t* err) {
    uint32_t bad = 0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t t = live_threshold(w[e]);
        if (t == 0xFFFFFFFFu) bad = 4u;
        thr[e] = t;
    }
    if (bad) atomicOr(err, bad);
}

hipError_t launch_edge_thresholds(const float* w, uint32_t* thr, int64_t m, uint32_t* err, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_edge_thresholds, dim3(4096), dim3(256), 0, s, w, thr, m, err);
    return hipGetLastError();
}

// X_j = Murmur3(LE32(j), seed+2) mod 2^31 (per-simulation word of Eq.
// hash_prob); HJ_j = Murmur3(LE32(j), seed+3) (hash(j) of the register init).
__global__ void k_sim_words(uint32_t* X, uint32_t* HJ, int J, uint32_t seed) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < J) {
        X[j] = mm3_key4((uint32_t)j, seed + 2u) & 0x7FFFFFFFu;
        HJ[j] = mm3_key4((uint32_t)j, seed + 3u);
    }
}

// int32 CSR offsets widened to the library's int64 copy.
__global__ void k_widen_offsets(const int32_t* __restrict__ src, int64_t* __restrict__ dst, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (int64_t)src[i];
}

hipError_t launch_widen_offsets(const int32_t* src, int64_t* dst, int64_t count, hipStream_t s) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_widen_offsets, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, count);
    return hipGetLastError();
}

hipError_t launch_sim_words(uint32_t* X, uint32_t* HJ, int J, uint32_t seed, hipStream_t s) {
    hipLaunchKernelGGL(k_sim_words, dim3((J + 255) / 256), dim3(256), 0, s, X, HJ, J, seed);
    return hipGetLastError();
}

// Marks the edges live in no sample: with h the edge's hash and t its
// threshold, the edge is live in sample j iff (X_j xor h) < t (Sec. 3.1), so it is
// dead in all J iff min_j (X_j xor h) >= t.  The sample words are read at
// wave-uniform addresses, four at a time (J is a multiple of 4), each load
// serving four edges per lane; a wave stops scanning samples once every edge
// it holds has one in which it is live.
__global__ __launch_bounds__(256) void k_dead_edges(int32_t* __restrict__ adj, const uint32_t* __restrict__ eh,
                                                    const uint32_t* __restrict__ thr,
                                                    uint32_t thr_const, int per_edge, const uint32_t* __restrict__ X,
                                                    int J, int64_t m) {
    constexpr int EPT = 4;  // edges per lane (e0 + 256 k): one load of sample words serves EPT edges
    const int64_t step = (int64_t)gridDim.x * blockDim.x * EPT;
    for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x * EPT + threadIdx.x; e0 - threadIdx.x < m; e0 += step) {
        uint32_t h[EPT], t[EPT], mn[EPT];
        bool in[EPT];
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int64_t e = e0 + (int64_t)k * blockDim.x;
            in[k] = e < m;
            h[k] = in[k] ? eh[e] : 0u;
            t[k] = in[k] ? (per_edge ? thr[e] : thr_const) : 0u;
            mn[k] = 0xFFFFFFFFu;
        }
        for (int j0 = 0; j0 < J; j0 += 16) {
            bool open = false;
#pragma unroll
            for (int k = 0; k < EPT; ++k) open = open || (in[k] && mn[k] >= t[k]);
            if (!__ballot(open)) break;  // every edge of the wave is live somewhere
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                if (j0 + 4 * g < J) {
                    const uint32_t* xg = X + j0 + 4 * g;
                    const uint32_t x0 = xg[0], x1 = xg[1], x2 = xg[2], x3 = xg[3];
#pragma unroll
                    for (int k = 0; k < EPT; ++k) {
                        mn[k] = min(min(mn[k], x0 ^ h[k]), x1 ^ h[k]);
                        mn[k] = min(min(mn[k], x2 ^ h[k]), x3 ^ h[k]);
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < EPT; ++k)
            if (in[k] && mn[k] >= t[k]) {
                int32_t* a = adj + e0 + (int64_t)k * blockDim.x;
                *a = (int32_t)((uint32_t)*a | DEAD_EDGE);
            }
    }
}

hipError_t launch_dead_edges(const DevGraph& g, const uint32_t* X, int J, hipStream_t s) {
    if (g.m == 0) return hipSuccess;
    if (J > 1024 || J % 4) return hipErrorInvalidValue;
    int64_t blocks = (g.m + 1023) / 1024;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_dead_edges, dim3((int)blocks), dim3(256), 0, s, g.adj, g.eh, g.thr, g.thr_const,
                       g.kind == THR_CONST ? 0 : 1, X, J, g.m);
    return hipGetLastError();
}

// Rows with more than heavy_deg out-edges are split into pieces.
// counts[0] = heavy rows, counts[1] = pieces.
__global__ void k_heavy_count(const int64_t* __restrict__ xadj, int64_t n, int64_t heavy_deg, int64_t piece,
                              unsigned long long* counts) {
    unsigned long long rows = 0, pieces = 0;
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = xadj[u + 1] - xadj[u];
        if (d > heavy_deg) {
            rows += 1;
            pieces += (unsigned long long)((d + piece - 1) / piece);
        }
    }
    rows = wave_sum(rows);
    pieces = wave_sum(pieces);
    if ((threadIdx.x & 63) == 0 && rows) {
        atomicAdd(&counts[0], rows);
        atomicAdd(&counts[1], pieces);
    }
}

hipError_t launch_heavy_count(const DevGraph& g, int64_t piece_edges, unsigned long long* counts, hipStream_t s) {
    hipLaunchKernelGGL(k_heavy_count, dim3(2048), dim3(256), 0, s, g.xadj, g.n, g.heavy_deg, piece_edges, counts);
    return hipGetLastError();
}

// Assigns heavy rows to slots (counts[2] = next row slot, counts[3] = next
// piece) and records each row's piece count; the order of slots does not
// affect any result.
__global__ void k_heavy_assign(const int64_t* __restrict__ xadj, int64_t n, int64_t heavy_deg, int64_t piece,
                               unsigned long long* counts, int32_t* hrow, int64_t* hpb, int64_t* hnp) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = xadj[u + 1] - xadj[u];
        if (d > heavy_deg) {
            const int64_t np = (d + piece - 1) / piece;
            const unsigned long long slot = atomicAdd(&counts[2], 1ull);
            const unsigned long long base = atomicAdd(&counts[3], (unsigned long long)np);
            hrow[slot] = (int32_t)u;
            hpb[slot] = (int64_t)base;
            hnp[slot] = np;
        }
    }
}

hipError_t launch_heavy_assign(const DevGraph& g, int64_t piece_edges, unsigned long long* counts, hipStream_t s) {
    if (g.nheavy == 0) return hipSuccess;
    hipLaunchKernelGGL(k_heavy_assign, dim3(2048), dim3(256), 0, s, g.xadj, g.n, g.heavy_deg, piece_edges, counts,
                       g.hrow, g.hpb, g.hpn);
    return hipGetLastError();
}

// Writes the pieces of every heavy row: pieces hpb[r] .. hpb[r] + hpn[r] - 1.
// Slot and piece base of a row come from two separate atomics, so the pieces
// of slot r are not followed by those of slot r + 1.
__global__ void k_heavy_pieces(const int64_t* __restrict__ xadj, const int32_t* __restrict__ hrow,
                               const int64_t* __restrict__ hpb, const int64_t* __restrict__ hnp, int64_t nheavy,
                               int64_t piece, int32_t* prow, int64_t* pe0, int64_t* pe1) {
    const int lane = threadIdx.x & 63;
    for (int64_t r = wave_index(); r < nheavy; r += wave_count()) {
        const int32_t u = hrow[r];
        const int64_t eb = xadj[u], ee = xadj[u + 1], base = hpb[r], np = hnp[r];
        for (int64_t c = lane; c < np; c += 64) {
            prow[base + c] = (int32_t)r;  // index of the heavy row (its slot)
            pe0[base + c] = eb + c * piece;
            pe1[base + c] = (eb + (c + 1) * piece < ee) ? eb + (c + 1) * piece : ee;
        }
    }
}

hipError_t launch_heavy_pieces(const DevGraph& g, int64_t piece_edges, hipStream_t s) {
    if (g.nheavy == 0) return hipSuccess;
    hipLaunchKernelGGL(k_heavy_pieces, dim3(1024), dim3(256), 0, s, g.xadj, g.hrow, g.hpb, g.hpn, g.nheavy,
                       piece_edges, g.prow, g.pe0, g.pe1);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Register initialisation (Alg. 1): M_v[j] = clz(hash(v) xor hash(j)), or 0
// for a blocked pair.  Writes both register buffers.
// ----------------------------------------------------------------------------
template <int G, int DW>
__global__ __launch_bounds__(256) void k_init(const uint32_t* __restrict__ HJ, const uint32_t* __restrict__ blk,
                                              uint32_t* __restrict__ A, uint32_t* __restrict__ B, int64_t n, int P,
                                              int PW, uint32_t seed1) {
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63, grp = lane / G, p = lane % G;
    uint32_t hj[DW][4];
#pragma unroll
    for (int i = 0; i < DW; ++i) {
        const int q = i * G + p;
#pragma unroll
        for (int k = 0; k < 4; ++k) hj[i][k] = q < P ? HJ[4 * q + k] : 0u;
    }
    for (int64_t base = wave_index() * RPW; base < n; base += wave_count() * RPW) {
        const int64_t u = base + grp;
        if (u >= n) continue;
        const uint32_t hv = mm3_key4((uint32_t)u, seed1);
#pragma unroll
        for (int i = 0; i < DW; ++i) {
            const int q = i * G + p;
            if (q >= P) continue;
            uint32_t w = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) w |= lead_zeros(hv ^ hj[i][k]) << (8 * k);
            if (blk) w &= unblocked_mask(blk, u, q, PW);
            A[u * P + q] = w;
            if (B) B[u * P + q] = w;
        }
    }
}

#define HFR_LAYOUT_DISPATCH(L, KERNEL_CALL)              \
    do {                                                 \
        if ((L).G == 4) {                                \
            constexpr int G_ = 4, DW_ = 1;               \
            KERNEL_CALL;                                 \
        } else if ((L).G == 8) {                         \
            constexpr int G_ = 8, DW_ = 1;               \
            KERNEL_CALL;                                 \
        } else if ((L).G == 16) {                        \
            constexpr int G_ = 16, DW_ = 1;              \
            KERNEL_CALL;                                 \
        } else if ((L).G == 32) {                        \
            constexpr int G_ = 32, DW_ = 1;              \
            KERNEL_CALL;                                 \
        } else if ((L).DW == 1) {                        \
            constexpr int G_ = 64, DW_ = 1;              \
            KERNEL_CALL;                                 \
        } else if ((L).DW == 2) {                        \
            constexpr int G_ = 64, DW_ = 2;              \
            KERNEL_CALL;                                 \
        } else {                                         \
            constexpr int G_ = 64, DW_ = 4;              \
            KERNEL_CALL;                                 \
        }                                                \
    } while (0)

Layout make_layout(int J) {
    Layout L;
    L.J = J;
    L.P = J / 4;
    L.PW = (L.P + 31) / 32;
    if (L.P <= 4) L.G = 4, L.DW = 1;
    else if (L.P <= 8) L.G = 8, L.DW = 1;
    else if (L.P <= 16) L.G = 16, L.DW = 1;
    else if (L.P <= 32) L.G = 32, L.DW = 1;
    else if (L.P <= 64) L.G = 64, L.DW = 1;
    else if (L.P <= 128) L.G = 64, L.DW = 2;
    else L.G = 64, L.DW = 4;
    return L;
}

static int grid_for_rows(int64_t rows_groups) {
    int64_t blocks = (rows_groups + 3) / 4;
    if (blocks < 1) blocks = 1;
    if (blocks > 8192) blocks = 8192;
    return (int)blocks;
}

hipError_t launch_init(const Layout& L, int64_t n, const uint32_t* HJ, uint32_t seed, const uint32_t* blk, uint32_t* A,
                       uint32_t* B, hipStream_t s) {
    const int grid = grid_for_rows((n + (64 / L.G) - 1) / (64 / L.G));
    HFR_LAYOUT_DISPATCH(L, hipLaunchKernelGGL((k_init<G_, DW_>), dim3(grid), dim3(256), 0, s, HJ, blk, A, B, n, L.P,
                                              L.PW, seed + 1u));
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Simulate sweep (Alg. 2), synchronous: reads M^t = A, writes M^{t+1} = B.
//
// Invariant before sweep t: B[u] = A[u] for every u not in L_t (for t = 0 the
// init kernel wrote both buffers).  Row u merges the rows of its out-
// neighbours v in L_t over the live samples; it is written to B iff it
// changed or u is in L_t (then B still holds M^{t-1}[u]).
//
// Dense sweep: every row is visited; a wave owns 32 consecutive rows per chunk
// and stores the chunk's L_{t+1} bitmap word with a plain store.  Sparse sweep
// (few live vertices): only the rows that can change are visited -- the
// in-neighbours of L_t, found through the reverse CSR, and L_t itself (for the
// copy rule); their L_{t+1} bits are set atomically.  Both visit exactly the
// rows with a live out-neighbour, so registers, traces and counts are the same.
// Rows with more than heavy_deg out-edges are split into pieces
// (k_sweep_heavy) and combined by k_sweep_heavy_fix.
// ----------------------------------------------------------------------------

// Live count |L_t| of a running sweep, or 0 when the sweep is past the
// stopping rule (the kernel then returns).
DEVI uint32_t sweep_live(const uint32_t* __restrict__ gate, uint32_t gate_thresh, int first, int64_t n) {
    if (first) return (uint32_t)n;
    const uint32_t live = gate_sum(gate);
    return live > gate_thresh ? live : 0u;
}

// A sweep after the first is sparse when the in-degrees of L_t sum to at most
// m / div: then listing the in-neighbours of L_t costs less than visiting
// every row.  The sum S_t is accumulated by the previous sweep.
DEVI bool sweep_sparse(const unsigned long long* __restrict__ sgate, int first, int64_t m, uint32_t div) {
    if (first || div == 0) return false;
    unsigned long long s = 0;
#pragma unroll
    for (int i = 0; i < NSLOT; ++i) s += sgate[i * SLOT_U64];
    return s * div <= (unsigned long long)m;
}

// A dense sweep after the first with at most coarse_live vertices in L_t tests
// heads against the coarse copy of L_t first (built by the frontier kernel).
DEVI bool sweep_coarse(uint32_t live, int first, bool sparse, const Frontier& fr) {
    return !first && !sparse && fr.coarse_live > 0 && live <= fr.coarse_live;
}

// Copies the coarse L_t of the sweep into LDS (cl[COARSE_WORDS]); returns the
// pointer the merges test against, nullptr when the sweep does not use it.
// Uniform over the workgroup.
DEVI const uint32_t* load_coarse(bool use, const Frontier& fr, uint32_t* cl) {
    if (!use) return nullptr;
    for (int i = threadIdx.x; i < fr.coarse_words; i += blockDim.x) cl[i] = fr.coarse[i];
    __syncthreads();
    return cl;
}


// First kernel of every sweep.  Zeroes the bitmap that will hold L_{t+2}; in a
// sparse sweep also marks the rows of L_t (the copy rule needs them) and lists
// the in-edge chunks of every vertex of L_t.
__global__ __launch_bounds__(256) void k_sweep_frontier(const uint32_t* __restrict__ gate, uint32_t gate_thresh,
                                                        const unsigned long long* __restrict__ sgate, int64_t m,
                                                        int first, int64_t n, const uint32_t* __restrict__ Lcur,
                                                        uint32_t* __restrict__ Lclear, Frontier fr, int parity,
                                                        const int64_t* __restrict__ rxadj) {
    const uint32_t live = sweep_live(gate, gate_thresh, first, n);
    if (!live) return;
    const int64_t nwords = (n + 31) >> 5;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int64_t w = tid; w < nwords + 1; w += stride) Lclear[w] = 0u;
    const bool sparse = sweep_sparse(sgate, first, m, fr.sparse_div);
    const int lane = threadIdx.x & 63;
    if (sweep_coarse(live, first, sparse, fr)) {
        // coarse word cw covers the 2^cs L_t words from cw << cs: lane l ORs k =
        // 2^cs / 64 of them, so coarse bit b is lanes 2b and 2b + 1
        const int cs = fr.coarse_shift;
        const int64_t k = (int64_t)1 << (cs - 6);
        for (int64_t cw = wave_index(); cw < fr.coarse_words; cw += wave_count()) {
            const int64_t w0 = (cw << cs) + lane * k;
            uint32_t any = 0;
            for (int64_t i = 0; i < k; ++i)
                if (w0 + i < nwords) any |= Lcur[w0 + i];
            const uint64_t bal = __ballot(any != 0u);
            uint32_t bits = 0;
#pragma unroll
            for (int b = 0; b < 32; ++b) bits |= (uint32_t)(((bal >> (2 * b)) | (bal >> (2 * b + 1))) & 1ull) << b;
            if (lane == 0) fr.coarse[cw] = bits;
        }
    }
    if (!sparse) return;
    uint32_t* cnt = fr.counts + 4 * parity;
    // uniform trip count per wave so that every lane takes part in the scan
    const int64_t span = ((nwords + stride - 1) / stride) * stride;
    for (int64_t w0 = tid - lane; w0 < span; w0 += stride) {
        const int64_t w = w0 + lane;
        const uint32_t bits = w < nwords ? Lcur[w] : 0u;
        uint32_t nitems = 0;
        for (uint32_t b = bits; b; b &= b - 1) {
            const int64_t v = w * 32 + __builtin_ctz(b);
            nitems += (uint32_t)((rxadj[v + 1] - rxadj[v] + fr.chunk - 1) / fr.chunk);
        }
        uint32_t ti;
        const uint32_t oi = wave_excl_scan(nitems, &ti);
        uint32_t bi = 0;
        if (lane == 0 && ti) bi = atomicAdd(&cnt[0], ti);
        bi = __shfl(bi, 0, 64) + oi;
        if (bits) {
            fr.mark[w] = bits;  // the mark words are zero outside a sparse sweep
            for (uint32_t b = bits; b; b &= b - 1) {
                const int64_t v = w * 32 + __builtin_ctz(b);
                const int64_t nc = (rxadj[v + 1] - rxadj[v] + fr.chunk - 1) / fr.chunk;
                for (int64_t c = 0; c < nc; ++c) fr.items[bi++] = make_int2((int)v, (int)c);
            }
        }
    }
}

// Sparse sweep: marks the source rows of the in-edges of L_t.  An in-edge from
// a row that is not split sets the row's bit in `mark`; an in-edge from a
// split row sets the bit of its 64-edge window in its piece's window mask.
// In-edges live in no sample (flagged in the reverse CSR) and in-edges from rows
// blocked in every sample mark nothing: such a row merges nothing through them.
// The sweep's edge visits -- in-edges of L_t whose source is not blocked in
// every sample -- are counted here, per source kind (split or not), so the row
// and piece kernels of a sparse sweep count only the rows they merge.
// Nothing is listed here: the marked rows are listed afterwards with one
// atomic per wave, and the piece kernel finds its pieces by scanning the
// window masks, so each in-edge costs one random access and no shared counter
// is contended.
__global__ __launch_bounds__(256) void k_sweep_expand(const uint32_t* __restrict__ gate, uint32_t gate_thresh,
                                                      const unsigned long long* __restrict__ sgate, int64_t m,
                                                      int first, int64_t n, Frontier fr, int parity,
                                                      const int64_t* __restrict__ rxadj,
                                                      const int2* __restrict__ rrec, int32_t wpp,
                                                      const uint32_t* __restrict__ fullblk,
                                                      unsigned long long* __restrict__ vis_light,
                                                      unsigned long long* __restrict__ vis_heavy) {
    __shared__ unsigned long long sh64[4];
    const uint32_t live = sweep_live(gate, gate_thresh, first, n);
    if (!live || !sweep_sparse(sgate, first, m, fr.sparse_div)) return;
    const uint32_t nitems = fr.counts[4 * parity];
    const int lane = threadIdx.x & 63;
    unsigned long long my_light = 0, my_heavy = 0;
    for (int64_t it = wave_index(); it < (int64_t)nitems; it += wave_count()) {
        const int2 item = fr.items[it];
        const int64_t vb = rxadj[item.x], ve = rxadj[item.x + 1];
        const int64_t e0 = vb + (int64_t)item.y * fr.chunk;
        const int64_t e1 = e0 + fr.chunk < ve ? e0 + fr.chunk : ve;
        for (int64_t e = e0 + lane; e < e1; e += 64) {
            const int2 rc = rrec[e];
            const int32_t a = rc.x;
            const int32_t u = adj_target(a);
            const int32_t wi = rc.y;
            if (fullblk && bit_of(fullblk, u)) continue;  // neither visited nor marked
            if (wi < 0)
                ++my_light;
            else
                ++my_heavy;
            if (adj_dead(a)) continue;
            // most rows are reached from several live vertices: test before
            // paying for the atomic
            uint32_t* word;
            uint32_t bit;
            if (wi < 0) {
                word = &fr.mark[u >> 5];
                bit = 1u << (u & 31);
            } else {
                const int32_t pc = wi / wpp;
                word = &fr.wmask[pc];
                bit = 1u << (wi - pc * wpp);
            }
            if ((*word & bit) == 0u) atomicOr(word, bit);
        }
    }
    const unsigned long long bl = block_sum256(my_light, sh64);
    const unsigned long long bh = block_sum256(my_heavy, sh64);
    if (threadIdx.x == 0) {
        const int slot = blockIdx.x % NSLOT;
        if (bl) atomicAdd(&vis_light[slot * SLOT_U64], bl);
        if (bh && vis_heavy) atomicAdd(&vis_heavy[slot * SLOT_U64], bh);
    }
}

// Sparse sweep: lists the marked rows (W) for the row kernels and clears the
// marks, with one counter atomic per workgroup.
__global__ __launch_bounds__(256) void k_sweep_compact(const uint32_t* __restrict__ gate, uint32_t gate_thresh,
                                                       const unsigned long long* __restrict__ sgate, int64_t m,
                                                       int first, int64_t n, Frontier fr, int parity) {
    const uint32_t live = sweep_live(gate, gate_thresh, first, n);
    if (!live || !sweep_sparse(sgate, first, m, fr.sparse_div)) return;
    uint32_t* cnt = fr.counts + 4 * parity;
    __shared__ uint32_t s_wtot[4];
    __shared__ uint32_t s_base;
    const int64_t nwords = (n + 31) >> 5;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // 256 words per workgroup and round, one counter atomic per workgroup
    for (int64_t c0 = (int64_t)blockIdx.x * 256; c0 < nwords; c0 += (int64_t)gridDim.x * 256) {
        const int64_t w = c0 + threadIdx.x;
        const uint32_t bits = w < nwords ? fr.mark[w] : 0u;
        if (bits) fr.mark[w] = 0u;
        uint32_t wtot;
        const uint32_t off = wave_excl_scan((uint32_t)__builtin_popcount(bits), &wtot);
        if (lane == 0) s_wtot[wv] = wtot;
        __syncthreads();
        uint32_t before = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k < wv) before += s_wtot[k];
            tot += s_wtot[k];
        }
        if (threadIdx.x == 0 && tot) s_base = atomicAdd(&cnt[1], tot);
        __syncthreads();
        if (tot) {
            uint32_t pos = s_base + before + off;
            for (uint32_t b = bits; b; b &= b - 1) fr.W[pos++] = (int32_t)(w * 32 + __builtin_ctz(b));
        }
        __syncthreads();  // s_wtot and s_base are reused by the next round
    }
}

// Last kernel of every sweep: zeroes the item counter of the next sweep.
__global__ __launch_bounds__(64) void k_sweep_cleanup(const uint32_t* __restrict__ gate, uint32_t gate_thresh,
                                                      int first, int64_t n, Frontier fr, int parity) {
    const uint32_t live = sweep_live(gate, gate_thresh, first, n);
    if (!live) return;
    if (threadIdx.x < 4) fr.counts[4 * (parity ^ 1) + threadIdx.x] = 0u;
}

template <int G, int DW, int KIND>
__global__ __launch_bounds__(256) void k_sweep_light(
    const int64_t* __restrict__ xadj, const int32_t* __restrict__ adj, EdgeHashes H,
    const uint32_t* __restrict__ thr, uint32_t thr_const, const uint32_t* __restrict__ X,
    const uint32_t* __restrict__ A, uint32_t* __restrict__ B, const uint32_t* __restrict__ Lcur,
    uint32_t* __restrict__ Lnext, const uint32_t* __restrict__ blk, const uint32_t* __restrict__ gate,
    uint32_t gate_thresh, uint32_t* __restrict__ cnt_out, unsigned long long* __restrict__ vis_out,
    const unsigned long long* __restrict__ sgate, unsigned long long* __restrict__ sum_out,
    const int64_t* __restrict__ rxadj, int64_t n, int64_t m, int P, int PW, int64_t heavy_deg, int first, Frontier fr,
    int parity, const uint32_t* __restrict__ fullblk) {
    __shared__ unsigned long long sh64[4];
    __shared__ uint32_t sh32[4];
    const uint32_t live = sweep_live(gate, gate_thresh, first, n);
    if (!live) return;
    const bool sparse = sweep_sparse(sgate, first, m, fr.sparse_div);
    unsigned long long my_sum = 0;
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63, grp = lane / G, p = lane % G;
    uint32_t x[DW][4];
    load_sim_words<G, DW>(X, P, p, x);
    const uint32_t ntv = to_vgpr(0u - thr_const);
    uint32_t my_cnt = 0;
    unsigned long long my_vis = 0, my_mrg = 0;
    if (!sparse) {
        const int64_t nwords = (n + 31) >> 5;
        for (int64_t c = wave_index(); c < nwords; c += wave_count()) {
            uint32_t word = 0;
            for (int rr = 0; rr < 32; rr += RPW) {
                const int64_t u = c * 32 + rr + grp;
                bool changed = false;
                if (u < n)
                    changed = sweep_row<G, DW, KIND>(u, xadj, adj, H, thr, ntv, x, A, B, Lcur, Lnext, blk, fullblk,
                                                     heavy_deg, P, PW, first, true, lane, p, my_vis, &my_mrg);
                if (changed && p == 0) my_sum += (unsigned long long)(rxadj[u + 1] - rxadj[u]);
                const uint64_t bal = __ballot(changed && p == 0);
#pragma unroll
                for (int g = 0; g < RPW; ++g) word |= (uint32_t)((bal >> (g * G)) & 1ull) << (rr + g);
            }
            if (lane == 0) {
                Lnext[c] = word;
                my_cnt += __builtin_popcount(word);
            }
        }
    } else {
        const int64_t nw = fr.counts[4 * parity + 1];
        for (int64_t base = wave_index() * RPW; base < nw; base += wave_count() * RPW) {
            const int64_t i = base + grp;
            bool changed = false;
            if (i < nw)
                changed = sweep_row<G, DW, KIND>(fr.W[i], xadj, adj, H, thr, ntv, x, A, B, Lcur, Lnext, blk,
                                                 fullblk, heavy_deg, P, PW, first, false, lane, p, my_vis, &my_mrg);
            if (changed && p == 0) {
                my_cnt += 1;
                my_sum += (unsigned long long)(rxadj[fr.W[i] + 1] - rxadj[fr.W[i]]);
            }
        }
    }
    if (sparse) my_vis = 0;  // a sparse sweep's visits are counted by k_sweep_expand
    const uint32_t bc = block_sum256(my_cnt, sh32);
    const unsigned long long bv = block_sum256(my_vis, sh64);
    const unsigned long long bm = block_sum256(my_mrg, sh64);
    const unsigned long long bs = block_sum256(my_sum, sh64);
    if (threadIdx.x == 0) {
        const int slot = blockIdx.x % NSLOT;
        if (bc) atomicAdd(&cnt_out[slot * SLOT_U32], bc);
        if (bv) atomicAdd(&vis_out[slot * SLOT_U64], bv);
        if (bm) atomicAdd(&vis_out[slot * SLOT_U64 + 1], bm);  // rows merged, beside the visits
        if (bs) atomicAdd(&sum_out[slot * SLOT_U64], bs);
    }
}

// Row kernel for one row per wave (R > 128): a wave takes 32 rows at a time
// (dense: 32 consecutive rows, one L_{t+1} word; sparse: 32 listed rows).
// Lane i < 32 reads the offsets of row i; the rows' out-edges are then read as
// one flat sequence, 64 per window, each lane finding its row by binary search
// over the rows' prefix offsets in LDS.  Live heads are merged in batches of UB
// row loads; the first load of a row also fetches the row itself (and its
// blocked bits), so finishing a row needs no extra round trip.  At one dword
// per lane (R = 256) the kernel runs at 7 waves per SIMD, a few spilled
// registers included (measured on the 2^24 weighted-cascade graph: 7% less
// row-kernel time than at 5 waves); wider rows keep 5.
template <int DW, int KIND, bool BLK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DW == 1 ? 7 : 5, 8))) void k_sweep_rows64(
    const int64_t* __restrict__ xadj, const int32_t* __restrict__ adj, EdgeHashes H,
    const uint32_t* __restrict__ thr, uint32_t thr_const, const uint32_t* __restrict__ X,
    const uint32_t* __restrict__ A, uint32_t* __restrict__ B, const uint32_t* __restrict__ Lcur,
    uint32_t* __restrict__ Lnext, const uint32_t* __restrict__ blk, const uint32_t* __restrict__ gate,
    uint32_t gate_thresh, uint32_t* __restrict__ cnt_out, unsigned long long* __restrict__ vis_out,
    const unsigned long long* __restrict__ sgate, unsigned long long* __restrict__ sum_out,
    const int64_t* __restrict__ rxadj, int64_t n, int64_t m, int P, int PW, int64_t heavy_deg, int first, Frontier fr,
    int parity, const uint32_t* __restrict__ fullblk, const int32_t* __restrict__ lrows, int64_t nlight) {
    __shared__ unsigned long long sh64[4];
    __shared__ uint32_t sh32[4];
    __shared__ uint32_t s_off[4][33];
    __shared__ int64_t s_x[4][32];
    __shared__ uint32_t s_coarse[COARSE_WORDS];
    const uint32_t live = sweep_live(gate, gate_thresh, first, n);
    if (!live) return;
    const bool sparse = sweep_sparse(sgate, first, m, fr.sparse_div);
    // dense: every row with 1..heavy_deg out-edges (rows without out-edges never
    // change and are never in L_t); sparse: the listed rows
    const int64_t nrows = sparse ? (int64_t)fr.counts[4 * parity + 1] : nlight;
    const int64_t nbatch = (nrows + 31) >> 5;
    // a workgroup none of whose waves has a batch leaves before any other load
    // (sparse sweeps late in a Simulate list a few rows for the whole grid)
    if ((int64_t)blockIdx.x * (blockDim.x >> 6) >= nbatch) return;
    const uint32_t* cl = load_coarse(sweep_coarse(live, first, sparse, fr), fr, s_coarse);
    const int cs = fr.coarse_shift;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t x[DW][4];
    load_sim_words<64, DW>(X, P, lane, x);
    const uint32_t ntv = to_vgpr(0u - thr_const);
    uint32_t my_cnt = 0;
    unsigned long long my_vis = 0, my_sum = 0, my_mrg = 0;
    for (int64_t c = wave_index(); c < nbatch; c += wave_count()) {
        // ---- the batch's rows: one per lane i < 32 (ascending in a dense sweep)
        int64_t u = -1;
        if (lane < 32) {
            const int64_t idx = c * 32 + lane;
            if (idx < nrows) u = sparse ? (int64_t)fr.W[idx] : (int64_t)lrows[idx];
        }
        int64_t eb = 0, ee = 0;
        bool inL = false;
        if (u >= 0) {
            eb = xadj[u];
            ee = xadj[u + 1];
            if (ee - eb > heavy_deg) {
                ee = eb;  // split row: handled by the piece kernels
            } else {
                inL = !first && bit_of(Lcur, u) != 0u;
                // blocked in every sample: cannot change, never in L
                if (BLK && ee > eb && bit_of(fullblk, u)) ee = eb;
            }
        }
        uint32_t total;
        const uint32_t off = wave_excl_scan((uint32_t)(ee - eb), &total);
        if (lane < 32) {
            s_off[wv][lane] = off;
            s_x[wv][lane] = eb;
        }
        if (lane == 32) s_off[wv][32] = total;
        __builtin_amdgcn_wave_barrier();
        const uint64_t inl_mask = __ballot(inL);
        uint32_t word = 0, touched = 0;
        int cur = -1;
        int64_t cur_u = 0;
        uint32_t cur_a[DW], cur_ub[DW];
        Acc acc[DW];
#pragma unroll
        for (int i = 0; i < DW; ++i) {
            cur_a[i] = 0u;
            cur_ub[i] = 0xFFFFFFFFu;
            acc[i].e = acc[i].o = 0u;
        }
        uint32_t vis = 0, mrg = 0;  // edges with a live head; rows merged
        // flat edge f of the batch -> (row r, edge id e); the next window's ids
        // are fetched while the current window is merged
        auto locate = [&](uint32_t f, int& r, int64_t& e) {
            int lo = 0, hi = 32;  // largest r with s_off[r] <= f
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_off[wv][mid] <= f) lo = mid; else hi = mid - 1;
            }
            r = lo < 31 ? lo : 31;  // lo = 32 only for lanes past the last edge
            e = s_x[wv][r] + (int64_t)(f - s_off[wv][r]);
        };
        int r_n;
        int64_t e_n;
        locate((uint32_t)lane, r_n, e_n);
        bool in_n = (uint32_t)lane < total;
        int32_t v_n = in_n ? adj[e_n] : 0;  // raw id (DEAD_EDGE possible)
        for (uint32_t f0 = 0; f0 < total; f0 += 64) {
            const int r = r_n;
            const int64_t e = e_n;
            const bool valid = in_n;
            const int32_t v = adj_target(v_n);
            const uint64_t dmask = __ballot(adj_dead(v_n));  // edges live in no sample
            const uint32_t fn = f0 + 64 + lane;
            locate(fn, r_n, e_n);
            in_n = fn < total;
            v_n = in_n ? adj[e_n] : 0;
            const bool lv = valid && (first || in_L(Lcur, cl, cs, v));
            uint64_t mask = __ballot(lv);
            if (!mask) continue;  // no live head: the window needs no hash or threshold
            vis += (uint32_t)__builtin_popcountll(mask);
            mask &= ~dmask;  // edges live in no sample merge nothing
            if (!mask) continue;
            mrg += (uint32_t)__builtin_popcountll(mask);
            // hashes and thresholds of the merged edges only; the row of lane's edge is r
            const bool mine = ((mask >> lane) & 1ull) != 0ull;
            const uint32_t su = (uint32_t)__shfl((int)u, r, 64);
            const uint32_t hh = mine ? edge_hash_of(H, e, su, (uint32_t)v) : 0u;
            uint32_t tt = 0u;
            if constexpr (KIND == THR_TARGET) tt = mine ? thr[v] : 0u;
            if constexpr (KIND == THR_EDGE) tt = mine ? thr[e] : 0u;
            // batches of NB live edges, NB the smallest of 1, 2, 4, UB that covers
            // the edges left (capped at UB); unused slots repeat the last one
            // (max-merge is idempotent), so every load is issued without a branch
            auto batch = [&](auto nbc) {
                constexpr int NB = decltype(nbc)::value;
                int idx[NB], rb[NB];
                int last = __builtin_ctzll(mask);
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    if (mask) last = __builtin_ctzll(mask);
                    idx[b] = last;
                    mask &= mask - 1;
                    rb[b] = __builtin_amdgcn_readlane(r, idx[b]);
                }
                uint32_t d[NB][DW];
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const int64_t vb = __builtin_amdgcn_readlane(v, idx[b]);
                    const uint32_t* __restrict__ row = A + vb * P;
#pragma unroll
                    for (int i = 0; i < DW; ++i) {
                        // lanes past the row (q >= P) read a valid dword of it; their
                        // results are masked from the change test and never stored
                        const int q = i * 64 + lane;
                        d[b][i] = row[q < P ? q : P - 1];
                    }
                }
                // keep the batch's loads ahead of the merges (no sinking to the uses)
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    if (rb[b] != cur) {
                        if (cur >= 0) {
                            bool ch = false;
#pragma unroll
                            for (int i = 0; i < DW; ++i) {
                                const uint32_t nw = acc_max(cur_a[i], acc[i]) & cur_ub[i];
                                ch = ch || (i * 64 + lane < P && nw != cur_a[i]);
                                cur_a[i] = nw;
                            }
                            const bool changed = __ballot(ch) != 0;
                            const bool il = (inl_mask >> cur) & 1ull;
                            if (changed || il) {
#pragma unroll
                                for (int i = 0; i < DW; ++i) {
                                    const int q = i * 64 + lane;
                                    if (q < P) B[cur_u * P + q] = cur_a[i];
                                }
                            }
                            if (changed) word |= 1u << cur;
                        }
                        cur = rb[b];
                        cur_u = __builtin_amdgcn_readlane((int)u, cur);
                        touched |= 1u << cur;
                        // the row's own registers are first needed when it is finished
#pragma unroll
                        for (int i = 0; i < DW; ++i) {
                            const int q = i * 64 + lane;
                            const int qc = q < P ? q : P - 1;
                            cur_a[i] = A[cur_u * P + qc];
                            cur_ub[i] = BLK ? unblocked_mask(blk, cur_u, qc, PW) : 0xFFFFFFFFu;
                            acc[i].e = acc[i].o = 0u;
                        }
                    }
                    const uint32_t hb = (uint32_t)__builtin_amdgcn_readlane((int)hh, idx[b]);
                    uint32_t nt = ntv;
                    if constexpr (KIND != THR_CONST) nt = 0u - (uint32_t)__builtin_amdgcn_readlane((int)tt, idx[b]);
#pragma unroll
                    for (int i = 0; i < DW; ++i)
                        merge_live(acc[i], d[b][i], x[i][0], x[i][1], x[i][2], x[i][3], hb, nt);
                }
            };
            while (mask) {
                const int nl = __builtin_popcountll(mask);
                if (DW == 1 && nl > UB)
                    batch(std::integral_constant<int, 2 * UB>{});
                else if (nl > 4)
                    batch(std::integral_constant<int, UB>{});
                else if (nl > 2)
                    batch(std::integral_constant<int, 4>{});
                else if (nl == 2)
                    batch(std::integral_constant<int, 2>{});
                else
                    batch(std::integral_constant<int, 1>{});
            }
        }
        if (cur >= 0) {
            bool ch = false;
#pragma unroll
            for (int i = 0; i < DW; ++i) {
                const uint32_t nw = acc_max(cur_a[i], acc[i]) & cur_ub[i];
                ch = ch || (i * 64 + lane < P && nw != cur_a[i]);
                cur_a[i] = nw;
            }
            const bool changed = __ballot(ch) != 0;
            const bool il = (inl_mask >> cur) & 1ull;
            if (changed || il) {
#pragma unroll
                for (int i = 0; i < DW; ++i) {
                    const int q = i * 64 + lane;
                    if (q < P) B[cur_u * P + q] = cur_a[i];
                }
            }
            if (changed) word |= 1u << cur;
        }
        // rows of L_t without a live out-neighbour: B still holds M^{t-1}; copy M^t
        for (uint32_t cp = (uint32_t)inl_mask & ~touched; cp; cp &= cp - 1) {
            const int rr = __builtin_ctz(cp);
            const int64_t uu = __builtin_amdgcn_readlane((int)u, rr);
#pragma unroll
            for (int i = 0; i < DW; ++i) {
                const int q = i * 64 + lane;
                if (q < P) B[uu * P + q] = A[uu * P + q];
            }
        }
        {
            // L_{t+1} starts zeroed; lanes that share an L word (the rows are sorted
            // in a dense sweep) OR their bits into the run's first lane, which
            // issues one atomic for the word
            const bool chg = lane < 32 && ((word >> lane) & 1u);
            const int32_t wd = u >= 0 ? (int32_t)(u >> 5) : -1 - lane;
            uint32_t bits = chg ? 1u << (u & 31) : 0u;
#pragma unroll
            for (int k = 1; k < 32; k <<= 1) {
                const uint32_t ob = __shfl_down(bits, k, 64);
                const int32_t ow = __shfl_down(wd, k, 64);
                if (lane + k < 32 && ow == wd) bits |= ob;
            }
            const int32_t pw = __shfl_up(wd, 1, 64);
            if (lane < 32 && bits && (lane == 0 || pw != wd)) atomicOr(&Lnext[wd], bits);
        }
        if (lane < 32 && ((word >> lane) & 1u)) my_sum += (unsigned long long)(rxadj[u + 1] - rxadj[u]);
        if (lane == 0) {
            my_cnt += __builtin_popcount(word);
            my_vis += vis;
            my_mrg += mrg;
        }
    }
    if (sparse) my_vis = 0;  // a sparse sweep's visits are counted by k_sweep_expand
    const uint32_t bc = block_sum256(my_cnt, sh32);
    const unsigned long long bv = block_sum256(my_vis, sh64);
    const unsigned long long bm = block_sum256(my_mrg, sh64);
    const unsigned long long bs = block_sum256(my_sum, sh64);
    if (threadIdx.x == 0) {
        const int slot = blockIdx.x % NSLOT;
        if (bc) atomicAdd(&cnt_out[slot * SLOT_U32], bc);
        if (bv) atomicAdd(&vis_out[slot * SLOT_U64], bv);
        if (bm) atomicAdd(&vis_out[slot * SLOT_U64 + 1], bm);  // rows merged, beside the visits
        if (bs) atomicAdd(&sum_out[slot * SLOT_U64], bs);
    }
}


// One G-lane group per piece of a split row: merge of the live rows of the
// piece's out-neighbours in L_t, written to part[piece].
constexpr int NSP = 2;  // marked pieces whose first windows a sparse sweep loads together
template <int G, int DW, int KIND>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7, 8))) void k_sweep_heavy(
    const int32_t* __restrict__ adj, EdgeHashes H, const uint32_t* __restrict__ thr,
    uint32_t thr_const, const uint32_t* __restrict__ X, const uint32_t* __restrict__ A,
    const uint32_t* __restrict__ Lcur, const uint32_t* __restrict__ blk, const uint32_t* __restrict__ gate,
    uint32_t gate_thresh, unsigned long long* __restrict__ vis_out, const int32_t* __restrict__ hrow,
    const int32_t* __restrict__ prow, const int64_t* __restrict__ pe0, const int64_t* __restrict__ pe1,
    uint32_t* __restrict__ part, uint32_t* __restrict__ part_any, int64_t npieces, int64_t n, int P, int PW,
    int first, Frontier fr, int parity, const unsigned long long* __restrict__ sgate, int64_t m,
    const uint32_t* __restrict__ fullblk, uint32_t* __restrict__ rtouch) {
    __shared__ unsigned long long sh64[4];
    __shared__ uint32_t s_coarse[COARSE_WORDS];
    const uint32_t live = sweep_live(gate, gate_thresh, first, n);
    if (!live) return;
    const bool sparse = sweep_sparse(sgate, first, m, fr.sparse_div);
    const uint32_t* cl = load_coarse(G == 64 && sweep_coarse(live, first, sparse, fr), fr, s_coarse);
    const int cs = fr.coarse_shift;
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63, grp = lane / G, p = lane % G;
    uint32_t x[DW][4];
    load_sim_words<G, DW>(X, P, p, x);
    const uint32_t ntv = to_vgpr(0u - thr_const);
    unsigned long long my_vis = 0;
    unsigned long long my_mrg = 0;  // rows merged (uniform over the group)
    // writes the partial row of piece pc of split row r (the merge of its live
    // edges, or of a run of consecutive pieces of r that starts at pc) and its
    // flag; vis is uniform over the group, a partial without live edges is
    // never read and a piece without a flag of this sweep is skipped by the
    // fix-up
    auto finish_piece = [&](const int64_t pc, const int32_t r, const uint32_t vis, const Acc (&acc)[DW]) {
        if (vis > 0) {
#pragma unroll
            for (int k = 0; k < DW; ++k) {
                const int q = k * G + p;
                if (q < P) part[pc * P + q] = acc[k].e | acc[k].o;
            }
        }
        if (p == 0) {
            if (vis > 0) {
                part_any[pc] = fr.stamp;
                rtouch[r] = fr.stamp;  // the row has a piece to combine in this sweep
            }
            my_vis += vis;
        }
    };
    // merges piece pc of split row r (vertex u), edges [b0, b1) (uniform over the
    // group); wm: its 64-edge windows to scan, all of them when 0; skip: the row
    // is blocked in every sample
    auto piece = [&](const int64_t pc, const int32_t r, const uint32_t u, const int64_t b0, const int64_t b1,
                     const uint32_t wm, const bool skip) {
        Acc acc[DW];
#pragma unroll
        for (int k = 0; k < DW; ++k) acc[k].e = acc[k].o = 0u;
        uint32_t vis = 0;
        if (!skip) {
            if (wm) {
                if constexpr (G == 64) {
                    vis = merge_marked_windows64<DW, KIND>(b0, b1, wm, u, adj, H, thr, ntv, A, Lcur, first, P, lane,
                                                           x, acc, nullptr, 0, &my_mrg);
                } else {
                    for (uint32_t left = wm; left; left &= left - 1) {
                        const int64_t w0 = b0 + 64 * (int64_t)__builtin_ctz(left);
                        const int64_t w1 = w0 + 64 < b1 ? w0 + 64 : b1;
                        vis += merge_edges<G, DW, KIND>(w0, w1, u, adj, H, thr, ntv, A, Lcur, first, P, lane, p, x,
                                                        acc, nullptr, 0, &my_mrg);
                    }
                }
            } else {
                vis = merge_edges<G, DW, KIND>(b0, b1, u, adj, H, thr, ntv, A, Lcur, first, P, lane, p, x, acc, cl,
                                               cs, &my_mrg);
            }
        }
        finish_piece(pc, r, vis, acc);
    };
    if (!sparse && G == 64) {
        // each wave takes `span` consecutive pieces (its share, <= 64), with their
        // table entries loaded lane-parallel; a run of consecutive pieces of one
        // row is merged into one partial row (the run's first piece's), so the
        // fix-up of a row with many pieces reads a few partials
        int64_t span = (npieces + wave_count() - 1) / wave_count();
        span = span < 1 ? 1 : (span > 64 ? 64 : span);
        for (int64_t base = wave_index() * span; base < npieces; base += wave_count() * span) {
            const int cnt = (int)(npieces - base < span ? npieces - base : span);
            int32_t rl = 0, ul = 0;
            int64_t b0l = 0, b1l = 0;
            bool skl = false;
            if (lane < cnt) {
                rl = prow[base + lane];
                b0l = pe0[base + lane];
                b1l = pe1[base + lane];
                ul = hrow[rl];
                skl = fullblk && bit_of(fullblk, ul) != 0u;
            }
            const uint64_t skipm = __ballot(skl);
            Acc acc[DW];
#pragma unroll
            for (int k = 0; k < DW; ++k) acc[k].e = acc[k].o = 0u;
            uint32_t vis = 0;
            int first_j = 0;
            int32_t run_r = __shfl(rl, 0, 64);
            for (int j = 0; j < cnt; ++j) {
                const int32_t r = __shfl(rl, j, 64);
                if (r != run_r) {
                    finish_piece(base + first_j, run_r, vis, acc);
#pragma unroll
                    for (int k = 0; k < DW; ++k) acc[k].e = acc[k].o = 0u;
                    vis = 0;
                    first_j = j;
                    run_r = r;
                }
                if (!((skipm >> j) & 1ull))
                    vis += merge_edges<G, DW, KIND>(__shfl(b0l, j, 64), __shfl(b1l, j, 64), (uint32_t)__shfl(ul, j, 64),
                                                    adj, H, thr, ntv, A, Lcur, first, P, lane, p, x, acc, cl, cs,
                                                    &my_mrg);
            }
            finish_piece(base + first_j, run_r, vis, acc);
        }
    } else if (!sparse) {
        // a group's pieces are i, i + stride, ...; the next piece's table entry is
        // loaded while the current piece is merged
        const int64_t stride = wave_count() * RPW;
        int64_t i = wave_index() * RPW + grp;
        int32_t r_n = 0;
        int64_t b0_n = 0, b1_n = 0;
        if (i < npieces) {
            r_n = prow[i];
            b0_n = pe0[i];
            b1_n = pe1[i];
        }
        for (; i - grp < npieces; i += stride) {
            const int32_t r = r_n;
            const int64_t b0 = b0_n, b1 = b1_n;
            if (i + stride < npieces) {
                r_n = prow[i + stride];
                b0_n = pe0[i + stride];
                b1_n = pe1[i + stride];
            }
            if (i < npieces) {
                const int32_t u = hrow[r];
                piece(i, r, (uint32_t)u, b0, b1, 0u, fullblk && bit_of(fullblk, u) != 0u);
            }
        }
    } else {
        // the pieces with a marked window: each wave scans `span` window masks
        // (its share, <= 64), clears the nonzero ones (this kernel is their last
        // reader in the sweep) and merges those pieces, RPW at a time
        int64_t span = (npieces + wave_count() - 1) / wave_count();
        span = span < 1 ? 1 : (span > 64 ? 64 : span);
        for (int64_t base = wave_index() * span; base < npieces; base += wave_count() * span) {
            uint32_t wm = 0;
            if (lane < span && base + lane < npieces) {
                wm = fr.wmask[base + lane];
                if (wm) fr.wmask[base + lane] = 0u;
            }
            // the table entries of every marked piece of the span, loaded at once
            int32_t rl = 0, ul = 0;
            int64_t b0l = 0, b1l = 0;
            bool skl = false;
            if (wm) {
                rl = prow[base + lane];
                b0l = pe0[base + lane];
                b1l = pe1[base + lane];
                ul = hrow[rl];
                skl = fullblk && bit_of(fullblk, ul) != 0u;
            }
            if constexpr (G == 64) {
                // NSP marked pieces at a time: the edge ids of each one's first marked
                // window are loaded, and their heads tested against L_t, together, so
                // that the pieces share those round trips; then each piece is merged
                // (its other marked windows, rare in a sparse sweep, after the first)
                for (uint64_t nz = __ballot(wm != 0u); nz;) {
                    // per slot: the piece's lane in the span, its table entry (wave-uniform,
                    // read from that lane) and the first marked window's edge ids
                    int js[NSP];
                    uint32_t wj[NSP], uq[NSP];
                    int32_t rq[NSP], vw[NSP];
                    int64_t w0[NSP], e1q[NSP];
                    bool val[NSP];
                    uint64_t dm[NSP], mw[NSP];
#pragma unroll
                    for (int q = 0; q < NSP; ++q) {
                        val[q] = nz != 0ull;
                        js[q] = val[q] ? __builtin_ctzll(nz) : 0;
                        nz &= nz - 1;
                        const int j = js[q];
                        wj[q] = (uint32_t)__builtin_amdgcn_readlane((int)wm, j);
                        rq[q] = __builtin_amdgcn_readlane(rl, j);
                        uq[q] = (uint32_t)__builtin_amdgcn_readlane(ul, j);
                        const int64_t b0q = readlane64(b0l, j);
                        e1q[q] = readlane64(b1l, j);
                        const bool skip = !val[q] || __builtin_amdgcn_readlane((int)skl, j) != 0;
                        w0[q] = skip || wj[q] == 0u ? e1q[q] : b0q + 64 * (int64_t)__builtin_ctz(wj[q]);
                        const bool in = w0[q] + lane < e1q[q];
                        const int32_t a = in ? adj[w0[q] + lane] : 0;
                        vw[q] = adj_target(a);
                        dm[q] = __ballot(adj_dead(a));
                    }
#pragma unroll
                    for (int q = 0; q < NSP; ++q) mw[q] = __ballot(w0[q] + lane < e1q[q] && bit_of(Lcur, vw[q]) != 0u);
#pragma unroll
                    for (int q = 0; q < NSP; ++q) {
                        if (!val[q]) continue;
                        Acc acc[DW];
#pragma unroll
                        for (int k = 0; k < DW; ++k) acc[k].e = acc[k].o = 0u;
                        uint32_t vis = 0;
                        if (w0[q] < e1q[q]) {  // not skipped (a window is never empty)
                            vis = (uint32_t)__builtin_popcountll(mw[q]);
                            const uint64_t mm = mw[q] & ~dm[q];  // edges live in no sample merge nothing
                            if (mm)
                                my_mrg += merge_window64<DW, KIND>(mm, w0[q] + lane, w0[q] + lane < e1q[q], vw[q],
                                                                   uq[q], H, thr, ntv, A, P, lane, x, acc);
                            const uint32_t rest = wj[q] & (wj[q] - 1u);
                            if (rest)
                                vis += merge_marked_windows64<DW, KIND>(w0[q] - 64 * (int64_t)__builtin_ctz(wj[q]),
                                                                        e1q[q], rest, uq[q], adj, H, thr, ntv, A,
                                                                        Lcur, first, P, lane, x, acc, nullptr, 0,
                                                                        &my_mrg);
                        }
                        finish_piece(base + js[q], rq[q], vis, acc);
                    }
                }
            } else {
                for (uint64_t nz = __ballot(wm != 0u); nz;) {
                    // group grp takes the grp-th marked piece left
                    uint64_t t = nz;
                    for (int k = 0; k < grp && t; ++k) t &= t - 1;
                    const int j = t ? __builtin_ctzll(t) : 0;
                    const uint32_t wj = (uint32_t)__shfl((int)wm, j, 64);
                    const int32_t r = __shfl(rl, j, 64);
                    const uint32_t u = (uint32_t)__shfl(ul, j, 64);
                    const int64_t b0 = __shfl(b0l, j, 64), b1 = __shfl(b1l, j, 64);
                    const bool sk = __shfl((int)skl, j, 64) != 0;
                    for (int k = 0; k < RPW && nz; ++k) nz &= nz - 1;
                    if (t) piece(base + j, r, u, b0, b1, wj, sk);
                }
            }
        }
    }
    if (sparse) my_vis = 0;  // a sparse sweep's visits are counted by k_sweep_expand
    const unsigned long long bv = block_sum256(my_vis, sh64);
    const unsigned long long bm = block_sum256(p == 0 ? my_mrg : 0ull, sh64);
    if (threadIdx.x == 0) {
        if (bv) atomicAdd(&vis_out[(blockIdx.x % NSLOT) * SLOT_U64], bv);
        if (bm) atomicAdd(&vis_out[(blockIdx.x % NSLOT) * SLOT_U64 + 1], bm);  // rows merged, beside the visits
    }
}

// One G-lane group per split row: combine the pieces merged in this sweep
// (flag == stamp) with the row itself.
template <int G, int DW>
__global__ __launch_bounds__(256) void k_sweep_heavy_fix(
    const uint32_t* __restrict__ A, uint32_t* __restrict__ B, const uint32_t* __restrict__ Lcur,
    uint32_t* __restrict__ Lnext, const uint32_t* __restrict__ blk, const uint32_t* __restrict__ gate,
    uint32_t gate_thresh, uint32_t* __restrict__ cnt_out, const int32_t* __restrict__ hrow,
    const int64_t* __restrict__ hpb, const int64_t* __restrict__ hpn, const uint32_t* __restrict__ part,
    const uint32_t* __restrict__ part_any, int64_t nheavy, int64_t n, int P, int PW, int first, Frontier fr,
    int parity, const unsigned long long* __restrict__ sgate, unsigned long long* __restrict__ sum_out,
    const int64_t* __restrict__ rxadj, int64_t m, const uint32_t* __restrict__ fullblk,
    const uint32_t* __restrict__ rtouch) {
    __shared__ uint32_t sh32[4];
    __shared__ unsigned long long sh64[4];
    const uint32_t live = sweep_live(gate, gate_thresh, first, n);
    if (!live) return;
    // dense and sparse sweeps alike: every split row, filtered by needs()
    const int64_t count = nheavy;
    const uint32_t stamp = fr.stamp;
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63, grp = lane / G, p = lane % G;
    uint32_t my_cnt = 0;
    unsigned long long my_sum = 0;
    // A row needs work only if a piece merged a live edge in this sweep (touch
    // stamp) or it is in L_t (copy rule); fix_row would leave any other row
    // untouched.  Rows are filtered with one ballot per wave-sized group.
    auto needs = [&](int64_t r, int64_t u) {
        return !(fullblk && bit_of(fullblk, u)) && (rtouch[r] == stamp || (!first && bit_of(Lcur, u)));
    };
    if constexpr (G == 64) {
        // each wave filters `span` rows at a time, span = its share of the rows (<= 64)
        int64_t span = (count + wave_count() - 1) / wave_count();
        span = span < 1 ? 1 : (span > 64 ? 64 : span);
        for (int64_t base = wave_index() * span; base < count; base += wave_count() * span) {
            const int64_t i = base + lane;
            int64_t r = 0, u = 0;
            bool need = false;
            if (lane < span && i < count) {
                r = i;
                u = hrow[r];
                need = needs(r, u);
            }
            // the rows that need work, two at a time (their loads interleaved)
            for (uint64_t mask = __ballot(need); mask;) {
                int64_t rr[2], uu[2];
                bool vv[2], ch[2];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    vv[t] = mask != 0ull;
                    const int j = vv[t] ? __builtin_ctzll(mask) : 0;
                    mask &= mask - 1;
                    rr[t] = __builtin_amdgcn_readlane((int)r, j);
                    uu[t] = __builtin_amdgcn_readlane((int)u, j);
                }
                fix_rows2<DW>(rr, uu, vv, A, B, Lcur, blk, hpb, hpn, part, part_any, stamp, P, PW, first, lane, ch);
#pragma unroll
                for (int t = 0; t < 2; ++t)
                    if (vv[t] && ch[t] && lane == 0) {
                        atomicOr(&Lnext[uu[t] >> 5], 1u << (uu[t] & 31));
                        my_cnt += 1;
                        my_sum += (unsigned long long)(rxadj[uu[t] + 1] - rxadj[uu[t]]);
                    }
            }
        }
    } else {
        for (int64_t base = wave_index() * RPW; base < count; base += wave_count() * RPW) {
            const int64_t i = base + grp;
            if (i >= count) continue;
            const int64_t r = i;
            const int64_t u = hrow[r];
            if (!needs(r, u)) continue;
            const bool changed =
                fix_row<G, DW>(r, u, A, B, Lcur, blk, hpb, hpn, part, part_any, stamp, P, PW, first, lane, p);
            if (changed && p == 0) {
                atomicOr(&Lnext[u >> 5], 1u << (u & 31));
                my_cnt += 1;
                my_sum += (unsigned long long)(rxadj[u + 1] - rxadj[u]);
            }
        }
    }
    const uint32_t bc = block_sum256(my_cnt, sh32);
    const unsigned long long bs = block_sum256(my_sum, sh64);
    if (threadIdx.x == 0) {
        if (bc) atomicAdd(&cnt_out[(blockIdx.x % NSLOT) * SLOT_U32], bc);
        if (bs) atomicAdd(&sum_out[(blockIdx.x % NSLOT) * SLOT_U64], bs);
    }
}

#define HFR_KIND_DISPATCH(kind, CALL)        \
    do {                                     \
        if ((kind) == THR_CONST) {           \
            constexpr int K_ = THR_CONST;    \
            CALL;                            \
        } else if ((kind) == THR_TARGET) {   \
            constexpr int K_ = THR_TARGET;   \
            CALL;                            \
        } else {                             \
            constexpr int K_ = THR_EDGE;     \
            CALL;                            \
        }                                    \
    } while (0)

hipError_t launch_sweep(const Layout& L, const DevGraph& g, const uint32_t* X, const SweepParams& sp, int grid,
                        hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, hipEvent_t ev2, hipEvent_t ev3) {
    const int64_t words = (g.n + 31) / 32;
    const int lg = grid > 0 ? grid : grid_for_rows(words);
    const int sg = 2048;  // grid of the list kernels
    hipLaunchKernelGGL(k_sweep_frontier, dim3(sg), dim3(256), 0, s, sp.gate, sp.gate_thresh, sp.sgate, g.m, sp.first,
                       g.n, sp.Lcur, sp.Lclear, sp.fr, sp.parity, g.rxadj);
    hipLaunchKernelGGL(k_sweep_expand, dim3(sg), dim3(256), 0, s, sp.gate, sp.gate_thresh, sp.sgate, g.m, sp.first, g.n,
                       sp.fr, sp.parity, g.rxadj, g.rrec, (int32_t)((g.piece_edges + 63) / 64), sp.fullblk,
                       sp.vis_out, g.npieces > 0 ? sp.vis_heavy_out : nullptr);
    hipLaunchKernelGGL(k_sweep_compact, dim3(sg), dim3(256), 0, s, sp.gate, sp.gate_thresh, sp.sgate, g.m, sp.first,
                       g.n, sp.fr, sp.parity);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    if (ev0) (void)hipEventRecord(ev0, s);
    if (L.G == 64) {
        const int rg = grid_for_rows((g.n + 31) / 32);
#define HFR_ROWS64(BLK_)                                                                                              \
    HFR_LAYOUT_DISPATCH(L, HFR_KIND_DISPATCH(g.kind, hipLaunchKernelGGL((k_sweep_rows64<DW_, K_, BLK_>), dim3(rg),     \
                                                                        dim3(256), 0, s, g.xadj, g.adj, hashes(g),    \
                                                                        g.thr, g.thr_const, X, sp.A, sp.B, sp.Lcur,   \
                                                                        sp.Lnext,                                     \
                                                                        sp.blk, sp.gate, sp.gate_thresh, sp.cnt_out,  \
                                                                        sp.vis_out, sp.sgate, sp.sum_out, g.rxadj,    \
                                                                        g.n, g.m, L.P, L.PW, g.heavy_deg, sp.first,   \
                                                                        sp.fr, sp.parity, sp.fullblk, g.lrows,        \
                                                                        g.nlight)))
        if (sp.blk)
            HFR_ROWS64(true);
        else
            HFR_ROWS64(false);
#undef HFR_ROWS64
    } else {
        HFR_LAYOUT_DISPATCH(L, HFR_KIND_DISPATCH(g.kind, hipLaunchKernelGGL((k_sweep_light<G_, DW_, K_>), dim3(lg),
                                                                            dim3(256), 0, s, g.xadj, g.adj,
                                                                            hashes(g), g.thr, g.thr_const, X, sp.A,
                                                                            sp.B, sp.Lcur,
                                                                            sp.Lnext, sp.blk, sp.gate, sp.gate_thresh,
                                                                            sp.cnt_out, sp.vis_out, sp.sgate,
                                                                            sp.sum_out, g.rxadj, g.n, g.m, L.P, L.PW,
                                                                            g.heavy_deg, sp.first, sp.fr, sp.parity,
                                                                            sp.fullblk)));
    }
    if (ev1) (void)hipEventRecord(ev1, s);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    if (ev2) (void)hipEventRecord(ev2, s);
    if (g.npieces > 0) {
        const int rpw = 64 / L.G;
        const int hg = grid_for_rows((g.npieces + rpw - 1) / rpw);
        HFR_LAYOUT_DISPATCH(L, HFR_KIND_DISPATCH(g.kind, hipLaunchKernelGGL((k_sweep_heavy<G_, DW_, K_>), dim3(hg),
                                                                            dim3(256), 0, s, g.adj, hashes(g), g.thr,
                                                                            g.thr_const, X, sp.A, sp.Lcur, sp.blk,
                                                                            sp.gate, sp.gate_thresh,
                                                                            sp.vis_heavy_out, g.hrow, g.prow, g.pe0,
                                                                            g.pe1, sp.part, sp.part_any, g.npieces,
                                                                            g.n, L.P, L.PW, sp.first, sp.fr,
                                                                            sp.parity, sp.sgate, g.m, sp.fullblk,
                                                                            sp.rtouch)));
        err = hipGetLastError();
        if (err != hipSuccess) return err;
        if (ev3) (void)hipEventRecord(ev3, s);
        const int fg = grid_for_rows((g.nheavy + rpw - 1) / rpw);
        HFR_LAYOUT_DISPATCH(L, hipLaunchKernelGGL((k_sweep_heavy_fix<G_, DW_>), dim3(fg), dim3(256), 0, s, sp.A, sp.B,
                                                  sp.Lcur, sp.Lnext, sp.blk, sp.gate, sp.gate_thresh, sp.cnt_out,
                                                  g.hrow, g.hpb, g.hpn, sp.part, sp.part_any, g.nheavy, g.n, L.P,
                                                  L.PW, sp.first, sp.fr, sp.parity, sp.sgate, sp.sum_out, g.rxadj,
                                                  g.m, sp.fullblk, sp.rtouch));
        err = hipGetLastError();
        if (err != hipSuccess) return err;
    } else if (ev3) {
        (void)hipEventRecord(ev3, s);
    }
    hipLaunchKernelGGL(k_sweep_cleanup, dim3(1), dim3(64), 0, s, sp.gate, sp.gate_thresh, sp.first, g.n, sp.fr,
                       sp.parity);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Reverse CSR (in-edges) for sparse sweeps, and the heavy slot of every row.
// ----------------------------------------------------------------------------

// Exclusive prefix sum of n u32 values into n+1 int64 offsets: block sums,
// a single-block scan of the sums, then a per-block scan with the offset.
constexpr int SCAN_BLOCK = 1024;

__global__ void k_scan_block_sums(const uint32_t* __restrict__ in, int64_t n, int64_t* sums) {
    __shared__ int64_t sh[4];
    const int64_t i0 = (int64_t)blockIdx.x * SCAN_BLOCK;
    int64_t s = 0;
    for (int k = threadIdx.x; k < SCAN_BLOCK; k += 256)
        if (i0 + k < n) s += in[i0 + k];
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

// Exclusive scan of the nb block sums in place (sums[nb] = total), one block of
// 1024 threads: each thread scans a contiguous run of ceil(nb / 1024) sums,
// offset by the scan of the run totals across the block.
__global__ __launch_bounds__(1024) void k_scan_sums(int64_t* sums, int64_t nb) {
    __shared__ int64_t sh[1024];
    const int t = threadIdx.x;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t b0 = t * per;
    const int64_t b1 = b0 + per < nb ? b0 + per : nb;
    int64_t loc = 0;
    for (int64_t b = b0; b < b1; ++b) loc += sums[b];
    sh[t] = loc;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t y = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += y;
        __syncthreads();
    }
    int64_t run = sh[t] - loc;
    for (int64_t b = b0; b < b1; ++b) {
        const int64_t v = sums[b];
        sums[b] = run;
        run += v;
    }
    if (t == 1023) sums[nb] = sh[1023];
}

__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t* __restrict__ in, int64_t n,
                                                    const int64_t* __restrict__ sums, int64_t* out) {
    // exclusive prefix of the block's SCAN_BLOCK values: 4 per thread, then a
    // scan of the thread totals across the block
    __shared__ int64_t sh_wave[4];
    const int64_t i0 = (int64_t)blockIdx.x * SCAN_BLOCK + 4 * threadIdx.x;
    int64_t v[4], t = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = i0 + k < n ? (int64_t)in[i0 + k] : 0;
        t += v[k];
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t incl = t;
#pragma unroll
    for (int k = 1; k < 64; k <<= 1) {
        const int64_t o = __shfl_up(incl, k, 64);
        if (lane >= k) incl += o;
    }
    if (lane == 63) sh_wave[w] = incl;
    __syncthreads();
    int64_t base = sums[blockIdx.x];
    for (int k = 0; k < w; ++k) base += sh_wave[k];
    int64_t run = base + incl - t;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (i0 + k < n) out[i0 + k] = run;
        run += v[k];
    }
    const int64_t nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    if (blockIdx.x == nb - 1 && threadIdx.x == 0) out[n] = sums[nb];
}

// rrec[cursor[v]++] = (u, window) for every edge (u, v); the order inside an in-row
// depends on scheduling, the set does not (graphs too large for the counting
// sort below).
__global__ void k_rev_scatter(const int64_t* __restrict__ xadj, const int32_t* __restrict__ adj, int64_t n,
                              int64_t* cursor, int2* rrec, const int32_t* __restrict__ hslot,
                              const int64_t* __restrict__ hpb, int64_t piece, int32_t wpp) {
    const int lane = threadIdx.x & 63;
    for (int64_t u = wave_index(); u < n; u += wave_count()) {
        const int64_t eb = xadj[u], ee = xadj[u + 1];
        const int32_t r = hslot[u];
        const int64_t base = r >= 0 ? hpb[r] : 0;
        for (int64_t e = eb + lane; e < ee; e += 64) {
            const int32_t v = adj_target(adj[e]);  // may run beside the flagging of dead edges
            const unsigned long long pos = atomicAdd((unsigned long long*)&cursor[v], 1ull);
            // 64-edge window of the edge within its piece (windows of piece c are
            // c * wpp .. c * wpp + wpp - 1)
            rrec[pos] = make_int2((int32_t)u,
                                  r >= 0 ? (int32_t)((base + (e - eb) / piece) * wpp + ((e - eb) % piece) / 64) : -1);
        }
    }
}

__global__ void k_copy_i64(const int64_t* __restrict__ a, int64_t* b, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

hipError_t launch_reverse_csr(const DevGraph& g, const uint32_t* indeg, int64_t* cursor, uint32_t* scan_tmp,
                              hipStream_t s) {
    const int64_t n = g.n;
    const int64_t nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    int64_t* sums = reinterpret_cast<int64_t*>(scan_tmp);  // nb + 1 entries
    hipLaunchKernelGGL(k_scan_block_sums, dim3((unsigned)nb), dim3(256), 0, s, indeg, n, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, sums, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, s, indeg, n, sums, g.rxadj);
    hipLaunchKernelGGL(k_copy_i64, dim3(4096), dim3(256), 0, s, g.rxadj, cursor, n);
    if (g.m > 0)
        hipLaunchKernelGGL(k_rev_scatter, dim3(8192), dim3(256), 0, s, g.xadj, g.adj, n, cursor, g.rrec,
                           g.hslot, g.hpb, g.piece_edges, (int32_t)((g.piece_edges + 63) / 64));
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Reverse CSR by a two-level counting sort on the target, without global
// atomics: (1) every workgroup counts its edges per bucket of 2^RB_SHIFT
// consecutive targets in LDS; (2) a scan of the counts, bucket-major, gives
// each workgroup its slice of every bucket; (3) the workgroups re-walk the same
// edges and write (target, source, window) records into their slices; (4) one
// workgroup per bucket counts the in-degrees of its targets in LDS, turns them
// into the offsets rxadj and places the records.  The edges of a workgroup are
// the same in (1) and (3): both walk the rows with at most heavy_deg edges,
// then the pieces of the split rows, with the same grids.  Step (4) shares a
// bucket with many records among several workgroups (chunks).
// ----------------------------------------------------------------------------
constexpr int RB_SHIFT = 13;          // targets per bucket: 8192 (32 KiB of LDS counters)
constexpr int RB_MAX_BUCKETS = 4096;  // so n <= 2^25
constexpr int RB_BLOCKS = 1024;       // workgroups per walk (light rows, then pieces)

template <bool PIECES>
__global__ __launch_bounds__(256) void k_rb_count(const int64_t* __restrict__ xadj, const int32_t* __restrict__ adj,
                                                  int64_t n, int64_t heavy_deg, const int32_t* __restrict__ hrow,
                                                  const int32_t* __restrict__ prow, const int64_t* __restrict__ pe0,
                                                  const int64_t* __restrict__ pe1, int64_t npieces, int nbk, int ncol,
                                                  int col, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[RB_MAX_BUCKETS];
    for (int i = threadIdx.x; i < nbk; i += blockDim.x) h[i] = 0u;
    __syncthreads();
    if constexpr (PIECES)
        for_piece_edges(hrow, prow, pe0, pe1, npieces,
                        [&](int64_t, int64_t e, int64_t, int64_t) { atomicAdd(&h[adj[e] >> RB_SHIFT], 1u); });
    else
        for_light_edges(xadj, n, heavy_deg, [&](int64_t, int64_t e) { atomicAdd(&h[adj[e] >> RB_SHIFT], 1u); });
    __syncthreads();
    for (int i = threadIdx.x; i < nbk; i += blockDim.x) hist[(int64_t)i * ncol + col + blockIdx.x] = h[i];
}

template <bool PIECES>
__global__ __launch_bounds__(256) void k_rb_scatter(const int64_t* __restrict__ xadj, const int32_t* __restrict__ adj,
                                                    int64_t n, int64_t heavy_deg, const int32_t* __restrict__ hrow,
                                                    const int32_t* __restrict__ prow, const int64_t* __restrict__ pe0,
                                                    const int64_t* __restrict__ pe1, int64_t npieces, int nbk,
                                                    int ncol, int col, const int64_t* __restrict__ off, int32_t wpp,
                                                    int32_t* __restrict__ tv, int32_t* __restrict__ tu,
                                                    int32_t* __restrict__ tw) {
    __shared__ int64_t base[RB_MAX_BUCKETS];
    __shared__ uint32_t cur[RB_MAX_BUCKETS];
    for (int i = threadIdx.x; i < nbk; i += blockDim.x) {
        base[i] = off[(int64_t)i * ncol + col + blockIdx.x];
        cur[i] = 0u;
    }
    __syncthreads();
    auto put = [&](int64_t u, int64_t e, int32_t w) {
        const int32_t v = adj[e];
        const int b = v >> RB_SHIFT;
        const int64_t pos = base[b] + atomicAdd(&cur[b], 1u);
        tv[pos] = v;
        tu[pos] = (int32_t)u;
        tw[pos] = w;
    };
    if constexpr (PIECES)
        // the 64-edge window of the edge within its piece: windows of piece pc
        // are pc * wpp .. pc * wpp + wpp - 1
        for_piece_edges(hrow, prow, pe0, pe1, npieces, [&](int64_t u, int64_t e, int64_t pc, int64_t b0) {
            put(u, e, (int32_t)(pc * wpp + (e - b0) / 64));
        });
    else
        for_light_edges(xadj, n, heavy_deg, [&](int64_t u, int64_t e) { put(u, e, -1); });
}

// The records of bucket b are [off[b * ncol], off[(b + 1) * ncol]); the
// bucket is cut into chunks of at most RB_CHUNK records (at least one chunk,
// also when empty), so that the hub buckets of skewed graphs are shared by
// many workgroups.  cstart[b] = first chunk of bucket b, cstart[nbk] = total.
constexpr int64_t RB_CHUNK = 1 << 17;

__global__ __launch_bounds__(1024) void k_rb_chunks(const int64_t* __restrict__ off, int ncol, int nbk,
                                                    int64_t* __restrict__ cstart) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int per = (nbk + 1023) / 1024;
    int64_t loc = 0;
    for (int k = 0; k < per; ++k) {
        const int64_t b = (int64_t)t * per + k;
        if (b < nbk) {
            const int64_t len = off[(b + 1) * ncol] - off[b * ncol];
            loc += len > 0 ? (len + RB_CHUNK - 1) / RB_CHUNK : 1;
        }
    }
    part[t] = loc;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int64_t y = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += y;
        __syncthreads();
    }
    int64_t run = part[t] - loc;
    for (int k = 0; k < per; ++k) {
        const int64_t b = (int64_t)t * per + k;
        if (b < nbk) {
            cstart[b] = run;
            const int64_t len = off[(b + 1) * ncol] - off[b * ncol];
            run += len > 0 ? (len + RB_CHUNK - 1) / RB_CHUNK : 1;
        }
    }
    if (t == 1023) cstart[nbk] = part[1023];
}

// Chunk c of the grid: its bucket b, target base v0 and records [r0, r1), and
// the bucket's first record s0.  False past the last chunk.
struct RbChunk {
    int64_t b, v0, s0, r0, r1;
};
DEVI bool rb_chunk(int64_t c, const int64_t* __restrict__ off, int ncol, int nbk, const int64_t* __restrict__ cstart,
                   RbChunk& ch) {
    if (c >= cstart[nbk]) return false;
    int lo = 0, hi = nbk - 1;  // last bucket with cstart <= c
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cstart[mid] <= c) lo = mid; else hi = mid - 1;
    }
    ch.b = lo;
    ch.v0 = (int64_t)lo << RB_SHIFT;
    ch.s0 = off[(int64_t)lo * ncol];
    const int64_t s1 = off[(int64_t)(lo + 1) * ncol];
    ch.r0 = ch.s0 + (c - cstart[lo]) * RB_CHUNK;
    ch.r1 = ch.r0 + RB_CHUNK < s1 ? ch.r0 + RB_CHUNK : s1;
    return true;
}

// Per chunk: the in-degree counts of its records' targets, ctab[c][t].
__global__ __launch_bounds__(1024) void k_rb_fcount(const int64_t* __restrict__ off, int ncol, int nbk,
                                                    const int64_t* __restrict__ cstart, const int32_t* __restrict__ tv,
                                                    uint32_t* __restrict__ ctab) {
    constexpr int BT = 1 << RB_SHIFT;
    __shared__ uint32_t cnt[BT];
    RbChunk ch;
    if (!rb_chunk(blockIdx.x, off, ncol, nbk, cstart, ch)) return;
    for (int i = threadIdx.x; i < BT; i += 1024) cnt[i] = 0u;
    __syncthreads();
    for (int64_t i = ch.r0 + threadIdx.x; i < ch.r1; i += 1024) atomicAdd(&cnt[tv[i] - ch.v0], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < BT; i += 1024) ctab[(int64_t)blockIdx.x * BT + i] = cnt[i];
}

// Per bucket: in-degrees and rxadj of its targets, and ctab[c][t] turned into
// the first slot (relative to the bucket's first record) of chunk c's records
// of target t.
__global__ __launch_bounds__(1024) void k_rb_fscan(const int64_t* __restrict__ off, int ncol, int nbk, int64_t n,
                                                   const int64_t* __restrict__ cstart, uint32_t* __restrict__ ctab,
                                                   uint32_t* __restrict__ indeg, int64_t* __restrict__ rxadj) {
    constexpr int BT = 1 << RB_SHIFT, PER = BT / 1024;
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int64_t c0 = cstart[b], c1 = cstart[b + 1];
    const int64_t s0 = off[b * ncol], v0 = b << RB_SHIFT;
    uint32_t deg[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) deg[k] = 0u;
    for (int64_t c = c0; c < c1; ++c)
#pragma unroll
        for (int k = 0; k < PER; ++k) deg[k] += ctab[c * BT + k * 1024 + t];
    // targets are k * 1024 + t: scan in that order, PER rounds of 1024
    int64_t base = 0;
    uint32_t first[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        part[t] = deg[k];
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int64_t y = t >= o ? part[t - o] : 0;
            __syncthreads();
            part[t] += y;
            __syncthreads();
        }
        const int64_t loc = base + part[t] - deg[k];
        first[k] = (uint32_t)loc;
        const int64_t v = v0 + k * 1024 + t;
        if (v < n) {
            indeg[v] = deg[k];
            rxadj[v] = s0 + loc;
        }
        base += part[1023];
        __syncthreads();
    }
    if (b == nbk - 1 && t == 0) rxadj[n] = off[(int64_t)nbk * ncol];
    for (int64_t c = c0; c < c1; ++c)
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int64_t i = c * BT + k * 1024 + t;
            const uint32_t x = ctab[i];
            ctab[i] = first[k];
            first[k] += x;
        }
}

// Per chunk: places its records at their slots (rrec).  With dt.mode
// set, a record whose edge is live in no sample gets DEAD_EDGE in its source
// id -- the test k_dead_edges applies to the out-edges, with the hash
// recomputed from (u, v) (Eq. hash) and a threshold that depends on the target
// only: constant p (mode 1), or the weighted cascade's 1/indeg(v) (mode 2), the
// in-degree being the length of v's in-edge list.  A sparse sweep marks no row
// for a flagged in-edge.
__global__ __launch_bounds__(1024) void k_rb_fplace(const int64_t* __restrict__ off, int ncol, int nbk,
                                                    const int64_t* __restrict__ cstart,
                                                    const uint32_t* __restrict__ ctab, const int32_t* __restrict__ tv,
                                                    const int32_t* __restrict__ tu, const int32_t* __restrict__ tw,
                                                    int2* __restrict__ rrec,
                                                    const int64_t* __restrict__ rxadj, DeadTest dt) {
    constexpr int BT = 1 << RB_SHIFT;
    __shared__ uint32_t cur[BT];
    RbChunk ch;
    if (!rb_chunk(blockIdx.x, off, ncol, nbk, cstart, ch)) return;
    for (int i = threadIdx.x; i < BT; i += 1024) cur[i] = ctab[(int64_t)blockIdx.x * BT + i];
    __syncthreads();
    // RPT records per thread (k0 + 1024 r), so that one load of sample words serves
    // RPT records; uniform trip count per wave, so that the sample scan's ballot
    // sees every lane
    constexpr int RPT = 4;
    const int64_t span = ((ch.r1 - ch.r0 + 1024 * RPT - 1) / (1024 * RPT)) * (1024 * RPT);
    for (int64_t k0 = threadIdx.x; k0 < span; k0 += 1024 * RPT) {
        int32_t v[RPT], u[RPT];
        bool in[RPT];
        uint32_t t[RPT], h[RPT], mn[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int64_t i = ch.r0 + k0 + 1024 * r;
            in[r] = i < ch.r1;
            v[r] = in[r] ? tv[i] : 0;
            u[r] = in[r] ? tu[i] : 0;
            mn[r] = 0xFFFFFFFFu;
            t[r] = 0u;
            h[r] = 0u;
            if (dt.mode) {
                t[r] = dt.mode == 2 ? (in[r] ? wc_threshold((uint32_t)(rxadj[v[r] + 1] - rxadj[v[r]])) : 0u)
                                    : dt.thr_const;
                h[r] = mm3_key8((uint32_t)u[r], (uint32_t)v[r], dt.seed) & 0x7FFFFFFFu;
            }
        }
        if (dt.mode) {
            for (int j0 = 0; j0 < dt.J; j0 += 16) {
                bool open = false;
#pragma unroll
                for (int r = 0; r < RPT; ++r) open = open || (in[r] && mn[r] >= t[r]);
                if (!__ballot(open)) break;  // every record of the wave is live somewhere
#pragma unroll
                for (int g = 0; g < 16; g += 4) {
                    if (j0 + g < dt.J) {
                        const uint32_t* xg = dt.X + j0 + g;
                        const uint32_t x0 = xg[0], x1 = xg[1], x2 = xg[2], x3 = xg[3];
#pragma unroll
                        for (int r = 0; r < RPT; ++r) {
                            mn[r] = min(min(mn[r], x0 ^ h[r]), x1 ^ h[r]);
                            mn[r] = min(min(mn[r], x2 ^ h[r]), x3 ^ h[r]);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            if (!in[r]) continue;
            const bool dead = dt.mode && mn[r] >= t[r];
            const int64_t p = ch.s0 + atomicAdd(&cur[v[r] - ch.v0], 1u);
            rrec[p] = make_int2(dead ? (int32_t)((uint32_t)u[r] | DEAD_EDGE) : u[r], tw[ch.r0 + k0 + 1024 * r]);
        }
    }
}

static int64_t rb_max_chunks(int64_t n, int64_t m) {
    const int64_t nbk = (n + (1 << RB_SHIFT) - 1) >> RB_SHIFT;
    return m / RB_CHUNK + nbk + 1;
}

bool rb_fits(int64_t n, int64_t m) {
    return n <= (int64_t)RB_MAX_BUCKETS << RB_SHIFT && m < (1ll << 31);
}

size_t rb_temp_bytes(int64_t n, int64_t m) {
    const int64_t nbk = (n + (1 << RB_SHIFT) - 1) >> RB_SHIFT;
    const int64_t cells = nbk * 2 * RB_BLOCKS;
    const int64_t nsb = (cells + SCAN_BLOCK - 1) / SCAN_BLOCK;
    auto al = [](int64_t b) { return (size_t)((b + 255) & ~int64_t(255)); };
    return al(4 * n) + 3 * al(4 * (m > 0 ? m : 1)) + al(4 * cells) + al(8 * (cells + 1)) + al(8 * (nsb + 2)) +
           al(8 * (nbk + 1)) + al(4 * rb_max_chunks(n, m) * (1 << RB_SHIFT));
}

// In-degrees (indeg) and the reverse CSR of g (rxadj, rrec) on stream
// s; tmp holds rb_temp_bytes(n, m) bytes, indeg at its start.
hipError_t launch_reverse_csr_buckets(const DevGraph& g, void* tmp, uint32_t** indeg_out, const DeadTest& dt,
                                      hipStream_t s) {
    const int64_t n = g.n, m = g.m;
    const int nbk = (int)((n + (1 << RB_SHIFT) - 1) >> RB_SHIFT);
    const int ncol = 2 * RB_BLOCKS;
    const int64_t cells = (int64_t)nbk * ncol;
    const int64_t nsb = (cells + SCAN_BLOCK - 1) / SCAN_BLOCK;
    auto al = [](int64_t b) { return (int64_t)((b + 255) & ~int64_t(255)); };
    char* p = static_cast<char*>(tmp);
    uint32_t* indeg = reinterpret_cast<uint32_t*>(p);
    p += al(4 * n);
    int32_t* tv = reinterpret_cast<int32_t*>(p);
    p += al(4 * (m > 0 ? m : 1));
    int32_t* tu = reinterpret_cast<int32_t*>(p);
    p += al(4 * (m > 0 ? m : 1));
    int32_t* tw = reinterpret_cast<int32_t*>(p);
    p += al(4 * (m > 0 ? m : 1));
    uint32_t* hist = reinterpret_cast<uint32_t*>(p);
    p += al(4 * cells);
    int64_t* off = reinterpret_cast<int64_t*>(p);
    p += al(8 * (cells + 1));
    int64_t* sums = reinterpret_cast<int64_t*>(p);
    p += al(8 * (nsb + 2));
    int64_t* cstart = reinterpret_cast<int64_t*>(p);
    p += al(8 * (nbk + 1));
    uint32_t* ctab = reinterpret_cast<uint32_t*>(p);
    const int64_t maxch = rb_max_chunks(n, m);
    *indeg_out = indeg;
    const int32_t wpp = (int32_t)((g.piece_edges + 63) / 64);
    // a workgroup that walks no edge still writes its (zero) counts
    hipLaunchKernelGGL((k_rb_count<false>), dim3(RB_BLOCKS), dim3(256), 0, s, g.xadj, g.adj, n, g.heavy_deg, g.hrow,
                       g.prow, g.pe0, g.pe1, g.npieces, nbk, ncol, 0, hist);
    hipLaunchKernelGGL((k_rb_count<true>), dim3(RB_BLOCKS), dim3(256), 0, s, g.xadj, g.adj, n, g.heavy_deg, g.hrow,
                       g.prow, g.pe0, g.pe1, g.npieces, nbk, ncol, RB_BLOCKS, hist);
    hipLaunchKernelGGL(k_scan_block_sums, dim3((unsigned)nsb), dim3(256), 0, s, hist, cells, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, sums, nsb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nsb), dim3(256), 0, s, hist, cells, sums, off);
    hipLaunchKernelGGL((k_rb_scatter<false>), dim3(RB_BLOCKS), dim3(256), 0, s, g.xadj, g.adj, n, g.heavy_deg, g.hrow,
                       g.prow, g.pe0, g.pe1, g.npieces, nbk, ncol, 0, off, wpp, tv, tu, tw);
    hipLaunchKernelGGL((k_rb_scatter<true>), dim3(RB_BLOCKS), dim3(256), 0, s, g.xadj, g.adj, n, g.heavy_deg, g.hrow,
                       g.prow, g.pe0, g.pe1, g.npieces, nbk, ncol, RB_BLOCKS, off, wpp, tv, tu, tw);
    hipLaunchKernelGGL(k_rb_chunks, dim3(1), dim3(1024), 0, s, off, ncol, nbk, cstart);
    hipLaunchKernelGGL(k_rb_fcount, dim3((unsigned)maxch), dim3(1024), 0, s, off, ncol, nbk, cstart, tv, ctab);
    hipLaunchKernelGGL(k_rb_fscan, dim3((unsigned)nbk), dim3(1024), 0, s, off, ncol, nbk, n, cstart, ctab, indeg,
                       g.rxadj);
    hipLaunchKernelGGL(k_rb_fplace, dim3((unsigned)maxch), dim3(1024), 0, s, off, ncol, nbk, cstart, ctab, tv, tu, tw,
                       g.rrec, g.rxadj, dt);
    return hipGetLastError();
}

// Rows with 1..heavy_deg out-edges, ascending: flag pass, scan, scatter.
__global__ void k_light_flags(const int64_t* __restrict__ xadj, int64_t n, int64_t heavy_deg, uint32_t* flags) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = xadj[u + 1] - xadj[u];
        flags[u] = (d >= 1 && d <= heavy_deg) ? 1u : 0u;
    }
}

__global__ void k_light_scatter(const uint32_t* __restrict__ flags, const int64_t* __restrict__ pos, int64_t n,
                                int32_t* lrows) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x)
        if (flags[u]) lrows[pos[u]] = (int32_t)u;
}

hipError_t launch_light_rows(const DevGraph& g, uint32_t* flags, int64_t* pos, uint32_t* scan_tmp, hipStream_t s) {
    const int64_t n = g.n;
    const int64_t nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    int64_t* sums = reinterpret_cast<int64_t*>(scan_tmp);  // nb + 1 entries
    hipLaunchKernelGGL(k_light_flags, dim3(4096), dim3(256), 0, s, g.xadj, n, g.heavy_deg, flags);
    hipLaunchKernelGGL(k_scan_block_sums, dim3((unsigned)nb), dim3(256), 0, s, flags, n, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, sums, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, s, flags, n, sums, pos);
    hipLaunchKernelGGL(k_light_scatter, dim3(4096), dim3(256), 0, s, flags, pos, n, g.lrows);
    return hipGetLastError();
}

// fullblk bit u = 1 iff vertex u is blocked in every sample.
__global__ void k_full_blocked(const uint32_t* __restrict__ blk, uint32_t* fullblk, int64_t n, int P, int PW) {
    const int64_t nwords = (n + 31) / 32;
    const int W = 4 * PW;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < nwords; w += (int64_t)gridDim.x * blockDim.x) {
        uint32_t bits = 0;
        for (int j = 0; j < 32; ++j) {
            const int64_t u = w * 32 + j;
            if (u >= n) break;
            bool all = true;
            for (int k = 0; k < W && all; ++k) all = (blk[u * W + k] | ~plane_valid_mask(k, P, PW)) == 0xFFFFFFFFu;
            if (all) bits |= 1u << j;
        }
        fullblk[w] = bits;
    }
}

hipError_t launch_full_blocked(const Layout& L, int64_t n, const uint32_t* blk, uint32_t* fullblk, hipStream_t s) {
    hipLaunchKernelGGL(k_full_blocked, dim3(2048), dim3(256), 0, s, blk, fullblk, n, L.P, L.PW);
    return hipGetLastError();
}

__global__ void k_heavy_slots(const int32_t* __restrict__ hrow, int64_t nheavy, int32_t* hslot) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nheavy; r += (int64_t)gridDim.x * blockDim.x)
        hslot[hrow[r]] = (int32_t)r;
}

hipError_t launch_heavy_slots(const DevGraph& g, hipStream_t s) {
    hipError_t err = launch_fill_u32(reinterpret_cast<uint32_t*>(g.hslot), 0xFFFFFFFFu, g.n, s);
    if (err != hipSuccess || g.nheavy == 0) return err;
    hipLaunchKernelGGL(k_heavy_slots, dim3(1024), dim3(256), 0, s, g.hrow, g.nheavy, g.hslot);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Greedy step (Alg. 1).
// ----------------------------------------------------------------------------

// score(v) = sum_j max(M_S'[j], M_v[j]) over v not in S; key = score << 32 |
// (2^32 - 1 - v), so the maximum key is the largest score with the lowest id.
template <int G, int DW>
__global__ __launch_bounds__(256) void k_argmax(const uint32_t* __restrict__ M, const uint32_t* __restrict__ MS,
                                                const uint8_t* __restrict__ inS, unsigned long long* key_out,
                                                int64_t n, int P) {
    __shared__ unsigned long long sh[4];
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63;
    unsigned long long best = best_score_rows<G, DW>(wave_index() * RPW, n, wave_count() * RPW, M, MS, inS, P);
    const int w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = sh[0];
        for (int i = 1; i < 4; ++i) b = sh[i] > b ? sh[i] : b;
        if (b) atomicMax(key_out, b);
    }
}

// The same argmax for rows of P = 16 DQ dwords: 16 lanes per row, lane p holding
// dwords [p DQ, p DQ + DQ) (16-byte loads), so a wave scores 4 rows per step with
// one 4-step reduction, two steps' loads in flight.
template <int DQ>
__global__ __launch_bounds__(256) void k_argmax16(const uint32_t* __restrict__ M, const uint32_t* __restrict__ MS,
                                                  const uint8_t* __restrict__ inS, unsigned long long* key_out,
                                                  int64_t n) {
    __shared__ unsigned long long sh[4];
    constexpr int P = 16 * DQ;
    const int lane = threadIdx.x & 63, grp = lane >> 4, p = lane & 15;
    uint32_t ms[DQ];
#pragma unroll
    for (int i = 0; i < DQ; ++i) ms[i] = MS[p * DQ + i];
    unsigned long long best = 0;
    const int64_t stride = wave_count() * 4;
    for (int64_t base = wave_index() * 4; base < n; base += 2 * stride) {
        const int64_t u0 = base + grp, u1 = base + stride + grp;
        const bool ok0 = u0 < n && inS[u0] == 0, ok1 = u1 < n && inS[u1] == 0;
        uint4 d0[DQ / 4], d1[DQ / 4];
#pragma unroll
        for (int c = 0; c < DQ / 4; ++c) {
            d0[c] = ok0 ? reinterpret_cast<const uint4*>(M + u0 * P + p * DQ)[c] : make_uint4(0u, 0u, 0u, 0u);
            d1[c] = ok1 ? reinterpret_cast<const uint4*>(M + u1 * P + p * DQ)[c] : make_uint4(0u, 0u, 0u, 0u);
        }
        uint32_t s0 = 0, s1 = 0;
#pragma unroll
        for (int c = 0; c < DQ / 4; ++c) {
            s0 = __builtin_amdgcn_sad_u8(byte_max(ms[4 * c], d0[c].x), 0u, s0);
            s0 = __builtin_amdgcn_sad_u8(byte_max(ms[4 * c + 1], d0[c].y), 0u, s0);
            s0 = __builtin_amdgcn_sad_u8(byte_max(ms[4 * c + 2], d0[c].z), 0u, s0);
            s0 = __builtin_amdgcn_sad_u8(byte_max(ms[4 * c + 3], d0[c].w), 0u, s0);
            s1 = __builtin_amdgcn_sad_u8(byte_max(ms[4 * c], d1[c].x), 0u, s1);
            s1 = __builtin_amdgcn_sad_u8(byte_max(ms[4 * c + 1], d1[c].y), 0u, s1);
            s1 = __builtin_amdgcn_sad_u8(byte_max(ms[4 * c + 2], d1[c].z), 0u, s1);
            s1 = __builtin_amdgcn_sad_u8(byte_max(ms[4 * c + 3], d1[c].w), 0u, s1);
        }
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) {
            s0 += __shfl_xor(s0, off, 64);
            s1 += __shfl_xor(s1, off, 64);
        }
        if (p == 0) {
            if (ok0) {
                const unsigned long long k0 = ((unsigned long long)s0 << 32) | (0xFFFFFFFFu - (uint32_t)u0);
                best = k0 > best ? k0 : best;
            }
            if (ok1) {
                const unsigned long long k1 = ((unsigned long long)s1 << 32) | (0xFFFFFFFFu - (uint32_t)u1);
                best = k1 > best ? k1 : best;
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(best, off, 64);
        best = o > best ? o : best;
    }
    const int w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long bb = sh[0];
        for (int i = 1; i < 4; ++i) bb = sh[i] > bb ? sh[i] : bb;
        if (bb) atomicMax(key_out, bb);
    }
}

hipError_t launch_argmax(const Layout& L, int64_t n, const uint32_t* M, const GreedyBufs& b, hipStream_t s) {
    if (L.P == 64 || L.P == 128 || L.P == 256) {
        const int grid = grid_for_rows((n + 7) / 8);  // 8 rows per wave and step pair
        if (L.P == 64)
            hipLaunchKernelGGL((k_argmax16<4>), dim3(grid), dim3(256), 0, s, M, b.MS, b.inS, b.key, n);
        else if (L.P == 128)
            hipLaunchKernelGGL((k_argmax16<8>), dim3(grid), dim3(256), 0, s, M, b.MS, b.inS, b.key, n);
        else
            hipLaunchKernelGGL((k_argmax16<16>), dim3(grid), dim3(256), 0, s, M, b.MS, b.inS, b.key, n);
        return hipGetLastError();
    }
    const int grid = grid_for_rows((n + (64 / L.G) - 1) / (64 / L.G));
    HFR_LAYOUT_DISPATCH(L, hipLaunchKernelGGL((k_argmax<G_, DW_>), dim3(grid), dim3(256), 0, s, M, b.MS, b.inS, b.key,
                                              n, L.P));
    return hipGetLastError();
}



// One wave: takes the argmax, records the step, computes e and starts the
// Monte-Carlo reach of s (see select_seed).
__global__ void k_select(const int64_t* __restrict__ xadj, const uint32_t* __restrict__ M, GreedyBufs b, StepRec* rec,
                         int32_t* seeds, int k, int J, int P, int PW, int32_t level_id, int64_t n) {
    const unsigned long long key = *b.key;
    uint32_t nch = 0, newcnt = 0;
    double e = 0.0;
    const bool ok = select_seed(key, n, J, P, PW, xadj, M, b.MS, b.merged, b.blk, b.F[0], b.Q[0], b.inS, b.stamp,
                                level_id, b.bfs_chunk, b.T, rec, seeds, k, &nch, &newcnt, &e);
    if (threadIdx.x == 0) {
        b.qsize[0] = nch;
        if (ok && newcnt) atomicAdd(&b.R[0], (unsigned long long)newcnt);
        *b.key = 0ull;
    }
}

hipError_t launch_select(const Layout& L, const DevGraph& g, const uint32_t* M, const GreedyBufs& b, StepRec* rec,
                         int32_t* seeds_dev, int k, int32_t level_id, hipStream_t s) {
    hipLaunchKernelGGL(k_select, dim3(1), dim3(64), 0, s, g.xadj, M, b, rec, seeds_dev, k, L.J, L.P, L.PW, level_id,
                       g.n);
    return hipGetLastError();
}

// Level 0 of a reach search from a vertex set: one wave per listed vertex s
// blocks every pair (s, j) not blocked yet, makes the new pairs its frontier
// and queues its out-edges once (stamp); repeated vertices add nothing.
__global__ void k_reach_start(const int64_t* __restrict__ xadj, GreedyBufs b, const int32_t* __restrict__ verts,
                              int count, int P, int PW, int32_t level_id) {
    const int lane = threadIdx.x & 63;
    const int W = 4 * PW;
    for (int64_t i = wave_index(); i < count; i += wave_count()) {
        const int64_t s = verts[i];
        const int64_t deg = xadj[s + 1] - xadj[s];
        uint32_t newcnt = 0;
        for (int w = lane; w < W; w += 64) {
            const uint32_t valid = plane_valid_mask(w, P, PW);
            const uint32_t nb = valid & ~atomicOr(&b.blk[s * W + w], valid);
            newcnt += __builtin_popcount(nb);
            if (deg > 0 && nb) atomicOr(&b.F[0][s * W + w], nb);
        }
        newcnt = wave_sum(newcnt);
        if (lane == 0 && newcnt) {
            atomicAdd(&b.R[0], (unsigned long long)newcnt);
            if (deg > 0 && atomicMax(&b.stamp[s], level_id) < level_id) {
                const int64_t nch = (deg + b.bfs_chunk - 1) / b.bfs_chunk;
                const uint32_t pos = atomicAdd(&b.qsize[0], (uint32_t)nch);
                for (int64_t c = 0; c < nch; ++c) b.Q[0][pos + c] = make_int2((int)s, (int)c);
            }
        }
    }
}

hipError_t launch_reach_start(const Layout& L, const DevGraph& g, const GreedyBufs& b, const int32_t* verts,
                              int count, int32_t level_id, hipStream_t s) {
    const int grid = (count + 3) / 4 < 1024 ? (count + 3) / 4 : 1024;
    hipLaunchKernelGGL(k_reach_start, dim3(grid), dim3(256), 0, s, g.xadj, b, verts, count, L.P, L.PW, level_id);
    return hipGetLastError();
}

// One BFS level over the queue of level `cur` (see bfs_expand_entries).
template <int G, int DW, int KIND>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_bfs_expand(const int64_t* __restrict__ xadj, const int32_t* __restrict__ adj,
                                                    EdgeHashes H, const uint32_t* __restrict__ thr,
                                                    uint32_t thr_const, const uint32_t* __restrict__ X, GreedyBufs b,
                                                    int cur, int32_t level_id_next, int P, int PW) {
    __shared__ unsigned long long sh64[4];
    const uint32_t size = b.qsize[cur % 3];
    if (size == 0) return;
    constexpr int RPW = 64 / G;
    const int p = (threadIdx.x & 63) % G;
    uint32_t x[DW][4];
    load_sim_words<G, DW>(X, P, p, x);
    const uint32_t ntv = to_vgpr(0u - thr_const);
    const unsigned long long my_new = bfs_expand_entries<G, DW, KIND, true, G == 64 ? 2 : 1>(
        wave_index() * RPW, (int64_t)size, wave_count() * RPW, xadj, adj, H, thr, ntv, x, b.F[cur & 1],
        b.F[(cur + 1) & 1], b.Q[cur & 1], b.Q[(cur + 1) & 1], &b.qsize[(cur + 1) % 3], b.blk, b.stamp, level_id_next,
        b.bfs_chunk, P, PW);
    const unsigned long long bn = block_sum256(my_new, sh64);
    if (threadIdx.x == 0 && bn) atomicAdd(&b.R[(blockIdx.x % NSLOT) * SLOT_U64], bn);
}

// Clears the frontier bits consumed at this level and recycles the ring counter
// of the previous level; qsize[3] counts levels that had work.
__global__ void k_bfs_cleanup(GreedyBufs b, int cur, int PW) {
    const uint32_t size = b.qsize[cur % 3];
    if (blockIdx.x == 0 && threadIdx.x == 0) b.qsize[(cur + 2) % 3] = 0u;  // level cur-1 is finished
    if (size == 0) return;
    uint32_t* Fc = b.F[cur & 1];
    const int2* Qc = b.Q[cur & 1];
    const int W = 4 * PW;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)size * W;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ent = i / W;
        const int2 qe = Qc[ent];
        if (qe.y == 0 && qe.x >= 0) Fc[(int64_t)qe.x * W + (i % W)] = 0u;  // holes have vertex -1
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) b.qsize[3] += 1u;
}

hipError_t launch_bfs_level(const Layout& L, const DevGraph& g, const uint32_t* X, const GreedyBufs& b, int level,
                            int32_t level_id_next, int grid, hipStream_t s) {
    // the queues hold BFS_RESV slots per wave of at most BFS_GRID workgroups beyond their entries
    if (grid < 1 || grid > BFS_GRID) return hipErrorInvalidValue;
    HFR_LAYOUT_DISPATCH(L, HFR_KIND_DISPATCH(g.kind, hipLaunchKernelGGL((k_bfs_expand<G_, DW_, K_>), dim3(grid),
                                                                        dim3(256), 0, s, g.xadj, g.adj, hashes(g),
                                                                        g.thr, g.thr_const, X, b, level, level_id_next,
                                                                        L.P, L.PW)));
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_bfs_cleanup, dim3(256), dim3(256), 0, s, b, level, L.PW);
    return hipGetLastError();
}

// Error-adaptive decision of Alg. 1 (one wave; see decide_step).
__global__ void k_decide(GreedyBufs b, StepRec* rec, int k, int K, double eps_g, double eps_l, int J, int P,
                         int32_t* rebuild_flag) {
    __shared__ int flags[2];
    const int lane = threadIdx.x;
    if (lane == 0) {
        unsigned long long R = 0;
        for (int i = 0; i < NSLOT; ++i) R += b.R[i * SLOT_U64];
        const unsigned long long R0 = *b.Rreb;
        int fresh = 0;
        const int rebuild = decide_step(R, R0, J, k, K, eps_g, eps_l, rec->e, rec, &fresh);
        if (rebuild) *b.Rreb = R;
        *rebuild_flag = rebuild;
        flags[0] = fresh;
        flags[1] = rebuild;
    }
    __syncthreads();
    if (k < K) {
        const bool keep = flags[0] != 0;
        for (int q = lane; q < P; q += 64) b.MS[q] = keep ? b.merged[q] : 0u;
    }
}

hipError_t launch_decide(const Layout& L, const GreedyBufs& b, StepRec* rec, int k, int K, double eps_g, double eps_l,
                         int32_t* rebuild_flag, hipStream_t s) {
    hipLaunchKernelGGL(k_decide, dim3(1), dim3(64), 0, s, b, rec, k, K, eps_g, eps_l, L.J, L.P, rebuild_flag);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Estimates (Eq. sketch-estimate): e = 2^(s/J) / 0.77351 with s the integer
// register sum, evaluated as 2^(s div J) * exp2((s mod J)/J) / 0.77351.
// ----------------------------------------------------------------------------
template <int G, int DW>
__global__ __launch_bounds__(256) void k_estimate_all(const uint32_t* __restrict__ M, const double* __restrict__ T,
                                                      float* out, int64_t n, int J, int P) {
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63, grp = lane / G, p = lane % G;
    for (int64_t base = wave_index() * RPW; base < n; base += wave_count() * RPW) {
        const int64_t u = base + grp;
        uint32_t s = 0;
        if (u < n) {
#pragma unroll
            for (int i = 0; i < DW; ++i) {
                const int q = i * G + p;
                if (q < P) s = __builtin_amdgcn_sad_u8(M[u * P + q], 0u, s);
            }
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (u < n && p == 0) out[u] = (float)estimate_from_sum(s, J, T);
    }
}

hipError_t launch_estimate_all(const Layout& L, int64_t n, const uint32_t* M, const double* T, float* out,
                               hipStream_t s) {
    const int grid = grid_for_rows((n + (64 / L.G) - 1) / (64 / L.G));
    HFR_LAYOUT_DISPATCH(L, hipLaunchKernelGGL((k_estimate_all<G_, DW_>), dim3(grid), dim3(256), 0, s, M, T, out, n, L.J,
                                              L.P));
    return hipGetLastError();
}

// Merge (Eq. sketch-merge) of the rows of `count` vertices, then estimate.
// One block of 256 threads; each thread owns dwords q = tid, tid + 256, ...
__global__ void k_estimate_set(const uint32_t* __restrict__ M, const int32_t* __restrict__ verts, int64_t count,
                               const double* __restrict__ T, float* out, int J, int P) {
    __shared__ uint32_t sh[4];
    uint32_t s = 0;
    for (int q = threadIdx.x; q < P; q += 256) {
        uint32_t acc = 0;
        for (int64_t i = 0; i < count; ++i) acc = byte_max(acc, M[(int64_t)verts[i] * P + q]);
        s = __builtin_amdgcn_sad_u8(acc, 0u, s);
    }
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) *out = (float)estimate_from_sum(s, J, T);
}

hipError_t launch_estimate_set(const Layout& L, const uint32_t* M, const int32_t* verts, int64_t count,
                               const double* T, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_estimate_set, dim3(1), dim3(256), 0, s, M, verts, count, T, out, L.J, L.P);
    return hipGetLastError();
}

// Blocked bits -> one byte per (vertex, register), vertex-major.
__global__ void k_blocked_to_bytes(const uint32_t* __restrict__ blk, uint8_t* out, int64_t n, int J, int P, int PW) {
    const int64_t total = n * J;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = i / J;
        const int j = (int)(i % J);
        const int q = j >> 2, k = j & 3;
        out[i] = (uint8_t)((blk[v * 4 * PW + k * PW + (q >> 5)] >> (q & 31)) & 1u);
    }
}

hipError_t launch_blocked_to_bytes(const Layout& L, int64_t n, const uint32_t* blk, uint8_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_blocked_to_bytes, dim3(4096), dim3(256), 0, s, blk, out, n, L.J, L.P, L.PW);
    return hipGetLastError();
}

}  // namespace hfr
