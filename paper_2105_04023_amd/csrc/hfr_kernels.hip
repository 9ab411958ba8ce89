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

#include "hfr_internal.h"

namespace hfr {

#define DEVI __device__ __forceinline__

// ----------------------------------------------------------------------------
// MurmurHash3 x86_32 for 4- and 8-byte keys (public-domain algorithm).
// ----------------------------------------------------------------------------
DEVI uint32_t rotl32(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }
DEVI uint32_t mm3_round(uint32_t h, uint32_t k) {
    k *= 0xcc9e2d51u;
    k = rotl32(k, 15);
    k *= 0x1b873593u;
    h ^= k;
    h = rotl32(h, 13);
    return h * 5u + 0xe6546b64u;
}
DEVI uint32_t mm3_tail(uint32_t h, uint32_t len) {
    h ^= len;
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}
DEVI uint32_t mm3_key4(uint32_t a, uint32_t seed) { return mm3_tail(mm3_round(seed, a), 4u); }
DEVI uint32_t mm3_key8(uint32_t a, uint32_t b, uint32_t seed) { return mm3_tail(mm3_round(mm3_round(seed, a), b), 8u); }

DEVI uint32_t lead_zeros(uint32_t x) { return x == 0u ? 32u : (uint32_t)__builtin_clz(x); }

// ----------------------------------------------------------------------------
// Packed byte helpers (register values are <= 32).
// ----------------------------------------------------------------------------
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

DEVI uint32_t pk_max16(uint32_t a, uint32_t b) {
    u16x2 x = __builtin_bit_cast(u16x2, a);
    u16x2 y = __builtin_bit_cast(u16x2, b);
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(x, y));
}

// Byte-wise max of two packed dwords.
DEVI uint32_t byte_max(uint32_t a, uint32_t b) {
    return pk_max16(a & 0x00FF00FFu, b & 0x00FF00FFu) | pk_max16(a & 0xFF00FF00u, b & 0xFF00FF00u);
}

// Accumulator of merged registers split into even bytes (0, 2) and odd bytes
// (1, 3) so that one v_pk_max_u16 merges two registers.
struct Acc {
    uint32_t e, o;
};

// Merge neighbour dword d into acc for the simulations whose edge is live.
// Simulation k of this dword is live iff (x_k xor hh) < thr; both sides are
// below 2^31, so the sign bit of (x_k xor hh) - thr is the live bit.  v_perm
// selectors 9 and 11 replicate bit 31 of the low / high source into a byte.
DEVI void merge_live(Acc& acc, uint32_t d, uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3, uint32_t hh,
                     uint32_t negthr) {
    uint32_t s0 = (x0 ^ hh) + negthr;
    uint32_t s1 = (x1 ^ hh) + negthr;
    uint32_t s2 = (x2 ^ hh) + negthr;
    uint32_t s3 = (x3 ^ hh) + negthr;
    uint32_t me = __builtin_amdgcn_perm(s2, s0, 0x0C0B0C09u);  // bytes 0, 2
    uint32_t mo = __builtin_amdgcn_perm(s3, s1, 0x0B0C090Cu);  // bytes 1, 3
    acc.e = pk_max16(acc.e, d & me);
    acc.o = pk_max16(acc.o, d & mo);
}

// Max of row dword a with an accumulator.
DEVI uint32_t acc_max(uint32_t a, const Acc& acc) {
    return pk_max16(a & 0x00FF00FFu, acc.e) | pk_max16(a & 0xFF00FF00u, acc.o);
}

DEVI uint32_t bit_of(const uint32_t* __restrict__ bm, int64_t v) { return (bm[v >> 5] >> (v & 31)) & 1u; }

// Byte mask of the unblocked registers of dword q of vertex u.
DEVI uint32_t unblocked_mask(const uint32_t* __restrict__ blk, int64_t u, int q, int PW) {
    const uint32_t* b = blk + u * 4 * PW + (q >> 5);
    const int s = q & 31;
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) m |= (((b[k * PW] >> s) & 1u) ? 0u : 0xFFu) << (8 * k);
    return m;
}

template <typename T>
DEVI T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the 256 threads of a block; result valid in thread 0.
template <typename T>
DEVI T block_sum256(T v, T* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    T r = 0;
    if (threadIdx.x == 0) r = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return r;
}

// True if any lane of this lane's G-lane group has `c` set.
template <int G>
DEVI bool group_any(bool c) {
    const uint64_t b = __ballot(c);
    if constexpr (G == 64) {
        return b != 0;
    } else {
        const int grp = (threadIdx.x & 63) / G;
        return ((b >> (grp * G)) & ((1ull << G) - 1)) != 0;
    }
}

template <int G>
DEVI bool group_all(bool c) {
    return !group_any<G>(!c);
}

DEVI int64_t wave_index() { return __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6)); }
DEVI int64_t wave_count() { return (int64_t)(gridDim.x * blockDim.x) >> 6; }

DEVI uint32_t gate_sum(const uint32_t* __restrict__ gate) {
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < NSLOT; ++i) s += gate[i * SLOT_U32];
    return s;
}

DEVI uint32_t edge_thr(int kind, uint32_t tconst, const uint32_t* __restrict__ thr, int64_t e, int32_t v) {
    return kind == THR_CONST ? tconst : (kind == THR_TARGET ? thr[v] : thr[e]);
}

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

// Eq. (hash): h(u, v) = Murmur3(LE32(u) || LE32(v)) mod 2^31.  One wave per
// row, lanes stride over its edges.
__global__ void k_edge_hash(const int64_t* __restrict__ xadj, const int32_t* __restrict__ adj, uint32_t* eh,
                            int64_t n, uint32_t seed) {
    const int lane = threadIdx.x & 63;
    for (int64_t u = wave_index(); u < n; u += wave_count()) {
        const int64_t eb = xadj[u], ee = xadj[u + 1];
        for (int64_t e = eb + lane; e < ee; e += 64) eh[e] = mm3_key8((uint32_t)u, (uint32_t)adj[e], seed) & 0x7FFFFFFFu;
    }
}

hipError_t launch_edge_hash(const DevGraph& g, uint32_t seed, hipStream_t s) {
    hipLaunchKernelGGL(k_edge_hash, dim3(8192), dim3(256), 0, s, g.xadj, g.adj, g.eh, g.n, seed);
    return hipGetLastError();
}

__global__ void k_indegree(const int32_t* __restrict__ adj, int64_t m, uint32_t* indeg) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&indeg[adj[e]], 1u);
}

hipError_t launch_indegree(const DevGraph& g, uint32_t* indeg, hipStream_t s) {
    if (g.m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_indegree, dim3(8192), dim3(256), 0, s, g.adj, g.m, indeg);
    return hipGetLastError();
}

// Weighted cascade (Sec. 2.1): w_uv = 1/d_v as the binary32 quotient
// 1.0f / (float)d_v.  For an integer-valued binary32 divisor below 2^24 in
// mantissa, the double quotient rounded to binary32 equals the correctly
// rounded binary32 quotient (its binary expansion has no run of 28 equal
// bits), so the double route is exact.
__global__ void k_wc_thresholds(const uint32_t* __restrict__ indeg, uint32_t* thr, int64_t n) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t d = indeg[v];
        if (d == 0) {
            thr[v] = 0;
            continue;
        }
        const float df = (float)d;
        const float w = (float)(1.0 / (double)df);
        thr[v] = live_threshold(w);
    }
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

hipError_t launch_sim_words(uint32_t* X, uint32_t* HJ, int J, uint32_t seed, hipStream_t s) {
    hipLaunchKernelGGL(k_sim_words, dim3((J + 255) / 256), dim3(256), 0, s, X, HJ, J, seed);
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
// changed or u is in L_t (then B still holds M^{t-1}[u]).  Rows with more
// than heavy_deg out-edges are handled by k_sweep_heavy / k_sweep_heavy_fix.
//
// A wave owns 32 consecutive rows per chunk and stores the chunk's L_{t+1}
// bitmap word with a plain store.
// ----------------------------------------------------------------------------

// Copies a wave-uniform value into a VGPR, so that v_xad_u32 can take the
// edge hash as its single scalar operand.
DEVI uint32_t to_vgpr(uint32_t s) {
    uint32_t v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
    return v;
}

constexpr int UB = 8;  // neighbour rows in flight per wave

// G = 64 (one row per wave): the row's out-edges are read 64 at a time with
// one coalesced load per array, the heads in L_t are found with one ballot,
// and the rows of up to UB live heads are loaded back-to-back before they are
// merged.  Returns the number of edges with a live head.
template <int DW, int KIND>
DEVI uint32_t merge_edges64(int64_t eb, int64_t ee, const int32_t* __restrict__ adj, const uint32_t* __restrict__ eh,
                            const uint32_t* __restrict__ thr, uint32_t ntv, const uint32_t* __restrict__ A,
                            const uint32_t* __restrict__ Lcur, int first, int P, int lane,
                            const uint32_t (&x)[DW][4], Acc (&acc)[DW]) {
    uint32_t vis = 0;
    for (int64_t w0 = eb; w0 < ee; w0 += 64) {
        const int64_t e = w0 + lane;
        const bool in = e < ee;
        const int32_t v = in ? adj[e] : 0;
        const bool lv = in && (first || bit_of(Lcur, v) != 0u);
        uint64_t mask = __ballot(lv);
        if (mask == 0) continue;
        vis += (uint32_t)__builtin_popcountll(mask);
        const uint32_t hh = lv ? eh[e] : 0u;
        uint32_t tt = 0u;
        if constexpr (KIND == THR_TARGET) tt = lv ? thr[v] : 0u;
        if constexpr (KIND == THR_EDGE) tt = lv ? thr[e] : 0u;
        while (mask) {
            const int pc = __builtin_popcountll(mask);
            const int cnt = pc < UB ? pc : UB;
            int idx[UB];
#pragma unroll
            for (int b = 0; b < UB; ++b) {
                idx[b] = mask ? __builtin_ctzll(mask) : 0;
                mask &= mask - 1;
            }
            uint32_t d[UB][DW];
#pragma unroll
            for (int b = 0; b < UB; ++b) {
#pragma unroll
                for (int i = 0; i < DW; ++i) d[b][i] = 0u;
                if (b < cnt) {
                    const int64_t vb = __builtin_amdgcn_readlane(v, idx[b]);
                    const uint32_t* __restrict__ row = A + vb * P;
#pragma unroll
                    for (int i = 0; i < DW; ++i) {
                        const int q = i * 64 + lane;
                        if (q < P) d[b][i] = row[q];
                    }
                }
            }
#pragma unroll
            for (int b = 0; b < UB; ++b) {
                if (b < cnt) {
                    const uint32_t hb = (uint32_t)__builtin_amdgcn_readlane((int)hh, idx[b]);
                    uint32_t nt = ntv;
                    if constexpr (KIND != THR_CONST) nt = 0u - (uint32_t)__builtin_amdgcn_readlane((int)tt, idx[b]);
#pragma unroll
                    for (int i = 0; i < DW; ++i) merge_live(acc[i], d[b][i], x[i][0], x[i][1], x[i][2], x[i][3], hb, nt);
                }
            }
        }
    }
    return vis;
}

// G < 64 (several rows per wave): each G-lane group walks its own row's edges.
template <int G, int DW, int KIND>
DEVI uint32_t merge_edges_grp(int64_t eb, int64_t ee, const int32_t* __restrict__ adj,
                              const uint32_t* __restrict__ eh, const uint32_t* __restrict__ thr, uint32_t ntv,
                              const uint32_t* __restrict__ A, const uint32_t* __restrict__ Lcur, int first, int P,
                              int p, const uint32_t (&x)[DW][4], Acc (&acc)[DW]) {
    uint32_t vis = 0;
    for (int64_t e = eb; e < ee; ++e) {
        const int32_t v = adj[e];
        if (!first && !bit_of(Lcur, v)) continue;
        ++vis;
        const uint32_t hh = eh[e];
        uint32_t nt = ntv;
        if constexpr (KIND == THR_TARGET) nt = 0u - thr[v];
        if constexpr (KIND == THR_EDGE) nt = 0u - thr[e];
        const uint32_t* __restrict__ row = A + (int64_t)v * P;
#pragma unroll
        for (int i = 0; i < DW; ++i) {
            const int q = i * G + p;
            if (q < P) merge_live(acc[i], row[q], x[i][0], x[i][1], x[i][2], x[i][3], hh, nt);
        }
    }
    return vis;
}

template <int G, int DW, int KIND>
DEVI uint32_t merge_edges(int64_t eb, int64_t ee, const int32_t* __restrict__ adj, const uint32_t* __restrict__ eh,
                          const uint32_t* __restrict__ thr, uint32_t ntv, const uint32_t* __restrict__ A,
                          const uint32_t* __restrict__ Lcur, int first, int P, int lane, int p,
                          const uint32_t (&x)[DW][4], Acc (&acc)[DW]) {
    if constexpr (G == 64)
        return merge_edges64<DW, KIND>(eb, ee, adj, eh, thr, ntv, A, Lcur, first, P, lane, x, acc);
    else
        return merge_edges_grp<G, DW, KIND>(eb, ee, adj, eh, thr, ntv, A, Lcur, first, P, p, x, acc);
}

template <int G, int DW>
DEVI void load_sim_words(const uint32_t* __restrict__ X, int P, int p, uint32_t (&x)[DW][4]) {
#pragma unroll
    for (int i = 0; i < DW; ++i) {
        const int q = i * G + p;
#pragma unroll
        for (int k = 0; k < 4; ++k) x[i][k] = q < P ? X[4 * q + k] : 0u;
    }
}

template <int G, int DW, int KIND>
__global__ __launch_bounds__(256) void k_sweep_light(
    const int64_t* __restrict__ xadj, const int32_t* __restrict__ adj, const uint32_t* __restrict__ eh,
    const uint32_t* __restrict__ thr, uint32_t thr_const, const uint32_t* __restrict__ X,
    const uint32_t* __restrict__ A, uint32_t* __restrict__ B, const uint32_t* __restrict__ Lcur,
    uint32_t* __restrict__ Lnext, const uint32_t* __restrict__ blk, const uint32_t* __restrict__ gate,
    uint32_t gate_thresh, uint32_t* __restrict__ cnt_out, unsigned long long* __restrict__ vis_out, int64_t n,
    int P, int PW, int64_t heavy_deg, int first) {
    __shared__ unsigned long long sh64[4];
    __shared__ uint32_t sh32[4];
    if (!first && gate_sum(gate) <= gate_thresh) return;
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63, grp = lane / G, p = lane % G;
    uint32_t x[DW][4];
    load_sim_words<G, DW>(X, P, p, x);
    const uint32_t ntv = to_vgpr(0u - thr_const);
    uint32_t my_cnt = 0;
    unsigned long long my_vis = 0;
    const int64_t nwords = (n + 31) >> 5;
    for (int64_t c = wave_index(); c < nwords; c += wave_count()) {
        uint32_t word = 0;
        for (int rr = 0; rr < 32; rr += RPW) {
            const int64_t u = c * 32 + rr + grp;
            bool changed = false;
            if (u < n) {
                const int64_t eb = xadj[u], ee = xadj[u + 1];
                const bool inL = first ? false : bit_of(Lcur, u) != 0;
                bool active = ee - eb <= heavy_deg && (ee > eb || inL);
                uint32_t ub[DW];
#pragma unroll
                for (int i = 0; i < DW; ++i) ub[i] = 0xFFFFFFFFu;
                if (active && blk) {
                    bool none = true;
#pragma unroll
                    for (int i = 0; i < DW; ++i) {
                        const int q = i * G + p;
                        if (q < P) {
                            ub[i] = unblocked_mask(blk, u, q, PW);
                            none = none && ub[i] == 0u;
                        }
                    }
                    active = !group_all<G>(none);
                }
                if (active) {
                    Acc acc[DW];
#pragma unroll
                    for (int i = 0; i < DW; ++i) acc[i].e = acc[i].o = 0u;
                    const uint32_t vis =
                        merge_edges<G, DW, KIND>(eb, ee, adj, eh, thr, ntv, A, Lcur, first, P, lane, p, x, acc);
                    if (p == 0) my_vis += vis;
                    if (vis > 0 || inL) {
                        bool ch = false;
                        uint32_t nw[DW];
#pragma unroll
                        for (int i = 0; i < DW; ++i) {
                            const int q = i * G + p;
                            nw[i] = 0;
                            if (q < P) {
                                const uint32_t a = A[u * P + q];
                                nw[i] = acc_max(a, acc[i]) & ub[i];
                                ch = ch || nw[i] != a;
                            }
                        }
                        changed = group_any<G>(ch);
                        if (changed || inL) {
#pragma unroll
                            for (int i = 0; i < DW; ++i) {
                                const int q = i * G + p;
                                if (q < P) B[u * P + q] = nw[i];
                            }
                        }
                    }
                }
            }
            const uint64_t bal = __ballot(changed && p == 0);
#pragma unroll
            for (int g = 0; g < RPW; ++g) word |= (uint32_t)((bal >> (g * G)) & 1ull) << (rr + g);
        }
        if (lane == 0) Lnext[c] = word;
        my_cnt += __builtin_popcount(word);
    }
    if (lane != 0) my_cnt = 0;
    const uint32_t bc = block_sum256(my_cnt, sh32);
    const unsigned long long bv = block_sum256(my_vis, sh64);
    if (threadIdx.x == 0) {
        const int slot = blockIdx.x % NSLOT;
        if (bc) atomicAdd(&cnt_out[slot * SLOT_U32], bc);
        if (bv) atomicAdd(&vis_out[slot * SLOT_U64], bv);
    }
}

// One G-lane group per piece of a split row: merge of the live rows of the
// piece's out-neighbours in L_t, written to part[piece].
template <int G, int DW, int KIND>
__global__ __launch_bounds__(256) void k_sweep_heavy(
    const int32_t* __restrict__ adj, const uint32_t* __restrict__ eh, const uint32_t* __restrict__ thr,
    uint32_t thr_const, const uint32_t* __restrict__ X, const uint32_t* __restrict__ A,
    const uint32_t* __restrict__ Lcur, const uint32_t* __restrict__ blk, const uint32_t* __restrict__ gate,
    uint32_t gate_thresh, unsigned long long* __restrict__ vis_out, const int32_t* __restrict__ hrow,
    const int32_t* __restrict__ prow, const int64_t* __restrict__ pe0, const int64_t* __restrict__ pe1,
    uint32_t* __restrict__ part, uint32_t* __restrict__ part_any, int64_t npieces, int P, int PW, int first) {
    __shared__ unsigned long long sh64[4];
    if (!first && gate_sum(gate) <= gate_thresh) return;
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63, grp = lane / G, p = lane % G;
    uint32_t x[DW][4];
    load_sim_words<G, DW>(X, P, p, x);
    const uint32_t ntv = to_vgpr(0u - thr_const);
    unsigned long long my_vis = 0;
    for (int64_t base = wave_index() * RPW; base < npieces; base += wave_count() * RPW) {
        const int64_t pc = base + grp;
        if (pc >= npieces) continue;
        const int64_t u = hrow[prow[pc]];
        bool skip = false;
        if (blk) {
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
        if (!skip) vis = merge_edges<G, DW, KIND>(pe0[pc], pe1[pc], adj, eh, thr, ntv, A, Lcur, first, P, lane, p, x, acc);
#pragma unroll
        for (int i = 0; i < DW; ++i) {
            const int q = i * G + p;
            if (q < P) part[pc * P + q] = acc[i].e | acc[i].o;
        }
        if (p == 0) {
            part_any[pc] = vis > 0 ? 1u : 0u;
            my_vis += vis;
        }
    }
    const unsigned long long bv = block_sum256(my_vis, sh64);
    if (threadIdx.x == 0 && bv) atomicAdd(&vis_out[(blockIdx.x % NSLOT) * SLOT_U64], bv);
}

// One G-lane group per split row: combine its pieces with its own row.
template <int G, int DW>
__global__ __launch_bounds__(256) void k_sweep_heavy_fix(
    const uint32_t* __restrict__ A, uint32_t* __restrict__ B, const uint32_t* __restrict__ Lcur,
    uint32_t* __restrict__ Lnext, const uint32_t* __restrict__ blk, const uint32_t* __restrict__ gate,
    uint32_t gate_thresh, uint32_t* __restrict__ cnt_out, const int32_t* __restrict__ hrow,
    const int64_t* __restrict__ hpb, const int64_t* __restrict__ hpn, const uint32_t* __restrict__ part,
    const uint32_t* __restrict__ part_any, int64_t nheavy, int P, int PW, int first) {
    __shared__ uint32_t sh32[4];
    if (!first && gate_sum(gate) <= gate_thresh) return;
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63, grp = lane / G, p = lane % G;
    uint32_t my_cnt = 0;
    for (int64_t base = wave_index() * RPW; base < nheavy; base += wave_count() * RPW) {
        const int64_t r = base + grp;
        bool changed = false;
        if (r < nheavy) {
            const int64_t u = hrow[r];
            const bool inL = first ? false : bit_of(Lcur, u) != 0;
            uint32_t ub[DW];
            bool none = true;
#pragma unroll
            for (int i = 0; i < DW; ++i) {
                const int q = i * G + p;
                ub[i] = 0xFFFFFFFFu;
                if (blk && q < P) {
                    ub[i] = unblocked_mask(blk, u, q, PW);
                    none = none && ub[i] == 0u;
                }
            }
            const bool skip = blk ? group_all<G>(none) : false;
            if (!skip) {
                const int64_t pb = hpb[r], pe = pb + hpn[r];
                uint32_t acc[DW];
                bool any = false;
#pragma unroll
                for (int i = 0; i < DW; ++i) acc[i] = 0u;
                for (int64_t pc = pb; pc < pe; ++pc) {
                    any = any || part_any[pc] != 0u;
#pragma unroll
                    for (int i = 0; i < DW; ++i) {
                        const int q = i * G + p;
                        if (q < P) acc[i] = byte_max(acc[i], part[pc * P + q]);
                    }
                }
                if (any || inL) {
                    bool ch = false;
                    uint32_t nw[DW];
#pragma unroll
                    for (int i = 0; i < DW; ++i) {
                        const int q = i * G + p;
                        nw[i] = 0;
                        if (q < P) {
                            const uint32_t a = A[u * P + q];
                            nw[i] = byte_max(a, acc[i]) & ub[i];
                            ch = ch || nw[i] != a;
                        }
                    }
                    changed = group_any<G>(ch);
                    if (changed || inL) {
#pragma unroll
                        for (int i = 0; i < DW; ++i) {
                            const int q = i * G + p;
                            if (q < P) B[u * P + q] = nw[i];
                        }
                    }
                    if (changed && p == 0) {
                        atomicOr(&Lnext[u >> 5], 1u << (u & 31));
                        my_cnt += 1;
                    }
                }
            }
        }
    }
    const uint32_t bc = block_sum256(my_cnt, sh32);
    if (threadIdx.x == 0 && bc) atomicAdd(&cnt_out[(blockIdx.x % NSLOT) * SLOT_U32], bc);
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
                        hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    const int64_t words = (g.n + 31) / 32;
    int lg = grid > 0 ? grid : grid_for_rows(words);
    if (ev0) (void)hipEventRecord(ev0, s);
    HFR_LAYOUT_DISPATCH(L, HFR_KIND_DISPATCH(g.kind, hipLaunchKernelGGL((k_sweep_light<G_, DW_, K_>), dim3(lg),
                                                                        dim3(256), 0, s, g.xadj, g.adj, g.eh, g.thr,
                                                                        g.thr_const, X, sp.A, sp.B, sp.Lcur, sp.Lnext,
                                                                        sp.blk, sp.gate, sp.gate_thresh, sp.cnt_out,
                                                                        sp.vis_out, g.n, L.P, L.PW, g.heavy_deg,
                                                                        sp.first)));
    if (ev1) (void)hipEventRecord(ev1, s);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    if (g.npieces > 0) {
        const int rpw = 64 / L.G;
        const int hg = grid_for_rows((g.npieces + rpw - 1) / rpw);
        HFR_LAYOUT_DISPATCH(L, HFR_KIND_DISPATCH(g.kind, hipLaunchKernelGGL((k_sweep_heavy<G_, DW_, K_>), dim3(hg),
                                                                            dim3(256), 0, s, g.adj, g.eh, g.thr,
                                                                            g.thr_const, X, sp.A, sp.Lcur, sp.blk,
                                                                            sp.gate, sp.gate_thresh, sp.vis_out,
                                                                            g.hrow, g.prow, g.pe0, g.pe1, sp.part,
                                                                            sp.part_any, g.npieces, L.P, L.PW,
                                                                            sp.first)));
        err = hipGetLastError();
        if (err != hipSuccess) return err;
        const int fg = grid_for_rows((g.nheavy + rpw - 1) / rpw);
        HFR_LAYOUT_DISPATCH(L, hipLaunchKernelGGL((k_sweep_heavy_fix<G_, DW_>), dim3(fg), dim3(256), 0, s, sp.A, sp.B,
                                                  sp.Lcur, sp.Lnext, sp.blk, sp.gate, sp.gate_thresh, sp.cnt_out,
                                                  g.hrow, g.hpb, g.hpn, sp.part, sp.part_any, g.nheavy, L.P,
                                                  L.PW, sp.first));
        err = hipGetLastError();
    }
    return err;
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
    const int lane = threadIdx.x & 63, grp = lane / G, p = lane % G;
    uint32_t ms[DW];
#pragma unroll
    for (int i = 0; i < DW; ++i) {
        const int q = i * G + p;
        ms[i] = q < P ? MS[q] : 0u;
    }
    unsigned long long best = 0;
    for (int64_t base = wave_index() * RPW; base < n; base += wave_count() * RPW) {
        const int64_t u = base + grp;
        const bool ok = u < n && inS[u] == 0;
        uint32_t s = 0;
        if (ok) {
#pragma unroll
            for (int i = 0; i < DW; ++i) {
                const int q = i * G + p;
                if (q < P) s = __builtin_amdgcn_sad_u8(byte_max(ms[i], M[u * P + q]), 0u, s);
            }
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (ok && p == 0) {
            const unsigned long long key = ((unsigned long long)s << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)u);
            best = key > best ? key : best;
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
        unsigned long long b = sh[0];
        for (int i = 1; i < 4; ++i) b = sh[i] > b ? sh[i] : b;
        if (b) atomicMax(key_out, b);
    }
}

hipError_t launch_argmax(const Layout& L, int64_t n, const uint32_t* M, const GreedyBufs& b, hipStream_t s) {
    const int grid = grid_for_rows((n + (64 / L.G) - 1) / (64 / L.G));
    HFR_LAYOUT_DISPATCH(L, hipLaunchKernelGGL((k_argmax<G_, DW_>), dim3(grid), dim3(256), 0, s, M, b.MS, b.inS, b.key,
                                              n, L.P));
    return hipGetLastError();
}

DEVI uint32_t plane_valid_mask(int w, int P, int PW) {
    const int ww = w % PW;  // word within the plane
    const int left = P - 32 * ww;
    return left >= 32 ? 0xFFFFFFFFu : (left <= 0 ? 0u : ((1u << left) - 1u));
}

DEVI double estimate_from_sum(uint32_t s, int J, const double* __restrict__ T) {
    const uint32_t q = s / (uint32_t)J, r = s % (uint32_t)J;
    return ldexp(T[r], (int)q) / 0.77351;
}

// One wave: takes the argmax, records the step, computes e = Estimate(Merge(M_S',
// M_s)) and starts the Monte-Carlo reach of s: every pair (s, j) not blocked
// yet becomes blocked and forms the level-0 frontier.
__global__ void k_select(const int64_t* __restrict__ xadj, const uint32_t* __restrict__ M, GreedyBufs b, StepRec* rec,
                         int32_t* seeds, int k, int J, int P, int PW, int32_t level_id, int64_t n) {
    const int lane = threadIdx.x;
    const unsigned long long key = *b.key;
    const int64_t s = (int64_t)(0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull));
    if (key == 0ull || s >= n) {  // no candidate: report and touch nothing else
        if (lane == 0) {
            rec->seed = -1;
            seeds[k] = -1;
            b.qsize[0] = 0u;
        }
        return;
    }
    uint32_t sum = 0;
    for (int q = lane; q < P; q += 64) {
        const uint32_t mg = byte_max(b.MS[q], M[s * P + q]);
        b.merged[q] = mg;
        sum = __builtin_amdgcn_sad_u8(mg, 0u, sum);
    }
    sum = wave_sum(sum);
    const int64_t deg = xadj[s + 1] - xadj[s];
    uint32_t newcnt = 0;
    for (int w = lane; w < 4 * PW; w += 64) {
        const uint32_t old = b.blk[s * 4 * PW + w];
        const uint32_t nb = ~old & plane_valid_mask(w, P, PW);
        b.blk[s * 4 * PW + w] = old | nb;
        newcnt += __builtin_popcount(nb);
        if (deg > 0) b.F[0][s * 4 * PW + w] = nb;
    }
    newcnt = wave_sum(newcnt);
    const int64_t nch = (deg > 0 && newcnt > 0) ? (deg + b.bfs_chunk - 1) / b.bfs_chunk : 0;
    for (int64_t c = lane; c < nch; c += 64) b.Q[0][c] = make_int2((int)s, (int)c);
    if (lane == 0) {
        b.inS[s] = 1;
        seeds[k] = (int32_t)s;
        rec->seed = (int32_t)s;
        rec->score = (int64_t)(key >> 32);
        rec->e = estimate_from_sum(sum, J, b.T);
        b.qsize[0] = (uint32_t)nch;
        if (nch) b.stamp[s] = level_id;
        if (newcnt) atomicAdd(&b.R[0], (unsigned long long)newcnt);
        *b.key = 0ull;
    }
}

hipError_t launch_select(const Layout& L, const DevGraph& g, const uint32_t* M, const GreedyBufs& b, StepRec* rec,
                         int32_t* seeds_dev, int k, int32_t level_id, hipStream_t s) {
    hipLaunchKernelGGL(k_select, dim3(1), dim3(64), 0, s, g.xadj, M, b, rec, seeds_dev, k, L.J, L.P, L.PW, level_id,
                       g.n);
    return hipGetLastError();
}

// One BFS level of the Monte-Carlo reach over all samples at once.  A queue
// entry is (vertex v, chunk c) covering at most bfs_chunk out-edges of v.  For
// each edge (v, w): the samples where the edge is live and v is in the
// frontier are OR-ed into w's blocked bits; bits that were not set before
// form w's frontier of the next level, and w is queued once per level.
template <int G, int DW>
__global__ __launch_bounds__(256) void k_bfs_expand(const int64_t* __restrict__ xadj, const int32_t* __restrict__ adj,
                                                    const uint32_t* __restrict__ eh, const uint32_t* __restrict__ thr,
                                                    uint32_t thr_const, int kind, const uint32_t* __restrict__ X,
                                                    GreedyBufs b, int cur, int32_t level_id_next, int P, int PW) {
    __shared__ unsigned long long sh64[4];
    const uint32_t size = b.qsize[cur % 3];
    if (size == 0) return;
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63, grp = lane / G, p = lane % G;
    const uint32_t* __restrict__ Fc = b.F[cur & 1];
    uint32_t* Fn = b.F[(cur + 1) & 1];
    const int2* __restrict__ Qc = b.Q[cur & 1];
    int2* Qn = b.Q[(cur + 1) & 1];
    uint32_t* qn = &b.qsize[(cur + 1) % 3];
    uint32_t x[DW][4];
#pragma unroll
    for (int i = 0; i < DW; ++i) {
        const int q = i * G + p;
#pragma unroll
        for (int k = 0; k < 4; ++k) x[i][k] = q < P ? X[4 * q + k] : 0u;
    }
    unsigned long long my_new = 0;
    const int W = 4 * PW;
    for (int64_t base = wave_index() * RPW; base < (int64_t)size; base += wave_count() * RPW) {
        const int64_t ent = base + grp;
        const bool ok = ent < (int64_t)size;
        int64_t e0 = 0, e1 = 0, v = 0;
        uint32_t fb[DW];  // frontier bits of this lane's 4*DW registers, bit (4i + k)
        if (ok) {
            const int2 qe = Qc[ent];
            v = qe.x;
            const int64_t vb = xadj[v], ve = xadj[v + 1];
            e0 = vb + (int64_t)qe.y * b.bfs_chunk;
            e1 = e0 + b.bfs_chunk < ve ? e0 + b.bfs_chunk : ve;
#pragma unroll
            for (int i = 0; i < DW; ++i) {
                const int q = i * G + p;
                uint32_t f = 0;
                if (q < P) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) f |= ((Fc[v * W + k * PW + (q >> 5)] >> (q & 31)) & 1u) << k;
                }
                fb[i] = f;
            }
        }
        for (int64_t e = e0; e < e1; ++e) {
            const int64_t w = adj[e];
            const uint32_t hh = eh[e];
            const uint32_t nt = 0u - edge_thr(kind, thr_const, thr, e, (int32_t)w);
            const int64_t wdeg = xadj[w + 1] - xadj[w];
            bool anynew = false;
#pragma unroll
            for (int i = 0; i < DW; ++i) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const bool c = (((x[i][k] ^ hh) + nt) >> 31) & (fb[i] >> k) & 1u;
                    const uint64_t bal = __ballot(c);
                    // plane word(s) this group contributes for (i, k)
                    if constexpr (G == 64) {
                        const uint32_t lo = (uint32_t)bal, hi = (uint32_t)(bal >> 32);
                        const int wlo = k * PW + 2 * i;
                        // lanes 0/1 of the wave issue the two atomics
                        uint32_t val = lane == 0 ? lo : (lane == 1 ? hi : 0u);
                        if (val) {
                            const int wi = wlo + lane;
                            const uint32_t old = atomicOr(&b.blk[w * W + wi], val);
                            const uint32_t nb = val & ~old;
                            if (nb) {
                                if (wdeg > 0) atomicOr(&Fn[w * W + wi], nb);
                                my_new += __builtin_popcount(nb);
                                anynew = true;
                            }
                        }
                    } else {
                        const uint32_t val = p == 0 ? (uint32_t)((bal >> (grp * G)) & ((1ull << G) - 1)) : 0u;
                        if (val) {
                            const int wi = k * PW;
                            const uint32_t old = atomicOr(&b.blk[w * W + wi], val);
                            const uint32_t nb = val & ~old;
                            if (nb) {
                                if (wdeg > 0) atomicOr(&Fn[w * W + wi], nb);
                                my_new += __builtin_popcount(nb);
                                anynew = true;
                            }
                        }
                    }
                }
            }
            const bool gnew = group_any<G>(anynew);
            if (gnew && wdeg > 0) {
                int64_t pos = 0, nch = 0;
                if (p == 0) {
                    const int32_t old = atomicMax(&b.stamp[w], level_id_next);
                    if (old < level_id_next) {
                        nch = (wdeg + b.bfs_chunk - 1) / b.bfs_chunk;
                        pos = atomicAdd(qn, (uint32_t)nch);
                    }
                }
                nch = __shfl(nch, grp * G, 64);
                pos = __shfl(pos, grp * G, 64);
                for (int64_t c = p; c < nch; c += G) Qn[pos + c] = make_int2((int)w, (int)c);
            }
        }
    }
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
        if (qe.y == 0) Fc[(int64_t)qe.x * W + (i % W)] = 0u;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) b.qsize[3] += 1u;
}

hipError_t launch_bfs_level(const Layout& L, const DevGraph& g, const uint32_t* X, const GreedyBufs& b, int level,
                            int32_t level_id_next, int grid, hipStream_t s) {
    HFR_LAYOUT_DISPATCH(L, hipLaunchKernelGGL((k_bfs_expand<G_, DW_>), dim3(grid), dim3(256), 0, s, g.xadj, g.adj, g.eh,
                                              g.thr, g.thr_const, g.kind, X, b, level, level_id_next, L.P, L.PW));
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_bfs_cleanup, dim3(256), dim3(256), 0, s, b, level, L.PW);
    return hipGetLastError();
}

// Error-adaptive decision of Alg. 1 in FP64 (one wave; lane 0 computes).
__global__ void k_decide(GreedyBufs b, StepRec* rec, int k, int K, double eps_g, double eps_l, int J, int P,
                         int32_t* rebuild_flag) {
    __shared__ int flags[2];
    const int lane = threadIdx.x;
    if (lane == 0) {
        unsigned long long R = 0;
        for (int i = 0; i < NSLOT; ++i) R += b.R[i * SLOT_U64];
        const unsigned long long R0 = *b.Rreb;
        const double sigma = (double)R / (double)J;
        const double delta = (double)(R - R0) / (double)J;
        const double e = rec->e;
        const double err_l = delta == 0.0 ? __builtin_inf() : fabs((e - delta) / delta);
        const double err_g = fabs((e - delta) / sigma);
        const int fresh = (err_l < eps_l) || (err_g < eps_g);
        const int rebuild = (k < K) && !fresh;
        rec->reach = (int64_t)R;
        rec->sigma = sigma;
        rec->delta = delta;
        rec->err_l = err_l;
        rec->err_g = err_g;
        rec->fresh = fresh;
        rec->rebuilt = rebuild;
        rec->sweeps = 0;
        rec->visits = 0;
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
