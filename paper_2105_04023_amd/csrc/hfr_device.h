// Device helpers shared by the kernels of the single-graph path and of the
// batched solver: Murmur3, packed register arithmetic, the fused live test,
// bit and wave utilities.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

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

// The 31-bit hash of edge e = (u, v) (Eq. hash): read from a precomputed array,
// or -- with eh null -- recomputed from the two ids (two Murmur3 rounds and the
// finaliser, about twenty integer instructions), which saves the 4-byte load
// and the cache line it costs a merged edge whose neighbours are not merged.
struct EdgeHashes {
    const uint32_t* eh;
    uint32_t seed;
};
DEVI uint32_t edge_hash_of(const EdgeHashes& H, int64_t e, uint32_t u, uint32_t v) {
    return H.eh ? H.eh[e] : (mm3_key8(u, v, H.seed) & 0x7FFFFFFFu);
}

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

// Whether head v is in L_t.  With cl set (a coarse copy of L_t in LDS, one bit
// per 2^cs vertices, set if any of them is in L_t), a head whose coarse bit is
// clear is answered without the load from the bitmap in memory.
DEVI bool in_L(const uint32_t* __restrict__ Lcur, const uint32_t* cl, int cs, int64_t v) {
    if (cl && ((cl[v >> (cs + 5)] >> ((v >> cs) & 31)) & 1u) == 0u) return false;
    return bit_of(Lcur, v) != 0u;
}

// Byte mask of the unblocked registers of dword q of vertex u.
DEVI uint32_t unblocked_mask(const uint32_t* __restrict__ blk, int64_t u, int q, int PW) {
    const uint32_t* b = blk + u * 4 * PW + (q >> 5);
    const int s = q & 31;
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) m |= (((b[k * PW] >> s) & 1u) ? 0u : 0xFFu) << (8 * k);
    return m;
}

DEVI uint32_t plane_valid_mask(int w, int P, int PW) {
    const int ww = w % PW;  // word within the plane
    const int left = P - 32 * ww;
    return left >= 32 ? 0xFFFFFFFFu : (left <= 0 ? 0u : ((1u << left) - 1u));
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

// Exclusive prefix of c over the wave and the wave total.
DEVI uint32_t wave_excl_scan(uint32_t c, uint32_t* total) {
    const int lane = threadIdx.x & 63;
    uint32_t x = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    *total = __shfl(x, 63, 64);
    return x - c;
}

// Lane j's value of x (j wave-uniform), as a scalar.
DEVI int64_t readlane64(int64_t x, int j) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)x >> 32), j);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

DEVI int64_t wave_index() { return __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6)); }
DEVI int64_t wave_count() { return (int64_t)(gridDim.x * blockDim.x) >> 6; }

DEVI uint32_t gate_sum(const uint32_t* __restrict__ gate) {
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < NSLOT; ++i) s += gate[i * SLOT_U32];
    return s;
}

// Weighted cascade (Sec. 2.1): w_uv = 1/d_v as the binary32 quotient
// 1.0f / (float)d_v, turned into its integer live threshold.  For an
// integer-valued binary32 divisor below 2^24 in mantissa, the double quotient
// rounded to binary32 equals the correctly rounded binary32 quotient (its
// binary expansion has no run of 28 equal bits), so the double route is exact.
// A vertex without in-edges gets threshold 0.
DEVI uint32_t wc_threshold(uint32_t d) {
    if (d == 0) return 0u;
    const float df = (float)d;
    const float w = (float)(1.0 / (double)df);
    return live_threshold(w);
}

// Copies a wave-uniform value into a VGPR, so that v_xad_u32 can take the
// edge hash as its single scalar operand.
DEVI uint32_t to_vgpr(uint32_t s) {
    uint32_t v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
    return v;
}

// Eq. (sketch-estimate) from the integer register sum s: 2^(s div J) *
// exp2((s mod J) / J) / 0.77351, with the exp2 table T computed on the host.
DEVI double estimate_from_sum(uint32_t s, int J, const double* __restrict__ T) {
    const uint32_t q = s / (uint32_t)J, r = s % (uint32_t)J;
    return ldexp(T[r], (int)q) / 0.77351;
}

// ----------------------------------------------------------------------------
// Merge of a row's out-edges (Alg. 2): for every out-neighbour v in L_t and
// every live sample, acc = max(acc, M^t[v]).
// ----------------------------------------------------------------------------
constexpr int UB = 8;  // neighbour rows in flight per wave (twice that with one dword per lane)

// G = 64: merges one window of up to 64 out-edges of row u, lane l holding edge
// e (in: the edge exists) with head v, `mask` the lanes whose head is in L_t (not
// empty, edges live in no sample already dropped).  The rows of up to UB heads
// are loaded back-to-back before they are merged.  Returns the number of rows
// merged.
template <int DW, int KIND>
DEVI uint32_t merge_window64(uint64_t mask, int64_t e, bool in, int32_t v, uint32_t u, const EdgeHashes& H,
                             const uint32_t* __restrict__ thr, uint32_t ntv, const uint32_t* __restrict__ A, int P,
                         int lane, const uint32_t (&x)[DW][4], Acc (&acc)[DW]) {
    // hashes and thresholds of the merged edges only: a sparse mask then
    // fetches only the cache lines it needs
    const uint32_t merged = (uint32_t)__builtin_popcountll(mask);
    const bool mine = ((mask >> lane) & 1ull) != 0ull;
    const uint32_t hh = mine ? edge_hash_of(H, e, u, (uint32_t)v) : 0u;
    uint32_t ntt = 0u;  // negated threshold
    if constexpr (KIND == THR_TARGET) ntt = 0u - (mine ? thr[v] : 0u);
    if constexpr (KIND == THR_EDGE) ntt = 0u - (mine ? thr[e] : 0u);
    // dword of a neighbour row this lane loads (lanes past the row load its last dword; their
    // results are never stored), unsigned so that a row load takes the row base as its
    // scalar address
    uint32_t qo[DW];
#pragma unroll
    for (int i = 0; i < DW; ++i) qo[i] = (uint32_t)(i * 64 + lane < P ? i * 64 + lane : P - 1);
    // batches of NB live edges, NB the smallest of 1, 2, 4, UB that covers the
    // edges left (capped at UB): unused slots repeat the last edge (max-merge is
    // idempotent), so every load of a batch is issued without a branch
    auto batch = [&](auto nbc) {
        constexpr int NB = decltype(nbc)::value;
        int idx[NB];
        int last = __builtin_ctzll(mask);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (mask) last = __builtin_ctzll(mask);
            idx[b] = last;
            mask &= mask - 1;
        }
        uint32_t d[NB][DW];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int64_t vb = __builtin_amdgcn_readlane(v, idx[b]);
            const uint32_t* __restrict__ row = A + vb * P;
#pragma unroll
            for (int i = 0; i < DW; ++i) d[b][i] = row[qo[i]];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const uint32_t hb = (uint32_t)__builtin_amdgcn_readlane((int)hh, idx[b]);
            uint32_t nt = ntv;
            // in a VGPR, so that each live test is one v_xad_u32 with hb as its scalar operand
            if constexpr (KIND != THR_CONST) nt = to_vgpr((uint32_t)__builtin_amdgcn_readlane((int)ntt, idx[b]));
#pragma unroll
            for (int i = 0; i < DW; ++i) merge_live(acc[i], d[b][i], x[i][0], x[i][1], x[i][2], x[i][3], hb, nt);
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
    return merged;
}

// G = 64 (one row per wave): the row's out-edges are read NW windows of 64
// at a time, with one coalesced load per window and array; the L_t tests of
// the NW windows are issued together, so that a sweep with few live heads
// waits on one round of dependent loads per NW windows.  Returns the number
// of edges with a live head.
constexpr int NW = 4;
template <int DW, int KIND>
DEVI uint32_t merge_edges64(int64_t eb, int64_t ee, uint32_t u, const int32_t* __restrict__ adj,
                            const EdgeHashes& H, const uint32_t* __restrict__ thr, uint32_t ntv, const uint32_t* __restrict__ A,
                            const uint32_t* __restrict__ Lcur, int first, int P, int lane,
                            const uint32_t (&x)[DW][4], Acc (&acc)[DW], const uint32_t* cl = nullptr, int cs = 0,
                            unsigned long long* mrg = nullptr) {
    uint32_t vis = 0;
    for (int64_t c0 = eb; c0 < ee; c0 += 64 * NW) {
        int32_t vw[NW];
        bool inw[NW];
        uint64_t dm[NW];  // edges live in no sample
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            inw[w] = c0 + 64 * w + lane < ee;
            const int32_t a = inw[w] ? adj[c0 + 64 * w + lane] : 0;
            vw[w] = adj_target(a);
            dm[w] = __ballot(adj_dead(a));
        }
        uint64_t mw[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) mw[w] = __ballot(inw[w] && (first || in_L(Lcur, cl, cs, vw[w])));
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            if (!mw[w]) continue;  // no live head: the window needs no hash or threshold
            vis += (uint32_t)__builtin_popcountll(mw[w]);
            const uint64_t mm = mw[w] & ~dm[w];  // edges live in no sample merge nothing
            if (!mm) continue;
            const uint32_t mg =
                merge_window64<DW, KIND>(mm, c0 + 64 * w + lane, inw[w], vw[w], u, H, thr, ntv, A, P, lane, x, acc);
            if (mrg) *mrg += mg;
        }
    }
    return vis;
}

// G = 64: merges the 64-edge windows of [eb, ee) named by the bits of wm
// (window i starts at eb + 64 i), NW of them at a time with their loads and
// L_t tests issued together.  Returns the number of edges with a live head.
template <int DW, int KIND>
DEVI uint32_t merge_marked_windows64(int64_t eb, int64_t ee, uint32_t wm, uint32_t u, const int32_t* __restrict__ adj,
                                     const EdgeHashes& H, const uint32_t* __restrict__ thr, uint32_t ntv,
                                     const uint32_t* __restrict__ A, const uint32_t* __restrict__ Lcur, int first,
                                     int P, int lane, const uint32_t (&x)[DW][4], Acc (&acc)[DW],
                                     const uint32_t* cl = nullptr, int cs = 0, unsigned long long* mrg = nullptr) {
    uint32_t vis = 0;
    while (wm) {
        int64_t w0[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            // past the last marked window: an empty window
            w0[w] = wm ? eb + 64 * (int64_t)__builtin_ctz(wm) : ee;
            wm &= wm - 1;
        }
        int32_t vw[NW];
        bool inw[NW];
        uint64_t dm[NW];  // edges live in no sample
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            inw[w] = w0[w] + lane < ee && w0[w] < ee;
            const int32_t a = inw[w] ? adj[w0[w] + lane] : 0;
            vw[w] = adj_target(a);
            dm[w] = __ballot(adj_dead(a));
        }
        uint64_t mw[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) mw[w] = __ballot(inw[w] && (first || in_L(Lcur, cl, cs, vw[w])));
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            if (!mw[w]) continue;
            vis += (uint32_t)__builtin_popcountll(mw[w]);
            const uint64_t mm = mw[w] & ~dm[w];  // edges live in no sample merge nothing
            if (!mm) continue;
            const uint32_t mg =
                merge_window64<DW, KIND>(mm, w0[w] + lane, inw[w], vw[w], u, H, thr, ntv, A, P, lane, x, acc);
            if (mrg) *mrg += mg;
        }
    }
    return vis;
}

// G < 64 (several rows per wave): each G-lane group reads its row's out-edges
// G at a time, finds the heads in L_t with one ballot and merges the rows of
// up to UB live heads per batch of loads.  Groups may diverge; shuffles only
// read lanes of the caller's own group.
template <int G, int DW, int KIND>
DEVI uint32_t merge_edges_grp(int64_t eb, int64_t ee, uint32_t u, const int32_t* __restrict__ adj,
                              const EdgeHashes& H, const uint32_t* __restrict__ thr, uint32_t ntv,
                              const uint32_t* __restrict__ A, const uint32_t* __restrict__ Lcur, int first, int P,
                              int lane, int p, const uint32_t (&x)[DW][4], Acc (&acc)[DW],
                              unsigned long long* mrg = nullptr) {
    const int gbase = lane - p;
    constexpr uint64_t GM = (1ull << G) - 1ull;
    uint32_t vis = 0;
    for (int64_t w0 = eb; w0 < ee; w0 += G) {
        const int64_t e = w0 + p;
        const bool in = e < ee;
        const int64_t ec = in ? e : ee - 1;  // lanes past the row re-read its last edge
        const int32_t a = adj[ec];
        const int32_t v = adj_target(a);
        const bool lv = in && (first || bit_of(Lcur, v) != 0u);
        uint64_t mask = (__ballot(lv) >> gbase) & GM;
        if (!mask) continue;  // no live head: the window needs no hash or threshold
        vis += (uint32_t)__builtin_popcountll(mask);
        mask &= ~(__ballot(in && adj_dead(a)) >> gbase);  // edges live in no sample merge nothing
        if (!mask) continue;
        if (mrg) *mrg += (uint32_t)__builtin_popcountll(mask);
        const uint32_t hh = edge_hash_of(H, ec, u, (uint32_t)v);
        uint32_t tt = 0u;
        if constexpr (KIND == THR_TARGET) tt = thr[v];
        if constexpr (KIND == THR_EDGE) tt = thr[ec];
        // batches as in merge_edges64, sized per group
        auto batch = [&](auto nbc) {
            constexpr int NB = decltype(nbc)::value;
            int idx[NB];
            int last = __builtin_ctzll(mask);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (mask) last = __builtin_ctzll(mask);
                idx[b] = last;
                mask &= mask - 1;
            }
            uint32_t d[NB][DW];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int64_t vb = __shfl(v, gbase + idx[b], 64);
                const uint32_t* __restrict__ row = A + vb * P;
#pragma unroll
                for (int i = 0; i < DW; ++i) {
                    const int q = i * G + p;
                    d[b][i] = row[q < P ? q : P - 1];
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const uint32_t hb = (uint32_t)__shfl((int)hh, gbase + idx[b], 64);
                uint32_t nt = ntv;
                if constexpr (KIND != THR_CONST) nt = 0u - (uint32_t)__shfl((int)tt, gbase + idx[b], 64);
#pragma unroll
                for (int i = 0; i < DW; ++i) merge_live(acc[i], d[b][i], x[i][0], x[i][1], x[i][2], x[i][3], hb, nt);
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
    return vis;
}

template <int G, int DW, int KIND>
DEVI uint32_t merge_edges(int64_t eb, int64_t ee, uint32_t u, const int32_t* __restrict__ adj, const EdgeHashes& H,
                          const uint32_t* __restrict__ thr, uint32_t ntv, const uint32_t* __restrict__ A,
                          const uint32_t* __restrict__ Lcur, int first, int P, int lane, int p,
                          const uint32_t (&x)[DW][4], Acc (&acc)[DW], const uint32_t* cl = nullptr, int cs = 0,
                          unsigned long long* mrg = nullptr) {
    if constexpr (G == 64)
        return merge_edges64<DW, KIND>(eb, ee, u, adj, H, thr, ntv, A, Lcur, first, P, lane, x, acc, cl, cs, mrg);
    else
        return merge_edges_grp<G, DW, KIND>(eb, ee, u, adj, H, thr, ntv, A, Lcur, first, P, lane, p, x, acc, mrg);
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

// Merge of one whole row (one G-lane group): returns true if it changed.
// dense_word: the caller stores L_{t+1} words itself; otherwise the bit is set
// atomically.
template <int G, int DW, int KIND>
DEVI bool sweep_row(int64_t u, const int64_t* __restrict__ xadj, const int32_t* __restrict__ adj,
                    const EdgeHashes& H, const uint32_t* __restrict__ thr, uint32_t ntv,
                    const uint32_t (&x)[DW][4], const uint32_t* __restrict__ A, uint32_t* __restrict__ B,
                    const uint32_t* __restrict__ Lcur, uint32_t* __restrict__ Lnext, const uint32_t* __restrict__ blk,
                    const uint32_t* __restrict__ fullblk, int64_t heavy_deg, int P, int PW, int first,
                    bool dense_word, int lane, int p, unsigned long long& my_vis,
                    unsigned long long* my_mrg = nullptr) {
    const int64_t eb = xadj[u], ee = xadj[u + 1];
    const bool inL = first ? false : bit_of(Lcur, u) != 0;
    bool active = ee - eb <= heavy_deg && (ee > eb || inL) && !(fullblk && bit_of(fullblk, u));
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
    if (!active) return false;
    Acc acc[DW];
#pragma unroll
    for (int i = 0; i < DW; ++i) acc[i].e = acc[i].o = 0u;
    unsigned long long mg = 0;
    const uint32_t vis =
        merge_edges<G, DW, KIND>(eb, ee, (uint32_t)u, adj, H, thr, ntv, A, Lcur, first, P, lane, p, x, acc, nullptr, 0,
                                 &mg);
    if (p == 0) {
        my_vis += vis;
        if (my_mrg) *my_mrg += mg;
    }
    if (vis == 0 && !inL) return false;
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
    const bool changed = group_any<G>(ch);
    if (changed || inL) {
#pragma unroll
        for (int i = 0; i < DW; ++i) {
            const int q = i * G + p;
            if (q < P) B[u * P + q] = nw[i];
        }
    }
    if (changed && !dense_word && p == 0) atomicOr(&Lnext[u >> 5], 1u << (u & 31));
    return changed;
}

// Split row u (slot r) after its pieces were merged: combines the partial
// rows flagged with this sweep's stamp with M^t[u] and writes B[u] when the
// row changed or u is in L_t.  Returns true if the row changed (uniform over
// the G-lane group).
template <int G, int DW>
DEVI bool fix_row(int64_t r, int64_t u, const uint32_t* __restrict__ A, uint32_t* __restrict__ B,
                  const uint32_t* __restrict__ Lcur, const uint32_t* __restrict__ blk, const int64_t* __restrict__ hpb,
                  const int64_t* __restrict__ hpn, const uint32_t* __restrict__ part,
                  const uint32_t* __restrict__ part_any, uint32_t stamp, int P, int PW, int first, int lane, int p) {
    const bool inL = first ? false : bit_of(Lcur, u) != 0;
    uint32_t ub[DW];
#pragma unroll
    for (int k = 0; k < DW; ++k) {
        const int q = k * G + p;
        ub[k] = (blk && q < P) ? unblocked_mask(blk, u, q, PW) : 0xFFFFFFFFu;
    }
    // the row's own registers are first needed after the pieces: load them now
    uint32_t a[DW];
#pragma unroll
    for (int k = 0; k < DW; ++k) {
        const int q = k * G + p;
        a[k] = A[u * P + (q < P ? q : P - 1)];
    }
    const int64_t pb = hpb[r], np = hpn[r];
    uint32_t acc[DW];
    bool any = false;
#pragma unroll
    for (int k = 0; k < DW; ++k) acc[k] = 0u;
    if constexpr (G == 64) {
        // 64 piece flags per load; the pieces of this sweep are merged 8 at a time
        for (int64_t c0 = 0; c0 < np; c0 += 64) {
            const bool hit = c0 + lane < np && part_any[pb + c0 + lane] == stamp;
            uint64_t mask = __ballot(hit);
            any = any || mask != 0ull;
            while (mask) {
                int idx[8];
                int last = __builtin_ctzll(mask);
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    if (mask) last = __builtin_ctzll(mask);
                    idx[b] = last;
                    mask &= mask - 1;
                }
                uint32_t pv[8][DW];
#pragma unroll
                for (int b = 0; b < 8; ++b) {
#pragma unroll
                    for (int k = 0; k < DW; ++k) {
                        const int q = k * 64 + lane;
                        pv[b][k] = part[(pb + c0 + idx[b]) * P + (q < P ? q : P - 1)];
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int b = 0; b < 8; ++b)
#pragma unroll
                    for (int k = 0; k < DW; ++k) acc[k] = byte_max(acc[k], pv[b][k]);
            }
        }
    } else {
        for (int64_t c = 0; c < np; ++c) {
            if (part_any[pb + c] != stamp) continue;
            any = true;
#pragma unroll
            for (int k = 0; k < DW; ++k) {
                const int q = k * G + p;
                if (q < P) acc[k] = byte_max(acc[k], part[(pb + c) * P + q]);
            }
        }
    }
    if (!any && !inL) return false;
    bool ch = false;
    uint32_t nw[DW];
#pragma unroll
    for (int k = 0; k < DW; ++k) {
        const int q = k * G + p;
        nw[k] = 0;
        if (q < P) {
            nw[k] = byte_max(a[k], acc[k]) & ub[k];
            ch = ch || nw[k] != a[k];
        }
    }
    const bool changed = group_any<G>(ch);
    if (changed || inL) {
#pragma unroll
        for (int k = 0; k < DW; ++k) {
            const int q = k * G + p;
            if (q < P) B[u * P + q] = nw[k];
        }
    }
    return changed;
}

// G = 64: fix_row for two split rows at once (val[t]: row t exists), their
// loads interleaved so that the two rows share their round trips: row words,
// blocked masks and piece ranges, then the piece flags 64 at a time and the
// flagged partial rows in batches of up to 8 per row.  A batch slot without a
// flagged piece re-reads the row's own registers, which the max leaves as they
// are.  changed[t] as fix_row returns it.
template <int DW>
DEVI void fix_rows2(const int64_t (&r)[2], const int64_t (&u)[2], const bool (&val)[2],
                    const uint32_t* __restrict__ A, uint32_t* __restrict__ B, const uint32_t* __restrict__ Lcur,
                    const uint32_t* __restrict__ blk, const int64_t* __restrict__ hpb,
                    const int64_t* __restrict__ hpn, const uint32_t* __restrict__ part,
                    const uint32_t* __restrict__ part_any, uint32_t stamp, int P, int PW, int first, int lane,
                    bool (&changed)[2]) {
    bool inL[2], any[2];
    uint32_t ub[2][DW], a[2][DW], acc[2][DW];
    int64_t pb[2], np[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        inL[t] = val[t] && !first && bit_of(Lcur, u[t]) != 0;
        any[t] = false;
        pb[t] = val[t] ? hpb[r[t]] : 0;
        np[t] = val[t] ? hpn[r[t]] : 0;
#pragma unroll
        for (int k = 0; k < DW; ++k) {
            const int q = k * 64 + lane;
            const int qc = q < P ? q : P - 1;
            ub[t][k] = (blk && q < P) ? unblocked_mask(blk, u[t], q, PW) : 0xFFFFFFFFu;
            a[t][k] = A[u[t] * P + qc];
            acc[t][k] = 0u;
        }
    }
    const int64_t npm = np[0] > np[1] ? np[0] : np[1];
    for (int64_t c0 = 0; c0 < npm; c0 += 64) {
        uint64_t mask[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const bool hit = c0 + lane < np[t] && part_any[pb[t] + c0 + lane] == stamp;
            mask[t] = __ballot(hit);
            any[t] = any[t] || mask[t] != 0ull;
        }
        while (mask[0] | mask[1]) {
            uint32_t pv[2][8][DW];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    // a flagged partial row, or (none left) the row's own registers
                    const uint32_t* src = A + u[t] * P;
                    if (mask[t]) {
                        const int j = __builtin_ctzll(mask[t]);
                        mask[t] &= mask[t] - 1;
                        src = part + (pb[t] + c0 + j) * P;
                    }
#pragma unroll
                    for (int k = 0; k < DW; ++k) {
                        const int q = k * 64 + lane;
                        pv[t][b][k] = src[q < P ? q : P - 1];
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int b = 0; b < 8; ++b)
#pragma unroll
                    for (int k = 0; k < DW; ++k) acc[t][k] = byte_max(acc[t][k], pv[t][b][k]);
        }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        changed[t] = false;
        if (!val[t] || (!any[t] && !inL[t])) continue;
        bool ch = false;
        uint32_t nw[DW];
#pragma unroll
        for (int k = 0; k < DW; ++k) {
            const int q = k * 64 + lane;
            nw[k] = 0;
            if (q < P) {
                nw[k] = byte_max(a[t][k], acc[t][k]) & ub[t][k];
                ch = ch || nw[k] != a[t][k];
            }
        }
        changed[t] = __ballot(ch) != 0ull;
        if (changed[t] || inL[t]) {
#pragma unroll
            for (int k = 0; k < DW; ++k) {
                const int q = k * 64 + lane;
                if (q < P) B[u[t] * P + q] = nw[k];
            }
        }
    }
}

// Greedy score (Alg. 1): score(u) = sum_j max(M_S'[j], M_u[j]) for u not in
// S, as the key score << 32 | (2^32 - 1 - u) so that the maximum key is the
// highest score with the lowest id.  The wave scores rows base + (lane / G)
// for base = b0, b0 + bstep, ... below b1 (uniform bounds) and returns the
// wave's best key (0 if none) in every lane.
template <int G, int DW>
DEVI unsigned long long best_score_rows(int64_t b0, int64_t b1, int64_t bstep, const uint32_t* __restrict__ M,
                                        const uint32_t* __restrict__ MS, const uint8_t* __restrict__ inS, int P) {
    const int lane = threadIdx.x & 63, grp = lane / G, p = lane % G;
    uint32_t ms[DW];
#pragma unroll
    for (int i = 0; i < DW; ++i) {
        const int q = i * G + p;
        ms[i] = q < P ? MS[q] : 0u;
    }
    unsigned long long best = 0;
    for (int64_t base = b0; base < b1; base += bstep) {
        const int64_t u = base + grp;
        const bool ok = u < b1 && inS[u] == 0;
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
    return best;
}

// Greedy step of Alg. 1 after the argmax (one wave, all lanes take part): s
// is the vertex of the maximum key.  Records s (seed, score), computes e =
// Estimate(Merge(M_S', M_s)) into merged, rec->e and *e_out, blocks every pair
// (s, j) not blocked yet and makes those pairs the level-0 frontier F0, with
// the queue entries Q0 covering s's out-edges.  Returns false (seed -1) when
// the key names no candidate.  *nch_out: queue entries; *newcnt_out: pairs
// blocked by this call (both uniform).
DEVI bool select_seed(unsigned long long key, int64_t n, int J, int P, int PW, const int64_t* __restrict__ xadj,
                      const uint32_t* __restrict__ M, const uint32_t* __restrict__ MS, uint32_t* merged, uint32_t* blk,
                      uint32_t* F0, int2* Q0, uint8_t* inS, int32_t* stamp, int32_t level_id, int bfs_chunk,
                      const double* __restrict__ T, StepRec* rec, int32_t* seeds, int k, uint32_t* nch_out,
                      uint32_t* newcnt_out, double* e_out) {
    const int lane = threadIdx.x & 63;
    const int64_t s = (int64_t)(0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull));
    *nch_out = 0;
    *newcnt_out = 0;
    *e_out = 0.0;
    if (key == 0ull || s >= n) {  // no candidate: report and touch nothing else
        if (lane == 0) {
            rec->seed = -1;
            seeds[k] = -1;
        }
        return false;
    }
    uint32_t sum = 0;
    for (int q = lane; q < P; q += 64) {
        const uint32_t mg = byte_max(MS[q], M[s * P + q]);
        merged[q] = mg;
        sum = __builtin_amdgcn_sad_u8(mg, 0u, sum);
    }
    sum = wave_sum(sum);
    const int64_t deg = xadj[s + 1] - xadj[s];
    const int W = 4 * PW;
    uint32_t newcnt = 0;
    for (int w = lane; w < W; w += 64) {
        const uint32_t old = blk[s * W + w];
        const uint32_t nb = ~old & plane_valid_mask(w, P, PW);
        blk[s * W + w] = old | nb;
        newcnt += __builtin_popcount(nb);
        if (deg > 0) F0[s * W + w] = nb;
    }
    newcnt = wave_sum(newcnt);
    const int64_t nch = (deg > 0 && newcnt > 0) ? (deg + bfs_chunk - 1) / bfs_chunk : 0;
    for (int64_t c = lane; c < nch; c += 64) Q0[c] = make_int2((int)s, (int)c);
    const double e = estimate_from_sum(sum, J, T);
    if (lane == 0) {
        inS[s] = 1;
        seeds[k] = (int32_t)s;
        rec->seed = (int32_t)s;
        rec->score = (int64_t)(key >> 32);
        rec->e = e;
        if (nch) stamp[s] = level_id;
    }
    *nch_out = (uint32_t)nch;
    *newcnt_out = newcnt;
    *e_out = e;
    return true;
}

// Error-adaptive decision of Alg. 1 in FP64 for step k (1-based) of K, from R
// blocked pairs now, R0 at the last rebuild and the step's estimate e: sigma =
// R / J, delta = (R - R0) / J, err_l = |(e - delta) / delta| (+inf when delta
// = 0), err_g = |(e - delta) / sigma|, fresh iff err_l < eps_l or err_g <
// eps_g; the sketches are rebuilt iff k < K and not fresh.  Fills rec (sweeps
// and visits 0) and returns the rebuild flag; *fresh_out receives fresh.
DEVI int decide_step(unsigned long long R, unsigned long long R0, int J, int k, int K, double eps_g, double eps_l,
                     double e, StepRec* rec, int* fresh_out) {
    const double sigma = (double)R / (double)J;
    const double delta = (double)(R - R0) / (double)J;
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
    *fresh_out = fresh;
    return rebuild;
}

// One BFS level of the Monte-Carlo reach over all samples at once.  A queue
// entry is (vertex v, chunk c) covering at most bfs_chunk out-edges of v.  For
// each edge (v, w): the samples where the edge is live and v is in the
// frontier are OR-ed into w's blocked bits; bits that were not set before
// form w's frontier of the next level, and w is queued once per level (the
// level id in stamp[w] guards the append).
//
// A G-lane group serves one entry: it reads G edges per window, tests every
// edge against its 4*DW registers per lane, and collects the edges with a
// candidate bit in a batch.  Lane p of the group owns word p % (4 PW) of edge
// slot p / (4 PW) of the batch, so one atomic instruction updates the blocked
// words of G / (4 PW) edges at once (8 edges at R = 256).  The wave serves
// entries base + (lane / G) for base = b0, b0 + bstep, ... below b1 (uniform
// bounds).  Returns the number of newly blocked pairs found by this lane.
//
// RESV (G = 64): a wave takes next-queue slots from the shared counter qn
// BFS_RESV at a time (or as many as one flush needs) instead of once per flush,
// so that the counter is not the level's serialisation point; the slots a wave
// reserved and did not fill become holes (vertex -1), which the next level and
// the cleanup skip.  The queue then needs BFS_RESV slots per wave of the launch
// beyond its entries.
template <int G, int DW, int KIND, bool RESV = false, int NE = 1>
DEVI unsigned long long bfs_expand_entries(int64_t b0, int64_t b1, int64_t bstep, const int64_t* __restrict__ xadj,
                                           const int32_t* __restrict__ adj, const EdgeHashes& H,
                                           const uint32_t* __restrict__ thr, uint32_t ntv, const uint32_t (&x)[DW][4],
                                           const uint32_t* __restrict__ Fc, uint32_t* Fn, const int2* __restrict__ Qc,
                                           int2* Qn, uint32_t* qn, uint32_t* blk, int32_t* stamp,
                                           int32_t level_id_next, int bfs_chunk, int P, int PW) {
    const int lane = threadIdx.x & 63, grp = lane / G, p = lane % G;
    const int W = 4 * PW;      // words of a vertex bitset = words of an edge's candidate set
    const int EPB = G / W;     // edges per batch (>= 1)
    const int sb = p / W, sw = p % W;
    const bool slot_ok = sb < EPB;
    const int sk = sw / PW, sww = sw % PW;  // plane and word-in-plane of this lane's word
    const uint64_t gmask = G == 64 ? ~0ull : ((1ull << G) - 1ull);
    const uint64_t wmask = W >= 64 ? ~0ull : ((1ull << W) - 1ull);
    unsigned long long my_new = 0;
    uint32_t rpos = 0, rend = 0;  // RESV: the wave's reserved slots not yet filled
    static_assert(NE == 1 || G == 64, "several entries per step need one entry per wave");
    // NE entries per step (base, base + bstep, ...): their records, edge ranges,
    // frontier bits and first windows of edges are loaded together, so that the
    // entries' round trips overlap; their candidate edges share the flush batches
    for (int64_t base = b0; base < b1; base += NE * bstep) {
        int2 qe[NE];
#pragma unroll
        for (int t = 0; t < NE; ++t) {
            const int64_t ent = base + t * bstep + grp;
            qe[t] = ent < b1 ? Qc[ent] : make_int2(-1, 0);
        }
        int64_t e0[NE], e1[NE];
        uint32_t src[NE];     // the entry's vertex: the source of its edges
        uint32_t fb[NE][DW];  // frontier bits of this lane's registers, bit (k) of fb[t][i] for register 4q+k
#pragma unroll
        for (int t = 0; t < NE; ++t) {
            e0[t] = e1[t] = 0;
            src[t] = 0;
#pragma unroll
            for (int i = 0; i < DW; ++i) fb[t][i] = 0u;
            if (qe[t].x >= 0) {  // not past b1, nor a hole
                const int64_t v = qe[t].x;
                src[t] = (uint32_t)v;
                const int64_t vb = xadj[v], ve = xadj[v + 1];
                e0[t] = vb + (int64_t)qe[t].y * bfs_chunk;
                e1[t] = e0[t] + bfs_chunk < ve ? e0[t] + bfs_chunk : ve;
#pragma unroll
                for (int i = 0; i < DW; ++i) {
                    const int q = i * G + p;
                    uint32_t f = 0;
                    if (q < P) {
#pragma unroll
                        for (int k = 0; k < 4; ++k) f |= ((Fc[v * W + k * PW + (q >> 5)] >> (q & 31)) & 1u) << k;
                    }
                    fb[t][i] = f;
                }
            }
        }
        uint32_t myval = 0;
        int64_t myw = 0;
        bool myslot = false;  // an edge was put in this lane's slot of the batch
        int nb = 0;
        auto flush = [&]() {
            uint32_t nbits = 0;
            // out-degree of the slot's target, loaded only for edges with a
            // candidate bit (it decides whether the target is queued)
            int64_t mywdeg = 0;
            if (myslot) mywdeg = xadj[myw + 1] - xadj[myw];
            // blocked bits are only ever set: a plain read that already shows every
            // candidate bit means the atomic could add nothing (a stale read only
            // costs an atomic)
            if (myval && (myval & ~blk[myw * W + sw]) != 0u) {
                const uint32_t old = atomicOr(&blk[myw * W + sw], myval);
                nbits = myval & ~old;
                if (nbits) {
                    if (mywdeg > 0) atomicOr(&Fn[myw * W + sw], nbits);
                    my_new += (unsigned long long)__builtin_popcount(nbits);
                }
            }
            const uint64_t bal = __ballot(nbits != 0u);
            const bool want = sw == 0 && slot_ok && mywdeg > 0 && ((bal >> (grp * G + sb * W)) & wmask) != 0ull;
            if constexpr (G == 64) {
                // the whole wave flushes together: the targets it queues take one
                // range of the next queue, with a single counter atomic
                uint32_t nch = 0;
                if (want && atomicMax(&stamp[myw], level_id_next) < level_id_next)
                    nch = (uint32_t)((mywdeg + bfs_chunk - 1) / bfs_chunk);
                uint32_t tot;
                const uint32_t off = wave_excl_scan(nch, &tot);
                if (tot && RESV) {
                    // the first `have` of the flush's entries fill the reserved slots, the
                    // rest a new block taken from the counter
                    const uint32_t have = rend - rpos;
                    uint32_t nb = rend, nend = rend;
                    if (tot > have) {
                        const uint32_t take = tot - have > (uint32_t)BFS_RESV ? tot - have : (uint32_t)BFS_RESV;
                        uint32_t blk0 = 0;
                        if (lane == 0) blk0 = atomicAdd(qn, take);
                        nb = __shfl(blk0, 0, 64);
                        nend = nb + take;
                    }
                    for (uint32_t c = 0; c < nch; ++c) {
                        const uint32_t i = off + c;
                        Qn[i < have ? rpos + i : nb + (i - have)] = make_int2((int)myw, (int)c);
                    }
                    if (tot > have) {
                        rpos = nb + (tot - have);
                        rend = nend;
                    } else {
                        rpos += tot;
                    }
                } else if (tot) {
                    uint32_t pos = 0;
                    if (lane == 0) pos = atomicAdd(qn, tot);
                    pos = __shfl(pos, 0, 64) + off;
                    for (uint32_t c = 0; c < nch; ++c) Qn[pos + c] = make_int2((int)myw, (int)c);
                }
            } else if (want) {
                const int32_t old = atomicMax(&stamp[myw], level_id_next);
                if (old < level_id_next) {
                    const int64_t nch = (mywdeg + bfs_chunk - 1) / bfs_chunk;
                    const uint32_t pos = atomicAdd(qn, (uint32_t)nch);
                    for (int64_t c = 0; c < nch; ++c) Qn[pos + c] = make_int2((int)myw, (int)c);
                }
            }
            myval = 0;
            myslot = false;
        };
        // the serial pass over one window's edges (lane p holds edge w0 + p with
        // head wv, hash hh and threshold tt; fbe: the entry's frontier bits)
        auto scan = [&](uint64_t todo, int nwin, uint32_t hh, uint32_t tt, int32_t wv, const uint32_t (&fbe)[DW]) {
            for (int jj = 0; G == 64 ? todo != 0ull : jj < nwin; ++jj) {
                int j = jj;
                if constexpr (G == 64) {
                    j = __builtin_ctzll(todo);
                    todo &= todo - 1;
                }
                uint32_t hb, nt = ntv;
                int32_t wj;
                if constexpr (G == 64) {
                    hb = (uint32_t)__builtin_amdgcn_readlane((int)hh, j);
                    if constexpr (KIND != THR_CONST) nt = 0u - (uint32_t)__builtin_amdgcn_readlane((int)tt, j);
                    wj = __builtin_amdgcn_readlane(wv, j);
                } else {
                    hb = __shfl(hh, grp * G + j, 64);
                    if constexpr (KIND != THR_CONST) nt = 0u - __shfl(tt, grp * G + j, 64);
                    wj = __shfl(wv, grp * G + j, 64);
                }
                uint32_t cw = 0;
                bool anyc = false;
#pragma unroll
                for (int i = 0; i < DW; ++i) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const bool c = (int32_t)((x[i][k] ^ hb) + nt) < 0 && ((fbe[i] >> k) & 1u);
                        const uint64_t bal = __ballot(c);
                        if constexpr (G == 64) {
                            const uint32_t lo = (uint32_t)bal, hi = (uint32_t)(bal >> 32);
                            if (sk == k && sww == 2 * i) cw = lo;
                            if (sk == k && sww == 2 * i + 1) cw = hi;
                            anyc = anyc || bal != 0ull;
                        } else {
                            const uint32_t gb = (uint32_t)((bal >> (grp * G)) & gmask);
                            if (sk == k) cw = gb;
                            anyc = anyc || gb != 0u;
                        }
                    }
                }
                if (!anyc) continue;
                if (sb == nb) {
                    myval = cw;
                    myw = wj;
                    myslot = slot_ok;
                }
                if (++nb == EPB) {
                    flush();
                    nb = 0;
                }
            }
        };
        // window [w0, w0 + G) of entry t: edge ids, heads, hashes and thresholds
        auto load_window = [&](int t, int64_t w0, bool& in, int32_t& wa, int32_t& wv, uint32_t& hh, uint32_t& tt) {
            const int64_t e = w0 + p;
            in = e < e1[t];
            wa = in ? adj[e] : 0;
            wv = adj_target(wa);
            hh = in ? edge_hash_of(H, e, src[t], (uint32_t)wv) : 0u;
            tt = 0u;
            if constexpr (KIND == THR_TARGET) tt = in ? thr[wv] : 0u;
            if constexpr (KIND == THR_EDGE) tt = in ? thr[e] : 0u;
        };
        // G = 64: only the window's edges live in some sample (an edge live in
        // none reaches nothing); groups scan their whole window
        auto todo_of = [&](bool in, int32_t wa) -> uint64_t {
            if constexpr (G == 64) return __ballot(in && !adj_dead(wa));
            return 0ull;
        };
        {
            bool in[NE];
            int32_t wa[NE], wv[NE];
            uint32_t hh[NE], tt[NE];
#pragma unroll
            for (int t = 0; t < NE; ++t) load_window(t, e0[t], in[t], wa[t], wv[t], hh[t], tt[t]);
#pragma unroll
            for (int t = 0; t < NE; ++t)
                scan(todo_of(in[t], wa[t]), (int)(e1[t] - e0[t] < G ? e1[t] - e0[t] : G), hh[t], tt[t], wv[t],
                     fb[t]);
        }
#pragma unroll
        for (int t = 0; t < NE; ++t) {
            for (int64_t w0 = e0[t] + G; w0 < e1[t]; w0 += G) {
                bool in;
                int32_t wa, wv;
                uint32_t hh, tt;
                load_window(t, w0, in, wa, wv, hh, tt);
                scan(todo_of(in, wa), (int)(e1[t] - w0 < G ? e1[t] - w0 : G), hh, tt, wv, fb[t]);
            }
        }
        if (nb > 0) flush();
    }
    if constexpr (RESV && G == 64)
        for (uint32_t h = rpos + lane; h < rend; h += 64) Qn[h] = make_int2(-1, 0);  // holes
    return my_new;
}

}  // namespace hfr
