/*
 * CPU oracle for the sketch-based influence-maximisation method of
 * Gokturk & Kaya, "Fast and Error-Adaptive Influence Maximization based on
 * Count-Distinct Sketches" (arXiv 2105.04023).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, single-threaded
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header, table or constant generator with the GPU library.
 *
 * Floating point is IEEE double, built with -ffp-contract=off.
 *
 * Where the paper leaves a point open, this file takes one reading, stated
 * next to the code that applies it:
 *   R1  Sweeps are synchronous (Jacobi): sweep t reads the registers of sweep
 *       t-1 only.
 *   R2  Only out-neighbours v that changed in the previous sweep (v in L) are
 *       merged; with L_0 = V this gives the same registers as merging all of
 *       them.
 *   R3  A (vertex, simulation) pair inside the seed set's reach is blocked: its
 *       register starts at 0 and never merges, so a rebuilt register holds the
 *       largest rank over the residual reach only.
 *   R4  hash(v) and hash(j) of the register initialisation are full 32-bit
 *       Murmur3 values with their own seeds; X_j is Murmur3 of j, 31 bits.
 *   R5  The live test compares the XOR value with an integer threshold equal
 *       to the number of 31-bit integers x with x < w * h_max.
 *   R6  The argmax excludes vertices already in S, compares integer register
 *       sums, and breaks ties to the lowest vertex id.
 *   R7  The Monte-Carlo reach uses the same hash samples as the sketches.
 *   R8  e is the estimate of Merge(M_S', M_s) taken before M_S' is merged.
 *   R9  No rebuild after the K-th seed (it cannot change S).
 *   R10 delta = 0 gives err_l = +inf.
 *   R11 The edge-visit count of a sweep is the number of edges (u, v) with v
 *       in L and u not blocked in every simulation (such a row cannot change).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* MurmurHash3, x86 32-bit variant (public-domain algorithm by A. Appleby),  */
/* written from its published description: 4-byte little-endian blocks are   */
/* scrambled with c1 = 0xcc9e2d51, rotl 15, c2 = 0x1b873593, mixed into the  */
/* state with rotl 13 and h*5 + 0xe6546b64; the tail bytes are scrambled the */
/* same way; the length is xored in and the 32-bit finaliser is applied.     */
/* ------------------------------------------------------------------------ */
static uint32_t rotl32(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }

uint32_t orc_murmur3_32(const uint8_t* key, uint64_t len, uint32_t seed) {
    const uint32_t c1 = 0xcc9e2d51u, c2 = 0x1b873593u;
    uint32_t h = seed;
    uint64_t nblocks = len / 4;
    for (uint64_t i = 0; i < nblocks; ++i) {
        uint32_t k = (uint32_t)key[4 * i] | ((uint32_t)key[4 * i + 1] << 8) | ((uint32_t)key[4 * i + 2] << 16) |
                     ((uint32_t)key[4 * i + 3] << 24);
        k *= c1;
        k = rotl32(k, 15);
        k *= c2;
        h ^= k;
        h = rotl32(h, 13);
        h = h * 5u + 0xe6546b64u;
    }
    const uint8_t* tail = key + 4 * nblocks;
    uint32_t k1 = 0;
    switch (len & 3) {
        case 3: k1 ^= (uint32_t)tail[2] << 16; /* fall through */
        case 2: k1 ^= (uint32_t)tail[1] << 8;  /* fall through */
        case 1:
            k1 ^= (uint32_t)tail[0];
            k1 *= c1;
            k1 = rotl32(k1, 15);
            k1 *= c2;
            h ^= k1;
    }
    h ^= (uint32_t)len;
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

static void le32(uint8_t* out, uint32_t x) {
    out[0] = (uint8_t)x;
    out[1] = (uint8_t)(x >> 8);
    out[2] = (uint8_t)(x >> 16);
    out[3] = (uint8_t)(x >> 24);
}

/* Eq. (hash): h(u,v) = Murmur3(u || v) mod 2^31, key = LE32(u) then LE32(v). */
uint32_t orc_edge_hash(int32_t u, int32_t v, uint32_t seed) {
    uint8_t key[8];
    le32(key, (uint32_t)u);
    le32(key + 4, (uint32_t)v);
    return orc_murmur3_32(key, 8, seed) % 2147483648u;
}

/* Sec. 3.1: the per-simulation random word X_j in [0, h_max] (reading R4). */
uint32_t orc_sim_word(int32_t j, uint32_t seed) {
    uint8_t key[4];
    le32(key, (uint32_t)j);
    return orc_murmur3_32(key, 4, seed + 2u) % 2147483648u;
}

/* Number of leading zero bits of a 32-bit word, counted one bit at a time; clz(0) = 32. */
static int clz32_plain(uint32_t y) {
    int n = 0;
    for (int b = 31; b >= 0; --b) {
        if (y & (1u << b)) break;
        ++n;
    }
    return n;
}

/* Alg. 1 register initialisation and Eq. (sketch-add): rank = clz(hash(v) xor hash(j)) (reading R4). */
uint8_t orc_rank(int32_t v, int32_t j, uint32_t seed) {
    uint8_t kv[4], kj[4];
    le32(kv, (uint32_t)v);
    le32(kj, (uint32_t)j);
    uint32_t hv = orc_murmur3_32(kv, 4, seed + 1u);
    uint32_t hj = orc_murmur3_32(kj, 4, seed + 3u);
    return (uint8_t)clz32_plain(hv ^ hj);
}

/*
 * Eq. (hash_prob) and the live-edge rule (reading R5): the edge is in sample j
 * iff (X_j xor h)/h_max < w, i.e. (X_j xor h) < w * (2^31 - 1) in exact
 * arithmetic.  The threshold is the count of such integers:
 * ceil(w * (2^31 - 1)), evaluated exactly from the binary32 value of w
 * (w = mant * 2^e, mant < 2^24, so mant * (2^31 - 1) < 2^55).
 * Returns 0xFFFFFFFF for w outside [0, 1] or NaN.
 */
uint32_t orc_threshold(float w) {
    if (!(w >= 0.0f && w <= 1.0f)) return 0xFFFFFFFFu;
    uint32_t bits;
    memcpy(&bits, &w, 4);
    uint32_t E = (bits >> 23) & 0xFF, F = bits & 0x7FFFFF;
    uint64_t mant;
    int e;
    if (E == 0) {
        mant = F;
        e = -149;
    } else {
        mant = (uint64_t)F | (1ull << 23);
        e = (int)E - 150;
    }
    if (mant == 0) return 0;
    uint64_t P = mant * 2147483647ull; /* w * h_max = P * 2^e, e < 0 here */
    int s = -e;
    if (s >= 64) return 1; /* 0 < value < 1 -> ceil is 1 */
    uint64_t q = P >> s;
    uint64_t rem = P & ((1ull << s) - 1);
    return (uint32_t)(q + (rem != 0));
}

int orc_live(uint32_t h, uint32_t x, uint32_t thr) { return (x ^ h) < thr; }

/*
 * Per-edge thresholds for a graph: kind 0 = constant w (p), kind 1 =
 * weighted cascade w_uv = 1/d_v with d_v the in-degree of v in the CSR as
 * given (computed as the binary32 quotient 1.0f / (float)d_v), kind 2 =
 * per-edge binary32 weights.  Returns 0, or -1 if a weight is outside [0,1].
 */
int orc_edge_thresholds(int64_t n, const int64_t* xadj, const int32_t* adj, int kind, float p, const float* per_edge,
                        uint32_t* thr_out) {
    int64_t m = xadj[n];
    if (kind == 0) {
        uint32_t t = orc_threshold(p);
        if (t == 0xFFFFFFFFu) return -1;
        for (int64_t e = 0; e < m; ++e) thr_out[e] = t;
    } else if (kind == 1) {
        int64_t* indeg = calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
        if (!indeg) return -2;
        for (int64_t e = 0; e < m; ++e) indeg[adj[e]]++;
        for (int64_t e = 0; e < m; ++e) thr_out[e] = orc_threshold(1.0f / (float)indeg[adj[e]]);
        free(indeg);
    } else {
        for (int64_t e = 0; e < m; ++e) {
            uint32_t t = orc_threshold(per_edge[e]);
            if (t == 0xFFFFFFFFu) return -1;
            thr_out[e] = t;
        }
    }
    return 0;
}

/*
 * Alg. 2 (Simulate) with the readings R1-R3.
 *
 *   M[v][j] = blocked(v,j) ? 0 : rank(v,j);  L = V
 *   while |L| > eps_c * n:
 *       M' = M
 *       for u, for v in A(u) with v in L, for j:
 *           if not blocked(u,j) and edge (u,v) live in sample j:
 *               M'[u][j] = max(M'[u][j], M[v][j])
 *       L = {u : M'[u] != M[u]};  M = M'
 *
 * M is n*J bytes, vertex-major (the J registers of a vertex are adjacent,
 * as in the implementation section).  blk is n*J bytes (nonzero = blocked)
 * or NULL.  trace_live[t] receives |L_t| for t = 0..sweeps (when t <
 * trace_cap) and trace_edges[t] the number of edges (u,v) with v in L_t
 * that sweep t visited.  max_sweeps < 0 means no bound.  Returns the number of
 * sweeps, or -1 on allocation failure.
 */
int64_t orc_simulate(int64_t n, const int64_t* xadj, const int32_t* adj, const uint32_t* thr_edge, int32_t J,
                     uint32_t seed, const uint8_t* blk, double eps_c, int64_t max_sweeps, uint8_t* M,
                     int64_t* trace_live, int64_t* trace_edges, int64_t trace_cap) {
    uint32_t* X = malloc(sizeof(uint32_t) * (size_t)J);
    uint8_t* Mn = malloc((size_t)(n * J > 0 ? n * J : 1));
    uint8_t* L = malloc((size_t)(n > 0 ? n : 1));
    uint8_t* Ln = malloc((size_t)(n > 0 ? n : 1));
    if (!X || !Mn || !L || !Ln) {
        free(X);
        free(Mn);
        free(L);
        free(Ln);
        return -1;
    }
    for (int32_t j = 0; j < J; ++j) X[j] = orc_sim_word(j, seed);
    for (int64_t v = 0; v < n; ++v)
        for (int32_t j = 0; j < J; ++j)
            M[v * J + j] = (blk && blk[v * J + j]) ? 0 : orc_rank((int32_t)v, j, seed);
    int64_t live = n;
    for (int64_t v = 0; v < n; ++v) L[v] = 1;
    int64_t t = 0;
    if (trace_cap > 0) trace_live[0] = live;
    while ((double)live > eps_c * (double)n && (max_sweeps < 0 || t < max_sweeps)) {
        memcpy(Mn, M, (size_t)(n * J));
        int64_t edges = 0;
        for (int64_t u = 0; u < n; ++u) {
            /* R11: a row blocked in every simulation can never change; its
             * edges are not visited (and not counted). */
            if (blk) {
                int32_t j = 0;
                while (j < J && blk[u * J + j]) ++j;
                if (j == J) continue;
            }
            for (int64_t e = xadj[u]; e < xadj[u + 1]; ++e) {
                int32_t v = adj[e];
                if (!L[v]) continue;
                ++edges;
                uint32_t h = orc_edge_hash((int32_t)u, v, seed);
                for (int32_t j = 0; j < J; ++j) {
                    if (blk && blk[u * J + j]) continue;
                    if (!orc_live(h, X[j], thr_edge[e])) continue;
                    if (M[(int64_t)v * J + j] > Mn[u * J + j]) Mn[u * J + j] = M[(int64_t)v * J + j];
                }
            }
        }
        live = 0;
        for (int64_t u = 0; u < n; ++u) {
            Ln[u] = memcmp(Mn + u * J, M + u * J, (size_t)J) != 0;
            live += Ln[u];
        }
        memcpy(M, Mn, (size_t)(n * J));
        memcpy(L, Ln, (size_t)n);
        if (t < trace_cap) trace_edges[t] = edges;
        ++t;
        if (t < trace_cap) trace_live[t] = live;
    }
    free(X);
    free(Mn);
    free(L);
    free(Ln);
    return t;
}

/*
 * Eq. (sketch-estimate): e = 2^(mean_j M[j]) / phi, phi = 0.77351.  The mean
 * is s/J with s the integer register sum; it is split into s = q*J + r so that
 * e = 2^q * 2^(r/J) / phi, with 2^(r/J) = exp2((double)r / (double)J).
 */
double orc_estimate(const uint8_t* row, int32_t J) {
    int64_t s = 0;
    for (int32_t j = 0; j < J; ++j) s += row[j];
    int64_t q = s / J, r = s % J;
    return ldexp(exp2((double)r / (double)J), (int)q) / 0.77351;
}

/*
 * Alg. 1, Monte-Carlo reach (reading R7): for every simulation j, a
 * breadth-first search from seed s over the edges live in sample j, marking
 * every reached (v, j) as blocked.  Pairs that are already blocked are not
 * entered again (the reach of S is closed under live edges).  Returns the
 * number of newly blocked pairs.
 */
int64_t orc_reach_add(int64_t n, const int64_t* xadj, const int32_t* adj, const uint32_t* thr_edge, int32_t J,
                      uint32_t seed, uint8_t* blk, int32_t s) {
    int32_t* queue = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!queue) return -1;
    int64_t added = 0;
    for (int32_t j = 0; j < J; ++j) {
        if (blk[(int64_t)s * J + j]) continue;
        uint32_t x = orc_sim_word(j, seed);
        int64_t head = 0, tail = 0;
        blk[(int64_t)s * J + j] = 1;
        queue[tail++] = s;
        ++added;
        while (head < tail) {
            int32_t u = queue[head++];
            for (int64_t e = xadj[u]; e < xadj[u + 1]; ++e) {
                int32_t v = adj[e];
                if (blk[(int64_t)v * J + j]) continue;
                if (!orc_live(orc_edge_hash(u, v, seed), x, thr_edge[e])) continue;
                blk[(int64_t)v * J + j] = 1;
                queue[tail++] = v;
                ++added;
            }
        }
    }
    free(queue);
    return added;
}

/* Per-step record of the greedy loop. */
typedef struct {
    int32_t seed;      /* s chosen at this step */
    int32_t rebuilt;   /* 1 if the sketches were rebuilt after this step */
    int32_t fresh;     /* 1 if err_l < eps_l or err_g < eps_g */
    int32_t sweeps;    /* sweeps of the rebuild Simulate (0 if none) */
    int64_t score;     /* integer register sum of Merge(M_S', M_s) */
    int64_t reach;     /* total blocked (v, j) pairs after this step */
    double e, sigma, delta, err_l, err_g;
    int64_t visits;    /* edge visits of the rebuild Simulate (edges with a live head, summed over sweeps) */
} orc_step;

/*
 * Observer of a greedy run, for recording expected values of long runs.  It is
 * called once after the build's Simulate (k = 0: M holds the build's registers,
 * sweeps and the two traces describe that Simulate, blk and st are NULL) and once
 * after every step k >= 1, when that step's record is complete and before its
 * rebuild (if any) starts: M then holds the registers the step used and blk the
 * blocked pairs after it, which is exactly the final state of a run with K = k
 * (no rebuild follows the last step, reading R9).  A nonzero return ends the run.
 */
typedef int (*orc_observer)(int32_t k, const uint8_t* M, const uint8_t* blk, const orc_step* st, int64_t sweeps,
                            const int64_t* trace_live, const int64_t* trace_edges, void* user);

/*
 * Alg. 1 (HyperFuseR) with the readings R1-R10:
 *
 *   M = Simulate(no blocks); M_S' = 0; varsigma = 0; S = {}
 *   for k = 1..K:
 *       s = argmax_{v not in S} sum_j max(M_S'[j], M[v][j])
 *       e = Estimate(Merge(M_S', M_s))
 *       block the reach of s in every sample; sigma = blocked pairs / J
 *       delta = sigma - varsigma; err_l = |(e-delta)/delta|; err_g = |(e-delta)/sigma|
 *       if k < K:
 *           if err_l < eps_l or err_g < eps_g: M_S' = Merge(M_S', M_s)
 *           else: M = Simulate(blocked = reach of S); M_S' = 0; varsigma = sigma
 *
 * sigma and delta are formed from integer pair counts: sigma = R / J,
 * delta = (R - R_at_last_rebuild) / J.  M (n*J bytes) holds the final
 * registers on return; blk (n*J bytes) the final blocked pairs (may be NULL
 * for an internal buffer).  build_sweeps/build_visits describe the initial
 * Simulate.  obs (may be NULL) is called as described above.  Returns 0, 1 if
 * the observer ended the run early, or -1 on allocation failure.
 */
int orc_greedy_observed(int64_t n, const int64_t* xadj, const int32_t* adj, const uint32_t* thr_edge, int32_t J,
                        uint32_t seed, int32_t K, double eps_g, double eps_l, double eps_c, uint8_t* M,
                        uint8_t* blk_out, orc_step* steps, int64_t* build_sweeps, int64_t* build_visits,
                        orc_observer obs, void* user) {
    uint8_t* blk = blk_out ? blk_out : calloc((size_t)(n * J > 0 ? n * J : 1), 1);
    uint8_t* inS = calloc((size_t)(n > 0 ? n : 1), 1);
    uint8_t* MS = calloc((size_t)J, 1);
    uint8_t* merged = malloc((size_t)J);
    int64_t cap = n + 2;
    int64_t* tl = malloc(sizeof(int64_t) * (size_t)cap);
    int64_t* te = malloc(sizeof(int64_t) * (size_t)cap);
    if (!blk || !inS || !MS || !merged || !tl || !te) return -1;
    if (blk_out) memset(blk, 0, (size_t)(n * J));
    int rc = 0;

    int64_t sw = orc_simulate(n, xadj, adj, thr_edge, J, seed, NULL, eps_c, -1, M, tl, te, cap);
    int64_t vis = 0;
    for (int64_t t = 0; t < sw && t < cap; ++t) vis += te[t];
    *build_sweeps = sw;
    *build_visits = vis;
    if (obs && obs(0, M, NULL, NULL, sw, tl, te, user)) rc = 1;

    int64_t R = 0, R_rebuild = 0;
    for (int32_t k = 1; k <= K && rc == 0; ++k) {
        int64_t best = -1;
        int32_t s = -1;
        for (int64_t v = 0; v < n; ++v) {
            if (inS[v]) continue;
            int64_t sc = 0;
            for (int32_t j = 0; j < J; ++j) sc += MS[j] > M[v * J + j] ? MS[j] : M[v * J + j];
            if (sc > best) {
                best = sc;
                s = (int32_t)v;
            }
        }
        inS[s] = 1;
        for (int32_t j = 0; j < J; ++j) merged[j] = MS[j] > M[(int64_t)s * J + j] ? MS[j] : M[(int64_t)s * J + j];
        double e = orc_estimate(merged, J);
        R += orc_reach_add(n, xadj, adj, thr_edge, J, seed, blk, s);
        double sigma = (double)R / (double)J;
        double delta = (double)(R - R_rebuild) / (double)J;
        double err_l = delta == 0.0 ? INFINITY : fabs((e - delta) / delta);
        double err_g = fabs((e - delta) / sigma);
        int fresh = (err_l < eps_l) || (err_g < eps_g);
        orc_step* st = &steps[k - 1];
        st->seed = s;
        st->score = best;
        st->reach = R;
        st->e = e;
        st->sigma = sigma;
        st->delta = delta;
        st->err_l = err_l;
        st->err_g = err_g;
        st->fresh = fresh;
        st->rebuilt = 0;
        st->sweeps = 0;
        st->visits = 0;
        if (obs && obs(k, M, blk, st, 0, NULL, NULL, user)) rc = 1;
        if (k < K && rc == 0) {
            if (fresh) {
                memcpy(MS, merged, (size_t)J);
            } else {
                int64_t rs = orc_simulate(n, xadj, adj, thr_edge, J, seed, blk, eps_c, -1, M, tl, te, cap);
                int64_t rv = 0;
                for (int64_t t = 0; t < rs && t < cap; ++t) rv += te[t];
                memset(MS, 0, (size_t)J);
                R_rebuild = R;
                st->rebuilt = 1;
                st->sweeps = (int32_t)rs;
                st->visits = rv;
            }
        }
    }
    if (!blk_out) free(blk);
    free(inS);
    free(MS);
    free(merged);
    free(tl);
    free(te);
    return rc;
}

/* Alg. 1 without an observer. */
int orc_greedy(int64_t n, const int64_t* xadj, const int32_t* adj, const uint32_t* thr_edge, int32_t J, uint32_t seed,
               int32_t K, double eps_g, double eps_l, double eps_c, uint8_t* M, uint8_t* blk_out, orc_step* steps,
               int64_t* build_sweeps, int64_t* build_visits) {
    return orc_greedy_observed(n, xadj, adj, thr_edge, J, seed, K, eps_g, eps_l, eps_c, M, blk_out, steps,
                               build_sweeps, build_visits, NULL, NULL);
}
