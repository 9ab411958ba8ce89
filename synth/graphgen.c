/*
 * Seeded synthetic graph generators (input synthesis only).
 *
 * This file holds no arithmetic of the influence-maximisation method: it only
 * produces directed graphs in CSR form (out-adjacency, rows sorted by target,
 * self-loops and duplicate edges removed).  Both the CPU oracle and the GPU
 * library consume the bytes it writes.
 *
 * Random numbers come from a counter-based generator: output(ctr) is the
 * SplitMix64 finaliser applied to base + (ctr + 1) * golden, so every draw is
 * a pure function of (seed, draw index) and the result does not depend on the
 * number of threads.
 *
 * R-MAT: each draw descends `scale` levels of the adjacency matrix; at every
 * level a 32-bit uniform value r picks quadrant (0,0) if r < A, (0,1) if
 * r < A+B, (1,0) if r < A+B+C, else (1,1), with A, B, C the quadrant
 * probabilities scaled to 2^32.  No noise, no vertex permutation.
 *
 * Erdos-Renyi: distinct ordered pairs (u, v), u != v, drawn uniformly by
 * rejection until m pairs are accepted.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t ctr_rand(uint64_t base, uint64_t ctr) {
    return sm64_mix(base + (ctr + 1) * GOLDEN);
}

static inline uint64_t seed_base(uint64_t seed) { return sm64_mix(seed ^ 0x6A09E667F3BCC909ULL); }

/* Scaled quadrant thresholds: floor(p * 2^32), computed from doubles. */
static void quad_thresholds(double a, double b, double c, uint64_t* ta, uint64_t* tab, uint64_t* tabc) {
    const double two32 = 4294967296.0;
    *ta = (uint64_t)(a * two32);
    *tab = (uint64_t)((a + b) * two32);
    *tabc = (uint64_t)((a + b + c) * two32);
}

/*
 * Draw `draws` R-MAT edges at the given scale; drop self-loops.
 * keys_out[i] = (u << 32) | v for the kept draws, in draw order.
 * Returns the number of kept draws.
 */
int64_t gg_rmat_draw(int scale, int64_t draws, double a, double b, double c, uint64_t seed, uint64_t* keys_out,
                     uint8_t* keep_tmp) {
    uint64_t ta, tab, tabc;
    quad_thresholds(a, b, c, &ta, &tab, &tabc);
    const uint64_t base = seed_base(seed);
    const int64_t words_per_draw = (scale + 1) / 2;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < draws; ++i) {
        uint64_t u = 0, v = 0;
        for (int l = 0; l < scale; ++l) {
            uint64_t w = ctr_rand(base, (uint64_t)(i * words_per_draw + l / 2));
            uint64_t r = (l & 1) ? (w >> 32) : (w & 0xFFFFFFFFULL);
            uint64_t ub = r >= tab;
            uint64_t vb = (r >= ta && r < tab) || (r >= tabc);
            u = (u << 1) | ub;
            v = (v << 1) | vb;
        }
        keys_out[i] = (u << 32) | v;
        keep_tmp[i] = (u != v);
    }
    int64_t k = 0;
    for (int64_t i = 0; i < draws; ++i)
        if (keep_tmp[i]) keys_out[k++] = keys_out[i];
    return k;
}

static int cmp_i32(const void* x, const void* y) {
    int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
    return (a > b) - (a < b);
}

/*
 * Turn (u << 32 | v) keys into a CSR with rows sorted by v and duplicates
 * removed.  xadj has n+1 entries; adj must hold cnt entries (the final edge
 * count is xadj[n] <= cnt).  row_tmp must hold n+1 int64 entries.
 * Returns the number of distinct edges.
 */
int64_t gg_keys_to_csr(const uint64_t* keys, int64_t cnt, int64_t n, int64_t* xadj, int32_t* adj, int64_t* row_tmp) {
    memset(row_tmp, 0, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t i = 0; i < cnt; ++i) row_tmp[(keys[i] >> 32) + 1]++;
    for (int64_t u = 0; u < n; ++u) row_tmp[u + 1] += row_tmp[u];
    /* scatter (stable, single-threaded) */
    int64_t* pos = xadj; /* reuse xadj as the running cursor */
    for (int64_t u = 0; u <= n; ++u) pos[u] = row_tmp[u];
    for (int64_t i = 0; i < cnt; ++i) {
        uint64_t u = keys[i] >> 32;
        adj[pos[u]++] = (int32_t)(keys[i] & 0xFFFFFFFFULL);
    }
    /* sort + unique each row in parallel, record new lengths */
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t u = 0; u < n; ++u) {
        int64_t b = row_tmp[u], e = row_tmp[u + 1];
        if (e - b > 1) qsort(adj + b, (size_t)(e - b), sizeof(int32_t), cmp_i32);
        int64_t w = b;
        for (int64_t i = b; i < e; ++i)
            if (i == b || adj[i] != adj[i - 1]) adj[w++] = adj[i];
        pos[u] = w - b; /* distinct length of row u (pos reused) */
    }
    /* compact rows to the front */
    int64_t out = 0;
    for (int64_t u = 0; u < n; ++u) {
        int64_t b = row_tmp[u], len = pos[u];
        if (out != b) memmove(adj + out, adj + b, sizeof(int32_t) * (size_t)len);
        row_tmp[u] = out;
        out += len;
    }
    for (int64_t u = 0; u < n; ++u) xadj[u] = row_tmp[u];
    xadj[n] = out;
    return out;
}

/* Open-addressing set of u64 keys (ER rejection). */
typedef struct {
    uint64_t* slots;
    uint64_t mask;
} u64set;

static int u64set_insert(u64set* s, uint64_t key) {
    uint64_t k = key + 1; /* 0 marks an empty slot */
    uint64_t i = sm64_mix(k) & s->mask;
    while (s->slots[i]) {
        if (s->slots[i] == k) return 0;
        i = (i + 1) & s->mask;
    }
    s->slots[i] = k;
    return 1;
}

/*
 * Erdos-Renyi: m distinct ordered pairs (u, v) with u != v, u, v uniform in
 * [0, n), accepted in draw order.  keys_out holds m keys.  Returns m, or -1 if
 * m exceeds n(n-1) or memory runs out.
 */
int64_t gg_er_draw(int64_t n, int64_t m, uint64_t seed, uint64_t* keys_out) {
    if (n < 2 || m > n * (n - 1)) return m == 0 ? 0 : -1;
    uint64_t cap = 1;
    while (cap < (uint64_t)m * 2 + 16) cap <<= 1;
    u64set s = {calloc(cap, sizeof(uint64_t)), cap - 1};
    if (!s.slots) return -1;
    const uint64_t base = seed_base(seed);
    uint64_t ctr = 0;
    int64_t k = 0;
    while (k < m) {
        uint64_t w = ctr_rand(base, ctr++);
        uint64_t u = ((w & 0xFFFFFFFFULL) * (uint64_t)n) >> 32;
        uint64_t v = ((w >> 32) * (uint64_t)n) >> 32;
        if (u == v) continue;
        uint64_t key = (u << 32) | v;
        if (u64set_insert(&s, key)) keys_out[k++] = key;
    }
    free(s.slots);
    return k;
}

/* Uniform 64-bit word for (seed, ctr): exposed so Python-side recipes draw from the same generator. */
uint64_t gg_rand64(uint64_t seed, uint64_t ctr) { return ctr_rand(seed_base(seed), ctr); }
