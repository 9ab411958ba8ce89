/*
 * im.h -- C ABI of the MI355X (gfx950) library for sketch-based influence
 * maximisation with hash-based fused sampling and error-adaptive rebuild
 * (Gokturk & Kaya, arXiv 2105.04023, "HyperFuseR").
 *
 * Conventions for every call:
 *  - Plain pointers and sizes only.  A pointer is a host pointer unless the
 *    argument or struct field says it is a device pointer.
 *  - Inputs are borrowed for the duration of the call and never retained.
 *  - Handles own their device memory until the matching *_free call.
 *  - Errors are returned as im_status; im_last_error() gives a thread-local
 *    message.  Validation errors leave existing handles unchanged.  A device
 *    error (IM_ERR_DEVICE) poisons the handle it happened on: later calls on
 *    it return IM_ERR_STATE.  The library never aborts the process.
 *  - Work is enqueued on the context's HIP stream; a call returns after the
 *    stream work it needs for its outputs has completed.
 *  - Calls on one handle are not thread-safe; distinct handles may be used from
 *    distinct threads when they belong to distinct contexts.
 */
#ifndef IM_H
#define IM_H

#include <stddef.h>
#include <stdint.h>

/* Entry points are the only symbols the shared library exports. */
#if defined(__GNUC__)
#define IM_API __attribute__((visibility("default")))
#else
#define IM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum im_status {
    IM_OK = 0,
    IM_ERR_INVALID_ARG = -1,   /* a scalar argument or pointer is invalid */
    IM_ERR_INVALID_GRAPH = -2, /* the CSR is malformed (offsets or ids out of range) */
    IM_ERR_OUT_OF_BUDGET = -3, /* the request exceeds the context's device-memory budget */
    IM_ERR_DEVICE = -4,        /* a HIP call failed */
    IM_ERR_STATE = -5          /* the handle is poisoned or in the wrong state */
} im_status;

/* Edge-probability model (Sec. 2.1): independent cascade with one constant
 * probability, weighted cascade w_uv = 1/d_v with d_v the in-degree of v, or
 * independent cascade with one binary32 probability per edge. */
typedef enum im_prob_kind {
    IM_PROB_CONSTANT = 0,
    IM_PROB_WEIGHTED_CASCADE = 1,
    IM_PROB_PER_EDGE = 2
} im_prob_kind;

/* Directed graph in compressed sparse rows over OUT-neighbours (Sec. 3.3):
 * the out-neighbours of vertex u are adj[xadj[u] .. xadj[u+1]-1].
 * Requirements: n >= 1, xadj[0] = 0, xadj nondecreasing, xadj[n] = m,
 * 0 <= adj[e] < n, n < 2^31.  Duplicate edges and self-loops are accepted
 * (they do not change the registers; they do count towards in-degrees for the
 * weighted cascade).  The offsets are int64 (offset_bits 0 or 64) or int32
 * (offset_bits 32, which needs m < 2^31); the library keeps its own int64
 * copy either way.  Any other offset_bits is IM_ERR_INVALID_ARG. */
typedef struct im_csr {
    int64_t n;
    int64_t m;
    const void* xadj;    /* n+1 offsets, int64_t or int32_t per offset_bits */
    const int32_t* adj;  /* m vertex ids */
    int32_t on_device;   /* 0: xadj/adj are host pointers; 1: device pointers on the context's device */
    int32_t offset_bits; /* 0 or 64: int64 offsets; 32: int32 offsets */
} im_csr;

/* Edge probabilities w_uv in [0, 1] (Sec. 2.1).  per_edge (kind PER_EDGE)
 * holds m binary32 values aligned with adj, resident where the CSR is. */
typedef struct im_probs {
    im_prob_kind kind;
    float p;
    const float* per_edge;
} im_probs;

/* Options of the sketch build.  eps_c is the early-exit ratio of Alg. 2:
 * sweeping stops once |L| <= eps_c * n (0 = run to the fixed point).  The
 * tuning fields select the work decomposition only; results do not depend on
 * them.  Zero means "library default". */
#define IM_BUILD_TIME_SWEEPS 1 /* record HIP-event timings of every sweep (im_sketch_get_sweep_log) */
#define IM_BUILD_IN_PLACE 2    /* in-place sweeps: a sweep reads registers this sweep already raised
                                  (the paper's own update order, Sec. 3.3).  Every Simulate, build
                                  and rebuilds, then reaches the same fixed point in at most as many
                                  sweeps; registers, estimates and seeds equal those of synchronous
                                  sweeps when eps_c = 0, while sweep and visit counts depend on the
                                  schedule (not reproducible). */
#define IM_BUILD_TIME_PIECES 8 /* record the sweep log with HIP-event timings of the split-row
                                  piece kernel only (heavy_ms; kernel_ms and sweep_ms are 0): two
                                  events per sweep instead of six, so the timing costs the sweeps
                                  less.  IM_BUILD_TIME_SWEEPS includes it. */
#define IM_BUILD_ATOMIC_REVERSE 4 /* build the reverse CSR (in-edges, for sparse sweeps) with global
                                     atomics on an auxiliary stream beside the first sweeps, the
                                     method used anyway when n > 2^25 or m >= 2^31; otherwise it
                                     is a counting sort on the build's stream.  Results are the
                                     same either way. */
typedef struct im_build_opts {
    double eps_c;
    int32_t heavy_degree; /* rows with more out-edges are split across waves (0: 64) */
    int32_t piece_edges;  /* edges per piece of a split row, at most 2048 (0: 256) */
    int32_t sparse_div;   /* sweep t > 0 visits only the rows next to L_t when the
                             in-degrees of L_t sum to at most m / sparse_div
                             (0: 8; < 0: never) */
    int32_t flags;        /* IM_BUILD_* bits */
} im_build_opts;

/* Thresholds of the error-adaptive rebuild (Sec. 3.2.1): the sketches are
 * kept when err_l < eps_l or err_g < eps_g, otherwise rebuilt.  The paper
 * uses eps_l = 0.3 and eps_g = 0.01. */
typedef struct im_select_opts {
    double eps_g;
    double eps_l;
} im_select_opts;

/* One greedy step of Alg. 1. */
typedef struct im_step {
    int32_t seed;    /* vertex added to S at this step */
    int32_t rebuilt; /* 1 if the sketches were rebuilt after this step */
    int32_t fresh;   /* 1 if err_l < eps_l or err_g < eps_g */
    int32_t sweeps;  /* sweeps of the rebuild (0 if none) */
    int64_t score;   /* integer register sum of Merge(M_S', M_s) */
    int64_t reach;   /* blocked (vertex, simulation) pairs after this step = sigma * R */
    double e;        /* Estimate(Merge(M_S', M_s)) */
    double sigma;    /* Monte-Carlo influence of S over the R samples */
    double delta;    /* sigma minus sigma at the last rebuild */
    double err_l;    /* |(e - delta) / delta| (+inf if delta = 0) */
    double err_g;    /* |(e - delta) / sigma| */
    int64_t visits;  /* edge visits (edges with a live head, summed over sweeps) of the rebuild */
} im_step;

typedef struct im_sketch_info {
    int64_t n;
    int64_t m;
    int32_t R;
    int32_t sweeps;        /* sweeps of the build */
    int64_t visits;        /* edges with a live head, summed over the build's sweeps */
    double build_ms;       /* device time of the build's Simulate (init + sweeps) */
    double prep_ms;        /* device time of graph upload, hashing and thresholds */
    size_t device_bytes;   /* device memory held by the sketch */
    int64_t heavy_rows;    /* rows split across waves */
    int64_t heavy_pieces;
} im_sketch_info;

typedef struct im_select_stats {
    int32_t rebuilds;
    int32_t reserved;
    int64_t rebuild_sweeps;
    int64_t rebuild_visits;
    int64_t bfs_levels;
    double device_ms; /* device time of im_select_seeds (events on the context stream) */
    double wall_ms;   /* host wall time of im_select_seeds */
} im_select_stats;

typedef struct im_ctx im_ctx;
typedef struct im_sketch im_sketch;

/* Device allocator hooks; both NULL selects hipMalloc/hipFree.  alloc returns a
 * device pointer aligned to 256 bytes, or NULL on failure. */
typedef void* (*im_alloc_fn)(size_t bytes, void* user);
typedef void (*im_free_fn)(void* ptr, void* user);

/* Creates a context on HIP device `device`.  `stream` is a hipStream_t (NULL =
 * the null stream) that must outlive the context.  hbm_budget bounds the
 * device bytes all sketches of this context may hold (0 = no bound). */
IM_API im_status im_ctx_create(int32_t device, void* stream, size_t hbm_budget, im_alloc_fn alloc, im_free_fn dealloc,
                        void* user, im_ctx** out);
IM_API void im_ctx_free(im_ctx* ctx);
/* Device bytes currently held by sketches of the context. */
IM_API size_t im_ctx_bytes_in_use(const im_ctx* ctx);

/* Device bytes a sketch of this shape would hold at its peak, the temporaries
 * of its preparation included (for admission by budget). */
IM_API size_t im_sketch_bytes_needed(int64_t n, int64_t m, int32_t R, im_prob_kind kind);

/*
 * Builds the per-vertex sketches (Alg. 1 initialisation and Alg. 2 Simulate).
 * Uploads or copies the graph, computes the 31-bit Murmur3 edge hashes
 * (Eq. hash), the per-simulation words X_j and the integer live thresholds of
 * Eq. (hash_prob), initialises M_v[j] = clz(hash(v) xor hash(j)), and runs
 * synchronous pull sweeps until |L| <= eps_c * n.
 * R: registers (= simulations) per vertex, a multiple of 4 in [4, 1024].
 * hash_seed: seed of every hash.  opts may be NULL.
 * On success *out owns the graph copy and the registers.
 */
IM_API im_status im_build_sketches(im_ctx* ctx, const im_csr* graph, const im_probs* probs, int32_t R, uint32_t hash_seed,
                            const im_build_opts* opts, im_sketch** out);

/*
 * Estimate (Eq. sketch-estimate, with the merge of Eq. sketch-merge) of the
 * union of the sketches of `count` vertices, from the registers of the build:
 * e = 2^(mean_j max_v M_v[j]) / 0.77351, returned as binary32.  verts is a host
 * array of ids in [0, n); count >= 1.
 */
IM_API im_status im_estimate(im_sketch* sk, const int32_t* verts, int64_t count, float* out_estimate);

/* Per-vertex estimates of the build's registers: out[v] = Estimate(M_v) as
 * binary32.  out holds n floats; out_on_device selects a device pointer. */
IM_API im_status im_estimate_all(im_sketch* sk, float* out, int32_t out_on_device);

/*
 * Greedy seed selection with error-adaptive rebuild (Alg. 1).  Starts from the
 * build's registers every time it is called (the build is kept), so repeated
 * calls with different K return consistent prefixes.  K in [1, n].
 * out_seeds: K ids.  out_steps: K records or NULL.  stats may be NULL.
 * opts NULL selects eps_g = 0.01, eps_l = 0.3.
 */
IM_API im_status im_select_seeds(im_sketch* sk, int32_t K, const im_select_opts* opts, int32_t* out_seeds,
                          im_step* out_steps, im_select_stats* stats);

/*
 * Greedy seed selection (Alg. 1) that reuses the sketch's last selection.
 * Every successful im_select_seeds, im_select_seeds_noalloc or
 * im_select_seeds_resume call on a sketch records its greedy run (K steps,
 * host memory).  When the thresholds equal that run's, this call answers K up
 * to its length from the record, with no device work (the first K steps of a
 * run are the run with K seeds: Alg. 1 rebuilds nothing after the last step),
 * and a larger K continues the run from its last step (whose rebuild decision
 * is taken again, now that a step follows) instead of starting from the
 * build.  Other thresholds, or no recorded run, start from the build as
 * im_select_seeds does.  Outputs are those im_select_seeds returns for the
 * same K and thresholds, bit for bit; stats->device_ms counts only this call's
 * device work (0 when answered from the record).  A failed call drops the
 * record.  Same arguments and errors as im_select_seeds.
 */
IM_API im_status im_select_seeds_resume(im_sketch* sk, int32_t K, const im_select_opts* opts, int32_t* out_seeds,
                                        im_step* out_steps, im_select_stats* stats);

/*
 * Allocation-free variant of im_select_seeds, for callers that cannot allocate
 * device memory during the call (code under stream capture, tight serving
 * loops, harnesses that forbid allocation).  Same arguments, results and
 * errors as im_select_seeds, with K in [1, IM_NOALLOC_MAX_K] (larger K:
 * IM_ERR_INVALID_ARG before any device work).  The per-call step records and
 * seeds live in a fixed 512 KiB device array that every GPU the library runs
 * on holds until the process ends; no device memory is allocated or freed.
 * All calls on one GPU share that array: calls that overlap in time on the
 * same GPU (from different threads or contexts) race and must be serialised
 * by the caller.  The context must have been created by im_ctx_create on that
 * GPU (which records the array's device address).
 */
#define IM_NOALLOC_MAX_K 4096
IM_API im_status im_select_seeds_noalloc(im_sketch* sk, int32_t K, const im_select_opts* opts, int32_t* out_seeds,
                                         im_step* out_steps, im_select_stats* stats);

/* Build information; trace of the build: live_counts[t] = |L_t| (t = 0..sweeps)
 * and edge_visits[t] = edges with a live head in sweep t (t < sweeps); cap
 * bounds both arrays; *written receives sweeps+1. */
IM_API im_status im_sketch_get_info(const im_sketch* sk, im_sketch_info* info);
IM_API im_status im_sketch_get_trace(const im_sketch* sk, int64_t* live_counts, int64_t* edge_visits, int32_t cap,
                              int32_t* written);

/* One sweep, recorded when the build was asked to time sweeps
 * (IM_BUILD_TIME_SWEEPS, or IM_BUILD_TIME_PIECES for heavy_ms alone): kernel_ms is the device time of the row
 * kernel, heavy_ms that of the split-row piece kernel, sweep_ms that of all
 * kernels of the sweep, from HIP events on the context stream; light_visits the edges
 * with a live head the row kernel visited, visits those of the whole sweep, live_next
 * |L_{t+1}|; light_merged and merged count the visited edges whose head's row was
 * merged, i.e. those live in at least one of the R samples (an edge live in none still
 * counts as visited, but its head's row, hash and threshold are not read).  ran = 0 marks a launch past the stopping rule (it returned at
 * once).  simulate numbers the Simulate calls of the sketch (0 = build,
 * later ones are rebuilds inside im_select_seeds). */
typedef struct im_sweep_rec {
    int32_t simulate;
    int32_t sweep;
    int32_t ran;
    float kernel_ms;  /* row kernel */
    float sweep_ms;   /* every kernel of the sweep */
    float heavy_ms;   /* split-row piece kernel */
    int64_t light_visits;
    int64_t visits;
    int64_t live;      /* |L_t| */
    int64_t live_next; /* |L_{t+1}| */
    int32_t sparse;    /* 1 if the sweep visited only the rows next to L_t */
    int32_t reserved;
    int64_t light_merged; /* edges of light_visits whose head's row was merged */
    int64_t merged;       /* the same over the whole sweep */
} im_sweep_rec;

/* Copies up to cap records of the sweep log; returns the number copied. */
IM_API int32_t im_sketch_get_sweep_log(const im_sketch* sk, im_sweep_rec* out, int32_t cap);
IM_API void im_sketch_clear_sweep_log(im_sketch* sk);

/* Copies registers to the host, n*R bytes, vertex-major (R registers of a
 * vertex adjacent).  which = 0: registers of the build; which = 1: registers
 * in force at the end of the greedy run the sketch holds (that of the last
 * selection call, or, after an im_select_seeds_resume answered from its
 * record, the recorded run's). */
IM_API im_status im_sketch_get_registers(const im_sketch* sk, int32_t which, uint8_t* out);

/* Copies the blocked pairs of the greedy run the sketch holds (the reach of
 * its S in every sample; which run: as for im_sketch_get_registers, which = 1)
 * to the host as n*R bytes (1 = blocked). */
IM_API im_status im_sketch_get_blocked(const im_sketch* sk, uint8_t* out);

IM_API void im_sketch_free(im_sketch* sk);

/*
 * Independent Monte-Carlo evaluation of a seed set: sigma(S) = (1/R) sum_j
 * |vertices reachable from S in sample j| over R samples drawn with
 * hash_seed (use a seed other than the selection's for samples independent of
 * the sketches): live-edge samples as in Eq. (hash_prob), then one
 * multi-source reach search over all samples at once (Alg. 1's reach step
 * from the whole set).  graph and probs as in im_build_sketches; seeds holds
 * count >= 1 host vertex ids (repeats allowed).  *out_sigma receives sigma,
 * *out_reach (may be NULL) the reached (vertex, sample) pairs.  Temporary
 * device memory comes from the context and is released before returning.
 */
IM_API im_status im_evaluate_influence(im_ctx* ctx, const im_csr* graph, const im_probs* probs, int32_t R,
                                       uint32_t hash_seed, const int32_t* seeds, int32_t count, double* out_sigma,
                                       int64_t* out_reach);

/*
 * ---------------------------------------------------------------------------
 * Batched solve: many independent problems (graphs of uneven sizes, edge
 * models and R) solved together by ONE persistent kernel launch, captured
 * once in a HIP graph at im_batch_create and replayed by im_batch_run.  Each
 * job computes exactly what im_build_sketches followed by im_select_seeds
 * computes for it alone (Alg. 1 with Alg. 2): the same registers, sweep
 * counts, edge visits, seeds and step records.  The work decomposition
 * (lanes per row, tile sizes, grid) never changes a result.
 * ---------------------------------------------------------------------------
 */
typedef struct im_batch_job {
    im_csr graph;        /* host or device CSR (graph.on_device); copied at create, not retained */
    im_probs probs;      /* per_edge resides where the CSR resides */
    int32_t R;           /* registers (= simulations) per vertex: a multiple of 4 in [4, 256] */
    int32_t K;           /* seeds to select, in [1, n] */
    uint32_t hash_seed;  /* seed of every hash, as in im_build_sketches */
    int32_t reserved;
    double eps_c;        /* early exit of every Simulate, as im_build_opts.eps_c */
    double eps_g, eps_l; /* rebuild thresholds, as im_select_opts (no defaults are substituted) */
} im_batch_job;

/* Work decomposition of the persistent solver.  Zero selects the default.
 * autotune = 1: im_batch_create solves the batch once per candidate
 * decomposition (lanes per row: the smallest power of two covering a row and
 * twice that; tile size; XCD pinning; grid), keeps the fastest, and fails with
 * IM_ERR_DEVICE if any two candidates disagree on a seed.  Fields set to
 * nonzero values are not varied. */
typedef struct im_batch_opts {
    int32_t autotune;
    int32_t lanes_per_row; /* power of two in [max(4, R_max/4), 64]; default the smallest */
    int32_t tile_edges;    /* edges per sweep tile; default 8192 */
    int32_t heavy_degree;  /* rows with more out-edges are split into pieces; default 512 */
    int32_t piece_edges;   /* edges per piece; default 512 */
    int32_t workgroups;    /* persistent grid, 256-thread workgroups; default 4 per compute unit */
    int32_t pin_edges;     /* jobs with at most this many edges run on one XCD each; default half
                              of one XCD's share of the batch's edges; negative: every job runs
                              on every XCD */
    int32_t reserved;
} im_batch_opts;

typedef struct im_batch_job_result {
    int32_t status;       /* IM_OK, or the device-side error that stopped this job */
    int32_t build_sweeps; /* sweeps of the build */
    int32_t rebuilds;
    int32_t reserved;
    int64_t build_visits; /* edges with a live head, summed over the build's sweeps */
    int64_t rebuild_sweeps;
    int64_t rebuild_visits;
    int64_t bfs_levels;   /* reach levels with work, over all steps */
} im_batch_job_result;

typedef struct im_batch_stats {
    double device_ms;   /* the replayed launch, from HIP events */
    double wall_ms;     /* host wall time of im_batch_run */
    int64_t tiles;      /* tiles processed */
    int64_t phases;     /* phase transitions over all jobs */
    int32_t lanes_per_row, tile_edges, heavy_degree, piece_edges, workgroups;
    int32_t candidates; /* decompositions the autotuner timed (0 without autotuning) */
} im_batch_stats;

typedef struct im_batch im_batch;

/* Validates and uploads every job (count >= 1), allocates all device state
 * through the context (IM_ERR_OUT_OF_BUDGET beyond its budget) and captures
 * the launch.  opts may be NULL.  On success *out owns everything. */
IM_API im_status im_batch_create(im_ctx* ctx, int32_t count, const im_batch_job* jobs, const im_batch_opts* opts,
                                 im_batch** out);
/* Solves every job (one graph launch on a stream of the batch, ordered after
 * work already enqueued on the context's stream) and waits for it.  May be
 * called repeatedly; each run starts from the uploaded graphs.  stats may be
 * NULL.  A device-side stop (watchdog) returns IM_ERR_DEVICE and poisons b. */
IM_API im_status im_batch_run(im_batch* b, im_batch_stats* stats);
/* Results of job `job` (the caller's index) from the last run: K seeds,
 * K step records (or NULL), counters (or NULL).  Returns the job's status. */
IM_API im_status im_batch_get_result(const im_batch* b, int32_t job, int32_t* out_seeds, im_step* out_steps,
                                     im_batch_job_result* res);
/* Registers of job `job` after the last run, n*R bytes vertex-major:
 * which = 0 those of the build, 1 those in force at the end of the greedy loop. */
IM_API im_status im_batch_get_registers(const im_batch* b, int32_t job, int32_t which, uint8_t* out);
/* Device bytes held by the batch. */
IM_API size_t im_batch_device_bytes(const im_batch* b);
IM_API void im_batch_free(im_batch* b);

/*
 * ---------------------------------------------------------------------------
 * Serving: requests (graph, edge model, R, K) over a pool of resident graphs,
 * answered by `slots` concurrent slots.  Each slot has its own host thread and
 * HIP stream, so requests of different slots overlap on the device.  Requests
 * wait in one queue; each free slot takes the oldest request it can start now,
 * so a request is admitted as soon as any slot and the memory it needs are
 * free.  Sketches stay resident in one pool and are reused, on whichever slot
 * runs the request, by later requests with the same (graph, model, p, R, hash
 * seed, eps_c); a sketch serves one request at a time, and a key whose copies
 * are all busy may get another copy, up to max_copies.  Selections go through
 * im_select_seeds_resume, so a request whose sketch copy last served the same
 * thresholds reuses or continues that greedy run; its result still equals
 * im_build_sketches + im_select_seeds run alone.  hbm_budget (0 = none) bounds the device memory of the resident graphs
 * plus all sketches: a build evicts idle sketches, least recently used first,
 * until it fits, and a request whose sketch cannot fit even alone fails with
 * IM_ERR_OUT_OF_BUDGET without evicting anything.
 * ---------------------------------------------------------------------------
 */
typedef struct im_server_opts {
    int32_t slots;      /* concurrent requests, in [1, 64] */
    int32_t max_copies; /* resident copies one sketch key may have, in [1, 64] (0: 1).  With
                           resumed selection a key's requests mostly need no device work, so a
                           second copy (a second build) pays only when requests of one key that
                           need new greedy steps overlap. */
    size_t hbm_budget;  /* device bytes for graphs and sketches; 0 = no bound */
} im_server_opts;

typedef struct im_request {
    int32_t graph;       /* id from im_server_add_graph */
    im_prob_kind kind;   /* IM_PROB_CONSTANT or IM_PROB_WEIGHTED_CASCADE */
    float p;             /* constant probability (kind IM_PROB_CONSTANT) */
    int32_t R;           /* multiple of 4 in [4, 1024] */
    int32_t K;           /* in [1, n] */
    uint32_t hash_seed;
    double eps_c;        /* as im_build_opts.eps_c */
    double eps_g, eps_l; /* as im_select_opts (no defaults are substituted) */
} im_request;

typedef struct im_response {
    int32_t status;        /* IM_OK, or the error of this request */
    int32_t slot;          /* slot that served it (-1: it never ran) */
    int32_t sketch_reused; /* 1 if its sketches were resident already */
    int32_t rebuilds;      /* rebuilds of its greedy selection */
    double queue_ms;       /* submit to start */
    double build_ms;       /* sketch build (0 when reused) */
    double select_ms;      /* greedy selection */
    double latency_ms;     /* submit to completion */
} im_response;

typedef struct im_server_stats {
    int64_t submitted, completed, failed;
    int64_t sketches_built, evictions, resident_sketches;
    size_t device_bytes;   /* graphs plus resident sketches */
} im_server_stats;

typedef struct im_server im_server;

IM_API im_status im_server_create(int32_t device, const im_server_opts* opts, im_server** out);
/* Copies a CSR (host or device) into the resident pool; all graphs are added
 * before the first request.  *out_graph receives its id. */
IM_API im_status im_server_add_graph(im_server* sv, const im_csr* graph, int32_t* out_graph);
/* Queues a request; out_seeds (K entries, host) must stay valid until
 * im_server_wait returns for *out_ticket.  Thread-safe. */
IM_API im_status im_server_submit(im_server* sv, const im_request* rq, int32_t* out_seeds, int64_t* out_ticket);
/* Blocks until the request is done; fills *out (may be NULL) and returns its status. */
IM_API im_status im_server_wait(im_server* sv, int64_t ticket, im_response* out);
/* Cancels a request that has not started: IM_OK, after which im_server_wait
 * returns IM_ERR_STATE for it (its out_seeds are not written); IM_ERR_STATE if
 * it already started, finished or the ticket is unknown.  Thread-safe. */
IM_API im_status im_server_cancel(im_server* sv, int64_t ticket);
IM_API im_status im_server_get_stats(im_server* sv, im_server_stats* out);
/* Finishes the queued requests, then frees every resource of the server. */
IM_API void im_server_free(im_server* sv);

/* Thread-local message of the last failed call on this thread ("" if none). */
IM_API const char* im_last_error(void);

/* Library version string. */
IM_API const char* im_version(void);

#ifdef __cplusplus
}
#endif

#endif /* IM_H */
