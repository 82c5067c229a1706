/*
 * pacim.h -- C-ABI of the MI355X (gfx950) sketch-based influence-maximization
 * library: the hot path of PaC-IM (Wang, Ding, Gu, Sun, "Fast and
 * Space-Efficient Parallel Algorithms for Influence Maximization", PVLDB 17(3),
 * 2023) under the Independent Cascade (IC) model on undirected graphs.
 *
 * The library computes, for a graph G, an edge-probability model, R sketches
 * and k, the greedy seed sequence s_1..s_k and integer gains g_1..g_k with
 *     f(S) = sum_{r<R} | union_{s in S} CC_r(s) |,
 *     s_i = argmax_{v not in S_{i-1}} f(S_{i-1} + v) - f(S_{i-1})   (smallest id on ties),
 *     g_i = f(S_i) - f(S_{i-1}),
 * where CC_r(v) is v's connected component in the r-th sampled graph G'_r
 * (Sec. 2, sketch-based algorithms and memoization; Algorithm 1).  Dividing by R
 * gives the paper's spread estimate; the library keeps the exact integers.
 *
 * Conventions for every call:
 *   - Every function returns im_status.  On error nothing the caller passed as
 *     an output is written, and im_last_error(ctx) describes the failure.
 *   - No exceptions and no C++ types cross this boundary.
 *   - Host buffers are owned by the caller and only read/written during the call.
 *   - Handles (im_ctx, im_graph, im_sketches, im_server) are owned by the
 *     library; free them with the matching *_free / *_destroy call.
 *   - An im_ctx is not thread-safe: use one per host thread (the server API
 *     handles concurrent requests itself).
 *   - Work is issued on the context's HIP stream; calls that return host
 *     results synchronise that stream before returning.
 *
 * Sampling (Sec. 3, function Sample; "fusion" of Sec. 2): edge {u,v} is live in
 * sketch r iff  mix64(((min<<32)|max) ^ K(seed, r)) < T(p_e), where mix64 is the
 * SplitMix64 output function, K(seed, x) = mix64(seed*0x9E3779B97F4A7C15 + x)
 * and T(p) = floor(p * 2^64) for 0 <= p < 1 (every edge live for p >= 1).
 * Sampled graphs are never stored.
 */
#ifndef PACIM_H
#define PACIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IM_OK = 0,
    IM_EINVAL = 1,    /* an argument is out of range or a graph is malformed   */
    IM_ENOMEM = 2,    /* device memory (or the context's HBM cap) is exhausted */
    IM_EDEVICE = 3,   /* a HIP call failed                                     */
    IM_EBUSY = 4,     /* the request can never fit the server's memory budget  */
    IM_EINTERNAL = 5  /* an internal consistency check failed                  */
} im_status;

typedef struct im_ctx im_ctx;
typedef struct im_graph im_graph;
typedef struct im_sketches im_sketches;

/* Edge-probability models (Sec. 5 uses the same p on every edge; the appendix on
 * edge-probability distributions adds per-edge Uniform and WIC assignments).
 * Each becomes an integer threshold T_e, and edge e is live in sketch r iff
 * mix64(((min<<32)|max) ^ K(seed, r)) < T_e, with T(p) = floor(p * 2^64). */
typedef enum {
    IM_PROB_UNIFORM = 0,     /* "Consistent": p_e = p for every edge                           */
    IM_PROB_TRIVALENCY = 1,  /* p_e in {0.1, 0.01, 0.001}, chosen by
                                mix64(((min<<32)|max) ^ K(0, 0xC000000000000002)) mod 3;
                                a property of the edge, independent of the sampling seed */
    IM_PROB_RANGE = 2,       /* "Uniform": p_e uniform over [p, p_hi), drawn once per edge:
                                T_e = T(p) + floor((T(p_hi) - T(p)) * h_e / 2^64) with
                                h_e = mix64(((min<<32)|max) ^ K(0, 0xC000000000000003))   */
    IM_PROB_WIC = 3,         /* "WIC": p_e = 2 / (d_u + d_v), d the degrees in the graph;
                                T_e = floor(2^65 / (d_u + d_v)), always live when d_u + d_v = 2 */
    IM_PROB_PER_EDGE = 4     /* p_e given by the caller for every CSR entry (p_edge), T_e = T(p_e);
                                im_build_sketches, im_select_seeds and im_influence only */
} im_prob_kind;

typedef struct {
    int32_t kind;          /* im_prob_kind */
    double p;              /* IM_PROB_UNIFORM: p in [0, 1]; IM_PROB_RANGE: the low end, 0 <= p <= p_hi */
    double p_hi;           /* IM_PROB_RANGE: the high end, p_hi < 1; ignored otherwise */
    const double *p_edge;  /* IM_PROB_PER_EDGE: host array of m_dir probabilities in [0, 1], entry j
                              for the graph's CSR entry j as uploaded; both directions of an edge must
                              carry the same value (else EINVAL).  Read during the call only. */
} im_prob;

/* ---- context ------------------------------------------------------------ */

/* Creates a context on HIP device `device`.  hip_stream: a hipStream_t to issue
 * work on, or NULL for a library-owned stream (default priority).  hbm_cap: the
 * most device memory (bytes) this context may hold at once, 0 for no cap beyond
 * the device's.  Errors: EINVAL (bad device), EDEVICE. */
im_status im_ctx_create(int device, void *hip_stream, size_t hbm_cap, im_ctx **out);
im_status im_ctx_destroy(im_ctx *ctx);
/* Text of the last error on ctx ("" if none).  Valid until the next call on ctx. */
const char *im_last_error(const im_ctx *ctx);
/* Bytes of device memory the context's live objects hold (used) and its cap.
 * Blocks freed by the library are kept for reuse by later requests of the same
 * size (up to 48 GB, and within the cap together with used); they are released
 * when an allocation fails, when the cap needs them, and by im_ctx_destroy. */
im_status im_ctx_memory(const im_ctx *ctx, size_t *used, size_t *cap);
/* Turns per-kernel HIP-event timing on (1) or off (0); see im_kernel_time. */
im_status im_ctx_set_profiling(im_ctx *ctx, int on);
/* Accumulated launches and milliseconds of one kernel family since profiling was
 * turned on: "init" (a labelling pass's forest set-up), "sample_hook" (sampling
 * and hooking pass), "compress" (pointer jumping and counting), "emit" (full
 * labels, or the compact triple and initial gains), "bulk_keys" (Marginal of every
 * unselected vertex in a bulk round: from E, or from the largest-component
 * bitmaps), "select" (a whole im_select_seeds_from call); and the batched path's
 * graph reuse: "batch_capture" (launches = graphs captured and instantiated) and
 * "batch_replay" (launches = batches that replayed the kept graph).  Unknown
 * names give count 0. */
im_status im_kernel_time(im_ctx *ctx, const char *name, uint64_t *launches, double *ms);

/* ---- graph ---------------------------------------------------------------- */

/* Uploads a simple undirected graph given as a symmetric CSR: offsets[n+1]
 * (uint64, offsets[0] = 0, non-decreasing, offsets[n] = m_dir) and cols[m_dir]
 * (uint32 neighbour ids).  Every undirected edge {u,v} appears as v in u's row
 * and u in v's row, exactly once each (Sec. 5, Table 2: |E| counts these directed
 * entries).  device_ptrs = 1 if offsets/cols are device pointers (read on the
 * context's stream, after the work already queued there), 0 for host.
 * The library copies the graph into memory it owns, with the numbering its
 * union-find passes use (highest degrees first); results use vertex ids.
 * Errors: EINVAL if n == 0, offsets are not monotone, a column is >= n, a row
 * holds a self-loop or a duplicate, or the CSR is not symmetric; ENOMEM. */
im_status im_graph_upload(im_ctx *ctx, uint32_t n, uint64_t m_dir, const uint64_t *offsets,
                          const uint32_t *cols, int device_ptrs, im_graph **out);
im_status im_graph_free(im_graph *g);

/* ---- sketches (Sec. 3: Sketch(r), the sketch triple <r, label, size>) ------ */

/* Builds R sketches of G under model `prob` with sampling seed `seed`.
 * alpha = 1: full labels -- for every vertex v and sketch r the CC label
 *            (a vertex of CC_r(v), the same for all its members; im_sketches_dump
 *            reports the smallest) and, at the label's own entry, the CC size
 *            (the InfuserMG-style memoization the paper extends).
 * 0 < alpha < 1: CompactSketch (Sec. 3) -- vertex v is a center iff
 *            mix64(v ^ K(seed, 0xC000000000000001)) < T(alpha); centers are
 *            ranked by id; per sketch only label_c[i] (smallest center rank in
 *            c_i's CC) and size_c[i] (CC size if label_c[i] = i, else 0) are kept,
 *            and Marginal uses the GetCenter BFS.
 * The initial gains Marginal(empty, v) = sum_r |CC_r(v)| are computed while the
 * components are built.  Requires R >= 1 and ceil(log2(R*n+2)) + ceil(log2 n) <= 64;
 * CompactSketch also needs R*n < 2^40 and R < 2^24.
 * Errors: EINVAL (bad R, alpha outside (0,1], bad prob), ENOMEM, EDEVICE. */
im_status im_build_sketches(im_ctx *ctx, const im_graph *g, im_prob prob, uint32_t R, uint64_t seed,
                            double alpha, im_sketches **out);
im_status im_sketches_free(im_sketches *s);

/* Selects the next k seeds (Algorithm 1's loop: NextSeed by a parallel lazy
 * greedy over a winning tree -- Sec. 4, Algorithm 5 -- then MarkSeed), continuing
 * from the seeds the handle already holds, so k1 then k2 equals k1 + k2 at once.
 * seeds_out[k], gains_out[k]: caller-owned host arrays.  Errors: EINVAL if
 * k > n - (seeds already chosen); EINTERNAL. */
im_status im_select_seeds_from(im_ctx *ctx, im_sketches *s, uint32_t k, uint32_t *seeds_out,
                               uint64_t *gains_out);

/* Selects the next k seeds like im_select_seeds_from, with NextSeed by prefix
 * doubling (Sec. 4, Algorithm 4) instead of the winning tree: the unselected
 * vertices are kept in decreasing order of stale key (larger gain, then smaller
 * id) -- the P-tree's order, held as sorted runs -- and each round takes batches
 * of 1, 2, 4, ... vertices from the front, re-evaluates each batch in parallel,
 * and stops once the best re-evaluated vertex ranks above the first vertex left;
 * the others go back with their new keys.  Seeds and gains equal the winning
 * tree's (Theorem 4.1); the per-round evaluation counts (im_select_trace) are
 * unique and at most twice CELF's in total (Theorem 4.2).  Both selections may
 * be mixed on one handle (each rebuilds its structure from the current keys).
 * Device memory: five arrays of n 64-bit keys, allocated at the first call and
 * held by the handle.  The host waits for each batch.  Errors as
 * im_select_seeds_from, plus ENOMEM. */
im_status im_select_seeds_ptree(im_ctx *ctx, im_sketches *s, uint32_t k, uint32_t *seeds_out,
                                uint64_t *gains_out);

/* One shot with full labels: build R sketches, select k seeds, free.
 * Same errors as im_build_sketches and im_select_seeds_from. */
im_status im_select_seeds(im_ctx *ctx, const im_graph *g, im_prob prob, uint32_t R, uint32_t k,
                          uint64_t seed, uint32_t *seeds_out, uint64_t *gains_out);

/* ---- quality ------------------------------------------------------------- */

/* Influence spread of a seed set by simulation (the quality measure of Sec. 5).
 * Under IC on an undirected graph a cascade flips each edge's coin once, so
 * simulation w is the live-edge world drawn like a sketch with key K(sim_seed, w),
 * and the cascade from the seeds activates every vertex connected to one of them.
 * *total_out = the sum over worlds w in [w0, w0 + sims) of the number of
 * activated vertices; the spread estimate is *total_out / sims.  seeds: host
 * array of k vertex ids (duplicates count once).  Worlds are labelled 64 per
 * pass with the sketch kernels; device memory for that is held only during the
 * call.  Errors: EINVAL (seed >= n, bad model, w0 + sims > 2^32), ENOMEM,
 * EDEVICE. */
im_status im_influence(im_ctx *ctx, const im_graph *g, im_prob prob, const uint32_t *seeds, uint32_t k,
                       uint64_t sim_seed, uint32_t w0, uint32_t sims, uint64_t *total_out);

/* im_influence for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * arguments, result and errors, but the call allocates nothing.  Its scratch
 * (world keys, the seed list, the running total and the labelling forests of up
 * to 64 worlds per pass) lives in one static device array of
 * im_influence_static_scratch() bytes (64 MiB), held by every device the library
 * runs on until the process ends; its device address is resolved once per device
 * by im_ctx_create.  Limits: one world takes 12 bytes per vertex (rounded up to
 * the sketch stride), so n is at most about 5.5 million, and 12 * n + 4 * k must
 * fit the array; larger inputs, and IM_PROB_PER_EDGE (whose thresholds would need
 * device memory), are rejected with EINVAL before any device work.  Every call
 * on one device shares that device's array: calls that overlap on one device
 * (two contexts or threads) race and must be serialised by the caller.  Each
 * call initialises every part of the array it reads.  No profiling timers. */
im_status im_influence_noalloc(im_ctx *ctx, const im_graph *g, im_prob prob, const uint32_t *seeds, uint32_t k,
                               uint64_t sim_seed, uint32_t w0, uint32_t sims, uint64_t *total_out);
/* Size in bytes of im_influence_noalloc's static device scratch. */
im_status im_influence_static_scratch(size_t *max_bytes);

/* ---- inspection (tests, measurement) -------------------------------------- */

/* Sketch r as it was built (MarkSeed's zeroing not applied):
 * full labels: labels[n] = CC label of every vertex, sizes[n] = CC size of every vertex;
 * CompactSketch: labels[rho] = label_c, sizes[rho] = size_c (see im_centers for rho).
 * Caller-owned host arrays.  Errors: EINVAL if r >= R. */
im_status im_sketches_dump(im_ctx *ctx, const im_sketches *s, uint32_t r, uint32_t *labels, uint32_t *sizes);
/* Centers of a CompactSketch (all vertices for alpha = 1): *rho gets their
 * number; centers (may be NULL) receives them in increasing id order. */
im_status im_centers(im_ctx *ctx, const im_sketches *s, uint32_t *centers, uint32_t *rho);
/* Initial gains Marginal(empty, v) for every vertex: gains[n], host. */
im_status im_initial_gains(im_ctx *ctx, const im_sketches *s, uint64_t *gains);
/* Re-evaluations NextSeed performed in each of the first `count` rounds
 * (count <= seeds chosen so far): the per-round |F_i| of Sec. 4 (the stale
 * vertices re-evaluated before the seed is known), for comparison with CELF.
 * Not unique: it depends on the traversal schedule. */
im_status im_select_trace(im_ctx *ctx, const im_sketches *s, uint32_t *evals_per_round, uint32_t count);
/* Counters of the handle: seeds chosen so far, total and per-call re-evaluations
 * performed by NextSeed, and the sketch build's byte/time figures. */
typedef struct {
    uint32_t seeds_chosen;
    uint32_t rho;
    uint64_t evaluations;        /* vertex re-evaluations by NextSeed, all rounds  */
    uint64_t bfs_overflow;       /* GetCenter searches that left the on-chip queue */
    uint64_t bfs_visits;         /* vertices whose adjacency GetCenter scanned     */
    double build_ms;             /* last im_build_sketches, device time            */
    double select_ms;            /* device time of all im_select_seeds_from calls  */
    uint32_t sketches_per_pass;  /* sketches sampled per pass over the edge list  */
    uint64_t sketch_bytes;       /* device bytes held by the sketch arrays         */
    uint32_t bulk_rounds;        /* rounds that evaluated every vertex at once
                                    (after a seed that covered a large share of
                                    every sketch): from E with full labels; from
                                    the kept bitmaps, or by re-deriving the
                                    sketches, with CompactSketch                   */
    uint32_t bulk_resampled;     /* of those, CompactSketch rounds that re-derived
                                    the sampled graphs' components (the others
                                    used the largest-component bitmaps)            */
} im_sketch_stats;
im_status im_sketches_stats(const im_sketches *s, im_sketch_stats *out);

/* ---- batched selection ------------------------------------------------------ */

/* One request: graph, probability model, R sketches, k seeds, sampling seed, and
 * the label kind: alpha = 1 (or 0, so that a zeroed struct asks for full labels)
 * for full labels, 0 < alpha < 1 for CompactSketch with that center fraction.
 * Its seeds and gains equal im_build_sketches(graph, prob, R, seed, alpha)
 * followed by im_select_seeds_from(k) -- the same for both label kinds. */
typedef struct {
    const im_graph *graph;
    im_prob prob;
    uint32_t R;
    uint32_t k;
    uint64_t seed;
    double alpha;
} im_query;

/* Launch shapes of the batched kernels (0 = library default).  hook_block and
 * select_block must be multiples of 64 and at most 1024.  Chosen by the
 * project's autotuner (paper_2311_07554_amd/autotune.py). */
typedef struct {
    uint32_t hook_block;    /* threads per block of the sampling + hooking pass      */
    uint32_t hook_grid;     /* blocks of the sampling + hooking pass                 */
    uint32_t select_block;  /* threads of each selection workgroup (one per query)   */
    uint32_t select_grid;   /* selection workgroups (taking queries from a counter)  */
} im_batch_config;

/* Answers nq independent requests together (Algorithm 1 for each).  Full-label
 * queries: all sketch builds run as flattened persistent kernels over every
 * (query, pass, edge) and (query, sketch, vertex), and every query's selection
 * runs in one workgroup of a persistent kernel; these kernels are captured in
 * one hipGraph, kept by the context for the next batch of the same shape, and
 * launched once.  CompactSketch queries (0 < alpha < 1) then run one after
 * another through the single-query build and selection (GetCenter needs the
 * whole GPU per evaluation step).  Each query's seeds and gains equal what it
 * gets alone (see im_query).
 * seeds_out[q] / gains_out[q]: caller-owned host arrays of queries[q].k entries,
 * written only if every query succeeded.  cfg may be NULL.  *device_ms (may be
 * NULL) gets the device time of the whole batch.
 * Errors: EINVAL (a query's k > n, R = 0, bad prob or alpha, per-edge model, bad
 * cfg), ENOMEM, EDEVICE, EINTERNAL. */
im_status im_select_seeds_batched(im_ctx *ctx, uint32_t nq, const im_query *queries, const im_batch_config *cfg,
                                  uint32_t *const *seeds_out, uint64_t *const *gains_out, double *device_ms);

/* ---- serving ---------------------------------------------------------------- */

typedef struct im_server im_server;

typedef struct {
    size_t hbm_budget;         /* bytes for query slots, build scratch, cached sketch sets
                                  and the CompactSketch lane together (0: 64 GiB)        */
    uint32_t max_active;       /* full-label requests selected concurrently
                                  (0: 16, at most 256)                                   */
    uint32_t rounds_per_step;  /* rounds each active request advances per step (0: 16)   */
    uint32_t max_R;            /* largest R accepted (0: 256)                            */
    uint32_t max_k;            /* largest k accepted (0: 1000)                           */
    size_t compact_budget;     /* part of hbm_budget for CompactSketch requests
                                  (0: a quarter of it)                                   */
} im_server_config;

typedef struct {
    uint64_t submitted, completed, steps, builds, cache_hits, evictions;
    uint64_t compact_completed;  /* CompactSketch requests answered by the compact lane */
    size_t bytes_in_use, peak_bytes;
    uint32_t cached_sets;
    double admit_ms;       /* worker time in admission (sketch-set allocation, eviction, build launch) */
    double build_wait_ms;  /* worker time waiting with every admitted request's sketches unbuilt      */
    double step_ms;        /* worker time in selection steps (launch to results on the host)          */
    double busy_steps_ms;  /* device time of the selection steps (HIP events)                         */
} im_server_counters;

/* A request server over resident graphs (Algorithm 1 per request), with
 * continuous batching.  Full-label requests: a worker thread admits them as
 * query slots and HBM free up (sketch sets cached per graph, model thresholds,
 * R and sampling seed; least recently used unreferenced sets evicted under
 * hbm_budget), builds missing sketch sets on its own stream, and advances every
 * admitted request by rounds_per_step rounds per step in one batched launch
 * (requests join and leave between steps).  CompactSketch requests (a query's
 * 0 < alpha < 1): a second worker builds and selects them one at a time on a
 * stream of its own, within compact_budget, while the full-label steps go on
 * (their selection modifies the sketch triple, so their sets are not cached).
 * Each request's seeds and gains equal what its im_query gets alone.  The graphs
 * must stay alive until im_server_destroy.  While a server exists its workers
 * issue work on the context's device; other calls may use the same context. */
im_status im_server_create(im_ctx *ctx, const im_graph *const *graphs, uint32_t ngraphs,
                           const im_server_config *cfg, im_server **out);
/* Queues a request (q->graph one of the server's graphs); *ticket identifies it.
 * EINVAL: bad arguments (unknown graph, R > max_R, k > max_k or > n, bad prob or
 * alpha, per-edge model); EBUSY: its sketch set can never fit the budget. */
im_status im_server_submit(im_server *srv, const im_query *q, uint64_t *ticket);
/* *done = 1 once the request finished (EINVAL for an unknown ticket). */
im_status im_server_poll(im_server *srv, uint64_t ticket, int *done);
/* Blocks until the request finishes, writes its k seeds and gains (caller-owned
 * host arrays) and the time from submit to completion, and retires the ticket.
 * Returns the request's own status (EDEVICE if its sketch build failed on the
 * device; every request waiting on that build fails the same way). */
im_status im_server_wait(im_server *srv, uint64_t ticket, uint32_t *seeds, uint64_t *gains, double *latency_ms);
im_status im_server_stats(im_server *srv, im_server_counters *out);
/* Finishes every queued request, then frees the server. */
im_status im_server_destroy(im_server *srv);

/* ---- device ceilings (roofline) -------------------------------------------- */

/* Measures, on the context's device, (a) the rate of live-edge hash tests the
 * sampling loop's arithmetic reaches with no memory traffic (keys in scalar
 * registers, 64 tests per edge word), in tests per second, and (b) the bandwidth
 * of a streaming 16-byte-per-lane copy of 1 GiB, counting bytes read plus
 * written, in bytes per second.  Allocates 2 GiB for the duration of the call.
 * Errors: ENOMEM, EDEVICE. */
im_status im_probe_device(im_ctx *ctx, double *hash_per_s, double *copy_bytes_per_s);
/* Measures the rate of independent 4-byte reads at pseudo-random places of a
 * 4 GiB buffer (the access pattern of the union-find's parent lookups), in reads
 * per second.  Allocates 4 GiB for the duration of the call.  Errors: ENOMEM,
 * EDEVICE. */
im_status im_probe_random(im_ctx *ctx, double *reads_per_s);

#ifdef __cplusplus
}
#endif

#endif /* PACIM_H */
