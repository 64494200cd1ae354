/*
 * trim.h -- C ABI of libtrim, parallel graph trimming on one MI355X (gfx950).
 *
 * Graph trimming (Def. Trimmed Graph, Section 2 of "Efficient Parallel Graph
 * Trimming by Arc-Consistency", arXiv 2107.12720) removes, until a fixed
 * point, every vertex that has no live successor.  The result is the greatest
 * vertex set in which every vertex keeps a successor inside the set.  Three
 * algorithms compute it:
 *
 *   TRIM_AC6  the AC-6-based algorithm (Section 6, Alg. par-ac-6-trim): each
 *             live vertex keeps one support, the first live successor found
 *             from its cursor; a removed vertex hands back only the vertices
 *             it supported.  Each edge is examined at most once.
 *   TRIM_AC4  the AC-4-based algorithm (Section 5, Alg. par-ac4trim): live
 *             out-degree counters, decremented over the transposed graph.
 *             Counters start from CSR offsets (AC4Trim*, Section 9.3).
 *   TRIM_AC3  the AC-3-based algorithm (Section 4, Alg. TraditionalTrim):
 *             repeated sweeps with the edge_index cursor of Section 8.  A
 *             sweep reads the statuses of its start (one sweep = one round),
 *             so the round count is alpha + 1 (Def. of alpha, Section 2.4).
 *
 * Conventions for every call:
 *  - Pointers marked (device) are device memory owned by the caller.  The
 *    library never frees or keeps them beyond the call's stream work.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  Calls
 *    only enqueue work on it and return; results are valid after the caller
 *    synchronises the stream.
 *  - Every call returns a trim_status_t.  Argument errors are detected on the
 *    host before anything is enqueued; trim_last_error() then returns a
 *    message for the calling thread.  Nothing aborts or throws across the ABI.
 *  - Outputs: live_bitmap has ceil(n/32) uint32 words; bit (v % 32) of word
 *    v / 32 is set iff v is LIVE.  Bits at positions >= n in the last word are
 *    zero.  worker_edges[p] receives the successor checks made by worker p
 *    (Section 9.3 counts traversed edges per worker); only their sum is a
 *    deterministic quantity.  All outputs are overwritten, never accumulated.
 *  - A trim_ctx owns the call's working memory and must not be used by two
 *    host threads or on two streams at the same time.
 */
#ifndef TRIM_H
#define TRIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TRIM_ABI_VERSION 3

typedef enum { TRIM_AC3 = 3, TRIM_AC4 = 4, TRIM_AC6 = 6 } trim_algo_t;

typedef enum {
    TRIM_OK = 0,
    TRIM_E_INVAL = -1,        /* bad argument (null pointer, size out of range) */
    TRIM_E_NOMEM = -2,        /* device working memory could not be allocated */
    TRIM_E_HIP = -3,          /* a HIP runtime call failed */
    TRIM_E_UNSUPPORTED = -4,  /* e.g. AC-4 on an implicit graph (no G^T) */
    TRIM_E_BADGRAPH = -5,     /* validate=1 found non-monotone offsets or bad targets */
    TRIM_E_STALLED = -6       /* a persistent kernel exceeded its step budget (watchdog):
                                 the call was abandoned and its outputs are invalid */
} trim_status_t;

typedef struct trim_ctx trim_ctx;

/* Explicit graph G = (V, E) in CSR (Section 2.1), plus G^T for AC-4. */
typedef struct {
    int32_t n;                /* vertices, 0 <= n <= 2^29 */
    int64_t m;                /* edges, == row_off[n], 0 <= m < 2^31 */
    const int32_t *row_off;   /* (device) n+1 non-decreasing offsets, row_off[0] == 0 */
    const int32_t *col;       /* (device) m targets in [0, n); successor order = array order */
    const int32_t *rrow_off;  /* (device) G^T offsets, n+1; AC-4 and two-sided only */
    const int32_t *rcol;      /* (device) G^T sources, m; AC-4 and two-sided only */
} trim_csr_t;

/*
 * Implicit graph G = (V, POST) (Section 2.1, on-the-fly property Section
 * 1.3): successors are computed when needed, nothing is stored.  With
 * fin() the SplitMix64 finalizer, n = 2^log2n:
 *   deg(v) = 0                              if fin(seed ^ TZ ^ (v<<8)) < zero_thr
 *          = 1 + #{j < 255 : fin(seed ^ TD ^ (v<<8)) >= deg_table[j]}   otherwise
 *   POST(v)[i] = fin(seed ^ TN ^ ((v<<8) | i)) & (n-1),   0 <= i < deg(v)
 * with TZ = 0x5A45524F00000000, TD = 0x4445470000000000,
 * TN = 0x4E42520000000000.  deg_table holds inverse-CDF thresholds, so
 * deg(v) <= 256.
 */
typedef struct {
    int32_t log2n;              /* 1 .. 29 */
    uint64_t seed;
    uint64_t zero_thr;
    const uint64_t *deg_table;  /* (device) 256 non-decreasing thresholds */
} trim_implicit_t;

/* Launch options; zero-initialise for defaults. */
typedef struct {
    int32_t block;      /* threads per workgroup of the sweep kernels (64..1024, 0 = 256) */
    int32_t workers;    /* persistent workgroups P (0 = sized from occupancy) */
    int32_t chunk;      /* AC-6: vertices claimed per dynamic work chunk of the first
                           sweep (Section 8, schedule(dynamic, s)); rounded up to a
                           multiple of block; 0 = automatic: 4096, or less for graphs
                           with fewer than 4096 * 4 vertices per CU (at least 256) */
    int32_t validate;   /* 1 = check offsets/targets on the device first (synchronises) */
    int32_t graph;      /* trim_batch only: 1 = capture the launch sequence into a HIP
                           graph on the first call and replay it while every argument
                           is unchanged (needs a non-NULL stream) */
    int32_t schedule;   /* schedule perturbation for race testing, bit flags:
                           TRIM_SCHED_REVERSE = the first sweep claims its chunks from
                           the last vertex down; TRIM_SCHED_JITTER = short
                           pseudo-random pauses inside the race windows (join versus
                           close, AC-4 decrements).  Results never depend on them. */
    int32_t budget;     /* watchdog: loop iterations a wavefront of a persistent kernel
                           (AC-6 and AC-4 propagation) may make, and polls a workgroup may
                           spend waiting at an AC-3 round barrier, before the call is
                           abandoned: every wavefront then exits normally, the outputs
                           are invalid and trim_ctx_status() returns TRIM_E_STALLED.
                           0 = TRIM_DEFAULT_BUDGET (a run that legitimately needs more
                           than that is longer than any workload here by over 10x). */
    int32_t flags;      /* TRIM_FLAG_* bits (0 = defaults) */
    int32_t rounds;     /* AC-6 on trim_csr and trim_implicit: register supports late
                           (see below).  0 or 1 = the plain algorithm;
                           2 .. TRIM_MAX_ROUNDS = R rounds; other calls and algorithms
                           take 0 or 1 only (TRIM_E_INVAL otherwise). */
} trim_opts_t;

/*
 * Late support registration (opts.rounds = R >= 2, AC-6 only).  On a shallow
 * graph (small alpha) most vertices keep the first successor they find, and
 * the supporting sets (Section 6.1) they join are never handed back: their
 * registration is the largest cost of the first sweep.  With R >= 2 the first
 * R - 1 repetitions are instead rounds of the AC-3-based algorithm with the
 * edge_index cursor (Sections 4.1 and 8), statuses read as they were at the
 * start of each round, and vertices without successors removed before round
 * 1 (as in the plain first sweep), so a vertex of peeling level l >= 2 goes
 * in round l - 1.  If a round removes nothing, that is the fixed point and
 * the call ends.  Otherwise round R re-checks every cursor the same way and
 * registers each vertex still live in the supporting set of the successor it
 * stops at, and the AC-6 propagation finishes from there.  The live set is
 * the same as without it.  Traversed edges count every cursor re-check:
 *   edges_total = sum_{dead, deg > 0} (deg + min(R, level - 1) - 1)
 *               + sum_live (fl + K),   K = min(R, max(alpha, 1)),
 * and stats.rechecks (the entries of the round lists from round 2 on) is the
 * excess over the plain AC-6 total, so edges_total - rechecks = T6.
 * stats.rounds = rounds run = K.  Working memory: 8 more bytes per vertex
 * (the round list), allocated on the first such call.
 */
#define TRIM_MAX_ROUNDS 64

/*
 * AC-6 (trim_csr, trim_csr_preset, trim_implicit, trim_batch,
 * trim_csr_noalloc): after the first sweep, a vertex whose support is its last
 * successor is removed exactly when that support is, so these links form a
 * forest whose trees fall with their roots.  By default (explicit graphs)
 * every tree whose root the first sweep already removed is taken out at once,
 * by pointer jumping in O(log depth) rounds, before the propagation starts;
 * the successor checks are the same.  TRIM_FLAG_STEPWISE instead propagates
 * those removals one at a time through the support lists, as the paper's
 * waiting sets do.  trim_implicit propagates stepwise unless TRIM_FLAG_FOREST
 * is given: the jump visits every tree member, also those under a root that
 * stays, which on a wide, shallow forest costs more than it saves (on the
 * 2^28-vertex hashed graph: 7.4 ms of jumping to save 3.3 ms of phases).
 * Deep, narrow trees (long chains) are what the collapse is for.
 */
#define TRIM_FLAG_STEPWISE 1
/* trim_implicit: collapse the forest (see above); ignored with STEPWISE. */
#define TRIM_FLAG_FOREST 4
/* trim_batch: trim the batch as one disjoint union (device-wide kernels)
 * instead of one workgroup per graph. */
#define TRIM_FLAG_BATCH_UNION 2

#define TRIM_DEFAULT_BUDGET (1 << 22)

#define TRIM_SCHED_REVERSE 1
#define TRIM_SCHED_JITTER 2

/* Per-call statistics, written to device memory. */
typedef struct {
    uint64_t edges_total;  /* sum of worker_edges: successor checks (AC-6, AC-3) or
                              reverse edges traversed (AC-4) */
    uint64_t n_live;       /* popcount of the live bitmap */
    uint64_t n_dead;       /* vertices removed */
    uint64_t rounds;       /* AC-3: sweeps run (alpha + 1); AC-6 with opts.rounds >= 2:
                              rounds run (see above); 0 otherwise */
    uint64_t queued;       /* AC-6/AC-4: work items that went through the shared queue */
    uint64_t edges_sweep;  /* AC-6: successor checks made by the first sweep */
    uint64_t closes;       /* AC-6: removed vertices whose support lists the propagation
                              closed (the forest collapse counts in `forest`) */
    uint64_t joins;        /* AC-6: support-list joins after the first sweep */
    uint64_t visited;      /* AC-6: support-list members handed back */
    uint64_t graph_edges;  /* AC-6: sum of out-degrees as generated or read (m) */
    uint64_t q_highwater;  /* AC-6/AC-4: largest number of items any wavefront's private
                              LDS queue held (the analogue of the bound on |Q_p| in
                              Section 9.2; capped by the 1,024-entry ring, beyond which
                              items go to the shared queue) */
    uint64_t edges_live;   /* two-sided AC-6: checks made by the vertices that stay live,
                              read off their final cursors (sum over live v of
                              fl_out(v) + 1 + fl_in(v) + 1, schedule independent); 0 for
                              the other calls */
    uint64_t stalled;      /* 1 if the watchdog abandoned the call (see opts.budget) */
    uint64_t forest;       /* AC-6: vertices removed by the forest collapse after the first
                              sweep (the vertices it left without a live successor, plus the
                              members of their last-successor trees); 0 with
                              TRIM_FLAG_STEPWISE */
    uint64_t jump_rounds;  /* AC-6: pointer-jumping rounds the forest collapse ran */
    uint64_t work_items;   /* AC-6: list entries the forest-collapse rounds processed;
                              AC-3: live-list entries processed over all rounds */
    uint64_t phases;       /* AC-6: level-synchronous phases of the propagation before its
                              asynchronous tail */
    uint64_t rechecks;     /* AC-6 with opts.rounds >= 2: cursor re-checks of rounds 2 ..
                              (counted in edges_total; edges_total - rechecks is the plain
                              AC-6 total); 0 otherwise */
} trim_stats_t;   /* 18 words */

/*
 * Per-kernel timing (for benchmarks).  With trim_ctx_set_timing(ctx, k),
 * 1 <= k <= 64, every later launch sequence on `ctx` records HIP events around
 * each of its kernels on the call's stream, and the events of the last k calls
 * are kept (k = 0 turns timing off; other values are TRIM_E_INVAL).  Calls
 * made under HIP graph capture, and the many-launch calls (trim_scc), record
 * nothing.  trim_ctx_kernel_times waits for the last call to finish and writes
 * up to `max` entries, the kept calls in call order and each call's kernels in
 * launch order: names[i] (a static string) and ms[i] (elapsed milliseconds).
 * Returns the number of entries written.  Reading does not wait for anything
 * before it, so a loop of up to k calls runs without host synchronisation and
 * is read once at its end.
 */
int trim_ctx_set_timing(trim_ctx *ctx, int enable);
int trim_ctx_kernel_times(trim_ctx *ctx, int max, const char **names, float *ms);

int trim_version(void);

/* Message of the last failed call on this host thread ("" if none). */
const char *trim_last_error(void);

/*
 * Create a context bound to HIP device `device`.  *out is NULL on failure.
 * mem_budget caps the device memory the context may hold (its control block
 * of about 1.1 MB included), in bytes; 0 = no cap.  A call whose working
 * memory would exceed the cap returns TRIM_E_NOMEM before enqueuing anything,
 * as does trim_ctx_create if the cap is below the control block.
 */
int trim_ctx_create(trim_ctx **out, int device, uint64_t mem_budget);
/* Device memory the context holds now, in bytes (working memory grows to the
 * largest graph seen and is kept for later calls). */
int trim_ctx_mem_used(trim_ctx *ctx, uint64_t *bytes);
/* Free a context and its working memory (NULL is ignored). */
int trim_ctx_destroy(trim_ctx *ctx);

/* Number of workers P for `algo` with `opts` (NULL = defaults); size of worker_edges.
 * opts.workers above trim_max_workers() is TRIM_E_INVAL here and in every call. */
int trim_num_workers(trim_ctx *ctx, int algo, const trim_opts_t *opts, int32_t *P);

/*
 * Largest opts.workers for `algo`: the persistent and cooperative kernels need
 * every workgroup resident at once.  AC-6 and AC-4: the occupancy limit
 * (resident workgroups per CU times CUs).  AC-3: two workgroups per CU (its
 * cooperative rounds kernel is not run at full occupancy; the round barrier
 * needs every workgroup resident, which the launch at the occupancy maximum
 * did not give).
 */
int trim_max_workers(trim_ctx *ctx, int algo, int32_t *P);

/*
 * Wait for the work enqueued on `stream` and report the watchdog of the last
 * trimming call made on `ctx`: TRIM_E_STALLED if a persistent kernel exceeded
 * its step budget (opts.budget), TRIM_OK otherwise, TRIM_E_HIP if the stream
 * reported an error.  The context stays usable after a stall: the next call
 * starts from a clean state.
 */
int trim_ctx_status(trim_ctx *ctx, void *stream);

/*
 * Trim an explicit graph with `algo`.  Output live_bitmap (device,
 * ceil(n/32) words), worker_edges (device, P entries from trim_num_workers),
 * stats (device, may be NULL).  AC-4 needs g->rrow_off and g->rcol
 * (TRIM_E_INVAL without them).  Self-loops keep their vertex; duplicate edges
 * are allowed and counted as separate edges.
 */
int trim_csr(trim_ctx *ctx, int algo, const trim_csr_t *g, const trim_opts_t *opts,
             uint32_t *live_bitmap, uint64_t *worker_edges, trim_stats_t *stats, void *stream);

/*
 * Trimming with some vertices removed before it starts: the vertex sampling
 * of the scalability experiments (Section 9), where unsampled vertices are set
 * to DEAD.  As trim_csr, plus preset_dead (device, ceil(n/32) words, the
 * live_bitmap layout; bits at positions >= n are ignored): a set bit removes
 * that vertex from the start.  The live set is the trimmed graph of the
 * subgraph the other vertices induce.  Preset vertices make no checks of
 * their own; a preset successor is passed like any removed one.  Totals:
 * AC-6 sum over vertices removed by trimming of deg + sum over live v of
 * (fl(v) + 1); AC-4 sum over every removed vertex, preset ones included, of
 * its in-degree (their removal is propagated); AC-3 as for trim_csr over the
 * vertices removed by trimming, alpha counting their peeling steps only.
 * stats.n_dead includes the preset vertices.  preset_dead may be NULL only
 * when n == 0 (TRIM_E_INVAL otherwise).
 */
int trim_csr_preset(trim_ctx *ctx, int algo, const trim_csr_t *g, const uint32_t *preset_dead,
                    const trim_opts_t *opts, uint32_t *live_bitmap, uint64_t *worker_edges,
                    trim_stats_t *stats, void *stream);

/*
 * Two-sided trimming of an explicit graph: the first improvement of Section
 * 4.1 for implementations that hold G^T, where a vertex must also keep a
 * live predecessor (its in-degree is checked too).  The result is the
 * greatest vertex set in which every vertex has a successor and a predecessor
 * inside the set, i.e. the vertices that reach a cycle and are reached from
 * one (a self-loop counts as a cycle).
 *   TRIM_AC6  every vertex keeps one support per side (a live successor and
 *             a live predecessor), each found by the AC-6 support search
 *             over its list in G or in G^T; a removed vertex hands back the
 *             vertices it supported on either side.  worker_edges count
 *             neighbour checks on both sides; their sum depends on the
 *             schedule for removed vertices only.
 *   TRIM_AC4  two counters per vertex (live successors, live predecessors),
 *             both from offsets; every removed vertex walks its predecessor
 *             and successor lists once, so the sum of worker_edges is
 *             sum over removed v of (out-degree + in-degree).
 *   TRIM_AC3  rounds with two edge_index cursors per vertex, one over G and
 *             one over G^T, reading the statuses of the round's start: in
 *             a round a vertex checks its successor cursor first and, only
 *             if a successor is left, its predecessor cursor.  Round r
 *             removes exactly the vertices of two-sided peeling step r, so
 *             stats.rounds = alpha + 1 and the sum of worker_edges is fixed
 *             (every check of a neighbour counts).  Uses the same extra
 *             context memory as AC-6.
 * g->rrow_off and g->rcol are required (TRIM_E_INVAL without them) and must
 * hold the transpose of (row_off, col); the in-side scans follow rcol's order.
 * opts.validate checks ranges and offsets of both, not that they are
 * transposes of each other.  Outputs as for trim_csr, with worker_edges
 * sized by trim_num_workers for the same algo.  Stats: closes + forest (AC-6)
 * count the vertices removed after the start, i.e. those that had a
 * successor and a predecessor; forest those the forest collapse removed (as
 * for the one-sided call, over the out-side last-successor links; 0 with
 * TRIM_FLAG_STEPWISE); n_dead all removed vertices.  AC-6 and AC-3 use 48
 * bytes per vertex of context memory beyond trim_csr (in-side lists and
 * records, a larger queue), 60 for graphs of up to 2^25 vertices (whose
 * out-side S_more lists are split as in the one-sided call), allocated on
 * the first call of either.
 */
int trim_csr_two_sided(trim_ctx *ctx, int algo, const trim_csr_t *g, const trim_opts_t *opts,
                       uint32_t *live_bitmap, uint64_t *worker_edges, trim_stats_t *stats,
                       void *stream);

/* Counts of one SCC decomposition (host memory). */
typedef struct {
    int64_t n_scc;         /* strongly connected components */
    int64_t trimmed;       /* vertices found as size-1 components by trimming */
    int64_t giant;         /* size of the pivot's component (forward-backward search) */
    int32_t trims;         /* two-sided trimming passes */
    int32_t color_rounds;  /* colouring rounds after the forward-backward search */
    int32_t color_sweeps;  /* max-label sweeps over all colouring rounds */
    int32_t search_levels; /* frontier levels of all searches */
    int64_t search_edges;  /* list entries examined by the forward and backward searches */
    int64_t search_ors;    /* mark fetch-ors the searches issued (a measure of contention:
                              at most 2 per vertex win) */
    double trim_ms;        /* host-timed phases: trimming passes, */
    double search_ms;      /* the pivot's forward-backward search, */
    double color_ms;       /* colouring rounds (without their trimming) */
    int64_t paired;        /* vertices found in components of two by the size-2 check */
    double size2_ms;       /* host-timed size-2 check */
} trim_scc_stats_t;

/*
 * Strongly connected components by forward-backward search with trimming,
 * the application of graph trimming in Section 1.1: two-sided trimming (as
 * trim_csr_two_sided with AC-6) takes out the size-1 components, a forward
 * and backward search from one pivot (the vertex with the largest
 * (outdeg+1)(indeg+1)) takes out its component, trimming runs again, and
 * colouring rounds (each unassigned vertex takes the largest id that reaches
 * it; a vertex keeping its own id is a root whose component is the vertices
 * of its colour that reach it) take out the rest, with trimming after each
 * round.  Between the search and the colouring, the size-2 check of
 * trim_size2 takes out components of two.  g->rrow_off and g->rcol are
 * required and must hold the transpose.
 * Output: label (device, n int32): label[v] is the id of one vertex of v's
 * component, so u and v share a component iff label[u] == label[v], and
 * label[label[v]] == label[v].  stats (host, may be NULL) receives the
 * counts.  The rounds and search levels are driven from the host: the call
 * synchronises `stream` once per level and returns when the labels are final.
 * Uses 96 bytes per vertex of context memory (the two-sided trimming arrays,
 * SCC marks and colours, two search frontiers and their prefix sums), 108
 * for graphs of up to 2^25 vertices (see trim_csr_two_sided).
 * TRIM_E_STALLED if a round made no progress (a guard; the method always
 * progresses).
 */
int trim_scc(trim_ctx *ctx, const trim_csr_t *g, const trim_opts_t *opts, int32_t *label,
             trim_scc_stats_t *stats, void *stream);

/*
 * Size-2 SCC trimming, the pattern check that follows size-1 trimming
 * (Section 1.1; the paper gives no algorithm, this is the check used here):
 * among the vertices not set in preset_dead (device bitmap as in
 * trim_csr_preset; NULL = none removed), u and v != u form a component of
 * two when each is the other's only remaining predecessor (nothing else
 * reaches them) or each is the other's only remaining successor (they reach
 * nothing else); a self-loop rules its vertex out.  Output partner (device,
 * n int32): the other vertex for paired vertices, -1 for all others
 * (including removed ones).  n_paired (host, may be NULL) receives the
 * number of paired vertices; passing it synchronises `stream`.  g->rrow_off
 * and g->rcol are required.  trim_scc runs this check once, after the
 * forward-backward search and the trimming that follows it.
 */
int trim_size2(trim_ctx *ctx, const trim_csr_t *g, const uint32_t *preset_dead, int32_t *partner,
               int64_t *n_paired, void *stream);

/*
 * Trim an implicit graph (AC-6 or AC-3 only; AC-4 needs G^T and returns
 * TRIM_E_UNSUPPORTED, Table trim: AC-4 lacks the on-the-fly property).
 * Outputs as for trim_csr with n = 2^log2n.
 */
int trim_implicit(trim_ctx *ctx, int algo, const trim_implicit_t *g, const trim_opts_t *opts,
                  uint32_t *live_bitmap, uint64_t *worker_edges, trim_stats_t *stats,
                  void *stream);

/*
 * AC-6 on G independent graphs packed into one CSR, in one launch sequence.
 * By default each graph is trimmed whole by one workgroup (graphs claimed
 * largest first; a graph's phases end at workgroup barriers, so graphs never
 * wait for each other), which suits many small and mid-sized graphs.  With
 * TRIM_FLAG_BATCH_UNION in opts.flags the batch is trimmed as one disjoint
 * union by the device-wide kernels of trim_csr, which suits a few large
 * graphs.  Both give the same bitmaps and per-graph totals.
 * Graph g owns vertices [vbase[g], vbase[g+1]) and their out-edges;
 * row_off (device, vbase[G]+1 entries) is absolute into col; col (device)
 * holds graph-local target ids in [0, vbase[g+1]-vbase[g]).  vbase and
 * bitmap_base are device int64 arrays of G+1 entries; graph g's bitmap starts
 * at word bitmap_base[g] of live_bitmaps and covers its n_g vertices
 * (bitmap_base[g+1] - bitmap_base[g] >= ceil(n_g/32)).  graph_edges (device,
 * G entries) receives each graph's successor checks.  total_n = vbase[G] and
 * total_m = row_off[total_n] are passed by value.
 */
int trim_batch(trim_ctx *ctx, int32_t G, const int64_t *vbase, const int32_t *row_off,
               const int32_t *col, int64_t total_n, int64_t total_m, const int64_t *bitmap_base,
               const trim_opts_t *opts, uint32_t *live_bitmaps, uint64_t *graph_edges,
               trim_stats_t *stats, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc): AC-6 on an
 * explicit graph exactly as trim_csr with TRIM_AC6, with no context and no
 * allocation of any kind.  The working memory is a fixed array inside the
 * library, one copy per GPU (about 69 MB, held until the process ends), on
 * the calling thread's current device.  The caller passes inputs and outputs
 * as for trim_csr; worker_edges needs opts.workers entries, or
 * TRIM_NOALLOC_WORKERS when opts.workers is 0.  g->rrow_off / g->rcol are
 * ignored.  TRIM_E_INVAL for n > TRIM_NOALLOC_MAX_N, opts.workers >
 * TRIM_NOALLOC_WORKERS, opts.graph != 0 or opts.rounds > 1 (late support
 * registration needs a round list it would have to allocate).  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (two streams, two threads) race
 * and must be serialised by the caller.  The watchdog (opts.budget) works as
 * for trim_csr; a stall shows in stats.stalled (no context to query).
 */
#define TRIM_NOALLOC_MAX_N (1 << 20)
#define TRIM_NOALLOC_WORKERS 512
int trim_csr_noalloc(const trim_csr_t *g, const trim_opts_t *opts, uint32_t *live_bitmap,
                     uint64_t *worker_edges, trim_stats_t *stats, void *stream);

/*
 * Learned successor order (AC-6 checks successors in list order; a live
 * vertex costs the index of its first live successor + 1 checks, Section 6.1
 * and the edge_index of Section 8).  A small network scores each edge u -> w
 * by how likely w is to stay live, and each successor list is reordered by
 * the score; this changes the traversed edges, never the live set.
 * Parameters: 1,377 values in this order -- W1[32][8], b1[32], W2[32][32]
 * (W2[out][in]), b2[32], w3[32], b3 -- as FP32 masters and BF16 copies
 * (uint16 bit patterns).  All arrays are device memory owned by the caller.
 */
#define TRIM_MLP_PARAMS 1377

/* indeg[v] (n entries) and src[e] (m entries: the source of edge e). */
int trim_mlp_prepare(trim_ctx *ctx, const trim_csr_t *g, int32_t *indeg, int32_t *src,
                     void *stream);

/*
 * Gradient of the mean binary cross-entropy "w is live" (labels: live_bitmap,
 * the trimmed set) over `count` sampled edges; edges with a non-live source
 * weigh 0.  Edges are edge_ids[0..count) if edge_ids is non-NULL, else hashed
 * samples of (seed, step).  Accumulates into grad[0..1376] and the loss into
 * grad[1377] (FP32, 1378 entries).
 */
int trim_mlp_grad(trim_ctx *ctx, const trim_csr_t *g, const int32_t *indeg, const int32_t *src,
                  const uint32_t *live_bitmap, const uint16_t *params_bf16,
                  const int64_t *edge_ids, int64_t count, uint64_t seed, int32_t step,
                  float *grad, void *stream);

/* One Adam step (step >= 1) on params; refreshes params_bf16 and clears grad. */
int trim_mlp_adam(trim_ctx *ctx, float *params, uint16_t *params_bf16, float *adam_m,
                  float *adam_v, float *grad, float lr, float beta1, float beta2, float eps,
                  int32_t step, void *stream);

/* scores[e] = the network's logit that the target of edge e stays live (its
 * probability is 1 / (1 + exp(-logit))) (m entries, CSR order).  Per-vertex features are first
 * tabulated in context memory (8 bytes per vertex, kept for later calls). */
int trim_mlp_score(trim_ctx *ctx, const trim_csr_t *g, const int32_t *indeg, const int32_t *src,
                   const uint16_t *params_bf16, float *scores, void *stream);

/* Reference orders: kind 0 keys[e] = log1p(outdeg(target)), kind 1 a hash of (seed, e). */
int trim_edge_keys(trim_ctx *ctx, const trim_csr_t *g, int32_t kind, uint64_t seed, float *keys,
                   void *stream);

/*
 * col_out = each successor list reordered by keys, larger first, in 16 equal
 * levels between lo and hi (clamped), stable within a level.  col_out (m
 * entries) must not alias g->col; row offsets are unchanged.
 */
int trim_order_by_key(trim_ctx *ctx, const trim_csr_t *g, const float *keys, float lo, float hi,
                      int32_t *col_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* TRIM_H */
