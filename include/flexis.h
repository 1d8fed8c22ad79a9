/*
 * flexis.h — C ABI of the MI355X (gfx950) support-counting library for
 * FLEXIS-style frequent subgraph mining (Sharma, Reinehr, Mehta, Wu,
 * "FLEXIS: FLExible Frequent Subgraph Mining using Maximal Independent
 * Sets", arXiv 2404.01585).
 *
 * One call answers the paper's metric step for one candidate pattern
 * (Algorithm 5, the matcher loop, and its per-candidate matcher of
 * Section 3.2.2): enumerate the embeddings of a labeled pattern in a
 * labeled data graph, take the greedy maximal independent set (mIS) of
 * those embeddings, and compare its size with the threshold tau of the
 * tau equation (Section 3.1.1).
 *
 * Conventions for every entry point:
 *   - Return value: FX_OK (0) or a negative fx_status.  On error the
 *     outputs are left untouched and fx_last_error() describes the cause.
 *   - Host pointers are only read during the call; the caller keeps
 *     ownership.  Device memory the library needs is allocated by the
 *     library and released by the matching destroy call.
 *   - All device work runs on the stream given in fx_ctx_opts (the
 *     caller's HIP stream, e.g. torch.cuda.current_stream().cuda_stream),
 *     and every call returns only after its results are on the host.
 *   - A context (and the graphs loaded into it) is used by one thread at a
 *     time; the server entry points are the exception and are thread-safe.
 *   - Vertex ids are the caller's ids 0..nv-1.  Labels are any int32 >= 0;
 *     the library maps them to a dense range internally.
 */
#ifndef FLEXIS_H
#define FLEXIS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fx_status;
enum {
    FX_OK = 0,
    FX_EINVAL = -1,   /* bad argument (NULL pointer, sigma <= 0, lambda outside [0,1], ...) */
    FX_EGRAPH = -2,   /* malformed data graph (see fx_graph_desc) */
    FX_EPATTERN = -3, /* malformed pattern (see fx_pattern) */
    FX_ENOMEM = -4,   /* device or host allocation failed */
    FX_EDEVICE = -5,  /* a HIP runtime call failed */
    FX_EBUSY = -6,    /* object still in use (destroy order) */
    FX_ETIMEOUT = -7, /* server wait timed out */
    FX_ELIMIT = -8    /* a size limit was exceeded (pattern > 16 vertices, > 65535 labels, ...) */
};

/* Result modes (Section 3.1.1, early termination at tau). */
enum {
    FX_MODE_FULL = 0,    /* exact support, verdict, embedding count and digest */
    FX_MODE_VERDICT = 1, /* verdict only; the search stops as soon as it is decided */
    FX_MODE_MNI = 2,     /* the minimum-image support of Section 2.4.4 instead of the
                            greedy: support = min over pattern vertices v of the
                            number of distinct data vertices v is mapped to by the
                            embeddings; tau = sigma (lambda is not used: it belongs
                            to the greedy metric); frequent = support >= max(sigma, 1);
                            embedding count and digest as in FULL (every embedding is
                            enumerated, the count cap only caps the reported count) */
    FX_MODE_MIS = 3      /* the exact maximum independent set of Section 2.4.2 (the
                            paper's gold-standard metric, NP-hard: small instances
                            only) instead of the greedy: support = the largest number
                            of pairwise vertex-disjoint embeddings; tau = sigma;
                            frequent = support >= max(sigma, 1); embedding_count =
                            |M| (exact); digest 0; rounds = search nodes.  FX_ELIMIT
                            beyond 4096 embeddings, 256 distinct vertex sets or 2^24
                            search nodes.  fx_support and fx_support_batch only. */
};

#define FX_MAX_PATTERN_VERTICES 16

typedef struct fx_ctx fx_ctx;
typedef struct fx_graph fx_graph;
typedef struct fx_server fx_server;

/* Context options.
 *   device            HIP device ordinal.
 *   hip_stream        hipStream_t to run on; NULL means the null stream.
 *   slice_rows        capacity, in partial embeddings, of each level of a
 *                     pattern's slice stack (0 = default 2^17): one step
 *                     writes at most this many partial embeddings of a level
 *                     (it may probe more candidates when few of them pass).  A
 *                     pattern's stack takes about slice_rows * (4 l + 25)
 *                     bytes per level l.  When few patterns are left, a
 *                     long-running pattern's stack may be moved to a larger
 *                     capacity (up to 2^23 rows, within mem_budget_bytes).
 *   count_cap         saturation cap of the embedding count (0 = 2^62).
 *   mem_budget_bytes  device memory the per-pattern stacks of one batch may
 *                     hold at once (0 = 64 GiB); patterns are admitted while
 *                     their projected stack bytes fit.
 *   run_index_bytes   largest label-run index a graph of this context may
 *                     build (0 = 8 GiB, -1 = none): for every vertex and every
 *                     (vertex label, edge label) pair, the adjacency position
 *                     where that run starts, 4 bytes each (built only for
 *                     graphs with fewer than 2^32 adjacency entries), and one
 *                     presence bit per (vertex, pair).  With it a candidate
 *                     run is one random access instead of two binary searches,
 *                     and the neighbour-label filter reads the smaller bit
 *                     array first.
 *   flags             bitwise or of FX_CTX_KERNEL_TIMING (bracket the kernels of
 *                     every step with HIP events on the context's stream and
 *                     accumulate their durations, see fx_ctx_stats) and
 *                     FX_CTX_NO_DIGEST (below). */
#define FX_CTX_KERNEL_TIMING 1u
/* FX_CTX_NO_DIGEST: FULL mode leaves digest at 0 and may count the embeddings
 * of a pattern whose last vertex is a leaf in closed form (run length minus
 * the already-matched vertices in the run) instead of one by one.  The count
 * is exact either way. */
#define FX_CTX_NO_DIGEST 2u
typedef struct {
    int32_t device;
    void *hip_stream;
    int64_t slice_rows;
    int64_t count_cap;
    int64_t mem_budget_bytes;
    int64_t run_index_bytes;
    uint32_t flags;
} fx_ctx_opts;

fx_status fx_ctx_create(const fx_ctx_opts *opts, fx_ctx **out);
/* Fails with FX_EBUSY while graphs loaded into the context still exist. */
fx_status fx_ctx_destroy(fx_ctx *ctx);

/* Data graph: an undirected simple labeled graph as symmetric CSR (the
 * paper loads its data graphs undirected, Section 4.1; vertex labels as in
 * Section 2.1.4, edge labels as in Section 2.3.4).
 *   num_vertices      nv >= 1.
 *   num_adj           2|E| adjacency entries.
 *   offset_bytes      4 (int32 row_ptr) or 8 (int64 row_ptr).
 *   row_ptr           [nv+1], row_ptr[0] = 0, non-decreasing, row_ptr[nv] = num_adj.
 *   col               [num_adj] int32 neighbour ids; each row strictly ascending,
 *                     no self-loops; (u,v) present iff (v,u) present.
 *   vlabel            [nv] int32 >= 0.
 *   elabel            [num_adj] int32 >= 0, or NULL for all-zero; the label of
 *                     (u,v) must equal the label of (v,u).
 *   on_device         0: the arrays are host memory; 1: device memory.  Either
 *                     way the library validates and builds its own copy, so the
 *                     arrays may be freed after the call.
 *   directed          0: undirected, as above.  1: a directed graph (Section 2.2
 *                     states the problem for labeled, directed graphs): row u
 *                     lists the heads v of the edges u -> v, strictly ascending,
 *                     no self-loops; (u,v) and (v,u) may both be present with
 *                     their own labels; no symmetry is required.  Patterns of a
 *                     directed graph are directed: fx_pattern edge (a, b) is
 *                     a -> b, and an embedding maps it onto a data edge
 *                     f(a) -> f(b) with the same label.
 * Errors: FX_EGRAPH for any violation above, FX_ELIMIT for more than 65535
 * distinct vertex labels, more than 65535 (32767 directed) distinct edge
 * labels or more than 2^31-1 vertices. */
typedef struct {
    int64_t num_vertices;
    int64_t num_adj;
    int32_t offset_bytes;
    const void *row_ptr;
    const int32_t *col;
    const int32_t *vlabel;
    const int32_t *elabel;
    int32_t on_device;
    int32_t directed;
} fx_graph_desc;

fx_status fx_graph_load(fx_ctx *ctx, const fx_graph_desc *desc, fx_graph **out);
fx_status fx_graph_destroy(fx_graph *g);

/* Pattern: a connected simple labeled graph with 1 <= n <= 16 vertices,
 * numbered 0..n-1 as submitted (the numbering fixes the greedy order, see
 * fx_support).  edges holds m pairs (a, b), elabel m labels or NULL for all
 * zero.  For a directed data graph the pair (a, b) is the edge a -> b, (a, b)
 * and (b, a) may both be present, and connected means weakly connected.  The
 * pattern is copied at call time.
 * Errors: FX_EPATTERN (disconnected, loops, repeated edges, bad endpoints),
 * FX_ELIMIT (n > 16). */
typedef struct {
    int32_t n, m;
    const int32_t *vlabel;
    const int32_t *edges;
    const int32_t *elabel;
} fx_pattern;

/* Per-pattern result.
 *   tau               threshold of the tau equation (Section 3.1.1) computed in
 *                     exact integer arithmetic with lambda rounded to parts per
 *                     million; the verdict uses max(tau, 1).
 *   support           FULL: size of the greedy mIS.  VERDICT: tau if frequent, else -1.
 *   frequent          1 iff support >= max(tau, 1).
 *   count_saturated   FULL: 1 iff |M| >= count_cap.
 *   embedding_count   FULL: min(|M|, count_cap).  VERDICT: -1.
 *   digest            FULL and not saturated: (sum mod 2^64, xor) of the
 *                     SplitMix64 hash chain of every embedding tuple (seeds
 *                     0x243f6a8885a308d3 and 0x13198a2e03707344); else 0.
 *   steps             expansion steps executed on the device.
 *   rounds            parallel greedy rounds executed on the device.
 *   device_ms         wall time from the start of the call (fx_support) or of the
 *                     batch (fx_support_batch) until the pattern's result was final.
 *   alg_bytes         algorithmic bytes of the query's expansion kernels (as in
 *                     fx_stats: probe plus scatter).
 *   sel_digest        FULL: (sum mod 2^64, xor) of the same hash chain over the
 *                     selected embeddings (the greedy mIS S).  S in rank order is
 *                     its tuples in lexicographic order, so the set fixes the
 *                     list; the digest identifies S without copying it.  Else 0.
 *   status            FX_OK, or the error of this query alone: fx_server_poll and
 *                     fx_server_wait return that error and also store it here
 *                     (for instance FX_ENOMEM for a query whose slice stack cannot
 *                     fit the memory budget even alone).  Every other call that
 *                     returns an error leaves its results untouched.
 *   exit              how the query ended: FX_EXIT_END (the search ran to its end),
 *                     FX_EXIT_REACHED (VERDICT: support reached tau, Section 3.1.1),
 *                     FX_EXIT_BOUND (VERDICT: the selections still possible --
 *                     at most one per root not yet finished, Section 3.2.2, and
 *                     at most the disjointness bound of Section 3.1.2 -- cannot
 *                     lift the support to tau: exactly infrequent), FX_EXIT_STATIC
 *                     (VERDICT: the disjointness bound alone is below tau, decided
 *                     before any device work), FX_EXIT_EMPTY (a label of the
 *                     pattern does not occur in the graph). */
enum {
    FX_EXIT_END = 0,
    FX_EXIT_REACHED = 1,
    FX_EXIT_BOUND = 2,
    FX_EXIT_STATIC = 3,
    FX_EXIT_EMPTY = 4
};
typedef struct {
    int64_t tau;
    int64_t support;
    int32_t frequent;
    int32_t count_saturated;
    int64_t embedding_count;
    uint64_t digest[2];
    int32_t steps;
    int32_t rounds;
    double device_ms;
    uint64_t alg_bytes;
    uint64_t sel_digest[2];
    int32_t status;
    int32_t exit;
} fx_result;

/* tau of the tau equation (Section 3.1.1):
 *   tau = floor(sigma * ((n-1) * lambda + 1) / n),
 * with lambda rounded to parts per million first.  Errors: FX_EINVAL for
 * sigma < 0, lambda outside [0,1] or n < 1. */
fx_status fx_tau(int64_t sigma, double lambda, int32_t n, int64_t *tau_out);

/* Support of one pattern (Algorithm 5 for a single candidate; Section 3.2.2).
 * Embeddings are the injective, label- and edge-label-preserving maps of
 * Section 2.1.4 (non-induced).  They are ranked lexicographically by
 * (f(0), ..., f(n-1)) and the greedy keeps every embedding that shares no
 * data vertex with an earlier kept one; support is the number kept.
 *   sigma >= 1, 0 <= lambda <= 1, mode FX_MODE_FULL, FX_MODE_VERDICT or
 *   FX_MODE_MNI (then support is the minimum-image count, see above). 
 *   selected (optional, host, [selected_cap * n] int32): FULL mode receives the
 *   first min(support, selected_cap) kept embeddings in rank order. */
fx_status fx_support(fx_graph *g, const fx_pattern *p, int64_t sigma, double lambda, int32_t mode,
                     fx_result *out, int32_t *selected, int64_t selected_cap);

/* All embeddings of a pattern in rank order (Section 2.4, the mapping set M).
 * Writes the first min(|M|, cap) tuples ([cap * n] int32, host) and sets
 * *count_out = |M| (exact, not capped by the context's count_cap). */
fx_status fx_enumerate(fx_graph *g, const fx_pattern *p, int32_t *rows, int64_t cap, int64_t *count_out);

/* A batch of patterns (one mining level, Algorithm 1's candidate set) in one
 * device pass.  Each pattern gets its own sigma[i], lambda[i]; results equal
 * those of fx_support called one by one. */
fx_status fx_support_batch(fx_graph *g, int32_t npat, const fx_pattern *pats, const int64_t *sigma,
                           const double *lambda, int32_t mode, fx_result *out);

/* Accumulated device statistics of a context (since creation or the last
 * reset).  Durations are only collected with FX_CTX_KERNEL_TIMING.
 *   probe_*     the expansion test kernel (one launch per step); for steps
 *               that take the single-pass expansion (the fused and
 *               fused_below tunables), that kernel (test and ordered write)
 *   scatter_*   the ordered write of surviving candidates (one launch per
 *               step, none for steps that take the single-pass expansion,
 *               whose write bytes are still counted here)
 *   greedy_*    the greedy mIS kernels (hash build and rounds)
 *   *_alg_bytes algorithmic bytes: bytes the operation must move at minimum
 *               on this layout (8-byte packed adjacency entries, 4-byte ids),
 *               counted on the device: candidate entries, partial rows and
 *               their run descriptors, every binary-search step of an
 *               adjacency test (8 bytes) and the used-set words read.
 *               Candidates of a slice that were probed but left for a later
 *               step (a slice stops at its row cap) are not counted.
 *   steps, syncs, queries   host-side counts.
 *   reoffered   candidates probed in a slice that stopped at its row cap and
 *               offered again in a later step (wasted probe work).
 *   probed      candidates offered to the probe in all steps.
 *   promotions  stacks moved to a larger slice capacity because few queries
 *               were left to share the device.
 *   host_ms     host time inside the engine's steps, waits excluded.
 *   wait_ms     host time waiting for each step's device work to finish.
 *   exits_reached, exits_bound   VERDICT queries that ended early with
 *               FX_EXIT_REACHED and FX_EXIT_BOUND (see fx_result.exit).
 *   lone_promotions   of the promotions, those that only the rule for VERDICT
 *               queries left nearly alone allowed (see the lone_* tunables of
 *               fx_ctx_set).
 *   *_ref_bytes reference algorithmic bytes, counted only with the ref_bytes
 *               tunable: a per-unit model of what the matching must move, apart
 *               from this implementation's own extras (4-byte ids, 1-byte
 *               labels, 8-byte row offsets): per root candidate 20; per expanded
 *               partial of level l, 4 l + 16 + 6 per neighbour read (the
 *               anchor's label run: rows are label-sorted); per candidate that
 *               reaches its adjacency tests, 4 ceil(log2(r + 1)) for each other
 *               earlier neighbour, r its run length; per row written at level
 *               l + 1, 4 (l + 1) (scatter); per complete embedding read by the
 *               greedy and per selection written, 4 n.
 *   probe_ref_row_bytes   the same model for plain rows: the anchor's whole row
 *               read and r = its degree.
 *   chains, chain_steps   device-scheduled chains run (one host
 *               synchronisation each) and the steps they ran (see the
 *               chain_* tunables of fx_ctx_set); steps, syncs and the launch
 *               counts include them. */
typedef struct {
    uint64_t probe_launches;
    double probe_ms;
    uint64_t probe_alg_bytes;
    uint64_t scatter_launches;
    double scatter_ms;
    uint64_t scatter_alg_bytes;
    uint64_t greedy_launches;
    double greedy_ms;
    uint64_t steps;
    uint64_t syncs;
    uint64_t queries;
    uint64_t reoffered;
    uint64_t promotions;
    double host_ms;
    double wait_ms;
    uint64_t exits_reached;
    uint64_t exits_bound;
    uint64_t lone_promotions;
    uint64_t probe_ref_bytes;
    uint64_t scatter_ref_bytes;
    uint64_t greedy_ref_bytes;
    uint64_t probed;
    uint64_t probe_ref_row_bytes;
    uint64_t chains;
    uint64_t chain_steps;
} fx_stats;

/* Copies the context's statistics into *out; reset != 0 zeroes them after. */
fx_status fx_ctx_stats(fx_ctx *ctx, fx_stats *out, int32_t reset);

/* Tunables of a context's engine, by name (results never depend on them;
 * they set the launch shape and the scheduling of later calls):
 *   slice_rows        level capacity of a pattern's slice stack [64, 2^26]
 *   step_candidates   flattened candidates per device step [2048, 2^31]
 *   items_per_thread  candidates per thread of the expansion kernels: 2, 4, 8
 *   last_span_init    complete embeddings per greedy slice [1, 2^26]
 *   lanes             pipeline lanes, each on its own stream: 1 to 3
 *   max_active        patterns in flight at once [1, 2^20]
 *   promote_after     steps a pattern runs before its stack may grow [0, 2^31)
 *   lone_growth       0/1: long VERDICT patterns left nearly alone may grow
 *                     their support-phase stacks
 *   lone_queries      ... once at most this many patterns are open [0, 2^31)
 *   lone_after        ... and the pattern has run this many steps [0, 2^31)
 *   chain_queries     once no pattern of a batch waits and at most this many
 *                     are in flight, their steps are scheduled on the device: a
 *                     chain of up to chain_steps steps, captured once in a HIP
 *                     graph, runs with one host synchronisation (single-pattern
 *                     calls keep host-scheduled steps) [0 (never), 64]
 *   chain_steps       steps per chain [1, 256]
 *   kernel_timing     0/1: as FX_CTX_KERNEL_TIMING (per-kernel timing needs the
 *                     host-scheduled steps: no chains while it is on)
 *   ref_bytes         0/1: also count the reference algorithmic bytes of
 *                     fx_stats (extra loads in the kernels: a counting pass)
 *   check_steps       0/1: check every step on the host -- its segment table
 *                     before the launch (candidate ranges inside their levels,
 *                     level rows and row caps inside the stacks, workgroups
 *                     inside the step's buffers) and the tile map the device
 *                     built after it; a violation fails the call with
 *                     FX_EDEVICE instead of launching (host-scheduled steps)
 *   fused             0/1: expand with the single-pass kernel (probe, ordered
 *                     write and run-length offsets in one launch, positions
 *                     found by a look-back over the preceding workgroups)
 *                     instead of five launches (probe, block scan, scatter,
 *                     block scan, offset fix-up); default 0 (the ordered
 *                     write waits on every earlier workgroup's probe, so a
 *                     slow tile holds up the writes of all tiles after it)
 *   fused_below       use the single-pass expansion also for host-scheduled
 *                     steps of at most this many workgroups [0, 2^31) (small
 *                     steps: a lone query, a single call); default 64
 *                     (one pattern per call on the 100K-vertex benchmark
 *                     graph: 2,321 to 2,565 patterns/s)
 * fx_autotune sets the first six.  Errors: FX_EINVAL for an unknown name or a
 * value out of range (the context is unchanged). */
fx_status fx_ctx_set(fx_ctx *ctx, const char *key, int64_t value);
fx_status fx_ctx_get(fx_ctx *ctx, const char *key, int64_t *value);

/* Continuous-batching server over a resident graph.  A worker thread with its
 * own HIP stream runs the batched engine; queries submitted from any thread
 * join the next device step as soon as a slot and stack memory are free
 * (admission by projected stack bytes), share every launch with the queries
 * already running, and are answered exactly as fx_support would answer them.
 * VERDICT queries leave as soon as their verdict is decided (Section 3.1.1).
 *   max_active        queries in flight (0 = 4096)
 *   slice_rows        level capacity per query (0 = the context's)
 *   mem_budget_bytes  device memory for in-flight stacks (0 = the context's)
 *   step_candidates   candidates per device step over all queries (0 = 2^25);
 *                     smaller steps lower latency, larger ones raise throughput
 *   flags             0 or FX_CTX_NO_DIGEST
 * fx_result.device_ms of a served query is its latency: submit to result.
 * The graph cannot be destroyed while a server uses it (FX_EBUSY). */
typedef struct {
    int32_t max_active;
    int64_t slice_rows;
    int64_t mem_budget_bytes;
    int64_t step_candidates;
    uint32_t flags;
} fx_server_opts;

fx_status fx_server_create(fx_graph *g, const fx_server_opts *opts, fx_server **out);
/* Thread-safe.  Validates sigma, lambda, mode and the pattern (errors are
 * returned here); the pattern is copied.  *ticket identifies the query. */
fx_status fx_server_submit(fx_server *s, const fx_pattern *p, int64_t sigma, double lambda, int32_t mode,
                           uint64_t *ticket);
/* Thread-safe.  *done = 1 and *out filled (the ticket is then released) once
 * the query is finished, else *done = 0.  FX_EINVAL for an unknown ticket. */
fx_status fx_server_poll(fx_server *s, uint64_t ticket, fx_result *out, int32_t *done);
/* Thread-safe.  Blocks until the query is finished (timeout_us < 0: no limit)
 * and releases the ticket; FX_ETIMEOUT when the limit passes first. */
fx_status fx_server_wait(fx_server *s, uint64_t ticket, int64_t timeout_us, fx_result *out);
/* Engine statistics of the server (steps, syncs, queries). */
fx_status fx_server_stats(fx_server *s, fx_stats *out);
/* Finishes every submitted query, then stops the worker and frees the server. */
fx_status fx_server_destroy(fx_server *s);

/* Autotuner of the batched launch shape.  Times fx_support_batch on the
 * given sample while it walks the tunables one at a time: candidates per
 * thread of the expansion kernels (2, 4, 8: the workgroup tile), candidates
 * per device step, the level capacity of a pattern's slice stack (the frontier
 * chunk), the complete embeddings per greedy slice (last_span_init), the
 * number of pipeline lanes (1: one device step at a time; 2 or 3: lanes on
 * their own streams, the host preparing one lane's step while the others'
 * run) and the patterns in flight at once.  The fastest setting is kept in the
 * context (later calls use it; results never depend on it).
 * cache_path (optional): a text file of tuned keys (architecture, graph shape,
 * largest pattern, mode); a cached key is applied without timing. */
typedef struct {
    int64_t slice_rows;
    int64_t step_candidates;
    int32_t items_per_thread;
    int32_t last_span_init;
    double best_ms;     /* sample time with the chosen setting */
    double default_ms;  /* sample time with the context's setting before tuning */
    int32_t trials;
    int32_t from_cache;
    int32_t lanes;
    int32_t max_active;
} fx_tune_result;

fx_status fx_autotune(fx_graph *g, int32_t npat, const fx_pattern *pats, const int64_t *sigma, const double *lambda,
                      int32_t mode, const char *cache_path, fx_tune_result *out);

/* Allocation-free variant of fx_support, for callers that cannot allocate
 * device memory during a call: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.  Same arguments and results as
 * fx_support without the selected list (modes FULL, VERDICT, MNI).  It makes
 * no device or pinned-host allocation (no hipMalloc, hipFree, hipHostMalloc
 * or allocating library routine): its device buffers -- per-step scratch, the
 * query's counters and its slice stack with the used-vertex bitmap -- live in
 * a static device array of FX_NOALLOC_SCRATCH_BYTES per GPU, held until the
 * process ends; its pinned staging and events are made by fx_ctx_create.  It
 * runs one query at a time with a stack capacity of 2^14 partial embeddings
 * per level and 2^22 candidates per device step (results never depend on
 * either).  Every call on a GPU shares that GPU's array: calls that overlap
 * on one GPU race.  Errors as fx_support, plus FX_ELIMIT when the query's
 * stack (about 2^14 * sum over levels l of (4 l + 21) bytes, plus |V| / 8
 * bytes of used-vertex bitmap, times (1 + n) bitmaps in MNI mode) does not
 * fit the array. */
#define FX_NOALLOC_SCRATCH_BYTES (64ull << 20)
fx_status fx_support_noalloc(fx_graph *g, const fx_pattern *p, int64_t sigma, double lambda, int32_t mode,
                             fx_result *out);

/* Device and pinned-host allocation calls the library has made so far in
 * this process (a check that a call allocated nothing). */
uint64_t fx_alloc_calls(void);

/* Thread-local description of the last error. */
const char *fx_last_error(void);

/* Library version string. */
const char *fx_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FLEXIS_H */
