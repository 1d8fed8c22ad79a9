// Host-side objects of the library (context, resident graph, query engine).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cstring>
#include <memory>
#include <cstdarg>
#include <cstdint>
#include <deque>
#include <functional>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/flexis.h"
#include "fx_internal.h"
#include "fx_check.h"
#include "fx_pool.h"

fx_status fx_fail(fx_status code, const char *fmt, ...);

#define FX_MAX_LANES 3  // pipeline lanes of an engine (each with its own stream and scratch)

// Runs fn(a, b) over the blocks [a, b) of `grain` indices of [0, n) on the
// calling thread and the library's worker threads (started on first use, at
// most 15, parked until the process ends).  Blocks are handed out through an
// atomic counter, so their order of execution is unspecified.  Callers from
// several threads take turns.  n <= grain runs inline.
void fx_parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)> &fn);

#define FX_HIP(call)                                                                                     \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess) return fx_fail(FX_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define FX_TRY(call)                \
    do {                            \
        fx_status s_ = (call);      \
        if (s_ != FX_OK) return s_; \
    } while (0)

// Number of device and pinned-host allocation calls the library has made
// (every hipMalloc / hipHostMalloc goes through DevBuf, HostBuf or the
// region pool's allocator, which count them).
extern std::atomic<uint64_t> fx_alloc_calls_made;

// Device allocation that remembers its size.  A borrowed buffer points into
// memory the library does not own (the static scratch array of the
// allocation-free entry point): ensure() never allocates for it and fails
// when it is too small, release() never frees it.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool borrowed = false;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release();
    fx_status ensure(size_t want);
    void borrow(void *q, size_t n)
    {
        release();
        p = q;
        bytes = n;
        borrowed = true;
    }
    template <class T>
    T *as() const { return (T *)p; }
};

// Pinned host allocation.
struct HostBuf {
    void *p = nullptr;
    size_t bytes = 0;
    HostBuf() = default;
    HostBuf(const HostBuf &) = delete;
    HostBuf &operator=(const HostBuf &) = delete;
    ~HostBuf() { release(); }
    void release();
    fx_status ensure(size_t want);
    template <class T>
    T *as() const { return (T *)p; }
};

// Tunables of an engine.
struct EngineParams {
    int64_t slice_rows = 1 << 17;          // level capacity of one query's stack
    int64_t count_cap = (int64_t)1 << 62;
    uint64_t step_candidates = 1ull << 25;  // flattened candidates per step, all queries together
    int32_t max_active = 4096;             // queries in flight
    uint32_t last_span_init = 4096;        // complete embeddings per greedy slice (support phase)
    int32_t items = 4;                     // candidates per thread in the expansion kernels (2, 4, 8)
    int32_t lanes = 2;                     // pipeline lanes (1 to FX_MAX_LANES)
    bool timing = false;
    bool no_digest = false;
    bool ref_bytes = false;   // count the reference algorithmic bytes (extra loads: a counting pass)
    bool check_steps = false; // check every step's segment table and tile map on the host (fx_check.h)
    bool fused = false;       // single-pass expansion kernel (else probe, scans, scatter, offset fix-up)
    int32_t fused_below = 64; // ... also for host-scheduled steps of at most this many workgroups
    bool lone_growth = true;  // long VERDICT queries left nearly alone may grow their support stacks
    int32_t chain_queries = 8;    // at most this many queries left (none waiting): device-scheduled steps
    int32_t chain_steps = 16;     // steps per chain (one host synchronisation each)
    int32_t promote_after = 16;   // steps a query has run before its stack may grow
    int32_t lone_queries = 2;     // open queries at or below which VERDICT support stacks grow freely
    int32_t lone_after = 1024;    // ... once the VERDICT query has run this many steps
};

// Buffers of one of the engine's pipeline lanes: what the host writes for a
// lane's step, and the summaries read back after it.
struct EngineLane {
    DevBuf stage_d, inits_d;           // stage: workgroup starts, then the segment table
    DevBuf cand, bcnt, boff, lsum, loff, tmap;  // per-step scratch of the expansion kernels
    DevBuf sstat;                               // block-scan state (scan_state_words of the step's workgroups)
    HostBuf stage_h, inits_h, sums_h;
    hipEvent_t done = nullptr;  // recorded after the lane's summary copy
    hipEvent_t evk[6] = {};     // kernel timing
};

// Device and pinned buffers of one engine (a context's, or a server's).  Lane
// 0 runs on the engine's stream, every other lane on a stream of its own, so
// the lanes' steps overlap on the device; each lane has its own scratch.
// A chain of device-scheduled steps captured in a HIP graph, with what it was
// captured for (the launch shape and every buffer its nodes point at).
struct ChainGraphKey {
    const void *graph;
    FxGraphDev dev;
    int32_t items, width, steps, max_q, fused;
    const void *bufs[9];
    size_t bytes;
    bool operator==(const ChainGraphKey &o) const { return memcmp(this, &o, sizeof(*this)) == 0; }
};

struct EngineWork {
    EngineWork();  // the pool allocates its chunks with hipMalloc
    RegionPool pool;
    DevBuf sums_d;
    EngineLane lane[FX_MAX_LANES];
    hipStream_t own_stream[FX_MAX_LANES - 1] = {};  // lanes 1.. (non-blocking, default priority)
    hipEvent_t start_ev = nullptr;  // orders those lanes after earlier work on the engine's stream
    // device-scheduled steps: control block, chained queries and their
    // segment table (device), their pinned mirror, the stream the captured
    // chain replays on, and the captured chain
    DevBuf chain_d;
    HostBuf chain_h;
    hipStream_t chain_stream = nullptr;
    struct ChainGraph {
        ChainGraphKey key{};
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        uint64_t used = 0;
    };
    static constexpr int kChainGraphs = 6;  // captured chains kept (chain lengths and shapes)
    ChainGraph chain[kChainGraphs];
    uint64_t chain_clock = 0;
    ~EngineWork();
    // Events of every lane, and streams for lanes 1 .. lanes-1 only.  The
    // hardware queues of a process are few (four by default) and streams are
    // mapped onto them in creation order, so a stream that is never used can
    // make two lanes share a queue, which serialises their kernels: the chain
    // stream is created on first use, and an engine with one lane (the
    // allocation-free path) creates none.
    fx_status init_events(int lanes);
    fx_status init_chain_stream();
    // the captured chain for `key`, or a free (least recently used) entry
    // for it after destroying what it held
    ChainGraph &chain_graph(const ChainGraphKey &key);
};

struct fx_ctx {
    int32_t device = 0;
    hipStream_t stream = nullptr;
    int64_t run_index_bytes = (int64_t)8 << 30;  // < 0: no label-run index
    EngineParams params;
    std::atomic<int> graphs{0};
    fx_stats stats{};
    EngineWork work;
    // the allocation-free entry point's engine buffers: device buffers carved
    // from the device's static scratch array, pinned host staging and events
    // made once here (fx_noalloc.hip)
    std::unique_ptr<EngineWork> na_work;
};

// Allocation-free support (fx_noalloc.hip).  fx_noalloc_setup runs once per
// context at creation, with the context's device current: it resolves the
// device address of that device's scratch array (once per device) and builds
// ctx->na_work over it.  fx_noalloc_params: the engine parameters the
// allocation-free path runs with (one query, one lane, a fixed step budget
// and slice capacity, stacks never moved).
fx_status fx_noalloc_setup(fx_ctx *c);
EngineParams fx_noalloc_params(const EngineParams &base);

struct fx_graph {
    fx_ctx *ctx = nullptr;
    std::atomic<int> servers{0};
    int64_t nv = 0, nadj = 0;
    std::vector<int32_t> vl_values, el_values;  // dense id -> caller's label
    std::unordered_map<int32_t, uint32_t> vl_map, el_map;
    std::vector<int64_t> bptr;                  // host copy of the label buckets' offsets
    DevBuf rowp, adj, bucket, bptr_d, runoff, keybits;
    FxGraphDev dev{};
    // directed graphs: each edge u -> v with dense label e is held twice, in
    // u's row with edge code 2e (outgoing) and in v's row with code 2e + 1
    // (incoming), so an edge of either direction is a (label, code) run
    bool directed = false;
};

// Matching plan of one pattern.
struct HostPlan {
    FxPlan plan{};
    bool empty = false;       // a label of the pattern does not occur in the graph
    bool symmetric = false;   // the plan has symmetry-breaking constraints
    int64_t upper_bound = 0;  // support <= min(nv / n, min_l |V_l| / cnt_l)
};

fx_status fx_check_pattern(const fx_pattern *p, bool directed = false);
int32_t fx_query_kind(int32_t mode);  // FX_MODE_* -> FX_Q_*
fx_status fx_build_plan(const fx_graph *G, const fx_pattern *p, HostPlan &hp);
fx_status fx_tau_checked(int64_t sigma, double lambda, int32_t n, int64_t *tau_out);

// One request to the engine.
enum FxQueryKind { FX_Q_FULL = 0, FX_Q_VERDICT = 1, FX_Q_LIST = 2, FX_Q_MNI = 3, FX_Q_MIS = 4 };

struct FxRequest {
    const fx_pattern *pattern = nullptr;
    void *user = nullptr;                // owner's tag (the server's ticket)
    int64_t sigma = 1;
    double lambda = 1.0;
    int32_t kind = FX_Q_FULL;
    fx_result *out = nullptr;            // result (FULL / VERDICT)
    int32_t *selected = nullptr;         // optional selected embeddings (FULL)
    int64_t selected_cap = 0;
    int32_t *list_rows = nullptr;        // listing output (LIST)
    int64_t list_cap = 0;
    int64_t *list_count = nullptr;
    fx_status status = FX_OK;            // per-request validation status
};

struct FxQuery;

// The multi-query engine: requests are added at any time; each step() admits
// pending requests while slots and memory allow, runs one device step for the
// active ones and reports finished requests through on_done.  Queries are
// split into lanes by slot (slot mod lanes), and step() serves the lanes in
// turn: it waits for a lane's previous device step, advances its queries and
// launches its next step while the other lanes' steps run on the device, so
// the host's work between steps is hidden behind device work.
class FxEngine {
public:
    FxEngine(fx_graph *G, EngineWork *W, hipStream_t s, const EngineParams &p, fx_stats *stats);
    ~FxEngine();
    FxEngine(const FxEngine &) = delete;
    FxEngine &operator=(const FxEngine &) = delete;
    // Validates and plans r.  Requests that are decided without device work
    // (invalid, a label absent from the graph, exact upper-bound reject) are
    // finished at once.
    void add(FxRequest *r);
    // add() for a whole batch: plans every request (on the worker threads
    // for a large batch), then queues them in order; if a pattern is
    // invalid, returns the error of the first such request and queues
    // nothing.
    fx_status add_all(FxRequest *reqs, size_t count);
    bool idle() const;
    fx_status step();
    std::function<void(FxRequest *)> on_done;

private:
    std::unique_ptr<FxQuery> prepare(FxRequest *r) const;  // plan and tau; touches no engine state
    void enqueue(std::unique_ptr<FxQuery> q);
    fx_status admit(int g);
    fx_status promote(FxQuery &q, int64_t new_cap);
    fx_status finish(FxQuery &q, const FxSummary &S);
    bool chain_ready() const;
    fx_status chain_step(double &waited);
    fx_status grow_stacks(std::vector<FxQuery *> &qs, uint64_t n_open);
    fx_status collect(int g, double &waited);
    fx_status launch(int g);
    void done(FxRequest *r);
    fx_graph *G_;
    EngineWork *W_;
    hipStream_t s_;
    hipStream_t ls_[FX_MAX_LANES];                                   // each lane's stream
    std::vector<std::pair<void *, size_t>> deferred_[FX_MAX_LANES];  // regions freed once the lane's work passed them
    EngineParams P_;
    fx_stats *stats_;
    std::deque<std::unique_ptr<FxQuery>> pending_;
    std::vector<std::unique_ptr<FxQuery>> active_[FX_MAX_LANES];  // by lane
    std::vector<int> free_slots_[FX_MAX_LANES];
    size_t rot_[FX_MAX_LANES] = {};
    bool in_flight_[FX_MAX_LANES] = {};
    int any_greedy_[FX_MAX_LANES] = {};
    int fused_[FX_MAX_LANES] = {};  // the lane's last step ran the single-pass expansion
    uint64_t nopen_[FX_MAX_LANES] = {};  // queries with candidates left, per lane, at its last launch
    int lane_ = 0;  // the lane the next step() serves
    int32_t chain_k_ = 0;  // steps of the last device-scheduled chain
    std::vector<FxStepSeg> step_view_[FX_MAX_LANES];  // the lane's step in flight, for check_steps
    uint32_t step_blocks_[FX_MAX_LANES] = {};
    std::chrono::steady_clock::time_point t0_;
    bool buffers_ready_ = false;
};

// Runs every request to completion, many at a time (at most max_active in
// flight).  Requests that fail validation get their status set; any device
// error aborts the run.
// chains: device-scheduled chains allowed (batches; a single query's few steps
// run faster host-scheduled: measured 2,291 against 1,810 one-call queries/s).
fx_status fx_engine_run(fx_graph *G, std::vector<FxRequest> &reqs, int32_t max_active, bool chains = true);
// The same over given buffers and parameters.
fx_status fx_engine_run_on(fx_graph *G, EngineWork *W, const EngineParams &p, std::vector<FxRequest> &reqs);
