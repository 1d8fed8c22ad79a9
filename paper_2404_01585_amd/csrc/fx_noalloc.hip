// Allocation-free support query (fx_support_noalloc).
//
// For callers that cannot allocate device memory during a call (code under
// HIP graph capture, tight serving loops, harnesses that forbid it).  Every
// device buffer the engine needs for one query -- the per-step scratch of the
// expansion kernels, the query's summary, the staged segment table and the
// query's slice stack with its used-vertex bitmap -- is carved from one
// file-scope device array, `scratch`, of FX_NOALLOC_SCRATCH_BYTES.  Each GPU
// the library runs on holds its own copy of the array until the process ends.
//
// The array's name is a host-side stand-in in host code, not a device
// address: its address on each device is resolved once, with that device
// current, by hipGetSymbolAddress when the first context on the device is
// created, and only that pointer is handed to kernels and copies.  The pinned
// host staging buffers and the events of this path are also made at context
// creation, so the entry point itself calls no allocating routine.
//
// Every call on a GPU shares that GPU's array and finds the previous call's
// contents there: the engine clears what must start at zero (the used-vertex
// bitmap and the query's counters, in its admission kernel) and writes every
// other buffer before reading it.  Calls that overlap on one GPU (from
// several threads or several contexts) race on the array.
#include <mutex>

#include "fx_host.h"

namespace {

constexpr size_t kScratchBytes = FX_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
constexpr uint64_t kStepCandidates = 1ull << 22;  // flattened candidates per step
constexpr int64_t kSliceRows = 1 << 14;           // level capacity of the query's stack

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

EngineParams fx_noalloc_params(const EngineParams &base)
{
    EngineParams p = base;
    p.max_active = 1;
    p.lanes = 1;
    p.step_candidates = kStepCandidates;
    p.slice_rows = kSliceRows;
    p.last_span_init = (uint32_t)std::min<int64_t>(p.last_span_init, kSliceRows);
    p.timing = false;
    p.lone_growth = false;
    p.promote_after = INT32_MAX;  // the stack never moves to a larger region
    p.chain_queries = 0;          // no device-scheduled chains (their graph and buffers are allocated)
    return p;
}

fx_status fx_noalloc_setup(fx_ctx *c)
{
    if (c->device < 0 || c->device >= kMaxDevices) return fx_fail(FX_ELIMIT, "device %d out of range", c->device);
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_scratch[c->device]) {
            void *ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr)
                return fx_fail(FX_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            g_scratch[c->device] = ptr;
        }
        base = g_scratch[c->device];
    }
    auto W = std::make_unique<EngineWork>();
    // per-step scratch sized for the largest grid any items-per-thread value
    // gives at the fixed step budget (one query: one segment)
    const uint64_t min_tile = (uint64_t)FX_BS * 2;
    const uint64_t max_blocks = (kStepCandidates + min_tile - 1) / min_tile + 1;
    // the probe's per-tile records: blocks x record bytes is largest for the
    // smallest tile (a record is 8 bytes per candidate slot plus 32)
    const size_t cand_bytes = (size_t)max_blocks * cand_tile_bytes(2);
    char *p = (char *)base;
    auto carve = [&](DevBuf &b, size_t bytes) {
        b.borrow(p, bytes);
        p += up256(bytes);
    };
    EngineLane &L = W->lane[0];
    carve(W->sums_d, sizeof(FxSummary));
    carve(L.cand, cand_bytes);
    carve(L.bcnt, max_blocks * 4);
    carve(L.boff, (max_blocks + 1) * 8);
    carve(L.lsum, max_blocks * 8);
    carve(L.loff, (max_blocks + 1) * 8);
    carve(L.sstat, (size_t)scan_state_words((uint32_t)max_blocks) * 8);
    carve(L.tmap, max_blocks * sizeof(FxTile));
    carve(L.stage_d, 4096);
    carve(L.inits_d, sizeof(FxInit));
    // the rest holds the query's stack: one pool chunk that never grows
    const size_t used = (size_t)(p - (char *)base);
    if (used + (1u << 20) > kScratchBytes) return fx_fail(FX_ELIMIT, "scratch array too small for its buffers");
    RegionPool::Chunk ch;
    ch.base = p;
    ch.size = kScratchBytes - used;
    ch.free_[0] = ch.size;
    W->pool.alloc_fn = nullptr;  // nothing beyond the chunk
    W->pool.free_fn = nullptr;
    W->pool.budget = ch.size;
    W->pool.held = ch.size;
    W->pool.chunks.push_back(std::move(ch));
    FX_TRY(L.stage_h.ensure(4096));
    FX_TRY(L.inits_h.ensure(sizeof(FxInit)));
    FX_TRY(L.sums_h.ensure(sizeof(FxSummary)));
    FX_TRY(W->init_events(1));  // one lane: no streams of its own
    c->na_work = std::move(W);
    return FX_OK;
}

extern "C" fx_status fx_support_noalloc(fx_graph *g, const fx_pattern *p, int64_t sigma, double lambda, int32_t mode,
                                        fx_result *out)
{
    if (!g || !out) return fx_fail(FX_EINVAL, "NULL argument");
    if (sigma < 1) return fx_fail(FX_EINVAL, "sigma must be >= 1");
    if (!(lambda >= 0.0 && lambda <= 1.0)) return fx_fail(FX_EINVAL, "lambda must lie in [0, 1]");
    if (mode != FX_MODE_FULL && mode != FX_MODE_VERDICT && mode != FX_MODE_MNI)
        return fx_fail(FX_EINVAL, "unknown mode %d", mode);
    fx_ctx *c = g->ctx;
    if (!c->na_work) return fx_fail(FX_EDEVICE, "the context has no scratch array");
    FX_HIP(hipSetDevice(c->device));
    const EngineParams P = fx_noalloc_params(c->params);
    std::vector<FxRequest> reqs(1);
    fx_result res{};
    FxRequest &r = reqs[0];
    r.pattern = p;
    r.sigma = sigma;
    r.lambda = lambda;
    r.kind = mode == FX_MODE_FULL ? FX_Q_FULL : (mode == FX_MODE_MNI ? FX_Q_MNI : FX_Q_VERDICT);
    r.out = &res;
    // a stack that does not fit the chunk is reported as FX_ENOMEM by the
    // engine's admission; name the limit instead
    FX_TRY(fx_engine_run_on(g, c->na_work.get(), P, reqs));
    if (r.status == FX_ENOMEM)
        return fx_fail(FX_ELIMIT, "the query needs more than the %zu-byte scratch array (%s)", kScratchBytes,
                       fx_last_error());
    if (r.status != FX_OK) return r.status;
    *out = res;
    return FX_OK;
}
