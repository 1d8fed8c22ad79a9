// C ABI entry points and host utilities of the support-counting library.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fx_host.h"
#include "fx_workers.h"

namespace {
thread_local std::string g_last_error;
}

fx_status fx_fail(fx_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

// ---------------------------------------------------------------------------
// Host worker threads
// ---------------------------------------------------------------------------

void fx_parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)> &fn)
{
    if (n <= 0) return;
    grain = std::max<int64_t>(grain, 1);
    if (n <= grain) {
        fn(0, n);
        return;
    }
    // never destroyed: the parked workers simply end with the process
    static HostWorkers *w = new HostWorkers();
    w->run(n, grain, fn);
}

// ---------------------------------------------------------------------------
// Buffers
// ---------------------------------------------------------------------------

std::atomic<uint64_t> fx_alloc_calls_made{0};

void DevBuf::release()
{
    if (p && !borrowed) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    borrowed = false;
}

fx_status DevBuf::ensure(size_t want)
{
    if (want <= bytes && p) return FX_OK;
    if (borrowed)
        return fx_fail(FX_ELIMIT, "a step needs %zu bytes of a scratch buffer of %zu bytes", want, bytes);
    release();
    const size_t b = std::max<size_t>(want, 256);
    fx_alloc_calls_made++;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
        p = nullptr;
        return fx_fail(FX_ENOMEM, "hipMalloc(%zu) failed: %s", b, hipGetErrorString(e));
    }
    bytes = b;
    return FX_OK;
}

void HostBuf::release()
{
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
}

fx_status HostBuf::ensure(size_t want)
{
    if (want <= bytes && p) return FX_OK;
    release();
    const size_t b = std::max<size_t>(want, 256);
    fx_alloc_calls_made++;
    hipError_t e = hipHostMalloc(&p, b, hipHostMallocDefault);
    if (e != hipSuccess) {
        p = nullptr;
        return fx_fail(FX_ENOMEM, "hipHostMalloc(%zu) failed: %s", b, hipGetErrorString(e));
    }
    bytes = b;
    return FX_OK;
}

// ---------------------------------------------------------------------------
// Small entry points
// ---------------------------------------------------------------------------

extern "C" const char *fx_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *fx_version(void) { return "flexis-mi355x 0.3 (gfx950)"; }

extern "C" uint64_t fx_alloc_calls(void) { return fx_alloc_calls_made.load(); }

// tau of the tau equation (Section 3.1.1): floor(sigma * ((n-1) lambda + 1) / n)
// with lambda rounded to parts per million, in exact integer arithmetic.
fx_status fx_tau_checked(int64_t sigma, double lambda, int32_t n, int64_t *tau_out)
{
    if (!tau_out) return fx_fail(FX_EINVAL, "tau_out is NULL");
    if (sigma < 0) return fx_fail(FX_EINVAL, "sigma must be >= 0");
    if (!(lambda >= 0.0 && lambda <= 1.0)) return fx_fail(FX_EINVAL, "lambda must lie in [0, 1]");
    if (n < 1) return fx_fail(FX_EINVAL, "n must be >= 1");
    const __int128 ppm = (__int128)llround(lambda * 1e6);
    const __int128 num = (__int128)sigma * ((__int128)(n - 1) * ppm + 1000000);
    const __int128 den = (__int128)n * 1000000;
    *tau_out = (int64_t)(num / den);
    return FX_OK;
}

extern "C" fx_status fx_tau(int64_t sigma, double lambda, int32_t n, int64_t *tau_out)
{
    return fx_tau_checked(sigma, lambda, n, tau_out);
}

extern "C" fx_status fx_ctx_create(const fx_ctx_opts *opts, fx_ctx **out)
{
    if (!out) return fx_fail(FX_EINVAL, "out is NULL");
    fx_ctx_opts o{};
    if (opts) o = *opts;
    if ((o.flags & ~(FX_CTX_KERNEL_TIMING | FX_CTX_NO_DIGEST)) != 0)
        return fx_fail(FX_EINVAL, "unknown flags 0x%x", o.flags);
    if (o.slice_rows < 0 || o.count_cap < 0 || o.mem_budget_bytes < 0 || o.run_index_bytes < -1)
        return fx_fail(FX_EINVAL, "slice_rows, count_cap, mem_budget_bytes must be >= 0, run_index_bytes >= -1");
    int ndev = 0;
    FX_HIP(hipGetDeviceCount(&ndev));
    if (o.device < 0 || o.device >= ndev)
        return fx_fail(FX_EINVAL, "device %d out of range (%d devices)", o.device, ndev);
    FX_HIP(hipSetDevice(o.device));
    fx_ctx *c = new fx_ctx();
    c->device = o.device;
    c->stream = (hipStream_t)o.hip_stream;
    if (o.slice_rows > 0)
        c->params.slice_rows = std::min<int64_t>(std::max<int64_t>(o.slice_rows, 64), (int64_t)1 << 26);
    if (o.count_cap > 0) c->params.count_cap = o.count_cap;
    c->work.pool.budget = o.mem_budget_bytes > 0 ? (size_t)o.mem_budget_bytes : ((size_t)64 << 30);
    if (o.run_index_bytes != 0) c->run_index_bytes = o.run_index_bytes;
    c->params.timing = (o.flags & FX_CTX_KERNEL_TIMING) != 0;
    c->params.no_digest = (o.flags & FX_CTX_NO_DIGEST) != 0;
    const fx_status st = fx_noalloc_setup(c);  // the device is current here
    if (st != FX_OK) {
        delete c;
        return st;
    }
    *out = c;
    return FX_OK;
}

extern "C" fx_status fx_ctx_destroy(fx_ctx *c)
{
    if (!c) return fx_fail(FX_EINVAL, "ctx is NULL");
    if (c->graphs.load() != 0) return fx_fail(FX_EBUSY, "%d graph(s) still loaded", c->graphs.load());
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    delete c;
    return FX_OK;
}

extern "C" fx_status fx_ctx_set(fx_ctx *c, const char *key, int64_t value)
{
    if (!c || !key) return fx_fail(FX_EINVAL, "NULL argument");
    EngineParams &P = c->params;
    const std::string k = key;
    auto in = [&](int64_t lo, int64_t hi) -> bool { return value >= lo && value <= hi; };
    if (k == "slice_rows" && in(64, (int64_t)1 << 26)) P.slice_rows = value;
    else if (k == "step_candidates" && in(FX_MAX_TILE, (int64_t)1 << 31)) P.step_candidates = (uint64_t)value;
    else if (k == "items_per_thread" && (value == 2 || value == 4 || value == 8)) P.items = (int32_t)value;
    else if (k == "last_span_init" && in(1, (int64_t)1 << 26)) P.last_span_init = (uint32_t)value;
    else if (k == "lanes" && in(1, FX_MAX_LANES)) P.lanes = (int32_t)value;
    else if (k == "max_active" && in(1, 1 << 20)) P.max_active = (int32_t)value;
    else if (k == "promote_after" && in(0, INT32_MAX)) P.promote_after = (int32_t)value;
    else if (k == "lone_queries" && in(0, INT32_MAX)) P.lone_queries = (int32_t)value;
    else if (k == "lone_after" && in(0, INT32_MAX)) P.lone_after = (int32_t)value;
    else if (k == "lone_growth" && in(0, 1)) P.lone_growth = value != 0;
    else if (k == "kernel_timing" && in(0, 1)) P.timing = value != 0;
    else if (k == "chain_queries" && in(0, 64)) P.chain_queries = (int32_t)value;
    else if (k == "chain_steps" && in(1, 256)) P.chain_steps = (int32_t)value;
    else if (k == "ref_bytes" && in(0, 1)) P.ref_bytes = value != 0;
    else if (k == "check_steps" && in(0, 1)) P.check_steps = value != 0;
    else if (k == "fused" && in(0, 1)) P.fused = value != 0;
    else if (k == "fused_below" && in(0, INT32_MAX)) P.fused_below = (int32_t)value;
    else return fx_fail(FX_EINVAL, "unknown tunable '%s' or value %lld out of range", key, (long long)value);
    return FX_OK;
}

extern "C" fx_status fx_ctx_get(fx_ctx *c, const char *key, int64_t *value)
{
    if (!c || !key || !value) return fx_fail(FX_EINVAL, "NULL argument");
    const EngineParams &P = c->params;
    const std::string k = key;
    if (k == "slice_rows") *value = P.slice_rows;
    else if (k == "step_candidates") *value = (int64_t)P.step_candidates;
    else if (k == "items_per_thread") *value = P.items;
    else if (k == "last_span_init") *value = P.last_span_init;
    else if (k == "lanes") *value = P.lanes;
    else if (k == "max_active") *value = P.max_active;
    else if (k == "promote_after") *value = P.promote_after;
    else if (k == "lone_queries") *value = P.lone_queries;
    else if (k == "lone_after") *value = P.lone_after;
    else if (k == "lone_growth") *value = P.lone_growth ? 1 : 0;
    else if (k == "kernel_timing") *value = P.timing ? 1 : 0;
    else if (k == "chain_queries") *value = P.chain_queries;
    else if (k == "chain_steps") *value = P.chain_steps;
    else if (k == "ref_bytes") *value = P.ref_bytes ? 1 : 0;
    else if (k == "check_steps") *value = P.check_steps ? 1 : 0;
    else if (k == "fused") *value = P.fused ? 1 : 0;
    else if (k == "fused_below") *value = P.fused_below;
    else return fx_fail(FX_EINVAL, "unknown tunable '%s'", key);
    return FX_OK;
}

extern "C" fx_status fx_ctx_stats(fx_ctx *c, fx_stats *out, int32_t reset)
{
    if (!c || !out) return fx_fail(FX_EINVAL, "NULL argument");
    *out = c->stats;
    if (reset) c->stats = fx_stats{};
    return FX_OK;
}

// ---------------------------------------------------------------------------
// Queries
// ---------------------------------------------------------------------------

int32_t fx_query_kind(int32_t mode)
{
    switch (mode) {
    case FX_MODE_FULL: return FX_Q_FULL;
    case FX_MODE_MNI: return FX_Q_MNI;
    case FX_MODE_MIS: return FX_Q_MIS;
    default: return FX_Q_VERDICT;
    }
}

extern "C" fx_status fx_support(fx_graph *g, const fx_pattern *p, int64_t sigma, double lambda, int32_t mode,
                                fx_result *out, int32_t *selected, int64_t selected_cap)
{
    if (!g || !out) return fx_fail(FX_EINVAL, "NULL argument");
    if (sigma < 1) return fx_fail(FX_EINVAL, "sigma must be >= 1");
    if (!(lambda >= 0.0 && lambda <= 1.0)) return fx_fail(FX_EINVAL, "lambda must lie in [0, 1]");
    if (mode != FX_MODE_FULL && mode != FX_MODE_VERDICT && mode != FX_MODE_MNI && mode != FX_MODE_MIS)
        return fx_fail(FX_EINVAL, "unknown mode %d", mode);
    if (selected_cap < 0 || (selected_cap > 0 && !selected)) return fx_fail(FX_EINVAL, "bad selected buffer");
    FX_HIP(hipSetDevice(g->ctx->device));
    std::vector<FxRequest> reqs(1);
    fx_result res{};
    FxRequest &r = reqs[0];
    r.pattern = p;
    r.sigma = sigma;
    r.lambda = lambda;
    r.kind = fx_query_kind(mode);
    r.out = &res;
    r.selected = selected;
    r.selected_cap = selected_cap;
    FX_TRY(fx_engine_run(g, reqs, 1, false));
    if (r.status != FX_OK) return r.status;
    *out = res;
    return FX_OK;
}

extern "C" fx_status fx_enumerate(fx_graph *g, const fx_pattern *p, int32_t *rows, int64_t cap, int64_t *count_out)
{
    if (!g || !count_out) return fx_fail(FX_EINVAL, "NULL argument");
    if (cap < 0 || (cap > 0 && !rows)) return fx_fail(FX_EINVAL, "bad output buffer");
    FX_HIP(hipSetDevice(g->ctx->device));
    std::vector<FxRequest> reqs(1);
    int64_t cnt = 0;
    FxRequest &r = reqs[0];
    r.pattern = p;
    r.kind = FX_Q_LIST;
    r.list_rows = rows;
    r.list_cap = cap;
    r.list_count = &cnt;
    FX_TRY(fx_engine_run(g, reqs, 1, false));
    if (r.status != FX_OK) return r.status;
    *count_out = cnt;
    return FX_OK;
}

extern "C" fx_status fx_support_batch(fx_graph *g, int32_t npat, const fx_pattern *pats, const int64_t *sigma,
                                      const double *lambda, int32_t mode, fx_result *out)
{
    if (!g || npat < 0 || (npat > 0 && (!pats || !sigma || !lambda || !out))) return fx_fail(FX_EINVAL, "bad batch");
    if (mode != FX_MODE_FULL && mode != FX_MODE_VERDICT && mode != FX_MODE_MNI && mode != FX_MODE_MIS)
        return fx_fail(FX_EINVAL, "unknown mode %d", mode);
    // sigma and lambda here; the patterns are checked when their plans are
    // built, for the whole batch before any device work
    for (int32_t i = 0; i < npat; i++) {
        if (sigma[i] < 1) return fx_fail(FX_EINVAL, "pattern %d: sigma must be >= 1", i);
        if (!(lambda[i] >= 0.0 && lambda[i] <= 1.0)) return fx_fail(FX_EINVAL, "pattern %d: lambda outside [0, 1]", i);
    }
    FX_HIP(hipSetDevice(g->ctx->device));
    std::vector<FxRequest> reqs(npat);
    std::vector<fx_result> res(npat);
    for (int32_t i = 0; i < npat; i++) {
        reqs[i].pattern = &pats[i];
        reqs[i].sigma = sigma[i];
        reqs[i].lambda = lambda[i];
        reqs[i].kind = fx_query_kind(mode);
        reqs[i].out = &res[i];
    }
    FX_TRY(fx_engine_run(g, reqs, g->ctx->params.max_active));
    for (int32_t i = 0; i < npat; i++)
        if (reqs[i].status != FX_OK) return reqs[i].status;
    std::copy(res.begin(), res.end(), out);
    return FX_OK;
}
