// Autotuner of the engine's launch shape.
//
// Times fx_support_batch on a caller's sample of patterns while it walks the
// tunables one at a time (coordinate descent): candidates per thread in the
// expansion kernels (the workgroup's tile), candidates per device step, the
// level capacity of a query's slice stack (the frontier chunk), and the first
// last-vertex slice of the greedy.  The fastest setting is kept in the
// context.  A cache file (one line per key: architecture, graph shape,
// largest pattern, mode) skips the timing when the key was tuned before.
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "fx_host.h"

namespace {

std::string tune_key(const fx_graph *G, int32_t npat, const fx_pattern *pats, int32_t mode)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, G->ctx->device) == hipSuccess) arch = prop.gcnArchName;
    for (auto &ch : arch)
        if (ch == ' ') ch = '_';
    int nmax = 0;
    for (int32_t i = 0; i < npat; i++) nmax = std::max(nmax, pats[i].n);
    std::ostringstream k;
    k << arch << "|nv=" << G->nv << "|adj=" << G->nadj << "|vl=" << G->vl_values.size() << "|el="
      << G->el_values.size() << "|n=" << nmax << "|mode=" << mode << "|digest=" << (G->ctx->params.no_digest ? 0 : 1) << "|v3";
    return k.str();
}

bool cache_lookup(const char *path, const std::string &key, EngineParams &p, double &ms)
{
    if (!path) return false;
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {  // the last line for a key wins
        std::istringstream in(line);
        std::string k;
        long long slice, step;
        int items, last, lanes, active;
        double t;
        if (in >> k >> slice >> step >> items >> last >> lanes >> active >> t && k == key) {
            p.max_active = active;
            p.slice_rows = slice;
            p.step_candidates = (uint64_t)step;
            p.items = items;
            p.last_span_init = (uint32_t)last;
            p.lanes = lanes;
            ms = t;
            found = true;
        }
    }
    return found;
}

void cache_store(const char *path, const std::string &key, const EngineParams &p, double ms)
{
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    f << key << " " << p.slice_rows << " " << p.step_candidates << " " << p.items << " " << p.last_span_init << " "
      << p.lanes << " " << p.max_active << " " << ms << "\n";
}

}  // namespace

extern "C" fx_status fx_autotune(fx_graph *g, int32_t npat, const fx_pattern *pats, const int64_t *sigma,
                                 const double *lambda, int32_t mode, const char *cache_path, fx_tune_result *out)
{
    if (!g || !out || npat <= 0 || !pats || !sigma || !lambda) return fx_fail(FX_EINVAL, "bad tuning sample");
    if (mode != FX_MODE_FULL && mode != FX_MODE_VERDICT) return fx_fail(FX_EINVAL, "unknown mode %d", mode);
    for (int32_t i = 0; i < npat; i++) {
        if (sigma[i] < 1) return fx_fail(FX_EINVAL, "pattern %d: sigma must be >= 1", i);
        if (!(lambda[i] >= 0.0 && lambda[i] <= 1.0)) return fx_fail(FX_EINVAL, "pattern %d: lambda outside [0, 1]", i);
        FX_TRY(fx_check_pattern(&pats[i], g->directed));
    }
    fx_ctx *c = g->ctx;
    FX_HIP(hipSetDevice(c->device));
    fx_tune_result r{};
    const std::string key = tune_key(g, npat, pats, mode);
    EngineParams cached = c->params;
    double cached_ms = 0;
    if (cache_lookup(cache_path, key, cached, cached_ms)) {
        c->params = cached;
        r.slice_rows = cached.slice_rows;
        r.step_candidates = (int64_t)cached.step_candidates;
        r.items_per_thread = cached.items;
        r.last_span_init = (int32_t)cached.last_span_init;
        r.lanes = cached.lanes;
        r.max_active = cached.max_active;
        r.best_ms = cached_ms;
        r.from_cache = 1;
        *out = r;
        return FX_OK;
    }
    std::vector<FxRequest> reqs(npat);
    std::vector<fx_result> res(npat);
    auto trial = [&](const EngineParams &p, double *ms) -> fx_status {
        const EngineParams keep = c->params;
        c->params = p;
        for (int32_t i = 0; i < npat; i++) {
            reqs[i] = FxRequest{};
            reqs[i].pattern = &pats[i];
            reqs[i].sigma = sigma[i];
            reqs[i].lambda = lambda[i];
            reqs[i].kind = mode == FX_MODE_FULL ? FX_Q_FULL : FX_Q_VERDICT;
            reqs[i].out = &res[i];
        }
        FX_HIP(c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize());
        const auto t0 = std::chrono::steady_clock::now();
        const fx_status st = fx_engine_run(g, reqs, p.max_active);
        *ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        c->params = keep;
        r.trials++;
        return st;
    };
    EngineParams best = c->params;
    double best_ms = 0, ms = 0;
    FX_TRY(trial(best, &ms));  // warm-up: workspace, region chunks
    FX_TRY(trial(best, &best_ms));
    r.default_ms = best_ms;
    auto sweep = [&](auto set, const std::vector<long long> &values) -> fx_status {
        EngineParams base = best;
        for (long long v : values) {
            EngineParams p = base;
            set(p, v);
            FX_TRY(trial(p, &ms));
            if (ms < best_ms) {
                best_ms = ms;
                best = p;
            }
        }
        return FX_OK;
    };
    FX_TRY(sweep([](EngineParams &p, long long v) { p.items = (int32_t)v; }, {2, 4, 8}));
    FX_TRY(sweep([](EngineParams &p, long long v) { p.step_candidates = (uint64_t)v; },
                 {1ll << 23, 1ll << 24, 1ll << 25, 1ll << 26}));
    FX_TRY(sweep([](EngineParams &p, long long v) { p.slice_rows = v; }, {1ll << 15, 1ll << 16, 1ll << 17, 1ll << 18}));
    FX_TRY(sweep([](EngineParams &p, long long v) { p.last_span_init = (uint32_t)v; }, {1024, 4096, 16384}));
    FX_TRY(sweep([](EngineParams &p, long long v) { p.lanes = (int32_t)v; }, {1, 2, 3}));
    FX_TRY(sweep([](EngineParams &p, long long v) { p.max_active = (int32_t)v; }, {4096, 16384}));
    c->params = best;
    cache_store(cache_path, key, best, best_ms);
    r.slice_rows = best.slice_rows;
    r.step_candidates = (int64_t)best.step_candidates;
    r.items_per_thread = best.items;
    r.last_span_init = (int32_t)best.last_span_init;
    r.lanes = best.lanes;
    r.max_active = best.max_active;
    r.best_ms = best_ms;
    *out = r;
    return FX_OK;
}
