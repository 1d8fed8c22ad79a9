// Continuous-batching query server.
//
// A worker thread owns a stream and an engine over a resident graph.  Queries
// submitted from any thread are handed to the engine between device steps;
// the engine admits them as soon as a slot and region memory are free, so
// queries that arrive while others run join the very next step and their
// work shares every launch with the queries already in flight.  Results are
// picked up with poll or wait.
#include <condition_variable>
#include <mutex>
#include <string>
#include <thread>

#include "fx_host.h"

namespace {

struct ServerTicket {
    uint64_t id = 0;
    std::vector<int32_t> vl, ed, el;  // the pattern, copied at submission
    fx_pattern pat{};
    FxRequest req;
    fx_result res{};
    std::chrono::steady_clock::time_point t_submit, t_done;
    bool done = false;
};

}  // namespace

struct fx_server {
    fx_graph *G = nullptr;
    hipStream_t stream = nullptr;
    EngineParams params;
    EngineWork work;
    fx_stats stats{};
    std::unique_ptr<FxEngine> engine;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<ServerTicket *> incoming;
    std::unordered_map<uint64_t, std::unique_ptr<ServerTicket>> tickets;
    uint64_t next_id = 1;
    bool stop = false;
    fx_status failed = FX_OK;
    std::string fail_msg;
};

namespace {

void server_loop(fx_server *S)
{
    (void)hipSetDevice(S->G->ctx->device);
    S->engine->on_done = [S](FxRequest *r) {
        ServerTicket *t = (ServerTicket *)r->user;
        std::lock_guard<std::mutex> lk(S->mu);
        t->done = true;
        t->t_done = std::chrono::steady_clock::now();
        t->res.device_ms = std::chrono::duration<double, std::milli>(t->t_done - t->t_submit).count();
        S->cv_done.notify_all();
    };
    while (true) {
        std::deque<ServerTicket *> batch;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] { return S->stop || !S->incoming.empty() || !S->engine->idle(); });
            if (S->stop && S->incoming.empty() && S->engine->idle()) break;
            batch.swap(S->incoming);
        }
        for (ServerTicket *t : batch) S->engine->add(&t->req);
        if (!S->engine->idle()) {
            const fx_status st = S->engine->step();
            if (st != FX_OK) {
                std::lock_guard<std::mutex> lk(S->mu);
                S->failed = st;
                S->fail_msg = fx_last_error();
                for (auto &kv : S->tickets)
                    if (!kv.second->done) {
                        kv.second->req.status = st;
                        kv.second->done = true;
                    }
                S->cv_done.notify_all();
                break;
            }
        }
    }
}

fx_status take_result(fx_server *S, std::unordered_map<uint64_t, std::unique_ptr<ServerTicket>>::iterator it,
                      fx_result *out)
{
    ServerTicket *t = it->second.get();
    const fx_status st = t->req.status;
    if (st == FX_OK) {
        *out = t->res;
    } else {  // the query's own error, also in the result
        *out = fx_result{};
        out->status = st;
    }
    S->tickets.erase(it);
    if (st != FX_OK) return fx_fail(st, "query failed: %s", S->failed != FX_OK ? S->fail_msg.c_str() : "invalid query");
    return FX_OK;
}

}  // namespace

extern "C" fx_status fx_server_create(fx_graph *g, const fx_server_opts *opts, fx_server **out)
{
    if (!g || !out) return fx_fail(FX_EINVAL, "NULL argument");
    fx_server_opts o{};
    if (opts) o = *opts;
    if (o.max_active < 0 || o.slice_rows < 0 || o.mem_budget_bytes < 0 || o.step_candidates < 0)
        return fx_fail(FX_EINVAL, "server options must be >= 0");
    if ((o.flags & ~FX_CTX_NO_DIGEST) != 0) return fx_fail(FX_EINVAL, "unknown server flags 0x%x", o.flags);
    FX_HIP(hipSetDevice(g->ctx->device));
    auto S = std::make_unique<fx_server>();
    S->G = g;
    S->params = g->ctx->params;
    S->params.timing = false;
    // queries arrive continuously, so "nearly alone" is a passing moment of a
    // server rather than the tail of a batch: measured on the cl100k sweep,
    // growing there cost 16% of the served capacity
    S->params.lone_growth = false;
    // a query that arrives while a device-scheduled chain runs would wait for
    // the whole chain: the server schedules every step on the host
    S->params.chain_queries = 0;
    if (o.max_active > 0) S->params.max_active = o.max_active;
    if (o.slice_rows > 0) S->params.slice_rows = std::min<int64_t>(std::max<int64_t>(o.slice_rows, 64), (int64_t)1 << 26);
    if (o.step_candidates > 0) S->params.step_candidates = (uint64_t)std::max<int64_t>(o.step_candidates, FX_MAX_TILE);
    if (o.flags & FX_CTX_NO_DIGEST) S->params.no_digest = true;
    S->work.pool.budget = o.mem_budget_bytes > 0 ? (size_t)o.mem_budget_bytes : g->ctx->work.pool.budget;
    FX_HIP(hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking));
    S->engine = std::make_unique<FxEngine>(g, &S->work, S->stream, S->params, &S->stats);
    g->servers++;
    fx_server *raw = S.release();
    raw->th = std::thread(server_loop, raw);
    *out = raw;
    return FX_OK;
}

extern "C" fx_status fx_server_submit(fx_server *S, const fx_pattern *p, int64_t sigma, double lambda, int32_t mode,
                                      uint64_t *ticket)
{
    if (!S || !p || !ticket) return fx_fail(FX_EINVAL, "NULL argument");
    if (sigma < 1) return fx_fail(FX_EINVAL, "sigma must be >= 1");
    if (!(lambda >= 0.0 && lambda <= 1.0)) return fx_fail(FX_EINVAL, "lambda must lie in [0, 1]");
    if (mode != FX_MODE_FULL && mode != FX_MODE_VERDICT && mode != FX_MODE_MNI)
        return fx_fail(FX_EINVAL, "unknown mode %d", mode);
    FX_TRY(fx_check_pattern(p, S->G->directed));
    auto t = std::make_unique<ServerTicket>();
    t->vl.assign(p->vlabel, p->vlabel + p->n);
    t->ed.assign(p->edges, p->edges + 2 * p->m);
    if (p->elabel) t->el.assign(p->elabel, p->elabel + p->m);
    else t->el.assign(p->m, 0);
    t->pat.n = p->n;
    t->pat.m = p->m;
    t->pat.vlabel = t->vl.data();
    t->pat.edges = t->ed.data();
    t->pat.elabel = t->el.data();
    t->req.pattern = &t->pat;
    t->req.sigma = sigma;
    t->req.lambda = lambda;
    t->req.kind = mode == FX_MODE_FULL ? FX_Q_FULL : (mode == FX_MODE_MNI ? FX_Q_MNI : FX_Q_VERDICT);
    t->req.out = &t->res;
    t->req.user = t.get();
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->failed != FX_OK) return fx_fail(S->failed, "server failed: %s", S->fail_msg.c_str());
    if (S->stop) return fx_fail(FX_EBUSY, "server is shutting down");
    t->id = S->next_id++;
    t->t_submit = std::chrono::steady_clock::now();
    *ticket = t->id;
    S->incoming.push_back(t.get());
    S->tickets[t->id] = std::move(t);
    S->cv_work.notify_one();
    return FX_OK;
}

extern "C" fx_status fx_server_poll(fx_server *S, uint64_t ticket, fx_result *out, int32_t *done)
{
    if (!S || !out || !done) return fx_fail(FX_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return fx_fail(FX_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (!it->second->done) {
        *done = 0;
        return FX_OK;
    }
    *done = 1;
    return take_result(S, it, out);
}

extern "C" fx_status fx_server_wait(fx_server *S, uint64_t ticket, int64_t timeout_us, fx_result *out)
{
    if (!S || !out) return fx_fail(FX_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return fx_fail(FX_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    ServerTicket *t = it->second.get();
    auto ready = [&] { return t->done; };
    if (timeout_us < 0) {
        S->cv_done.wait(lk, ready);
    } else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
        return fx_fail(FX_ETIMEOUT, "ticket %llu not done after %lld us", (unsigned long long)ticket,
                       (long long)timeout_us);
    }
    return take_result(S, S->tickets.find(ticket), out);
}

extern "C" fx_status fx_server_stats(fx_server *S, fx_stats *out)
{
    if (!S || !out) return fx_fail(FX_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->stats;
    return FX_OK;
}

extern "C" fx_status fx_server_destroy(fx_server *S)
{
    if (!S) return fx_fail(FX_EINVAL, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;  // queued and running queries are finished first
    }
    S->cv_work.notify_all();
    if (S->th.joinable()) S->th.join();
    (void)hipSetDevice(S->G->ctx->device);
    if (S->stream) (void)hipStreamSynchronize(S->stream);
    S->engine.reset();
    if (S->stream) (void)hipStreamDestroy(S->stream);
    S->G->servers--;
    delete S;
    return FX_OK;
}
