// Pattern plans and the multi-query engine.
//
// A query's slice stack holds, for every level l (l pattern vertices
// matched), the partial embeddings of the current slice of level l-1 and
// each one's candidate run for pattern vertex l.  A step expands one slice
// of the deepest level that still has unexpanded candidates, so complete
// embeddings appear in rank order (lexicographic in submitted vertex order,
// ascending ids).  Every step serves all active queries at once: each
// contributes one segment to the same kernel launches, and the host reads
// all their counters with one copy and one synchronisation.
//
// Phases of a query:
//   support  partial embeddings and candidates that meet the used-vertex set
//            U are dropped (the bitmap of the matcher in Section 3.2.2); the
//            complete embeddings of each slice go through the greedy, which
//            extends U.  In VERDICT mode the query ends as soon as the
//            support reaches tau (the early termination of Section 3.1.1).
//   count    (FULL mode) every embedding is enumerated again without U and
//            counted and hashed at the last vertex, up to the count cap.
//   list     (fx_enumerate) every complete embedding is written out.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <numeric>

#include "fx_host.h"
#include "fx_sym.h"

// ---------------------------------------------------------------------------
// Pattern plan
// ---------------------------------------------------------------------------

fx_status fx_check_pattern(const fx_pattern *p, bool directed)
{
    if (!p) return fx_fail(FX_EINVAL, "pattern is NULL");
    if (p->n > FX_MAXN) return fx_fail(FX_ELIMIT, "pattern has %d vertices; at most %d", p->n, FX_MAXN);
    if (p->n < 1 || p->m < 0) return fx_fail(FX_EPATTERN, "pattern needs n >= 1 and m >= 0");
    if (!p->vlabel || (p->m > 0 && !p->edges)) return fx_fail(FX_EINVAL, "pattern arrays are NULL");
    const int n = p->n;
    bool adj[FX_MAXN][FX_MAXN] = {};  // undirected: either order; directed: a -> b
    bool any[FX_MAXN][FX_MAXN] = {};  // connected in either direction
    for (int k = 0; k < p->m; k++) {
        int a = p->edges[2 * k], b = p->edges[2 * k + 1];
        if (a < 0 || b < 0 || a >= n || b >= n) return fx_fail(FX_EPATTERN, "edge %d has an endpoint out of range", k);
        if (a == b) return fx_fail(FX_EPATTERN, "edge %d is a loop", k);
        if (adj[a][b]) return fx_fail(FX_EPATTERN, "edge %d repeats an edge", k);
        if (p->elabel && p->elabel[k] < 0) return fx_fail(FX_EPATTERN, "edge %d has a negative label", k);
        adj[a][b] = true;
        if (!directed) adj[b][a] = true;
        any[a][b] = any[b][a] = true;
    }
    for (int i = 0; i < n; i++)
        if (p->vlabel[i] < 0) return fx_fail(FX_EPATTERN, "vertex %d has a negative label", i);
    bool seen[FX_MAXN] = {};
    int stack[FX_MAXN], top = 0, cnt = 1;
    seen[0] = true;
    stack[top++] = 0;
    while (top) {
        int x = stack[--top];
        for (int y = 0; y < n; y++)
            if (any[x][y] && !seen[y]) {
                seen[y] = true;
                cnt++;
                stack[top++] = y;
            }
    }
    if (cnt != n) return fx_fail(FX_EPATTERN, "pattern is not connected");
    return FX_OK;
}

fx_status fx_build_plan(const fx_graph *G, const fx_pattern *p, HostPlan &hp)
{
    FX_TRY(fx_check_pattern(p, G->directed));
    const int n = p->n;
    FxPlan &P = hp.plan;
    memset(&P, 0, sizeof(P));
    P.n = n;
    // ed[a][b]: dense label of the pattern edge a -> b (undirected: both
    // orders), or -1.  code(a, b): the edge code an edge between a and b has
    // in the row of f(a) -- its dense label, or for a directed graph 2 label
    // (outgoing from a) or 2 label + 1 (incoming into a).
    int32_t ed[FX_MAXN][FX_MAXN];
    for (int a = 0; a < n; a++)
        for (int b = 0; b < n; b++) ed[a][b] = -1;
    for (int i = 0; i < n; i++) {
        auto it = G->vl_map.find(p->vlabel[i]);
        if (it == G->vl_map.end()) hp.empty = true;
        else P.vl[i] = (uint16_t)it->second;
    }
    for (int k = 0; k < p->m; k++) {
        int a = p->edges[2 * k], b = p->edges[2 * k + 1];
        int32_t lab = p->elabel ? p->elabel[k] : 0;
        auto it = G->el_map.find(lab);
        int32_t d = 0;
        if (it == G->el_map.end()) hp.empty = true;
        else d = (int32_t)it->second;
        ed[a][b] = d;
        if (!G->directed) ed[b][a] = d;
    }
    // the (neighbour, edge code) pairs of vertex a towards vertex b
    auto codes = [&](int a, int b, int32_t *out) {
        int c = 0;
        if (!G->directed) {
            if (ed[a][b] >= 0) out[c++] = ed[a][b];
        } else {
            if (ed[a][b] >= 0) out[c++] = 2 * ed[a][b];      // a -> b: outgoing in a's row
            if (ed[b][a] >= 0) out[c++] = 2 * ed[b][a] + 1;  // b -> a: incoming in a's row
        }
        return c;
    };
    for (int i = 0; i < n; i++) {
        P.nback[i] = 0;
        for (int b = 0; b < i; b++) {
            int32_t cs[2];
            const int c = codes(b, i, cs);
            if (P.nback[i] + c > FX_MAXN)
                return fx_fail(FX_ELIMIT, "vertex %d has more than %d edges to earlier vertices", i, FX_MAXN);
            for (int k = 0; k < c; k++) {  // a reciprocal pair gives two constraints
                P.back[i][P.nback[i]] = (int8_t)b;
                P.bel[i][P.nback[i]] = (uint16_t)cs[k];
                P.nback[i]++;
            }
        }
        // neighbour-label filter over later neighbours: worthwhile for the
        // root and for vertices that need two or more later neighbours
        std::pair<uint32_t, int> need_buf[2 * FX_MAXN];
        int nneed = 0;
        int later = 0;
        for (int j = i + 1; j < n; j++) {
            int32_t cs[2];
            const int c = codes(i, j, cs);
            for (int k = 0; k < c; k++) {
                later++;
                const uint32_t key = ((uint32_t)P.vl[j] << 16) | (uint32_t)cs[k];
                bool found = false;
                for (int q = 0; q < nneed; q++)
                    if (need_buf[q].first == key) {
                        need_buf[q].second++;
                        found = true;
                    }
                if (!found) need_buf[nneed++] = {key, 1};
            }
        }
        P.nnlf[i] = 0;
        if (i < n - 1 && (i == 0 || later >= 2)) {
            std::stable_sort(need_buf, need_buf + nneed, [](auto &x, auto &y) { return x.second > y.second; });
            for (int q = 0; q < nneed; q++) {
                if (P.nnlf[i] == FX_NLF) break;
                P.nlf_key[i][P.nnlf[i]] = need_buf[q].first;
                P.nlf_need[i][P.nnlf[i]] = (uint8_t)need_buf[q].second;
                P.nnlf[i]++;
            }
        }
    }
    // symmetry breaking: automorphisms must keep every pair's edges, with
    // their directions; each ordered pair gets the class of (a -> b, b -> a)
    int32_t el[FX_MAXN][FX_MAXN];
    {
        std::vector<std::pair<int32_t, int32_t>> cls;
        for (int a = 0; a < n; a++)
            for (int b = 0; b < n; b++) {
                el[a][b] = -1;
                if (ed[a][b] < 0 && ed[b][a] < 0) continue;
                const std::pair<int32_t, int32_t> key{ed[a][b], ed[b][a]};
                size_t c = 0;
                while (c < cls.size() && cls[c] != key) c++;
                if (c == cls.size()) cls.push_back(key);
                el[a][b] = (int32_t)c;
            }
    }
    fx_symmetry_constraints(n, p->vlabel, el, P.sym_lt);
    for (int i = 0; i < n; i++) hp.symmetric = hp.symmetric || P.sym_lt[i] != 0;
    // upper bound on any independent set: disjoint images (bound of Section 3.1.2)
    int64_t ub = G->nv / n;
    if (!hp.empty) {
        for (int i = 0; i < n; i++) {  // label multiplicity, counted at its first vertex
            int c = 0, first = i;
            for (int j = 0; j < n; j++)
                if (P.vl[j] == P.vl[i]) {
                    c++;
                    if (j < first) first = j;
                }
            if (first != i) continue;
            const int64_t sz = G->bptr[P.vl[i] + 1] - G->bptr[P.vl[i]];
            ub = std::min<int64_t>(ub, sz / c);
        }
    } else {
        ub = 0;
    }
    hp.upper_bound = ub;
    return FX_OK;
}


// ---------------------------------------------------------------------------
// Engine
// ---------------------------------------------------------------------------

namespace {

constexpr uint64_t kCountSpan = FX_COUNT_SPAN;  // least last-vertex candidates per counting step
constexpr double kFill = FX_FILL;                // aim a slice at this fraction of the rows it may write
constexpr int64_t kPromoteCap = 1 << 23;     // largest slice capacity a stack is moved to

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Stage buffer of a step: workgroup starts of up to `segs` segments (plus the
// end), then the segment table.
size_t stage_off(size_t segs) { return align256((segs + 1) * 4); }
size_t stage_bytes(size_t segs, size_t table) { return stage_off(segs) + table * sizeof(FxSeg); }

enum { PH_SUPPORT = 0, PH_COUNT = 1, PH_LIST = 2 };

bool wants_selection(const FxRequest &r) { return r.kind == FX_Q_FULL && r.selected && r.selected_cap > 0; }

}  // namespace

struct FxQuery {
    FxRequest *req = nullptr;
    HostPlan hp;
    int n = 0;
    int64_t tau = 0, tau_eff = 1;
    int phase = PH_SUPPORT;
    int slot = -1;
    void *region = nullptr;
    size_t region_bytes = 0;
    int64_t cap = 0;
    FxLevelDev lev[FX_MAXN + 1]{};
    uint32_t *U = nullptr;
    uint32_t *img = nullptr;                 // image bitmaps (minimum-image support), after U
    unsigned long long *mni = nullptr;       // per-vertex image counts [FX_MAXN], then the minimum
    FxPlan *plan = nullptr;
    int32_t *sel_rows = nullptr;
    int64_t *sel_rank = nullptr;
    uint64_t T[FX_MAXN + 1]{}, cur[FX_MAXN + 1]{};
    int64_t nparts[FX_MAXN + 1]{};
    int64_t rank_base = 0;
    uint32_t last_span = 0;                // complete embeddings per greedy slice
    double rate[FX_MAXN + 1]{};            // passing fraction of each level's last slice
    uint64_t alg_probe_seen = 0;           // probe bytes read back so far
    double alg_probe_credit = 0;           // of those, the share of the candidates taken
    uint64_t ref_probe_seen = 0;           // the same for the reference bytes (counting pass)
    double ref_probe_credit = 0;
    uint64_t ref_row_seen = 0;
    double ref_row_credit = 0;
    uint64_t probed_support = 0;           // candidates probed in the support phase
    int32_t steps = 0;
    int deep = -1;                         // deepest level with candidates left (-1: none)
    int lane = 0;
    int exit = FX_EXIT_END;                // how the query ended (fx_result.exit)
    uint64_t last_ufiltered = 0;           // candidates U has removed, as of the last step read back
    int32_t *mis_rows = nullptr;           // exact-MIS mode: every embedding, collected on the device
    uint64_t *mis_hash = nullptr;
    FxMisOut *mis_out = nullptr;
    bool chain_done = false;               // finished in a device-scheduled chain
    int64_t listed = 0;
    // the segment of the current step (-1: none)
    int seg_l = -1, seg_kind = 0;
    uint64_t seg_t0 = 0;
    uint32_t seg_span = 0;
};

namespace {

size_t region_size(const FxQuery &q, int64_t nv)
{
    const int n = q.n;
    const size_t C = (size_t)q.cap;
    size_t b = 0;
    b += align256(8) + align256(4) + align256(1) + align256(16);  // level 0
    for (int l = 1; l < n; l++)
        b += align256(C * l * 4) + align256(C * 8) + align256(C * 4) + align256(C) + align256((C + 1) * 8);
    b += align256(C * n * 4);  // complete embeddings
    b += align256(((size_t)nv + 31) / 32 * 4 * (q.req->kind == FX_Q_MNI ? 1 + n : 1)) + align256(sizeof(FxPlan));
    if (q.req->kind == FX_Q_MNI) b += align256((FX_MAXN + 1) * 8);
    if (wants_selection(*q.req)) {
        const size_t k = (size_t)nv / n + 1;
        b += align256(k * n * 4) + align256(k * 8);
    }
    if (q.req->kind == FX_Q_MIS)
        b += align256((size_t)FX_MIS_MAX_EMB * n * 4) + align256((size_t)FX_MIS_MAX_EMB * 8) + align256(sizeof(FxMisOut));
    return b;
}

void carve(FxQuery &q, int64_t nv)
{
    char *p = (char *)q.region;
    auto take = [&](size_t bytes) {
        void *r = p;
        p += align256(bytes);
        return r;
    };
    const int n = q.n;
    const size_t C = (size_t)q.cap;
    q.lev[0].lo = (int64_t *)take(8);
    q.lev[0].len = (int32_t *)take(4);
    q.lev[0].anc = (int8_t *)take(1);
    q.lev[0].off = (int64_t *)take(16);
    q.lev[0].rows = nullptr;
    for (int l = 1; l < n; l++) {
        q.lev[l].rows = (int32_t *)take(C * l * 4);
        q.lev[l].lo = (int64_t *)take(C * 8);
        q.lev[l].len = (int32_t *)take(C * 4);
        q.lev[l].anc = (int8_t *)take(C);
        q.lev[l].off = (int64_t *)take((C + 1) * 8);
    }
    q.lev[n] = FxLevelDev{};
    q.lev[n].rows = (int32_t *)take(C * n * 4);
    const size_t words = ((size_t)nv + 31) / 32;
    const bool mni = q.req->kind == FX_Q_MNI;
    q.U = (uint32_t *)take(words * 4 * (mni ? 1 + n : 1));  // the image bitmaps follow U
    q.img = mni ? q.U + words : nullptr;
    q.mni = mni ? (unsigned long long *)take((FX_MAXN + 1) * 8) : nullptr;
    q.plan = (FxPlan *)take(sizeof(FxPlan));
    q.sel_rows = nullptr;
    q.sel_rank = nullptr;
    if (wants_selection(*q.req)) {
        const size_t k = (size_t)nv / n + 1;
        q.sel_rows = (int32_t *)take(k * n * 4);
        q.sel_rank = (int64_t *)take(k * 8);
    }
    q.mis_rows = nullptr;
    q.mis_hash = nullptr;
    q.mis_out = nullptr;
    if (q.req->kind == FX_Q_MIS) {
        q.mis_rows = (int32_t *)take((size_t)FX_MIS_MAX_EMB * n * 4);
        q.mis_hash = (uint64_t *)take((size_t)FX_MIS_MAX_EMB * 8);
        q.mis_out = (FxMisOut *)take(sizeof(FxMisOut));
    }
}

int deepest_open_level(const FxQuery &q)
{
    for (int l = q.n - 1; l >= 0; l--)
        if (q.cur[l] < q.T[l]) return l;
    return -1;
}

void restart_stack(FxQuery &q, const fx_graph *G)
{
    const uint32_t vl0 = q.hp.plan.vl[0];
    for (int l = 0; l <= q.n; l++) q.T[l] = q.cur[l] = 0, q.nparts[l] = 0;
    q.T[0] = (uint64_t)(G->bptr[vl0 + 1] - G->bptr[vl0]);
    q.nparts[0] = 1;
    q.deep = deepest_open_level(q);
}

}  // namespace

namespace {

bool hip_region_alloc(void **p, size_t bytes)
{
    fx_alloc_calls_made++;
    if (hipMalloc(p, bytes) == hipSuccess) return true;
    (void)hipGetLastError();
    *p = nullptr;
    return false;
}

void hip_region_free(void *p) { (void)hipFree(p); }

}  // namespace

EngineWork::EngineWork()
{
    pool.alloc_fn = hip_region_alloc;
    pool.free_fn = hip_region_free;
}

EngineWork::~EngineWork()
{
    for (auto &L : lane) {
        if (L.done) (void)hipEventDestroy(L.done);
        for (auto &e : L.evk)
            if (e) (void)hipEventDestroy(e);
    }
    if (start_ev) (void)hipEventDestroy(start_ev);
    for (auto &st : own_stream)
        if (st) {
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
    for (auto &c : chain) {
        if (c.exec) (void)hipGraphExecDestroy(c.exec);
        if (c.graph) (void)hipGraphDestroy(c.graph);
    }
    if (chain_stream) {
        (void)hipStreamSynchronize(chain_stream);
        (void)hipStreamDestroy(chain_stream);
    }
}

EngineWork::ChainGraph &EngineWork::chain_graph(const ChainGraphKey &key)
{
    ChainGraph *lru = &chain[0];
    for (auto &c : chain) {
        if (c.exec && c.key == key) {
            c.used = ++chain_clock;
            return c;
        }
        if (c.used < lru->used) lru = &c;
    }
    if (lru->exec) (void)hipGraphExecDestroy(lru->exec);
    if (lru->graph) (void)hipGraphDestroy(lru->graph);
    *lru = ChainGraph{};
    lru->key = key;
    lru->used = ++chain_clock;
    return *lru;
}

fx_status EngineWork::init_events(int lanes)
{
    for (auto &L : lane) {
        if (!L.done) FX_HIP(hipEventCreateWithFlags(&L.done, hipEventDisableTiming));
        for (auto &e : L.evk)
            if (!e) FX_HIP(hipEventCreate(&e));
    }
    if (!start_ev) FX_HIP(hipEventCreateWithFlags(&start_ev, hipEventDisableTiming));
    for (int g = 0; g + 1 < lanes && g < FX_MAX_LANES - 1; g++)
        if (!own_stream[g]) FX_HIP(hipStreamCreateWithFlags(&own_stream[g], hipStreamNonBlocking));
    return FX_OK;
}

fx_status EngineWork::init_chain_stream()
{
    if (!chain_stream) FX_HIP(hipStreamCreateWithFlags(&chain_stream, hipStreamNonBlocking));
    return FX_OK;
}

FxEngine::FxEngine(fx_graph *G, EngineWork *W, hipStream_t s, const EngineParams &p, fx_stats *stats)
    : G_(G), W_(W), s_(s), P_(p), stats_(stats), t0_(std::chrono::steady_clock::now())
{
    for (auto &st : ls_) st = s;
    if (P_.max_active < 1) P_.max_active = 1;
    // a segment's span is a 32-bit count
    P_.step_candidates = std::min<uint64_t>(std::max<uint64_t>(P_.step_candidates, FX_MAX_TILE), 1ull << 31);
    P_.lanes = std::min<int32_t>(std::max<int32_t>(P_.lanes, 1), FX_MAX_LANES);
    for (int k = P_.max_active - 1; k >= 0; k--) free_slots_[k % P_.lanes].push_back(k);
}

FxEngine::~FxEngine()
{
    // after an error, queries may still be running: let their work finish
    // before their stack memory goes back to the pool
    bool busy = false;
    for (int g = 0; g < FX_MAX_LANES; g++) busy = busy || !active_[g].empty() || !deferred_[g].empty();
    if (busy)
        for (int g = 0; g < P_.lanes; g++) (void)hipStreamSynchronize(ls_[g]);
    for (auto &A : active_)
        for (auto &q : A)
            if (q->region) W_->pool.give(q->region, q->region_bytes);
    for (auto &D : deferred_)
        for (auto &r : D) W_->pool.give(r.first, r.second);
}

bool FxEngine::idle() const
{
    if (!pending_.empty()) return false;
    for (const auto &A : active_)
        if (!A.empty()) return false;
    return true;
}

void FxEngine::done(FxRequest *r)
{
    if (on_done) on_done(r);
}

std::unique_ptr<FxQuery> FxEngine::prepare(FxRequest *r) const
{
    auto q = std::make_unique<FxQuery>();
    q->req = r;
    r->status = fx_build_plan(G_, r->pattern, q->hp);
    if (r->status != FX_OK) return q;
    q->n = r->pattern->n;
    if (r->kind != FX_Q_LIST) {
        r->status = fx_tau_checked(r->sigma, r->lambda, q->n, &q->tau);
        if (r->status != FX_OK) return q;
        // the minimum-image and maximum-independent-set thresholds are sigma itself
        if (r->kind == FX_Q_MNI || r->kind == FX_Q_MIS) q->tau = r->sigma;
        q->tau_eff = std::max<int64_t>(q->tau, 1);
    }
    return q;
}

void FxEngine::add(FxRequest *r) { enqueue(prepare(r)); }

fx_status FxEngine::add_all(FxRequest *reqs, size_t count)
{
    std::vector<std::unique_ptr<FxQuery>> qs(count);
    fx_parallel_for((int64_t)count, 256, [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; i++) qs[i] = prepare(&reqs[i]);
    });
    for (size_t i = 0; i < count; i++)
        if (reqs[i].status != FX_OK) {
            // again on this thread, for the error message
            HostPlan hp;
            const fx_status st = fx_build_plan(G_, reqs[i].pattern, hp);
            return st != FX_OK ? st : reqs[i].status;
        }
    for (auto &q : qs) enqueue(std::move(q));
    return FX_OK;
}

void FxEngine::enqueue(std::unique_ptr<FxQuery> q)
{
    FxRequest *r = q->req;
    if (r->status != FX_OK) return done(r);
    fx_result res{};
    res.tau = q->tau;
    res.status = FX_OK;
    if (q->hp.empty) {  // some label never occurs: M is empty
        res.exit = FX_EXIT_EMPTY;
        if (r->kind == FX_Q_LIST) {
            *r->list_count = 0;
        } else {
            res.support = r->kind == FX_Q_VERDICT ? -1 : 0;
            res.embedding_count = r->kind == FX_Q_VERDICT ? -1 : 0;
            *r->out = res;
        }
        return done(r);
    }
    if (r->kind == FX_Q_VERDICT && q->hp.upper_bound < q->tau_eff) {  // support can never reach tau
        res.exit = FX_EXIT_STATIC;
        res.support = -1;
        res.embedding_count = -1;
        *r->out = res;
        return done(r);
    }
    q->phase = (r->kind == FX_Q_LIST || r->kind == FX_Q_MIS) ? PH_LIST : (r->kind == FX_Q_MNI ? PH_COUNT : PH_SUPPORT);
    q->cap = P_.slice_rows;
    q->last_span = (uint32_t)std::min<int64_t>(P_.last_span_init, q->cap);
    for (auto &r : q->rate) r = 1.0;
    pending_.push_back(std::move(q));
}

fx_status FxEngine::finish(FxQuery &q, const FxSummary &S)
{
    FxRequest &r = *q.req;
    if (q.phase == PH_LIST && r.kind == FX_Q_MIS) {
        fx_result res{};
        res.tau = q.tau;
        res.steps = q.steps;
        res.status = FX_OK;
        res.exit = FX_EXIT_END;
        res.embedding_count = q.listed;
        res.device_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0_).count();
        if (q.listed > FX_MIS_MAX_EMB) {
            r.status = fx_fail(FX_ELIMIT, "exact MIS: more than %d embeddings", FX_MIS_MAX_EMB);
        } else {
            FxMisOut mo{};
            hipStream_t st = ls_[q.lane];
            FX_HIP(fx_launch_mis(st, q.mis_rows, (int32_t)q.listed, q.n, q.mis_hash, q.mis_out));
            FX_HIP(hipMemcpyAsync(&mo, q.mis_out, sizeof(mo), hipMemcpyDeviceToHost, st));
            FX_HIP(hipStreamSynchronize(st));
            if (mo.status == 1)
                r.status = fx_fail(FX_ELIMIT, "exact MIS: %d distinct vertex sets, at most %d", mo.sets,
                                   FX_MIS_MAX_SETS);
            else if (mo.status != 0)
                r.status = fx_fail(FX_ELIMIT, "exact MIS: the search needs more than %u nodes", FX_MIS_MAX_NODES);
            res.support = mo.mis;
            res.rounds = (int32_t)std::min<uint64_t>(mo.nodes, INT32_MAX);
        }
        res.frequent = res.support >= q.tau_eff;
        *r.out = res;
    } else if (q.phase == PH_LIST) {
        *r.list_count = q.listed;  // rows written at the last level (a capped slice re-offers the rest)
    } else {
        fx_result res{};
        res.tau = q.tau;
        res.steps = q.steps;
        res.rounds = (int32_t)S.rounds;
        res.alg_bytes = (uint64_t)q.alg_probe_credit + S.alg_scatter;
        res.device_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0_).count();
        res.status = FX_OK;
        res.exit = q.exit;
        if (q.exit == FX_EXIT_REACHED) stats_->exits_reached++;
        if (q.exit == FX_EXIT_BOUND) stats_->exits_bound++;
        if (r.kind == FX_Q_VERDICT) {
            res.frequent = (int64_t)S.support >= q.tau_eff;
            res.support = res.frequent ? q.tau : -1;
            res.embedding_count = -1;
        } else {
            res.support = (int64_t)S.support;
            if (r.kind == FX_Q_MNI) {
                unsigned long long m = 0;
                hipStream_t st = ls_[q.lane];
                FX_HIP(fx_launch_mni(st, q.img, ((uint64_t)G_->nv + 31) / 32, q.n, q.mni, q.mni + FX_MAXN));
                FX_HIP(hipMemcpyAsync(&m, q.mni + FX_MAXN, 8, hipMemcpyDeviceToHost, st));
                FX_HIP(hipStreamSynchronize(st));
                res.support = (int64_t)m;
            }
            res.frequent = res.support >= q.tau_eff;
            const bool sat = (int64_t)S.count >= P_.count_cap;
            res.count_saturated = sat;
            res.embedding_count = sat ? P_.count_cap : (int64_t)S.count;
            if (!sat && !P_.no_digest) {
                res.digest[0] = S.digest0;
                res.digest[1] = S.digest1;
            }
            if (r.kind == FX_Q_FULL) {
                res.sel_digest[0] = S.sel_d0;
                res.sel_digest[1] = S.sel_d1;
            }
            if (wants_selection(r) && S.support > 0) {
                const int64_t k = (int64_t)S.support;
                std::vector<int32_t> rows((size_t)k * q.n);
                std::vector<int64_t> rank(k);
                hipStream_t st = ls_[q.lane];
                FX_HIP(hipMemcpyAsync(rows.data(), q.sel_rows, rows.size() * 4, hipMemcpyDeviceToHost, st));
                FX_HIP(hipMemcpyAsync(rank.data(), q.sel_rank, rank.size() * 8, hipMemcpyDeviceToHost, st));
                FX_HIP(hipStreamSynchronize(st));
                std::vector<int64_t> idx(k);
                std::iota(idx.begin(), idx.end(), 0);
                std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return rank[a] < rank[b]; });
                const int64_t w = std::min<int64_t>(k, r.selected_cap);
                for (int64_t i = 0; i < w; i++)
                    memcpy(r.selected + i * q.n, rows.data() + idx[i] * q.n, (size_t)q.n * 4);
            }
        }
        *r.out = res;
    }
    stats_->probe_alg_bytes += (uint64_t)q.alg_probe_credit;
    stats_->scatter_alg_bytes += S.alg_scatter;
    stats_->probe_ref_bytes += (uint64_t)q.ref_probe_credit;
    stats_->probe_ref_row_bytes += (uint64_t)q.ref_row_credit;
    stats_->scatter_ref_bytes += S.ref_scatter;
    stats_->greedy_ref_bytes += S.ref_greedy;
    stats_->queries++;
    W_->pool.give(q.region, q.region_bytes);
    q.region = nullptr;
    free_slots_[q.slot % P_.lanes].push_back(q.slot);  // slots stay with their lane (slot mod lanes)
    q.slot = -1;
    done(&r);
    return FX_OK;
}

// Admission into lane g: as many pending queries as its slots and memory allow.
fx_status FxEngine::admit(int g)
{
    const int64_t nv = G_->nv;
    const uint64_t u_words = ((uint64_t)nv + 31) / 32;
    EngineLane &L = W_->lane[g];
    FxInit *inits = L.inits_h.as<FxInit>();
    FxSummary *sums_d = W_->sums_d.as<FxSummary>();
    int ninit = 0;
    while (!pending_.empty() && !free_slots_[g].empty()) {
        FxQuery &q = *pending_.front();
        const size_t bytes = region_size(q, nv);
        if (!W_->pool.take(bytes, &q.region)) {
            // wait until running queries free their regions
            bool running = ninit > 0;
            for (const auto &A : active_) running = running || !A.empty();
            if (running) break;
            // it cannot fit even alone
            q.req->status = fx_fail(FX_ENOMEM, "query region of %zu bytes does not fit in the %zu-byte budget",
                                    bytes, W_->pool.budget);
            FxRequest *r = q.req;
            pending_.pop_front();
            done(r);
            continue;
        }
        q.region_bytes = bytes;
        carve(q, nv);
        q.slot = free_slots_[g].back();
        q.lane = g;
        free_slots_[g].pop_back();
        FxInit &I = inits[ninit++];
        I.plan = q.hp.plan;
        I.plan_dst = q.plan;
        I.lev0 = q.lev[0];
        I.U = q.U;
        I.sum = sums_d + q.slot;
        I.u_words = u_words * (q.req->kind == FX_Q_MNI ? 1 + (uint64_t)q.n : 1);  // U and the image bitmaps
        I.clear_u = 1;
        I.clear_sum = 1;
        restart_stack(q, G_);
        active_[g].push_back(std::move(pending_.front()));
        pending_.pop_front();
    }
    if (ninit) {
        FX_HIP(hipMemcpyAsync(L.inits_d.p, inits, (size_t)ninit * sizeof(FxInit), hipMemcpyHostToDevice, ls_[g]));
        FX_HIP(fx_launch_init(ls_[g], G_->dev, L.inits_d.as<FxInit>(), ninit));
    }
    return FX_OK;
}

// Moves q's stack to a region with new_cap rows per level (when the pool has
// room; otherwise q keeps its stack).  Every level that still has candidates
// left is copied on the stream, so the next step sees the same stack with
// room for larger slices.
fx_status FxEngine::promote(FxQuery &q, int64_t new_cap)
{
    const int64_t nv = G_->nv;
    FxQuery old;
    old.n = q.n;
    old.req = q.req;
    old.cap = q.cap;
    old.region = q.region;
    old.region_bytes = q.region_bytes;
    for (int l = 0; l <= q.n; l++) old.lev[l] = q.lev[l];
    old.U = q.U;
    old.plan = q.plan;
    old.sel_rows = q.sel_rows;
    old.sel_rank = q.sel_rank;
    old.mis_rows = q.mis_rows;
    q.cap = new_cap;
    const size_t bytes = region_size(q, nv);
    void *region = nullptr;
    if (!W_->pool.take(bytes, &region)) {
        q.cap = old.cap;
        return FX_OK;
    }
    q.region = region;
    q.region_bytes = bytes;
    carve(q, nv);
    auto cp = [&](void *dst, const void *src, size_t b) -> fx_status {
        if (b) FX_HIP(hipMemcpyAsync(dst, src, b, hipMemcpyDeviceToDevice, ls_[q.lane]));
        return FX_OK;
    };
    FX_TRY(cp(q.lev[0].lo, old.lev[0].lo, 8));
    FX_TRY(cp(q.lev[0].len, old.lev[0].len, 4));
    FX_TRY(cp(q.lev[0].anc, old.lev[0].anc, 1));
    FX_TRY(cp(q.lev[0].off, old.lev[0].off, 16));
    const int deep = q.deep;
    for (int l = 1; l <= deep; l++) {
        const size_t np = (size_t)q.nparts[l];
        if (np == 0) continue;
        FX_TRY(cp(q.lev[l].rows, old.lev[l].rows, np * l * 4));
        FX_TRY(cp(q.lev[l].lo, old.lev[l].lo, np * 8));
        FX_TRY(cp(q.lev[l].len, old.lev[l].len, np * 4));
        FX_TRY(cp(q.lev[l].anc, old.lev[l].anc, np));
        FX_TRY(cp(q.lev[l].off, old.lev[l].off, (np + 1) * 8));
    }
    FX_TRY(cp(q.U, old.U, ((size_t)nv + 31) / 32 * 4 * (q.img ? 1 + (size_t)q.n : 1)));  // U and images
    FX_TRY(cp(q.plan, old.plan, sizeof(FxPlan)));
    if (q.sel_rows) {
        const size_t k = (size_t)nv / q.n + 1;
        FX_TRY(cp(q.sel_rows, old.sel_rows, k * q.n * 4));
        FX_TRY(cp(q.sel_rank, old.sel_rank, k * 8));
    }
    if (q.mis_rows && q.listed > 0)  // the embeddings collected so far (exact-MIS mode)
        FX_TRY(cp(q.mis_rows, old.mis_rows, (size_t)std::min<int64_t>(q.listed, FX_MIS_MAX_EMB) * q.n * 4));
    // the copies read the old region on this lane's stream: it goes back to
    // the pool once the lane's next step has been waited for (the other lanes
    // run on other streams and could reuse it too early)
    deferred_[q.lane].push_back({old.region, old.region_bytes});
    q.last_span = (uint32_t)std::min<int64_t>(P_.last_span_init, q.cap);
    stats_->promotions++;
    return FX_OK;
}

fx_status FxEngine::step()
{
    using clk = std::chrono::steady_clock;
    const auto h0 = clk::now();
    double waited = 0;
    struct HostTime {  // adds this step's host time to the statistics on every exit
        fx_stats *st;
        clk::time_point h0;
        double *waited;
        ~HostTime()
        {
            const double ms = std::chrono::duration<double, std::milli>(clk::now() - h0).count();
            st->host_ms += ms - *waited;
            st->wait_ms += *waited;
        }
    } host_time{stats_, h0, &waited};
    if (!buffers_ready_) {  // grow-only buffers sized for these parameters
        const int32_t A = P_.max_active;
        const uint64_t tile = (uint64_t)FX_BS * P_.items;
        const uint64_t max_blocks = (P_.step_candidates + tile - 1) / tile + (uint64_t)A;
        FX_TRY(W_->sums_d.ensure((size_t)A * sizeof(FxSummary)));
        for (int g = 0; g < P_.lanes; g++) {
            EngineLane &L = W_->lane[g];
            FX_TRY(L.cand.ensure(max_blocks * cand_tile_bytes(P_.items)));
            FX_TRY(L.bcnt.ensure(max_blocks * 4));
            FX_TRY(L.boff.ensure((max_blocks + 1) * 8));
            FX_TRY(L.lsum.ensure(max_blocks * 8));
            FX_TRY(L.loff.ensure((max_blocks + 1) * 8));
            FX_TRY(L.sstat.ensure((size_t)scan_state_words((uint32_t)max_blocks) * 8));
            FX_TRY(L.tmap.ensure(max_blocks * sizeof(FxTile)));
            FX_TRY(L.stage_d.ensure(stage_bytes(A, A)));
            FX_TRY(L.stage_h.ensure(stage_bytes(A, A)));
            FX_TRY(L.inits_d.ensure((size_t)A * sizeof(FxInit)));
            FX_TRY(L.inits_h.ensure((size_t)A * sizeof(FxInit)));
            FX_TRY(L.sums_h.ensure((size_t)A * sizeof(FxSummary)));
        }
        FX_TRY(W_->init_events(P_.lanes));
        if (P_.lanes > 1) {
            // lanes 1.. start after whatever the caller queued on the engine's stream
            FX_HIP(hipEventRecord(W_->start_ev, s_));
            for (int g = 1; g < P_.lanes; g++) {
                ls_[g] = W_->own_stream[g - 1];
                FX_HIP(hipStreamWaitEvent(ls_[g], W_->start_ev, 0));
            }
        }
        buffers_ready_ = true;
    }
    if (chain_ready()) return chain_step(waited);
    const int g = lane_;
    lane_ = (lane_ + 1) % P_.lanes;
    if (in_flight_[g]) FX_TRY(collect(g, waited));
    FX_TRY(admit(g));
    if (!active_[g].empty()) FX_TRY(launch(g));
    return FX_OK;
}

// Moves the stacks of long-running queries that now have the device nearly
// to themselves to a larger capacity (room for slices of their share of a
// step).  In the support phase the slice size is also the granularity at
// which selections prune the search through U: larger slices expand partials
// that a selection would have removed (measured: twice the probe work on
// cl1m).  A support-phase stack grows only while U has removed under 1/64 of
// its candidates -- or, for a VERDICT query that has run lone_after steps,
// once at most lone_queries queries are left: then the device is idle between
// their small steps, and fewer, larger steps finish sooner despite the extra
// expansion (cl1m: half the steps, 40% more patterns/s).  FULL queries keep
// the rule: their batch tail also holds other queries' counting, and the
// extra expansion cost 10% there; short queries keep it too (a single VERDICT
// call grew from the start and ran 3x slower).
fx_status FxEngine::grow_stacks(std::vector<FxQuery *> &qs, uint64_t n_open)
{
    const uint64_t share = P_.step_candidates / std::max<uint64_t>(n_open, 1);
    const bool lone = P_.lone_growth && n_open <= (uint64_t)std::max<int32_t>(P_.lone_queries, 0);
    for (FxQuery *qp : qs) {
        FxQuery &q = *qp;
        const bool free_growth = lone && q.req->kind == FX_Q_VERDICT && q.steps >= P_.lone_after;
        const bool u_ok = q.phase != PH_SUPPORT || (q.probed_support > 0 && q.last_ufiltered * 64 <= q.probed_support);
        if (!free_growth && !u_ok) continue;
        if (q.steps < P_.promote_after || q.cap >= kPromoteCap || share < 4 * (uint64_t)q.cap) continue;
        if (q.deep < 0) continue;
        uint64_t left = 0;  // largest candidate range still open: no slice needs more rows
        for (int l = 0; l < q.n; l++) left = std::max<uint64_t>(left, q.T[l] - q.cur[l]);
        int64_t nc = q.cap;
        while (nc < kPromoteCap && (uint64_t)nc * 2 <= share && (uint64_t)nc < left) nc *= 2;
        if (nc > q.cap) {
            const uint64_t before = stats_->promotions;
            FX_TRY(promote(q, nc));
            if (!u_ok && stats_->promotions > before) stats_->lone_promotions++;  // only the lone rule allowed it
        }
    }
    return FX_OK;
}

// Builds and launches lane g's next device step: one segment per active
// query of the lane, within the step's candidate budget, then the copy of
// the summaries and the lane's completion event.
fx_status FxEngine::launch(int g)
{
    EngineLane &L = W_->lane[g];
    auto &act = active_[g];
    step_view_[g].clear();
    // the stage buffer holds the workgroup starts, then the segment table,
    // so one copy uploads both
    const size_t seg_off = stage_off(act.size());
    uint32_t *blk0 = L.stage_h.as<uint32_t>();
    FxSeg *segs = (FxSeg *)((char *)L.stage_h.p + seg_off);
    FxSummary *sums_d = W_->sums_d.as<FxSummary>();
    int nsegs = 0;
    uint64_t budget = P_.step_candidates;
    uint32_t nblocks = 0;
    int any_inner = 0, any_greedy = 0, maxn = 1;
    const size_t A = act.size();
    uint64_t mine = 0;  // open queries of this lane; the other lanes' counts are from their last launches
    for (auto &qp : act) {
        qp->seg_l = -1;
        mine += qp->deep >= 0;
    }
    nopen_[g] = mine;
    uint64_t n_open = mine;  // a query gets one step of its lane in every `lanes` steps
    for (int h = 0; h < P_.lanes; h++)
        if (h != g) n_open += nopen_[h];
    // a query's fair share of the step; a slice may take more candidates
    // than its level holds rows when few of them pass (the row cap bounds
    // what is written, see k_scatter)
    const uint64_t share = P_.step_candidates / std::max<uint64_t>(n_open, 1);
    {
        std::vector<FxQuery *> qs;
        for (auto &qp : act) qs.push_back(qp.get());
        FX_TRY(grow_stacks(qs, n_open));
    }
    for (size_t k = 0; k < A && budget > 0; k++) {
        FxQuery &q = *act[(rot_[g] + k) % A];
        const int l = q.deep;
        if (l < 0) continue;
        const bool last = (l == q.n - 1);
        int kind, flags = 0;
        uint64_t out_cap = (uint64_t)q.cap;  // rows the segment may write
        if (q.phase == PH_SUPPORT) {
            flags = FX_PROBE_UFILTER | (q.hp.symmetric ? FX_PROBE_SYM : 0);
            kind = last ? FX_SEG_GREEDY : FX_SEG_INNER;
            if (last) out_cap = std::min<uint64_t>(q.last_span, (uint64_t)q.cap);
        } else if (q.phase == PH_COUNT) {
            // without a digest, a leaf last vertex is counted in closed form
            // from the partials of vertex n-2 (level n-1 is never built)
            // (the minimum-image support needs every last-vertex image: no closed form)
            const bool mni = q.req->kind == FX_Q_MNI;
            const bool leaf = P_.no_digest && !mni && q.n >= 2 && q.hp.plan.nback[q.n - 1] == 1;
            const bool end = leaf ? (l == q.n - 2) : last;
            flags = end ? (leaf ? FX_PROBE_LEAF
                                : (FX_PROBE_COUNT | (P_.no_digest ? 0 : FX_PROBE_HASH) | (mni ? FX_PROBE_IMAGES : 0)))
                        : 0;
            kind = end ? FX_SEG_COUNT : FX_SEG_INNER;
        } else {
            kind = last ? FX_SEG_LIST : FX_SEG_INNER;
        }
        uint64_t want;
        if (kind == FX_SEG_COUNT) {
            want = std::max<uint64_t>(kCountSpan, share);
        } else {
            // expected passes = rate * span: aim at kFill of the row cap
            const double r = std::max(q.rate[l], 1e-9);
            want = r >= 1.0 ? out_cap : (uint64_t)std::min(kFill * (double)out_cap / r, 2147483648.0);
            want = std::min<uint64_t>(std::max<uint64_t>(want, out_cap), std::max<uint64_t>(out_cap, share));
        }
        const uint64_t span = std::min<uint64_t>(std::min<uint64_t>(q.T[l] - q.cur[l], want), budget);
        if (span == 0) continue;
        if (P_.ref_bytes) flags |= FX_PROBE_REF;
        FxSeg &S = segs[nsegs];
        S.in = q.lev[l];
        S.out = q.lev[l + 1];
        S.plan = q.plan;
        S.U = q.U;
        S.sum = sums_d + q.slot;
        S.sel_rows = q.sel_rows;
        S.sel_rank = q.sel_rank;
        S.img = q.img;
        S.img_words = ((uint64_t)G_->nv + 31) / 32;
        S.nparts = q.nparts[l];
        S.t0 = q.cur[l];
        S.rank_base = q.rank_base;
        S.span = (uint32_t)span;
        S.out_cap = (uint32_t)std::min<uint64_t>(out_cap, 0xffffffffu);
        S.blk0 = nblocks;
        S.n = q.n;
        S.l = l;
        S.flags = flags;
        S.kind = kind;
        blk0[nsegs] = nblocks;
        nblocks += (uint32_t)((span + (uint64_t)FX_BS * P_.items - 1) / ((uint64_t)FX_BS * P_.items));
        budget -= span;
        if (P_.check_steps) {
            FxStepSeg v{};
            v.n = S.n;
            v.l = S.l;
            v.kind = S.kind;
            v.leaf = (S.flags & FX_PROBE_LEAF) != 0;
            v.t0 = S.t0;
            v.span = S.span;
            v.level_total = q.T[l];
            v.nparts = S.nparts;
            v.cap = q.cap;
            v.out_cap = S.out_cap;
            v.blk0 = S.blk0;
            step_view_[g].push_back(v);
        }
        q.seg_l = l;
        q.seg_kind = kind;
        q.seg_t0 = q.cur[l];
        q.seg_span = (uint32_t)span;
        any_inner |= kind == FX_SEG_INNER;
        any_greedy |= kind == FX_SEG_GREEDY;
        maxn = std::max(maxn, q.n);
        nsegs++;
    }
    rot_[g]++;
    if (nsegs == 0) return fx_fail(FX_EDEVICE, "engine stalled with %zu active queries", A);
    blk0[nsegs] = nblocks;
    if (P_.check_steps) {  // every range the kernels will index, against the buffers sized for it
        const std::vector<FxStepSeg> &view = step_view_[g];
        const uint64_t tile = (uint64_t)FX_BS * P_.items;
        const uint64_t max_blocks = L.bcnt.bytes / 4;
        const std::string err = fx_check_segments(view, nblocks, (uint32_t)tile, max_blocks, P_.step_candidates);
        if (!err.empty()) return fx_fail(FX_EDEVICE, "step check failed before the launch: %s", err.c_str());
        step_blocks_[g] = nblocks;
    }
    hipStream_t st = ls_[g];
    FX_HIP(hipMemcpyAsync(L.stage_d.p, L.stage_h.p, seg_off + (size_t)nsegs * sizeof(FxSeg), hipMemcpyHostToDevice,
                          st));
    hipEvent_t *ev = P_.timing ? L.evk : nullptr;
    // small steps (a lone query, a single call) take the single-pass form:
    // two launches fewer per step, and few tiles to wait on in its ordered write
    const int fused = (P_.fused || nblocks <= (uint32_t)std::max<int32_t>(P_.fused_below, 0)) ? 1 : 0;
    fused_[g] = fused;
    FX_HIP(fx_launch_step(st, G_->dev, (const FxSeg *)((char *)L.stage_d.p + seg_off), L.stage_d.as<uint32_t>(),
                          nsegs, nblocks, P_.items, maxn, L.tmap.as<FxTile>(), L.cand.as<int32_t>(), L.bcnt.as<uint32_t>(),
                          L.boff.as<uint64_t>(), L.lsum.as<uint64_t>(), L.loff.as<uint64_t>(), L.sstat.as<uint64_t>(),
                          ev ? ev[0] : nullptr,
                          ev ? ev[1] : nullptr, ev ? ev[2] : nullptr, ev ? ev[3] : nullptr, ev ? ev[4] : nullptr,
                          ev ? ev[5] : nullptr, any_inner, any_greedy, fused));
    int hi = 0;
    for (auto &qp : act) hi = std::max(hi, qp->slot + 1);
    FX_HIP(hipMemcpyAsync(L.sums_h.p, sums_d, (size_t)hi * sizeof(FxSummary), hipMemcpyDeviceToHost, st));
    FX_HIP(hipEventRecord(L.done, st));
    in_flight_[g] = true;
    any_greedy_[g] = any_greedy;
    return FX_OK;
}

// Waits for lane g's device step, advances its queries, retires the finished
// ones and moves FULL queries to their counting phase.
fx_status FxEngine::collect(int g, double &waited)
{
    EngineLane &L = W_->lane[g];
    auto &act = active_[g];
    {
        const auto w0 = std::chrono::steady_clock::now();
        FX_HIP(hipEventSynchronize(L.done));
        waited += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - w0).count();
    }
    in_flight_[g] = false;
    if (P_.check_steps) {  // the tile map the device built for this step
        std::vector<FxStepTile> tiles(step_blocks_[g]);
        static_assert(sizeof(FxStepTile) == sizeof(FxTile), "tile views mirror FxTile");
        if (!tiles.empty()) {
            FX_HIP(hipMemcpyAsync(tiles.data(), L.tmap.p, tiles.size() * sizeof(FxTile), hipMemcpyDeviceToHost, ls_[g]));
            FX_HIP(hipStreamSynchronize(ls_[g]));
        }
        const std::string err = fx_check_tiles(step_view_[g], tiles, (uint32_t)(FX_BS * P_.items));
        if (!err.empty()) return fx_fail(FX_EDEVICE, "step check failed after the step: %s", err.c_str());
    }
    for (auto &r : deferred_[g]) W_->pool.give(r.first, r.second);
    deferred_[g].clear();
    const FxSummary *sums_h = L.sums_h.as<FxSummary>();
    stats_->steps++;
    stats_->syncs++;
    stats_->probe_launches++;
    if (!fused_[g]) stats_->scatter_launches++;
    if (any_greedy_[g]) stats_->greedy_launches++;
    if (P_.timing) {
        float ms = 0;
        FX_HIP(hipEventElapsedTime(&ms, L.evk[0], L.evk[1]));
        stats_->probe_ms += ms;
        if (!fused_[g]) {
            FX_HIP(hipEventElapsedTime(&ms, L.evk[2], L.evk[3]));
            stats_->scatter_ms += ms;
        }
        FX_HIP(hipEventElapsedTime(&ms, L.evk[4], L.evk[5]));
        stats_->greedy_ms += ms;
    }

    // ---- advance every query that took part
    for (auto &qp : act) {
        FxQuery &q = *qp;
        if (q.seg_l < 0) continue;
        const FxSummary &S = sums_h[q.slot];
        if (S.error) return fx_fail(FX_EDEVICE, "device consistency check failed (greedy round limit)");
        const int l = q.seg_l;
        const uint64_t taken = S.consumed;
        if (taken == 0 || taken > q.seg_span)
            return fx_fail(FX_EDEVICE, "internal: segment took %llu of %u candidates", (unsigned long long)taken,
                           q.seg_span);
        q.cur[l] = q.seg_t0 + taken;
        stats_->reoffered += q.seg_span - taken;
        stats_->probed += q.seg_span;
        if (q.phase == PH_SUPPORT) q.probed_support += q.seg_span;
        q.rate[l] = (double)S.passes / (double)q.seg_span;
        q.last_ufiltered = S.ufiltered;
        q.alg_probe_credit += (double)(S.alg_probe - q.alg_probe_seen) * (double)taken / (double)q.seg_span;
        q.alg_probe_seen = S.alg_probe;
        q.ref_probe_credit += (double)(S.ref_probe - q.ref_probe_seen) * (double)taken / (double)q.seg_span;
        q.ref_probe_seen = S.ref_probe;
        q.ref_row_credit += (double)(S.ref_probe_row - q.ref_row_seen) * (double)taken / (double)q.seg_span;
        q.ref_row_seen = S.ref_probe_row;
        q.steps++;
        q.seg_l = -1;
        const uint64_t N = S.total_out;
        if (q.seg_kind == FX_SEG_INNER) {
            q.nparts[l + 1] = (int64_t)N;
            q.T[l + 1] = S.t_next;
            q.cur[l + 1] = 0;
        } else if (q.seg_kind == FX_SEG_GREEDY) {
            q.rank_base += (int64_t)N;
        } else if (q.seg_kind == FX_SEG_LIST && q.req->kind == FX_Q_MIS) {
            // collected on the device; past the limit the query ends with an error
            if (q.listed + (int64_t)N <= FX_MIS_MAX_EMB && N > 0)
                FX_HIP(hipMemcpyAsync(q.mis_rows + q.listed * q.n, q.lev[q.n].rows, (size_t)N * q.n * 4,
                                      hipMemcpyDeviceToDevice, ls_[g]));
            q.listed += (int64_t)N;
        } else if (q.seg_kind == FX_SEG_LIST) {
            FxRequest &r = *q.req;
            const int64_t take = std::min<int64_t>((int64_t)N, std::max<int64_t>(0, r.list_cap - q.listed));
            if (take > 0) {
                FX_HIP(hipMemcpyAsync(r.list_rows + q.listed * q.n, q.lev[q.n].rows, (size_t)take * q.n * 4,
                                      hipMemcpyDeviceToHost, ls_[g]));
                FX_HIP(hipStreamSynchronize(ls_[g]));
            }
            q.listed += (int64_t)N;
        }
        q.deep = deepest_open_level(q);
    }
    // ---- retire finished queries, move FULL queries to their counting phase
    for (size_t k = 0; k < act.size();) {
        FxQuery &q = *act[k];
        const FxSummary &S = sums_h[q.slot];
        bool fin = false;
        if (q.phase == PH_SUPPORT && q.req->kind == FX_Q_VERDICT) {
            const int64_t sup = (int64_t)S.support;
            if (sup >= q.tau_eff) {  // early termination at tau (Section 3.1.1)
                fin = true;
                q.exit = FX_EXIT_REACHED;
            } else if (q.deep >= 0) {
                // exactly infrequent once the selections still possible cannot
                // reach tau: a later selection has its own root (one per root,
                // Section 3.2.2) among the level-0 candidates not yet expanded
                // and the roots of the current level-1 slice (every open partial
                // descends from one of them); and all selections are disjoint,
                // so at most the upper bound of Section 3.1.2 exist in total
                uint64_t roots = q.T[0] - q.cur[0];
                if (q.deep >= 1) roots += (uint64_t)q.nparts[1];
                const int64_t room = std::max<int64_t>(q.hp.upper_bound - sup, 0);
                const int64_t possible = std::min<int64_t>((int64_t)std::min<uint64_t>(roots, INT64_MAX), room);
                if (sup + possible < q.tau_eff) {
                    fin = true;
                    q.exit = FX_EXIT_BOUND;
                }
            }
        }
        // (the minimum-image support needs every embedding: the cap only caps its count)
        if (q.phase == PH_COUNT && q.req->kind != FX_Q_MNI && (int64_t)S.count >= P_.count_cap) fin = true;
        if (q.req->kind == FX_Q_MIS && q.listed > FX_MIS_MAX_EMB) fin = true;  // reported as FX_ELIMIT
        if (!fin && q.deep < 0) {
            if (q.phase == PH_SUPPORT && q.req->kind == FX_Q_FULL) {
                q.phase = PH_COUNT;  // level 0 is unchanged; restart the cursors
                restart_stack(q, G_);
            } else {
                fin = true;
            }
        }
        if (fin) {
            FX_TRY(finish(q, sums_h[q.slot]));
            act[k] = std::move(act.back());
            act.pop_back();
        } else {
            k++;
        }
    }
    return FX_OK;
}

// ---------------------------------------------------------------------------
// Device-scheduled chains
// ---------------------------------------------------------------------------

namespace {

constexpr size_t kChainCtlBytes = 256;

size_t chain_layout(int32_t max_q, size_t *cq_off, size_t *blk0_off, size_t *segs_off)
{
    *cq_off = kChainCtlBytes;
    *blk0_off = align256(*cq_off + (size_t)max_q * sizeof(FxChainQuery));
    *segs_off = align256(*blk0_off + ((size_t)max_q + 1) * 4);
    return align256(*segs_off + (size_t)max_q * sizeof(FxSeg));
}

}  // namespace

// Chains run once no query waits for admission, at most chain_queries are in
// flight, and no query lists its embeddings (a listing copies rows out every
// step).  Per-kernel timing needs the host-scheduled steps.
bool FxEngine::chain_ready() const
{
    if (P_.chain_queries <= 0 || P_.chain_steps <= 0 || P_.timing || P_.check_steps || !pending_.empty())
        return false;
    size_t total = 0;
    for (int g = 0; g < P_.lanes; g++) {
        total += active_[g].size();
        for (const auto &q : active_[g])
            if (q->phase == PH_LIST) return false;
    }
    return total > 0 && total <= (size_t)P_.chain_queries;
}

// One chain: every lane's step in flight is collected, the open queries'
// state goes to the device, the captured chain of chain_steps steps runs
// (its scheduler kernel advances, retires and schedules the queries between
// steps), and the state comes back: finished queries are retired here, the
// others continue in the next chain or in host-scheduled steps.
fx_status FxEngine::chain_step(double &waited)
{
    for (int g = 0; g < P_.lanes; g++)
        if (in_flight_[g]) FX_TRY(collect(g, waited));
    std::vector<FxQuery *> qs;
    uint64_t n_open = 0;
    int maxn = 1;
    for (int g = 0; g < P_.lanes; g++)
        for (auto &qp : active_[g]) {
            qs.push_back(qp.get());
            n_open += qp->deep >= 0;
            maxn = std::max(maxn, qp->n);
        }
    if (qs.empty()) return FX_OK;
    FX_TRY(grow_stacks(qs, n_open));
    const int32_t max_q = P_.chain_queries;
    size_t cq_off, blk0_off, segs_off;
    const size_t bytes = chain_layout(max_q, &cq_off, &blk0_off, &segs_off);
    FX_TRY(W_->chain_d.ensure(bytes));
    FX_TRY(W_->chain_h.ensure(bytes));
    char *hb = (char *)W_->chain_h.p;
    char *db = (char *)W_->chain_d.p;
    FxChainCtl *ctl_h = (FxChainCtl *)hb;
    FxChainQuery *cq_h = (FxChainQuery *)(hb + cq_off);
    memset(ctl_h, 0, sizeof(FxChainCtl));
    ctl_h->nq = (int32_t)qs.size();
    ctl_h->budget = P_.step_candidates;
    FxSummary *sums_d = W_->sums_d.as<FxSummary>();
    const uint64_t words = ((uint64_t)G_->nv + 31) / 32;
    for (size_t i = 0; i < qs.size(); i++) {
        FxQuery &q = *qs[i];
        FxChainQuery &c = cq_h[i];
        memset(&c, 0, sizeof(c));
        for (int l = 0; l <= q.n; l++) c.lev[l] = q.lev[l];
        c.plan = q.plan;
        c.U = q.U;
        c.sum = sums_d + q.slot;
        c.sel_rows = q.sel_rows;
        c.sel_rank = q.sel_rank;
        c.img = q.img;
        c.img_words = words;
        c.cap = q.cap;
        c.tau_eff = q.tau_eff;
        c.upper_bound = q.hp.upper_bound;
        c.count_cap = P_.count_cap;
        c.bucket0 = (uint64_t)(G_->bptr[q.hp.plan.vl[0] + 1] - G_->bptr[q.hp.plan.vl[0]]);
        c.last_span = q.last_span;
        c.n = q.n;
        c.verdict = q.req->kind == FX_Q_VERDICT;
        c.mni = q.req->kind == FX_Q_MNI;
        c.full = q.req->kind == FX_Q_FULL;
        c.sym = q.hp.symmetric;
        c.leaf_count = P_.no_digest && !c.mni && q.n >= 2 && q.hp.plan.nback[q.n - 1] == 1;
        c.hash = !P_.no_digest;
        c.ref_bytes = P_.ref_bytes;
        c.phase = q.phase == PH_SUPPORT ? FX_CQ_SUPPORT : FX_CQ_COUNT;
        c.deep = q.deep;
        c.exit = q.exit;
        c.steps = q.steps;
        for (int l = 0; l <= FX_MAXN; l++) {
            c.T[l] = q.T[l];
            c.cur[l] = q.cur[l];
            c.nparts[l] = q.nparts[l];
            c.rate[l] = q.rate[l];
        }
        c.rank_base = q.rank_base;
        c.probed_support = q.probed_support;
        c.alg_probe_seen = q.alg_probe_seen;
        c.alg_probe_credit = q.alg_probe_credit;
        c.ref_probe_seen = q.ref_probe_seen;
        c.ref_probe_credit = q.ref_probe_credit;
        c.ref_row_seen = q.ref_row_seen;
        c.ref_row_credit = q.ref_row_credit;
        c.seg_l = -1;
    }
    // the chain runs on its own stream, after everything queued on the lanes
    FX_TRY(W_->init_chain_stream());
    hipStream_t cs = W_->chain_stream;
    for (int g = 0; g < P_.lanes; g++) {
        FX_HIP(hipEventRecord(W_->lane[g].done, ls_[g]));
        FX_HIP(hipStreamWaitEvent(cs, W_->lane[g].done, 0));
    }
    EngineLane &L = W_->lane[0];
    ChainGraphKey key{};
    key.graph = G_;
    key.dev = G_->dev;
    key.items = P_.items;
    key.width = maxn <= 4 ? 4 : (maxn <= 8 ? 8 : FX_MAXN);
    // chains start short and double while queries stay open: a query that
    // ends after a few steps does not sit through a long chain's empty steps
    key.steps = chain_k_ = std::min<int32_t>(chain_k_ ? 2 * chain_k_ : 2, std::max<int32_t>(P_.chain_steps, 1));
    key.max_q = max_q;
    key.fused = P_.fused ? 1 : 0;
    const void *bufs[9] = {hb, db, L.tmap.p, L.cand.p, L.bcnt.p, L.boff.p, L.lsum.p, L.loff.p, L.sstat.p};
    memcpy(key.bufs, bufs, sizeof(bufs));
    key.bytes = bytes;
    EngineWork::ChainGraph &cg = W_->chain_graph(key);
    if (!cg.exec) {
        if (cg.graph) (void)hipGraphDestroy(cg.graph);
        cg.graph = nullptr;
        FX_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipMemcpyAsync(db, hb, bytes, hipMemcpyHostToDevice, cs);
        if (e == hipSuccess)
            e = fx_launch_chain(cs, G_->dev, (FxChainQuery *)(db + cq_off), (FxChainCtl *)db, max_q, key.steps,
                                (FxSeg *)(db + segs_off), (uint32_t *)(db + blk0_off), P_.items, key.width,
                                L.tmap.as<FxTile>(), L.cand.as<int32_t>(), L.bcnt.as<uint32_t>(),
                                L.boff.as<uint64_t>(), L.lsum.as<uint64_t>(), L.loff.as<uint64_t>(),
                                L.sstat.as<uint64_t>(), key.fused);
        if (e == hipSuccess) e = hipMemcpyAsync(hb, db, bytes, hipMemcpyDeviceToHost, cs);
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fx_fail(FX_EDEVICE, "capturing the device-scheduled chain failed: %s",
                           hipGetErrorString(e != hipSuccess ? e : e2));
        }
        cg.graph = graph;
        const hipError_t e3 = hipGraphInstantiate(&cg.exec, graph, nullptr, nullptr, 0);
        if (e3 != hipSuccess) {
            cg.exec = nullptr;
            return fx_fail(FX_EDEVICE, "instantiating the device-scheduled chain failed: %s", hipGetErrorString(e3));
        }
    }
    FX_HIP(hipGraphLaunch(cg.exec, cs));
    {
        const auto w0 = std::chrono::steady_clock::now();
        FX_HIP(hipStreamSynchronize(cs));
        waited += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - w0).count();
    }
    // stack regions freed by promotions: the chain has run past them
    for (int g = 0; g < FX_MAX_LANES; g++) {
        for (auto &r : deferred_[g]) W_->pool.give(r.first, r.second);
        deferred_[g].clear();
    }
    const uint32_t ran = ctl_h->steps;
    stats_->chains++;
    stats_->chain_steps += ran;
    stats_->steps += ran;
    stats_->syncs++;
    stats_->probe_launches += ran;
    if (!P_.fused) stats_->scatter_launches += ran;
    stats_->greedy_launches += ran;
    bool any_done = false;
    for (size_t i = 0; i < qs.size(); i++) {
        FxQuery &q = *qs[i];
        const FxChainQuery &c = cq_h[i];
        if (c.error) return fx_fail(FX_EDEVICE, "device consistency check failed in a device-scheduled step");
        for (int l = 0; l <= FX_MAXN; l++) {
            q.T[l] = c.T[l];
            q.cur[l] = c.cur[l];
            q.nparts[l] = c.nparts[l];
            q.rate[l] = c.rate[l];
        }
        q.phase = c.phase == FX_CQ_SUPPORT ? PH_SUPPORT : PH_COUNT;
        q.deep = c.deep;
        q.exit = c.exit;
        q.steps = c.steps;
        q.rank_base = c.rank_base;
        q.probed_support = c.probed_support;
        q.alg_probe_seen = c.alg_probe_seen;
        q.alg_probe_credit = c.alg_probe_credit;
        q.ref_probe_seen = c.ref_probe_seen;
        q.ref_probe_credit = c.ref_probe_credit;
        q.ref_row_seen = c.ref_row_seen;
        q.ref_row_credit = c.ref_row_credit;
        q.last_ufiltered = c.last.ufiltered;
        q.seg_l = -1;
        stats_->reoffered += c.reoffered;
        stats_->probed += c.probed;
        if (c.done) {
            FX_TRY(finish(q, c.last));
            q.chain_done = true;
            any_done = true;
        }
    }
    if (any_done)
        for (int g = 0; g < FX_MAX_LANES; g++) {
            auto &act = active_[g];
            for (size_t k = 0; k < act.size();) {
                if (act[k]->chain_done) {
                    act[k] = std::move(act.back());
                    act.pop_back();
                } else {
                    k++;
                }
            }
        }
    return FX_OK;
}

fx_status fx_engine_run_on(fx_graph *G, EngineWork *W, const EngineParams &p, std::vector<FxRequest> &reqs)
{
    fx_ctx *c = G->ctx;
    FxEngine eng(G, W, c->stream, p, &c->stats);
    FX_TRY(eng.add_all(reqs.data(), reqs.size()));
    while (!eng.idle()) FX_TRY(eng.step());
    return FX_OK;
}

fx_status fx_engine_run(fx_graph *G, std::vector<FxRequest> &reqs, int32_t max_active, bool chains)
{
    fx_ctx *c = G->ctx;
    EngineParams p = c->params;
    if (!chains) p.chain_queries = 0;
    p.max_active = std::max<int32_t>(1, std::min<int32_t>(max_active, (int32_t)std::max<size_t>(reqs.size(), 1)));
    return fx_engine_run_on(G, &c->work, p, reqs);
}
