// C ABI and host runtime of the support-counting library.
//
// fx_graph_load validates the caller's CSR, maps labels to a dense range,
// packs every adjacency entry as (neighbour label, edge label, id) and sorts
// each row by that key, and builds per-label vertex buckets; the result
// stays resident on the device.
//
// fx_support runs one pattern: it builds the matching plan (pattern vertices
// in submitted order, so embeddings come out in rank order), then drives the
// slice stack on the device.  Each step expands one slice of the deepest
// level that still has unexpanded candidates (a depth-first order over
// slices), so complete embeddings appear in rank order and the greedy of
// Section 2.4.3 can be applied slice by slice: the used-vertex set U carried
// from slice to slice is the bitmap of the matcher in Section 3.2.2, and
// partial embeddings that meet U are dropped (they could never be selected).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/flexis.h"
#include "fx_internal.h"

namespace {

thread_local std::string g_last_error;

fx_status fail(fx_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define FX_HIP(call)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess) return fail(FX_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define FX_TRY(call)                     \
    do {                                 \
        fx_status s_ = (call);           \
        if (s_ != FX_OK) return s_;      \
    } while (0)

// Device allocation that remembers its size.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    fx_status ensure(size_t want)
    {
        if (want <= bytes && p) return FX_OK;
        release();
        size_t b = std::max<size_t>(want, 256);
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            p = nullptr;
            return fail(FX_ENOMEM, "hipMalloc(%zu) failed: %s", b, hipGetErrorString(e));
        }
        bytes = b;
        return FX_OK;
    }
    template <class T>
    T *as() const { return (T *)p; }
};

int64_t parallel_for_chunks(int64_t n, const std::function<void(int64_t, int64_t)> &fn)
{
    unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 200000 || hw == 1) {
        fn(0, n);
        return 1;
    }
    std::vector<std::thread> th;
    int64_t per = (n + hw - 1) / hw;
    for (unsigned t = 0; t < hw; t++) {
        int64_t a = t * per, b = std::min(n, a + per);
        if (a >= b) break;
        th.emplace_back(fn, a, b);
    }
    for (auto &x : th) x.join();
    return (int64_t)th.size();
}

}  // namespace

// ---------------------------------------------------------------------------
// Objects
// ---------------------------------------------------------------------------

struct fx_ctx {
    int32_t device = 0;
    hipStream_t stream = nullptr;
    int64_t slice_rows = 1 << 20;
    int64_t count_cap = (int64_t)1 << 62;
    std::atomic<int> graphs{0};

    // workspace (grown on demand)
    DevBuf lev_rows[FX_MAXN + 1], lev_lo[FX_MAXN + 1], lev_len[FX_MAXN + 1], lev_anc[FX_MAXN + 1],
        lev_off[FX_MAXN + 1];
    DevBuf flag, bcnt, boff, bsum, hkey, hval, slot, state, rem, plan, summary, U, sel_rows, sel_rank;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    FxSummary *host_sum = nullptr;  // pinned
};

struct fx_graph {
    fx_ctx *ctx = nullptr;
    int64_t nv = 0, nadj = 0;
    std::vector<int32_t> vl_values, el_values;   // dense id -> caller's label
    std::unordered_map<int32_t, uint32_t> vl_map, el_map;
    std::vector<int64_t> bptr;                   // host copy of the label buckets' offsets
    DevBuf rowp, adj, bucket, bptr_d;
    FxGraphDev dev{};
};

// ---------------------------------------------------------------------------
// Small C entry points
// ---------------------------------------------------------------------------

extern "C" const char *fx_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *fx_version(void) { return "flexis-mi355x 0.1 (gfx950)"; }

// tau of the tau equation (Section 3.1.1), lambda rounded to parts per million.
extern "C" fx_status fx_tau(int64_t sigma, double lambda, int32_t n, int64_t *tau_out)
{
    if (!tau_out) return fail(FX_EINVAL, "tau_out is NULL");
    if (sigma < 0) return fail(FX_EINVAL, "sigma must be >= 0");
    if (!(lambda >= 0.0 && lambda <= 1.0)) return fail(FX_EINVAL, "lambda must lie in [0, 1]");
    if (n < 1) return fail(FX_EINVAL, "n must be >= 1");
    const __int128 ppm = (__int128)llround(lambda * 1e6);
    const __int128 num = (__int128)sigma * ((__int128)(n - 1) * ppm + 1000000);
    const __int128 den = (__int128)n * 1000000;
    *tau_out = (int64_t)(num / den);
    return FX_OK;
}

extern "C" fx_status fx_ctx_create(const fx_ctx_opts *opts, fx_ctx **out)
{
    if (!out) return fail(FX_EINVAL, "out is NULL");
    fx_ctx_opts o{};
    if (opts) o = *opts;
    if (o.flags != 0) return fail(FX_EINVAL, "flags must be 0");
    if (o.slice_rows < 0 || o.count_cap < 0) return fail(FX_EINVAL, "slice_rows and count_cap must be >= 0");
    int ndev = 0;
    FX_HIP(hipGetDeviceCount(&ndev));
    if (o.device < 0 || o.device >= ndev) return fail(FX_EINVAL, "device %d out of range (%d devices)", o.device, ndev);
    FX_HIP(hipSetDevice(o.device));
    fx_ctx *c = new fx_ctx();
    c->device = o.device;
    c->stream = (hipStream_t)o.hip_stream;
    if (o.slice_rows > 0) c->slice_rows = std::max<int64_t>(o.slice_rows, 64);
    if (c->slice_rows > (int64_t)1 << 28) c->slice_rows = (int64_t)1 << 28;
    if (o.count_cap > 0) c->count_cap = o.count_cap;
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        hipHostMalloc((void **)&c->host_sum, sizeof(FxSummary), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return fail(FX_EDEVICE, "event or pinned allocation failed");
    }
    *out = c;
    return FX_OK;
}

extern "C" fx_status fx_ctx_destroy(fx_ctx *c)
{
    if (!c) return fail(FX_EINVAL, "ctx is NULL");
    if (c->graphs.load() != 0) return fail(FX_EBUSY, "%d graph(s) still loaded", c->graphs.load());
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->host_sum) (void)hipHostFree(c->host_sum);
    delete c;
    return FX_OK;
}

// ---------------------------------------------------------------------------
// Graph residency
// ---------------------------------------------------------------------------

namespace {

fx_status validate_and_pack(const fx_graph_desc *d, const int64_t *rp, const int32_t *col, const int32_t *vlab,
                            const int32_t *elab, fx_graph *G, std::vector<uint64_t> &adj,
                            std::vector<int32_t> &bucket)
{
    const int64_t nv = d->num_vertices, na = d->num_adj;
    if (rp[0] != 0 || rp[nv] != na) return fail(FX_EGRAPH, "row_ptr[0] must be 0 and row_ptr[nv] = num_adj");
    for (int64_t v = 0; v < nv; v++)
        if (rp[v + 1] < rp[v]) return fail(FX_EGRAPH, "row_ptr decreases at vertex %lld", (long long)v);
    for (int64_t v = 0; v < nv; v++)
        if (vlab[v] < 0) return fail(FX_EGRAPH, "negative vertex label at %lld", (long long)v);
    // rows ascending, in range, no self loops, labels >= 0
    std::atomic<int64_t> bad{-1};
    parallel_for_chunks(nv, [&](int64_t a, int64_t b) {
        for (int64_t v = a; v < b && bad.load(std::memory_order_relaxed) < 0; v++) {
            for (int64_t k = rp[v]; k < rp[v + 1]; k++) {
                int32_t w = col[k];
                if (w < 0 || w >= nv || w == v || (k > rp[v] && col[k - 1] >= w) || (elab && elab[k] < 0)) {
                    bad.store(v);
                    break;
                }
            }
        }
    });
    if (bad.load() >= 0)
        return fail(FX_EGRAPH, "row %lld: neighbour out of range, self-loop, duplicate, unsorted or negative label",
                    (long long)bad.load());
    // symmetry with equal edge labels
    parallel_for_chunks(nv, [&](int64_t a, int64_t b) {
        for (int64_t v = a; v < b && bad.load(std::memory_order_relaxed) < 0; v++) {
            for (int64_t k = rp[v]; k < rp[v + 1]; k++) {
                int32_t w = col[k];
                const int32_t *beg = col + rp[w], *end = col + rp[w + 1];
                const int32_t *it = std::lower_bound(beg, end, (int32_t)v);
                if (it == end || *it != v || (elab && elab[it - col] != elab[k])) {
                    bad.store(v);
                    break;
                }
            }
        }
    });
    if (bad.load() >= 0)
        return fail(FX_EGRAPH, "row %lld: adjacency not symmetric or edge labels differ by direction",
                    (long long)bad.load());
    // dense label maps
    std::vector<int32_t> vals(vlab, vlab + nv);
    std::sort(vals.begin(), vals.end());
    vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
    if (vals.size() > 65535) return fail(FX_ELIMIT, "more than 65535 distinct vertex labels");
    G->vl_values = vals;
    for (size_t i = 0; i < vals.size(); i++) G->vl_map[vals[i]] = (uint32_t)i;
    std::vector<int32_t> evals;
    if (elab) {
        evals.assign(elab, elab + na);
        std::sort(evals.begin(), evals.end());
        evals.erase(std::unique(evals.begin(), evals.end()), evals.end());
    }
    if (evals.empty()) evals.push_back(0);
    if (evals.size() > 65535) return fail(FX_ELIMIT, "more than 65535 distinct edge labels");
    G->el_values = evals;
    for (size_t i = 0; i < evals.size(); i++) G->el_map[evals[i]] = (uint32_t)i;
    std::vector<uint16_t> dvl(nv);
    for (int64_t v = 0; v < nv; v++) dvl[v] = (uint16_t)G->vl_map[vlab[v]];
    // packed rows
    adj.resize(na);
    parallel_for_chunks(nv, [&](int64_t a, int64_t b) {
        for (int64_t v = a; v < b; v++) {
            for (int64_t k = rp[v]; k < rp[v + 1]; k++) {
                uint32_t w = (uint32_t)col[k];
                uint32_t el = elab ? (uint32_t)(std::lower_bound(G->el_values.begin(), G->el_values.end(), elab[k]) -
                                                G->el_values.begin())
                                   : 0u;
                adj[k] = ((uint64_t)dvl[w] << 48) | ((uint64_t)el << 32) | w;
            }
            std::sort(adj.begin() + rp[v], adj.begin() + rp[v + 1]);
        }
    });
    // label buckets (counting sort, ascending id within a label)
    const size_t L = vals.size();
    G->bptr.assign(L + 1, 0);
    for (int64_t v = 0; v < nv; v++) G->bptr[dvl[v] + 1]++;
    for (size_t l = 0; l < L; l++) G->bptr[l + 1] += G->bptr[l];
    bucket.resize(nv);
    std::vector<int64_t> fill(G->bptr.begin(), G->bptr.end() - 1);
    for (int64_t v = 0; v < nv; v++) bucket[fill[dvl[v]]++] = (int32_t)v;
    return FX_OK;
}

}  // namespace

extern "C" fx_status fx_graph_load(fx_ctx *ctx, const fx_graph_desc *d, fx_graph **out)
{
    if (!ctx || !d || !out) return fail(FX_EINVAL, "NULL argument");
    if (d->num_vertices < 1) return fail(FX_EGRAPH, "num_vertices must be >= 1");
    if (d->num_vertices > 0x7fffffffLL) return fail(FX_ELIMIT, "more than 2^31-1 vertices");
    if (d->num_adj < 0) return fail(FX_EGRAPH, "num_adj must be >= 0");
    if (d->offset_bytes != 4 && d->offset_bytes != 8) return fail(FX_EINVAL, "offset_bytes must be 4 or 8");
    if (!d->row_ptr || !d->vlabel || (d->num_adj > 0 && !d->col)) return fail(FX_EINVAL, "NULL array in graph desc");
    FX_HIP(hipSetDevice(ctx->device));
    const int64_t nv = d->num_vertices, na = d->num_adj;
    // host views of the caller's arrays
    std::vector<int64_t> rp(nv + 1);
    std::vector<int32_t> colv, vlv, elv;
    const int32_t *col = d->col, *vlab = d->vlabel, *elab = d->elabel;
    std::vector<uint8_t> rp_raw((size_t)(nv + 1) * d->offset_bytes);
    if (d->on_device) {
        FX_HIP(hipMemcpy(rp_raw.data(), d->row_ptr, rp_raw.size(), hipMemcpyDeviceToHost));
        colv.resize(na);
        vlv.resize(nv);
        if (na) FX_HIP(hipMemcpy(colv.data(), d->col, na * 4, hipMemcpyDeviceToHost));
        FX_HIP(hipMemcpy(vlv.data(), d->vlabel, nv * 4, hipMemcpyDeviceToHost));
        col = colv.data();
        vlab = vlv.data();
        if (d->elabel) {
            elv.resize(na);
            if (na) FX_HIP(hipMemcpy(elv.data(), d->elabel, na * 4, hipMemcpyDeviceToHost));
            elab = elv.data();
        }
    } else {
        memcpy(rp_raw.data(), d->row_ptr, rp_raw.size());
    }
    if (d->offset_bytes == 4) {
        const int32_t *r = (const int32_t *)rp_raw.data();
        for (int64_t i = 0; i <= nv; i++) rp[i] = r[i];
    } else {
        memcpy(rp.data(), rp_raw.data(), rp_raw.size());
    }
    fx_graph *G = new fx_graph();
    G->ctx = ctx;
    G->nv = nv;
    G->nadj = na;
    std::vector<uint64_t> adj;
    std::vector<int32_t> bucket;
    fx_status st = validate_and_pack(d, rp.data(), col, vlab, elab, G, adj, bucket);
    if (st != FX_OK) {
        delete G;
        return st;
    }
    st = G->rowp.ensure((nv + 1) * 8);
    if (st == FX_OK) st = G->adj.ensure(std::max<int64_t>(na, 1) * 8);
    if (st == FX_OK) st = G->bucket.ensure(nv * 4);
    if (st == FX_OK) st = G->bptr_d.ensure(G->bptr.size() * 8);
    if (st != FX_OK) {
        delete G;
        return st;
    }
    hipError_t e = hipMemcpy(G->rowp.p, rp.data(), (nv + 1) * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess && na) e = hipMemcpy(G->adj.p, adj.data(), na * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(G->bucket.p, bucket.data(), nv * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(G->bptr_d.p, G->bptr.data(), G->bptr.size() * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        delete G;
        return fail(FX_EDEVICE, "graph upload failed: %s", hipGetErrorString(e));
    }
    G->dev.nv = nv;
    G->dev.nadj = na;
    G->dev.rowp = G->rowp.as<int64_t>();
    G->dev.adj = G->adj.as<uint64_t>();
    G->dev.bucket = G->bucket.as<int32_t>();
    G->dev.bptr = G->bptr_d.as<int64_t>();
    G->dev.nvl = (int32_t)G->vl_values.size();
    G->dev.nel = (int32_t)G->el_values.size();
    ctx->graphs++;
    *out = G;
    return FX_OK;
}

extern "C" fx_status fx_graph_destroy(fx_graph *g)
{
    if (!g) return fail(FX_EINVAL, "graph is NULL");
    (void)hipSetDevice(g->ctx->device);
    g->ctx->graphs--;
    delete g;
    return FX_OK;
}

// ---------------------------------------------------------------------------
// Pattern plan
// ---------------------------------------------------------------------------

namespace {

struct HostPlan {
    FxPlan plan{};
    bool empty = false;          // a label of the pattern does not occur in the graph
    int64_t upper_bound = 0;     // support <= min(nv / n, min_l |V_l| / cnt_l)
};

fx_status check_pattern(const fx_pattern *p)
{
    if (!p) return fail(FX_EINVAL, "pattern is NULL");
    if (p->n > FX_MAXN) return fail(FX_ELIMIT, "pattern has %d vertices; at most %d", p->n, FX_MAXN);
    if (p->n < 1 || p->m < 0) return fail(FX_EPATTERN, "pattern needs n >= 1 and m >= 0");
    if (!p->vlabel || (p->m > 0 && !p->edges)) return fail(FX_EINVAL, "pattern arrays are NULL");
    const int n = p->n;
    bool adj[FX_MAXN][FX_MAXN] = {};
    for (int k = 0; k < p->m; k++) {
        int a = p->edges[2 * k], b = p->edges[2 * k + 1];
        if (a < 0 || b < 0 || a >= n || b >= n) return fail(FX_EPATTERN, "edge %d has an endpoint out of range", k);
        if (a == b) return fail(FX_EPATTERN, "edge %d is a loop", k);
        if (adj[a][b]) return fail(FX_EPATTERN, "edge %d repeats an edge", k);
        if (p->elabel && p->elabel[k] < 0) return fail(FX_EPATTERN, "edge %d has a negative label", k);
        adj[a][b] = adj[b][a] = true;
    }
    for (int i = 0; i < n; i++)
        if (p->vlabel[i] < 0) return fail(FX_EPATTERN, "vertex %d has a negative label", i);
    bool seen[FX_MAXN] = {};
    int stack[FX_MAXN], top = 0, cnt = 1;
    seen[0] = true;
    stack[top++] = 0;
    while (top) {
        int x = stack[--top];
        for (int y = 0; y < n; y++)
            if (adj[x][y] && !seen[y]) {
                seen[y] = true;
                cnt++;
                stack[top++] = y;
            }
    }
    if (cnt != n) return fail(FX_EPATTERN, "pattern is not connected");
    return FX_OK;
}

fx_status build_plan(const fx_graph *G, const fx_pattern *p, HostPlan &hp)
{
    FX_TRY(check_pattern(p));
    const int n = p->n;
    FxPlan &P = hp.plan;
    memset(&P, 0, sizeof(P));
    P.n = n;
    int32_t el[FX_MAXN][FX_MAXN];
    for (int a = 0; a < n; a++)
        for (int b = 0; b < n; b++) el[a][b] = -1;
    for (int i = 0; i < n; i++) {
        auto it = G->vl_map.find(p->vlabel[i]);
        if (it == G->vl_map.end()) hp.empty = true;
        else P.vl[i] = it->second;
    }
    for (int k = 0; k < p->m; k++) {
        int a = p->edges[2 * k], b = p->edges[2 * k + 1];
        int32_t lab = p->elabel ? p->elabel[k] : 0;
        auto it = G->el_map.find(lab);
        if (it == G->el_map.end()) {
            hp.empty = true;
            el[a][b] = el[b][a] = 0;
        } else {
            el[a][b] = el[b][a] = (int32_t)it->second;
        }
    }
    for (int i = 0; i < n; i++) {
        P.nback[i] = 0;
        for (int b = 0; b < i; b++)
            if (el[b][i] >= 0) {
                P.back[i][P.nback[i]] = b;
                P.bel[i][P.nback[i]] = (uint32_t)el[b][i];
                P.nback[i]++;
            }
        // neighbour-label filter over later neighbours: worthwhile for the
        // root and for vertices that need two or more later neighbours
        std::vector<std::pair<uint64_t, int>> need;
        int later = 0;
        for (int j = i + 1; j < n; j++)
            if (el[i][j] >= 0) {
                later++;
                uint64_t key = ((uint64_t)P.vl[j] << 48) | ((uint64_t)el[i][j] << 32);
                bool found = false;
                for (auto &q : need)
                    if (q.first == key) {
                        q.second++;
                        found = true;
                    }
                if (!found) need.push_back({key, 1});
            }
        P.nnlf[i] = 0;
        if (i < n - 1 && (i == 0 || later >= 2)) {
            std::sort(need.begin(), need.end(), [](auto &x, auto &y) { return x.second > y.second; });
            for (auto &q : need) {
                if (P.nnlf[i] == FX_NLF) break;
                P.nlf_key[i][P.nnlf[i]] = q.first;
                P.nlf_need[i][P.nnlf[i]] = q.second;
                P.nnlf[i]++;
            }
        }
    }
    // upper bound on any independent set: disjoint images (bound of Section 3.1.2)
    int64_t ub = G->nv / n;
    if (!hp.empty) {
        std::unordered_map<uint32_t, int> cnt;
        for (int i = 0; i < n; i++) cnt[P.vl[i]]++;
        for (auto &kv : cnt) {
            int64_t sz = G->bptr[kv.first + 1] - G->bptr[kv.first];
            ub = std::min<int64_t>(ub, sz / kv.second);
        }
    } else {
        ub = 0;
    }
    hp.upper_bound = ub;
    return FX_OK;
}

// ---------------------------------------------------------------------------
// The per-pattern engine
// ---------------------------------------------------------------------------

enum RunKind { RUN_SUPPORT, RUN_LIST };

struct RunOut {
    int64_t support = 0;
    uint64_t count = 0;
    uint64_t digest0 = 0, digest1 = 0;
    bool count_done = false;   // counting ran to the end (not cut at the cap)
    int32_t steps = 0, rounds = 0;
    double ms = 0;
};

fx_status ensure_workspace(fx_ctx *c, const fx_graph *G, int n)
{
    const int64_t C = c->slice_rows;
    for (int l = 0; l <= n; l++) {
        const int64_t cap = (l == 0) ? 1 : C;
        FX_TRY(c->lev_rows[l].ensure((size_t)cap * std::max(l, 1) * 4));
        FX_TRY(c->lev_lo[l].ensure((size_t)cap * 8));
        FX_TRY(c->lev_len[l].ensure((size_t)cap * 4));
        FX_TRY(c->lev_anc[l].ensure((size_t)cap));
        FX_TRY(c->lev_off[l].ensure((size_t)(cap + 1) * 8));
    }
    const int64_t nblk = (C + FX_BS - 1) / FX_BS;
    FX_TRY(c->flag.ensure(C));
    FX_TRY(c->bcnt.ensure(nblk * 4));
    FX_TRY(c->boff.ensure(nblk * 8));
    FX_TRY(c->bsum.ensure(((C + FX_BS * FX_SCAN_ITEMS - 1) / (FX_BS * FX_SCAN_ITEMS) + 1) * 8));
    FX_TRY(c->slot.ensure((size_t)C * n * 4));
    FX_TRY(c->state.ensure(C));
    FX_TRY(c->rem.ensure(FX_RMAX * 4));
    FX_TRY(c->plan.ensure(sizeof(FxPlan)));
    FX_TRY(c->summary.ensure(sizeof(FxSummary)));
    FX_TRY(c->U.ensure(((G->nv + 31) / 32) * 4));
    FX_TRY(c->sel_rows.ensure((size_t)(G->nv / n + 1) * n * 4));
    FX_TRY(c->sel_rank.ensure((size_t)(G->nv / n + 1) * 8));
    return FX_OK;
}

FxLevelDev level_view(fx_ctx *c, int l)
{
    FxLevelDev v;
    v.rows = c->lev_rows[l].as<int32_t>();
    v.lo = c->lev_lo[l].as<int64_t>();
    v.len = c->lev_len[l].as<int32_t>();
    v.anc = c->lev_anc[l].as<int8_t>();
    v.off = c->lev_off[l].as<int64_t>();
    return v;
}

uint64_t pow2_at_least(uint64_t x)
{
    uint64_t p = 2;
    while (p < x) p <<= 1;
    return p;
}

fx_status read_summary(fx_ctx *c)
{
    FX_HIP(hipMemcpyAsync(c->host_sum, c->summary.p, sizeof(FxSummary), hipMemcpyDeviceToHost, c->stream));
    FX_HIP(hipStreamSynchronize(c->stream));
    return FX_OK;
}

// Runs one pattern.  kind RUN_SUPPORT: greedy support (+ count/digest while
// `count_on`, stopping the count at count_cap); stop_at > 0 stops once that
// many embeddings are selected.  kind RUN_LIST: every embedding is
// materialised and copied to list_out (first list_cap rows) and counted.
fx_status run_pattern(fx_ctx *c, fx_graph *G, const HostPlan &hp, RunKind kind, bool count_on, int64_t stop_at,
                      int64_t count_cap, RunOut &ro, int32_t *list_out, int64_t list_cap,
                      std::vector<int32_t> *sel_host)
{
    const int n = hp.plan.n;
    const int64_t C = c->slice_rows;
    hipStream_t s = c->stream;
    FX_TRY(ensure_workspace(c, G, n));
    FX_HIP(hipEventRecord(c->ev0, s));
    FX_HIP(hipMemcpyAsync(c->plan.p, &hp.plan, sizeof(FxPlan), hipMemcpyHostToDevice, s));
    FX_HIP(fx_launch_fill_u32(s, c->summary.as<uint32_t>(), sizeof(FxSummary) / 4, 0u));
    FX_HIP(fx_launch_fill_u32(s, c->U.as<uint32_t>(), (G->nv + 31) / 32, 0u));
    const FxPlan *dplan = c->plan.as<FxPlan>();
    FX_HIP(fx_launch_level0(s, G->dev, dplan, level_view(c, 0)));

    const uint32_t vl0 = hp.plan.vl[0];
    std::vector<uint64_t> T(n + 1, 0), cur(n + 1, 0);
    std::vector<int64_t> nparts(n + 1, 0);
    T[0] = (uint64_t)(G->bptr[vl0 + 1] - G->bptr[vl0]);
    nparts[0] = 1;
    int64_t rank_base = 0;
    int64_t listed = 0;
    bool counting = count_on || kind == RUN_LIST;
    uint32_t total_rounds = 0;
    int32_t steps = 0;
    uint64_t support = 0;

    while (true) {
        int l = -1;
        for (int k = n - 1; k >= 0; k--)
            if (cur[k] < T[k]) {
                l = k;
                break;
            }
        if (l < 0) break;
        const uint64_t t0 = cur[l];
        const uint64_t t1 = std::min<uint64_t>(T[l], t0 + (uint64_t)C);
        cur[l] = t1;
        const bool last = (l == n - 1);
        int32_t flags = 0;
        if (kind == RUN_SUPPORT) {
            if (!counting) flags |= FX_PROBE_UFILTER;
            else if (last) flags |= FX_PROBE_UFILTER | FX_PROBE_COUNT;
        } else if (last) {
            flags |= FX_PROBE_COUNT;
        }
        const FxLevelDev in = level_view(c, l), outl = level_view(c, l + 1);
        const uint32_t nblk = (uint32_t)((t1 - t0 + FX_BS - 1) / FX_BS);
        FX_HIP(fx_launch_probe(s, G->dev, dplan, n, l, in, nparts[l], t0, t1, flags, c->U.as<uint32_t>(),
                               c->flag.as<uint8_t>(), c->bcnt.as<uint32_t>(), c->summary.as<FxSummary>()));
        FX_HIP(fx_launch_scan_blocks(s, c->bcnt.as<uint32_t>(), nblk, c->boff.as<uint64_t>(),
                                     c->summary.as<FxSummary>()));
        FX_HIP(fx_launch_scatter(s, G->dev, dplan, n, l, in, nparts[l], t0, t1, c->flag.as<uint8_t>(),
                                 c->boff.as<uint64_t>(), outl));
        if (!last) FX_HIP(fx_launch_scan_len(s, outl, t1 - t0, c->bsum.as<int64_t>(), c->summary.as<FxSummary>()));
        FX_TRY(read_summary(c));
        steps++;
        const uint64_t N = c->host_sum->total_out;
        if (!last) {
            nparts[l + 1] = (int64_t)N;
            T[l + 1] = c->host_sum->t_next;
            cur[l + 1] = 0;
        } else if (kind == RUN_LIST) {
            const int64_t take = std::min<int64_t>((int64_t)N, std::max<int64_t>(0, list_cap - listed));
            if (take > 0 && list_out)
                FX_HIP(hipMemcpy(list_out + listed * n, outl.rows, (size_t)take * n * 4, hipMemcpyDeviceToHost));
            listed += (int64_t)N;
        } else if (N > 0) {
            // greedy over this slice's complete embeddings (all disjoint from U)
            const uint64_t hsize = pow2_at_least(2 * N * (uint64_t)n);
            FX_TRY(c->hkey.ensure(hsize * 4));
            FX_TRY(c->hval.ensure(hsize * 8));
            FX_HIP(fx_launch_greedy_init(s, outl.rows, n, N, c->hkey.as<int32_t>(),
                                         c->hval.as<unsigned long long>(), hsize, c->slot.as<int32_t>(),
                                         c->state.as<uint8_t>(), c->rem.as<uint32_t>(), c->summary.as<FxSummary>()));
            uint32_t r = 0;
            while (true) {
                const uint32_t batch = 4;
                for (uint32_t k = 0; k < batch; k++, r++)
                    FX_HIP(fx_launch_greedy_round(s, outl.rows, n, N, c->hval.as<unsigned long long>(),
                                                  c->slot.as<int32_t>(), c->state.as<uint8_t>(),
                                                  c->rem.as<uint32_t>(), r, c->U.as<uint32_t>(),
                                                  c->sel_rows.as<int32_t>(), c->sel_rank.as<int64_t>(), rank_base,
                                                  c->summary.as<FxSummary>()));
                uint32_t remv = 0;
                FX_HIP(hipMemcpyAsync(&remv, c->rem.as<uint32_t>() + ((r - 1) % FX_RMAX), 4, hipMemcpyDeviceToHost,
                                      s));
                FX_HIP(hipStreamSynchronize(s));
                if (remv == 0) break;
                if ((uint64_t)r > N + 8)  // every round selects the minimum undecided embedding
                    return fail(FX_EDEVICE, "greedy did not converge after %u rounds on %llu rows", r,
                                (unsigned long long)N);
            }
            total_rounds += r;
            rank_base += (int64_t)N;
            FX_TRY(read_summary(c));
        }
        support = c->host_sum->support;
        if (stop_at > 0 && (int64_t)support >= stop_at) break;
        if (kind == RUN_SUPPORT && counting && (int64_t)c->host_sum->count >= count_cap) {
            counting = false;  // saturated: finish the support with the used-set filter
        }
    }
    FX_HIP(hipEventRecord(c->ev1, s));
    FX_TRY(read_summary(c));
    float ms = 0;
    FX_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    ro.support = (int64_t)c->host_sum->support;
    ro.count = kind == RUN_LIST ? (uint64_t)listed : c->host_sum->count;
    ro.digest0 = c->host_sum->digest0;
    ro.digest1 = c->host_sum->digest1;
    ro.count_done = counting;
    ro.steps = steps;
    ro.rounds = (int32_t)total_rounds;
    ro.ms = ms;
    if (sel_host && ro.support > 0) {
        const int64_t k = ro.support;
        std::vector<int32_t> rows((size_t)k * n);
        std::vector<int64_t> rank(k);
        FX_HIP(hipMemcpy(rows.data(), c->sel_rows.p, (size_t)k * n * 4, hipMemcpyDeviceToHost));
        FX_HIP(hipMemcpy(rank.data(), c->sel_rank.p, (size_t)k * 8, hipMemcpyDeviceToHost));
        std::vector<int64_t> idx(k);
        std::iota(idx.begin(), idx.end(), 0);
        std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return rank[a] < rank[b]; });
        sel_host->resize((size_t)k * n);
        for (int64_t i = 0; i < k; i++)
            memcpy(sel_host->data() + i * n, rows.data() + idx[i] * n, (size_t)n * 4);
    }
    return FX_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Queries
// ---------------------------------------------------------------------------

extern "C" fx_status fx_support(fx_graph *g, const fx_pattern *p, int64_t sigma, double lambda, int32_t mode,
                                fx_result *out, int32_t *selected, int64_t selected_cap)
{
    if (!g || !out) return fail(FX_EINVAL, "NULL argument");
    if (sigma < 1) return fail(FX_EINVAL, "sigma must be >= 1");
    if (!(lambda >= 0.0 && lambda <= 1.0)) return fail(FX_EINVAL, "lambda must lie in [0, 1]");
    if (mode != FX_MODE_FULL && mode != FX_MODE_VERDICT) return fail(FX_EINVAL, "unknown mode %d", mode);
    if (selected_cap < 0) return fail(FX_EINVAL, "selected_cap must be >= 0");
    fx_ctx *c = g->ctx;
    FX_HIP(hipSetDevice(c->device));
    HostPlan hp;
    FX_TRY(build_plan(g, p, hp));
    const int n = p->n;
    int64_t tau = 0;
    FX_TRY(fx_tau(sigma, lambda, n, &tau));
    const int64_t tau_eff = std::max<int64_t>(tau, 1);
    fx_result r{};
    r.tau = tau;
    if (hp.empty) {  // some label never occurs: M is empty
        r.support = mode == FX_MODE_VERDICT ? -1 : 0;
        r.frequent = 0;
        r.embedding_count = mode == FX_MODE_VERDICT ? -1 : 0;
        *out = r;
        return FX_OK;
    }
    if (mode == FX_MODE_VERDICT) {
        if (hp.upper_bound < tau_eff) {  // exact: support can never reach tau
            r.support = -1;
            r.frequent = 0;
            r.embedding_count = -1;
            *out = r;
            return FX_OK;
        }
        RunOut ro;
        FX_TRY(run_pattern(c, g, hp, RUN_SUPPORT, false, tau_eff, c->count_cap, ro, nullptr, 0, nullptr));
        r.frequent = ro.support >= tau_eff;
        r.support = r.frequent ? tau : -1;
        r.embedding_count = -1;
        r.steps = ro.steps;
        r.rounds = ro.rounds;
        r.device_ms = ro.ms;
        *out = r;
        return FX_OK;
    }
    RunOut ro;
    std::vector<int32_t> sel;
    FX_TRY(run_pattern(c, g, hp, RUN_SUPPORT, true, 0, c->count_cap, ro, nullptr, 0,
                       (selected && selected_cap > 0) ? &sel : nullptr));
    r.support = ro.support;
    r.frequent = ro.support >= tau_eff;
    const bool sat = (int64_t)ro.count >= c->count_cap;
    r.count_saturated = sat;
    r.embedding_count = sat ? c->count_cap : (int64_t)ro.count;
    if (!sat) {
        r.digest[0] = ro.digest0;
        r.digest[1] = ro.digest1;
    }
    r.steps = ro.steps;
    r.rounds = ro.rounds;
    r.device_ms = ro.ms;
    if (selected && selected_cap > 0) {
        const int64_t k = std::min<int64_t>(selected_cap, ro.support);
        memcpy(selected, sel.data(), (size_t)k * n * 4);
    }
    *out = r;
    return FX_OK;
}

extern "C" fx_status fx_enumerate(fx_graph *g, const fx_pattern *p, int32_t *rows, int64_t cap, int64_t *count_out)
{
    if (!g || !count_out) return fail(FX_EINVAL, "NULL argument");
    if (cap < 0 || (cap > 0 && !rows)) return fail(FX_EINVAL, "bad output buffer");
    fx_ctx *c = g->ctx;
    FX_HIP(hipSetDevice(c->device));
    HostPlan hp;
    FX_TRY(build_plan(g, p, hp));
    if (hp.empty) {
        *count_out = 0;
        return FX_OK;
    }
    RunOut ro;
    FX_TRY(run_pattern(c, g, hp, RUN_LIST, true, 0, INT64_MAX, ro, rows, cap, nullptr));
    *count_out = (int64_t)ro.count;
    return FX_OK;
}

extern "C" fx_status fx_support_batch(fx_graph *g, int32_t npat, const fx_pattern *pats, const int64_t *sigma,
                                      const double *lambda, int32_t mode, fx_result *out)
{
    if (!g || npat < 0 || (npat > 0 && (!pats || !sigma || !lambda || !out))) return fail(FX_EINVAL, "bad batch");
    for (int32_t i = 0; i < npat; i++) FX_TRY(fx_support(g, &pats[i], sigma[i], lambda[i], mode, &out[i], nullptr, 0));
    return FX_OK;
}
