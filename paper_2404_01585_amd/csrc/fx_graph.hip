// Graph residency: validation of the caller's CSR, dense labels, packed and
// label-sorted adjacency, per-label vertex buckets.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <vector>

#include "fx_host.h"

namespace {

// Per-vertex loops of the graph checks and index build: inline for small
// graphs, else in blocks on the library's worker threads.
void parallel_for_chunks(int64_t n, const std::function<void(int64_t, int64_t)> &fn)
{
    if (n < 200000) {
        fn(0, n);
        return;
    }
    fx_parallel_for(n, std::max<int64_t>(n / 256, 4096), fn);
}

}  // namespace

// ---------------------------------------------------------------------------
// Graph residency
// ---------------------------------------------------------------------------

namespace {

fx_status validate_and_pack(const fx_graph_desc *d, const int64_t *rp, const int32_t *col, const int32_t *vlab,
                            const int32_t *elab, fx_graph *G, std::vector<uint64_t> &adj,
                            std::vector<int32_t> &bucket)
{
    const int64_t nv = d->num_vertices, na = d->num_adj;
    if (rp[0] != 0 || rp[nv] != na) return fx_fail(FX_EGRAPH, "row_ptr[0] must be 0 and row_ptr[nv] = num_adj");
    for (int64_t v = 0; v < nv; v++)
        if (rp[v + 1] < rp[v]) return fx_fail(FX_EGRAPH, "row_ptr decreases at vertex %lld", (long long)v);
    for (int64_t v = 0; v < nv; v++)
        if (vlab[v] < 0) return fx_fail(FX_EGRAPH, "negative vertex label at %lld", (long long)v);
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
        return fx_fail(FX_EGRAPH, "row %lld: neighbour out of range, self-loop, duplicate, unsorted or negative label",
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
        return fx_fail(FX_EGRAPH, "row %lld: adjacency not symmetric or edge labels differ by direction",
                    (long long)bad.load());
    // dense label maps
    std::vector<int32_t> vals(vlab, vlab + nv);
    std::sort(vals.begin(), vals.end());
    vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
    if (vals.size() > 65535) return fx_fail(FX_ELIMIT, "more than 65535 distinct vertex labels");
    G->vl_values = vals;
    for (size_t i = 0; i < vals.size(); i++) G->vl_map[vals[i]] = (uint32_t)i;
    std::vector<int32_t> evals;
    if (elab) {
        evals.assign(elab, elab + na);
        std::sort(evals.begin(), evals.end());
        evals.erase(std::unique(evals.begin(), evals.end()), evals.end());
    }
    if (evals.empty()) evals.push_back(0);
    if (evals.size() > 65535) return fx_fail(FX_ELIMIT, "more than 65535 distinct edge labels");
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

// A directed graph: the caller's rows list out-neighbours.  The packed
// adjacency holds every edge u -> v twice: in u's row with code 2e (out) and
// in v's row with code 2e + 1 (in), e the dense label; rp_sym receives the
// rows of that symmetric form (twice the entries).
fx_status validate_and_pack_directed(const fx_graph_desc *d, const int64_t *rp, const int32_t *col,
                                     const int32_t *vlab, const int32_t *elab, fx_graph *G,
                                     std::vector<uint64_t> &adj, std::vector<int32_t> &bucket,
                                     std::vector<int64_t> &rp_sym)
{
    const int64_t nv = d->num_vertices, na = d->num_adj;
    if (rp[0] != 0 || rp[nv] != na) return fx_fail(FX_EGRAPH, "row_ptr[0] must be 0 and row_ptr[nv] = num_adj");
    for (int64_t v = 0; v < nv; v++)
        if (rp[v + 1] < rp[v]) return fx_fail(FX_EGRAPH, "row_ptr decreases at vertex %lld", (long long)v);
    for (int64_t v = 0; v < nv; v++)
        if (vlab[v] < 0) return fx_fail(FX_EGRAPH, "negative vertex label at %lld", (long long)v);
    for (int64_t v = 0; v < nv; v++)
        for (int64_t k = rp[v]; k < rp[v + 1]; k++) {
            const int32_t w = col[k];
            if (w < 0 || w >= nv || w == v || (k > rp[v] && col[k - 1] >= w) || (elab && elab[k] < 0))
                return fx_fail(FX_EGRAPH,
                               "row %lld: head out of range, self-loop, duplicate, unsorted or negative label",
                               (long long)v);
        }
    std::vector<int32_t> vals(vlab, vlab + nv);
    std::sort(vals.begin(), vals.end());
    vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
    if (vals.size() > 65535) return fx_fail(FX_ELIMIT, "more than 65535 distinct vertex labels");
    G->vl_values = vals;
    for (size_t i = 0; i < vals.size(); i++) G->vl_map[vals[i]] = (uint32_t)i;
    std::vector<int32_t> evals;
    if (elab) {
        evals.assign(elab, elab + na);
        std::sort(evals.begin(), evals.end());
        evals.erase(std::unique(evals.begin(), evals.end()), evals.end());
    }
    if (evals.empty()) evals.push_back(0);
    if (evals.size() > 32767) return fx_fail(FX_ELIMIT, "more than 32767 distinct edge labels in a directed graph");
    G->el_values = evals;
    for (size_t i = 0; i < evals.size(); i++) G->el_map[evals[i]] = (uint32_t)i;
    std::vector<uint16_t> dvl(nv);
    for (int64_t v = 0; v < nv; v++) dvl[v] = (uint16_t)G->vl_map[vlab[v]];
    rp_sym.assign(nv + 1, 0);
    for (int64_t u = 0; u < nv; u++) {
        rp_sym[u + 1] += rp[u + 1] - rp[u];
        for (int64_t k = rp[u]; k < rp[u + 1]; k++) rp_sym[col[k] + 1]++;
    }
    for (int64_t v = 0; v < nv; v++) rp_sym[v + 1] += rp_sym[v];
    adj.resize(2 * na);
    std::vector<int64_t> fill(rp_sym.begin(), rp_sym.end() - 1);
    for (int64_t u = 0; u < nv; u++)
        for (int64_t k = rp[u]; k < rp[u + 1]; k++) {
            const uint32_t w = (uint32_t)col[k];
            const uint64_t e = elab ? (uint64_t)(std::lower_bound(evals.begin(), evals.end(), elab[k]) - evals.begin())
                                    : 0u;
            adj[fill[u]++] = ((uint64_t)dvl[w] << 48) | ((2 * e) << 32) | w;           // u -> w, out of u
            adj[fill[w]++] = ((uint64_t)dvl[u] << 48) | ((2 * e + 1) << 32) | (uint32_t)u;  // into w
        }
    parallel_for_chunks(nv, [&](int64_t a, int64_t b) {
        for (int64_t v = a; v < b; v++) std::sort(adj.begin() + rp_sym[v], adj.begin() + rp_sym[v + 1]);
    });
    const size_t L = vals.size();
    G->bptr.assign(L + 1, 0);
    for (int64_t v = 0; v < nv; v++) G->bptr[dvl[v] + 1]++;
    for (size_t l = 0; l < L; l++) G->bptr[l + 1] += G->bptr[l];
    bucket.resize(nv);
    std::vector<int64_t> bf(G->bptr.begin(), G->bptr.end() - 1);
    for (int64_t v = 0; v < nv; v++) bucket[bf[dvl[v]]++] = (int32_t)v;
    G->directed = true;
    return FX_OK;
}

}  // namespace

extern "C" fx_status fx_graph_load(fx_ctx *ctx, const fx_graph_desc *d, fx_graph **out)
{
    if (!ctx || !d || !out) return fx_fail(FX_EINVAL, "NULL argument");
    if (d->num_vertices < 1) return fx_fail(FX_EGRAPH, "num_vertices must be >= 1");
    if (d->num_vertices > 0x7fffffffLL) return fx_fail(FX_ELIMIT, "more than 2^31-1 vertices");
    if (d->num_adj < 0) return fx_fail(FX_EGRAPH, "num_adj must be >= 0");
    if (d->offset_bytes != 4 && d->offset_bytes != 8) return fx_fail(FX_EINVAL, "offset_bytes must be 4 or 8");
    if (!d->row_ptr || !d->vlabel || (d->num_adj > 0 && !d->col)) return fx_fail(FX_EINVAL, "NULL array in graph desc");
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
    fx_status st;
    if (d->directed) {
        std::vector<int64_t> rp_sym;
        st = validate_and_pack_directed(d, rp.data(), col, vlab, elab, G, adj, bucket, rp_sym);
        rp.swap(rp_sym);  // the device rows are the symmetric form
        G->nadj = 2 * na;
    } else {
        st = validate_and_pack(d, rp.data(), col, vlab, elab, G, adj, bucket);
    }
    if (st != FX_OK) {
        delete G;
        return st;
    }
    const int64_t nadj = G->nadj;
    st = G->rowp.ensure((nv + 1) * 8);
    if (st == FX_OK) st = G->adj.ensure(std::max<int64_t>(nadj, 1) * 8);
    if (st == FX_OK) st = G->bucket.ensure(nv * 4);
    if (st == FX_OK) st = G->bptr_d.ensure(G->bptr.size() * 8);
    if (st != FX_OK) {
        delete G;
        return st;
    }
    hipError_t e = hipMemcpy(G->rowp.p, rp.data(), (nv + 1) * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess && nadj) e = hipMemcpy(G->adj.p, adj.data(), nadj * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(G->bucket.p, bucket.data(), nv * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(G->bptr_d.p, G->bptr.data(), G->bptr.size() * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        delete G;
        return fx_fail(FX_EDEVICE, "graph upload failed: %s", hipGetErrorString(e));
    }
    G->dev.nv = nv;
    G->dev.nadj = nadj;
    G->dev.rowp = G->rowp.as<int64_t>();
    G->dev.adj = G->adj.as<uint64_t>();
    G->dev.bucket = G->bucket.as<int32_t>();
    G->dev.bptr = G->bptr_d.as<int64_t>();
    G->dev.nvl = (int32_t)G->vl_values.size();
    G->dev.nel = (int32_t)G->el_values.size() * (G->directed ? 2 : 1);  // edge codes
    G->dev.nkeys = G->dev.nvl * G->dev.nel;
    G->dev.runoff = nullptr;
    // label-run index: the absolute adjacency position of every (vertex, key)
    // run, in one flat array (the run of (v, k) is [R[v K + k], R[v K + k + 1]),
    // the last key of v ending where v + 1 starts); positions are 32-bit, so
    // the index needs fewer than 2^32 adjacency entries
    const uint64_t K = (uint64_t)G->dev.nkeys;
    const uint64_t VW = ((uint64_t)nv + 31) / 32;  // words of one key's vertex bitmap
    const uint64_t index_bytes = ((uint64_t)nv * K + 1) * 4 + K * VW * 4;
    G->dev.vwords = (int32_t)VW;
    G->dev.keybits = nullptr;
    if (ctx->run_index_bytes >= 0 && index_bytes <= (uint64_t)ctx->run_index_bytes && nadj < 0xffffffffLL) {
        std::vector<uint32_t> ro(nv * K + 1);
        std::vector<uint32_t> kb(K * VW, 0u);
        const int32_t nel = G->dev.nel;
        parallel_for_chunks(nv, [&](int64_t a, int64_t b) {
            for (int64_t v = a; v < b; v++) {
                uint32_t *r = ro.data() + v * K;
                const int64_t base = rp[v], end = rp[v + 1];
                uint64_t k = 0;
                for (int64_t i = base; i < end; i++) {  // the row is sorted by key
                    const uint64_t e = adj[i];
                    const uint64_t key = (e >> 48) * (uint64_t)nel + ((e >> 32) & 0xffffu);
                    while (k <= key) r[k++] = (uint32_t)i;
                    // neighbouring vertices share a word across chunks: an atomic or
                    __atomic_fetch_or(&kb[key * VW + (uint64_t)v / 32], 1u << (v % 32), __ATOMIC_RELAXED);
                }
                while (k < K) r[k++] = (uint32_t)end;
            }
        });
        ro[nv * K] = (uint32_t)nadj;
        if (G->runoff.ensure(ro.size() * 4) == FX_OK && G->keybits.ensure(kb.size() * 4) == FX_OK &&
            hipMemcpy(G->runoff.p, ro.data(), ro.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(G->keybits.p, kb.data(), kb.size() * 4, hipMemcpyHostToDevice) == hipSuccess) {
            G->dev.runoff = G->runoff.as<uint32_t>();
            G->dev.keybits = G->keybits.as<uint32_t>();
        }
    }
    ctx->graphs++;
    *out = G;
    return FX_OK;
}

extern "C" fx_status fx_graph_destroy(fx_graph *g)
{
    if (!g) return fx_fail(FX_EINVAL, "graph is NULL");
    if (g->servers.load() != 0) return fx_fail(FX_EBUSY, "%d server(s) still use the graph", g->servers.load());
    (void)hipSetDevice(g->ctx->device);
    g->ctx->graphs--;
    delete g;
    return FX_OK;
}

