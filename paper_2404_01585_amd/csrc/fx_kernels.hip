// gfx950 kernels of the support-counting path.
//
// The enumeration is a lexicographic slice-by-slice expansion of partial
// embeddings (pattern vertices matched in submitted order, candidates in
// ascending id).  A step takes a contiguous range of the flattened candidate
// space of one level -- every (partial, candidate) pair, one thread each --
// tests the candidates (Section 2.1.4: label, injectivity, every pattern edge
// to an earlier vertex present in the data graph with the right edge label),
// and writes the survivors to the next level with an order-preserving
// ballot/prefix-sum compaction, so rows stay in rank order.
//
// Complete embeddings feed the greedy maximal independent set (Section 2.4.3):
// data vertices are hashed to slots (the overlap structure), and rounds select
// every undecided embedding whose rank is the minimum in all of its slots;
// this is the lexicographically-first MIS, i.e. exactly the sequential greedy
// of the matcher in Section 3.2.2.
#include "fx_internal.h"
#include "../../include/flexis.h"

namespace {

constexpr uint64_t kSeed1 = 0x243f6a8885a308d3ULL;
constexpr uint64_t kSeed2 = 0x13198a2e03707344ULL;

// SplitMix64 output function (Steele, Lea, Flood 2014; Vigna's constants).
__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    uint64_t z = x + 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t run_key(uint32_t vl, uint32_t el)
{
    return ((uint64_t)vl << 48) | ((uint64_t)el << 32);
}

// Binary search narrows a range down to at most SCAN entries; those are
// then read with independent loads (one memory round trip instead of a chain
// of dependent ones: most label runs are a few entries long).  The loads in
// flight hold registers, so kernels with a wider partial row (W) scan fewer:
// SCAN = 32 / W.
template <int W>
constexpr int scan_width() { return 32 / W; }

// First index in adj[lo, hi) whose value is >= key.  `bytes` grows by the 8
// bytes of every entry the search reads (its algorithmic traffic).
template <int SCAN>
__device__ __forceinline__ int64_t lower_bound64(const uint64_t *__restrict__ a, int64_t lo, int64_t hi, uint64_t key,
                                                 uint32_t &bytes)
{
    while (hi - lo > SCAN) {
        int64_t mid = lo + ((hi - lo) >> 1);
        bytes += 8;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    const int64_t n = hi - lo;
    uint64_t v[SCAN];
#pragma unroll
    for (int j = 0; j < SCAN; j++)
        if (j < n) v[j] = a[lo + j];
    int64_t below = 0;
#pragma unroll
    for (int j = 0; j < SCAN; j++) below += (j < n && v[j] < key) ? 1 : 0;
    bytes += 8u * (uint32_t)n;
    return lo + below;
}

// Does the sorted range a[lo, hi) hold key?
template <int SCAN>
__device__ __forceinline__ bool contains64(const uint64_t *__restrict__ a, int64_t lo, int64_t hi, uint64_t key,
                                           uint32_t &bytes)
{
    while (hi - lo > SCAN) {
        int64_t mid = lo + ((hi - lo) >> 1);
        const uint64_t m = a[mid];
        bytes += 8;
        if (m == key) return true;
        if (m < key) lo = mid + 1;
        else hi = mid;
    }
    const int64_t n = hi - lo;
    uint64_t v[SCAN];
#pragma unroll
    for (int j = 0; j < SCAN; j++)
        if (j < n) v[j] = a[lo + j];
    bool found = false;
#pragma unroll
    for (int j = 0; j < SCAN; j++) found = found | (j < n && v[j] == key);
    bytes += 8u * (uint32_t)n;
    return found;
}

// The run of neighbours of u with the given (label, elabel) key: two
// adjacent positions of the label-run index when the graph has one (one
// random access), else two binary searches over u's row.
template <int SCAN>
__device__ __forceinline__ void run_of(const FxGraphDev &g, int32_t u, uint64_t key, int64_t &lo, int32_t &len,
                                       uint32_t &bytes)
{
    if (g.runoff) {
        const uint32_t kidx = (uint32_t)(key >> 48) * (uint32_t)g.nel + (uint32_t)((key >> 32) & 0xffffu);
        const uint32_t *r = g.runoff + (uint64_t)(uint32_t)u * (uint32_t)g.nkeys + kidx;
        const uint32_t a = r[0], b = r[1];
        lo = a;
        len = (int32_t)(b - a);
        bytes += 8;
        return;
    }
    int64_t a = g.rowp[u], b = g.rowp[u + 1];
    bytes += 16;
    int64_t s = lower_bound64<SCAN>(g.adj, a, b, key, bytes);
    int64_t e = lower_bound64<SCAN>(g.adj, s, b, key + (1ULL << 32), bytes);
    lo = s;
    len = (int32_t)(e - s);
}

// Does the row of u contain the packed entry (label, elabel, id)?  A binary
// search inside the entry's (label, elabel) run.
template <int SCAN>
__device__ __forceinline__ bool has_entry(const FxGraphDev &g, int32_t u, uint64_t entry, uint32_t &bytes)
{
    int64_t lo, hi;
    if (g.runoff) {
        int32_t len;
        run_of<SCAN>(g, u, entry & 0xffffffff00000000ULL, lo, len, bytes);
        hi = lo + len;
    } else {
        lo = g.rowp[u];
        hi = g.rowp[u + 1];
        bytes += 16;
    }
    return contains64<SCAN>(g.adj, lo, hi, entry, bytes);
}

__device__ __forceinline__ bool is_used(const uint32_t *__restrict__ U, int32_t v)
{
    return (U[(uint32_t)v >> 5] >> ((uint32_t)v & 31u)) & 1u;
}

// Largest p in [0, nparts) with off[p] <= t (off[0] = 0 <= t < off[nparts]).
__device__ __forceinline__ int64_t find_part(const int64_t *__restrict__ off, int64_t nparts, uint64_t t)
{
    int64_t lo = 0, hi = nparts;
    while (hi - lo > 1) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if ((uint64_t)off[mid] <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

// W: register width of the partial row, at least the largest pattern size of
// the launch (4, 8 or FX_MAXN); a narrower row keeps fewer registers live and
// unrolls fewer compares.
template <int W>
struct Cand {
    int32_t v[W];        // the partial row (first l entries)
    int32_t c;           // candidate for pattern vertex l
    int32_t anc;         // back edge of vertex l whose run produced c (-1: bucket)
    bool first;          // first candidate of its partial
};

// The partials a workgroup's tile of candidates [tfirst, tlast] touches:
// [p0, p0 + np).  When they are few, their offsets are staged in LDS and a
// map from each of the tile's candidates to its partial is built there (see
// map_tile_parts), so a thread finds its partial with one LDS read.  Called
// by every thread.
struct TileMap {
    int64_t p0;
    int64_t np;
    bool staged;
    uint64_t t0;            // flattened index of the tile's first candidate
    const uint32_t *pk;     // partial of each of the tile's candidates, from p0 (staged tiles)
};

// LDS of the tile map: the staged offsets and the candidate-to-partial map
// of a tile of up to TILE candidates.
template <int TILE>
struct TileLds {
    int64_t s_off[FX_LDSP + 1];
    uint32_t pk[TILE];
    uint32_t wmax[FX_BS / 64];
};

// Stages the offsets (and clears the partial map) without the barrier; the
// caller syncs, then calls map_tile_parts.
template <int TILE>
__device__ __forceinline__ TileMap map_tile_async(const int64_t *__restrict__ off, const FxTile &T, uint64_t t0,
                                                  TileLds<TILE> &L)
{
    TileMap m;
    m.p0 = T.p0;
    m.np = T.np;
    m.staged = m.np + 1 <= FX_LDSP;
    m.t0 = t0;
    m.pk = L.pk;
    if (m.staged) {
        for (int64_t k = threadIdx.x; k <= m.np; k += FX_BS) L.s_off[k] = off[m.p0 + k];  // off[p1 + 1] exists
        if (m.np > 1)
            for (uint32_t i = threadIdx.x; i < (uint32_t)TILE; i += FX_BS) L.pk[i] = 0;
    }
    return m;
}

// After the barrier that follows map_tile_async: every partial k >= 1 whose
// first candidate lies in the tile marks that slot with k (an LDS atomic max:
// partials without candidates start where the next one does, and the last of
// them owns the slot), then a workgroup-wide prefix max over the slots gives
// every candidate its partial.  One LDS read per candidate afterwards instead
// of a binary search over the staged offsets.  Ends with a barrier.
template <int TILE>
__device__ __forceinline__ void map_tile_parts(const TileMap &m, TileLds<TILE> &L)
{
    if (!m.staged || m.np <= 1) return;  // uniform: one partial needs no map
    constexpr int PER = TILE / FX_BS;
    for (int64_t k = 1 + threadIdx.x; k <= m.np; k += FX_BS) {
        const uint64_t rel = (uint64_t)L.s_off[k] - m.t0;  // > 0: p0 is the last partial starting at or before t0
        if (rel < (uint64_t)TILE) atomicMax(&L.pk[rel], (uint32_t)k);
    }
    __syncthreads();
    const uint32_t wave = threadIdx.x >> 6, lane = __lane_id();
    uint32_t v[PER], run = 0;
#pragma unroll
    for (int j = 0; j < PER; j++) {
        run = max(run, L.pk[threadIdx.x * PER + j]);
        v[j] = run;
    }
    uint32_t inc = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(inc, o);
        if (lane >= (uint32_t)o) inc = max(inc, u);
    }
    uint32_t before = __shfl_up(inc, 1);
    if (lane == 0) before = 0;
    if (lane == 63) L.wmax[wave] = inc;
    __syncthreads();
    for (uint32_t w = 0; w < wave; w++) before = max(before, L.wmax[w]);
#pragma unroll
    for (int j = 0; j < PER; j++) L.pk[threadIdx.x * PER + j] = max(before, v[j]);
    __syncthreads();
}

template <int TILE>
__device__ __forceinline__ TileMap map_tile(const int64_t *__restrict__ off, const FxTile &T, uint64_t t0,
                                            TileLds<TILE> &L)
{
    const TileMap m = map_tile_async<TILE>(off, T, t0, L);
    __syncthreads();
    map_tile_parts<TILE>(m, L);
    return m;
}

// Partial of flattened candidate t (t inside the tile of m).
__device__ __forceinline__ int64_t tile_part(const TileMap &m, const int64_t *__restrict__ off, uint64_t t)
{
    if (m.np <= 1) return m.p0;
    if (m.staged) return m.p0 + (int64_t)m.pk[t - m.t0];
    int64_t lo = 0, hi = m.np;  // largest k with offset[p0 + k] <= t
    {
        while (hi - lo > 1) {
            int64_t mid = (lo + hi) >> 1;
            if ((uint64_t)off[m.p0 + mid] <= t) lo = mid;
            else hi = mid;
        }
    }
    return m.p0 + lo;
}

// Loads partial p and its candidate at flattened index t.
template <int W>
__device__ __forceinline__ void load_cand(const FxGraphDev &g, const FxLevelDev &in, int32_t l, int64_t p,
                                          uint64_t t, Cand<W> &x)
{
    int64_t j = (int64_t)(t - (uint64_t)in.off[p]);
    const int32_t *row = in.rows + p * l;
#pragma unroll
    for (int k = 0; k < W; k++)
        x.v[k] = (k < l) ? row[k] : -1;
    x.anc = in.anc[p];
    x.first = (j == 0);
    int64_t base = in.lo[p];
    x.c = x.anc >= 0 ? (int32_t)(uint32_t)(g.adj[base + j] & 0xffffffffULL) : g.bucket[base + j];
}

template <int W>
__device__ __forceinline__ int32_t pick(const int32_t (&v)[W], int32_t b)
{
    int32_t r = -1;
#pragma unroll
    for (int k = 0; k < W; k++)
        r = (k == b) ? v[k] : r;
    return r;
}

// Candidate test of Section 2.1.4 for pattern vertex i = l.
template <int W>
__device__ __forceinline__ bool feasible(const FxGraphDev &g, const FxPlan *__restrict__ plan, int32_t n, int32_t l,
                                         bool sym, const Cand<W> &x, uint32_t &bytes)
{
#pragma unroll
    for (int k = 0; k < W; k++)
        if (k < l && x.v[k] == x.c) return false;  // injective
    if (sym) {  // only the smallest embedding of each automorphism orbit
        const uint32_t lt = plan->sym_lt[l];
#pragma unroll
        for (int k = 0; k < W; k++)
            if (k < l && ((lt >> k) & 1u) && x.v[k] >= x.c) return false;
    }
    const int32_t i = l;
    const uint32_t vl = plan->vl[i];
    const int32_t nb = plan->nback[i];
    for (int kk = 0; kk < nb; kk++) {
        int32_t b = plan->back[i][kk];
        if (kk == x.anc) continue;  // the run it came from already matches
        uint64_t entry = run_key(vl, plan->bel[i][kk]) | (uint32_t)x.c;
        if (!has_entry<scan_width<W>()>(g, pick(x.v, b), entry, bytes)) return false;
    }
    if (i < n - 1) {  // neighbour-label filter for the later neighbours of i
        const int32_t nf = plan->nnlf[i];
        for (int k = 0; k < nf; k++) {
            const uint32_t nk = plan->nlf_key[i][k];
            const int32_t need = plan->nlf_need[i][k];
            if (g.keybits) {  // presence first: one word of the key's vertex bitmap
                const uint32_t kidx = (nk >> 16) * (uint32_t)g.nel + (nk & 0xffffu);
                const uint32_t w = g.keybits[(uint64_t)kidx * (uint64_t)g.vwords + ((uint32_t)x.c >> 5)];
                bytes += 4;
                if (!((w >> ((uint32_t)x.c & 31u)) & 1u)) return false;
                if (need <= 1) continue;
            }
            int64_t lo;
            int32_t len;
            run_of<scan_width<W>()>(g, x.c, run_key(nk >> 16, nk & 0xffffu), lo, len, bytes);
            if (len < need) return false;
        }
    }
    return true;
}

template <int W>
__device__ __forceinline__ bool touches_used(const uint32_t *__restrict__ U, const Cand<W> &x, int32_t l)
{
    if (is_used(U, x.c)) return true;
#pragma unroll
    for (int k = 0; k < W; k++)
        if (k < l && is_used(U, x.v[k])) return true;
    return false;
}

// Reference algorithmic bytes (the counting pass only).  A per-unit model of
// what the matching itself must move, apart from this implementation's own
// extras (pass flags, run descriptors, used-set words, binary-search probes of
// the run index): 4-byte ids, 1-byte labels, 8-byte row offsets.
//   root candidate (label bucket)      4 (id) + 16 (its two row offsets)
//   partial expanded at level l        4 l (its row) + 16 (anchor's offsets)
//                                      + 6 per neighbour read (id, edge label,
//                                      neighbour label)
//   candidate tested against an earlier
//   neighbour b other than the anchor  4 ceil(log2(r + 1)) (a binary search
//                                      over r entries)
//   row written at level l + 1         4 (l + 1)
//   greedy                             4 n per complete embedding read and
//                                      4 n per selected embedding written
// With label-sorted rows the neighbours read are the anchor's run of the
// vertex's (label, edge label) and r is the length of b's run (ref_probe);
// with plain rows they are the anchor's whole row and r = deg(f(b))
// (ref_probe_row, the same model for a layout without label-sorted rows).
__device__ __forceinline__ uint32_t bit_length(uint64_t d) { return d ? 64u - (uint32_t)__clzll(d) : 0u; }

__device__ __forceinline__ uint64_t degree(const FxGraphDev &g, int32_t u)
{
    return (uint64_t)(g.rowp[u + 1] - g.rowp[u]);
}

template <int W>
__device__ __forceinline__ void ref_back_edges(const FxGraphDev &g, const FxPlan *__restrict__ plan, int32_t l,
                                               const Cand<W> &x, unsigned long long &run_b, unsigned long long &row_b)
{
    const int32_t nb = plan->nback[l];
    const uint32_t vl = plan->vl[l];
    for (int kk = 0; kk < nb; kk++) {
        const int32_t a = plan->back[l][kk];
        if (kk == x.anc) continue;
        const int32_t u = pick(x.v, a);
        int64_t lo;
        int32_t len;
        uint32_t ignored = 0;
        run_of<scan_width<W>()>(g, u, run_key(vl, plan->bel[l][kk]), lo, len, ignored);
        run_b += 4u * bit_length((uint64_t)len);
        row_b += 4u * bit_length(degree(g, u));
    }
}

// Injectivity and the symmetry-breaking order alone (the tests before any
// adjacency probe).
template <int W>
__device__ __forceinline__ bool distinct_and_ordered(const FxPlan *__restrict__ plan, int32_t l, bool sym,
                                                     const Cand<W> &x)
{
#pragma unroll
    for (int k = 0; k < W; k++)
        if (k < l && x.v[k] == x.c) return false;
    if (sym) {
        const uint32_t lt = plan->sym_lt[l];
#pragma unroll
        for (int k = 0; k < W; k++)
            if (k < l && ((lt >> k) & 1u) && x.v[k] >= x.c) return false;
    }
    return true;
}

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const uint32_t lane = __lane_id();
    return lane == 0 ? 0ULL : ((~0ULL) >> (64 - lane));
}

// ---------------------------------------------------------------------------
// Expansion: probe (test + per-block counts) and scatter (ordered write).
// ---------------------------------------------------------------------------

// One thread per expansion workgroup b: its segment (the last s with
// blk0s[s] <= b) and the partials of its tile, by binary searches over the
// level's candidate offsets -- done here once instead of at the start of
// every workgroup of the probe, the scatter and the offset fix-up.
template <int ITEMS>
__device__ __forceinline__ void tile_map_one(const FxSeg *__restrict__ segs, const uint32_t *__restrict__ blk0s,
                                             int32_t nsegs, uint32_t b, FxTile *tmap)
{
    constexpr uint32_t TILE = FX_BS * ITEMS;
    int32_t lo = 0, hi = nsegs;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (blk0s[mid] <= b) lo = mid;
        else hi = mid;
    }
    const FxSeg &S = segs[lo];
    const uint32_t tile0 = (b - S.blk0) * TILE;
    const uint32_t tile_n = min(TILE, S.span - tile0);
    const int64_t p0 = find_part(S.in.off, S.nparts, S.t0 + tile0);
    const int64_t p1 = find_part(S.in.off, S.nparts, S.t0 + tile0 + tile_n - 1);
    FxTile t;
    t.seg = lo;
    t.np = (int32_t)(p1 - p0 + 1);
    t.p0 = p0;
    tmap[b] = t;
}

// For the single-pass expansion (cstat non-null) it also clears the tiles'
// status words and the ticket counter; with sstat, the two block scans'
// status words and tickets.
template <int ITEMS>
__global__ __launch_bounds__(FX_BS) void k_tile_map(const FxSeg *__restrict__ segs, const uint32_t *__restrict__ blk0s,
                                                    int32_t nsegs, uint32_t nblocks, FxTile *tmap, uint64_t *cstat,
                                                    uint64_t *lstat, uint32_t *ticket, uint64_t *sstat)
{
    const uint32_t b = blockIdx.x * FX_BS + threadIdx.x;
    if (sstat && b < scan_state_words(nblocks)) sstat[b] = 0;
    if (b < nblocks) {
        tile_map_one<ITEMS>(segs, blk0s, nsegs, b, tmap);
        if (cstat) {
            cstat[b] = 0;
            lstat[b] = 0;
            if (b == 0) *ticket = 0;
        }
    }
}

// The same over a fixed grid, with the step's size from the scheduler.
template <int ITEMS>
__global__ __launch_bounds__(FX_BS) void k_tile_map_chain(const FxSeg *__restrict__ segs,
                                                          const uint32_t *__restrict__ blk0s, const FxChainCtl *ctl,
                                                          FxTile *tmap, uint64_t *cstat, uint64_t *lstat,
                                                          uint32_t *ticket, uint64_t *sstat)
{
    const uint32_t nb = ctl->nblocks;
    const int32_t ns = (int32_t)ctl->nsegs;
    if (sstat)
        for (uint32_t b = blockIdx.x * FX_BS + threadIdx.x; b < scan_state_words(nb); b += gridDim.x * FX_BS)
            sstat[b] = 0;
    for (uint32_t b = blockIdx.x * FX_BS + threadIdx.x; b < nb; b += gridDim.x * FX_BS) {
        tile_map_one<ITEMS>(segs, blk0s, ns, b, tmap);
        if (cstat) {
            cstat[b] = 0;
            lstat[b] = 0;
        }
    }
    if (cstat && blockIdx.x == 0 && threadIdx.x == 0) *ticket = 0;
}

template <int W>
__device__ __forceinline__ void tuple_hash(const Cand<W> &x, int32_t l, uint64_t &h1, uint64_t &h2)
{
    uint64_t a = kSeed1, b = kSeed2;
#pragma unroll
    for (int k = 0; k < W; k++) {
        if (k < l) {
            a = mix64(a ^ (uint64_t)(uint32_t)x.v[k]);
            b = mix64(b ^ (uint64_t)(uint32_t)x.v[k]);
        }
    }
    h1 = mix64(a ^ (uint64_t)(uint32_t)x.c);
    h2 = mix64(b ^ (uint64_t)(uint32_t)x.c);
}

// Marks the images of one embedding (x.v[0..l), x.c): data vertex f(k) in
// the bitmap of pattern vertex k.  A word is read before the atomic OR, so a
// vertex already marked (the common case: many embeddings share a partial)
// costs no atomic.
template <int W>
__device__ __forceinline__ void mark_images(uint32_t *img, uint64_t words, const Cand<W> &x, int32_t l)
{
#pragma unroll
    for (int k = 0; k < W; k++) {  // fully unrolled: x.v stays in registers (l < W)
        if (k <= l) {
            const uint32_t v = (uint32_t)(k == l ? x.c : x.v[k]);
            uint32_t *w = img + (uint64_t)k * words + (v >> 5);
            const uint32_t bit = 1u << (v & 31u);
            if (!(*w & bit)) atomicOr(w, bit);
        }
    }
}

// Embeddings completing the partial (x.v[0..l), x.c) when the last pattern
// vertex i = l + 1 is a leaf whose only earlier neighbour is a: every vertex
// of the run of a's image with i's (label, edge label) is a valid image,
// except the already-matched vertices that lie in that run (injectivity).
template <int W>
__device__ __forceinline__ uint64_t leaf_count(const FxGraphDev &g, const FxPlan *__restrict__ plan, int32_t l,
                                               const Cand<W> &x, uint32_t &bytes)
{
    const int32_t i = l + 1;
    const int32_t a = plan->back[i][0];
    const uint32_t vl = plan->vl[i];
    const uint64_t key = run_key(vl, plan->bel[i][0]);
    const int32_t u = (a == l) ? x.c : pick(x.v, a);
    int64_t lo;
    int32_t len;
    run_of<scan_width<W>()>(g, u, key, lo, len, bytes);
    int64_t c = len;
    for (int k = 0; k <= l; k++) {
        if (k == a || plan->vl[k] != vl) continue;
        const int32_t w = (k == l) ? x.c : pick(x.v, k);
        if (has_entry<scan_width<W>()>(g, u, key | (uint32_t)w, bytes)) c--;
    }
    return (uint64_t)c;
}

// Test every candidate of a workgroup's tile (ITEMS per thread, strided by
// the workgroup size so each item pass covers consecutive candidates).  Per
// item, the wave's ballot of the candidates that pass (bal).  Per candidate,
// without COMPACT: at cv[it * FX_BS + threadIdx.x] its vertex id (-1 when it
// does not pass) and at pi[...] its partial relative to the tile's first.
// With COMPACT, only the passing candidates, in order within their (item,
// wave) region of 64 slots: the vertex id, and the partial with the
// candidate's lane in the top 6 bits (a partial index is below 2^26: the
// slice capacity is at most 2^26 rows).
// Counting segments count (and hash) here; the per-query counters and byte
// tallies are added with one atomic per wave.
template <int TILE>
struct ProbeLds {
    TileLds<TILE> map;
    uint8_t s_dead[FX_LDSP];
    uint32_t wcnt[FX_BS / 64];
};

template <int ITEMS, int W, bool COMPACT>
__device__ __forceinline__ TileMap probe_core(const FxGraphDev &g, const FxSeg &S, const FxTile &T, const uint32_t blk,
                                              ProbeLds<FX_BS * ITEMS> &lds, uint64_t (&bal)[ITEMS], int32_t *cv,
                                              int32_t *pi)
{
    constexpr uint32_t TILE = FX_BS * ITEMS;
    uint8_t *s_dead = lds.s_dead;
    const int32_t l = S.l, n = S.n, flags = S.flags;
    const uint32_t tile0 = (blk - S.blk0) * TILE;
    const TileMap m = map_tile<TILE>(S.in.off, T, S.t0 + tile0, lds.map);
    const bool ufilter = (flags & FX_PROBE_UFILTER) != 0;
    uint32_t bytes = 0;
    // The used-set test of a partial's own vertices, once per partial of the
    // tile (a partial with many candidates is tested once, not per candidate).
    const bool pdead = ufilter && m.staged;
    if (pdead) {
        for (int64_t k = threadIdx.x; k < m.np; k += FX_BS) {
            const int32_t *row = S.in.rows + (m.p0 + k) * l;
            bool d = false;
            for (int32_t j = 0; j < l; j++) d = d || is_used(S.U, row[j]);
            s_dead[k] = d ? 1 : 0;
            bytes += 4u * (uint32_t)l;
        }
        __syncthreads();
    }
    const bool count = (flags & FX_PROBE_COUNT) != 0;
    const bool leaf = (flags & FX_PROBE_LEAF) != 0;
    const bool hash = (flags & FX_PROBE_HASH) != 0;
    const bool images = (flags & FX_PROBE_IMAGES) != 0;
    const bool sym = (flags & FX_PROBE_SYM) != 0;
    const bool ref = (flags & FX_PROBE_REF) != 0;
    uint32_t uout = 0;
    unsigned long long cnt = 0;
    unsigned long long rbytes = 0, dbytes = 0;  // reference algorithmic bytes (counting pass): run, row model
    uint64_t h1 = 0, h2 = 0;
#pragma unroll
    for (int it = 0; it < ITEMS; it++) {
        const uint32_t tl = tile0 + it * FX_BS + threadIdx.x;
        bool mat = false;
        int32_t c_out = 0, pk_out = 0;
        if (tl < S.span) {
            const uint64_t t = S.t0 + tl;
            Cand<W> x;
            const int64_t p = tile_part(m, S.in.off, t);
            load_cand(g, S.in, l, p, t, x);
            c_out = x.c;
            pk_out = (int32_t)(p - m.p0);
            if (!COMPACT && pi) pi[it * FX_BS + threadIdx.x] = pk_out;
            // candidate entry + the pass word; the partial row and its run descriptor once
            bytes += (x.anc >= 0 ? 8u : 4u) + 4u;
            if (x.first || tl == tile0) bytes += 4u * (uint32_t)l + 21u;
            if (ref) {
                const unsigned long long own = x.first ? 4u * (uint32_t)l : 0u;  // the partial's row, once
                rbytes += own;
                dbytes += own;
                if (x.anc < 0) {  // a label-bucket candidate and its offsets
                    rbytes += 20u;
                    dbytes += 20u;
                } else if (x.first) {  // the anchor's run, or its whole row
                    rbytes += 16u + 6u * (unsigned long long)S.in.len[p];
                    dbytes += 16u + 6u * degree(g, pick(x.v, S.plan->back[l][x.anc]));
                }
            }
            bool ok = true;
            if (ufilter) {
                if (pdead) {
                    ok = !s_dead[p - m.p0] && !is_used(S.U, x.c);
                    bytes += 4u;
                } else {
                    ok = !touches_used(S.U, x, l);
                    bytes += 4u * (uint32_t)(l + 1);
                }
                uout += ok ? 0u : 1u;
            }
            if (ref && ok && distinct_and_ordered(S.plan, l, sym, x)) ref_back_edges(g, S.plan, l, x, rbytes, dbytes);
            if (ok) ok = feasible(g, S.plan, n, l, sym, x, bytes);
            if (ref && ok && leaf) {  // the last vertex's expansion, counted in closed form here
                const int32_t a = S.plan->back[l + 1][0];
                const int32_t u = a == l ? x.c : pick(x.v, a);
                int64_t lo;
                int32_t len;
                uint32_t ignored = 0;
                run_of<scan_width<W>()>(g, u, run_key(S.plan->vl[l + 1], S.plan->bel[l + 1][0]), lo, len, ignored);
                rbytes += 4u * (uint32_t)(l + 1) + 16u + 6u * (unsigned long long)len;
                dbytes += 4u * (uint32_t)(l + 1) + 16u + 6u * degree(g, u);
            }
            if (ok) {
                if (count) {
                    cnt++;
                    if (hash) {
                        uint64_t a, b;
                        tuple_hash(x, l, a, b);
                        h1 += a;
                        h2 ^= b;
                    }
                    if (images) mark_images(S.img, S.img_words, x, l);
                }
                if (leaf) cnt += leaf_count(g, S.plan, l, x, bytes);
                mat = S.kind != FX_SEG_COUNT;
            }
            if (!COMPACT) cv[it * FX_BS + threadIdx.x] = mat ? x.c : -1;
        }
        bal[it] = __ballot(mat);
        if (COMPACT && mat) {
            const uint32_t slot = it * FX_BS + (threadIdx.x & ~63u) + (uint32_t)__popcll(bal[it] & lanemask_lt());
            cv[slot] = c_out;
            pi[slot] = (int32_t)(((uint32_t)__lane_id() << 26) | (uint32_t)pk_out);
        }
    }
    if (count || leaf) {  // uniform across the workgroup
        unsigned long long c = cnt;
        unsigned long long s1 = h1, s2 = h2;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            c += __shfl_xor(c, o);
            s1 += __shfl_xor(s1, o);
            s2 ^= __shfl_xor(s2, o);
        }
        if (__lane_id() == 0 && c) {
            atomicAdd(&S.sum->count, c);
            atomicAdd(&S.sum->digest0, s1);
            atomicXor(&S.sum->digest1, s2);
        }
    }
    {
        unsigned long long b = bytes;
        uint32_t uo = uout;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            b += __shfl_xor(b, o);
            uo += __shfl_xor(uo, o);
        }
        if (__lane_id() == 0) {
            if (b) atomicAdd(&S.sum->alg_probe, b);
            if (uo) atomicAdd(&S.sum->ufiltered, (unsigned long long)uo);
        }
    }
    if (ref) {  // uniform across the workgroup
        unsigned long long r = rbytes, d = dbytes;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            r += __shfl_xor(r, o);
            d += __shfl_xor(d, o);
        }
        if (__lane_id() == 0 && r) atomicAdd(&S.sum->ref_probe, r);
        if (__lane_id() == 0 && d) atomicAdd(&S.sum->ref_probe_row, d);
    }
    return m;
}

// Probe pass of the multi-kernel expansion: the tile's passing candidates
// compacted per (item, wave) region with their partials, the regions'
// counts (cand_tile_bytes per tile), and the number of passes per workgroup.
template <int ITEMS, int W>
__device__ __forceinline__ void probe_tile(const FxGraphDev &g, const FxSeg *__restrict__ segs,
                                           const FxTile *__restrict__ tmap, int32_t *cand, uint32_t *bcnt,
                                           const uint32_t blk, ProbeLds<FX_BS * ITEMS> &lds)
{
    constexpr uint32_t TILE = FX_BS * ITEMS;
    const FxTile T = tmap[blk];
    const FxSeg &S = segs[__builtin_amdgcn_readfirstlane(T.seg)];
    int32_t *crec = (int32_t *)((char *)cand + (size_t)blk * cand_tile_bytes(ITEMS));
    uint64_t bal[ITEMS];
    probe_core<ITEMS, W, true>(g, S, T, blk, lds, bal, crec, crec + TILE);
    uint32_t passed = 0;
#pragma unroll
    for (int it = 0; it < ITEMS; it++) passed += (uint32_t)__popcll(bal[it]);
    if (__lane_id() == 0) {
        uint8_t *rc = (uint8_t *)(crec + 2 * TILE);
        const uint32_t wave = threadIdx.x >> 6;
#pragma unroll
        for (int it = 0; it < ITEMS; it++) rc[it * (FX_BS / 64) + wave] = (uint8_t)__popcll(bal[it]);
        lds.wcnt[wave] = passed;
    }
    __syncthreads();
    if (threadIdx.x == 0) bcnt[blk] = lds.wcnt[0] + lds.wcnt[1] + lds.wcnt[2] + lds.wcnt[3];
}

template <int ITEMS, int W>
__global__ __launch_bounds__(FX_BS) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_probe(
    FxGraphDev g, const FxSeg *__restrict__ segs, const FxTile *__restrict__ tmap, int32_t *cand, uint32_t *bcnt)
{
    __shared__ ProbeLds<FX_BS * ITEMS> lds;
    probe_tile<ITEMS, W>(g, segs, tmap, cand, bcnt, blockIdx.x, lds);
}

template <int ITEMS, int W>
__global__ __launch_bounds__(FX_BS) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_probe_chain(
    FxGraphDev g, const FxSeg *__restrict__ segs, const FxTile *__restrict__ tmap, int32_t *cand, uint32_t *bcnt,
    const FxChainCtl *ctl)
{
    __shared__ ProbeLds<FX_BS * ITEMS> lds;
    const uint32_t nb = ctl->nblocks;
    for (uint32_t b = blockIdx.x; b < nb; b += gridDim.x) {
        probe_tile<ITEMS, W>(g, segs, tmap, cand, bcnt, b, lds);
        __syncthreads();  // the tile's LDS is reused by the next
    }
}

// Decoupled look-back over ordered workgroups (the block scans and the
// single-pass expansion).  Status word of a tile: bits 63..62 the state (0 not
// ready, 1 the tile's own total, 2 the inclusive prefix of its segment up to
// the tile), bits 61..0 the value.  k_tile_map clears the words of a step's
// tiles before the launch.
constexpr uint64_t kStatAgg = 1ull << 62;
constexpr uint64_t kStatPre = 2ull << 62;
constexpr uint64_t kStatVal = (1ull << 62) - 1;

__device__ __forceinline__ void stat_put(uint64_t *st, uint32_t b, uint64_t w)
{
    __hip_atomic_store(st + b, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of the values of tiles s0..b-1 (b > s0), called by one whole wave.  The
// wave reads the status words of up to 64 preceding tiles at once; if a tile
// nearer than the nearest inclusive prefix is not ready it reads the window
// again after a short sleep, else it adds the totals down to that prefix (or
// all 64 and moves on).  The wait ends: every tile s0..b-1 got its ticket
// before b, so it is running or done, and it publishes its total before it
// waits on anything itself; tile s0 publishes an inclusive prefix.
__device__ uint64_t look_back(const uint64_t *st, uint32_t b, uint32_t s0)
{
    const uint32_t lane = __lane_id();
    uint64_t sum = 0;
    int64_t top = (int64_t)b - 1;  // nearest tile not yet added
    while (top >= (int64_t)s0) {   // uniform across the wave
        const int64_t j = top - (int64_t)lane;
        const uint64_t w = j >= (int64_t)s0 ? __hip_atomic_load(st + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                            : kStatPre;  // lanes before the segment: never reached
        const uint32_t state = (uint32_t)(w >> 62);
        const uint64_t pm = __ballot(state == 2), xm = __ballot(state == 0);
        const uint64_t upto = pm ? (((pm & (~pm + 1)) << 1) - 1) : ~0ull;  // lanes down to the nearest prefix
        if (xm & upto) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        unsigned long long v = ((upto >> lane) & 1ull) ? (w & kStatVal) : 0ull;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
        sum += v;
        if (pm) break;
        top -= 64;
    }
    return sum;
}

// Exclusive prefix of a tile's value within its segment, published on the
// way: the tile's total first, then its inclusive prefix.  Called by wave 0.
__device__ __forceinline__ uint64_t tile_prefix(uint64_t *st, uint32_t blk, uint32_t s0, uint64_t agg)
{
    const bool lead = __lane_id() == 0;
    if (blk == s0) {
        if (lead) stat_put(st, blk, kStatPre | agg);
        return 0;
    }
    if (lead) stat_put(st, blk, kStatAgg | agg);
    const uint64_t excl = look_back(st, blk, s0);
    if (lead) stat_put(st, blk, kStatPre | (excl + agg));
    return excl;
}

// Exclusive scan of per-workgroup values (n of them; out[n] receives the
// total): chunks of kScanChunk values, one workgroup each, taken by ticket;
// each workgroup scans its chunk (4 values per thread, a shuffle scan per
// wave, the wave totals in LDS) and finds the chunk's prefix by look-back.
// A step's scan state (sstat, cleared by k_tile_map) holds, per scan (which =
// 0, 1), scan_chunks(n) status words and the ticket counter after them.  Every chunk is the same small amount of work, so the
// look-back rarely waits.
struct ScanLds {
    unsigned long long wt[FX_BS / 64];
    unsigned long long excl;
    uint32_t chunk;
};

template <class T>
__device__ __forceinline__ void scan_chunk(const T *__restrict__ vals, uint32_t n, uint64_t *out, uint64_t *st,
                                           uint32_t c, uint32_t nch, ScanLds &lds)
{
    constexpr uint32_t PER = kScanChunk / FX_BS;
    const uint32_t wave = threadIdx.x >> 6, lane = __lane_id();
    const uint32_t base = c * kScanChunk + threadIdx.x * PER;
    unsigned long long v[PER], sum = 0;
#pragma unroll
    for (uint32_t k = 0; k < PER; k++) {
        v[k] = base + k < n ? (unsigned long long)vals[base + k] : 0ull;
        sum += v[k];
    }
    unsigned long long inc = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long u = __shfl_up(inc, o);
        if (lane >= (uint32_t)o) inc += u;
    }
    if (lane == 63) lds.wt[wave] = inc;
    __syncthreads();
    unsigned long long agg = 0, woff = 0;
#pragma unroll
    for (uint32_t w = 0; w < FX_BS / 64; w++) {
        agg += lds.wt[w];
        woff += w < wave ? lds.wt[w] : 0ull;
    }
    if (wave == 0) {
        const uint64_t e = tile_prefix(st, c, 0, agg);
        if (lane == 0) lds.excl = e;
    }
    __syncthreads();
    unsigned long long run = lds.excl + woff + inc - sum;
#pragma unroll
    for (uint32_t k = 0; k < PER; k++) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (c == nch - 1 && threadIdx.x == 0) out[n] = lds.excl + agg;
}

template <class T>
__global__ __launch_bounds__(FX_BS) void k_scan_blocks(const T *__restrict__ vals, uint32_t n, uint64_t *out,
                                                       uint64_t *sstat, uint32_t which)
{
    __shared__ ScanLds lds;
    const uint32_t nch = scan_chunks(n);
    uint64_t *st = sstat + which * (nch + 1);  // the step's first or second scan
    if (threadIdx.x == 0) lds.chunk = atomicAdd(reinterpret_cast<uint32_t *>(st + nch), 1u);
    __syncthreads();
    scan_chunk<T>(vals, n, out, st, lds.chunk, nch, lds);
}

// The same over a fixed grid, with the count from the scheduler.
template <class T>
__global__ __launch_bounds__(FX_BS) void k_scan_blocks_chain(const T *__restrict__ vals, const FxChainCtl *ctl,
                                                             uint64_t *out, uint64_t *sstat, uint32_t which)
{
    __shared__ ScanLds lds;
    const uint32_t n = ctl->nblocks;
    const uint32_t nch = scan_chunks(n);
    uint64_t *st = sstat + which * (nch + 1);
    for (;;) {
        if (threadIdx.x == 0) lds.chunk = atomicAdd(reinterpret_cast<uint32_t *>(st + nch), 1u);
        __syncthreads();
        const uint32_t c = lds.chunk;
        if (c >= nch) break;  // uniform across the workgroup
        scan_chunk<T>(vals, n, out, st, c, nch, lds);
        __syncthreads();  // LDS reused by the next chunk
    }
}

// Ordered write of the passing candidates of each segment into its level l+1
// (position = passes before it in the segment, in candidate order), with the
// candidate run of the next pattern vertex for inner levels.  A workgroup
// takes its tile's passing candidates from the probe's compacted output, one
// thread each in candidate order (the regions' counts give each one's
// region).  For inner segments it also writes each new row's prefix of run
// lengths within this workgroup's rows to off[] and the workgroup's total to
// lsum[]; k_fix_off adds the workgroup offsets after a scan of lsum.  A
// segment writes at most out_cap rows: when more candidates pass, writing
// stops at the out_cap-th and the summary records how many candidates that
// took (the rest are probed again in a later step), so a slice may span many
// more candidates than the level holds rows.
template <int ITEMS>
struct ScatterLds {
    uint32_t rpre[FX_BS * ITEMS / 64];     // passes before each (item, wave) region of the tile
    unsigned long long ltot[FX_BS / 64];   // run-length totals of the waves in a round
};

template <int ITEMS, int W>
__device__ __forceinline__ void scatter_tile(const FxGraphDev &g, const FxSeg *__restrict__ segs,
                                             const FxTile *__restrict__ tmap, const int32_t *__restrict__ cand,
                                             const uint64_t *__restrict__ boff, uint64_t *lsum, const uint32_t blk,
                                             ScatterLds<ITEMS> &lds)
{
    constexpr uint32_t TILE = FX_BS * ITEMS;
    constexpr uint32_t NR = TILE / 64;  // regions: (item, wave)
    static_assert(NR <= 64, "one wave scans the region counts");
    const int32_t *crec = (const int32_t *)((const char *)cand + (size_t)blk * cand_tile_bytes(ITEMS));
    const FxTile T = tmap[blk];
    // loads that do not depend on the segment first, so their latencies
    // overlap the segment's
    const uint64_t b_lo = boff[blk], b_hi = boff[blk + 1];
    const uint32_t rc = threadIdx.x < NR ? (uint32_t)((const uint8_t *)(crec + 2 * TILE))[threadIdx.x] : 0u;
    const FxSeg &S = segs[__builtin_amdgcn_readfirstlane(T.seg)];
    const int32_t l = S.l, n = S.n;
    const uint64_t seg_base = boff[S.blk0];
    const uint64_t seg_pass = boff[S.blk0 + (S.span + TILE - 1) / TILE] - seg_base;
    const uint64_t cap = S.kind == FX_SEG_COUNT ? seg_pass : (uint64_t)S.out_cap;
    const bool overflow = seg_pass > cap;
    if (blk == S.blk0 && threadIdx.x == 0) {
        S.sum->passes = seg_pass;
        S.sum->total_out = overflow ? cap : seg_pass;
        if (!overflow) S.sum->consumed = S.span;
    }
    if (S.kind != FX_SEG_INNER && threadIdx.x == 0) lsum[blk] = 0;
    if (S.kind == FX_SEG_COUNT) return;  // nothing is written for a counting segment
    // a tile without passing candidates, or whose passes all fall past the row
    // cap, writes nothing (its run-length total is 0); uniform per workgroup
    if (b_hi == b_lo || b_lo - seg_base >= cap) {
        if (threadIdx.x == 0) lsum[blk] = 0;
        return;
    }
    const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
    if (threadIdx.x < 64) {  // exclusive prefix of the region counts
        uint32_t inc = rc;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(inc, o);
            if (lane >= (uint32_t)o) inc += u;
        }
        if (lane < NR) lds.rpre[lane] = inc - rc;
    }
    __syncthreads();
    const uint32_t nsurv = (uint32_t)(b_hi - b_lo);  // at most TILE
    const uint32_t tile0 = (blk - S.blk0) * TILE;
    const uint64_t row0 = b_lo - seg_base;          // output row of the tile's first pass
    const int32_t w1 = l + 1;
    const int32_t *in_rows = S.in.rows + T.p0 * l;  // the tile's first partial
    uint32_t bytes = 0, written = 0;
    uint64_t lbefore = 0;                           // run lengths of the tile's earlier rounds
    for (uint32_t j0 = 0; j0 < nsurv; j0 += FX_BS) {  // uniform
        const uint32_t j = j0 + threadIdx.x;          // this thread's pass, in candidate order
        const uint64_t p_out = row0 + j;
        bool f = false;
        int32_t len = 0;
        if (j < nsurv) {
            uint32_t lo = 0, hi = NR;  // the last region starting at or before pass j
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (lds.rpre[mid] <= j) lo = mid;
                else hi = mid;
            }
            const uint32_t slot = lo * 64 + (j - lds.rpre[lo]);
            const int32_t c = crec[slot];
            const uint32_t pw = (uint32_t)crec[TILE + slot];
            const int32_t pk = (int32_t)(pw & ((1u << 26) - 1u));
            const uint32_t tl = tile0 + lo * 64 + (pw >> 26);  // the candidate's index in the segment's span
            if (overflow && p_out == cap - 1) S.sum->consumed = tl + 1;  // the last row that fits
            f = p_out < cap;
            if (f) {
                const int32_t *row = in_rows + (int64_t)pk * l;
                int32_t v[W];
#pragma unroll
                for (int k = 0; k < W; k++) v[k] = (k < l) ? row[k] : -1;
                int32_t *dst = S.out.rows + p_out * (uint32_t)w1;
#pragma unroll
                for (int k = 0; k < W; k++)
                    if (k < l) dst[k] = v[k];
                dst[l] = c;
                bytes += 8u + 4u * (uint32_t)(l + w1) + (w1 < n ? 21u : 0u);
                written++;
                if (w1 < n) {
                    // candidate run of the next pattern vertex i2 = l + 1: the
                    // shortest run among its earlier neighbours, or its label bucket
                    const FxPlan *plan = S.plan;
                    const int32_t i2 = w1;
                    const uint32_t vl = plan->vl[i2];
                    const int32_t nb = plan->nback[i2];
                    int64_t best_lo = 0;
                    int32_t best_len = 0;
                    int32_t best_anc = -1;
                    if (nb == 0) {
                        best_lo = g.bptr[vl];
                        best_len = (int32_t)(g.bptr[vl + 1] - g.bptr[vl]);
                    } else {
                        best_len = 0x7fffffff;
                        for (int kk = 0; kk < nb; kk++) {
                            const int32_t b = plan->back[i2][kk];
                            const int32_t u = (b == l) ? c : pick(v, b);
                            int64_t rlo;
                            int32_t rlen;
                            run_of<scan_width<W>()>(g, u, run_key(vl, plan->bel[i2][kk]), rlo, rlen, bytes);
                            if (rlen < best_len) {
                                best_len = rlen;
                                best_lo = rlo;
                                best_anc = kk;
                            }
                        }
                    }
                    S.out.lo[p_out] = best_lo;
                    S.out.len[p_out] = best_len;
                    S.out.anc[p_out] = (int8_t)best_anc;
                    len = best_len;
                }
            }
        }
        if (S.kind == FX_SEG_INNER) {  // uniform: run lengths before each new row, in pass order
            long long inc = len;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const long long u = __shfl_up(inc, o);
                if (lane >= (uint32_t)o) inc += u;
            }
            if (lane == 63) lds.ltot[wave] = (unsigned long long)inc;
            __syncthreads();
            uint64_t mine = lbefore, tot = 0;
#pragma unroll
            for (uint32_t w = 0; w < FX_BS / 64; w++) {
                tot += lds.ltot[w];
                mine += w < wave ? lds.ltot[w] : 0ull;
            }
            if (f) S.out.off[p_out] = (int64_t)(mine + (uint64_t)(inc - len));
            lbefore += tot;
            __syncthreads();  // ltot is reused by the next round
        }
    }
    if (S.kind == FX_SEG_INNER && threadIdx.x == 0) lsum[blk] = lbefore;
    unsigned long long b = bytes;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) b += __shfl_xor(b, o);
    if (lane == 0 && b) atomicAdd(&S.sum->alg_scatter, b);
    if (S.flags & FX_PROBE_REF) {  // reference bytes: the rows written, 4 (l + 1) each
        unsigned long long r = 4ull * written * (uint32_t)w1;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) r += __shfl_xor(r, o);
        if (lane == 0 && r) atomicAdd(&S.sum->ref_scatter, r);
    }
}

template <int ITEMS, int W>
__global__ __launch_bounds__(FX_BS) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_scatter(
    FxGraphDev g, const FxSeg *__restrict__ segs, const FxTile *__restrict__ tmap, const int32_t *__restrict__ cand,
    const uint64_t *__restrict__ boff, uint64_t *lsum)
{
    __shared__ ScatterLds<ITEMS> lds;
    scatter_tile<ITEMS, W>(g, segs, tmap, cand, boff, lsum, blockIdx.x, lds);
}

template <int ITEMS, int W>
__global__ __launch_bounds__(FX_BS) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_scatter_chain(
    FxGraphDev g, const FxSeg *__restrict__ segs, const FxTile *__restrict__ tmap, const int32_t *__restrict__ cand,
    const uint64_t *__restrict__ boff, uint64_t *lsum, const FxChainCtl *ctl)
{
    __shared__ ScatterLds<ITEMS> lds;
    const uint32_t nb = ctl->nblocks;
    for (uint32_t b = blockIdx.x; b < nb; b += gridDim.x) {
        scatter_tile<ITEMS, W>(g, segs, tmap, cand, boff, lsum, b, lds);
        __syncthreads();  // the tile's LDS is reused by the next
    }
}

// Adds each workgroup's offset (scan of lsum within its segment) to the
// run-length prefixes k_scatter wrote, and closes each inner level with
// off[N] and the level's candidate total.
template <int ITEMS>
__device__ __forceinline__ void fix_off_tile(const FxSeg *__restrict__ segs, const FxTile *__restrict__ tmap,
                                             const uint64_t *__restrict__ boff, const uint64_t *__restrict__ loff,
                                             const uint32_t blk)
{
    constexpr uint32_t TILE = FX_BS * ITEMS;
    const FxSeg &S = segs[__builtin_amdgcn_readfirstlane(tmap[blk].seg)];
    if (S.kind != FX_SEG_INNER) return;
    const uint64_t seg_base = boff[S.blk0];
    const uint64_t cap = S.out_cap;
    const uint64_t r0 = min(boff[blk] - seg_base, cap), r1 = min(boff[blk + 1] - seg_base, cap);
    const uint64_t add = loff[blk] - loff[S.blk0];
    if (add)
        for (uint64_t r = r0 + threadIdx.x; r < r1; r += FX_BS) S.out.off[r] += (int64_t)add;
    if (blk == S.blk0 && threadIdx.x == 0) {
        const uint32_t nblk = (S.span + TILE - 1) / TILE;
        const uint64_t N = min(boff[S.blk0 + nblk] - seg_base, cap);
        const uint64_t total = loff[S.blk0 + nblk] - loff[S.blk0];
        S.out.off[N] = (int64_t)total;
        S.sum->t_next = total;
    }
}

template <int ITEMS>
__global__ __launch_bounds__(FX_BS) void k_fix_off(const FxSeg *__restrict__ segs, const FxTile *__restrict__ tmap,
                                                   const uint64_t *__restrict__ boff, const uint64_t *__restrict__ loff)
{
    fix_off_tile<ITEMS>(segs, tmap, boff, loff, blockIdx.x);
}

template <int ITEMS>
__global__ __launch_bounds__(FX_BS) void k_fix_off_chain(const FxSeg *__restrict__ segs,
                                                         const FxTile *__restrict__ tmap,
                                                         const uint64_t *__restrict__ boff,
                                                         const uint64_t *__restrict__ loff, const FxChainCtl *ctl)
{
    const uint32_t nb = ctl->nblocks;
    for (uint32_t b = blockIdx.x; b < nb; b += gridDim.x) fix_off_tile<ITEMS>(segs, tmap, boff, loff, b);
}

// ---------------------------------------------------------------------------
// Single-pass expansion: probe, ordered write and run-length offsets of a
// step in one kernel.  Each workgroup takes a ticket (tiles are handed out in
// tile order), probes its tile, and finds the passes before it in its segment
// by a decoupled look-back over the status words of the preceding tiles; it
// then writes its rows and, for inner segments, finds the run lengths before
// them the same way.  Replaces the probe, the two block scans, the scatter and
// the offset fix-up of the multi-kernel form, with the same output.
// ---------------------------------------------------------------------------

template <int ITEMS>
struct ExpandLds {
    ProbeLds<FX_BS * ITEMS> probe;
    int32_t cv[FX_BS * ITEMS];  // candidate ids (-1: did not pass)
    int32_t pi[FX_BS * ITEMS];  // their partials, relative to the tile's first
    uint32_t wc[ITEMS][FX_BS / 64];
    unsigned long long lt[ITEMS][FX_BS / 64];
    unsigned long long excl, lexcl;
    uint32_t tile;
};

template <int ITEMS, int W>
__device__ __forceinline__ void expand_tile(const FxGraphDev &g, const FxSeg *__restrict__ segs,
                                            const FxTile *__restrict__ tmap, uint64_t *cstat, uint64_t *lstat,
                                            const uint32_t blk, ExpandLds<ITEMS> &lds)
{
    constexpr uint32_t TILE = FX_BS * ITEMS;
    const FxTile T = tmap[blk];
    const FxSeg &S = segs[__builtin_amdgcn_readfirstlane(T.seg)];
    uint64_t bal[ITEMS];
    const TileMap m = probe_core<ITEMS, W, false>(g, S, T, blk, lds.probe, bal, lds.cv, lds.pi);
    const int32_t l = S.l, n = S.n;
    const uint32_t tile0 = (blk - S.blk0) * TILE;
    const uint32_t nblk = (S.span + TILE - 1) / TILE;
    const bool last = blk == S.blk0 + nblk - 1;
    if (S.kind == FX_SEG_COUNT) {  // nothing is written; no tile of the segment waits on another
        if (blk == S.blk0 && threadIdx.x == 0) {
            S.sum->passes = 0;
            S.sum->total_out = 0;
            S.sum->consumed = S.span;
        }
        return;
    }
    const uint32_t wave = threadIdx.x >> 6, lane = __lane_id();
#pragma unroll
    for (int it = 0; it < ITEMS; it++)
        if (lane == 0) lds.wc[it][wave] = (uint32_t)__popcll(bal[it]);
    __syncthreads();
    uint64_t agg = 0;
#pragma unroll
    for (int it = 0; it < ITEMS; it++)
        for (uint32_t w = 0; w < FX_BS / 64; w++) agg += lds.wc[it][w];
    if (wave == 0) {
        const uint64_t e = tile_prefix(cstat, blk, S.blk0, agg);
        if (lane == 0) lds.excl = e;
    }
    __syncthreads();
    const uint64_t excl = lds.excl;
    const uint64_t cap = S.out_cap;
    const int32_t w1 = l + 1;
    uint32_t bytes = 0;
    uint64_t pos = excl;
    // row of each item in the segment's output (written when < out_cap); kept
    // as the wave's ballot plus counts, and recomputed where needed
    auto row_of = [&](int it, uint64_t base) -> uint64_t {
        uint64_t po = base + (uint64_t)__popcll(bal[it] & lanemask_lt());
        for (uint32_t w = 0; w < wave; w++) po += lds.wc[it][w];
        return po;
    };
    int32_t lens[ITEMS];
    uint32_t written = 0;  // rows this thread wrote (the reference byte tally)
#pragma unroll
    for (int it = 0; it < ITEMS; it++) {
        const uint32_t tl = tile0 + it * FX_BS + threadIdx.x;
        const bool mat = (bal[it] >> lane) & 1ull;
        lens[it] = 0;
        const uint64_t po = row_of(it, pos);
        // the first pass past the row cap: it and the candidates after it are
        // probed again in a later step
        if (mat && po == cap) S.sum->consumed = tl;
        const bool f = mat && po < cap;
        const uint32_t p_out = (uint32_t)po;
        bytes += f ? 4u * (uint32_t)(l + w1) + (w1 < n ? 21u : 0u) : 0u;
        written += f ? 1u : 0u;
        if (f) {
            Cand<W> x;
            const int32_t *row = S.in.rows + (m.p0 + lds.pi[it * FX_BS + threadIdx.x]) * l;
#pragma unroll
            for (int k = 0; k < W; k++) x.v[k] = (k < l) ? row[k] : -1;
            x.c = lds.cv[it * FX_BS + threadIdx.x];
            int32_t *dst = S.out.rows + (uint64_t)p_out * (uint32_t)w1;
#pragma unroll
            for (int k = 0; k < W; k++)
                if (k < l) dst[k] = x.v[k];
            dst[l] = x.c;
            if (w1 < n) {
                // candidate run of the next pattern vertex i2 = l + 1: the
                // shortest run among its earlier neighbours, or its label bucket
                const FxPlan *plan = S.plan;
                const int32_t i2 = w1;
                const uint32_t vl = plan->vl[i2];
                const int32_t nb = plan->nback[i2];
                int64_t best_lo = 0;
                int32_t best_len = 0;
                int32_t best_anc = -1;
                if (nb == 0) {
                    best_lo = g.bptr[vl];
                    best_len = (int32_t)(g.bptr[vl + 1] - g.bptr[vl]);
                } else {
                    best_len = 0x7fffffff;
                    for (int kk = 0; kk < nb; kk++) {
                        const int32_t b = plan->back[i2][kk];
                        const int32_t u = (b == l) ? x.c : pick(x.v, b);
                        int64_t lo;
                        int32_t len;
                        run_of<scan_width<W>()>(g, u, run_key(vl, plan->bel[i2][kk]), lo, len, bytes);
                        if (len < best_len) {
                            best_len = len;
                            best_lo = lo;
                            best_anc = kk;
                        }
                    }
                }
                S.out.lo[p_out] = best_lo;
                S.out.len[p_out] = best_len;
                S.out.anc[p_out] = (int8_t)best_anc;
                lens[it] = best_len;
            }
        }
        for (uint32_t w = 0; w < FX_BS / 64; w++) pos += lds.wc[it][w];
    }
    const uint64_t seg_pass = excl + agg;  // meaningful in the segment's last tile
    const uint64_t nout = seg_pass < cap ? seg_pass : cap;
    if (last && threadIdx.x == 0) {
        S.sum->passes = seg_pass;
        S.sum->total_out = nout;
        if (seg_pass <= cap) S.sum->consumed = S.span;
    }
    if (S.kind == FX_SEG_INNER) {  // uniform across the workgroup
        // run lengths before each new row: wave totals per item, the tile's
        // prefix in its segment by look-back, then each lane's scan in its wave
#pragma unroll
        for (int it = 0; it < ITEMS; it++) {
            unsigned long long tot = (unsigned long long)lens[it];
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) tot += __shfl_xor(tot, o);
            if (lane == 0) lds.lt[it][wave] = tot;
        }
        __syncthreads();
        uint64_t lagg = 0;
#pragma unroll
        for (int it = 0; it < ITEMS; it++)
            for (uint32_t w = 0; w < FX_BS / 64; w++) lagg += lds.lt[it][w];
        if (wave == 0) {
            const uint64_t e = tile_prefix(lstat, blk, S.blk0, lagg);
            if (lane == 0) lds.lexcl = e;
        }
        __syncthreads();
        uint64_t before = lds.lexcl;
        uint64_t rows = excl;
#pragma unroll
        for (int it = 0; it < ITEMS; it++) {
            long long inc = lens[it];
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const long long u = __shfl_up(inc, o);
                if (lane >= (uint32_t)o) inc += u;
            }
            uint64_t mine = before;
            for (uint32_t w = 0; w < wave; w++) mine += lds.lt[it][w];
            const uint64_t po = row_of(it, rows);
            if (((bal[it] >> lane) & 1ull) && po < cap) S.out.off[po] = (int64_t)(mine + (uint64_t)(inc - lens[it]));
            for (uint32_t w = 0; w < FX_BS / 64; w++) {
                before += lds.lt[it][w];
                rows += lds.wc[it][w];
            }
        }
        if (last && threadIdx.x == 0) {  // close the level: off[N] and its candidate total
            S.out.off[nout] = (int64_t)before;
            S.sum->t_next = before;
        }
    }
    unsigned long long b = bytes;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) b += __shfl_xor(b, o);
    if (lane == 0 && b) atomicAdd(&S.sum->alg_scatter, b);
    if (S.flags & FX_PROBE_REF) {  // reference bytes: the rows written, 4 (l + 1) each
        unsigned long long r = 4ull * written * (uint32_t)w1;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) r += __shfl_xor(r, o);
        if (lane == 0 && r) atomicAdd(&S.sum->ref_scatter, r);
    }
}

// One workgroup per tile; the tile is the workgroup's ticket, not its index.
template <int ITEMS, int W>
__global__ __launch_bounds__(FX_BS) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_expand(
    FxGraphDev g, const FxSeg *__restrict__ segs, const FxTile *__restrict__ tmap, uint64_t *cstat, uint64_t *lstat,
    uint32_t *ticket)
{
    __shared__ ExpandLds<ITEMS> lds;
    if (threadIdx.x == 0) lds.tile = atomicAdd(ticket, 1u);
    __syncthreads();
    expand_tile<ITEMS, W>(g, segs, tmap, cstat, lstat, lds.tile, lds);
}

// The same over a fixed grid: each workgroup takes tickets until they pass
// the step's tile count from the scheduler.
template <int ITEMS, int W>
__global__ __launch_bounds__(FX_BS) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_expand_chain(
    FxGraphDev g, const FxSeg *__restrict__ segs, const FxTile *__restrict__ tmap, uint64_t *cstat, uint64_t *lstat,
    uint32_t *ticket, const FxChainCtl *ctl)
{
    __shared__ ExpandLds<ITEMS> lds;
    const uint32_t nb = ctl->nblocks;
    for (;;) {
        if (threadIdx.x == 0) lds.tile = atomicAdd(ticket, 1u);
        __syncthreads();
        const uint32_t b = lds.tile;
        if (b >= nb) break;  // uniform across the workgroup
        expand_tile<ITEMS, W>(g, segs, tmap, cstat, lstat, b, lds);
        __syncthreads();  // the tile's LDS (and its ticket) is reused by the next
    }
}

// ---------------------------------------------------------------------------
// Greedy maximal independent set of one query's complete embeddings of this
// step, in rank order, one workgroup per query (Section 2.4.3; the used set U
// is the bitmap of Section 3.2.2).  Embeddings are taken in chunks of at most
// FX_GREEDY_VN vertices.  Per chunk: drop embeddings that meet U, hash their
// data vertices into LDS slots (the overlap structure), then run rounds: every
// undecided embedding writes ((~round) << 16 | rank) into its slots with an
// atomic min, and is selected when it holds the minimum of all its slots --
// i.e. it ranks below every undecided embedding it overlaps.  Slot value 0
// marks a slot taken by a selected embedding; an undecided embedding that
// meets one is dropped.  The lowest-ranked undecided embedding always wins
// its round, so a chunk ends after at most (embeddings) rounds, and the
// selection equals the sequential greedy's.  The rounds touch LDS only; the
// chunk's selections go to U, the support count and the selection list in
// one pass after it.  The first chunk skips the U test: the probe has just
// tested every embedding against the same U.
// ---------------------------------------------------------------------------

// Slot of data vertex v in a table of 2^bits slots (Fibonacci hashing: the
// top bits of the product with 2^64 / golden ratio).
__device__ __forceinline__ uint32_t lds_hash(int32_t v, uint32_t bits)
{
    return (uint32_t)(((uint64_t)(uint32_t)v * 0x9e3779b97f4a7c15ULL) >> (64 - bits));
}

__device__ __forceinline__ bool used_coherent(const uint32_t *U, int32_t v)
{
    // bypass the per-CU cache: this workgroup sets bits of U while it runs
    const uint32_t w = __hip_atomic_load(&U[(uint32_t)v >> 5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (w >> ((uint32_t)v & 31u)) & 1u;
}

// Sequential finish of a chunk by one wave, once the parallel rounds make
// little progress (long chains of overlapping embeddings need one round per
// link).  The wave walks the undecided embeddings in rank order, 64 at a
// time: a lane whose slots are taken is dropped; otherwise the lowest
// undecided lane is the lowest-ranked undecided embedding, so it is selected,
// its slots are taken, and the lanes sharing a slot with it are dropped.
// Decided embeddings of the rounds before are consistent with the sequential
// greedy (a selected embedding has no undecided lower-ranked neighbour), so
// the result is still the sequential greedy's.  Selections are marked 3; the
// caller writes them out.
__device__ void greedy_tail(uint8_t *state, const uint16_t *slot, uint32_t *hval, uint32_t nb, int32_t n)
{
    const uint32_t lane = threadIdx.x;  // wave 0
    for (uint32_t base = 0; base < nb; base += 64) {
        const uint32_t e = base + lane;
        const bool und = e < nb && state[e] == 0;
        uint32_t s[FX_MAXN];
        bool blocked = false;
#pragma unroll
        for (int j = 0; j < FX_MAXN; j++) {
            s[j] = (und && j < n) ? (uint32_t)slot[e * n + j] : 0xffffffffu;
            if (und && j < n) blocked = blocked || hval[s[j]] == 0u;
        }
        if (und && blocked) state[e] = 2;
        uint64_t M = __ballot(und && !blocked);
        while (M) {
            const uint32_t f = (uint32_t)__ffsll((unsigned long long)M) - 1;
            const uint32_t ef = base + f;
            bool conf = false;
            for (int j = 0; j < n; j++) {
                const uint32_t fs = slot[ef * n + j];
#pragma unroll
                for (int k = 0; k < FX_MAXN; k++) conf = conf || s[k] == fs;
                if (lane == (uint32_t)j) hval[fs] = 0u;
            }
            const bool in_m = (M >> lane) & 1ull;
            const bool drop = in_m && lane != f && conf;
            if (lane == f) state[e] = 3;
            if (drop) state[e] = 2;
            M &= ~(1ull << f);
            M &= ~__ballot(drop);
        }
    }
}

template <bool CHAIN>
__global__ __launch_bounds__(FX_BS) void k_greedy(const FxSeg *__restrict__ segs, const FxChainCtl *ctl)
{
    static_assert(FX_GREEDY_H == 4096 && 2 * FX_GREEDY_VN <= FX_GREEDY_H, "a chunk's vertices fill at most half");
    // 32-bit slot keys: a chunk's ranks and rounds (at most one per embedding)
    // stay below 2^16, and no key is 0 (the taken mark)
    static_assert(FX_GREEDY_VN < 0xffff, "rank and round must fit 16 bits");
    __shared__ int32_t hkey[FX_GREEDY_H];
    __shared__ uint32_t hval[FX_GREEDY_H];  // (~round) << 16 | rank in chunk; 0 = taken
    __shared__ uint16_t slot[FX_GREEDY_VN];
    __shared__ uint8_t state[FX_GREEDY_VN];  // 0 undecided, 1 selected, 2 out, 3 selected by the tail
    __shared__ uint32_t undecided, nsel;
    __shared__ unsigned long long sel_base;
    if (CHAIN && blockIdx.x >= ctl->nsegs) return;  // a fixed grid: one workgroup per possible segment
    const FxSeg &S = segs[blockIdx.x];
    if (S.kind != FX_SEG_GREEDY) return;
    const int32_t n = S.n;
    const uint64_t N = S.sum->total_out;
    const int32_t *rows = S.out.rows;
    const uint32_t B = FX_GREEDY_VN / (uint32_t)n;  // embeddings per chunk
    constexpr uint32_t kTailBelow = 64;              // undecided embeddings one wave finishes
    uint32_t rounds_total = 0;
    unsigned long long selected_total = 0;           // (thread 0) selections of this launch
    for (uint64_t c0 = 0; c0 < N; c0 += B) {
        const uint32_t nb = (uint32_t)((N - c0) < B ? (N - c0) : B);
        // a table of at least twice the chunk's vertices (at least 64 slots):
        // small chunks clear and probe only that part of the LDS table
        uint32_t hbits = 6;
        while ((1u << hbits) < 2 * nb * (uint32_t)n) hbits++;
        const uint32_t hmask = (1u << hbits) - 1;
        for (uint32_t k = threadIdx.x; k <= hmask; k += FX_BS) {
            hkey[k] = -1;
            hval[k] = ~0u;
        }
        if (threadIdx.x == 0) nsel = 0;
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < nb; e += FX_BS) {
            const int32_t *row = rows + (c0 + e) * n;
            // the probe tested every embedding against U as it stood before
            // this launch; only selections of earlier chunks can have changed it
            bool out = false;
            if (c0 > 0)
                for (int j = 0; j < n; j++) out = out || used_coherent(S.U, row[j]);
            state[e] = out ? 2 : 0;
            if (!out) {
                for (int j = 0; j < n; j++) {
                    const int32_t v = row[j];
                    uint32_t h = lds_hash(v, hbits);
                    while (true) {  // linear probing; at most H/2 keys per chunk
                        const int32_t prev = atomicCAS(&hkey[h], -1, v);
                        if (prev == -1 || prev == v) break;
                        h = (h + 1) & hmask;
                    }
                    slot[e * n + j] = (uint16_t)h;
                }
            }
        }
        __syncthreads();
        // rounds touch LDS only; the selections are written out after the chunk
        bool tail = false;
        uint32_t prev_und = nb;
        for (uint32_t r = 0; r <= nb; r++) {  // a chunk needs at most nb rounds
            if (threadIdx.x == 0) undecided = 0;
            for (uint32_t e = threadIdx.x; e < nb; e += FX_BS) {
                if (state[e] != 0) continue;
                bool out = false;
                for (int j = 0; j < n; j++) out = out || (hval[slot[e * n + j]] == 0u);
                if (out) {
                    state[e] = 2;
                    continue;
                }
                const uint32_t key = ((0xffffu - r) << 16) | e;
                for (int j = 0; j < n; j++) atomicMin(&hval[slot[e * n + j]], key);
            }
            __syncthreads();
            uint32_t mine_undecided = 0;
            for (uint32_t e = threadIdx.x; e < nb; e += FX_BS) {
                if (state[e] != 0) continue;
                const uint32_t key = ((0xffffu - r) << 16) | e;
                bool mine = true;
                for (int j = 0; j < n; j++) mine = mine && (hval[slot[e * n + j]] == key);
                if (mine) {
                    state[e] = 1;
                    for (int j = 0; j < n; j++) hval[slot[e * n + j]] = 0u;
                } else {
                    mine_undecided++;
                }
            }
            if (mine_undecided) atomicAdd(&undecided, mine_undecided);
            __syncthreads();
            const uint32_t und = undecided;
            rounds_total++;
            __syncthreads();  // everyone has read `undecided` before it is reset
            if (und == 0) break;
            // few left, or a round that decided under 1/8 of them: chains
            if (und <= kTailBelow || (r >= 1 && (prev_und - und) * 8 < prev_und)) {
                tail = true;
                break;
            }
            prev_und = und;
            if (r == nb && threadIdx.x == 0) atomicAdd(&S.sum->error, 1ULL);  // cannot happen
        }
        if (tail) {  // uniform
            if (threadIdx.x < 64) greedy_tail(state, slot, hval, nb, n);
            __syncthreads();
        }
        // write out the chunk's selections: U bits, the support count and,
        // when asked for, the selected rows with their ranks
        constexpr int kPer = (FX_GREEDY_VN + FX_BS - 1) / FX_BS;  // embeddings of a chunk per thread
        uint32_t my_pos[kPer];
        uint64_t sh1 = 0, sh2 = 0;  // digest of the selected set (same hash chain as the count's)
#pragma unroll
        for (int k = 0; k < kPer; k++) {
            const uint32_t e = threadIdx.x + (uint32_t)k * FX_BS;
            my_pos[k] = 0xffffffffu;
            if (e >= nb || (state[e] != 1 && state[e] != 3)) continue;
            const int32_t *row = rows + (c0 + e) * n;
            uint64_t a = kSeed1, b = kSeed2;
            for (int j = 0; j < n; j++) {
                const uint32_t v = (uint32_t)row[j];
                atomicOr(&S.U[v >> 5], 1u << (v & 31u));
                a = mix64(a ^ (uint64_t)v);
                b = mix64(b ^ (uint64_t)v);
            }
            sh1 += a;
            sh2 ^= b;
            my_pos[k] = atomicAdd(&nsel, 1u);
        }
        {
            unsigned long long s1 = sh1, s2 = sh2;
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                s1 += __shfl_xor(s1, o);
                s2 ^= __shfl_xor(s2, o);
            }
            if (__lane_id() == 0 && (s1 | s2)) {
                atomicAdd(&S.sum->sel_d0, s1);
                atomicXor(&S.sum->sel_d1, s2);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned long long c = nsel;
            sel_base = c ? atomicAdd(&S.sum->support, c) : 0ULL;
            selected_total += c;
        }
        if (S.sel_rows) {  // selections are kept only when the caller asked for them
            __syncthreads();
            const unsigned long long base = sel_base;
#pragma unroll
            for (int k = 0; k < kPer; k++) {
                const uint32_t e = threadIdx.x + (uint32_t)k * FX_BS;
                if (my_pos[k] == 0xffffffffu) continue;
                const int32_t *row = rows + (c0 + e) * n;
                const unsigned long long pos = base + my_pos[k];
                for (int j = 0; j < n; j++) S.sel_rows[pos * n + j] = row[j];
                S.sel_rank[pos] = S.rank_base + (int64_t)(c0 + e);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(&S.sum->rounds, (unsigned long long)rounds_total);
        if (S.flags & FX_PROBE_REF)  // reference bytes: every embedding read once, the selections written
            atomicAdd(&S.sum->ref_greedy, 4ull * (unsigned long long)n * (N + selected_total));
    }
}

// ---------------------------------------------------------------------------
// Device scheduler of a chain of steps (one thread).  It does for the chained
// queries what the engine's host side does between two steps: advance every
// query from the counters of its last segment, retire the finished ones
// (VERDICT at tau or at the exactness bound, the count cap, an exhausted
// search; a FULL query moves from its support phase to its count phase), and
// choose every open query's next segment: the deepest level with candidates
// left, a span aimed at the rows the segment may write from the level's last
// passing rate, within the query's share of the step's candidates.
// ---------------------------------------------------------------------------

__device__ int32_t chain_deepest(const FxChainQuery &q)
{
    for (int32_t l = q.n - 1; l >= 0; l--)
        if (q.cur[l] < q.T[l]) return l;
    return -1;
}

__device__ void chain_restart(FxChainQuery &q)
{
    for (int l = 0; l <= q.n; l++) q.T[l] = q.cur[l] = 0, q.nparts[l] = 0;
    q.T[0] = q.bucket0;
    q.nparts[0] = 1;
    q.deep = chain_deepest(q);
}

__device__ void chain_advance(FxChainQuery &q)
{
    q.last = *q.sum;
    if (q.seg_l < 0) return;
    const FxSummary &S = q.last;
    const int32_t l = q.seg_l;
    const uint64_t taken = S.consumed;
    q.seg_l = -1;
    if (S.error || taken == 0 || taken > q.seg_span) {
        q.error = 1;
        q.done = 1;
        return;
    }
    const double share = (double)taken / (double)q.seg_span;
    q.cur[l] = q.seg_t0 + taken;
    q.reoffered += q.seg_span - taken;
    q.probed += q.seg_span;
    if (q.phase == FX_CQ_SUPPORT) q.probed_support += q.seg_span;
    q.rate[l] = (double)S.passes / (double)q.seg_span;
    q.alg_probe_credit += (double)(S.alg_probe - q.alg_probe_seen) * share;
    q.alg_probe_seen = S.alg_probe;
    q.ref_probe_credit += (double)(S.ref_probe - q.ref_probe_seen) * share;
    q.ref_probe_seen = S.ref_probe;
    q.ref_row_credit += (double)(S.ref_probe_row - q.ref_row_seen) * share;
    q.ref_row_seen = S.ref_probe_row;
    q.steps++;
    if (q.seg_kind == FX_SEG_INNER) {
        q.nparts[l + 1] = (int64_t)S.total_out;
        q.T[l + 1] = S.t_next;
        q.cur[l + 1] = 0;
    } else if (q.seg_kind == FX_SEG_GREEDY) {
        q.rank_base += (int64_t)S.total_out;
    }
    q.deep = chain_deepest(q);
}

__device__ void chain_check(FxChainQuery &q)
{
    if (q.done) return;
    const FxSummary &S = q.last;
    bool fin = false;
    if (q.phase == FX_CQ_SUPPORT && q.verdict) {
        const int64_t sup = (int64_t)S.support;
        if (sup >= q.tau_eff) {
            fin = true;
            q.exit = FX_EXIT_REACHED;
        } else if (q.deep >= 0) {
            uint64_t roots = q.T[0] - q.cur[0];
            if (q.deep >= 1) roots += (uint64_t)q.nparts[1];
            const int64_t room = q.upper_bound - sup > 0 ? q.upper_bound - sup : 0;
            const int64_t possible = roots < (uint64_t)room ? (int64_t)roots : room;
            if (sup + possible < q.tau_eff) {
                fin = true;
                q.exit = FX_EXIT_BOUND;
            }
        }
    }
    if (q.phase == FX_CQ_COUNT && !q.mni && (int64_t)S.count >= q.count_cap) fin = true;
    if (!fin && q.deep < 0) {
        if (q.phase == FX_CQ_SUPPORT && q.full) {
            q.phase = FX_CQ_COUNT;
            chain_restart(q);
        } else {
            fin = true;
        }
    }
    if (fin) q.done = 1;
}

__global__ void k_sched(FxChainQuery *qs, FxChainCtl *ctl, FxSeg *segs, uint32_t *blk0s, uint32_t tile, int32_t final)
{
    if (threadIdx.x != 0) return;
    const int32_t nq = ctl->nq;
    uint64_t n_open = 0;
    for (int32_t k = 0; k < nq; k++) {
        FxChainQuery &q = qs[k];
        chain_advance(q);
        chain_check(q);
        n_open += (!q.done && q.deep >= 0) ? 1 : 0;
    }
    uint32_t nsegs = 0, nblocks = 0;
    if (!final) {
        uint64_t budget = ctl->budget;
        const uint64_t share = ctl->budget / (n_open > 0 ? n_open : 1);
        for (int32_t k = 0; k < nq && budget > 0; k++) {
            FxChainQuery &q = qs[(ctl->rot + (uint32_t)k) % (uint32_t)nq];
            if (q.done || q.deep < 0) continue;
            const int32_t l = q.deep;
            const bool last = l == q.n - 1;
            int32_t kind, flags = 0;
            uint64_t out_cap = (uint64_t)q.cap;
            if (q.phase == FX_CQ_SUPPORT) {
                flags = FX_PROBE_UFILTER | (q.sym ? FX_PROBE_SYM : 0);
                kind = last ? FX_SEG_GREEDY : FX_SEG_INNER;
                if (last) out_cap = q.last_span < (uint64_t)q.cap ? q.last_span : (uint64_t)q.cap;
            } else {
                const bool end = q.leaf_count ? (l == q.n - 2) : last;
                flags = end ? (q.leaf_count ? FX_PROBE_LEAF
                                            : (FX_PROBE_COUNT | (q.hash ? FX_PROBE_HASH : 0) |
                                               (q.mni ? FX_PROBE_IMAGES : 0)))
                            : 0;
                kind = end ? FX_SEG_COUNT : FX_SEG_INNER;
            }
            uint64_t want;
            if (kind == FX_SEG_COUNT) {
                want = FX_COUNT_SPAN > share ? FX_COUNT_SPAN : share;
            } else {
                const double r = q.rate[l] > 1e-9 ? q.rate[l] : 1e-9;
                if (r >= 1.0) {
                    want = out_cap;
                } else {
                    const double w = FX_FILL * (double)out_cap / r;
                    want = (uint64_t)(w < 2147483648.0 ? w : 2147483648.0);
                }
                if (want < out_cap) want = out_cap;
                const uint64_t hi = out_cap > share ? out_cap : share;
                if (want > hi) want = hi;
            }
            uint64_t span = q.T[l] - q.cur[l];
            if (span > want) span = want;
            if (span > budget) span = budget;
            if (span == 0) continue;
            if (q.ref_bytes) flags |= FX_PROBE_REF;
            FxSeg &S = segs[nsegs];
            S.in = q.lev[l];
            S.out = q.lev[l + 1];
            S.plan = q.plan;
            S.U = q.U;
            S.sum = q.sum;
            S.sel_rows = q.sel_rows;
            S.sel_rank = q.sel_rank;
            S.img = q.img;
            S.img_words = q.img_words;
            S.nparts = q.nparts[l];
            S.t0 = q.cur[l];
            S.rank_base = q.rank_base;
            S.span = (uint32_t)span;
            S.out_cap = (uint32_t)(out_cap < 0xffffffffull ? out_cap : 0xffffffffull);
            S.blk0 = nblocks;
            S.n = q.n;
            S.l = l;
            S.flags = flags;
            S.kind = kind;
            blk0s[nsegs] = nblocks;
            nblocks += (uint32_t)((span + tile - 1) / tile);
            budget -= span;
            q.seg_l = l;
            q.seg_kind = kind;
            q.seg_t0 = q.cur[l];
            q.seg_span = (uint32_t)span;
            nsegs++;
        }
        ctl->rot++;
        if (nsegs) ctl->steps++;
    }
    blk0s[nsegs] = nblocks;
    ctl->nsegs = nsegs;
    ctl->nblocks = nblocks;
}

// ---------------------------------------------------------------------------
// Exact maximum independent set (Section 2.4.2) for small instances: one
// workgroup.  Embeddings with the same vertex set are interchangeable for
// independence, so each row's ids are sorted, rows are reduced to distinct
// sets (first occurrence kept), the overlap relation of the sets becomes LDS
// bitsets, and one lane searches for a largest independent set by branch and
// bound: take the open set that overlaps most open sets, search with it
// (dropping everything it overlaps) and without it, and prune a branch that
// cannot beat the best found.  Bounds: independent sets never share a vertex,
// so among the open sets at most one per distinct smallest vertex, and one
// per distinct largest vertex, can be chosen -- and at most (the vertices the
// open sets cover) / n of them (when the sets cover at most 256 vertices).
// ---------------------------------------------------------------------------

constexpr int kMisWords = FX_MIS_MAX_SETS / 64;

__global__ __launch_bounds__(256) void k_mis(int32_t *rows, int32_t count, int32_t n, uint64_t *hash_scratch,
                                             FxMisOut *out)
{
    __shared__ int32_t set_first[FX_MIS_MAX_SETS];     // row of each distinct set
    __shared__ uint8_t grp_lo[FX_MIS_MAX_SETS];        // class of the set's smallest vertex
    __shared__ uint8_t grp_hi[FX_MIS_MAX_SETS];        // class of the set's largest vertex
    __shared__ uint64_t vmask[FX_MIS_MAX_SETS][kMisWords];  // the set's vertices, as local ids
    __shared__ int32_t local_ids[FX_MIS_MAX_SETS];     // data vertex of each local id
    __shared__ int32_t nlocal;
    __shared__ uint64_t adj[FX_MIS_MAX_SETS][kMisWords];  // overlap bitsets
    __shared__ uint64_t stack_p[FX_MIS_MAX_SETS + 2][kMisWords];
    __shared__ int32_t stack_size[FX_MIS_MAX_SETS + 2];
    __shared__ int32_t nsets;
    // 1. sort every row's vertex ids; hash the sorted row
    for (int32_t r = threadIdx.x; r < count; r += blockDim.x) {
        int32_t *row = rows + (int64_t)r * n;
        for (int32_t a = 1; a < n; a++) {  // insertion sort, n <= 16
            const int32_t v = row[a];
            int32_t b = a - 1;
            while (b >= 0 && row[b] > v) {
                row[b + 1] = row[b];
                b--;
            }
            row[b + 1] = v;
        }
        uint64_t h = kSeed1;
        for (int32_t a = 0; a < n; a++) h = mix64(h ^ (uint64_t)(uint32_t)row[a]);
        hash_scratch[r] = h;
    }
    __syncthreads();
    // 2. distinct sets: row r is kept when no earlier row holds the same set
    //    (taken in row order by one wave so the kept rows stay ordered; the
    //    running count is a wave-uniform register)
    if (threadIdx.x < 64) {
        int32_t kept = 0;
        for (int32_t base = 0; base < count; base += 64) {
            const int32_t r = base + (int32_t)threadIdx.x;
            bool first = r < count;
            if (first) {
                const uint64_t h = hash_scratch[r];
                const int32_t *row = rows + (int64_t)r * n;
                for (int32_t q = 0; q < r && first; q++) {
                    if (hash_scratch[q] != h) continue;
                    const int32_t *other = rows + (int64_t)q * n;
                    bool same = true;
                    for (int32_t a = 0; a < n; a++) same = same && other[a] == row[a];
                    first = !same;
                }
            }
            const uint64_t m = __ballot(first);
            const int32_t k = kept + __popcll(m & lanemask_lt());
            if (first && k < FX_MIS_MAX_SETS) set_first[k] = r;
            kept += __popcll(m);
        }
        if (threadIdx.x == 0) nsets = kept;
    }
    __syncthreads();
    const int32_t K = nsets < FX_MIS_MAX_SETS ? nsets : FX_MIS_MAX_SETS;
    if (nsets > FX_MIS_MAX_SETS) {
        if (threadIdx.x == 0) {
            out->mis = -1;
            out->sets = nsets;
            out->status = 1;
            out->nodes = 0;
        }
        return;
    }
    // 3. overlap bitsets of the distinct sets (sorted rows: a merge)
    for (int32_t i = threadIdx.x; i < FX_MIS_MAX_SETS; i += blockDim.x)
        for (int w = 0; w < kMisWords; w++) adj[i][w] = 0;
    __syncthreads();
    for (int32_t pq = threadIdx.x; pq < K * K; pq += blockDim.x) {
        const int32_t i = pq / K, j = pq % K;
        if (i == j) continue;
        const int32_t *a = rows + (int64_t)set_first[i] * n;
        const int32_t *b = rows + (int64_t)set_first[j] * n;
        int32_t x = 0, y = 0;
        bool meet = false;
        while (x < n && y < n && !meet) {
            if (a[x] == b[y]) meet = true;
            else if (a[x] < b[y]) x++;
            else y++;
        }
        if (meet) atomicOr((unsigned long long *)&adj[i][j >> 6], 1ull << (j & 63));
    }
    // classes of equal smallest (largest) vertex, numbered by their first set
    for (int32_t i = threadIdx.x; i < K; i += blockDim.x) {
        const int32_t *a = rows + (int64_t)set_first[i] * n;
        int32_t lo = i, hi = i;
        for (int32_t j = 0; j < i; j++) {
            const int32_t *b = rows + (int64_t)set_first[j] * n;
            if (lo == i && b[0] == a[0]) lo = j;
            if (hi == i && b[n - 1] == a[n - 1]) hi = j;
        }
        grp_lo[i] = (uint8_t)lo;
        grp_hi[i] = (uint8_t)hi;
    }
    // local ids of the vertices the sets cover (at most 256, else no cover bound)
    if (threadIdx.x == 0) {
        int32_t nl = 0;
        for (int32_t i = 0; i < K && nl >= 0; i++) {
            const int32_t *a = rows + (int64_t)set_first[i] * n;
            for (int w = 0; w < kMisWords; w++) vmask[i][w] = 0;
            for (int32_t x = 0; x < n && nl >= 0; x++) {
                int32_t id = -1;
                for (int32_t q = 0; q < nl; q++)
                    if (local_ids[q] == a[x]) id = q;
                if (id < 0) {
                    if (nl == FX_MIS_MAX_SETS) {
                        nl = -1;
                        break;
                    }
                    local_ids[nl] = a[x];
                    id = nl++;
                }
                vmask[i][id >> 6] |= 1ull << (id & 63);
            }
        }
        nlocal = nl;
    }
    __syncthreads();
    // 4. branch and bound (one lane)
    if (threadIdx.x != 0) return;
    const bool cover_bound = nlocal >= 0;
    int32_t best = 0;
    uint64_t nodes = 0;
    int32_t top = 0;
    for (int w = 0; w < kMisWords; w++) {
        const int32_t lo = w * 64;
        stack_p[0][w] = K >= lo + 64 ? ~0ull : (K > lo ? ((1ull << (K - lo)) - 1) : 0ull);
    }
    stack_size[0] = 0;
    top = 1;
    int32_t status = 0;
    while (top > 0) {
        top--;
        uint64_t P[kMisWords];
        int32_t open = 0;
        for (int w = 0; w < kMisWords; w++) {
            P[w] = stack_p[top][w];
            open += __popcll(P[w]);
        }
        const int32_t size = stack_size[top];
        if (++nodes > FX_MIS_MAX_NODES) {
            status = 2;
            break;
        }
        if (size + open <= best) continue;
        if (open == 0) {
            best = size;  // size > best here
            continue;
        }
        // the bounds, and the open set with the most open neighbours
        uint64_t cl[kMisWords] = {}, ch[kMisWords] = {}, cv[kMisWords] = {};
        int32_t v = -1, vdeg = -1;
        for (int w = 0; w < kMisWords; w++) {
            uint64_t m = P[w];
            while (m) {
                const int32_t i = w * 64 + __ffsll((unsigned long long)m) - 1;
                m &= m - 1;
                cl[grp_lo[i] >> 6] |= 1ull << (grp_lo[i] & 63);
                ch[grp_hi[i] >> 6] |= 1ull << (grp_hi[i] & 63);
                if (cover_bound)
                    for (int u = 0; u < kMisWords; u++) cv[u] |= vmask[i][u];
                int32_t d = 0;
                for (int u = 0; u < kMisWords; u++) d += __popcll(adj[i][u] & P[u]);
                if (d > vdeg) {
                    vdeg = d;
                    v = i;
                }
            }
        }
        int32_t blo = 0, bhi = 0, bcv = 0;
        for (int w = 0; w < kMisWords; w++) {
            blo += __popcll(cl[w]);
            bhi += __popcll(ch[w]);
            bcv += __popcll(cv[w]);
        }
        int32_t bound = blo < bhi ? blo : bhi;
        if (cover_bound && bcv / n < bound) bound = bcv / n;
        if (size + bound <= best) continue;
        if (vdeg == 0) {  // no open set overlaps another: take them all
            best = size + open > best ? size + open : best;
            continue;
        }
        // without v (searched second), then with v (searched first)
        for (int w = 0; w < kMisWords; w++) stack_p[top][w] = P[w];
        stack_p[top][v >> 6] &= ~(1ull << (v & 63));
        stack_size[top] = size;
        top++;
        for (int w = 0; w < kMisWords; w++) stack_p[top][w] = P[w] & ~adj[v][w];
        stack_p[top][v >> 6] &= ~(1ull << (v & 63));
        stack_size[top] = size + 1;
        top++;
    }
    out->mis = status ? -1 : best;
    out->sets = K;
    out->status = status;
    out->nodes = nodes;
}

// Admission / phase start of queries: level 0 is the single empty partial
// whose candidate run is the label bucket of pattern vertex 0.
__global__ void k_init(FxGraphDev g, const FxInit *__restrict__ inits)
{
    const FxInit &I = inits[blockIdx.x];
    {
        const uint32_t *src = (const uint32_t *)&I.plan;
        uint32_t *dst = (uint32_t *)I.plan_dst;
        for (uint32_t k = threadIdx.x; k < sizeof(FxPlan) / 4; k += blockDim.x) dst[k] = src[k];
    }
    __syncthreads();  // the plan is read below
    if (I.clear_u)
        for (uint64_t k = threadIdx.x; k < I.u_words; k += blockDim.x) I.U[k] = 0u;
    if (I.clear_sum && threadIdx.x < sizeof(FxSummary) / 8) ((unsigned long long *)I.sum)[threadIdx.x] = 0ULL;
    if (threadIdx.x == 0) {
        const uint32_t vl = I.plan.vl[0];
        I.lev0.lo[0] = g.bptr[vl];
        I.lev0.len[0] = (int32_t)(g.bptr[vl + 1] - g.bptr[vl]);
        I.lev0.anc[0] = -1;
        I.lev0.off[0] = 0;
        I.lev0.off[1] = g.bptr[vl + 1] - g.bptr[vl];
    }
}

// Set bits of image bitmap blockIdx.x.
__global__ __launch_bounds__(1024) void k_mni_count(const uint32_t *__restrict__ img, uint64_t words,
                                                    unsigned long long *counts)
{
    __shared__ unsigned long long part[1024 / 64];
    const uint32_t *b = img + (uint64_t)blockIdx.x * words;
    unsigned long long c = 0;
    for (uint64_t k = threadIdx.x; k < words; k += 1024) c += (unsigned long long)__popc(b[k]);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o);
    if (__lane_id() == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < 1024 / 64; w++) t += part[w];
        counts[blockIdx.x] = t;
    }
}

__global__ void k_mni_min(const unsigned long long *__restrict__ counts, int32_t n, unsigned long long *out)
{
    if (threadIdx.x != 0) return;
    unsigned long long m = counts[0];
    for (int32_t j = 1; j < n; j++) m = counts[j] < m ? counts[j] : m;
    *out = m;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t fx_launch_init(hipStream_t s, const FxGraphDev &g, const FxInit *inits, int32_t ninit)
{
    if (ninit <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init, dim3(ninit), dim3(256), 0, s, g, inits);
    return hipGetLastError();
}

hipError_t fx_launch_mni(hipStream_t s, const uint32_t *img, uint64_t words, int32_t n,
                         unsigned long long *counts, unsigned long long *out)
{
    if (n <= 0 || n > FX_MAXN) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mni_count, dim3(n), dim3(1024), 0, s, img, words, counts);
    hipLaunchKernelGGL(k_mni_min, dim3(1), dim3(64), 0, s, counts, n, out);
    return hipGetLastError();
}

template <int ITEMS, int W>
hipError_t launch_step_items(hipStream_t s, const FxGraphDev &g, const FxSeg *segs, const uint32_t *blk0s,
                             int32_t nsegs, uint32_t nblocks, FxTile *tmap, int32_t *cand, uint32_t *bcnt, uint64_t *boff,
                             uint64_t *lsum, uint64_t *loff, uint64_t *sstat, hipEvent_t probe_begin,
                             hipEvent_t probe_end,
                             hipEvent_t scatter_begin, hipEvent_t scatter_end, hipEvent_t greedy_begin,
                             hipEvent_t greedy_end, int32_t any_inner, int32_t any_greedy, int32_t fused)
{
    hipError_t e;
    if (fused) {  // single pass: boff / loff hold the tiles' status words, lsum the ticket counter
        uint32_t *ticket = reinterpret_cast<uint32_t *>(lsum);
        hipLaunchKernelGGL(k_tile_map<ITEMS>, dim3((nblocks + FX_BS - 1) / FX_BS), dim3(FX_BS), 0, s, segs, blk0s,
                           nsegs, nblocks, tmap, boff, loff, ticket, nullptr);
        if (probe_begin && (e = hipEventRecord(probe_begin, s)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_expand<ITEMS, W>), dim3(nblocks), dim3(FX_BS), 0, s, g, segs, tmap, boff, loff, ticket);
        if (probe_end && (e = hipEventRecord(probe_end, s)) != hipSuccess) return e;
        if (greedy_begin && (e = hipEventRecord(greedy_begin, s)) != hipSuccess) return e;
        if (any_greedy) hipLaunchKernelGGL(k_greedy<false>, dim3(nsegs), dim3(FX_BS), 0, s, segs, nullptr);
        if (greedy_end && (e = hipEventRecord(greedy_end, s)) != hipSuccess) return e;
        return hipGetLastError();
    }
    const uint32_t nch = scan_chunks(nblocks);
    const uint32_t nmap = max(nblocks, scan_state_words(nblocks));
    hipLaunchKernelGGL(k_tile_map<ITEMS>, dim3((nmap + FX_BS - 1) / FX_BS), dim3(FX_BS), 0, s, segs, blk0s, nsegs,
                       nblocks, tmap, nullptr, nullptr, nullptr, sstat);
    if (probe_begin && (e = hipEventRecord(probe_begin, s)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_probe<ITEMS, W>), dim3(nblocks), dim3(FX_BS), 0, s, g, segs, tmap, cand, bcnt);
    if (probe_end && (e = hipEventRecord(probe_end, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_blocks<uint32_t>, dim3(nch), dim3(FX_BS), 0, s, bcnt, nblocks, boff, sstat, 0u);
    if (scatter_begin && (e = hipEventRecord(scatter_begin, s)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_scatter<ITEMS, W>), dim3(nblocks), dim3(FX_BS), 0, s, g, segs, tmap, cand, boff, lsum);
    if (scatter_end && (e = hipEventRecord(scatter_end, s)) != hipSuccess) return e;
    if (any_inner) {
        hipLaunchKernelGGL(k_scan_blocks<uint64_t>, dim3(nch), dim3(FX_BS), 0, s, lsum, nblocks, loff, sstat, 1u);
        hipLaunchKernelGGL(k_fix_off<ITEMS>, dim3(nblocks), dim3(FX_BS), 0, s, segs, tmap, boff, loff);
    }
    if (greedy_begin && (e = hipEventRecord(greedy_begin, s)) != hipSuccess) return e;
    if (any_greedy) hipLaunchKernelGGL(k_greedy<false>, dim3(nsegs), dim3(FX_BS), 0, s, segs, nullptr);
    if (greedy_end && (e = hipEventRecord(greedy_end, s)) != hipSuccess) return e;
    return hipGetLastError();
}

template <int ITEMS, int W>
hipError_t launch_chain_items(hipStream_t s, const FxGraphDev &g, FxChainQuery *cq, FxChainCtl *ctl, int32_t max_q,
                              int32_t steps, FxSeg *segs, uint32_t *blk0s, FxTile *tmap, int32_t *cand, uint32_t *bcnt,
                              uint64_t *boff, uint64_t *lsum, uint64_t *loff, uint64_t *sstat, int32_t fused)
{
    constexpr uint32_t TILE = FX_BS * ITEMS;
    // enough workgroups to fill the chip at the expansion kernels' occupancy
    // (8 waves per SIMD, 4 waves per workgroup: 8 per CU on 256 CUs); each
    // loops over the tiles the scheduler announced
    constexpr uint32_t kGrid = 2048, kMapGrid = 64, kScanGrid = 128;
    if (fused) {
        uint32_t *ticket = reinterpret_cast<uint32_t *>(lsum);
        for (int32_t k = 0; k < steps; k++) {
            hipLaunchKernelGGL(k_sched, dim3(1), dim3(64), 0, s, cq, ctl, segs, blk0s, TILE, 0);
            hipLaunchKernelGGL(k_tile_map_chain<ITEMS>, dim3(kMapGrid), dim3(FX_BS), 0, s, segs, blk0s, ctl, tmap,
                               boff, loff, ticket, nullptr);
            hipLaunchKernelGGL((k_expand_chain<ITEMS, W>), dim3(kGrid), dim3(FX_BS), 0, s, g, segs, tmap, boff, loff,
                               ticket, ctl);
            hipLaunchKernelGGL(k_greedy<true>, dim3(max_q), dim3(FX_BS), 0, s, segs, ctl);
        }
        hipLaunchKernelGGL(k_sched, dim3(1), dim3(64), 0, s, cq, ctl, segs, blk0s, TILE, 1);
        return hipGetLastError();
    }
    for (int32_t k = 0; k < steps; k++) {
        hipLaunchKernelGGL(k_sched, dim3(1), dim3(64), 0, s, cq, ctl, segs, blk0s, TILE, 0);
        hipLaunchKernelGGL(k_tile_map_chain<ITEMS>, dim3(kMapGrid), dim3(FX_BS), 0, s, segs, blk0s, ctl, tmap, nullptr,
                           nullptr, nullptr, sstat);
        hipLaunchKernelGGL((k_probe_chain<ITEMS, W>), dim3(kGrid), dim3(FX_BS), 0, s, g, segs, tmap, cand, bcnt, ctl);
        hipLaunchKernelGGL(k_scan_blocks_chain<uint32_t>, dim3(kScanGrid), dim3(FX_BS), 0, s, bcnt, ctl, boff, sstat, 0u);
        hipLaunchKernelGGL((k_scatter_chain<ITEMS, W>), dim3(kGrid), dim3(FX_BS), 0, s, g, segs, tmap, cand, boff,
                           lsum, ctl);
        hipLaunchKernelGGL(k_scan_blocks_chain<uint64_t>, dim3(kScanGrid), dim3(FX_BS), 0, s, lsum, ctl, loff, sstat,
                           1u);
        hipLaunchKernelGGL(k_fix_off_chain<ITEMS>, dim3(kGrid), dim3(FX_BS), 0, s, segs, tmap, boff, loff, ctl);
        hipLaunchKernelGGL(k_greedy<true>, dim3(max_q), dim3(FX_BS), 0, s, segs, ctl);
    }
    hipLaunchKernelGGL(k_sched, dim3(1), dim3(64), 0, s, cq, ctl, segs, blk0s, TILE, 1);
    return hipGetLastError();
}

template <int W>
hipError_t launch_chain_width(hipStream_t s, const FxGraphDev &g, FxChainQuery *cq, FxChainCtl *ctl, int32_t max_q,
                              int32_t steps, FxSeg *segs, uint32_t *blk0s, int32_t items, FxTile *tmap, int32_t *cand,
                              uint32_t *bcnt, uint64_t *boff, uint64_t *lsum, uint64_t *loff, uint64_t *sstat,
                              int32_t fused)
{
    switch (items) {
    case 2:
        return launch_chain_items<2, W>(s, g, cq, ctl, max_q, steps, segs, blk0s, tmap, cand, bcnt, boff, lsum, loff,
                                        sstat, fused);
    case 8:
        return launch_chain_items<8, W>(s, g, cq, ctl, max_q, steps, segs, blk0s, tmap, cand, bcnt, boff, lsum, loff,
                                        sstat, fused);
    default:
        return launch_chain_items<4, W>(s, g, cq, ctl, max_q, steps, segs, blk0s, tmap, cand, bcnt, boff, lsum, loff,
                                        sstat, fused);
    }
}

template <int W>
hipError_t launch_step_width(hipStream_t s, const FxGraphDev &g, const FxSeg *segs, const uint32_t *blk0s,
                             int32_t nsegs, uint32_t nblocks, int32_t items, FxTile *tmap, int32_t *cand,
                             uint32_t *bcnt, uint64_t *boff, uint64_t *lsum, uint64_t *loff, uint64_t *sstat,
                             hipEvent_t probe_begin,
                             hipEvent_t probe_end, hipEvent_t scatter_begin, hipEvent_t scatter_end,
                             hipEvent_t greedy_begin, hipEvent_t greedy_end, int32_t any_inner, int32_t any_greedy,
                             int32_t fused)
{
    switch (items) {
    case 2:
        return launch_step_items<2, W>(s, g, segs, blk0s, nsegs, nblocks, tmap, cand, bcnt, boff, lsum, loff,
                                       sstat, probe_begin, probe_end, scatter_begin, scatter_end, greedy_begin, greedy_end,
                                       any_inner, any_greedy, fused);
    case 8:
        return launch_step_items<8, W>(s, g, segs, blk0s, nsegs, nblocks, tmap, cand, bcnt, boff, lsum, loff,
                                       sstat, probe_begin, probe_end, scatter_begin, scatter_end, greedy_begin, greedy_end,
                                       any_inner, any_greedy, fused);
    default:
        return launch_step_items<4, W>(s, g, segs, blk0s, nsegs, nblocks, tmap, cand, bcnt, boff, lsum, loff,
                                       sstat, probe_begin, probe_end, scatter_begin, scatter_end, greedy_begin, greedy_end,
                                       any_inner, any_greedy, fused);
    }
}

hipError_t fx_launch_step(hipStream_t s, const FxGraphDev &g, const FxSeg *segs, const uint32_t *blk0s,
                          int32_t nsegs, uint32_t nblocks, int32_t items, int32_t maxn, FxTile *tmap, int32_t *cand,
                          uint32_t *bcnt, uint64_t *boff, uint64_t *lsum, uint64_t *loff, uint64_t *sstat,
                          hipEvent_t probe_begin,
                          hipEvent_t probe_end, hipEvent_t scatter_begin, hipEvent_t scatter_end,
                          hipEvent_t greedy_begin, hipEvent_t greedy_end, int32_t any_inner, int32_t any_greedy,
                          int32_t fused)
{
    if (maxn < 1 || maxn > FX_MAXN) return hipErrorInvalidValue;
    if (maxn <= 4)
        return launch_step_width<4>(s, g, segs, blk0s, nsegs, nblocks, items, tmap, cand, bcnt, boff, lsum, loff,
                                    sstat, probe_begin, probe_end, scatter_begin, scatter_end, greedy_begin, greedy_end,
                                    any_inner, any_greedy, fused);
    if (maxn <= 8)
        return launch_step_width<8>(s, g, segs, blk0s, nsegs, nblocks, items, tmap, cand, bcnt, boff, lsum, loff,
                                    sstat, probe_begin, probe_end, scatter_begin, scatter_end, greedy_begin, greedy_end,
                                    any_inner, any_greedy, fused);
    return launch_step_width<FX_MAXN>(s, g, segs, blk0s, nsegs, nblocks, items, tmap, cand, bcnt, boff, lsum, loff,
                                      sstat, probe_begin, probe_end, scatter_begin, scatter_end, greedy_begin, greedy_end,
                                      any_inner, any_greedy, fused);
}

hipError_t fx_launch_chain(hipStream_t s, const FxGraphDev &g, FxChainQuery *cq, FxChainCtl *ctl, int32_t max_q,
                           int32_t steps, FxSeg *segs, uint32_t *blk0s, int32_t items, int32_t maxn, FxTile *tmap,
                           int32_t *cand, uint32_t *bcnt, uint64_t *boff, uint64_t *lsum, uint64_t *loff,
                           uint64_t *sstat, int32_t fused)
{
    if (maxn < 1 || maxn > FX_MAXN || max_q < 1 || steps < 1) return hipErrorInvalidValue;
    if (maxn <= 4)
        return launch_chain_width<4>(s, g, cq, ctl, max_q, steps, segs, blk0s, items, tmap, cand, bcnt, boff, lsum,
                                     loff, sstat, fused);
    if (maxn <= 8)
        return launch_chain_width<8>(s, g, cq, ctl, max_q, steps, segs, blk0s, items, tmap, cand, bcnt, boff, lsum,
                                     loff, sstat, fused);
    return launch_chain_width<FX_MAXN>(s, g, cq, ctl, max_q, steps, segs, blk0s, items, tmap, cand, bcnt, boff, lsum,
                                       loff, sstat, fused);
}

hipError_t fx_launch_mis(hipStream_t s, int32_t *rows, int32_t count, int32_t n, uint64_t *hash_scratch,
                         FxMisOut *out)
{
    if (n < 1 || n > FX_MAXN || count < 0 || count > FX_MIS_MAX_EMB) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mis, dim3(1), dim3(256), 0, s, rows, count, n, hash_scratch, out);
    return hipGetLastError();
}
