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

// First index in adj[lo, hi) whose value is >= key.
__device__ __forceinline__ int64_t lower_bound64(const uint64_t *__restrict__ a, int64_t lo, int64_t hi, uint64_t key)
{
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Does the row of u contain the packed entry (label, elabel, id)?
__device__ __forceinline__ bool has_entry(const FxGraphDev &g, int32_t u, uint64_t entry)
{
    int64_t lo = g.rowp[u], hi = g.rowp[u + 1];
    int64_t k = lower_bound64(g.adj, lo, hi, entry);
    return k < hi && g.adj[k] == entry;
}

// The run of neighbours of u with the given (label, elabel) key.
__device__ __forceinline__ void run_of(const FxGraphDev &g, int32_t u, uint64_t key, int64_t &lo, int32_t &len)
{
    int64_t a = g.rowp[u], b = g.rowp[u + 1];
    int64_t s = lower_bound64(g.adj, a, b, key);
    int64_t e = lower_bound64(g.adj, s, b, key + (1ULL << 32));
    lo = s;
    len = (int32_t)(e - s);
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

struct Cand {
    int32_t v[FX_MAXN];  // the partial row (first l entries)
    int32_t c;           // candidate for pattern vertex l
    int32_t anc;         // pattern vertex whose run produced c (-1: bucket)
};

// Loads the partial and the candidate behind flattened index t.
__device__ __forceinline__ void load_cand(const FxGraphDev &g, const FxLevelDev &in, int32_t l, int64_t nparts,
                                          uint64_t t, Cand &x)
{
    int64_t p = find_part(in.off, nparts, t);
    int64_t j = (int64_t)(t - (uint64_t)in.off[p]);
    const int32_t *row = in.rows + p * l;
#pragma unroll
    for (int k = 0; k < FX_MAXN; k++)
        x.v[k] = (k < l) ? row[k] : -1;
    x.anc = in.anc[p];
    int64_t base = in.lo[p];
    x.c = x.anc >= 0 ? (int32_t)(uint32_t)(g.adj[base + j] & 0xffffffffULL) : g.bucket[base + j];
}

__device__ __forceinline__ int32_t pick(const int32_t (&v)[FX_MAXN], int32_t b)
{
    int32_t r = -1;
#pragma unroll
    for (int k = 0; k < FX_MAXN; k++)
        r = (k == b) ? v[k] : r;
    return r;
}

// Candidate test of Section 2.1.4 for pattern vertex i = l.
__device__ __forceinline__ bool feasible(const FxGraphDev &g, const FxPlan *__restrict__ plan, int32_t n, int32_t l,
                                         const Cand &x)
{
#pragma unroll
    for (int k = 0; k < FX_MAXN; k++)
        if (k < l && x.v[k] == x.c) return false;  // injective
    const int32_t i = l;
    const uint32_t vl = plan->vl[i];
    const int32_t nb = plan->nback[i];
    for (int kk = 0; kk < nb; kk++) {
        int32_t b = plan->back[i][kk];
        if (b == x.anc) continue;  // the run it came from already matches
        uint64_t entry = run_key(vl, plan->bel[i][kk]) | (uint32_t)x.c;
        if (!has_entry(g, pick(x.v, b), entry)) return false;
    }
    if (i < n - 1) {  // neighbour-label filter for the later neighbours of i
        const int32_t nf = plan->nnlf[i];
        for (int k = 0; k < nf; k++) {
            int64_t lo;
            int32_t len;
            run_of(g, x.c, plan->nlf_key[i][k], lo, len);
            if (len < plan->nlf_need[i][k]) return false;
        }
    }
    return true;
}

__device__ __forceinline__ bool touches_used(const uint32_t *__restrict__ U, const Cand &x, int32_t l)
{
    if (is_used(U, x.c)) return true;
#pragma unroll
    for (int k = 0; k < FX_MAXN; k++)
        if (k < l && is_used(U, x.v[k])) return true;
    return false;
}

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const uint32_t lane = __lane_id();
    return lane == 0 ? 0ULL : ((~0ULL) >> (64 - lane));
}

// ---------------------------------------------------------------------------
// Expansion: probe (test + per-block counts) and scatter (ordered write).
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(FX_BS) void k_probe(FxGraphDev g, const FxPlan *__restrict__ plan, int32_t n, int32_t l,
                                                 FxLevelDev in, int64_t nparts, uint64_t t0, uint32_t span,
                                                 int32_t flags, const uint32_t *__restrict__ U, uint8_t *flag,
                                                 uint32_t *bcnt, FxSummary *sum)
{
    __shared__ uint32_t wcnt[FX_BS / 64];
    const uint32_t tl = blockIdx.x * FX_BS + threadIdx.x;
    bool mat = false, cnt = false;
    uint64_t h1 = 0, h2 = 0;
    if (tl < span) {
        Cand x;
        load_cand(g, in, l, nparts, t0 + tl, x);
        const bool ufilter = (flags & FX_PROBE_UFILTER) != 0;
        const bool count = (flags & FX_PROBE_COUNT) != 0;
        bool ok = true;
        bool used = false;
        if (ufilter) used = touches_used(U, x, l);
        if (ufilter && !count && used) ok = false;  // nothing to count: prune early
        if (ok) ok = feasible(g, plan, n, l, x);
        if (ok) {
            mat = !(ufilter && used);
            if (count) {
                cnt = true;
                uint64_t a = kSeed1, b = kSeed2;
#pragma unroll
                for (int k = 0; k < FX_MAXN; k++) {
                    if (k < l) {
                        a = mix64(a ^ (uint64_t)(uint32_t)x.v[k]);
                        b = mix64(b ^ (uint64_t)(uint32_t)x.v[k]);
                    }
                }
                h1 = mix64(a ^ (uint64_t)(uint32_t)x.c);
                h2 = mix64(b ^ (uint64_t)(uint32_t)x.c);
            }
        }
        flag[tl] = mat ? 1 : 0;
    }
    const uint64_t bal = __ballot(mat);
    const uint32_t wave = threadIdx.x >> 6;
    if (__lane_id() == 0) wcnt[wave] = (uint32_t)__popcll(bal);
    if (flags & FX_PROBE_COUNT) {
        unsigned long long c = cnt ? 1ULL : 0ULL;
        unsigned long long s1 = h1, s2 = h2;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            c += __shfl_xor(c, o);
            s1 += __shfl_xor(s1, o);
            s2 ^= __shfl_xor(s2, o);
        }
        if (__lane_id() == 0 && c) {
            atomicAdd(&sum->count, c);
            atomicAdd(&sum->digest0, s1);
            atomicXor(&sum->digest1, s2);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
#pragma unroll
        for (int w = 0; w < FX_BS / 64; w++) s += wcnt[w];
        bcnt[blockIdx.x] = s;
    }
}

// Exclusive scan of the per-block counts (one workgroup of 1024 threads).
__global__ __launch_bounds__(1024) void k_scan_blocks(const uint32_t *__restrict__ bcnt, uint32_t nblocks,
                                                      uint64_t *boff, FxSummary *sum)
{
    __shared__ uint64_t part[1024];
    const uint32_t per = (nblocks + 1023) / 1024;
    const uint32_t beg = threadIdx.x * per;
    uint64_t s = 0;
    for (uint32_t k = 0; k < per; k++)
        if (beg + k < nblocks) s += bcnt[beg + k];
    part[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t o = 1; o < 1024; o <<= 1) {  // Hillis-Steele inclusive scan
        uint64_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint64_t run = threadIdx.x ? part[threadIdx.x - 1] : 0;
    for (uint32_t k = 0; k < per; k++)
        if (beg + k < nblocks) {
            boff[beg + k] = run;
            run += bcnt[beg + k];
        }
    if (threadIdx.x == 1023) sum->total_out = part[1023];
}

__global__ __launch_bounds__(FX_BS) void k_scatter(FxGraphDev g, const FxPlan *__restrict__ plan, int32_t n, int32_t l,
                                                   FxLevelDev in, int64_t nparts, uint64_t t0, uint32_t span,
                                                   const uint8_t *__restrict__ flag, const uint64_t *__restrict__ boff,
                                                   FxLevelDev out)
{
    __shared__ uint32_t wcnt[FX_BS / 64];
    const uint32_t tl = blockIdx.x * FX_BS + threadIdx.x;
    const bool f = tl < span && flag[tl];
    const uint64_t bal = __ballot(f);
    const uint32_t wave = threadIdx.x >> 6;
    if (__lane_id() == 0) wcnt[wave] = (uint32_t)__popcll(bal);
    __syncthreads();
    if (!f) return;
    uint64_t pos = boff[blockIdx.x] + (uint64_t)__popcll(bal & lanemask_lt());
    for (uint32_t w = 0; w < wave; w++) pos += wcnt[w];

    Cand x;
    load_cand(g, in, l, nparts, t0 + tl, x);
    const int32_t w1 = l + 1;
    int32_t *dst = out.rows + pos * w1;
#pragma unroll
    for (int k = 0; k < FX_MAXN; k++)
        if (k < l) dst[k] = x.v[k];
    dst[l] = x.c;
    if (w1 < n) {
        // candidate run of the next pattern vertex i2 = l + 1: the shortest
        // run among its earlier neighbours, or its label bucket.
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
                int32_t b = plan->back[i2][kk];
                int32_t u = (b == l) ? x.c : pick(x.v, b);
                int64_t lo;
                int32_t len;
                run_of(g, u, run_key(vl, plan->bel[i2][kk]), lo, len);
                if (len < best_len) {
                    best_len = len;
                    best_lo = lo;
                    best_anc = b;
                }
            }
        }
        out.lo[pos] = best_lo;
        out.len[pos] = best_len;
        out.anc[pos] = (int8_t)best_anc;
    }
}

// ---------------------------------------------------------------------------
// Exclusive scan of the run lengths of a new level (three passes).
// ---------------------------------------------------------------------------

constexpr uint32_t kScanTile = FX_BS * FX_SCAN_ITEMS;

__global__ __launch_bounds__(FX_BS) void k_scan_len_a(FxLevelDev lev, const FxSummary *sum, int64_t *bsum)
{
    __shared__ int64_t red[FX_BS];
    const uint64_t N = sum->total_out;
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    if (base >= N) return;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < FX_SCAN_ITEMS; k++) {
        uint64_t i = base + threadIdx.x * FX_SCAN_ITEMS + k;
        if (i < N) s += lev.len[i];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t o = FX_BS / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(1024) void k_scan_len_b(int64_t *bsum, FxSummary *sum)
{
    __shared__ int64_t part[1024];
    const uint64_t N = sum->total_out;
    const uint64_t nb = (N + kScanTile - 1) / kScanTile;
    const uint64_t per = (nb + 1023) / 1024;
    const uint64_t beg = threadIdx.x * per;
    int64_t s = 0;
    for (uint64_t k = 0; k < per; k++)
        if (beg + k < nb) s += bsum[beg + k];
    part[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t o = 1; o < 1024; o <<= 1) {
        int64_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t run = threadIdx.x ? part[threadIdx.x - 1] : 0;
    for (uint64_t k = 0; k < per; k++)
        if (beg + k < nb) {
            int64_t v = bsum[beg + k];
            bsum[beg + k] = run;
            run += v;
        }
    if (threadIdx.x == 1023) sum->t_next = (unsigned long long)part[1023];
}

__global__ __launch_bounds__(FX_BS) void k_scan_len_c(FxLevelDev lev, const FxSummary *sum, const int64_t *bsum)
{
    __shared__ int64_t part[FX_BS];
    const uint64_t N = sum->total_out;
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    if (blockIdx.x == 0 && threadIdx.x == 0) lev.off[N] = (int64_t)sum->t_next;
    if (base >= N) return;
    int64_t v[FX_SCAN_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < FX_SCAN_ITEMS; k++) {
        uint64_t i = base + threadIdx.x * FX_SCAN_ITEMS + k;
        v[k] = i < N ? lev.len[i] : 0;
        s += v[k];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t o = 1; o < FX_BS; o <<= 1) {
        int64_t t = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += t;
        __syncthreads();
    }
    int64_t run = bsum[blockIdx.x] + (threadIdx.x ? part[threadIdx.x - 1] : 0);
#pragma unroll
    for (int k = 0; k < FX_SCAN_ITEMS; k++) {
        uint64_t i = base + threadIdx.x * FX_SCAN_ITEMS + k;
        if (i < N) lev.off[i] = run;
        run += v[k];
    }
}

// ---------------------------------------------------------------------------
// Greedy maximal independent set over one slice of complete embeddings.
// Slot value: min over contending embeddings of ((~round) << 32 | rank); a
// later round's keys are smaller than every stale key, so slots need no reset
// between rounds.  Value 0 marks a slot taken by a selected embedding.
// ---------------------------------------------------------------------------

// Fibonacci hashing: the top log2(size) bits of v * 2^64/phi.
__device__ __forceinline__ uint64_t hash_slot(int32_t v, uint64_t mask)
{
    const uint32_t bits = (uint32_t)__popcll(mask);
    return ((uint64_t)(uint32_t)v * 0x9e3779b97f4a7c15ULL) >> (64 - bits);
}

__global__ __launch_bounds__(FX_BS) void k_greedy_init(const int32_t *__restrict__ rows, int32_t n, uint64_t nrows,
                                                       int32_t *hkey, uint64_t hmask, int32_t *slot,
                                                       uint8_t *state)
{
    const uint64_t e = (uint64_t)blockIdx.x * FX_BS + threadIdx.x;
    if (e >= nrows) return;
    for (int j = 0; j < n; j++) {
        const int32_t v = rows[e * n + j];
        uint64_t h = hash_slot(v, hmask);
        while (true) {  // linear probing; the table has >= 2x as many slots as keys
            int32_t prev = atomicCAS(&hkey[h], -1, v);
            if (prev == -1 || prev == v) break;
            h = (h + 1) & hmask;
        }
        slot[e * n + j] = (int32_t)h;
    }
    state[e] = 0;
}

__global__ __launch_bounds__(FX_BS) void k_greedy_min(int32_t n, uint64_t nrows, unsigned long long *hval,
                                                      const int32_t *__restrict__ slot, uint8_t *state,
                                                      const uint32_t *rem, uint32_t round)
{
    if ((round % FX_RMAX) != 0 && rem[(round - 1) % FX_RMAX] == 0) return;
    const uint64_t e = (uint64_t)blockIdx.x * FX_BS + threadIdx.x;
    if (e >= nrows || state[e] != 0) return;
    for (int j = 0; j < n; j++)
        if (hval[slot[e * n + j]] == 0ULL) {  // meets a selected embedding
            state[e] = 2;
            return;
        }
    const unsigned long long key = ((unsigned long long)(0xffffffffu - round) << 32) | (uint32_t)e;
    for (int j = 0; j < n; j++) atomicMin(&hval[slot[e * n + j]], key);
}

__global__ __launch_bounds__(FX_BS) void k_greedy_sel(const int32_t *__restrict__ rows, int32_t n, uint64_t nrows,
                                                      unsigned long long *hval, const int32_t *__restrict__ slot,
                                                      uint8_t *state, uint32_t *rem, uint32_t round, uint32_t *U,
                                                      int32_t *sel_rows, int64_t *sel_rank, int64_t rank_base,
                                                      FxSummary *sum)
{
    if ((round % FX_RMAX) != 0 && rem[(round - 1) % FX_RMAX] == 0) return;
    const uint64_t e = (uint64_t)blockIdx.x * FX_BS + threadIdx.x;
    bool still = false;
    if (e < nrows && state[e] == 0) {
        const unsigned long long key = ((unsigned long long)(0xffffffffu - round) << 32) | (uint32_t)e;
        bool mine = true;
        for (int j = 0; j < n; j++) mine = mine && (hval[slot[e * n + j]] == key);
        if (mine) {
            state[e] = 1;
            for (int j = 0; j < n; j++) {
                hval[slot[e * n + j]] = 0ULL;
                const uint32_t v = (uint32_t)rows[e * n + j];
                atomicOr(&U[v >> 5], 1u << (v & 31u));
            }
            const unsigned long long pos = atomicAdd(&sum->support, 1ULL);
            for (int j = 0; j < n; j++) sel_rows[pos * n + j] = rows[e * n + j];
            sel_rank[pos] = rank_base + (int64_t)e;
        } else {
            still = true;
        }
    }
    const uint64_t bal = __ballot(still);
    if (__lane_id() == 0 && bal) atomicAdd(&rem[round % FX_RMAX], (uint32_t)__popcll(bal));
}

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_level0(FxGraphDev g, const FxPlan *__restrict__ plan, FxLevelDev lev)
{
    if (threadIdx.x != 0) return;
    const uint32_t vl = plan->vl[0];
    lev.lo[0] = g.bptr[vl];
    lev.len[0] = (int32_t)(g.bptr[vl + 1] - g.bptr[vl]);
    lev.anc[0] = -1;
    lev.off[0] = 0;
    lev.off[1] = g.bptr[vl + 1] - g.bptr[vl];
}

inline uint32_t blocks_for(uint64_t n, uint32_t bs) { return (uint32_t)((n + bs - 1) / bs); }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t fx_launch_probe(hipStream_t s, const FxGraphDev &g, const FxPlan *plan, int32_t n, int32_t l,
                           const FxLevelDev &in, int64_t nparts, uint64_t t0, uint64_t t1, int32_t flags,
                           const uint32_t *U, uint8_t *flag, uint32_t *bcnt, FxSummary *sum)
{
    const uint32_t span = (uint32_t)(t1 - t0);
    hipLaunchKernelGGL(k_probe, dim3(blocks_for(span, FX_BS)), dim3(FX_BS), 0, s, g, plan, n, l, in, nparts, t0, span,
                       flags, U, flag, bcnt, sum);
    return hipGetLastError();
}

hipError_t fx_launch_scan_blocks(hipStream_t s, const uint32_t *bcnt, uint32_t nblocks, uint64_t *boff,
                                 FxSummary *sum)
{
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, bcnt, nblocks, boff, sum);
    return hipGetLastError();
}

hipError_t fx_launch_scatter(hipStream_t s, const FxGraphDev &g, const FxPlan *plan, int32_t n, int32_t l,
                             const FxLevelDev &in, int64_t nparts, uint64_t t0, uint64_t t1,
                             const uint8_t *flag, const uint64_t *boff, const FxLevelDev &out)
{
    const uint32_t span = (uint32_t)(t1 - t0);
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(span, FX_BS)), dim3(FX_BS), 0, s, g, plan, n, l, in, nparts, t0,
                       span, flag, boff, out);
    return hipGetLastError();
}

hipError_t fx_launch_scan_len(hipStream_t s, const FxLevelDev &lev, uint64_t max_rows, int64_t *bsum,
                              FxSummary *sum)
{
    const uint32_t nb = blocks_for(max_rows > 0 ? max_rows : 1, kScanTile);
    hipLaunchKernelGGL(k_scan_len_a, dim3(nb), dim3(FX_BS), 0, s, lev, sum, bsum);
    hipLaunchKernelGGL(k_scan_len_b, dim3(1), dim3(1024), 0, s, bsum, sum);
    hipLaunchKernelGGL(k_scan_len_c, dim3(nb), dim3(FX_BS), 0, s, lev, sum, bsum);
    return hipGetLastError();
}

hipError_t fx_launch_greedy_init(hipStream_t s, const int32_t *rows, int32_t n, uint64_t nrows, int32_t *hkey,
                                 unsigned long long *hval, uint64_t hsize, int32_t *slot, uint8_t *state,
                                 uint32_t *rem, FxSummary *sum)
{
    (void)sum;
    hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, s, (uint32_t *)hkey, hsize, 0xffffffffu);
    hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, s, (uint32_t *)hval, 2 * hsize, 0xffffffffu);
    hipLaunchKernelGGL(k_fill_u32, dim3(16), dim3(256), 0, s, rem, (uint64_t)FX_RMAX, 0u);
    hipLaunchKernelGGL(k_greedy_init, dim3(blocks_for(nrows, FX_BS)), dim3(FX_BS), 0, s, rows, n, nrows, hkey,
                       hsize - 1, slot, state);
    return hipGetLastError();
}

hipError_t fx_launch_greedy_round(hipStream_t s, const int32_t *rows, int32_t n, uint64_t nrows,
                                  unsigned long long *hval, const int32_t *slot, uint8_t *state, uint32_t *rem,
                                  uint32_t round, uint32_t *U, int32_t *sel_rows, int64_t *sel_rank,
                                  int64_t rank_base, FxSummary *sum)
{
    const uint32_t nb = blocks_for(nrows, FX_BS);
    if (round != 0 && (round % FX_RMAX) == 0)
        hipLaunchKernelGGL(k_fill_u32, dim3(16), dim3(256), 0, s, rem, (uint64_t)FX_RMAX, 0u);
    hipLaunchKernelGGL(k_greedy_min, dim3(nb), dim3(FX_BS), 0, s, n, nrows, hval, slot, state, rem, round);
    hipLaunchKernelGGL(k_greedy_sel, dim3(nb), dim3(FX_BS), 0, s, rows, n, nrows, hval, slot, state, rem, round, U,
                       sel_rows, sel_rank, rank_base, sum);
    return hipGetLastError();
}

hipError_t fx_launch_fill_u32(hipStream_t s, uint32_t *p, uint64_t n, uint32_t v)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t fx_launch_level0(hipStream_t s, const FxGraphDev &g, const FxPlan *plan, FxLevelDev lev0)
{
    hipLaunchKernelGGL(k_level0, dim3(1), dim3(64), 0, s, g, plan, lev0);
    return hipGetLastError();
}
