// Internal declarations shared by the host runtime and the gfx950 kernels.
//
// Device layout of a data graph (built once by fx_graph_load):
//   rowp   int64 [nv+1]        CSR offsets
//   adj    uint64 [2|E|]       packed adjacency entry
//                                bits 63..48  dense vertex label of the neighbour
//                                bits 47..32  dense edge label
//                                bits 31..0   neighbour id
//                              each row sorted ascending by the packed value, so
//                              the neighbours with a given (vertex label, edge
//                              label) form one contiguous run in ascending id.
//   bucket int32 [nv]          vertex ids grouped by dense label, ascending id
//   bptr   int64 [L+1]         start of each label group in bucket
//   runoff uint32 [nv*K + 1]   label-run index, K = (vertex labels) x (edge labels):
//                              runoff[v*K + k] = position in adj of the first
//                              neighbour of v with key >= k (k = label * nel +
//                              elabel), so the run of (v, k) is
//                              [runoff[v*K + k], runoff[v*K + k + 1]) and
//                              runoff[nv*K] = 2|E|.  Built when it fits the
//                              index budget and 2|E| < 2^32; otherwise runs are
//                              found by binary search.
//   keybits uint32 [K * VW]    with the run index: key-major vertex bitmaps,
//                              VW = ceil(nv/32); bit v of key k's bitmap is set
//                              when v has a neighbour with key k (the
//                              neighbour-label filter's common question, "at
//                              least one").  The workgroups of a segment test
//                              one key, so its |V|/8-byte bitmap stays in L2.
//
// A pattern plan fixes, for every pattern vertex i (in submitted order), its
// dense label, its earlier neighbours b < i with the edge label of (b, i),
// and a neighbour-label filter for its later neighbours.
//
// Every expansion step runs over a list of segments: one per active query,
// each a contiguous range of the flattened candidate space of one level of
// that query's slice stack.  Workgroups never straddle two segments.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define FX_MAXN 16
#define FX_NLF 4
#define FX_BS 256            // threads per workgroup for the streaming kernels
#define FX_MAX_TILE (FX_BS * 8)  // most candidates per expansion workgroup (8 per thread)
#define FX_LDSP 1024         // partial offsets a workgroup stages in LDS

// The probe's output per expansion workgroup (tile of FX_BS * items
// candidates): the passing candidates' vertex ids, compacted within each
// (item, wave) region of 64 candidate slots in candidate order; for each, its
// partial relative to the tile's first with the candidate's lane in the top 6
// bits; and the passing count of every region (at most 32 regions).
__host__ __device__ constexpr size_t cand_tile_bytes(int items) { return (size_t)FX_BS * items * 8 + 32; }

// Block scans of a step: chunks of kScanChunk per-workgroup values, each
// chunk's prefix found by look-back; a step's scan state is two scans' status
// words and tickets.
constexpr uint32_t kScanChunk = 1024;
__host__ __device__ inline uint32_t scan_chunks(uint32_t n) { return n ? (n + kScanChunk - 1) / kScanChunk : 1; }
__host__ __device__ inline uint32_t scan_state_words(uint32_t n) { return 2 * (scan_chunks(n) + 1); }
#define FX_GREEDY_H 4096     // LDS hash slots of the per-query greedy
#define FX_GREEDY_VN 2048    // embedding-vertices per greedy chunk (<= H / 2)
#define FX_FILL 0.8          // a slice aims at this fraction of the rows it may write
#define FX_COUNT_SPAN (1ull << 22)  // least last-vertex candidates of a counting slice

// Dense labels fit 16 bits (more than 65535 distinct labels is FX_ELIMIT).
struct FxPlan {
    int32_t n;
    uint16_t vl[FX_MAXN];                 // dense vertex label of pattern vertex i
    int8_t nback[FX_MAXN];                // number of earlier neighbours of i
    int8_t nnlf[FX_MAXN];                 // neighbour-label filter entries for i
    int8_t back[FX_MAXN][FX_MAXN];        // earlier neighbours of i (one entry per edge: a
                                          // reciprocal pair of a directed pattern gives two)
    uint16_t bel[FX_MAXN][FX_MAXN];       // edge code of that edge in the row of back[i][k]
    uint32_t nlf_key[FX_MAXN][FX_NLF];    // (label << 16 | elabel) of later neighbours
    uint8_t nlf_need[FX_MAXN][FX_NLF];    // how many such neighbours i needs
    uint16_t sym_lt[FX_MAXN];             // bit j: f(j) < f(i) (support phase only)
};
static_assert(sizeof(FxPlan) % 4 == 0, "the plan is copied in 32-bit words");

struct FxGraphDev {
    int64_t nv;
    int64_t nadj;
    const int64_t *rowp;
    const uint64_t *adj;
    const int32_t *bucket;
    const int64_t *bptr;
    int32_t nvl;   // dense vertex labels
    int32_t nel;   // dense edge labels
    const uint32_t *runoff;  // label-run index or nullptr
    int32_t nkeys;           // nvl * nel
    int32_t vwords;          // 32-bit words of one key's vertex bitmap in keybits
    const uint32_t *keybits; // key-presence bits or nullptr (with the run index)
};

// Device-side counters of one query, read by the host once per step.
struct FxSummary {
    unsigned long long total_out;   // rows materialised by the query's last segment
    unsigned long long t_next;      // candidate-space size of the new level
    unsigned long long count;       // embeddings counted so far
    unsigned long long digest0;     // sum of hashes (mod 2^64)
    unsigned long long digest1;     // xor of hashes
    unsigned long long support;     // embeddings selected so far
    unsigned long long rounds;      // greedy rounds run so far
    unsigned long long alg_probe;   // algorithmic bytes of the probe launches
    unsigned long long alg_scatter; // algorithmic bytes of the scatter launches
    unsigned long long error;       // nonzero: a device-side consistency check failed
    unsigned long long passes;      // candidates of the last segment that passed (before the row cap)
    unsigned long long consumed;    // candidates of the last segment taken (the rest are offered again)
    unsigned long long ufiltered;   // candidates the used set U has removed so far
    unsigned long long sel_d0;      // sum of the hashes of the selected embeddings (mod 2^64)
    unsigned long long sel_d1;      // xor of their second hashes
    // reference algorithmic bytes (counted only with FX_PROBE_REF): the bytes
    // the matching must move by a per-unit model (see k_probe, k_scatter,
    // k_greedy); ref_probe_row is the same model reading whole adjacency rows
    unsigned long long ref_probe;
    unsigned long long ref_scatter;
    unsigned long long ref_greedy;
    unsigned long long ref_probe_row;
};

// One level of a slice stack: partial embeddings with l matched vertices
// and, for each, the candidate run of pattern vertex l.
struct FxLevelDev {
    int32_t *rows;   // [cap * l]
    int64_t *lo;     // start of the candidate run (index into adj, or into bucket if anc < 0)
    int32_t *len;    // length of the run
    int8_t *anc;     // the back edge (index into the plan's back[l]) whose run is used, -1: a label bucket
    int64_t *off;    // exclusive prefix of len, [cap + 1]
};

// What a segment does with the candidates that pass.
enum : int32_t {
    FX_SEG_INNER = 0,    // write them to level l+1 (with their next candidate run)
    FX_SEG_GREEDY = 1,   // last vertex: write the complete embeddings, then run the greedy
    FX_SEG_COUNT = 2,    // count (and hash) the complete embeddings they give; nothing is written
    FX_SEG_LIST = 3,     // last vertex: write the complete embeddings (listing)
};

// Probe flags
enum : int32_t {
    FX_PROBE_UFILTER = 1,   // pass only candidates whose partial and vertex avoid the used set U
    FX_PROBE_COUNT = 2,     // count (and hash) every valid candidate of the last vertex
    FX_PROBE_LEAF = 4,      // candidates of vertex n-2: add the closed-form count of the last
                            // vertex, a leaf with a single earlier neighbour (no hashing)
    FX_PROBE_HASH = 8,      // with FX_PROBE_COUNT: also hash every counted embedding
    FX_PROBE_IMAGES = 16,   // with FX_PROBE_COUNT: mark every counted embedding's images
    FX_PROBE_SYM = 32,      // apply the plan's symmetry-breaking constraints (support phase)
    FX_PROBE_REF = 64,      // also count the reference algorithmic bytes (a counting pass: extra loads)
};

struct FxSeg {
    FxLevelDev in;          // level l of the query
    FxLevelDev out;         // level l+1 of the query
    const FxPlan *plan;
    uint32_t *U;            // used-vertex bitmap of the query
    FxSummary *sum;
    int32_t *sel_rows;      // selected embeddings (append)
    int64_t *sel_rank;      // their ranks
    uint32_t *img;          // image bitmaps of the pattern vertices (minimum-image support)
    uint64_t img_words;     // words per image bitmap
    int64_t nparts;         // rows in level l
    uint64_t t0;            // first flattened candidate of the slice
    int64_t rank_base;      // rank of the first complete embedding this step writes
    uint32_t span;          // candidates in the slice
    uint32_t out_cap;       // rows of level l+1 this segment may write; the candidates after the
                            // out_cap-th passing one are left for a later step
    uint32_t blk0;          // first workgroup of this segment in the launch (FX_BS * items candidates each)
    int32_t n, l;
    int32_t flags;          // FX_PROBE_*
    int32_t kind;           // FX_SEG_*
};

// Where an expansion workgroup's tile lies: its segment and the partials its
// candidates belong to, [p0, p0 + np).  Found once per step by k_tile_map.
struct FxTile {
    int32_t seg;
    int32_t np;
    int64_t p0;
};

// Per-query initialisation at admission: plan upload, U and counters cleared,
// level 0 set up.
struct FxInit {
    FxPlan plan;            // copied to plan_dst
    FxPlan *plan_dst;
    FxLevelDev lev0;
    uint32_t *U;            // cleared when clear_u != 0
    FxSummary *sum;         // cleared when clear_sum != 0
    uint64_t u_words;
    int32_t clear_u, clear_sum;
};

// ---------------------------------------------------------------------------
// Device-scheduled steps.  When few queries are left, the engine hands them
// to a chain of steps that runs without the host: each step starts with a
// one-workgroup scheduler kernel that advances every query from its last
// step's counters (as the host would), decides which queries are finished,
// and writes the next segment table; the expansion and greedy kernels then
// run over a fixed grid and loop over the tiles the scheduler announced.  A
// chain of K steps is captured once in a HIP graph and replayed; the host
// reads the queries' state back once per chain instead of once per step.
// ---------------------------------------------------------------------------

enum : int32_t { FX_CQ_SUPPORT = 0, FX_CQ_COUNT = 1 };  // phase of a chained query

struct FxChainQuery {
    // fixed while the query runs
    FxLevelDev lev[FX_MAXN + 1];
    const FxPlan *plan;
    uint32_t *U;
    FxSummary *sum;
    int32_t *sel_rows;
    int64_t *sel_rank;
    uint32_t *img;
    uint64_t img_words;
    int64_t cap;            // rows per level of its stack
    int64_t tau_eff;
    int64_t upper_bound;    // disjointness bound on the support
    int64_t count_cap;
    uint64_t bucket0;       // candidates of level 0 (the label bucket of vertex 0)
    uint32_t last_span;     // complete embeddings per greedy slice
    int32_t n;
    int32_t verdict;        // VERDICT mode: ends at tau or at the exactness bound
    int32_t mni;            // minimum-image mode: no support phase, no count cap
    int32_t full;           // FULL mode: the count phase follows the support phase
    int32_t sym;            // symmetry-breaking constraints in the support phase
    int32_t leaf_count;     // count phase: the leaf last vertex is counted in closed form
    int32_t hash;           // count phase: hash every embedding
    int32_t ref_bytes;      // count the reference algorithmic bytes
    // advanced by the scheduler
    int32_t phase;          // FX_CQ_*
    int32_t deep;           // deepest level with candidates left, -1: none
    int32_t done;           // finished (the host retires it)
    int32_t exit;           // fx_result.exit
    int32_t steps;
    int32_t error;          // nonzero: a consistency check failed
    uint64_t T[FX_MAXN + 1], cur[FX_MAXN + 1];
    int64_t nparts[FX_MAXN + 1];
    double rate[FX_MAXN + 1];
    int64_t rank_base;
    uint64_t probed_support, probed, reoffered;
    uint64_t alg_probe_seen, ref_probe_seen, ref_row_seen;
    double alg_probe_credit, ref_probe_credit, ref_row_credit;
    // the segment in flight
    int32_t seg_l, seg_kind;
    uint64_t seg_t0;
    uint32_t seg_span;
    uint32_t pad0;
    FxSummary last;         // the counters as of the last advance
};

struct FxChainCtl {
    int32_t nq;             // chained queries
    uint32_t nsegs;         // segments of the step in flight
    uint32_t nblocks;       // expansion workgroups (tiles) of the step in flight
    uint32_t rot;           // rotates which query the step budget serves first
    uint32_t steps;         // steps that had at least one segment
    uint32_t error;
    uint64_t budget;        // candidates per step, all queries together
};

// Exact maximum independent set of a pattern's embeddings (Section 2.4.2),
// for small instances: at most FX_MIS_MAX_EMB embeddings, at most
// FX_MIS_MAX_SETS distinct vertex sets, at most FX_MIS_MAX_NODES search nodes.
#define FX_MIS_MAX_EMB 4096
#define FX_MIS_MAX_SETS 256
#define FX_MIS_MAX_NODES (1u << 24)

struct FxMisOut {
    int64_t mis;        // size of a maximum independent set
    int32_t sets;       // distinct vertex sets
    int32_t status;     // 0 ok, 1 too many distinct sets, 2 the search budget ran out
    uint64_t nodes;     // branch-and-bound nodes visited
};

// Launchers (fx_kernels.hip).  All return the hipError_t of the launches.
// The exact maximum independent set of `count` embeddings of n vertices
// (rows, device, sorted in place), into *out.
hipError_t fx_launch_mis(hipStream_t s, int32_t *rows, int32_t count, int32_t n, uint64_t *hash_scratch,
                         FxMisOut *out);
hipError_t fx_launch_init(hipStream_t s, const FxGraphDev &g, const FxInit *inits, int32_t ninit);
// Minimum-image support from n image bitmaps of `words` words each: counts[j]
// = set bits of bitmap j, then *out = min_j counts[j].
hipError_t fx_launch_mni(hipStream_t s, const uint32_t *img, uint64_t words, int32_t n,
                         unsigned long long *counts, unsigned long long *out);
// One step: probe, scan, scatter (+ run-length prefix fix-up), greedy -- or,
// with fused, the single-pass expansion kernel (boff and loff then hold the
// tiles' status words, lsum the ticket counter) and the greedy.  sstat holds
// the block scans' state, scan_state_words(nblocks) words.  items
// (2, 4 or 8) is the number of candidates per thread; segment j owns
// ceil(span_j / (FX_BS * items)) consecutive workgroups starting at blk0s[j].
// maxn is the largest pattern size among the segments (it picks the register
// width of a partial row).
hipError_t fx_launch_step(hipStream_t s, const FxGraphDev &g, const FxSeg *segs, const uint32_t *blk0s,
                          int32_t nsegs, uint32_t nblocks, int32_t items, int32_t maxn, FxTile *tmap, int32_t *cand,
                          uint32_t *bcnt, uint64_t *boff, uint64_t *lsum, uint64_t *loff, uint64_t *sstat,
                          hipEvent_t probe_begin,
                          hipEvent_t probe_end, hipEvent_t scatter_begin, hipEvent_t scatter_end,
                          hipEvent_t greedy_begin, hipEvent_t greedy_end, int32_t any_inner, int32_t any_greedy,
                          int32_t fused);
// Enqueues `steps` device-scheduled steps over the chained queries in cq
// (ctl->nq of them, at most max_q), then a final advance, on stream s.  The
// scratch buffers must hold ceil(ctl->budget / (FX_BS * items)) + max_q
// tiles; segs and blk0s room for max_q segments.
hipError_t fx_launch_chain(hipStream_t s, const FxGraphDev &g, FxChainQuery *cq, FxChainCtl *ctl, int32_t max_q,
                           int32_t steps, FxSeg *segs, uint32_t *blk0s, int32_t items, int32_t maxn, FxTile *tmap,
                           int32_t *cand, uint32_t *bcnt, uint64_t *boff, uint64_t *lsum, uint64_t *loff,
                           uint64_t *sstat, int32_t fused);
