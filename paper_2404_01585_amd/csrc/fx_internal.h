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
//
// A pattern plan fixes, for every pattern vertex i (in submitted order), its
// dense label, its earlier neighbours b < i with the edge label of (b, i),
// and a neighbour-label filter for its later neighbours.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define FX_MAXN 16
#define FX_NLF 4
#define FX_BS 256           // threads per workgroup for the streaming kernels
#define FX_SCAN_ITEMS 4     // items per thread in the span scan
#define FX_RMAX 4096        // greedy rounds tracked per clear of the round counters

struct FxPlan {
    int32_t n;
    uint32_t vl[FX_MAXN];                 // dense vertex label of pattern vertex i
    int32_t nback[FX_MAXN];               // number of earlier neighbours of i
    int32_t back[FX_MAXN][FX_MAXN];       // earlier neighbours of i
    uint32_t bel[FX_MAXN][FX_MAXN];       // dense edge label of (back[i][k], i)
    int32_t nnlf[FX_MAXN];                // neighbour-label filter entries for i
    uint64_t nlf_key[FX_MAXN][FX_NLF];    // (label << 48 | elabel << 32) of later neighbours
    int32_t nlf_need[FX_MAXN][FX_NLF];    // how many such neighbours i needs
};

struct FxGraphDev {
    int64_t nv;
    int64_t nadj;
    const int64_t *rowp;
    const uint64_t *adj;
    const int32_t *bucket;
    const int64_t *bptr;
    int32_t nvl;   // dense vertex labels
    int32_t nel;   // dense edge labels
};

// Device-side counters of one query.  Written by kernels, read by the host
// once per step.
struct FxSummary {
    unsigned long long total_out;   // rows materialised by the last expansion
    unsigned long long t_next;      // candidate-space size of the new level
    unsigned long long count;       // embeddings counted so far
    unsigned long long digest0;     // sum of hashes (mod 2^64)
    unsigned long long digest1;     // xor of hashes
    unsigned long long support;     // embeddings selected so far
    unsigned long long hsize;       // hash-table size of the current greedy
    unsigned long long pad;
};

// One level of the slice stack: partial embeddings with l matched vertices
// and, for each, the candidate run of pattern vertex l.
struct FxLevelDev {
    int32_t *rows;   // [cap * l]
    int64_t *lo;     // start of the candidate run (index into adj, or into bucket if anc < 0)
    int32_t *len;    // length of the run
    int8_t *anc;     // pattern vertex whose neighbour run is used, -1 for a label bucket
    int64_t *off;    // exclusive prefix of len, [cap + 1]
};

// Probe modes
enum : int32_t {
    FX_PROBE_UFILTER = 1,   // materialise only candidates disjoint from the used set U
    FX_PROBE_COUNT = 2,     // count (and hash) every valid candidate of the last vertex
};

struct FxWork;  // host-side workspace (fx_api.hip)

// Launchers (fx_kernels.hip).  All return hipError_t of the launch.
hipError_t fx_launch_probe(hipStream_t s, const FxGraphDev &g, const FxPlan *plan, int32_t n, int32_t l,
                           const FxLevelDev &in, int64_t nparts, uint64_t t0, uint64_t t1, int32_t flags,
                           const uint32_t *U, uint8_t *flag, uint32_t *bcnt, FxSummary *sum);
hipError_t fx_launch_scan_blocks(hipStream_t s, const uint32_t *bcnt, uint32_t nblocks, uint64_t *boff,
                                 FxSummary *sum);
hipError_t fx_launch_scatter(hipStream_t s, const FxGraphDev &g, const FxPlan *plan, int32_t n, int32_t l,
                             const FxLevelDev &in, int64_t nparts, uint64_t t0, uint64_t t1,
                             const uint8_t *flag, const uint64_t *boff, const FxLevelDev &out);
hipError_t fx_launch_scan_len(hipStream_t s, const FxLevelDev &lev, uint64_t max_rows, int64_t *bsum,
                              FxSummary *sum);
hipError_t fx_launch_greedy_init(hipStream_t s, const int32_t *rows, int32_t n, uint64_t nrows,
                                 int32_t *hkey, unsigned long long *hval, uint64_t hsize, int32_t *slot,
                                 uint8_t *state, uint32_t *rem, FxSummary *sum);
hipError_t fx_launch_greedy_round(hipStream_t s, const int32_t *rows, int32_t n, uint64_t nrows,
                                  unsigned long long *hval, const int32_t *slot, uint8_t *state, uint32_t *rem,
                                  uint32_t round, uint32_t *U, int32_t *sel_rows, int64_t *sel_rank,
                                  int64_t rank_base, FxSummary *sum);
hipError_t fx_launch_fill_u32(hipStream_t s, uint32_t *p, uint64_t n, uint32_t v);
hipError_t fx_launch_level0(hipStream_t s, const FxGraphDev &g, const FxPlan *plan, FxLevelDev lev0);
