/*
 * Plain CPU oracle for FLEXIS support counting (arXiv 2404.01585).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header, table or helper with the
 * HIP library; it is written from the paper's definitions:
 *
 *   - subgraph isomorphism (Section 2.1.4): an embedding is an injective
 *     map f from pattern vertices to data vertices that preserves vertex
 *     labels and maps every pattern edge onto a data edge; extra data edges
 *     are allowed (non-induced).  Edge labels must match (Section 2.3.4
 *     turns edge labels into vertex labels; checking them directly is the
 *     same condition).
 *   - the mapping set M (Section 2.4) and independence (Section 2.4.1):
 *     two mappings are independent when they share no data vertex.
 *   - the maximal independent set mIS (Section 2.4.3), computed the way the
 *     modified matcher of Section 3.2.2 does it: a depth-first search in
 *     pattern-vertex order with a used-vertex bitmap and a per-root stop
 *     flag, which selects embeddings greedily in lexicographic order.
 *   - the threshold tau (Section 3.1.1, the equation for tau).
 *   - MNI (Section 2.4.4), used only as an invariant (mIS <= MNI).
 *   - directed graphs (Section 2.2 states the problem for labeled, directed
 *     graphs): with og_graph.directed set, row u lists the heads of the edges
 *     u -> v, a pattern edge (a, b) is a -> b, and an embedding maps it onto
 *     a data edge f(a) -> f(b) with the same label.
 *
 * Everything is exact integer arithmetic except tau's lambda, which is
 * quantised to parts per million before the integer floor (a reading of the
 * tau equation; doubles round the floor wrongly for some inputs).
 *
 * The greedy order: embeddings are ranked lexicographically by the tuple
 * (f(0), ..., f(n-1)) in the submitted pattern-vertex numbering, and data
 * vertices by the caller's ids.  The paper leaves the order to its matcher;
 * this is the order its depth-first search produces when it matches pattern
 * vertices in submitted order and tries candidates in ascending id.
 *
 * Two independent forms of the support are provided and cross-checked by
 * the tests:
 *   og_support_literal : enumerate all of M, sort it, run the greedy
 *                        (the definition written out step by step);
 *   og_support_stream  : the depth-first search with used-vertex bitmap and
 *                        per-root stop flag (the matcher of Section 3.2.2),
 *                        with optional stop once tau selections exist.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define OG_MAXN 16

typedef struct {
    int64_t nv;
    const int64_t *row_ptr; /* [nv+1] */
    const int32_t *col;     /* ascending per row */
    const int32_t *vlabel;  /* [nv] */
    const int32_t *elabel;  /* [row_ptr[nv]] */
    int32_t directed;       /* 0: symmetric rows; 1: row u holds the heads of u's edges */
} og_graph;

typedef struct {
    int32_t n, m;
    const int32_t *vlabel; /* [n] */
    const int32_t *edges;  /* [2m] pairs (a, b) */
    const int32_t *elabel; /* [m] */
} og_pattern;

/* ------------------------------------------------------------------ */
/* tau (Section 3.1.1, equation for tau):                              */
/*   tau = floor(sigma * (1 - 1/n) * lambda + sigma / n)               */
/*       = floor(sigma * ((n-1) * lambda + 1) / n)                     */
/* lambda is taken in parts per million, so the floor is exact.        */
/* ------------------------------------------------------------------ */
int64_t og_tau(int64_t sigma, double lambda, int32_t n)
{
    long long lam_ppm = llround(lambda * 1000000.0);
    __int128 num = (__int128)sigma * ((__int128)(n - 1) * lam_ppm + 1000000);
    __int128 den = (__int128)n * 1000000;
    __int128 q = num / den;
    if (num % den != 0 && num < 0) q -= 1; /* floor for negatives (never used) */
    return (int64_t)q;
}

/* ------------------------------------------------------------------ */
/* data-graph helpers                                                  */
/* ------------------------------------------------------------------ */

/* Label of data edge {u, v}, or -1 when u and v are not adjacent.      */
static int32_t og_edge_label(const og_graph *g, int32_t u, int32_t v)
{
    int64_t lo = g->row_ptr[u], hi = g->row_ptr[u + 1];
    while (lo < hi) { /* binary search in the ascending row of u */
        int64_t mid = lo + (hi - lo) / 2;
        if (g->col[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    if (lo < g->row_ptr[u + 1] && g->col[lo] == v) return g->elabel[lo];
    return -1;
}

/* Label of the pattern edge a -> b (directed), or -1.                  */
static int32_t og_pattern_arc(const og_pattern *p, int a, int b)
{
    for (int k = 0; k < p->m; k++)
        if (p->edges[2 * k] == a && p->edges[2 * k + 1] == b) return p->elabel ? p->elabel[k] : 0;
    return -1;
}

/* Label of pattern edge {a, b}, or -1.                                 */
static int32_t og_pattern_edge(const og_pattern *p, int a, int b)
{
    for (int k = 0; k < p->m; k++) {
        int x = p->edges[2 * k], y = p->edges[2 * k + 1];
        if ((x == a && y == b) || (x == b && y == a)) return p->elabel ? p->elabel[k] : 0;
    }
    return -1;
}

/* ------------------------------------------------------------------ */
/* Embedding enumeration (Section 2.1.4 and Section 2.4).              */
/* Pattern vertices are matched in submitted order 0..n-1; candidates  */
/* for vertex i are tried in ascending data-vertex id, so embeddings   */
/* come out in lexicographic order of (f(0), ..., f(n-1)).             */
/* ------------------------------------------------------------------ */

typedef struct og_dfs og_dfs;
/* return value of the visitor: 0 continue, 1 abandon the current root,
 * 2 stop everything */
typedef int (*og_visit_fn)(og_dfs *s);

struct og_dfs {
    const og_graph *g;
    const og_pattern *p;
    int n;
    int32_t f[OG_MAXN];
    int32_t back_lab[OG_MAXN][OG_MAXN]; /* label of pattern edge (a, i), a < i, or -1 */
    int32_t arc_lab[OG_MAXN][OG_MAXN];  /* directed: label of the pattern edge a -> b, or -1 */
    int first_back[OG_MAXN];            /* smallest earlier neighbour of i, or -1 (directed: the
                                           smallest earlier a with an edge a -> i) */
    const uint8_t *skip;                /* optional: data vertices that may not be used */
    og_visit_fn visit;
    void *user;
};

/* Can data vertex w be the image of pattern vertex i, given f[0..i-1]? */
static int og_feasible(og_dfs *s, int i, int32_t w)
{
    if (s->g->vlabel[w] != s->p->vlabel[i]) return 0;
    if (s->skip && s->skip[w]) return 0;
    for (int a = 0; a < i; a++)
        if (s->f[a] == w) return 0; /* injective */
    if (s->g->directed) {
        for (int a = 0; a < i; a++) {
            if (s->arc_lab[a][i] >= 0 && og_edge_label(s->g, s->f[a], w) != s->arc_lab[a][i]) return 0;
            if (s->arc_lab[i][a] >= 0 && og_edge_label(s->g, w, s->f[a]) != s->arc_lab[i][a]) return 0;
        }
        return 1;
    }
    for (int a = 0; a < i; a++) {
        int32_t want = s->back_lab[a][i];
        if (want < 0) continue;
        if (og_edge_label(s->g, s->f[a], w) != want) return 0;
    }
    return 1;
}

/* Returns 0 normally, 1 when the visitor abandoned the root, 2 to stop. */
static int og_rec(og_dfs *s, int i)
{
    if (i == s->n) return s->visit(s);
    int b = s->first_back[i];
    if (b >= 0) {
        int32_t u = s->f[b];
        for (int64_t k = s->g->row_ptr[u]; k < s->g->row_ptr[u + 1]; k++) {
            int32_t w = s->g->col[k];
            if (!og_feasible(s, i, w)) continue;
            s->f[i] = w;
            int r = og_rec(s, i + 1);
            if (r == 2) return 2;
            if (r == 1 && i > 0) return 1; /* unwind up to the root */
        }
    } else {
        for (int64_t w = 0; w < s->g->nv; w++) {
            if (!og_feasible(s, i, (int32_t)w)) continue;
            s->f[i] = (int32_t)w;
            int r = og_rec(s, i + 1);
            if (r == 2) return 2;
            if (r == 1 && i > 0) return 1;
        }
    }
    return 0;
}

static void og_dfs_init(og_dfs *s, const og_graph *g, const og_pattern *p)
{
    memset(s, 0, sizeof(*s));
    s->g = g;
    s->p = p;
    s->n = p->n;
    for (int i = 0; i < p->n; i++) {
        s->first_back[i] = -1;
        for (int a = 0; a < p->n; a++) s->back_lab[a][i] = -1;
    }
    for (int a = 0; a < p->n; a++)
        for (int b = 0; b < p->n; b++) s->arc_lab[a][b] = g->directed ? og_pattern_arc(p, a, b) : -1;
    for (int i = 0; i < p->n; i++)
        for (int a = 0; a < i; a++) {
            s->back_lab[a][i] = og_pattern_edge(p, a, i);
            /* candidates of i come from the row of f(a): in a directed graph
             * that row holds f(a)'s out-neighbours, so only an edge a -> i */
            const int from = g->directed ? s->arc_lab[a][i] >= 0 : s->back_lab[a][i] >= 0;
            if (from && s->first_back[i] < 0) s->first_back[i] = a;
        }
}

/* Rejects malformed patterns: n outside [1, 16], bad endpoints, loops,
 * repeated edges, or a disconnected pattern.  Returns 0 when valid.  With
 * `directed`, (a, b) and (b, a) are different edges and connected means
 * weakly connected. */
static int og_check_pattern_d(const og_pattern *p, int directed)
{
    if (p->n < 1 || p->n > OG_MAXN || p->m < 0) return -1;
    for (int k = 0; k < p->m; k++) {
        int a = p->edges[2 * k], b = p->edges[2 * k + 1];
        if (a < 0 || b < 0 || a >= p->n || b >= p->n || a == b) return -1;
        for (int j = 0; j < k; j++) {
            int x = p->edges[2 * j], y = p->edges[2 * j + 1];
            if ((x == a && y == b) || (!directed && x == b && y == a)) return -1;
        }
    }
    /* connectivity by repeated relaxation */
    int reach[OG_MAXN] = {0};
    reach[0] = 1;
    for (int it = 0; it < p->n; it++)
        for (int k = 0; k < p->m; k++) {
            int a = p->edges[2 * k], b = p->edges[2 * k + 1];
            if (reach[a] || reach[b]) reach[a] = reach[b] = 1;
        }
    for (int i = 0; i < p->n; i++)
        if (!reach[i]) return -1;
    return 0;
}

int og_check_pattern(const og_pattern *p) { return og_check_pattern_d(p, 0); }

static int og_check(const og_graph *g, const og_pattern *p) { return og_check_pattern_d(p, g->directed); }

/* ------------------------------------------------------------------ */
/* Literal form: list M, sort it, then the greedy (Section 2.4.3).     */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t *rows;
    int64_t count, cap;
    int stored_all;
} og_list;

static int og_visit_list(og_dfs *s)
{
    og_list *L = (og_list *)s->user;
    if (L->count < L->cap) memcpy(L->rows + L->count * s->n, s->f, sizeof(int32_t) * s->n);
    else L->stored_all = 0;
    L->count++;
    return 0;
}

static int og_n_for_cmp;
static int og_cmp_rows(const void *x, const void *y)
{
    const int32_t *a = (const int32_t *)x, *b = (const int32_t *)y;
    for (int j = 0; j < og_n_for_cmp; j++) {
        if (a[j] < b[j]) return -1;
        if (a[j] > b[j]) return 1;
    }
    return 0;
}

/* Enumerates M.  Writes min(|M|, cap) rows of n vertex ids, sorted
 * lexicographically, into out.  Returns |M| (or -1 on a bad pattern).
 * When |M| > cap the rows written are the lexicographically first cap. */
int64_t og_enumerate(const og_graph *g, const og_pattern *p, int32_t *out, int64_t cap)
{
    if (og_check(g, p)) return -1;
    og_dfs s;
    og_dfs_init(&s, g, p);
    og_list L = {out, 0, cap, 1};
    s.visit = og_visit_list;
    s.user = &L;
    og_rec(&s, 0);
    int64_t kept = L.count < cap ? L.count : cap;
    og_n_for_cmp = p->n;
    qsort(out, (size_t)kept, sizeof(int32_t) * p->n, og_cmp_rows); /* step 2: order */
    return L.count;
}

/* Sequential greedy over rows already in rank order (Section 2.4.3 with
 * the used-vertex bitmap of Section 3.2.2): keep a row iff it shares no
 * vertex with the rows kept before it.  Writes kept row indices to sel
 * (if not NULL) and returns how many rows were kept. */
int64_t og_greedy_rows(const int32_t *rows, int64_t count, int32_t n, int64_t nv, int64_t *sel)
{
    uint8_t *used = (uint8_t *)calloc((size_t)nv, 1);
    int64_t k = 0;
    for (int64_t r = 0; r < count; r++) {
        const int32_t *e = rows + r * n;
        int clash = 0;
        for (int j = 0; j < n; j++)
            if (used[e[j]]) clash = 1;
        if (clash) continue;
        for (int j = 0; j < n; j++) used[e[j]] = 1;
        if (sel) sel[k] = r;
        k++;
    }
    free(used);
    return k;
}

/* Literal support: enumerate M (must fit in cap rows), sort, greedy.
 * Writes the selected tuples in rank order to sel_out (room for
 * sel_cap rows).  Returns the support, -1 on a bad pattern and -2 when M
 * does not fit in cap rows. */
int64_t og_support_literal(const og_graph *g, const og_pattern *p, int64_t cap,
                           int32_t *sel_out, int64_t sel_cap)
{
    int32_t *rows = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1) * p->n);
    int64_t cnt = og_enumerate(g, p, rows, cap);
    if (cnt < 0) { free(rows); return -1; }
    if (cnt > cap) { free(rows); return -2; }
    int64_t *sel = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cnt > 0 ? cnt : 1));
    int64_t k = og_greedy_rows(rows, cnt, p->n, g->nv, sel);
    for (int64_t i = 0; i < k && i < sel_cap; i++)
        memcpy(sel_out + i * p->n, rows + sel[i] * p->n, sizeof(int32_t) * p->n);
    free(sel);
    free(rows);
    return k;
}

/* ------------------------------------------------------------------ */
/* Streaming form (Section 3.2.2): depth-first search with a used-     */
/* vertex bitmap shared by the whole search and a per-root stop flag:  */
/* after a match the search leaves the current root; the bitmap keeps  */
/* later matches disjoint.  Optionally stops once `stop_at` embeddings */
/* are selected (the early termination at tau of Section 3.1.1).       */
/* ------------------------------------------------------------------ */

typedef struct {
    uint8_t *used;
    int32_t *sel_out;
    int64_t sel_cap, support, stop_at;
} og_stream;

static int og_visit_stream(og_dfs *s)
{
    og_stream *S = (og_stream *)s->user;
    for (int j = 0; j < s->n; j++) S->used[s->f[j]] = 1;
    if (S->sel_out && S->support < S->sel_cap)
        memcpy(S->sel_out + S->support * s->n, s->f, sizeof(int32_t) * s->n);
    S->support++;
    if (S->stop_at > 0 && S->support >= S->stop_at) return 2;
    return 1; /* abandon this root */
}

int64_t og_support_stream(const og_graph *g, const og_pattern *p, int64_t stop_at,
                          int32_t *sel_out, int64_t sel_cap)
{
    if (og_check(g, p)) return -1;
    og_dfs s;
    og_dfs_init(&s, g, p);
    og_stream S;
    S.used = (uint8_t *)calloc((size_t)g->nv, 1);
    S.sel_out = sel_out;
    S.sel_cap = sel_cap;
    S.support = 0;
    S.stop_at = stop_at;
    s.skip = S.used;
    s.visit = og_visit_stream;
    s.user = &S;
    og_rec(&s, 0);
    free(S.used);
    return S.support;
}

/* ------------------------------------------------------------------ */
/* Embedding count and order-independent digest of M.                  */
/* The digest hashes each tuple with the SplitMix64 finaliser (Steele, */
/* Lea and Flood, OOPSLA 2014; constants as published by Vigna):       */
/*   h(e; s): x = s; for each j: x = mix(x xor f(j)).                  */
/* digest[0] = sum of h(e; S1) mod 2^64, digest[1] = xor of h(e; S2).  */
/* ------------------------------------------------------------------ */

static uint64_t og_mix(uint64_t x)
{
    uint64_t z = x + 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t og_tuple_hash(const int32_t *e, int32_t n, uint64_t seed)
{
    uint64_t x = seed;
    for (int j = 0; j < n; j++) x = og_mix(x ^ (uint64_t)(uint32_t)e[j]);
    return x;
}

#define OG_SEED1 0x243f6a8885a308d3ULL
#define OG_SEED2 0x13198a2e03707344ULL

typedef struct {
    int64_t count, cap;
    uint64_t d0, d1;
} og_counter;

static int og_visit_count(og_dfs *s)
{
    og_counter *C = (og_counter *)s->user;
    C->count++;
    C->d0 += og_tuple_hash(s->f, s->n, OG_SEED1);
    C->d1 ^= og_tuple_hash(s->f, s->n, OG_SEED2);
    if (C->count >= C->cap) return 2;
    return 0;
}

/* The same digest over a list of rows (for instance the selected set S,
 * whose rank order is the lexicographic order of its tuples, so the set
 * fixes the list): digest_out[0] = sum of h(e; S1), digest_out[1] = xor of
 * h(e; S2) over the `count` rows of n ids each. */
void og_rows_digest(const int32_t *rows, int64_t count, int32_t n, uint64_t *digest_out)
{
    uint64_t d0 = 0, d1 = 0;
    for (int64_t r = 0; r < count; r++) {
        d0 += og_tuple_hash(rows + r * n, n, OG_SEED1);
        d1 ^= og_tuple_hash(rows + r * n, n, OG_SEED2);
    }
    digest_out[0] = d0;
    digest_out[1] = d1;
}

/* count_out = min(|M|, cap); saturated_out = (|M| >= cap); digest of M
 * (meaningful only when not saturated). Returns 0, or -1 on a bad pattern. */
int og_count(const og_graph *g, const og_pattern *p, int64_t cap, int64_t *count_out,
             int32_t *saturated_out, uint64_t *digest_out)
{
    if (og_check(g, p)) return -1;
    og_dfs s;
    og_dfs_init(&s, g, p);
    og_counter C = {0, cap, 0, 0};
    s.visit = og_visit_count;
    s.user = &C;
    if (cap > 0) og_rec(&s, 0);
    *count_out = C.count;
    *saturated_out = C.count >= cap;
    digest_out[0] = C.d0;
    digest_out[1] = C.d1;
    return 0;
}

/* ------------------------------------------------------------------ */
/* MNI (Section 2.4.4): min over pattern vertices of the number of     */
/* distinct images.                                                     */
/* ------------------------------------------------------------------ */

typedef struct {
    uint8_t *img; /* n * nv flags */
    int64_t nv;
} og_mni_state;

static int og_visit_mni(og_dfs *s)
{
    og_mni_state *M = (og_mni_state *)s->user;
    for (int j = 0; j < s->n; j++) M->img[(int64_t)j * M->nv + s->f[j]] = 1;
    return 0;
}

int64_t og_mni(const og_graph *g, const og_pattern *p)
{
    if (og_check(g, p)) return -1;
    og_dfs s;
    og_dfs_init(&s, g, p);
    og_mni_state M;
    M.nv = g->nv;
    M.img = (uint8_t *)calloc((size_t)(p->n * g->nv), 1);
    s.visit = og_visit_mni;
    s.user = &M;
    og_rec(&s, 0);
    int64_t best = -1;
    for (int j = 0; j < p->n; j++) {
        int64_t c = 0;
        for (int64_t v = 0; v < g->nv; v++) c += M.img[(int64_t)j * g->nv + v];
        if (best < 0 || c < best) best = c;
    }
    free(M.img);
    return best;
}
