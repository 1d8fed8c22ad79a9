// Symmetry-breaking constraints of a pattern (host code only, no HIP types,
// so it builds and is tested on the CPU).
#pragma once

#include <stdint.h>

#ifndef FX_MAXN
#define FX_MAXN 16
#endif

// Backtracking search for an automorphism of the pattern (labels and labelled
// edges preserved) with some images forced (img[i] >= 0).  Counts its nodes
// against a budget; budget < 0 afterwards means the search was cut short.
struct AutSearch {
    int n = 0;
    const int32_t *vl = nullptr;
    const int32_t (*el)[FX_MAXN] = nullptr;
    int deg[FX_MAXN] = {};
    int img[FX_MAXN];
    bool used[FX_MAXN];
    int64_t budget = 0;

    bool fits(int i, int w) const
    {
        if (vl[w] != vl[i] || deg[w] != deg[i]) return false;
        for (int u = 0; u < i; u++)
            if (el[u][i] != el[img[u]][w]) return false;
        return true;
    }

    bool rec(int i)
    {
        if (--budget < 0) return false;
        if (i == n) return true;
        if (img[i] >= 0) return fits(i, img[i]) && rec(i + 1);
        for (int w = 0; w < n; w++) {
            if (used[w] || !fits(i, w)) continue;
            img[i] = w;
            used[w] = true;
            if (rec(i + 1)) return true;
            img[i] = -1;
            used[w] = false;
        }
        return false;
    }
};

// Symmetry breaking for the support phase.  The automorphisms of P permute the
// embeddings of one vertex set among themselves; the greedy over embeddings
// in lexicographic order keeps an embedding only if it is the first of its
// set, so it is enough to enumerate the lexicographically smallest member of
// each such orbit.  Walking the vertices in order 0, 1, ..., with the group
// shrunk to the stabiliser of the vertices already walked, every vertex w in
// the orbit of v (always w > v) gets the constraint f(v) < f(w); the members
// that meet all constraints are exactly the smallest ones.  Sets lt[w] bit v
// for each constraint.  A subset of the constraints (the search budget, in
// search nodes for the whole pattern, ran out) still keeps every smallest
// member, so the result stays exact.  The default budget bounds a plan's
// search at about a millisecond.
inline void fx_symmetry_constraints(int n, const int32_t *vl, const int32_t (*el)[FX_MAXN], uint16_t *lt,
                                    int64_t budget = 50000)
{
    AutSearch A;
    A.n = n;
    A.vl = vl;
    A.el = el;
    A.budget = budget;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) A.deg[i] += el[i][j] >= 0;
    bool fixed[FX_MAXN] = {};
    for (int v = 0; v < n; v++) {
        for (int w = v + 1; w < n; w++) {
            if (vl[w] != vl[v] || A.deg[w] != A.deg[v]) continue;
            for (int k = 0; k < n; k++) {
                A.img[k] = fixed[k] ? k : -1;
                A.used[k] = fixed[k];
            }
            A.img[v] = w;
            A.used[w] = true;
            const bool found = A.rec(0);
            if (A.budget < 0) return;
            if (found) lt[w] |= (uint16_t)(1u << v);
        }
        fixed[v] = true;
    }
}

