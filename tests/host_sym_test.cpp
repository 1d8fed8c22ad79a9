// Driver for tests/test_host_sym.py: reads patterns from stdin and prints the
// symmetry-breaking masks of paper_2404_01585_amd/csrc/fx_sym.h.
// Input: count, then per pattern a search budget (0: the library's default),
// n, n vertex labels and the n x n matrix of edge labels (-1: no edge).
// Output: one line of n masks per pattern.
#include <cstdio>

#include "fx_sym.h"

int main()
{
    int count = 0;
    if (std::scanf("%d", &count) != 1) return 1;
    for (int c = 0; c < count; c++) {
        long long budget = 0;
        int n = 0;
        if (std::scanf("%lld %d", &budget, &n) != 2 || n < 1 || n > FX_MAXN) return 1;
        int32_t vl[FX_MAXN] = {};
        int32_t el[FX_MAXN][FX_MAXN];
        for (int i = 0; i < n; i++)
            if (std::scanf("%d", &vl[i]) != 1) return 1;
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++)
                if (std::scanf("%d", &el[i][j]) != 1) return 1;
        uint16_t lt[FX_MAXN] = {};
        if (budget > 0) fx_symmetry_constraints(n, vl, el, lt, budget);
        else fx_symmetry_constraints(n, vl, el, lt);
        for (int i = 0; i < n; i++) std::printf("%d%c", (int)lt[i], i + 1 < n ? ' ' : '\n');
    }
    return 0;
}
