// Randomised check of the stack-memory pool (paper_2404_01585_amd/csrc/fx_pool.h)
// with a malloc-backed allocator: live regions never overlap and stay inside
// their chunks, the byte accounting holds, the budget is respected, and once
// everything is given back and flushed every chunk is one free range again.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <utility>
#include <vector>

#include "fx_pool.h"

static bool alloc_host(void **p, size_t bytes)
{
    *p = std::malloc(bytes);
    return *p != nullptr;
}

static void free_host(void *p) { std::free(p); }

#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                                   \
        }                                                               \
    } while (0)

int main()
{
    std::mt19937_64 rng(12345);
    for (int trial = 0; trial < 20; trial++) {
        RegionPool pool;
        pool.alloc_fn = alloc_host;
        pool.free_fn = free_host;
        pool.chunk_bytes = (size_t)1 << 20;
        pool.budget = (size_t)(1 + trial % 4) << 20;
        const size_t sizes[] = {256, 1000, 4096, 70000, 300000, 999999};
        std::vector<std::pair<char *, size_t>> live;
        size_t live_bytes = 0;
        for (int step = 0; step < 4000; step++) {
            if (live.empty() || rng() % 100 < 55) {
                const size_t want = sizes[rng() % 6] + rng() % 300;
                void *p = nullptr;
                if (pool.take(want, &p)) {
                    const size_t b = RegionPool::round(want);
                    char *q = (char *)p;
                    bool inside = false;
                    for (auto &c : pool.chunks) inside = inside || (q >= c.base && q + b <= c.base + c.size);
                    CHECK(inside);
                    for (auto &r : live) CHECK(q + b <= r.first || r.first + r.second <= q);
                    live.push_back({q, b});
                    live_bytes += b;
                } else {
                    CHECK(p == nullptr);
                }
            } else {
                const size_t k = rng() % live.size();
                pool.give(live[k].first, live[k].second);
                live_bytes -= live[k].second;
                live[k] = live.back();
                live.pop_back();
            }
            CHECK(pool.in_use == live_bytes);
            CHECK(pool.held <= pool.budget);
        }
        for (auto &r : live) pool.give(r.first, r.second);
        pool.flush();
        CHECK(pool.in_use == 0);
        for (auto &c : pool.chunks) CHECK(c.free_.size() == 1 && c.free_.begin()->first == 0 &&
                                          c.free_.begin()->second == c.size);
    }
    std::printf("ok\n");
    return 0;
}
