// Check of the host worker threads (paper_2404_01585_amd/csrc/fx_workers.h):
// every index of a job is visited exactly once, whatever the block size;
// back-to-back jobs of different sizes; callers on several threads at once
// take turns; a pool is destroyed cleanly after use and without use.
#include <atomic>
#include <cstdio>
#include <memory>
#include <thread>
#include <vector>

#include "fx_workers.h"

#define CHECK(c)                                                                 \
    do {                                                                         \
        if (!(c)) {                                                              \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                                            \
        }                                                                        \
    } while (0)

static int one_job(HostWorkers &w, int64_t n, int64_t grain)
{
    std::unique_ptr<std::atomic<int>[]> hits(new std::atomic<int>[n > 0 ? n : 1]);
    for (int64_t i = 0; i < n; i++) hits[i] = 0;
    std::atomic<int64_t> sum{0};
    w.run(n, grain, [&](int64_t a, int64_t b) {
        if (a < 0 || b > n || a >= b || b - a > grain) sum.fetch_add(1LL << 50);  // a malformed block
        for (int64_t i = a; i < b; i++) {
            hits[i].fetch_add(1);
            sum.fetch_add(i);
        }
    });
    for (int64_t i = 0; i < n; i++) CHECK(hits[i].load() == 1);
    CHECK(sum.load() == (n > 0 ? n * (n - 1) / 2 : 0));
    return 0;
}

int main()
{
    {
        HostWorkers unused(4);  // never started
    }
    {
        HostWorkers w(5);
        const int64_t sizes[] = {0, 1, 2, 7, 64, 1000, 4097, 100000};
        const int64_t grains[] = {1, 3, 64, 256, 5000};
        for (int64_t n : sizes)
            for (int64_t g : grains)
                if (one_job(w, n, g)) return 1;
        CHECK(w.threads() == 4);
    }
    {
        HostWorkers w(8);
        std::atomic<int> failed{0};
        std::vector<std::thread> callers;
        for (int c = 0; c < 4; c++)
            callers.emplace_back([&, c] {
                for (int j = 0; j < 50; j++)
                    if (one_job(w, 1000 + 37 * j + c, 1 + (j % 9) * 17)) failed++;
            });
        for (auto &t : callers) t.join();
        CHECK(failed.load() == 0);
    }
    std::printf("ok\n");
    return 0;
}
