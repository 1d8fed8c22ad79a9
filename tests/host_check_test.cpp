// The host-side step checks (paper_2404_01585_amd/csrc/fx_check.h): a step
// laid out the way the engine lays one out passes; each way a segment table
// or a tile map could point outside its buffers is caught.
#include <cstdio>
#include <string>
#include <vector>

#include "fx_check.h"

#define CHECK(c)                                                                \
    do {                                                                        \
        if (!(c)) {                                                             \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                                           \
        }                                                                       \
    } while (0)

static std::vector<FxStepSeg> good_step(uint32_t tile, uint32_t *nblocks)
{
    // three queries: a root slice, an inner slice and a greedy slice
    std::vector<FxStepSeg> v;
    FxStepSeg a{};
    a.n = 3; a.l = 0; a.kind = 0; a.t0 = 0; a.span = 5000; a.level_total = 20000; a.nparts = 1; a.cap = 64;
    a.out_cap = 64;
    FxStepSeg b{};
    b.n = 4; b.l = 2; b.kind = 0; b.t0 = 100; b.span = 1500; b.level_total = 1600; b.nparts = 64; b.cap = 64;
    b.out_cap = 64;
    FxStepSeg c{};
    c.n = 3; c.l = 2; c.kind = 1; c.t0 = 0; c.span = 33; c.level_total = 33; c.nparts = 10; c.cap = 64;
    c.out_cap = 16;
    uint32_t blocks = 0;
    for (FxStepSeg *s : {&a, &b, &c}) {
        s->blk0 = blocks;
        blocks += (uint32_t)((s->span + tile - 1) / tile);
        v.push_back(*s);
    }
    *nblocks = blocks;
    return v;
}

int main()
{
    const uint32_t tile = 1024;
    uint32_t nb = 0;
    std::vector<FxStepSeg> v = good_step(tile, &nb);
    CHECK(fx_check_segments(v, nb, tile, 1000, 1u << 20).empty());
    // each mutation must be caught
    auto bad = [&](auto mutate, uint32_t blocks, uint64_t max_blocks = 1000, uint64_t budget = 1u << 20) {
        std::vector<FxStepSeg> w = v;
        mutate(w);
        return !fx_check_segments(w, blocks, tile, max_blocks, budget).empty();
    };
    CHECK(bad([](auto &w) { w[1].t0 = 200; }, nb));                      // range past the level's candidates
    CHECK(bad([](auto &w) { w[1].nparts = 65; }, nb));                   // level rows beyond the stack
    CHECK(bad([](auto &w) { w[0].nparts = 2; }, nb));                    // level 0 has one (empty) row
    CHECK(bad([](auto &w) { w[2].out_cap = 65; }, nb));                  // row cap beyond the stack
    CHECK(bad([](auto &w) { w[2].out_cap = 0; }, nb));                   // nothing may be written
    CHECK(bad([](auto &w) { w[1].blk0 += 1; }, nb));                     // workgroups overlap / gap
    CHECK(bad([](auto &w) { w[0].span = 0; }, nb));                      // empty segment
    CHECK(bad([](auto &w) { w[0].l = 3; }, nb));                         // level beyond the pattern
    CHECK(bad([](auto &w) { w[0].kind = 1; }, nb));                      // greedy before the last vertex
    CHECK(bad([](auto &w) { w[1].l = 3; w[1].kind = 0; w[1].level_total = 100000; }, nb));  // inner at the last vertex
    CHECK(bad([](auto &w) { w[2].kind = 2; w[2].l = 0; }, nb));          // counting at a wrong level
    CHECK(bad([](auto &) {}, nb + 1));                                  // launch size disagrees
    CHECK(bad([](auto &) {}, nb, nb - 1));                              // more workgroups than buffers
    CHECK(bad([](auto &) {}, nb, 1000, 4000));                          // more candidates than the budget
    // a counting segment of vertex n-2 is fine when the last vertex is a leaf
    {
        std::vector<FxStepSeg> w = v;
        w[2].kind = 2;
        w[2].l = 1;
        w[2].leaf = 1;
        w[2].nparts = 1 > 0 ? 10 : 0;
        CHECK(fx_check_segments(w, nb, tile, 1000, 1u << 20).empty());
        w[2].leaf = 0;
        CHECK(!fx_check_segments(w, nb, tile, 1000, 1u << 20).empty());
    }
    // tile map: a correct one, then wrong segments and partial ranges
    std::vector<FxStepTile> tiles;
    for (size_t k = 0; k < v.size(); k++) {
        const uint32_t blocks = (uint32_t)((v[k].span + tile - 1) / tile);
        for (uint32_t b = 0; b < blocks; b++) {
            FxStepTile t{};
            t.seg = (int32_t)k;
            t.p0 = 0;
            t.np = (int32_t)(v[k].nparts < 4 ? v[k].nparts : 4);
            tiles.push_back(t);
        }
    }
    CHECK(tiles.size() == nb);
    CHECK(fx_check_tiles(v, tiles, tile).empty());
    {
        auto t = tiles;
        t[0].seg = 2;  // a workgroup of segment 0 attributed to segment 2
        CHECK(!fx_check_tiles(v, t, tile).empty());
    }
    {
        auto t = tiles;
        t.back().p0 = 9;  // partials [9, 13) of a 10-row level
        CHECK(!fx_check_tiles(v, t, tile).empty());
    }
    {
        auto t = tiles;
        t[1].seg = -1;
        CHECK(!fx_check_tiles(v, t, tile).empty());
    }
    {
        auto t = tiles;
        t[3].np = 0;
        CHECK(!fx_check_tiles(v, t, tile).empty());
    }
    std::printf("ok\n");
    return 0;
}
