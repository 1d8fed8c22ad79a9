// Host-side consistency checks of a device step (no HIP types, so they build
// and are tested on the CPU).  With the check_steps tunable on, the engine
// checks every step's segment table before the launch and the tile map the
// device built for it afterwards: every range a kernel will index -- the
// level rows it reads, the rows it may write, the workgroup tiles -- must lie
// inside the buffers the host sized for it.  A failure is reported as an
// error instead of a launch that would read or write out of bounds.
#pragma once

#include <stdint.h>

#include <cstdio>
#include <string>
#include <vector>

// What the host knows about one segment of a step.
struct FxStepSeg {
    int32_t n;           // pattern vertices
    int32_t l;           // level expanded (vertices matched)
    int32_t kind;        // 0 inner, 1 greedy, 2 count, 3 list
    int32_t leaf;        // a count segment of vertex n-2 (the leaf last vertex counted in closed form)
    uint64_t t0, span;   // candidate range [t0, t0 + span) of the level
    uint64_t level_total;  // candidates of the level (T[l])
    int64_t nparts;      // rows of the level (1 at level 0)
    int64_t cap;         // rows per level of the stack
    uint64_t out_cap;    // rows the segment may write at level l + 1
    uint32_t blk0;       // first workgroup
};

// One workgroup's tile as the device mapped it.
struct FxStepTile {
    int32_t seg;
    int32_t np;
    int64_t p0;
};

// Checks a step's segment table; tile = candidates per workgroup,
// max_blocks = workgroups the step's buffers hold, budget = candidates per
// step.  Returns "" or the first violation.
inline std::string fx_check_segments(const std::vector<FxStepSeg> &segs, uint32_t nblocks, uint32_t tile,
                                     uint64_t max_blocks, uint64_t budget)
{
    char buf[256];
    uint64_t blocks = 0, cands = 0;
    for (size_t k = 0; k < segs.size(); k++) {
        const FxStepSeg &s = segs[k];
        auto fail = [&](const char *what) {
            std::snprintf(buf, sizeof(buf), "segment %zu (n %d, l %d, kind %d): %s", k, s.n, s.l, s.kind, what);
            return std::string(buf);
        };
        if (s.n < 1 || s.n > 16) return fail("pattern size outside [1, 16]");
        if (s.l < 0 || s.l >= s.n) return fail("level outside [0, n)");
        if (s.span == 0) return fail("empty span");
        if (s.span > 0xffffffffull) return fail("span beyond 32 bits");
        if (s.t0 + s.span > s.level_total) return fail("candidate range past the level's candidates");
        if (s.l == 0 ? s.nparts != 1 : (s.nparts < 1 || s.nparts > s.cap)) return fail("level rows outside the stack");
        if (s.kind == 0 && s.l + 1 >= s.n) return fail("inner segment at the last vertex");
        if ((s.kind == 1 || s.kind == 3) && s.l != s.n - 1) return fail("complete embeddings before the last vertex");
        if (s.kind == 2 && s.l != s.n - 1 && !(s.leaf && s.l == s.n - 2)) return fail("counting segment at a wrong level");
        if (s.kind != 2 && (s.out_cap == 0 || s.out_cap > (uint64_t)s.cap)) return fail("row cap outside the stack");
        if (s.blk0 != blocks) return fail("first workgroup does not follow the previous segment");
        blocks += (s.span + tile - 1) / tile;
        cands += s.span;
    }
    if (blocks != nblocks) {
        std::snprintf(buf, sizeof(buf), "step has %u workgroups, its segments %llu", nblocks,
                      (unsigned long long)blocks);
        return buf;
    }
    if (blocks > max_blocks) {
        std::snprintf(buf, sizeof(buf), "step needs %llu workgroups, its buffers hold %llu",
                      (unsigned long long)blocks, (unsigned long long)max_blocks);
        return buf;
    }
    if (cands > budget) return "step takes more candidates than its budget";
    return "";
}

// Checks the tile map the device built for the step: every workgroup's
// segment is the one whose workgroups contain it, and its partials lie inside
// that segment's level rows.
inline std::string fx_check_tiles(const std::vector<FxStepSeg> &segs, const std::vector<FxStepTile> &tiles,
                                  uint32_t tile)
{
    char buf[256];
    for (size_t b = 0; b < tiles.size(); b++) {
        const FxStepTile &t = tiles[b];
        if (t.seg < 0 || (size_t)t.seg >= segs.size()) {
            std::snprintf(buf, sizeof(buf), "tile %zu: segment %d out of range", b, t.seg);
            return buf;
        }
        const FxStepSeg &s = segs[t.seg];
        const uint64_t nblk = (s.span + tile - 1) / tile;
        if (b < s.blk0 || b >= s.blk0 + nblk) {
            std::snprintf(buf, sizeof(buf), "tile %zu: not a workgroup of segment %d", b, t.seg);
            return buf;
        }
        if (t.np < 1 || t.p0 < 0 || t.p0 + t.np > s.nparts) {
            std::snprintf(buf, sizeof(buf), "tile %zu: partials [%lld, %lld) outside the level's %lld rows", b,
                          (long long)t.p0, (long long)(t.p0 + t.np), (long long)s.nparts);
            return buf;
        }
    }
    return "";
}
