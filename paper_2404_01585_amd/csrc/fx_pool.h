// Device memory for the per-query slice stacks (host-side bookkeeping only;
// no HIP types, so the allocator logic builds and is tested on the CPU).
//
// Chunks are allocated once (up to a byte budget) and carved first-fit, with
// freed ranges merged back.  Admission control of the engine is "can this
// query's region be carved".  Nothing is returned to the runtime before the
// pool is destroyed, so steady-state admission makes no allocation call
// (hipFree would synchronise the device).
//
// Freed regions are first kept per exact size: the queries of one batch have
// a handful of region sizes (one per pattern size and slice capacity), so a
// region is usually handed out again in O(1) instead of after a first-fit
// walk over a fragmented free map.  The cached regions go back into the free
// map (merged) before the pool asks for a new chunk.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <iterator>
#include <map>
#include <unordered_map>
#include <vector>

struct RegionPool {
    using AllocFn = bool (*)(void **p, size_t bytes);  // true on success
    using FreeFn = void (*)(void *p);

    struct Chunk {
        char *base = nullptr;
        size_t size = 0;
        std::map<size_t, size_t> free_;  // offset -> length, non-adjacent ranges
    };
    std::vector<Chunk> chunks;
    std::unordered_map<size_t, std::vector<char *>> cached;  // exact size -> freed regions
    size_t in_use = 0, held = 0, budget = 0;
    size_t chunk_bytes = (size_t)4 << 30;
    AllocFn alloc_fn = nullptr;
    FreeFn free_fn = nullptr;

    RegionPool() = default;
    RegionPool(const RegionPool &) = delete;
    RegionPool &operator=(const RegionPool &) = delete;
    ~RegionPool()
    {
        for (auto &c : chunks)
            if (c.base && free_fn) free_fn(c.base);
    }

    static size_t round(size_t bytes) { return (bytes + 255) & ~(size_t)255; }

    // A region of `bytes` (rounded up to 256), or false when nothing fits
    // within the budget or the allocator fails.
    bool take(size_t bytes, void **out)
    {
        bytes = round(bytes);
        *out = nullptr;
        auto hit = cached.find(bytes);
        if (hit != cached.end() && !hit->second.empty()) {
            *out = hit->second.back();
            hit->second.pop_back();
            in_use += bytes;
            return true;
        }
        if (first_fit(bytes, out)) return true;
        if (flush() && first_fit(bytes, out)) return true;
        if (held + bytes > budget || !alloc_fn) return false;
        Chunk c;
        c.size = std::min(std::max(bytes, chunk_bytes), budget - held);
        void *base = nullptr;
        if (!alloc_fn(&base, c.size)) return false;
        c.base = (char *)base;
        held += c.size;
        if (c.size > bytes) c.free_[bytes] = c.size - bytes;
        *out = c.base;
        in_use += bytes;
        chunks.push_back(std::move(c));
        return true;
    }

    void give(void *p, size_t bytes)
    {
        if (!p) return;
        bytes = round(bytes);
        cached[bytes].push_back((char *)p);
        in_use -= bytes;
    }

    // Returns every cached region to the free maps; true if there was any.
    bool flush()
    {
        bool any = false;
        for (auto &kv : cached) {
            for (char *p : kv.second) merge_back(p, kv.first);
            any = any || !kv.second.empty();
            kv.second.clear();
        }
        return any;
    }

private:
    bool first_fit(size_t bytes, void **out)
    {
        for (auto &c : chunks)
            for (auto it = c.free_.begin(); it != c.free_.end(); ++it)
                if (it->second >= bytes) {
                    const size_t off = it->first, len = it->second;
                    c.free_.erase(it);
                    if (len > bytes) c.free_[off + bytes] = len - bytes;
                    *out = c.base + off;
                    in_use += bytes;
                    return true;
                }
        return false;
    }

    void merge_back(char *q, size_t bytes)
    {
        for (auto &c : chunks) {
            if (q < c.base || q >= c.base + c.size) continue;
            size_t off = (size_t)(q - c.base), len = bytes;
            auto next = c.free_.lower_bound(off);
            if (next != c.free_.end() && next->first == off + len) {  // merge with the following range
                len += next->second;
                next = c.free_.erase(next);
            }
            if (next != c.free_.begin()) {  // merge with the preceding range
                auto prev = std::prev(next);
                if (prev->first + prev->second == off) {
                    off = prev->first;
                    len += prev->second;
                    c.free_.erase(prev);
                }
            }
            c.free_[off] = len;
            return;
        }
    }
};
