// First-fit allocator of byte ranges inside one device arena (the request
// server's HBM budget).  Host code only: it hands out offsets, the caller
// owns the memory.  Free ranges are kept sorted by offset and coalesced with
// both neighbours on release; every request is rounded up to kAlign.
#pragma once

#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>

namespace pit {

constexpr size_t kArenaAlign = 256;
inline size_t arena_round(size_t x) { return (x + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }

struct Arena {
    std::map<size_t, size_t> free;  // offset -> size
    size_t used = 0;
    void init(size_t off, size_t size)
    {
        free.clear();
        if (size) free[off] = size;
        used = 0;
    }
    bool alloc(size_t bytes, size_t &off)
    {
        bytes = arena_round(bytes);
        for (auto it = free.begin(); it != free.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const size_t rest = it->second - bytes;
            free.erase(it);
            if (rest) free[off + bytes] = rest;
            used += bytes;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = arena_round(bytes);
        used -= bytes;
        auto it = free.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free.erase(nx);
        }
        if (it != free.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free.erase(it);
            }
        }
    }
    size_t largest() const
    {
        size_t m = 0;
        for (auto &kv : free) m = std::max(m, kv.second);
        return m;
    }
};

}  // namespace pit
