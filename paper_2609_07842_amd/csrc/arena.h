// arena.h -- first-fit allocator of contiguous index ranges, the bookkeeping behind a
// replica pool's particle slots, bricks, cells and caller-order indices (host only).
#pragma once
#include <cstdint>
#include <iterator>
#include <map>

namespace vbc {

// Free ranges of [0, cap) as start -> length; take(n) returns the start of the first free
// range of at least n (or -1) and keeps its remainder; give(start, n) returns a range and
// merges it with free neighbours, so that free ranges never touch.
struct Arena {
    std::map<int64_t, int64_t> free;
    void init(int64_t cap)
    {
        free.clear();
        if (cap > 0) free[0] = cap;
    }
    int64_t take(int64_t n)
    {
        if (n <= 0) return 0;
        for (auto it = free.begin(); it != free.end(); ++it) {
            if (it->second < n) continue;
            int64_t start = it->first, len = it->second;
            free.erase(it);
            if (len > n) free[start + n] = len - n;
            return start;
        }
        return -1;
    }
    void give(int64_t start, int64_t n)
    {
        if (n <= 0) return;
        auto it = free.emplace(start, n).first;
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
};

}  // namespace vbc
