// First-fit allocator of byte ranges inside one device buffer, used by the
// serving scheduler to reserve each request's tile-list memory.  Plain C++
// (no device code), so its host logic is testable on its own.
#pragma once
#include <cstddef>
#include <iterator>
#include <map>

namespace qgs {

inline size_t pool_align(size_t x) { return (x + 255) & ~(size_t)255; }

// Ranges are 256-byte aligned; released ranges merge with free neighbours.
struct Pool {
    std::map<size_t, size_t> free_;  // offset -> length
    size_t size = 0, used = 0, peak = 0;
    void init(size_t n)
    {
        size = n;
        used = peak = 0;
        free_.clear();
        if (n) free_[0] = n;
    }
    bool alloc(size_t bytes, size_t &off)
    {
        bytes = pool_align(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                used += bytes;
                if (used > peak) peak = used;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = pool_align(bytes);
        used -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

}  // namespace qgs
