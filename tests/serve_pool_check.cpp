// Randomised check of the serving pool allocator (host code only).
#include <cassert>
#include <cstdio>
#include <random>
#include <vector>

#include "serve_pool.hpp"

int main()
{
    using qgs::Pool;
    std::mt19937_64 rng(7);
    for (int trial = 0; trial < 200; ++trial) {
        Pool pool;
        const size_t size = 256 * (1 + rng() % 4096);
        pool.init(size);
        struct Blk { size_t off, len; };
        std::vector<Blk> live;
        for (int step = 0; step < 2000; ++step) {
            if (live.empty() || rng() % 3 != 0) {
                const size_t len = 1 + rng() % (size / 8 + 1);
                size_t off;
                if (pool.alloc(len, off)) {
                    const size_t a = qgs::pool_align(len);
                    assert(off % 256 == 0 && off + a <= size);
                    for (auto &b : live)  // no overlap with live blocks
                        assert(off + a <= b.off || b.off + qgs::pool_align(b.len) <= off);
                    live.push_back({off, len});
                } else {
                    // refused only if no free range is large enough
                    for (auto &f : pool.free_) assert(f.second < qgs::pool_align(len));
                }
            } else {
                const size_t k = rng() % live.size();
                pool.release(live[k].off, live[k].len);
                live.erase(live.begin() + k);
            }
            size_t used = 0;
            for (auto &b : live) used += qgs::pool_align(b.len);
            assert(used == pool.used && pool.peak >= pool.used && pool.peak <= size);
            // free ranges are disjoint, sorted and never adjacent (fully merged)
            size_t prev_end = 0, free_total = 0;
            bool first = true;
            for (auto &f : pool.free_) {
                assert(first || f.first > prev_end);
                prev_end = f.first + f.second;
                free_total += f.second;
                first = false;
            }
            assert(free_total + used == size);
        }
        for (auto &b : live) pool.release(b.off, b.len);
        assert(pool.used == 0 && pool.free_.size() == 1 && pool.free_.begin()->second == size);
    }
    std::puts("pool ok");
    return 0;
}
