// Host reference for the order in which the rasterizers take tiles: for each
// tile, the largest over its four 8 x 8 pixel blocks of the number of the
// tile's list entries whose pixel rectangle meets the block and whose
// pre-test conic does too (conic_meets_block, the kernels' own host-callable
// code).  Reads DIR/records.bin (n x 32 words), DIR/ranges.bin (tiles x 2
// uint32) and DIR/prims.bin (the sorted primitive ids); writes DIR/cost.bin
// (tiles uint32).  Usage: block_work_check DIR tiles_x.  Compiled for the
// host only.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "qgs_device.hpp"

using namespace qgs;

template <typename T>
static std::vector<T> read_all(const std::string &path)
{
    std::vector<T> v;
    FILE *f = std::fopen(path.c_str(), "rb");
    if (!f) return v;
    std::fseek(f, 0, SEEK_END);
    const long bytes = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    v.resize((size_t)bytes / sizeof(T));
    if (std::fread(v.data(), sizeof(T), v.size(), f) != v.size()) v.clear();
    std::fclose(f);
    return v;
}

int main(int argc, char **argv)
{
    if (argc < 3) return 2;
    const std::string dir = argv[1];
    const int tiles_x = std::atoi(argv[2]);
    const std::vector<float4> recs = read_all<float4>(dir + "/records.bin");
    const std::vector<uint32_t> ranges = read_all<uint32_t>(dir + "/ranges.bin");
    const std::vector<uint32_t> prims = read_all<uint32_t>(dir + "/prims.bin");
    const size_t ntiles = ranges.size() / 2;
    std::vector<uint32_t> cost(ntiles, 0u);
    for (size_t t = 0; t < ntiles; ++t) {
        const int tx = (int)(t % (size_t)tiles_x), ty = (int)(t / (size_t)tiles_x);
        for (int k = 0; k < 4; ++k) {
            const int wx0 = tx * TILE + (k & 1) * 8, wy0 = ty * TILE + (k >> 1) * 8;
            uint32_t c = 0;
            for (uint32_t i = ranges[2 * t]; i < ranges[2 * t + 1]; ++i) {
                if (i >= prims.size() || 8 * (size_t)prims[i] + 8 > recs.size()) return 3;
                const float4 *rec = recs.data() + 8 * (size_t)prims[i];
                int32_t rc[4];
                std::memcpy(rc, &rec[0], sizeof rc);  // x0, x1, y0, y1
                if (rc[1] < wx0 || rc[0] > wx0 + 7 || rc[3] < wy0 || rc[2] > wy0 + 7) continue;
                if (conic_meets_block(rec, (float)wx0, (float)wy0)) ++c;
            }
            cost[t] = c > cost[t] ? c : cost[t];
        }
    }
    FILE *f = std::fopen((dir + "/cost.bin").c_str(), "wb");
    if (!f) return 4;
    const size_t w = std::fwrite(cost.data(), sizeof(uint32_t), ntiles, f);
    std::fclose(f);
    return w == ntiles ? 0 : 5;
}
