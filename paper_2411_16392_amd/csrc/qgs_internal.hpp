// Internal launch interfaces between the C ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qgs.h"

namespace qgs {

// Rasterizer constants shared by forward and backward (passed by value).
struct RasterParams {
    float fx, fy, cx, cy, ifx, ify;
    int32_t width, height, tiles_x, tiles_y;
    float near_plane, k2, alpha_min, alpha_max, T_eps, A_eps;
    float bg[3];
    uint32_t flags;
};

struct PreprocessArgs {
    const float *center, *quat, *scale, *curv, *opacity, *rgb;
    int64_t n;
    qgs_camera cam;
    float near_plane, k_sigma, alpha_min;
    void *records;
    uint32_t *depth_key;
    int32_t *rect;
    uint32_t *tiles;
    double *conic;
    double *frame;  // optional
    const float *sh;  // optional SH colour [n][K][3]
    int sh_degree;
    int tight;        // QGS_TIGHT_BOUND: the chord-bound local box
};

struct PreprocessBwdArgs {
    const float *center, *quat, *scale;
    const float *sh;  // optional SH colour [n][K][3]
    int sh_degree;
    int64_t n;
    qgs_camera cam;
    const float *grad_rec;  // [n][16]
    const uint32_t *tiles;
    qgs_scene_grads out;
    int accumulate;
};

hipError_t launch_preprocess(const PreprocessArgs &a, hipStream_t stream);
hipError_t launch_preprocess_bwd(const PreprocessBwdArgs &a, hipStream_t stream);

// ---- bin / sort --------------------------------------------------------------

// Elements per block of the radix passes: the per-primitive depth sort and
// the per-pair tile sort.  A pass over m elements uses a count table of
// 256 * ceil(m / chunk) entries (SortWorkspace::hist).
constexpr uint64_t DEPTH_SORT_CHUNK = 1024;
constexpr uint64_t TILE_SORT_CHUNK = 4096;
// Elements per workgroup of the device-wide scans (count tables, offsets): a
// scan of m elements keeps ceil(m / SCAN_CHUNK) partial sums.
constexpr int SCAN_CHUNK = 1024;

struct SortWorkspace {
    uint32_t *dkA, *dvA, *dkB, *dvB;  // depth keys / primitive ids, ping-pong [n]
    uint64_t *off;                    // [n + 1] pair offsets in depth order
    uint64_t *part;                   // scan partials
    uint32_t *hist;                   // [256][nblocks]
    uint32_t *tileT, *primT;          // pair ping-pong [capacity]
    uint32_t *emit_prim;              // primitive of each emitted pair [capacity]
    uint32_t *dkeyT;                  // per-tile depth key of each emitted pair [capacity]
    uint32_t *blk_cost;               // forward work of each 8 x 8 block [4 tiles], or NULL
    size_t bytes;
};

// Layout of the bin_sort workspace inside `base` (NULL base: sizes only).
SortWorkspace sort_workspace_layout(void *base, int64_t n, uint64_t capacity, uint64_t ntiles);

// Tiles by decreasing cost[t] (max4: the largest of cost[4 t .. 4 t + 3]; null
// cost: by list length, from ranges), the longest-processing-time-first order;
// one workgroup.
hipError_t launch_tile_order(const uint32_t *ranges, const uint32_t *cost, uint32_t ntiles, uint32_t *order,
                             hipStream_t stream, bool max4 = false);

struct BinSortArgs {
    int64_t n;
    const uint32_t *depth_key, *tiles;
    const int32_t *rect;
    const double *conic;
    qgs_camera cam;
    uint32_t *pair_offset;
    int32_t tiles_x, tiles_y;
    uint32_t *pair_tile, *pair_prim, *emit_to_sorted, *ranges, *tile_order, *counters;
    uint64_t capacity;
    const double *frame;  // non-null: key pairs by the per-tile depth
    float near_plane;
    // the records (non-null: tiles ordered by the forward's block work)
    const float *records = nullptr;
};

// Phase 1: depth sort, offsets, counters.  Phase 2: emission, tile sort, ranges
// with grids sized for `n_pairs_bound` pairs (the exact count, or the capacity).
hipError_t bin_sort_phase1(const BinSortArgs &a, const SortWorkspace &ws, hipStream_t stream);
hipError_t bin_sort_phase2(const BinSortArgs &a, const SortWorkspace &ws, uint64_t n_pairs_bound,
                           hipStream_t stream);

// ---- rasterizer --------------------------------------------------------------

struct RasterArgs {
    const float *records;  // [n][32]
    const uint32_t *pair_prim, *pair_tile, *ranges, *tile_order, *counters;
    const uint32_t *pair_offset, *tiles, *emit_to_sorted;
    int32_t tiles_x, tiles_y;
    // the backward's own order of 8 x 8 blocks (id 4 tile + block), taking the
    // place of tile_order when set; NULL elsewhere
    const uint32_t *block_order = nullptr;
};

struct FwdOut {
    float *color, *depth, *normal, *T_final;
    uint32_t *last;
    uint32_t flags;      // QGS_RESORT selects the resort kernels
    uint32_t *counters;  // counters[2..4] of the tile lists, or null
    // geometry maps: all set or all null
    float *curvature, *median_depth, *distortion;
    uint32_t *median_pos;
    // replay bitmap for the backward (both or null)
    uint64_t *steps;
    uint32_t *step_count;
    // caller events recorded just before and after the rasterizer kernel (or null)
    hipEvent_t ev_begin = nullptr, ev_end = nullptr;
};

struct BwdIn {
    const float *T_final;
    const uint32_t *last;
    const float *dcolor, *ddepth, *dnormal;
    // geometry gradients (any may be null) and the forward maps they need
    const float *dcurvature, *dmedian, *ddistortion;
    const float *depth, *distortion;
    const uint32_t *median_pos;
    // the forward's colour, normal and curvature (the front-to-back adjoint of
    // the resort mode needs every composited output)
    const float *color, *normal, *curvature;
    // the forward's replay bitmap (both or null)
    const uint64_t *steps;
    const uint32_t *step_count;
    uint32_t flags;
    // caller events recorded just before and after the rasterizer kernel (or null)
    hipEvent_t ev_begin = nullptr, ev_end = nullptr;
};

hipError_t launch_render_fwd(const RasterArgs &a, const RasterParams &p, const FwdOut &o, hipStream_t stream);
// order_ws: [2][tiles] u32 for the backward's own tile order (by the entries
// the replay bitmap makes each tile visit); null: the lists' tile order.
hipError_t launch_render_bwd(const RasterArgs &a, const RasterParams &p, const BwdIn &in, float *grad_rec,
                             float *pair_scratch, uint32_t *order_ws, int64_t n_prims, uint64_t capacity,
                             hipStream_t stream);

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, uint64_t n, hipStream_t stream);

}  // namespace qgs
