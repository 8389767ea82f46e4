// Tile|depth key lists: integer-only, bit-exact (the tile test is the FP64
// conic test of qgs_keys.hpp, with the same decisions as the preprocess).
//
// The required order is a stable sort of the 64-bit keys (tile << 32 | depth)
// emitted primitive by primitive (tiles row-major within each rectangle).  An
// LSD radix sort of those keys would first sort by the depth bits; since all
// pairs of one primitive share its depth, that part is done once per
// primitive instead of once per pair: the primitives are radix-sorted by depth
// key (stable, so ties keep primitive order), their pairs are emitted in that
// order, and a stable radix sort by tile id finishes the job.  The result is
// identical to the 64-bit sort; the pair arrays move 2 passes x 8 bytes instead
// of ceil((32 + tile bits) / 8) passes x 12 bytes.
//
// Radix passes are 8-bit LSD passes in three kernels: per-block digit counts,
// a device-wide exclusive scan of the digit-major count table, and a scatter
// that ranks each element stably inside its block (wave ballots on the digit
// bits, then per-wave counts in LDS), stages the block's elements in LDS in
// digit order and writes them out in contiguous runs.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qgs_device.hpp"
#include "qgs_internal.hpp"
#include "qgs_keys.hpp"

namespace qgs {

constexpr int RS_THREADS = 256;
// elements per thread of a radix block: small for the per-primitive depth
// sort (more blocks for a small array), large for the per-pair tile sort
constexpr int RS_ITEMS_DEPTH = (int)(DEPTH_SORT_CHUNK / RS_THREADS);
constexpr int RS_ITEMS_TILE = (int)(TILE_SORT_CHUNK / RS_THREADS);
static_assert(RS_ITEMS_DEPTH * RS_THREADS == (int)DEPTH_SORT_CHUNK && RS_ITEMS_TILE * RS_THREADS == (int)TILE_SORT_CHUNK,
              "radix chunks");
// arrays up to this size are scanned by a single workgroup (one kernel
// instead of three; a workgroup's sequential chunks are slow for more)
constexpr uint64_t SCAN_SINGLE_MAX = 8192;

static inline uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// element count: a host bound, or the pair count on the device (0 on overflow)
struct Count {
    const uint32_t *counters;  // null: use n
    uint64_t n;
    __device__ inline uint64_t get() const
    {
        if (!counters) return n;
        if (counters[1]) return 0;
        const uint64_t c = counters[0];
        return c < n ? c : n;
    }
};

// ---------------------------------------------------------------------------
// block-wide exclusive scan of one value per thread (256 threads)
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline T wave_incl_scan(T v, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const T o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

template <typename T>
__device__ inline T block_excl_scan(T v, T *s_wave /* [4] */, T &total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const T inc = wave_incl_scan(v, lane);
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    T pre = 0;
    for (int w = 0; w < wave; ++w) pre += s_wave[w];
    total = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
    __syncthreads();
    return pre + inc - v;
}

// ---------------------------------------------------------------------------
// device-wide exclusive scan: partial sums per SCAN_CHUNK-element chunk, then each
// chunk's scan plus the sum of the partials before it
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_scan_partials(const T *in, uint64_t n, T *part)
{
    __shared__ T s_wave[4];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_CHUNK;
    T acc = 0;
    for (int k = 0; k < SCAN_CHUNK / 256; ++k) {
        const uint64_t i = base + (uint64_t)k * 256 + threadIdx.x;
        if (i < n) acc += in[i];
    }
    T total;
    (void)block_excl_scan(acc, s_wave, total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// Each block adds the sum of the partials before it (its own short reduction:
// there are n / SCAN_CHUNK partials) to the exclusive scan of its chunk; the last
// block also writes the grand total.
template <typename T>
__global__ __launch_bounds__(256) void k_scan_apply(const T *in, T *out, uint64_t n, const T *part, T *grand_total)
{
    __shared__ T s_wave[4];
    T pre = 0;
    for (uint64_t k0 = 0; k0 < blockIdx.x; k0 += 256) {
        const uint64_t k = k0 + threadIdx.x;
        T tot;
        (void)block_excl_scan(k < blockIdx.x ? part[k] : (T)0, s_wave, tot);
        pre += tot;
    }
    // blocked arrangement: thread t owns items [t*16, t*16 + 16) of the chunk
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_CHUNK + (uint64_t)threadIdx.x * (SCAN_CHUNK / 256);
    T v[SCAN_CHUNK / 256];
    T acc = 0;
#pragma unroll
    for (int k = 0; k < SCAN_CHUNK / 256; ++k) {
        const uint64_t i = base + k;
        v[k] = i < n ? in[i] : 0;
        acc += v[k];
    }
    T total;
    T run = block_excl_scan(acc, s_wave, total) + pre;
#pragma unroll
    for (int k = 0; k < SCAN_CHUNK / 256; ++k) {
        const uint64_t i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
    if (grand_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *grand_total = pre + total;
}

// exclusive scan of a small array by one 1024-thread workgroup: each thread
// sums a contiguous chunk, the chunk sums are scanned, each chunk is rewritten
// (in == out allowed)
template <typename T>
__global__ __launch_bounds__(1024) void k_scan_single(const T *in, T *out, uint64_t n)
{
    __shared__ T s_w[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t per = (n + 1023) / 1024;
    const uint64_t b = (uint64_t)tid * per, e = b + per < n ? b + per : n;
    T acc = 0;
    for (uint64_t i = b; i < e; ++i) acc += in[i];
    const T inc = wave_incl_scan(acc, lane);
    if (lane == 63) s_w[wave] = inc;
    __syncthreads();
    T run = inc - acc;
    for (int w = 0; w < wave; ++w) run += s_w[w];
    for (uint64_t i = b; i < e; ++i) {
        const T v = in[i];
        out[i] = run;
        run += v;
    }
}

template <typename T>
static hipError_t device_excl_scan(const T *in, T *out, uint64_t n, T *part, T *grand_total, hipStream_t stream)
{
    const uint64_t nb = cdiv(n, SCAN_CHUNK);
    if (nb == 0) return hipSuccess;
    if (n <= SCAN_SINGLE_MAX && !grand_total) {
        hipLaunchKernelGGL(k_scan_single<T>, dim3(1), dim3(1024), 0, stream, in, out, n);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_partials<T>, dim3((unsigned)nb), dim3(256), 0, stream, in, n, part);
    hipLaunchKernelGGL(k_scan_apply<T>, dim3((unsigned)nb), dim3(256), 0, stream, in, out, n, (const T *)part,
                       grand_total);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// radix pass kernels (u32 keys, u32 values, 8-bit digit at `shift`)
// ---------------------------------------------------------------------------
template <int RS_ITEMS>
__global__ __launch_bounds__(RS_THREADS) void k_radix_hist(const uint32_t *keys, Count cnt, int shift, uint32_t *hist,
                                                           uint32_t nblocks)
{
    constexpr int RS_CHUNK = RS_THREADS * RS_ITEMS;
    __shared__ uint32_t h[4][256];
    for (int i = threadIdx.x; i < 1024; i += RS_THREADS) (&h[0][0])[i] = 0;
    __syncthreads();
    const uint64_t n = cnt.get();
    const uint64_t base = (uint64_t)blockIdx.x * RS_CHUNK;
    const int wave = threadIdx.x >> 6;
    for (int k = 0; k < RS_ITEMS; ++k) {
        const uint64_t i = base + (uint64_t)k * RS_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&h[wave][(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    const int d = threadIdx.x;
    hist[(uint64_t)d * nblocks + blockIdx.x] = h[0][d] + h[1][d] + h[2][d] + h[3][d];
}

template <int RS_ITEMS>
__global__ __launch_bounds__(RS_THREADS) void k_radix_scatter(const uint32_t *keys_in, const uint32_t *vals_in,
                                                              uint32_t *keys_out, uint32_t *vals_out, Count cnt,
                                                              int shift, const uint32_t *hist_scan, uint32_t nblocks)
{
    // Each wave ranks its own contiguous segment of RS_ITEMS * 64 elements
    // (element base + 64 (RS_ITEMS wave + k) + lane): lanes holding the same
    // digit are found with eight ballots, the lowest of them adds the group to
    // the wave's running digit count in LDS, so the wave needs no barrier.
    // The block then offsets each wave by the counts of the waves before it.
    constexpr int RS_CHUNK = RS_THREADS * RS_ITEMS;
    constexpr int NW = RS_THREADS / 64;
    __shared__ uint32_t s_keys[RS_CHUNK];
    __shared__ uint32_t s_vals[RS_CHUNK];
    __shared__ uint32_t wcnt[NW][256];
    __shared__ uint32_t lstart[256];
    __shared__ uint32_t goff[256];
    __shared__ uint32_t s_wave[4];

    const uint64_t n = cnt.get();
    const uint64_t base = (uint64_t)blockIdx.x * RS_CHUNK;
    if (base >= n) return;  // uniform for the block
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int w = 0; w < NW; ++w) wcnt[w][tid] = 0;
    goff[tid] = hist_scan[(uint64_t)tid * nblocks + blockIdx.x];
    __syncthreads();

    const uint64_t seg = base + (uint64_t)wave * (RS_ITEMS * 64);
    uint32_t key[RS_ITEMS], val[RS_ITEMS], rank[RS_ITEMS];
#pragma unroll
    for (int k = 0; k < RS_ITEMS; ++k) {
        const uint64_t i = seg + (uint64_t)k * 64 + lane;
        key[k] = i < n ? keys_in[i] : 0u;
        val[k] = i < n ? vals_in[i] : 0u;
    }
    const uint64_t lt = __lanemask_lt();
#pragma unroll
    for (int k = 0; k < RS_ITEMS; ++k) {
        const uint64_t i = seg + (uint64_t)k * 64 + lane;
        const bool valid = i < n;
        const uint32_t d = (key[k] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        if (!valid) peers = 0;
        const uint32_t r_in = (uint32_t)__popcll(peers & lt);
        const uint32_t before = valid ? wcnt[wave][d] : 0u;
        rank[k] = before + r_in;
        // every lane has read the running count before the leader adds
        __builtin_amdgcn_wave_barrier();
        if (valid && r_in == 0) wcnt[wave][d] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // digit d: offsets of the waves within the block's run of d, and the run's start
    uint32_t tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const uint32_t c = wcnt[w][tid];
        wcnt[w][tid] = tot;
        tot += c;
    }
    uint32_t total;
    lstart[tid] = block_excl_scan(tot, s_wave, total);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RS_ITEMS; ++k) {
        const uint64_t i = seg + (uint64_t)k * 64 + lane;
        if (i < n) {
            const uint32_t d = (key[k] >> shift) & 255u;
            const uint32_t pos = lstart[d] + wcnt[wave][d] + rank[k];
            s_keys[pos] = key[k];
            s_vals[pos] = val[k];
        }
    }
    __syncthreads();
    const uint32_t m = (uint32_t)((n - base) < (uint64_t)RS_CHUNK ? (n - base) : (uint64_t)RS_CHUNK);
    for (uint32_t i = tid; i < m; i += RS_THREADS) {
        const uint32_t kk = s_keys[i];
        const uint32_t d = (kk >> shift) & 255u;
        const uint32_t dst = goff[d] + (i - lstart[d]);
        keys_out[dst] = kk;
        vals_out[dst] = s_vals[i];
    }
}

// one stable 8-bit pass; grid sized for `bound` elements
template <int RS_ITEMS>
static hipError_t radix_pass(const uint32_t *ki, const uint32_t *vi, uint32_t *ko, uint32_t *vo, Count cnt,
                             uint64_t bound, int shift, const SortWorkspace &ws, hipStream_t stream)
{
    const uint64_t nb = cdiv(bound, (uint64_t)RS_THREADS * RS_ITEMS);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_radix_hist<RS_ITEMS>, dim3((unsigned)nb), dim3(RS_THREADS), 0, stream, ki, cnt, shift,
                       ws.hist, (uint32_t)nb);
    hipError_t e = device_excl_scan<uint32_t>(ws.hist, ws.hist, 256 * nb, reinterpret_cast<uint32_t *>(ws.part),
                                              (uint32_t *)nullptr, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter<RS_ITEMS>, dim3((unsigned)nb), dim3(RS_THREADS), 0, stream, ki, vi, ko, vo,
                       cnt, shift, (const uint32_t *)ws.hist, (uint32_t)nb);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// bin / sort stages
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_depth_init(const uint32_t *depth_key, const uint32_t *tiles, int64_t n,
                                                    uint32_t *keys, uint32_t *vals)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    // primitives without tiles emit no pairs; they sort last
    keys[p] = tiles[p] ? depth_key[p] : 0xFFFFFFFFu;
    vals[p] = (uint32_t)p;
}

__global__ __launch_bounds__(256) void k_gather_tiles(const uint32_t *order, const uint32_t *tiles, int64_t n,
                                                      uint64_t *out)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    out[r] = tiles[order[r]];
}

__global__ void k_set_counters(const uint64_t *total, uint64_t capacity, uint32_t *counters)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const uint64_t t = *total;
        counters[0] = t > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)t;
        counters[1] = t > capacity ? 1u : 0u;
        for (int i = 2; i < 8; ++i) counters[i] = 0u;
    }
}

// pair_offset[p] = first emission index of primitive p
__global__ __launch_bounds__(256) void k_pair_offsets(const uint32_t *order, const uint64_t *off, int64_t n,
                                                      uint32_t *pair_offset)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint64_t o = off[r];
    pair_offset[order[r]] = o > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)o;
}

// Primitives in depth order (one per thread, the tests spread over the wave):
// emits the pairs of the tiles of each rectangle that pass the conic test,
// row-major, at the primitive's offset.  The value of a pair is its emission
// index (EMIT_INDEX, with emit_prim[e] = its primitive, for the emission map)
// or directly its primitive.  The decisions are those the preprocess counted
// with the same test.
// Block tags of the emitted pairs, in emission order (a primitive's pairs
// are consecutive, so its record words are read once per run of pairs): bits
// tag_shift .. tag_shift + 3 of a pair's tile id are set for the 8 x 8 blocks
// of the tile the forward will visit the pair for, where the pixel rectangle
// meets the block and so does the pre-test conic (conic_meets_block, the
// forward's own per-batch filter).  The tile sort looks only at the bits
// below tag_shift, so the tags ride along to the ranges pass, which counts
// them per block and strips them.
__global__ __launch_bounds__(256) void k_tag_blocks(uint32_t *keys, const uint32_t *prim_of, Count cnt,
                                                    const float4 *__restrict__ recs, int32_t tiles_x,
                                                    uint32_t tag_shift)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt.get()) return;
    const uint32_t t = keys[i];
    const float4 *rec = recs + (size_t)prim_of[i] * 8;
    const int4 r = *reinterpret_cast<const int4 *>(rec);  // x0, x1, y0, y1
    const int tx = (int)(t % (uint32_t)tiles_x), ty = (int)(t / (uint32_t)tiles_x);
    uint32_t m = 0u;  // blocks the pixel rectangle meets
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int wx0 = tx * TILE + (k & 1) * 8, wy0 = ty * TILE + (k >> 1) * 8;
        m |= (r.y < wx0 || r.x > wx0 + 7 || r.w < wy0 || r.z > wy0 + 7) ? 0u : 1u << k;
    }
    if (m) m &= conic_meets_blocks4(rec, tx * TILE, ty * TILE);
    keys[i] = t | (m << tag_shift);
}

template <bool EMIT_INDEX>
__global__ __launch_bounds__(256) void k_emit(const uint32_t *order, const uint64_t *off, const int32_t *rect,
                                              const double *conic, int64_t n, qgs_camera cam, int32_t tiles_x,
                                              const uint32_t *counters, uint32_t *out_tile, uint32_t *out_emit,
                                              uint32_t *emit_prim, const double *frame, uint32_t *out_dkey,
                                              float near_plane)
{
    __shared__ ConicLane s_cl[64];
    if (counters[1]) return;  // overflow: the same for every thread
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    ConicLane cl = {};
    if (r < n) {
        const uint64_t base = off[r], cnt = off[r + 1] - base;
        if (cnt > 0) {
            const uint32_t p = order[r];
            const int32_t *rc = rect + 4 * (size_t)p;
            const double *C = conic + 8 * (size_t)p;
            for (int i = 0; i < 6; ++i) cl.C[i] = C[i];
            cl.cok = C[6] != 0.0 ? 1u : 0u;
            if (cl.cok) conic_center(cl.C, cl.mx, cl.my, cl.ia, cl.ic);
            // the counting pass's decisions for a rectangle of at most 64 tiles
            cl.mask = reinterpret_cast<const uint64_t *>(C)[7];
            if ((uint64_t)(rc[2] - rc[0] + 1) * (uint64_t)(rc[3] - rc[1] + 1) <= 64u) cl.cok |= 2u;
            cl.base = base;
            cl.cnt = (uint32_t)cnt;
            cl.prim = p;
            cl.tx0 = rc[0];
            cl.ty0 = rc[1];
            cl.nx = rc[2] - rc[0] + 1;
            cl.ny = rc[3] - rc[1] + 1;
        }
    }
    (void)wave_conic_tiles<true, EMIT_INDEX>(s_cl + (threadIdx.x & ~63u), cl, cam, tiles_x, out_tile, out_emit,
                                             emit_prim, frame, out_dkey, (double)near_plane);
}

// tile-depth lists: after the depth passes the values are emission indices;
// fetch each pair's tile as the key of the tile passes
__global__ __launch_bounds__(256) void k_gather_tile_keys(const uint32_t *tile_by_emit, const uint32_t *vals, Count cnt,
                                                          uint32_t *keys_out, uint32_t *vals_out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t n = cnt.get();
    if (i >= n) return;
    const uint32_t e = vals[i];
    if (e >= n) return;  // cannot happen for lists built here
    keys_out[i] = tile_by_emit[e];
    vals_out[i] = e;
}

// After the sort the values are emission indices: replace them by primitive
// ids and record where each emitted pair landed.
__global__ __launch_bounds__(256) void k_gather_prims(const uint32_t *emit_prim, Count cnt, uint32_t *pair_prim,
                                                      uint32_t *emit_to_sorted)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t n = cnt.get();
    if (i >= n) return;
    const uint32_t e = pair_prim[i];
    if (e >= n) return;  // cannot happen for lists built here
    pair_prim[i] = emit_prim[e];
    if (emit_to_sorted) emit_to_sorted[e] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, uint32_t v, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Each tile's range in the sorted lists, one wave per 256 consecutive pairs
// (64 at a time).  With tag_shift > 0 the tile ids still carry the emission's
// block tags (bits tag_shift .. tag_shift + 3): they are stripped here, and
// each wave adds its pairs' tags per (tile, block) into blk[4 t + k], holding
// the counts of its current tile until the tile changes (so a long list costs
// four atomics per 256 pairs).
__global__ __launch_bounds__(256) void k_ranges(uint32_t *tile, Count cnt, uint32_t *ranges, uint32_t ntiles,
                                                uint32_t tag_shift, uint32_t *blk)
{
    const uint64_t n = cnt.get();
    const int lane = threadIdx.x & 63;
    const uint64_t base = ((uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6)) * 256u;
    const uint32_t low = tag_shift ? (1u << tag_shift) - 1u : 0xFFFFFFFFu;
    uint32_t pend_t = 0xFFFFFFFFu, pend[4] = {0u, 0u, 0u, 0u};
    auto flush = [&]() {
        if (pend_t == 0xFFFFFFFFu) return;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (lane == 0 && pend[k]) atomicAdd(blk + 4 * (uint64_t)pend_t + k, pend[k]);
    };
    for (int j = 0; j < 4; ++j) {
        if (base + 64u * (uint64_t)j >= n) break;  // whole wave
        const uint64_t i = base + 64u * (uint64_t)j + (uint64_t)lane;
        const uint32_t key = i < n ? tile[i] : 0u;
        const uint32_t t = key & low;
        const bool in = i < n && t < ntiles;  // t < ntiles always holds for lists built here
        if (in) {
            if (i == 0 || (tile[i - 1] & low) != t) ranges[2 * (uint64_t)t] = (uint32_t)i;
            if (i == n - 1 || (tile[i + 1] & low) != t) ranges[2 * (uint64_t)t + 1] = (uint32_t)(i + 1);
        }
        if (!tag_shift) continue;  // uniform
        // (neighbours may read a stripped or an unstripped id: both mask to t)
        if (i < n) tile[i] = t;
        uint64_t todo = __ballot(in);
        while (todo != 0ull) {
            const int l0 = __builtin_ctzll(todo);
            const uint32_t t0 = (uint32_t)__builtin_amdgcn_readlane((int)t, l0);
            const bool mine = in && t == t0;
            todo &= ~__ballot(mine);
            if (t0 != pend_t) {
                flush();
                pend_t = t0;
                pend[0] = pend[1] = pend[2] = pend[3] = 0u;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) pend[k] += (uint32_t)__popcll(__ballot(mine && ((key >> (tag_shift + k)) & 1u)));
        }
    }
    if (tag_shift) flush();
}

// Tiles in decreasing order of cost: the rasterizer's workgroups take tiles in
// this order, so that the costliest start first and the ones that start last
// are the cheapest (longest-processing-time-first order).  The cost is cost[t],
// the largest of cost[4 t .. 4 t + 3] (max4: per-block costs), or, with no
// cost array, the tile's list length.  Counting sort over 4096
// cost classes: one per value below 2048, then classes 16 wide up to 34800
// (higher costs share the top class); order inside a class is arbitrary.
constexpr int TO_CLASSES = 4096;
__device__ inline uint32_t cost_class(uint32_t c)
{
    uint32_t b = c < 2048u ? c : 2048u + ((c - 2048u) >> 4);
    b = b < (uint32_t)TO_CLASSES - 1u ? b : (uint32_t)TO_CLASSES - 1u;
    return (uint32_t)TO_CLASSES - 1u - b;  // costliest first
}

__global__ __launch_bounds__(1024) void k_tile_order(const uint32_t *ranges, const uint32_t *cost, uint32_t ntiles,
                                                     uint32_t *order, bool max4)
{
    auto tile_cost = [&](uint32_t t) -> uint32_t {
        if (!cost) return ranges[2 * t + 1] - ranges[2 * t];
        if (!max4) return cost[t];
        const uint4 v = reinterpret_cast<const uint4 *>(cost)[t];
        const uint32_t m = v.x > v.y ? v.x : v.y, m2 = v.z > v.w ? v.z : v.w;
        return m > m2 ? m : m2;
    };
    __shared__ uint32_t cnt[TO_CLASSES];
    __shared__ uint32_t s_w[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < TO_CLASSES; i += 1024) cnt[i] = 0;
    __syncthreads();
    for (uint32_t t = tid; t < ntiles; t += blockDim.x) atomicAdd(&cnt[cost_class(tile_cost(t))], 1u);
    __syncthreads();
    // exclusive scan of the class counts: thread t owns classes 4t .. 4t + 3
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = cnt[4 * tid + k];
        sum += v[k];
    }
    const uint32_t inc = wave_incl_scan(sum, lane);
    if (lane == 63) s_w[wave] = inc;
    __syncthreads();
    uint32_t run = inc - sum;
    for (int w = 0; w < wave; ++w) run += s_w[w];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        cnt[4 * tid + k] = run;
        run += v[k];
    }
    __syncthreads();
    for (uint32_t t = tid; t < ntiles; t += blockDim.x) order[atomicAdd(&cnt[cost_class(tile_cost(t))], 1u)] = t;
}

hipError_t launch_tile_order(const uint32_t *ranges, const uint32_t *cost, uint32_t ntiles, uint32_t *order,
                             hipStream_t stream, bool max4)
{
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), 0, stream, ranges, cost, ntiles, order, max4);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, uint64_t n, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, stream, p, v, n);
    return hipGetLastError();
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

SortWorkspace sort_workspace_layout(void *base, int64_t n, uint64_t capacity, uint64_t ntiles)
{
    SortWorkspace w{};
    const uint64_t nn = (uint64_t)(n > 0 ? n : 1);
    const uint64_t nb_depth = cdiv(nn, (uint64_t)RS_THREADS * RS_ITEMS_DEPTH);
    const uint64_t nb_tile = cdiv(capacity > 0 ? capacity : 1, (uint64_t)RS_THREADS * RS_ITEMS_TILE);
    const uint64_t nbmax = (nb_depth > nb_tile ? nb_depth : nb_tile) + 1;
    const uint64_t nparts = cdiv(nn + 1, SCAN_CHUNK) + cdiv(256 * nbmax, SCAN_CHUNK) + 64;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return base ? (void *)((char *)base + at) : nullptr;
    };
    w.dkA = (uint32_t *)take(4 * nn);
    w.dvA = (uint32_t *)take(4 * nn);
    w.dkB = (uint32_t *)take(4 * nn);
    w.dvB = (uint32_t *)take(4 * nn);
    w.off = (uint64_t *)take(8 * (nn + 1));
    w.part = (uint64_t *)take(8 * nparts);
    w.hist = (uint32_t *)take(4 * 256 * nbmax);
    w.tileT = (uint32_t *)take(4 * (capacity > 0 ? capacity : 1));
    w.primT = (uint32_t *)take(4 * (capacity > 0 ? capacity : 1));
    w.emit_prim = (uint32_t *)take(4 * (capacity > 0 ? capacity : 1));
    w.dkeyT = (uint32_t *)take(4 * (capacity > 0 ? capacity : 1));
    w.blk_cost = (uint32_t *)take(16 * (ntiles > 0 ? ntiles : 1));
    w.bytes = o;
    return w;
}

hipError_t bin_sort_phase1(const BinSortArgs &a, const SortWorkspace &ws, hipStream_t stream)
{
    const int64_t n = a.n;
    const unsigned pb = (unsigned)cdiv((uint64_t)(n > 0 ? n : 1), 256);
    if (n > 0) {
        hipLaunchKernelGGL(k_depth_init, dim3(pb), dim3(256), 0, stream, a.depth_key, a.tiles, n, ws.dkA, ws.dvA);
        // 4 stable passes over the 32-bit depth keys: A -> B -> A -> B -> A
        Count c{nullptr, (uint64_t)n};
        hipError_t e;
        e = radix_pass<RS_ITEMS_DEPTH>(ws.dkA, ws.dvA, ws.dkB, ws.dvB, c, n, 0, ws, stream);
        if (e != hipSuccess) return e;
        e = radix_pass<RS_ITEMS_DEPTH>(ws.dkB, ws.dvB, ws.dkA, ws.dvA, c, n, 8, ws, stream);
        if (e != hipSuccess) return e;
        e = radix_pass<RS_ITEMS_DEPTH>(ws.dkA, ws.dvA, ws.dkB, ws.dvB, c, n, 16, ws, stream);
        if (e != hipSuccess) return e;
        e = radix_pass<RS_ITEMS_DEPTH>(ws.dkB, ws.dvB, ws.dkA, ws.dvA, c, n, 24, ws, stream);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_gather_tiles, dim3(pb), dim3(256), 0, stream, ws.dvA, a.tiles, n, ws.off);
        e = device_excl_scan<uint64_t>(ws.off, ws.off, (uint64_t)n, ws.part, ws.off + n, stream);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_pair_offsets, dim3(pb), dim3(256), 0, stream, ws.dvA, ws.off, n, a.pair_offset);
    } else {
        hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(ws.off), 0u, 2, stream);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_set_counters, dim3(1), dim3(64), 0, stream, ws.off + (n > 0 ? n : 0), a.capacity,
                       a.counters);
    return hipGetLastError();
}

static hipError_t emit_sort_ranges(const BinSortArgs &a, const SortWorkspace &ws, uint64_t bound, int passes,
                                   uint64_t ntiles, uint32_t tag_shift, hipStream_t stream);

hipError_t bin_sort_phase2(const BinSortArgs &a, const SortWorkspace &ws, uint64_t bound, hipStream_t stream)
{
    const int64_t n = a.n;
    const uint64_t ntiles = (uint64_t)a.tiles_x * (uint64_t)a.tiles_y;
    int bits = 1;
    while ((1ull << bits) < ntiles) ++bits;
    const int passes = (bits + 7) / 8;
    hipError_t e = launch_fill_u32(a.ranges, 0u, 2 * ntiles, stream);
    if (e != hipSuccess) return e;
    // the tiles' order by their forward work when the records and room for
    // the block counts are there (centre-depth lists; the tags need 4 bits
    // above the tile bits the sort passes look at), else by list length
    const bool tags = a.tile_order && a.records && ws.blk_cost && !a.frame && passes < 4;
    if (tags) e = launch_fill_u32(ws.blk_cost, 0u, 4 * ntiles, stream);
    if (e != hipSuccess) return e;
    if (bound > a.capacity) bound = a.capacity;
    if (n > 0 && bound > 0) e = emit_sort_ranges(a, ws, bound, passes, ntiles, tags ? 8u * passes : 0u, stream);
    if (e != hipSuccess) return e;
    // the tile order is written on every path: the rasterizer reads it for
    // every workgroup, also when there are no pairs
    if (a.tile_order)
        e = launch_tile_order(a.ranges, tags ? ws.blk_cost : nullptr, (uint32_t)ntiles, a.tile_order, stream, tags);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

static hipError_t emit_sort_ranges(const BinSortArgs &a, const SortWorkspace &ws, uint64_t bound, int passes,
                                   uint64_t ntiles, uint32_t tag_shift, hipStream_t stream)
{
    const float4 *recs = reinterpret_cast<const float4 *>(a.records);
    const int64_t n = a.n;
    hipError_t e = hipSuccess;
    const bool emit_map = a.emit_to_sorted != nullptr;
    Count c{a.counters, bound};
    const unsigned eb = (unsigned)cdiv((uint64_t)n, 64), gb = (unsigned)cdiv(bound, 256);
    uint32_t *ki, *vi;
    bool values_are_emission = emit_map;
    if (a.frame) {
        // per-tile depth keys: emission writes (tile, depth key, emission
        // index, primitive) by emission index; four stable passes over the
        // depth key, then the tile passes on the gathered tiles (ties keep the
        // emission order: centre depth, then primitive)
        hipLaunchKernelGGL(k_emit<true>, dim3(eb), dim3(64), 0, stream, ws.dvA, ws.off, a.rect, a.conic, n, a.cam,
                           a.tiles_x, a.counters, ws.tileT, ws.primT, ws.emit_prim, a.frame, ws.dkeyT,
                           a.near_plane);
        uint32_t *dk = ws.dkeyT, *dv = ws.primT, *ak = a.pair_tile, *av = a.pair_prim;
        for (int pass = 0; pass < 4; ++pass) {
            e = radix_pass<RS_ITEMS_TILE>(dk, dv, ak, av, c, bound, 8 * pass, ws, stream);
            if (e != hipSuccess) return e;
            uint32_t *tk = dk, *tv = dv;
            dk = ak; dv = av; ak = tk; av = tv;
        }
        // (dk, dv) = (ws.dkeyT, ws.primT): sorted by depth key, values are
        // emission indices; start the tile passes where they end in the lists
        ki = (passes % 2 == 0) ? a.pair_tile : ws.dkeyT;
        vi = (passes % 2 == 0) ? a.pair_prim : ws.primT;
        hipLaunchKernelGGL(k_gather_tile_keys, dim3(gb), dim3(256), 0, stream, (const uint32_t *)ws.tileT,
                           (const uint32_t *)ws.primT, c, ki, vi);
        values_are_emission = true;
    } else {
        // emit into the buffers that make the final pass land in the caller's lists
        ki = (passes % 2 == 0) ? a.pair_tile : ws.tileT;
        vi = (passes % 2 == 0) ? a.pair_prim : ws.primT;
        if (emit_map)
            hipLaunchKernelGGL(k_emit<true>, dim3(eb), dim3(64), 0, stream, ws.dvA, ws.off, a.rect, a.conic, n,
                               a.cam, a.tiles_x, a.counters, ki, vi, ws.emit_prim, (const double *)nullptr,
                               (uint32_t *)nullptr, 0.0f);
        else
            hipLaunchKernelGGL(k_emit<false>, dim3(eb), dim3(64), 0, stream, ws.dvA, ws.off, a.rect, a.conic, n,
                               a.cam, a.tiles_x, a.counters, ki, vi, ws.emit_prim, (const double *)nullptr,
                               (uint32_t *)nullptr, 0.0f);
        if (tag_shift)
            hipLaunchKernelGGL(k_tag_blocks, dim3(gb), dim3(256), 0, stream, ki,
                               emit_map ? (const uint32_t *)ws.emit_prim : (const uint32_t *)vi, c, recs, a.tiles_x,
                               tag_shift);
    }
    for (int pass = 0; pass < passes; ++pass) {
        uint32_t *ko = (ki == a.pair_tile) ? (a.frame ? ws.dkeyT : ws.tileT) : a.pair_tile;
        uint32_t *vo = (vi == a.pair_prim) ? ws.primT : a.pair_prim;
        e = radix_pass<RS_ITEMS_TILE>(ki, vi, ko, vo, c, bound, 8 * pass, ws, stream);
        if (e != hipSuccess) return e;
        ki = ko;
        vi = vo;
    }
    if (values_are_emission)
        hipLaunchKernelGGL(k_gather_prims, dim3(gb), dim3(256), 0, stream, (const uint32_t *)ws.emit_prim, c,
                           a.pair_prim, a.emit_to_sorted);
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)cdiv(bound, 1024)), dim3(256), 0, stream, a.pair_tile, c, a.ranges,
                       (uint32_t)ntiles, tag_shift, ws.blk_cost);
    return hipGetLastError();
}

}  // namespace qgs
