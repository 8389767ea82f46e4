// Screen-space conic test of a tile, shared by the preprocess (tile counts)
// and the emission kernel (tile lists), so that both take the same decisions.
//
// The conic C = {c00, c01, c11, c02, c12, c22} is the image of an ellipsoid
// enclosing a primitive's support in normalised camera coordinates
// (x, y) = ((u - cx) / fx, (v - cy) / fy):
//     f(x, y) = c00 x^2 + 2 c01 x y + c11 y^2 + 2 c02 x + 2 c12 y + c22 <= 0
// inside.  f is a convex quadratic on the image plane, so the tile's rectangle
// of pixel centres (widened by 1/64 pixel) meets the interior iff f's
// minimiser lies in the rectangle or the minimum of f along one of the four
// edges is <= 0.  FP64, fixed operation order, no contraction.  Divisions are
// taken once per primitive (1/det, 1/a, 1/c) and once per camera (1/fx,
// 1/fy); the per-tile test multiplies.
#pragma once
#include <hip/hip_runtime.h>

#include "qgs.h"

namespace qgs {

__device__ inline double conic_eval(const double *C, double x, double y)
{
#pragma clang fp contract(off)
    return ((C[0] * x + 2.0 * C[1] * y + 2.0 * C[3]) * x + (C[2] * y + 2.0 * C[4]) * y) + C[5];
}

__device__ inline double clamp_d(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Per-primitive constants of the test: the conic's centre (minimiser of f)
// and the reciprocals 1/a, 1/c of the edge minimisers.
__device__ inline void conic_center(const double *C, double &mx, double &my, double &ia, double &ic)
{
#pragma clang fp contract(off)
    const double a = C[0], b = C[1], c = C[2], d = C[3], e = C[4];
    const double idet = 1.0 / (a * c - b * b);
    mx = (b * e - c * d) * idet;
    my = (b * d - a * e) * idet;
    ia = 1.0 / a;
    ic = 1.0 / c;
}

// ifx = 1/fx, ify = 1/fy
__device__ inline bool conic_tile_hit(const double *C, double mx, double my, double ia, double ic, int tx, int ty,
                                      const qgs_camera &cam, double ifx, double ify)
{
#pragma clang fp contract(off)
    const double cx = cam.cx, cy = cam.cy;
    const double pad_px = 1.0 / 64.0;
    const int ux0 = tx * 16, ux1 = (tx * 16 + 15) < cam.width - 1 ? tx * 16 + 15 : cam.width - 1;
    const int vy0 = ty * 16, vy1 = (ty * 16 + 15) < cam.height - 1 ? ty * 16 + 15 : cam.height - 1;
    const double x0 = ((((double)ux0 + 0.5) - pad_px) - cx) * ifx, x1 = ((((double)ux1 + 0.5) + pad_px) - cx) * ifx;
    const double y0 = ((((double)vy0 + 0.5) - pad_px) - cy) * ify, y1 = ((((double)vy1 + 0.5) + pad_px) - cy) * ify;
    const double b = C[1], d = C[3], e = C[4];
    if (mx >= x0 && mx <= x1 && my >= y0 && my <= y1) return true;
    const double xs[2] = {x0, x1}, ys[2] = {y0, y1};
    for (int k = 0; k < 2; ++k) {
        const double y = clamp_d(-(b * xs[k] + e) * ic, y0, y1);
        if (conic_eval(C, xs[k], y) <= 0.0) return true;
        const double x = clamp_d(-(b * ys[k] + d) * ia, x0, x1);
        if (conic_eval(C, x, ys[k]) <= 0.0) return true;
    }
    return false;
}

// Per-tile sort depth (supplement, per-tile sorting): the camera depth at which
// the ray through tile (tx, ty)'s pixel nearest the projected vertex meets the
// paraboloid; the smallest root beyond the near plane, or the centre depth if
// there is none.  F: the primitive's frame (c_cam, Rc, projected vertex,
// lambda_1, lambda_2).  FP64, fixed operation order, no contraction; returns
// the bits of the depth rounded to FP32.
__device__ inline uint32_t tile_depth_bits(const double *F, int tx, int ty, const qgs_camera &cam, double near_d)
{
#pragma clang fp contract(off)
    const double fx = cam.fx, fy = cam.fy, cx = cam.cx, cy = cam.cy;
    const int ux0 = tx * 16, ux1 = (tx * 16 + 15) < cam.width - 1 ? tx * 16 + 15 : cam.width - 1;
    const int vy0 = ty * 16, vy1 = (ty * 16 + 15) < cam.height - 1 ? ty * 16 + 15 : cam.height - 1;
    const double fu = floor(F[12]), fv = floor(F[13]);
    const int px = fu < (double)ux0 ? ux0 : (fu > (double)ux1 ? ux1 : (int)fu);
    const int py = fv < (double)vy0 ? vy0 : (fv > (double)vy1 ? vy1 : (int)fv);
    const double dx = (((double)px + 0.5) - cx) / fx, dy = (((double)py + 0.5) - cy) / fy;
    double o[3], e[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        o[k] = -((F[3 + k] * F[0] + F[6 + k] * F[1]) + F[9 + k] * F[2]);
        e[k] = (F[3 + k] * dx + F[6 + k] * dy) + F[9 + k];
    }
    const double l1 = F[14], l2 = F[15];
    const double A = (l1 * e[0]) * e[0] + (l2 * e[1]) * e[1];
    const double B = 2.0 * ((l1 * o[0]) * e[0] + (l2 * o[1]) * e[1]) - e[2];
    const double C = ((l1 * o[0]) * o[0] + (l2 * o[1]) * o[1]) - o[2];
    double r0 = 0.0, r1 = 0.0;
    int nr = 0;
    if (fabs(A) <= 1e-12 * ((e[0] * e[0] + e[1] * e[1]) + e[2] * e[2])) {
        if (B != 0.0) {
            r0 = -C / B;
            nr = 1;
        }
    } else {
        const double D = B * B - 4.0 * (A * C);
        if (D >= 0.0) {
            const double sq = sqrt(D);
            const double q = -0.5 * (B + (B >= 0.0 ? sq : -sq));
            if (q != 0.0) {
                r0 = q / A;
                r1 = C / q;
                nr = 2;
            }
        }
    }
    double z = F[2];
    bool found = false;
    if (nr >= 1 && r0 > near_d) {
        z = r0;
        found = true;
    }
    if (nr >= 2 && r1 > near_d && (!found || r1 < z)) z = r1;
    return __float_as_uint((float)z);
}

// ---------------------------------------------------------------------------
// Wave-cooperative tile tests.  A primitive's candidate tiles are the tiles of
// its rectangle, row-major.  Rather than one thread looping over its own
// primitive's candidates (a wave then waits for its largest primitive), the
// wave's candidates are numbered consecutively (an inclusive scan of the
// per-lane counts) and processed 64 at a time, candidate c on lane c mod 64.
// Each lane stages its primitive in LDS; a candidate finds its owner by binary
// search over the scan.  The decisions are those of conic_tile_hit, so counts
// and emitted tiles are the same as a per-primitive loop's.  The counting pass
// also returns, for a rectangle of at most 64 tiles, its decisions as a bit
// mask (bit k: the k-th tile, row-major); the emission pass reads a lane's
// decisions from that mask when it has one (cok bit 1) instead of testing
// again, so both passes take the same decisions.
// ---------------------------------------------------------------------------
struct ConicLane {
    double C[6];
    double mx, my, ia, ic;
    uint64_t base;               // first emission index (emission only)
    int32_t tx0, ty0, nx, ny;    // tile rectangle, nx * ny candidates (0: none)
    uint32_t excl, cnt, prim;
    uint32_t cok;                // bit 0: the conic bounds the support; bit 1: `mask` holds the decisions
    uint64_t mask;               // decisions of the counting pass (cok bit 1)
};

__device__ inline uint32_t wave_incl_scan_u32(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// number of lanes whose inclusive count is <= c (the owner of candidate c);
// every lane of the wave must call it
__device__ inline int wave_owner(uint32_t incl, uint32_t c)
{
    int o = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
        if (__shfl(incl, o + step - 1, 64) <= c) o += step;
    return o;
}

// bits [lo, hi) of a 64-bit lane mask, clamped to [0, 64)
__device__ inline uint64_t lane_range_mask(int64_t lo, int64_t hi)
{
    lo = lo < 0 ? 0 : (lo > 64 ? 64 : lo);
    hi = hi < 0 ? 0 : (hi > 64 ? 64 : hi);
    if (hi <= lo) return 0ull;
    const uint64_t below_hi = hi >= 64 ? ~0ull : ((1ull << hi) - 1ull);
    const uint64_t below_lo = (1ull << lo) - 1ull;
    return below_hi & ~below_lo;
}

// Counts (and with EMIT writes) the tiles of each lane's rectangle that pass
// the conic test (every tile when cok == 0).  s_wave: this wave's 64 LDS
// entries.  Must be reached by every thread of the workgroup (one barrier; the
// kernels run one-wave workgroups).
// EMIT: a hit of primitive `prim` with rank k among its hits goes to emission
// index base + k (if k < cnt): out_tile = tile id, and out_emit = the index
// with emit_prim = prim (EMIT_INDEX), or out_emit = prim.
// mask_out (counting pass, may be NULL): the lane's decisions as a bit mask
// when its rectangle has at most 64 tiles, else 0.
template <bool EMIT, bool EMIT_INDEX = true>
__device__ inline uint32_t wave_conic_tiles(ConicLane *s_wave, const ConicLane &me, const qgs_camera &cam,
                                            int tiles_x, uint32_t *out_tile, uint32_t *out_emit, uint32_t *emit_prim,
                                            const double *frame = nullptr, uint32_t *out_dkey = nullptr,
                                            double near_d = 0.0, uint64_t *mask_out = nullptr)
{
    const int lane = threadIdx.x & 63;
    const uint32_t R = (me.nx > 0 && me.ny > 0) ? (uint32_t)me.nx * (uint32_t)me.ny : 0u;
    const double ifx = 1.0 / (double)cam.fx, ify = 1.0 / (double)cam.fy;
    const uint32_t incl = wave_incl_scan_u32(R), excl = incl - R;
    const uint32_t total = __shfl(incl, 63, 64);
    s_wave[lane] = me;
    s_wave[lane].excl = excl;
    if (!EMIT) s_wave[lane].mask = 0ull;
    __syncthreads();
    uint32_t hits = 0;
    for (uint32_t base = 0; base < total; base += 64) {
        const uint32_t c = base + (uint32_t)lane;
        const int o = wave_owner(incl, c);
        const uint32_t run_o = EMIT ? __shfl(hits, o & 63, 64) : 0u;
        bool hit = false;
        int tx = 0, ty = 0;
        if (c < total) {
            const ConicLane &q = s_wave[o];
            const uint32_t loc = c - q.excl;
            tx = q.tx0 + (int)(loc % (uint32_t)q.nx);
            ty = q.ty0 + (int)(loc / (uint32_t)q.nx);
            if (EMIT && (q.cok & 2u))
                hit = ((q.mask >> loc) & 1ull) != 0ull;
            else
                hit = (q.cok & 1u) == 0u || conic_tile_hit(q.C, q.mx, q.my, q.ia, q.ic, tx, ty, cam, ifx, ify);
        }
        if (!EMIT && mask_out && hit) {
            // the owner's decision bit, in its staged copy (LDS atomic)
            const ConicLane &q = s_wave[o];
            const uint32_t loc = c - q.excl;
            if ((uint32_t)q.nx * (uint32_t)q.ny <= 64u) atomicOr(&s_wave[o].mask, 1ull << loc);
        }
        const uint64_t bal = __ballot(hit);
        if (EMIT && hit) {
            const ConicLane &q = s_wave[o];
            const uint32_t k = run_o + (uint32_t)__popcll(bal & lane_range_mask((int64_t)q.excl - (int64_t)base, lane));
            if (k < q.cnt) {
                const uint64_t e = q.base + k;
                out_tile[e] = (uint32_t)(ty * tiles_x + tx);
                if (out_dkey) out_dkey[e] = tile_depth_bits(frame + 16 * (size_t)q.prim, tx, ty, cam, near_d);
                if (EMIT_INDEX) {
                    out_emit[e] = (uint32_t)e;
                    emit_prim[e] = q.prim;
                } else {
                    out_emit[e] = q.prim;
                }
            }
        }
        hits += (uint32_t)__popcll(bal & lane_range_mask((int64_t)excl - (int64_t)base, (int64_t)incl - (int64_t)base));
    }
    if (mask_out) *mask_out = R <= 64u ? s_wave[lane].mask : 0ull;
    return hits;
}

}  // namespace qgs
