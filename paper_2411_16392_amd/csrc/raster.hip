// Tile rasterizer, forward and backward.
//
// Four one-wave workgroups per 16 x 16 tile (a finished wave's slot takes new
// work at once; with four-wave workgroups about a fifth of the wave slots sat
// empty in mid-kernel); the forward gives a tile's four workgroups ids 8
// apart, so they run on one XCD and share its L2; wave w owns the 8 x 8
// block (w & 1, w >> 1) of the tile, lane l the pixel (l & 7, l >> 3) in it.
// The resort kernels run the same way.  The waves
// walk the tile's list independently, without LDS or barriers: 64 entries at
// a time, lane i fetches entry b + i's primitive id and pixel rectangle (one
// batch ahead), a ballot keeps the entries whose rectangle
// meets the wave's block, and only those are visited; the forwards also drop
// entries whose pre-test conic misses the block (conic_meets_block, one test
// per lane and batch instead of a wave step per entry).  A visited entry's
// 128-byte record is read with a wave-uniform address, i.e. by scalar loads
// into scalar registers, once per wave.  Each lane first applies the conic
// pre-test (no per-lane rectangle test: it removed almost nothing the conic
// keeps); the intersection runs only if some lane passes it.
//
// Forward (Eq. 1, compositing front to back): a wave stops once every lane is
// done (ballot).  It can also mark, per block and 64-entry batch, the entries
// some pixel blended (the replay bitmap).
// Backward (supplement, back-to-front adjoint): each pixel starts at its last
// blended entry, recovers T_i = T_{i+1} / (1 - alpha_i), and keeps the suffix
// sum S_i = sum_{j>i} w_j X_j + T_final bg, so dX/dalpha_i = T_i X_i - S_i /
// (1 - alpha_i).  With the replay bitmap a wave visits only the marked
// entries (the others change nothing).  A visited entry's 14 per-primitive
// gradient fields are reduce-scattered over the wave and added to global
// memory by 14 lanes with one atomic instruction; the deterministic variant
// stores them into the pair's slot for the wave and a second pass sums the
// slots in a fixed order.  The gradient arithmetic, which takes no decision,
// may contract into fma; everything that decides (hit, root, cut-off,
// alpha) is evaluated without contraction, identically in both passes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qgs_device.hpp"
#include "qgs_internal.hpp"

#pragma clang fp contract(off)

// Minimum number of waves per SIMD the compiler is asked to fit (0: no request).
// For the forward, 7 makes the compiler keep the scalar registers to 94, which
// lets 8 waves share a SIMD (about 100 would allow 7); asking for 8 costs
// more instructions than the occupancy gains.  For the backward, 7 holds it
// to 72 vector registers (7 waves per SIMD) without spills; the geometry
// variant needs 88 and is left to the compiler (5).
#ifndef QGS_FWD_MIN_WAVES
#define QGS_FWD_MIN_WAVES 7
#endif
#ifndef QGS_BWD_MIN_WAVES
#define QGS_BWD_MIN_WAVES 7
#endif
#ifndef QGS_BWD_GEO_MIN_WAVES
#define QGS_BWD_GEO_MIN_WAVES 5
#endif

namespace qgs {

template <int CTRL, int ROW_MASK = 0xF>
__device__ inline float dpp_f(float v)
{
    // lanes whose source is outside the row read 0; rows outside ROW_MASK keep 0
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, true));
}

// Wave totals of the NGRAD gradient fields over the lanes with `mine` set,
// transposed through LDS: s_red is the wave's block of 16 rows of RED_ROW
// floats, zero on entry and again on return (rows NGRAD.. stay zero).  Each
// such lane writes field f to row f, column lane; lane l then sums the 16
// values of row l / 4 in columns l % 4, l % 4 + 4, ..., l % 4 + 60 and the
// quad adds its four partial sums, so lane 4 f (f < NGRAD) ends with the total
// of field f.  Fixed order, so the result is reproducible.  The row pitch of
// 68 words puts the rows 4 banks apart: a half-wave of the column reads hits
// 32 different banks.  Called by the whole wave (its workgroup), so the
// barriers only order its LDS accesses; about a third of the VALU work of a
// shuffle-based reduce-scatter.
constexpr int RED_ROW = 68;
__device__ inline float wave_reduce_lds(float *s_red, const float (&gr)[NGRAD], bool mine)
{
    const int lane = threadIdx.x & 63;
    if (mine) {
#pragma unroll
        for (int f = 0; f < NGRAD; ++f) s_red[f * RED_ROW + lane] = gr[f];
    }
    __syncthreads();
    const float *src = s_red + (lane >> 2) * RED_ROW + (lane & 3);
    float v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = src[4 * k];
#pragma unroll
    for (int f = 0; f < NGRAD; ++f) s_red[f * RED_ROW + lane] = 0.0f;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] += v[k + 8];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] += v[k + 4];
    v[0] += v[2];
    v[1] += v[3];
    float tot = v[0] + v[1];
    tot += dpp_f<0x4E>(tot);  // quad_perm [2, 3, 0, 1]
    tot += dpp_f<0xB1>(tot);  // quad_perm [1, 0, 3, 2]
    return tot;
}

// zeroes the wave's reduction block (all 16 rows)
__device__ inline void clear_reduce_lds(float *s_red)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int f = 0; f < 16; ++f) s_red[f * RED_ROW + lane] = 0.0f;
}

// Words 4..31 of primitive pj's record (everything past the rectangle) into
// rw[4..31], fetched in one round of scalar loads before any is used: the
// empty asm makes the values live in scalar registers here, so the pre-test,
// the primitive and the colour words then need no further wait (the compiler
// otherwise issues them as three dependent rounds, one per use).
__device__ inline void load_record_words(const float4 *__restrict__ recs, uint32_t pj, float (&rw)[32])
{
    float4 rv[8];
#pragma unroll
    for (int q = 1; q < 8; ++q) rv[q] = recs[(size_t)pj * 8 + q];
#pragma unroll
    for (int q = 1; q < 8; ++q) {
        __asm__ volatile("" : : "s"(rv[q].x), "s"(rv[q].y), "s"(rv[q].z), "s"(rv[q].w));
        rw[4 * q] = rv[q].x;
        rw[4 * q + 1] = rv[q].y;
        rw[4 * q + 2] = rv[q].z;
        rw[4 * q + 3] = rv[q].w;
    }
}

__device__ inline uint32_t wave_max_u32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
// GEO: also the curvature, median-depth and depth-distortion maps.  NRM:
// accumulate depth and normal (off for colour-only rendering).  COUNT: the
// work counters of QGS_COUNT_EVALS (a separate instantiation, so that the
// plain forward carries none of their per-step bookkeeping).
//
// First word of the replay bitmap of 8 x 8 block `wave` of tile `tile`, whose
// list is [start, start + len): tiles take 4 ceil(len / 64) words each from
// word 4 (floor(start / 64) + tile) on, which never overlaps the next tile's
// (its start is at least start + len); at most 4 (capacity / 64 + tiles + 1)
// words in all.
__device__ inline size_t replay_base(uint32_t start, uint32_t len, int tile, int wave)
{
    return 4 * ((size_t)(start >> 6) + (size_t)tile) + (size_t)wave * ((len + 63u) >> 6);
}

// Each wave walks its tile's list on its own, with no LDS and no barrier: the
// list is read 64 entries at a time (lane i fetches entry b + i's primitive id
// two batches ahead and its pixel rectangle one batch ahead), a ballot selects
// the entries whose rectangle and pre-test conic meet the wave's 8 x 8 block,
// and only those are visited.  A
// visited entry's record is read with a wave-uniform address, so it is
// fetched once for the wave (scalar loads) and sits in scalar registers.
// `recs` is a.records again and `replay` o.steps, as restrict arguments: the
// records are never written here, which keeps the scalar loads legal although
// the loop stores replay words.
template <bool GEO, bool NRM, bool COUNT>
#if QGS_FWD_MIN_WAVES > 0
// Launched as one-wave workgroups (4 per tile); BLOCK only bounds the size.
__global__ __launch_bounds__(BLOCK, QGS_FWD_MIN_WAVES) void k_render_fwd(RasterArgs a, RasterParams P, FwdOut o,
                                                                         const float4 *__restrict__ recs,
                                                                         uint64_t *__restrict__ replay)
#else
__global__ __launch_bounds__(BLOCK) void k_render_fwd(RasterArgs a, RasterParams P, FwdOut o,
                                                      const float4 *__restrict__ recs, uint64_t *__restrict__ replay)
#endif
{
    // workgroup ids 32 G + 8 k + x take block k of the tile in position 8 G + x
    // of the order: consecutive ids go to the 8 XCDs in turn, so a tile's four
    // blocks share one XCD (and its L2) and the tiles still start in order
    const uint32_t ntl = (uint32_t)(P.tiles_x * P.tiles_y);
    const uint32_t grp = blockIdx.x >> 5, r32 = blockIdx.x & 31u;
    const uint32_t left = ntl - 8u * grp, mg = left < 8u ? left : 8u;
    const uint32_t slot = mg == 8u ? 8u * grp + (r32 & 7u) : 8u * grp + r32 % mg;
    const uint32_t kblk = mg == 8u ? r32 >> 3 : r32 / mg;
    const int tile = a.tile_order ? (int)a.tile_order[slot] : (int)slot;
    if ((unsigned)tile >= (unsigned)(P.tiles_x * P.tiles_y)) return;  // whole workgroup; cannot happen for lists built here
    const int tx = tile % P.tiles_x, ty = tile / P.tiles_x;
    const int tid = threadIdx.x, lane = tid & 63, wave = (int)kblk;
    const int wx0 = tx * TILE + (wave & 1) * 8, wy0 = ty * TILE + (wave >> 1) * 8;
    const int px = wx0 + (lane & 7), py = wy0 + (lane >> 3);
    const bool inside = px < P.width && py < P.height;
    const uint32_t start = a.ranges[2 * tile], n = a.ranges[2 * tile + 1] - start;
    const PixelRay ray = make_ray(px, py, P);

    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, dep = 0.0f, n0 = 0.0f, n1 = 0.0f, n2 = 0.0f;
    uint32_t last = 0, stop_pos = 0, n_eval = 0, n_blend = 0, w_rect = 0, w_eval = 0, w_blend = 0;
    bool done = !inside;
    // geometry: curvature sum, median depth and its position, and the running
    // sum of weights, mean depth and distortion
    float kk = 0.0f, med = 0.0f, gW = 0.0f, gm = 0.0f, gL = 0.0f;
    uint32_t med_pos = 0;
    // replay bitmap of this block: bit j of word w set when some pixel blended entry 64 w + j
    uint64_t *bm = replay ? replay + replay_base(start, n, tile, wave) : nullptr;
    uint32_t n_words = 0;

    // batch fetch: lane i holds entry b + i's primitive and rectangle
    // primitive ids two batches ahead, rectangles one batch ahead
    uint32_t nxt_pid = 0, nn_pid = 0;
    int4 nxt_rect = make_int4(0, -1, 0, -1);
    if ((uint32_t)lane < n) {
        nxt_pid = a.pair_prim[start + lane];
        nxt_rect = *reinterpret_cast<const int4 *>(recs + (size_t)nxt_pid * 8);
    }
    if (64u + (uint32_t)lane < n) nn_pid = a.pair_prim[start + 64 + lane];
    bool wave_alive = __ballot(!done) != 0ull;
    for (uint32_t b = 0; b < n && wave_alive; b += 64) {
        const uint32_t cur_pid = nxt_pid;
        const int4 cur_rect = nxt_rect;
        // entries whose rectangle and pre-test conic meet the block (the
        // conic test's loads come before the next batch's, so waiting for
        // them leaves those in flight)
        bool rel = b + (uint32_t)lane < n && !(cur_rect.y < wx0 || cur_rect.x > wx0 + 7 ||
                                                 cur_rect.w < wy0 || cur_rect.z > wy0 + 7);
        if (rel) rel = conic_meets_block(recs + (size_t)cur_pid * 8, (float)wx0, (float)wy0);
        nxt_pid = nn_pid;
        if (b + 64 + (uint32_t)lane < n) nxt_rect = *reinterpret_cast<const int4 *>(recs + (size_t)nxt_pid * 8);
        if (b + 128 + (uint32_t)lane < n) nn_pid = a.pair_prim[start + b + 128 + lane];
        uint64_t m = __ballot(rel);
        uint64_t blended = 0ull;
        while (m != 0ull && wave_alive) {
            const int j = __builtin_ctzll(m);
            m &= m - 1ull;
            if (COUNT) ++w_rect;
            const uint32_t pj = (uint32_t)__builtin_amdgcn_readlane((int)cur_pid, j);
            float rw[32];
            load_record_words(recs, pj, rw);
            const float *w = rw;
            float dxp, dyp;
            // bitwise and: the pre-test runs on every lane, with no branch
            const bool lane_on = conic_offsets(w, ray, dxp, dyp) & !done;
            if (__ballot(lane_on) == 0ull) continue;
            if (COUNT) ++w_eval;
            const uint32_t pos1 = b + (uint32_t)j + 1u;
            if (lane_on) {
                Prim p;
                load_prim(w, P, p);
                Hit H;
                if (COUNT) ++n_eval;
                if (ray_hit(p, ray, P, dxp, dyp, H)) {
                    const float G = __expf(-0.5f * H.E);
                    const float alpha = fminf(P.alpha_max, p.op * G);
                    if (alpha >= P.alpha_min) {
                        const float Tn = T * (1.0f - alpha);
                        if (Tn < P.T_eps) {
                            done = true;
                            stop_pos = pos1;
                        } else {
                            const float wgt = alpha * T;
                            const float4 cr = *reinterpret_cast<const float4 *>(w + 24);
                            c0 = __builtin_fmaf(wgt, cr.y, c0);
                            c1 = __builtin_fmaf(wgt, cr.z, c1);
                            c2 = __builtin_fmaf(wgt, cr.w, c2);
                            const float t = (p.Zc + H.s) * ray.enorm;
                            float nl[3], il = 0.0f;
                            if (NRM || GEO) {
                                dep = __builtin_fmaf(wgt, t, dep);
                                const float f = hit_normal(p, H, nl, il);
                                const float wf = wgt * f;
                                n0 = __builtin_fmaf(wf, __builtin_fmaf(p.R[0], nl[0], __builtin_fmaf(p.R[1], nl[1], p.R[2] * nl[2])), n0);
                                n1 = __builtin_fmaf(wf, __builtin_fmaf(p.R[3], nl[0], __builtin_fmaf(p.R[4], nl[1], p.R[5] * nl[2])), n1);
                                n2 = __builtin_fmaf(wf, __builtin_fmaf(p.R[6], nl[0], __builtin_fmaf(p.R[7], nl[1], p.R[8] * nl[2])), n2);
                            }
                            if (GEO) {
                                kk = __builtin_fmaf(wgt, hit_curvature(p, il), kk);
                                if (T > 0.5f && (med_pos == 0u || t > med)) {
                                    med = t;
                                    med_pos = pos1;
                                }
                                // L += w (L / W + W (t - mean)^2); W += w; mean += w (t - mean) / W
                                const float dtm = t - gm;
                                const float Xd = gW > 0.0f ? __builtin_fmaf(gW * dtm, dtm, gL * __builtin_amdgcn_rcpf(gW)) : 0.0f;
                                gL = __builtin_fmaf(wgt, Xd, gL);
                                gW += wgt;
                                gm = __builtin_fmaf(wgt * __builtin_amdgcn_rcpf(gW), dtm, gm);
                            }
                            T = Tn;
                            last = pos1;
                            if (COUNT) ++n_blend;
                        }
                    }
                }
            }
            if (COUNT || bm) {
                const bool any_blend = __ballot(last == pos1) != 0ull;
                if (COUNT) w_blend += any_blend ? 1u : 0u;
                if (any_blend) blended |= 1ull << j;
            }
            wave_alive = __ballot(!done) != 0ull;
        }
        if (bm) {
            bm[b >> 6] = blended;  // every lane stores the same word
            n_words = (b >> 6) + 1u;
        }
    }

    if (o.step_count && lane == 0) o.step_count[4 * tile + wave] = n_words;
    if (inside) {
        const size_t hw = (size_t)P.width * P.height, pix = (size_t)py * P.width + px;
        o.color[pix] = c0 + T * P.bg[0];
        o.color[hw + pix] = c1 + T * P.bg[1];
        o.color[2 * hw + pix] = c2 + T * P.bg[2];
        if (NRM || GEO) {
            o.depth[pix] = dep;
            o.normal[pix] = n0;
            o.normal[hw + pix] = n1;
            o.normal[2 * hw + pix] = n2;
        }
        if (o.T_final) o.T_final[pix] = T;
        if (o.last) o.last[pix] = last;
        if (GEO) {
            o.curvature[pix] = kk;
            o.median_depth[pix] = med;
            o.distortion[pix] = gL;
            o.median_pos[pix] = med_pos;
        }
    }
    if (COUNT) {
        // list entries processed per pixel (up to and including a stop),
        // intersections evaluated, pairs blended
        uint32_t c[3] = {inside ? (stop_pos ? stop_pos : n) : 0u, n_eval, n_blend};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uint32_t v = c[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0 && v) atomicAdd(o.counters + 2 + k, v);
        }
        // per-wave step counts (the same in every lane)
        if (lane == 0 && w_rect) atomicAdd(o.counters + 5, w_rect);
        if (lane == 0 && w_eval) atomicAdd(o.counters + 6, w_eval);
        if (lane == 0 && w_blend) atomicAdd(o.counters + 7, w_blend);
    }
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
// adjoint of one blended entry: writes every field of gr (the entry's
// contribution to the primitive's record gradient).  dt: gradient with
// respect to the hit depth t; qn: the normal map's upstream gradient in the
// local frame, Rc^T gn; dK (GEO): with respect to the curvature value K at
// the hit.  Each sum starts from its first term (no addition to a zero).
template <bool GEO>
__device__ inline void entry_grad(const Prim &p, const float rgb[3], const PixelRay &ray, const RasterParams &P,
                                  const Hit &H, float G, float dalpha, float w, const float gc[3], float dt,
                                  const float qn[3], float dK, float *gr)
{
    // gradient arithmetic only (no decisions): products may fuse into fma
#pragma clang fp contract(fast)
    // colour and depth outputs
    gr[G_R] = gc[0] * w;
    gr[G_G] = gc[1] * w;
    gr[G_B] = gc[2] * w;
    const float dz = dt * ray.enorm;  // t = (Zc + s) |e|
    float dx, dy, dphi0, dphi1, dphi2, gl1, gl2;
    // normal output: n_cam = f Rc nl, nl = v / |v|, v = (-2 l1 x, -2 l2 y, 1)
    {
        float nl[3], il;
        const float f = hit_normal(p, H, nl, il);
        // Rc^T (w gn)
        const float q0 = qn[0] * w, q1 = qn[1] * w, q2 = qn[2] * w;
        // rotation: dphi = n_f x (Rc^T g), n_f = f nl, plus the terms below
        const float nf0 = f * nl[0], nf1 = f * nl[1], nf2 = f * nl[2];
        dphi0 = nf1 * q2 - nf2 * q1;
        dphi1 = nf2 * q0 - nf0 * q2;
        dphi2 = nf0 * q1 - nf1 * q0;
        // through the normalisation
        const float d0 = f * q0, d1 = f * q1, d2 = f * q2;
        const float dot = nl[0] * d0 + nl[1] * d1 + nl[2] * d2;
        const float dv0 = (d0 - nl[0] * dot) * il, dv1 = (d1 - nl[1] * dot) * il;
        gl1 = -2.0f * H.x * dv0;
        gl2 = -2.0f * H.y * dv1;
        dx = -2.0f * p.l1 * dv0;
        dy = -2.0f * p.l2 * dv1;
        // curvature output: K = 4 l1 l2 / D^2, D = 1 + 4 l1^2 x^2 + 4 l2^2 y^2 = 1 / il^2
        if (GEO) {
            const float i2 = il * il, i4 = i2 * i2;
            const float K = 4.0f * p.l1 * p.l2 * i4;
            const float dD = -2.0f * K * i2 * dK;
            gl1 += 4.0f * p.l2 * i4 * dK + 8.0f * p.l1 * H.x * H.x * dD;
            gl2 += 4.0f * p.l1 * i4 * dK + 8.0f * p.l2 * H.y * H.y * dD;
            dx += 8.0f * p.l1 * p.l1 * H.x * dD;
            dy += 8.0f * p.l2 * p.l2 * H.y * dD;
        }
    }
    // alpha = min(alpha_max, op G), G = exp(-E / 2), E = g(u)^2 Q
    float dG = 0.0f, gop = 0.0f;
    if (p.op * G < P.alpha_max) {
        gop = dalpha * G;
        dG = dalpha * p.op;
    }
    gr[G_OP] = gop;
    const float dE = -0.5f * G * dG;
    const float dQ = H.g * H.g * dE;
    const float du = 2.0f * H.g * gprime(H.u) * H.Q * dE;
    const float xx = H.x * H.x, yy = H.y * H.y;
    dx += 2.0f * p.k1 * H.x * dQ;
    dy += 2.0f * p.k2 * H.y * dQ;
    gr[G_K1] = xx * dQ;
    gr[G_K2] = yy * dQ;
    // u = 2 |h| / rho, h = l1 x^2 + l2 y^2
    if (H.rho2 > 0.0f && du != 0.0f) {
        const float irho = __builtin_amdgcn_rsqf(H.rho2);
        const float sg = H.h > 0.0f ? 1.0f : (H.h < 0.0f ? -1.0f : 0.0f);
        const float dh = du * 2.0f * sg * irho;
        const float drho = -du * 2.0f * __builtin_fabsf(H.h) * irho * irho;
        gl1 += xx * dh;
        gl2 += yy * dh;
        dx += (2.0f * p.l1 * dh + drho * irho) * H.x;
        dy += (2.0f * p.l2 * dh + drho * irho) * H.y;
    }
    // x = m0 + s e0, y = m1 + s e1, z = Zc + s
    float dm0 = dx, dm1 = dy;
    float de0 = H.s * dx, de1 = H.s * dy;
    const float ds = __builtin_fmaf(H.e0, dx, __builtin_fmaf(H.e1, dy, dz));
    // root of A s^2 + B s + C = 0 (implicit differentiation)
    const float iF = __builtin_amdgcn_rcpf(__builtin_fmaf(2.0f * H.A, H.s, H.B));
    const float dA = -H.s * H.s * iF * ds;
    const float dB = -H.s * iF * ds;
    const float dC = -iF * ds;
    // A = l1 e0^2 + l2 e1^2
    gl1 += H.e0 * H.e0 * dA;
    gl2 += H.e1 * H.e1 * dA;
    de0 += 2.0f * p.l1 * H.e0 * dA;
    de1 += 2.0f * p.l2 * H.e1 * dA;
    // B = 2 (l1 m0 e0 + l2 m1 e1) - e2
    gl1 += 2.0f * H.m0 * H.e0 * dB;
    gl2 += 2.0f * H.m1 * H.e1 * dB;
    dm0 += 2.0f * p.l1 * H.e0 * dB;
    dm1 += 2.0f * p.l2 * H.e1 * dB;
    de0 += 2.0f * p.l1 * H.m0 * dB;
    de1 += 2.0f * p.l2 * H.m1 * dB;
    const float de2 = -dB;
    // C = l1 m0^2 + l2 m1^2 - m2
    gl1 += H.m0 * H.m0 * dC;
    gl2 += H.m1 * H.m1 * dC;
    dm0 += 2.0f * p.l1 * H.m0 * dC;
    dm1 += 2.0f * p.l2 * H.m1 * dC;
    const float dm2 = -dC;
    // mhat = Rc^T m, ehat = Rc^T e: dphi += dm x m + de x e
    dphi0 += dm1 * H.m2 - dm2 * H.m1 + de1 * H.e2 - de2 * H.e1;
    dphi1 += dm2 * H.m0 - dm0 * H.m2 + de2 * H.e0 - de0 * H.e2;
    dphi2 += dm0 * H.m1 - dm1 * H.m0 + de0 * H.e1 - de1 * H.e0;
    // m = (kx dxp, ky dyp, 0), kx = Zc / fx, dxp = u + 0.5 - u_c
    const float dmx = __builtin_fmaf(p.R[0], dm0, __builtin_fmaf(p.R[1], dm1, p.R[2] * dm2));
    const float dmy = __builtin_fmaf(p.R[3], dm0, __builtin_fmaf(p.R[4], dm1, p.R[5] * dm2));
    gr[G_L1] = gl1;
    gr[G_L2] = gl2;
    gr[G_UC] = -dmx * p.kx;
    gr[G_VC] = -dmy * p.ky;
    gr[G_ZC] = dz + (dmx * H.dxp * P.ifx + dmy * H.dyp * P.ify);
    gr[G_PHI0] = dphi0;
    gr[G_PHI1] = dphi1;
    gr[G_PHI2] = dphi2;
}

// The backward walks each wave's entries from its pixels' largest `last` down
// to the first, with the same per-wave list reading as the forward.  A
// visited entry's per-lane gradients are reduce-scattered over the wave, and
// the 14 field totals go to memory from 14 lanes in one instruction: atomic
// adds into the primitive's record gradient, or (DET) a store into the pair's
// slot for this wave, summed later in a fixed order.
template <bool DET, bool GEO>
// `recs` is a.records again, as a restrict argument: the records are never
// written here, which lets the compiler read them with scalar loads although
// the loop stores gradients.
// Launched as one-wave workgroups (4 per tile); BLOCK only bounds the size.
__global__ __launch_bounds__(BLOCK, GEO ? QGS_BWD_GEO_MIN_WAVES : QGS_BWD_MIN_WAVES) void k_render_bwd(
    RasterArgs a, RasterParams P, BwdIn in, const float4 *__restrict__ recs, float *__restrict__ grad_rec,
    float *__restrict__ pair_scratch)
{
    // the block: from the backward's block order, or the tile order's tile
    const uint32_t bid = a.block_order ? a.block_order[blockIdx.x]
                                       : 4u * (a.tile_order ? a.tile_order[blockIdx.x >> 2] : (blockIdx.x >> 2)) +
                                             (blockIdx.x & 3u);
    const int tile = (int)(bid >> 2);
    if ((unsigned)tile >= (unsigned)(P.tiles_x * P.tiles_y)) return;  // whole workgroup; cannot happen for lists built here
    const int tx = tile % P.tiles_x, ty = tile / P.tiles_x;
    const int tid = threadIdx.x, lane = tid & 63, wave = (int)(bid & 3u);
    __shared__ float s_red[16 * RED_ROW];  // the wave's gradient reduction block
    clear_reduce_lds(s_red);
    const int wx0 = tx * TILE + (wave & 1) * 8, wy0 = ty * TILE + (wave >> 1) * 8;
    const int px = wx0 + (lane & 7), py = wy0 + (lane >> 3);
    const bool inside = px < P.width && py < P.height;
    const uint32_t start = a.ranges[2 * tile], list_len = a.ranges[2 * tile + 1] - start;
    const PixelRay ray = make_ray(px, py, P);
    
    const size_t hw = (size_t)P.width * P.height, pix = (size_t)py * P.width + px;
    float T = 1.0f, gc[3] = {0, 0, 0}, gd = 0.0f, gn[3] = {0, 0, 0};
    uint32_t last = 0;
    if (inside) {
        T = in.T_final[pix];
        last = in.last[pix];
        if (in.dcolor) {
            gc[0] = in.dcolor[pix];
            gc[1] = in.dcolor[hw + pix];
            gc[2] = in.dcolor[2 * hw + pix];
        }
        if (in.ddepth) gd = in.ddepth[pix];
        if (in.dnormal) {
            gn[0] = in.dnormal[pix];
            gn[1] = in.dnormal[hw + pix];
            gn[2] = in.dnormal[2 * hw + pix];
        }
    }
    // geometry: upstream gradients and the pixel's final sum of weights W,
    // mean depth and distortion L; the distortion adjoint is the linear one
    // with X_i = dL/dw_i = L / W + W (t_i - mean)^2, plus dL/dt_i = 2 w_i W (t_i - mean)
    float gK = 0.0f, gmed = 0.0f, gdist = 0.0f, gW = 0.0f, gm = 0.0f, gLW = 0.0f;
    uint32_t med_pos = 0;
    if (GEO && inside) {
        if (in.dcurvature) gK = in.dcurvature[pix];
        if (in.dmedian) gmed = in.dmedian[pix];
        if (in.ddistortion) gdist = in.ddistortion[pix];
        med_pos = in.median_pos[pix];
        gW = 1.0f - T;
        if (gW > 0.0f) {
            const float iW = __builtin_amdgcn_rcpf(gW);
            gm = in.depth[pix] * iW;
            gLW = in.distortion[pix] * iW;
        }
    }
    // composited channels: colour, depth, normal; GEO adds curvature and
    // distortion
    constexpr int NX = GEO ? 9 : 7;
    // The upstream gradients gx are fixed per pixel, so only the contraction
    // gS = sum_c gx_c S_c of the suffix sums is needed: dX/dalpha_i contracted
    // with gx is T_i gX_i - gS_i / (1 - alpha_i), gX_i = sum_c gx_c X_c, and
    // gS grows by w_i gX_i (colour starts with the background term).
    float gS = T * ((gc[0] * P.bg[0] + gc[1] * P.bg[1]) + gc[2] * P.bg[2]);
    // adjoint of visited entry `pos` (primitive pj)
    auto visit = [&](uint32_t pos, uint32_t pj) {
        const float *wr = reinterpret_cast<const float *>(recs + (size_t)pj * 8);
        float dxp, dyp;
        const bool lane_on = conic_offsets(wr, ray, dxp, dyp) & (pos < last);
        if (__ballot(lane_on) == 0ull) return;
        // written only by contributing lanes; the others give zeros below
        // (one select per field, instead of zeroing on every other path)
        float gr[NGRAD];
        bool contrib = false;
        if (lane_on) {
            Prim p;
            load_prim(wr, P, p);
            Hit H;
            if (ray_hit(p, ray, P, dxp, dyp, H)) {
                const float G = __expf(-0.5f * H.E);
                const float alpha = fminf(P.alpha_max, p.op * G);
                if (alpha >= P.alpha_min) {
#pragma clang fp contract(fast)
                    contrib = true;
                    const float4 cr = *reinterpret_cast<const float4 *>(wr + 24);
                    const float rgb[3] = {cr.y, cr.z, cr.w};
                    const float om = 1.0f - alpha;
                    const float iom = __builtin_amdgcn_rcpf(om);
                    const float Ti = T * iom;
                    const float w = alpha * Ti;
                    float X[NX];
                    X[0] = rgb[0];
                    X[1] = rgb[1];
                    X[2] = rgb[2];
                    const float t = (p.Zc + H.s) * ray.enorm;
                    X[3] = t;
                    float nl[3], il;
                    const float f = hit_normal(p, H, nl, il);
                    // gn . (f Rc nl) = f (Rc^T gn) . nl
                    float qn[3];
                    qn[0] = __builtin_fmaf(p.R[0], gn[0], __builtin_fmaf(p.R[3], gn[1], p.R[6] * gn[2]));
                    qn[1] = __builtin_fmaf(p.R[1], gn[0], __builtin_fmaf(p.R[4], gn[1], p.R[7] * gn[2]));
                    qn[2] = __builtin_fmaf(p.R[2], gn[0], __builtin_fmaf(p.R[5], gn[1], p.R[8] * gn[2]));
                    X[4] = f * __builtin_fmaf(qn[0], nl[0], __builtin_fmaf(qn[1], nl[1], qn[2] * nl[2]));
                    X[5] = 0.0f;
                    X[6] = 0.0f;
                    float gx[NX] = {gc[0], gc[1], gc[2], gd, 1.0f, 0.0f, 0.0f};
                    float dt = gd * w;
                    if (GEO) {
                        const float dtm = t - gm;
                        X[7] = hit_curvature(p, il);
                        X[8] = __builtin_fmaf(gW * dtm, dtm, gLW);
                        gx[7] = gK;
                        gx[8] = gdist;
                        dt = __builtin_fmaf(gdist * 2.0f * w * gW, dtm, dt);
                        if (pos + 1u == med_pos) dt += gmed;
                    }
                    float gX = 0.0f;
#pragma unroll
                    for (int c = 0; c < NX; ++c) gX += gx[c] * X[c];
                    const float dalpha = Ti * gX - gS * iom;
                    gS = __builtin_fmaf(w, gX, gS);
                    T = Ti;
                    entry_grad<GEO>(p, rgb, ray, P, H, G, dalpha, w, gc, dt, qn, GEO ? gK * w : 0.0f, gr);
                }
            }
        }
        if (__ballot(contrib) != 0ull) {
            // lane 4f (f < NGRAD) ends with the wave total of field f
            const float tot = wave_reduce_lds(s_red, gr, contrib);
            const int f = lane >> 2;
            if ((lane & 3) == 0 && f < NGRAD) {
                if (DET)
                    pair_scratch[((size_t)start + pos) * 64 + wave * 16 + f] = tot;
                else if (tot != 0.0f)
                    unsafeAtomicAdd(grad_rec + (size_t)pj * 16 + f, tot);
            }
        }
    };

    if (in.steps) {
        // replay: only the entries some pixel of this block blended, last first
        const uint32_t nw_max = (list_len + 63u) >> 6;
        uint32_t nw = in.step_count[4 * tile + wave];
        nw = nw < nw_max ? nw : nw_max;
        const uint64_t *bm = in.steps + replay_base(start, list_len, tile, wave);
        uint32_t nxt_pid = 0;
        int32_t w = (int32_t)nw - 1;
        if (w >= 0 && (uint32_t)(64 * w + lane) < list_len) nxt_pid = a.pair_prim[start + 64 * w + lane];
        for (; w >= 0; --w) {
            const uint32_t cur_pid = nxt_pid;
            nxt_pid = 0;
            if (w >= 1) nxt_pid = a.pair_prim[start + 64 * (w - 1) + lane];  // word w - 1 is full
            uint64_t m = bm[w];
            while (m != 0ull) {
                const int j = 63 - __builtin_clzll(m);
                m &= ~(1ull << j);
                const uint32_t pos = 64u * (uint32_t)w + (uint32_t)j;
                if (pos >= list_len) continue;  // not written by a matching forward
                visit(pos, (uint32_t)__builtin_amdgcn_readlane((int)cur_pid, j));
            }
        }
        return;
    }

    // never walk past the tile's list, whatever `last` holds
    const uint32_t wmax = wave_max_u32(last);
    const uint32_t nmax = wmax < list_len ? wmax : list_len;

    // batch fetch, backwards: lane i holds entry lo + i of [lo, lo + 64)
    uint32_t nxt_pid = 0;
    int4 nxt_rect = make_int4(0, -1, 0, -1);
    int32_t lo = ((int32_t)nmax - 1) & ~63;  // first batch: the one holding entry nmax - 1
    if (nmax > 0 && (uint32_t)(lo + lane) < nmax) {
        nxt_pid = a.pair_prim[start + lo + lane];
        nxt_rect = *reinterpret_cast<const int4 *>(recs + (size_t)nxt_pid * 8);
    }
    for (; nmax > 0 && lo >= 0; lo -= 64) {
        const uint32_t cur_pid = nxt_pid;
        const int4 cur_rect = nxt_rect;
        if (lo >= 64) {
            nxt_pid = a.pair_prim[start + lo - 64 + lane];
            nxt_rect = *reinterpret_cast<const int4 *>(recs + (size_t)nxt_pid * 8);
        }
        const bool rel = (uint32_t)(lo + lane) < nmax && !(cur_rect.y < wx0 || cur_rect.x > wx0 + 7 ||
                                                         cur_rect.w < wy0 || cur_rect.z > wy0 + 7);
        uint64_t m = __ballot(rel);
        while (m != 0ull) {
            const int j = 63 - __builtin_clzll(m);
            m &= ~(1ull << j);
            visit((uint32_t)(lo + j), (uint32_t)__builtin_amdgcn_readlane((int)cur_pid, j));
        }
    }
}

// deterministic second pass: sum each primitive's per-pair partials in
// emission order (its pairs are pair_offset[p] ... + tiles[p] - 1 there),
// each pair's four per-wave slots in wave order
__global__ __launch_bounds__(256) void k_det_reduce(const float *pair_scratch, const uint32_t *pair_offset,
                                                    const uint32_t *tiles, const uint32_t *emit_to_sorted, int64_t n,
                                                    uint64_t capacity, float *grad_rec)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    float acc[NGRAD];
#pragma unroll
    for (int f = 0; f < NGRAD; ++f) acc[f] = 0.0f;
    const uint32_t cnt = tiles[p], e0 = pair_offset[p];
    for (uint32_t k = 0; k < cnt; ++k) {
        if ((uint64_t)e0 + k >= capacity) break;  // cannot happen for lists built here
        const uint32_t i = emit_to_sorted[e0 + k];
        if (i >= capacity) continue;  // cannot happen for lists built with the map
        const float *src = pair_scratch + (size_t)i * 64;
        for (int wv = 0; wv < 4; ++wv)
#pragma unroll
            for (int f = 0; f < NGRAD; ++f) acc[f] += src[16 * wv + f];
    }
#pragma unroll
    for (int f = 0; f < NGRAD; ++f) grad_rec[16 * p + f] = acc[f];
    grad_rec[16 * p + 14] = 0.0f;
    grad_rec[16 * p + 15] = 0.0f;
}

// ---------------------------------------------------------------------------
// resort mode (supplement, per-pixel resorting)
// ---------------------------------------------------------------------------
// Each lane keeps its accepted hits in a buffer of RS_K entries; when the
// buffer is full the nearest (smallest t, the earliest list position among
// equal t) is blended, and at the end of the list the rest in the same way.
// The buffer lives in registers: it is kept sorted by (t, position) and every
// access uses a compile-time index (insertion shifts by one slot, the nearest
// is slot 0), so no array is ever indexed at run time.
constexpr int RS_K = 8;

template <int NF>
struct ResortBuf {
    float t[RS_K];
    float f[NF][RS_K];
    uint32_t pid[RS_K], pos[RS_K];
    int cnt;

    __device__ inline void insert(float xt, const float (&xf)[NF], uint32_t xpid, uint32_t xpos)
    {
        // entries already held come first on equal t (their positions are smaller)
#pragma unroll
        for (int i = RS_K - 1; i >= 0; --i) {
            if (i > cnt) continue;
            const bool keep = i < cnt && t[i] <= xt;
            if (keep) continue;
            const int j = i > 0 ? i - 1 : 0;
            const bool here = i == 0 || t[j] <= xt;
            t[i] = here ? xt : t[j];
#pragma unroll
            for (int k = 0; k < NF; ++k) f[k][i] = here ? xf[k] : f[k][j];
            pid[i] = here ? xpid : pid[j];
            pos[i] = here ? xpos : pos[j];
        }
        ++cnt;
    }

    // removes the nearest entry (slot 0) into the outputs
    __device__ inline void pop(float &xt, float (&xf)[NF], uint32_t &xpid, uint32_t &xpos)
    {
        xt = t[0];
#pragma unroll
        for (int k = 0; k < NF; ++k) xf[k] = f[k][0];
        xpid = pid[0];
        xpos = pos[0];
#pragma unroll
        for (int i = 0; i + 1 < RS_K; ++i) {
            t[i] = t[i + 1];
#pragma unroll
            for (int k = 0; k < NF; ++k) f[k][i] = f[k][i + 1];
            pid[i] = pid[i + 1];
            pos[i] = pos[i + 1];
        }
        --cnt;
    }
};

// local ray direction e = Rc^T (xn, yn, 1), as in ray_hit
__device__ inline void local_dir(const Prim &p, const PixelRay &r, float &e0, float &e1, float &e2)
{
    e0 = __builtin_fmaf(p.R[0], r.xn, __builtin_fmaf(p.R[3], r.yn, p.R[6]));
    e1 = __builtin_fmaf(p.R[1], r.xn, __builtin_fmaf(p.R[4], r.yn, p.R[7]));
    e2 = __builtin_fmaf(p.R[2], r.xn, __builtin_fmaf(p.R[5], r.yn, p.R[8]));
}

template <bool GEO>
__global__ __launch_bounds__(BLOCK) void k_render_fwd_rs(RasterArgs a, RasterParams P, FwdOut o,
                                                         const float4 *__restrict__ recs, uint64_t *__restrict__ replay)
{
    // one-wave workgroups, ids mapped as in k_render_fwd (a tile's four blocks
    // on one XCD, the tiles in order)
    const uint32_t ntl = (uint32_t)(P.tiles_x * P.tiles_y);
    const uint32_t grp = blockIdx.x >> 5, r32 = blockIdx.x & 31u;
    const uint32_t left = ntl - 8u * grp, mg = left < 8u ? left : 8u;
    const uint32_t slot = mg == 8u ? 8u * grp + (r32 & 7u) : 8u * grp + r32 % mg;
    const uint32_t kblk = mg == 8u ? r32 >> 3 : r32 / mg;
    const int tile = a.tile_order ? (int)a.tile_order[slot] : (int)slot;
    if ((unsigned)tile >= (unsigned)(P.tiles_x * P.tiles_y)) return;  // whole workgroup; cannot happen for lists built here
    const int tx = tile % P.tiles_x, ty = tile / P.tiles_x;
    const int tid = threadIdx.x, lane = tid & 63, wave = (int)kblk;
    const int wx0 = tx * TILE + (wave & 1) * 8, wy0 = ty * TILE + (wave >> 1) * 8;
    const int px = wx0 + (lane & 7), py = wy0 + (lane >> 3);
    const bool inside = px < P.width && py < P.height;
    const uint32_t start = a.ranges[2 * tile], n = a.ranges[2 * tile + 1] - start;
    const PixelRay ray = make_ray(px, py, P);

    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, dep = 0.0f, n0 = 0.0f, n1 = 0.0f, n2 = 0.0f;
    uint32_t last = 0, stop_pos = 0, n_eval = 0, n_blend = 0;
    bool done = !inside;
    float kk = 0.0f, med = 0.0f, gW = 0.0f, gm = 0.0f, gL = 0.0f;
    uint32_t med_pos = 0;
    ResortBuf<3> buf;  // fields: alpha, x, y
    buf.cnt = 0;
    // replay bitmap of this block: bit j of word w set when some pixel took entry 64 w + j in
    uint64_t *bm = replay ? replay + replay_base(start, n, tile, wave) : nullptr;
    uint32_t n_words = 0;

    // blend the nearest pending hit (per lane)
    auto pop_blend = [&]() {
        float t, fv[3];
        uint32_t pid, pos1;
        buf.pop(t, fv, pid, pos1);
        const float alpha = fv[0], x = fv[1], y = fv[2];
        const float Tn = T * (1.0f - alpha);
        if (Tn < P.T_eps) {
            done = true;
            stop_pos = last;
            return;
        }
        const float wgt = alpha * T;
        const float *w = reinterpret_cast<const float *>(recs + (size_t)pid * 8);
        Prim p;
        load_prim(w, P, p);
        Hit H;
        H.x = x;
        H.y = y;
        local_dir(p, ray, H.e0, H.e1, H.e2);
        c0 = __builtin_fmaf(wgt, w[25], c0);
        c1 = __builtin_fmaf(wgt, w[26], c1);
        c2 = __builtin_fmaf(wgt, w[27], c2);
        dep = __builtin_fmaf(wgt, t, dep);
        float nl[3], il;
        const float f = hit_normal(p, H, nl, il);
        const float wf = wgt * f;
        n0 = __builtin_fmaf(wf, __builtin_fmaf(p.R[0], nl[0], __builtin_fmaf(p.R[1], nl[1], p.R[2] * nl[2])), n0);
        n1 = __builtin_fmaf(wf, __builtin_fmaf(p.R[3], nl[0], __builtin_fmaf(p.R[4], nl[1], p.R[5] * nl[2])), n1);
        n2 = __builtin_fmaf(wf, __builtin_fmaf(p.R[6], nl[0], __builtin_fmaf(p.R[7], nl[1], p.R[8] * nl[2])), n2);
        if (GEO) {
            kk = __builtin_fmaf(wgt, hit_curvature(p, il), kk);
            if (T > 0.5f && (med_pos == 0u || t > med)) {
                med = t;
                med_pos = pos1;
            }
            const float dtm = t - gm;
            const float Xd = gW > 0.0f ? __builtin_fmaf(gW * dtm, dtm, gL * __builtin_amdgcn_rcpf(gW)) : 0.0f;
            gL = __builtin_fmaf(wgt, Xd, gL);
            gW += wgt;
            gm = __builtin_fmaf(wgt * __builtin_amdgcn_rcpf(gW), dtm, gm);
        }
        T = Tn;
        ++n_blend;
    };

    // primitive ids two batches ahead, rectangles one batch ahead
    uint32_t nxt_pid = 0, nn_pid = 0;
    int4 nxt_rect = make_int4(0, -1, 0, -1);
    if ((uint32_t)lane < n) {
        nxt_pid = a.pair_prim[start + lane];
        nxt_rect = *reinterpret_cast<const int4 *>(recs + (size_t)nxt_pid * 8);
    }
    if (64u + (uint32_t)lane < n) nn_pid = a.pair_prim[start + 64 + lane];
    bool wave_alive = __ballot(!done) != 0ull;
    for (uint32_t b = 0; b < n && wave_alive; b += 64) {
        const uint32_t cur_pid = nxt_pid;
        const int4 cur_rect = nxt_rect;
        // entries whose rectangle and pre-test conic meet the block (the
        // conic test's loads come before the next batch's, so waiting for
        // them leaves those in flight)
        bool rel = b + (uint32_t)lane < n && !(cur_rect.y < wx0 || cur_rect.x > wx0 + 7 ||
                                                 cur_rect.w < wy0 || cur_rect.z > wy0 + 7);
        if (rel) rel = conic_meets_block(recs + (size_t)cur_pid * 8, (float)wx0, (float)wy0);
        nxt_pid = nn_pid;
        if (b + 64 + (uint32_t)lane < n) nxt_rect = *reinterpret_cast<const int4 *>(recs + (size_t)nxt_pid * 8);
        if (b + 128 + (uint32_t)lane < n) nn_pid = a.pair_prim[start + b + 128 + lane];
        uint64_t m = __ballot(rel);
        uint64_t taken = 0ull;
        while (m != 0ull && wave_alive) {
            const int j = __builtin_ctzll(m);
            m &= m - 1ull;
            const uint32_t pj = (uint32_t)__builtin_amdgcn_readlane((int)cur_pid, j);
            float rw[32];
            load_record_words(recs, pj, rw);
            const float *w = rw;
            float dxp, dyp;
            const bool lane_on = conic_offsets(w, ray, dxp, dyp) & !done;
            if (__ballot(lane_on) == 0ull) continue;
            const uint32_t pos1 = b + (uint32_t)j + 1u;
            if (lane_on) {
                Prim p;
                load_prim(w, P, p);
                Hit H;
                ++n_eval;
                if (ray_hit(p, ray, P, dxp, dyp, H)) {
                    const float G = __expf(-0.5f * H.E);
                    const float alpha = fminf(P.alpha_max, p.op * G);
                    if (alpha >= P.alpha_min) {
                        const float t = (p.Zc + H.s) * ray.enorm;
                        const float fv[3] = {alpha, H.x, H.y};
                        buf.insert(t, fv, pj, pos1);
                        last = pos1;
                        if (buf.cnt == RS_K) pop_blend();
                    }
                }
            }
            if (bm && __ballot(last == pos1) != 0ull) taken |= 1ull << j;
            wave_alive = __ballot(!done) != 0ull;
        }
        if (bm) {
            bm[b >> 6] = taken;  // every lane stores the same word
            n_words = (b >> 6) + 1u;
        }
    }
    if (o.step_count && lane == 0) o.step_count[4 * tile + wave] = n_words;
    // end of the list: blend what is pending, nearest first
    while (buf.cnt > 0 && !done) pop_blend();

    if (inside) {
        const size_t hw = (size_t)P.width * P.height, pix = (size_t)py * P.width + px;
        o.color[pix] = c0 + T * P.bg[0];
        o.color[hw + pix] = c1 + T * P.bg[1];
        o.color[2 * hw + pix] = c2 + T * P.bg[2];
        o.depth[pix] = dep;
        o.normal[pix] = n0;
        o.normal[hw + pix] = n1;
        o.normal[2 * hw + pix] = n2;
        if (o.T_final) o.T_final[pix] = T;
        // the backward replays the entries up to the last one this pixel took in
        if (o.last) o.last[pix] = last;
        if (GEO) {
            o.curvature[pix] = kk;
            o.median_depth[pix] = med;
            o.distortion[pix] = gL;
            o.median_pos[pix] = med_pos;
        }
    }
    if (o.counters) {
        uint32_t c[3] = {inside ? (stop_pos ? stop_pos : n) : 0u, n_eval, n_blend};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uint32_t v = c[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0 && v) atomicAdd(o.counters + 2 + k, v);
        }
    }
}

// Backward of the resort mode, front to back (supplement, front-to-back form
// of the adjoint): each pixel replays the forward's entries and buffer up to
// its `last`, keeping T_i and the prefix sums P_i = sum_{j<i} w_j X_j, so the
// suffix after entry i is S_i = X_hat - P_i - w_i X_i with X_hat the forward's
// output, and dX/dalpha_i = T_i X_i - S_i / (1 - alpha_i).  A blended entry's
// hit is recomputed from its record (lanes blend different entries at a
// step), and the lanes of a step that blended the same primitive are reduced
// together: one reduce-scatter and one 14-lane atomic per distinct primitive
// (or, DET, an add into the pair's slot for this wave).
template <bool DET, bool GEO>
__global__ __launch_bounds__(BLOCK) void k_render_bwd_rs(RasterArgs a, RasterParams P, BwdIn in,
                                                         const float4 *__restrict__ recs,
                                                         float *__restrict__ grad_rec, float *__restrict__ pair_scratch)
{
    // one-wave workgroups: the block from the backward's block order, or the
    // tile order's tile
    const uint32_t bid = a.block_order ? a.block_order[blockIdx.x]
                                       : 4u * (a.tile_order ? a.tile_order[blockIdx.x >> 2] : (blockIdx.x >> 2)) +
                                             (blockIdx.x & 3u);
    const int tile = (int)(bid >> 2);
    if ((unsigned)tile >= (unsigned)(P.tiles_x * P.tiles_y)) return;  // whole workgroup; cannot happen for lists built here
    const int tx = tile % P.tiles_x, ty = tile / P.tiles_x;
    const int tid = threadIdx.x, lane = tid & 63, wave = (int)(bid & 3u);
    __shared__ float s_red[16 * RED_ROW];  // the wave's gradient reduction block
    clear_reduce_lds(s_red);
    const int wx0 = tx * TILE + (wave & 1) * 8, wy0 = ty * TILE + (wave >> 1) * 8;
    const int px = wx0 + (lane & 7), py = wy0 + (lane >> 3);
    const bool inside = px < P.width && py < P.height;
    const uint32_t start = a.ranges[2 * tile], list_len = a.ranges[2 * tile + 1] - start;
    const PixelRay ray = make_ray(px, py, P);

    const size_t hw = (size_t)P.width * P.height, pix = (size_t)py * P.width + px;
    constexpr int NX = GEO ? 9 : 7;
    float gc[3] = {0, 0, 0}, gd = 0.0f, gn[3] = {0, 0, 0};
    float Xh[NX];
#pragma unroll
    for (int c = 0; c < NX; ++c) Xh[c] = 0.0f;
    uint32_t last = 0;
    float T = 1.0f;
    if (inside) {
        last = in.last[pix];
        if (in.dcolor) {
            gc[0] = in.dcolor[pix];
            gc[1] = in.dcolor[hw + pix];
            gc[2] = in.dcolor[2 * hw + pix];
        }
        if (in.ddepth) gd = in.ddepth[pix];
        if (in.dnormal) {
            gn[0] = in.dnormal[pix];
            gn[1] = in.dnormal[hw + pix];
            gn[2] = in.dnormal[2 * hw + pix];
        }
        Xh[0] = in.color[pix];
        Xh[1] = in.color[hw + pix];
        Xh[2] = in.color[2 * hw + pix];
        Xh[3] = in.depth[pix];
        Xh[4] = in.normal[pix];
        Xh[5] = in.normal[hw + pix];
        Xh[6] = in.normal[2 * hw + pix];
    }
    float gK = 0.0f, gmed = 0.0f, gdist = 0.0f, gW = 0.0f, gm = 0.0f, gLW = 0.0f;
    uint32_t med_pos = 0;
    if (GEO && inside) {
        if (in.dcurvature) gK = in.dcurvature[pix];
        if (in.dmedian) gmed = in.dmedian[pix];
        if (in.ddistortion) gdist = in.ddistortion[pix];
        med_pos = in.median_pos[pix];
        gW = 1.0f - in.T_final[pix];
        const float L = in.distortion[pix];
        if (gW > 0.0f) {
            const float iW = __builtin_amdgcn_rcpf(gW);
            gm = in.depth[pix] * iW;
            gLW = L * iW;
        }
        Xh[7] = in.curvature[pix];
        Xh[8] = 2.0f * L;  // sum_i w_i (L / W + W (t_i - mean)^2)
    }
    // the forward's outputs and the prefix sums contracted with the upstream
    // gradients: gXh = sum_c gx_c Xhat_c, gPf = sum_c gx_c sum_{j<i} w_j X_jc
    float gXh = ((gc[0] * Xh[0] + gc[1] * Xh[1]) + gc[2] * Xh[2]) + gd * Xh[3] +
                ((gn[0] * Xh[4] + gn[1] * Xh[5]) + gn[2] * Xh[6]);
    if (GEO) gXh += gK * Xh[7] + gdist * Xh[8];
    float gPf = 0.0f;
    bool done = !inside;
    ResortBuf<1> buf;  // field: alpha
    buf.cnt = 0;

    // blend-backward of the nearest pending hit: per-lane gradient in gr
    auto pop_grad = [&](float (&gr)[NGRAD], uint32_t &g_pid, uint32_t &g_pos) -> bool {
        float tq, fv[1];
        uint32_t pid, pos1;
        buf.pop(tq, fv, pid, pos1);
        const float alpha = fv[0];
        const float om = 1.0f - alpha;
        const float Tn = T * om;
        if (Tn < P.T_eps) {
            done = true;
            return false;
        }
        const float *wr = reinterpret_cast<const float *>(recs + (size_t)pid * 8);
        Prim p;
        load_prim(wr, P, p);
        float dxp, dyp;
        (void)conic_offsets(wr, ray, dxp, dyp);
        Hit H;
        if (!ray_hit(p, ray, P, dxp, dyp, H)) {  // cannot happen: the same hit was accepted before
            T = Tn;
            return false;
        }
        const float G = __expf(-0.5f * H.E);
        const float w = alpha * T;
        const float iom = __builtin_amdgcn_rcpf(om);
        float X[NX];
        X[0] = wr[25];
        X[1] = wr[26];
        X[2] = wr[27];
        const float t = (p.Zc + H.s) * ray.enorm;
        X[3] = t;
        float nl[3], il;
        const float f = hit_normal(p, H, nl, il);
        // gn . (f Rc nl) = f (Rc^T gn) . nl
        float qn[3];
        qn[0] = __builtin_fmaf(p.R[0], gn[0], __builtin_fmaf(p.R[3], gn[1], p.R[6] * gn[2]));
        qn[1] = __builtin_fmaf(p.R[1], gn[0], __builtin_fmaf(p.R[4], gn[1], p.R[7] * gn[2]));
        qn[2] = __builtin_fmaf(p.R[2], gn[0], __builtin_fmaf(p.R[5], gn[1], p.R[8] * gn[2]));
        X[4] = f * __builtin_fmaf(qn[0], nl[0], __builtin_fmaf(qn[1], nl[1], qn[2] * nl[2]));
        X[5] = 0.0f;
        X[6] = 0.0f;
        float gx[NX] = {gc[0], gc[1], gc[2], gd, 1.0f, 0.0f, 0.0f};
        float dt = gd * w;
        if (GEO) {
            const float dtm = t - gm;
            X[7] = hit_curvature(p, il);
            X[8] = __builtin_fmaf(gW * dtm, dtm, gLW);
            gx[7] = gK;
            gx[8] = gdist;
            dt = __builtin_fmaf(gdist * 2.0f * w * gW, dtm, dt);
            if (pos1 == med_pos) dt += gmed;
        }
        // contracted with the fixed upstream gradients: the suffix after this
        // entry is gXh - gPf - w gX
        float gX = 0.0f;
#pragma unroll
        for (int c = 0; c < NX; ++c) gX += gx[c] * X[c];
        const float dalpha = T * gX - ((gXh - gPf) - w * gX) * iom;
        gPf = __builtin_fmaf(w, gX, gPf);
        const float rgb[3] = {X[0], X[1], X[2]};
        entry_grad<GEO>(p, rgb, ray, P, H, G, dalpha, w, gc, dt, qn, GEO ? gK * w : 0.0f, gr);
        T = Tn;
        g_pid = pid;
        g_pos = pos1;
        return true;
    };

    // the lanes of this step that blended the same primitive are reduced together
    auto flush_grads = [&](const float (&gr)[NGRAD], bool has, uint32_t g_pid, uint32_t g_pos) {
        uint64_t rem = __ballot(has);
        while (rem != 0ull) {
            const int l0 = __builtin_ctzll(rem);
            const uint32_t pid0 = (uint32_t)__builtin_amdgcn_readlane((int)g_pid, l0);
            const uint32_t pos0 = (uint32_t)__builtin_amdgcn_readlane((int)g_pos, l0);
            const bool mine = has && g_pid == pid0;
            rem &= ~__ballot(mine);
            const float tot = wave_reduce_lds(s_red, gr, mine);
            const int f = lane >> 2;
            if ((lane & 3) == 0 && f < NGRAD) {
                if (DET) {
                    // the pair's slot for this wave; only this wave adds to it
                    float *dst = pair_scratch + ((size_t)start + pos0 - 1u) * 64 + wave * 16 + f;
                    *dst += tot;
                } else if (tot != 0.0f) {
                    unsafeAtomicAdd(grad_rec + (size_t)pid0 * 16 + f, tot);
                }
            }
        }
    };

    // replay of visited entry pos1 - 1 (primitive pj)
    auto visit = [&](uint32_t pos1, uint32_t pj) {
        const float *w = reinterpret_cast<const float *>(recs + (size_t)pj * 8);
        float dxp, dyp;
        const bool lane_on = !done && pos1 <= last && conic_offsets(w, ray, dxp, dyp);
        if (__ballot(lane_on) == 0ull) return;
        float gr[NGRAD];
#pragma unroll
        for (int f = 0; f < NGRAD; ++f) gr[f] = 0.0f;
        bool has = false;
        uint32_t g_pid = 0, g_pos = 0;
        if (lane_on) {
            Prim p;
            load_prim(w, P, p);
            Hit H;
            if (ray_hit(p, ray, P, dxp, dyp, H)) {
                const float G = __expf(-0.5f * H.E);
                const float alpha = fminf(P.alpha_max, p.op * G);
                if (alpha >= P.alpha_min) {
                    const float fv[1] = {alpha};
                    buf.insert((p.Zc + H.s) * ray.enorm, fv, pj, pos1);
                    if (buf.cnt == RS_K) has = pop_grad(gr, g_pid, g_pos);
                }
            }
        }
        if (__ballot(has) != 0ull) flush_grads(gr, has, g_pid, g_pos);
    };

    if (in.steps) {
        // only the entries some pixel of this block took into its buffer, in list order
        const uint32_t nw_max = (list_len + 63u) >> 6;
        uint32_t nw = in.step_count[4 * tile + wave];
        nw = nw < nw_max ? nw : nw_max;
        const uint64_t *bm = in.steps + replay_base(start, list_len, tile, wave);
        uint32_t nxt_pid = 0;
        if (nw > 0 && (uint32_t)lane < list_len) nxt_pid = a.pair_prim[start + lane];
        for (uint32_t w = 0; w < nw; ++w) {
            const uint32_t cur_pid = nxt_pid;
            nxt_pid = 0;
            if (w + 1 < nw && 64 * (w + 1) + (uint32_t)lane < list_len) nxt_pid = a.pair_prim[start + 64 * (w + 1) + lane];
            uint64_t m = bm[w];
            while (m != 0ull) {
                const int j = __builtin_ctzll(m);
                m &= m - 1ull;
                const uint32_t pos = 64u * w + (uint32_t)j;
                if (pos >= list_len) continue;  // not written by a matching forward
                visit(pos + 1u, (uint32_t)__builtin_amdgcn_readlane((int)cur_pid, j));
            }
        }
    } else {
        const uint32_t wmax = wave_max_u32(last);
        const uint32_t nmax = wmax < list_len ? wmax : list_len;
        uint32_t nxt_pid = 0;
        int4 nxt_rect = make_int4(0, -1, 0, -1);
        if ((uint32_t)lane < nmax) {
            nxt_pid = a.pair_prim[start + lane];
            nxt_rect = *reinterpret_cast<const int4 *>(recs + (size_t)nxt_pid * 8);
        }
        for (uint32_t b = 0; b < nmax; b += 64) {
            const uint32_t cur_pid = nxt_pid;
            const int4 cur_rect = nxt_rect;
            if (b + 64 + (uint32_t)lane < nmax) {
                nxt_pid = a.pair_prim[start + b + 64 + lane];
                nxt_rect = *reinterpret_cast<const int4 *>(recs + (size_t)nxt_pid * 8);
            }
            const bool rel = b + (uint32_t)lane < nmax && !(cur_rect.y < wx0 || cur_rect.x > wx0 + 7 ||
                                                              cur_rect.w < wy0 || cur_rect.z > wy0 + 7);
            uint64_t m = __ballot(rel);
            while (m != 0ull) {
                const int j = __builtin_ctzll(m);
                m &= m - 1ull;
                visit(b + (uint32_t)j + 1u, (uint32_t)__builtin_amdgcn_readlane((int)cur_pid, j));
            }
        }
    }
    // end of the replay: the pending hits, nearest first
    while (__ballot(buf.cnt > 0 && !done) != 0ull) {
        float gr[NGRAD];
#pragma unroll
        for (int f = 0; f < NGRAD; ++f) gr[f] = 0.0f;
        bool has = false;
        uint32_t g_pid = 0, g_pos = 0;
        if (buf.cnt > 0 && !done) has = pop_grad(gr, g_pid, g_pos);
        if (__ballot(has) != 0ull) flush_grads(gr, has, g_pid, g_pos);
    }
}

// Records a caller's event (if any) on the stream.
static inline hipError_t mark(hipEvent_t ev, hipStream_t stream)
{
    return ev ? hipEventRecord(ev, stream) : hipSuccess;
}

hipError_t launch_render_fwd(const RasterArgs &a, const RasterParams &p, const FwdOut &o, hipStream_t stream)
{
    const unsigned ntiles = (unsigned)(p.tiles_x * p.tiles_y);
    hipError_t e = mark(o.ev_begin, stream);
    if (e != hipSuccess) return e;
    const float4 *recs = reinterpret_cast<const float4 *>(a.records);
    if (ntiles == 0) {
    } else if (o.flags & QGS_RESORT) {
        if (o.curvature)
            hipLaunchKernelGGL((k_render_fwd_rs<true>), dim3(4 * ntiles), dim3(64), 0, stream, a, p, o, recs, o.steps);
        else
            hipLaunchKernelGGL((k_render_fwd_rs<false>), dim3(4 * ntiles), dim3(64), 0, stream, a, p, o, recs,
                               o.steps);
    } else {
        const dim3 grid(4 * ntiles), wave(64);
        const bool cnt = o.counters != nullptr;
        if (o.curvature && cnt)
            hipLaunchKernelGGL((k_render_fwd<true, true, true>), grid, wave, 0, stream, a, p, o, recs, o.steps);
        else if (o.curvature)
            hipLaunchKernelGGL((k_render_fwd<true, true, false>), grid, wave, 0, stream, a, p, o, recs, o.steps);
        else if (o.depth && cnt)
            hipLaunchKernelGGL((k_render_fwd<false, true, true>), grid, wave, 0, stream, a, p, o, recs, o.steps);
        else if (o.depth)
            hipLaunchKernelGGL((k_render_fwd<false, true, false>), grid, wave, 0, stream, a, p, o, recs, o.steps);
        else if (cnt)
            hipLaunchKernelGGL((k_render_fwd<false, false, true>), grid, wave, 0, stream, a, p, o, recs, o.steps);
        else
            hipLaunchKernelGGL((k_render_fwd<false, false, false>), grid, wave, 0, stream, a, p, o, recs, o.steps);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return mark(o.ev_end, stream);
}

// Backward work of each 8 x 8 block: the entries it visits, i.e. the set bits
// of its replay words; per block (cost[4 t + w], per_block) or per tile (the
// largest of its four, cost[t]).  One wave per tile, its lanes striding over
// each block's words.
__global__ __launch_bounds__(256) void k_bwd_cost(const uint32_t *ranges, const uint64_t *steps,
                                                  const uint32_t *step_count, uint32_t ntiles, uint32_t *cost,
                                                  bool per_block)
{
    const uint32_t t = blockIdx.x * 4u + (threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    if (t >= ntiles) return;  // whole wave
    const uint32_t start = ranges[2 * t], len = ranges[2 * t + 1] - start;
    const uint32_t nw_max = (len + 63u) >> 6;
    uint32_t c = 0;
    for (int w = 0; w < 4; ++w) {
        uint32_t nw = step_count[4 * t + w];
        nw = nw < nw_max ? nw : nw_max;
        const uint64_t *bm = steps + replay_base(start, len, (int)t, w);
        uint32_t v = 0;
        for (uint32_t k = lane; k < nw; k += 64u) v += (uint32_t)__popcll(bm[k]);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (per_block && lane == 0) cost[4 * t + w] = v;
        c = v > c ? v : c;
    }
    if (!per_block && lane == 0) cost[t] = c;
}

hipError_t launch_render_bwd(const RasterArgs &a_in, const RasterParams &p, const BwdIn &in, float *grad_rec,
                             float *pair_scratch, uint32_t *order_ws, int64_t n_prims, uint64_t capacity,
                             hipStream_t stream)
{
    const unsigned ntiles = (unsigned)(p.tiles_x * p.tiles_y);
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(grad_rec), 0u, (uint64_t)n_prims * 16, stream);
    if (e != hipSuccess) return e;
    RasterArgs a = a_in;
    if (ntiles > 0 && order_ws && in.steps) {
        // the 8 x 8 blocks (one-wave workgroups) in decreasing order of the
        // entries they visit
        const unsigned nu = 4u * ntiles;
        hipLaunchKernelGGL(k_bwd_cost, dim3((ntiles + 3) / 4), dim3(256), 0, stream, a.ranges, in.steps,
                           in.step_count, ntiles, order_ws, true);
        e = launch_tile_order(a.ranges, order_ws, nu, order_ws + nu, stream);
        if (e != hipSuccess) return e;
        a.block_order = order_ws + nu;
    }
    if (ntiles > 0 && pair_scratch) {
        e = launch_fill_u32(reinterpret_cast<uint32_t *>(pair_scratch), 0u, capacity * 64, stream);
        if (e != hipSuccess) return e;
    }
    const bool geo = in.dcurvature || in.dmedian || in.ddistortion;
    const bool det = pair_scratch != nullptr;
    const float4 *recs = reinterpret_cast<const float4 *>(a.records);
    const dim3 grid(4 * ntiles), wave(64);
    e = mark(in.ev_begin, stream);
    if (e != hipSuccess) return e;
    if (ntiles == 0) {
    } else if (in.flags & QGS_RESORT) {
        if (det && geo)
            hipLaunchKernelGGL((k_render_bwd_rs<true, true>), grid, wave, 0, stream, a, p, in, recs, grad_rec,
                               pair_scratch);
        else if (det)
            hipLaunchKernelGGL((k_render_bwd_rs<true, false>), grid, wave, 0, stream, a, p, in, recs, grad_rec,
                               pair_scratch);
        else if (geo)
            hipLaunchKernelGGL((k_render_bwd_rs<false, true>), grid, wave, 0, stream, a, p, in, recs, grad_rec,
                               pair_scratch);
        else
            hipLaunchKernelGGL((k_render_bwd_rs<false, false>), grid, wave, 0, stream, a, p, in, recs, grad_rec,
                               pair_scratch);
    } else {
        if (det && geo)
            hipLaunchKernelGGL((k_render_bwd<true, true>), grid, wave, 0, stream, a, p, in, recs, grad_rec,
                               pair_scratch);
        else if (det)
            hipLaunchKernelGGL((k_render_bwd<true, false>), grid, wave, 0, stream, a, p, in, recs, grad_rec,
                               pair_scratch);
        else if (geo)
            hipLaunchKernelGGL((k_render_bwd<false, true>), grid, wave, 0, stream, a, p, in, recs, grad_rec,
                               pair_scratch);
        else
            hipLaunchKernelGGL((k_render_bwd<false, false>), grid, wave, 0, stream, a, p, in, recs, grad_rec,
                               pair_scratch);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = mark(in.ev_end, stream);
    if (e != hipSuccess) return e;
    if (ntiles > 0 && det && n_prims > 0)
        hipLaunchKernelGGL(k_det_reduce, dim3((unsigned)((n_prims + 255) / 256)), dim3(256), 0, stream,
                           (const float *)pair_scratch, a.pair_offset, a.tiles, a.emit_to_sorted, n_prims, capacity,
                           grad_rec);
    return hipGetLastError();
}

}  // namespace qgs
