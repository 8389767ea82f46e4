// Device-side pieces shared by the rasterizer kernels: the primitive record,
// per-pixel ray set-up and the ray-paraboloid hit with root selection.
//
// Geometry is evaluated in a centre-relative frame.  With the centre at camera
// depth Zc and the pixel ray P(z) = z (xn, yn, 1), write z = Zc + s:
//     P - c_cam = m + s e,   m = Zc (dxp / fx, dyp / fy, 0),   e = (xn, yn, 1),
// where dxp = u + 0.5 - u_c is the pixel's offset from the projected centre.  The
// preprocess stores u_c as an integer plus a fraction, so dxp is exact to FP32
// rounding of a small number, and every term above is of the size of the
// primitive: FP32 keeps its relative precision where the camera-origin form
// ohat + t dhat would cancel |ohat| / sigma (10^3 and more) digits away.  In the
// local frame mhat = Rc^T m, ehat = Rc^T e, and substituting phat = mhat + s ehat
// into z = lambda1 x^2 + lambda2 y^2 (supplement, ray-splat intersection) gives
// A s^2 + B s + C = 0 with
//     A = l1 e0^2 + l2 e1^2,  B = 2 (l1 m0 e0 + l2 m1 e1) - e2,  C = l1 m0^2 + l2 m1^2 - m2.
// A is the unit-ray A of the paper scaled by |e|^2, so the small-|A| test uses
// A_eps |e|^2.  The discriminant is the same in s as in the camera-origin t.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qgs_internal.hpp"

namespace qgs {

constexpr int TILE = 16;
constexpr int BLOCK = 256;
constexpr int REC_WORDS = 32;
constexpr int NGRAD = 14;  // per-(tile, primitive) gradient fields

// record word offsets (layout documented in qgs.h)
enum : int {
    R_PX0 = 0, R_PX1 = 1, R_PY0 = 2, R_PY1 = 3,
    R_U = 4, R_HU = 5, R_V = 6, R_HV = 7,
    R_ZC = 8, R_L1 = 9, R_L2 = 10, R_OP = 11,
    R_K1 = 12, R_K2 = 13, R_CA = 14, R_CB = 15,
    R_ROT = 16, R_RGB = 25, R_CC = 28, R_CD = 29, R_CE = 30, R_ZL = 31
};

// slack of the FP32 conic pre-test (the conic is normalised to -1 at the
// projected centre and 0 on its boundary, and encloses the support with a
// relative margin of 2^-10)
constexpr float CONIC_SLACK = 1e-3f;

// gradient field order within a record gradient (16 floats, 14 used)
enum : int {
    G_PHI0 = 0, G_PHI1 = 1, G_PHI2 = 2, G_ZC = 3, G_UC = 4, G_VC = 5,
    G_L1 = 6, G_L2 = 7, G_K1 = 8, G_K2 = 9, G_OP = 10, G_R = 11, G_G = 12, G_B = 13
};

struct PixelRay {
    float fpx, fpy;   // integer pixel coordinates as floats
    float xn, yn;     // normalised image coordinates of the pixel centre
    float e2, enorm;  // |e|^2 and |e| for e = (xn, yn, 1)
};

__device__ inline PixelRay make_ray(int px, int py, const RasterParams &P)
{
    PixelRay r;
    r.fpx = (float)px;
    r.fpy = (float)py;
    r.xn = (((float)px + 0.5f) - P.cx) / P.fx;
    r.yn = (((float)py + 0.5f) - P.cy) / P.fy;
    r.e2 = __builtin_fmaf(r.xn, r.xn, __builtin_fmaf(r.yn, r.yn, 1.0f));
    r.enorm = __builtin_amdgcn_sqrtf(r.e2);
    return r;
}

// Geometry of one primitive, as loaded from its record.  The centre sits at
// (Xc, Yc, Zc + zl) with Zc its FP32 depth and zl the rounding residual; the
// pixel offsets are measured at depth Zc, so the offset from the centre has
// the camera-z component -zl, i.e. mz = -zl Rc^T z in the local frame.
struct Prim {
    float U, hu, V, hv, Zc, l1, l2, op, k1, k2, kx, ky;
    float R[9];  // camera-from-local rotation, row-major R[3 i + j]
    float mz[3];  // local-frame offset -zl Rc^T z
};

__device__ inline void load_prim(const float *w, const RasterParams &P, Prim &p)
{
    const float4 a = *reinterpret_cast<const float4 *>(w + 4);
    const float4 b = *reinterpret_cast<const float4 *>(w + 8);
    const float2 c = *reinterpret_cast<const float2 *>(w + 12);
    const float4 d = *reinterpret_cast<const float4 *>(w + 16);
    const float4 e = *reinterpret_cast<const float4 *>(w + 20);
    const float f = w[24];
    p.U = a.x; p.hu = a.y; p.V = a.z; p.hv = a.w;
    p.Zc = b.x; p.l1 = b.y; p.l2 = b.z; p.op = b.w;
    p.k1 = c.x; p.k2 = c.y;
    p.kx = p.Zc * P.ifx;
    p.ky = p.Zc * P.ify;
    p.R[0] = d.x; p.R[1] = d.y; p.R[2] = d.z; p.R[3] = d.w;
    p.R[4] = e.x; p.R[5] = e.y; p.R[6] = e.z; p.R[7] = e.w;
    p.R[8] = f;
    const float zl = w[R_ZL];
    p.mz[0] = -zl * p.R[6];
    p.mz[1] = -zl * p.R[7];
    p.mz[2] = -zl * p.R[8];
}

// Offset of the pixel centre from the projected centre, dxp = u + 0.5 - u_c,
// from the integer + fraction split of u_c (exact to the rounding of a small
// number), and the conic pre-test: false means the pixel's ray misses the
// ellipsoid that encloses the support.
__host__ __device__ inline bool conic_offsets(const float *w, const PixelRay &r, float &dxp, float &dyp)
{
    const float4 a = *reinterpret_cast<const float4 *>(w + 4);
    dxp = (r.fpx - a.x) + a.y;
    dyp = (r.fpy - a.z) + a.w;
    const float2 c1 = *reinterpret_cast<const float2 *>(w + 14);
    const float4 c2 = *reinterpret_cast<const float4 *>(w + 28);
    const float fx_ = __builtin_fmaf(c1.x, dxp, __builtin_fmaf(c1.y, dyp, c2.y));
    const float fy_ = __builtin_fmaf(c2.x, dyp, c2.z);
    const float f = __builtin_fmaf(fx_, dxp, __builtin_fmaf(fy_, dyp, -1.0f));
    return f <= CONIC_SLACK;
}

// Conservative test of the pre-test conic of conic_offsets against the 8 x 8
// pixel block whose top-left pixel is (bx, by): false only where no pixel of
// the block can pass the pre-test.  In pixel offsets from the projected
// centre the conic is f = a x^2 + b x y + c y^2 + d x + e y - 1, which is -1
// at the origin.  With a, c > 0, each connected part of {f <= t} either holds
// the origin (it is convex if f is) or is unbounded, so unless the origin lies
// in the block's box of offsets the set meets the box only across the box's
// boundary; on each of the four edges f is a convex quadratic of one variable,
// smallest at its clamped vertex.  FP32 rounding of these minima and of the
// per-pixel values stays below 2^-19 of the sum of absolute terms over the
// box, which the threshold adds.  (Host-callable, like conic_offsets, for the
// brute-force check of this bound over the pixels of a block.)
// The test of one block past its early outcomes (X0 .. Y1: the block's box of
// pixel offsets; a, c > 0; ha = 0.5 / a, hc = 0.5 / c)
__host__ __device__ inline bool conic_block_edges(float X0, float X1, float Y0, float Y1, float a, float b, float c,
                                                  float d, float e, float ha, float hc)
{
    float fmin;
    {
        // edges x = X0, X1: vertex at y = -(b X + e) / (2 c)
        const float y0 = fminf(fmaxf(-__builtin_fmaf(b, X0, e) * hc, Y0), Y1);
        const float y1 = fminf(fmaxf(-__builtin_fmaf(b, X1, e) * hc, Y0), Y1);
        const float f0 = __builtin_fmaf(__builtin_fmaf(a, X0, __builtin_fmaf(b, y0, d)), X0, __builtin_fmaf(__builtin_fmaf(c, y0, e), y0, -1.0f));
        const float f1 = __builtin_fmaf(__builtin_fmaf(a, X1, __builtin_fmaf(b, y1, d)), X1, __builtin_fmaf(__builtin_fmaf(c, y1, e), y1, -1.0f));
        // edges y = Y0, Y1: vertex at x = -(b Y + d) / (2 a)
        const float x0 = fminf(fmaxf(-__builtin_fmaf(b, Y0, d) * ha, X0), X1);
        const float x1 = fminf(fmaxf(-__builtin_fmaf(b, Y1, d) * ha, X0), X1);
        const float f2 = __builtin_fmaf(__builtin_fmaf(a, x0, __builtin_fmaf(b, Y0, d)), x0, __builtin_fmaf(__builtin_fmaf(c, Y0, e), Y0, -1.0f));
        const float f3 = __builtin_fmaf(__builtin_fmaf(a, x1, __builtin_fmaf(b, Y1, d)), x1, __builtin_fmaf(__builtin_fmaf(c, Y1, e), Y1, -1.0f));
        fmin = fminf(fminf(f0, f1), fminf(f2, f3));
    }
    const float xm = fmaxf(__builtin_fabsf(X0), __builtin_fabsf(X1)), ym = fmaxf(__builtin_fabsf(Y0), __builtin_fabsf(Y1));
    const float S = __builtin_fmaf(a * xm, xm, __builtin_fmaf(__builtin_fabsf(b) * xm, ym, __builtin_fmaf(c * ym, ym, __builtin_fmaf(__builtin_fabsf(d), xm, __builtin_fmaf(__builtin_fabsf(e), ym, 1.0f)))));
    return fmin <= __builtin_fmaf(0x1p-19f, S, CONIC_SLACK);
}

__host__ __device__ inline bool conic_meets_block(const float4 *__restrict__ rec, float bx, float by)
{
    const float4 cu = rec[1];  // record words 4..7: U, 0.5 - frac(u_c), V, 0.5 - frac(v_c)
    const float2 ab = *reinterpret_cast<const float2 *>(reinterpret_cast<const float *>(rec) + 14);
    const float4 cz = rec[7];  // words 28..31: c, d, e, zl
    const float X0 = (bx - cu.x) + cu.y, X1 = X0 + 7.0f;
    const float Y0 = (by - cu.z) + cu.w, Y1 = Y0 + 7.0f;
    const float a = ab.x, b = ab.y, c = cz.x, d = cz.y, e = cz.z;
    if (X0 <= 0.0f && X1 >= 0.0f && Y0 <= 0.0f && Y1 >= 0.0f) return true;
    if (!(a > 0.0f && c > 0.0f)) return true;
    const float ha = 0.5f / a, hc = 0.5f / c;  // once per batch entry: plain divisions
    return conic_block_edges(X0, X1, Y0, Y1, a, b, c, d, e, ha, hc);
}

// conic_meets_block for the four 8 x 8 blocks of the tile whose top-left pixel
// is (x0, y0), bit k for the block at (x0 + 8 (k & 1), y0 + 8 (k >> 1)); the
// same decisions, with the two divisions taken once
__device__ inline uint32_t conic_meets_blocks4(const float4 *__restrict__ rec, int x0, int y0)
{
    const float4 cu = rec[1];
    const float2 ab = *reinterpret_cast<const float2 *>(reinterpret_cast<const float *>(rec) + 14);
    const float4 cz = rec[7];
    const float a = ab.x, b = ab.y, c = cz.x, d = cz.y, e = cz.z;
    if (!(a > 0.0f && c > 0.0f)) return 0xFu;
    const float ha = 0.5f / a, hc = 0.5f / c;
    uint32_t m = 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float X0 = ((float)(x0 + 8 * (k & 1)) - cu.x) + cu.y, X1 = X0 + 7.0f;
        const float Y0 = ((float)(y0 + 8 * (k >> 1)) - cu.z) + cu.w, Y1 = Y0 + 7.0f;
        const bool in = (X0 <= 0.0f && X1 >= 0.0f && Y0 <= 0.0f && Y1 >= 0.0f) ||
                        conic_block_edges(X0, X1, Y0, Y1, a, b, c, d, e, ha, hc);
        m |= (in ? 1u : 0u) << k;
    }
    return m;
}

// arc-length factor g(u) = l / rho for u = 2 |a| rho (geodesic equation, Sec.
// 3.2) and its derivative.  g and h = g' / u are analytic in v = u^2 with the
// nearest singularity at v = -1, so for u <= 1 they are polynomials in v from
// Chebyshev interpolation (gen_arc_poly.py: relative error 9.5e-8 and 1.3e-7
// in FP32, no transcendental and no branch between series and closed form);
// above, the closed form.
// highest degree first
constexpr float G_POLY[7] = {-0.00024931385996751487f, 0.0013209348544478416f, -0.003705431940034032f,
                             0.008731926791369915f, -0.02496938779950142f, 0.16666482388973236f, 1.0f};
constexpr float H_POLY[9] = {0.000549668213352561f, -0.0031673528719693422f, 0.008671113289892673f,
                             -0.015905411913990974f, 0.023939577862620354f, -0.03455767035484314f,
                             0.053556177765131f, -0.09999944269657135f, 0.3333333432674408f};

__device__ inline float gfun(float u)
{
    if (u <= 1.0f) {
        const float v = u * u;
        float acc = G_POLY[0];
#pragma unroll
        for (int k = 1; k < 7; ++k) acc = __builtin_fmaf(acc, v, G_POLY[k]);
        return acc;
    }
    const float s = __builtin_amdgcn_sqrtf(__builtin_fmaf(u, u, 1.0f));
    const float ash = __logf(u + s);
    return (ash + u * s) * __builtin_amdgcn_rcpf(2.0f * u);
}

__device__ inline float gprime(float u)
{
    if (u <= 1.0f) {
        const float v = u * u;
        float acc = H_POLY[0];
#pragma unroll
        for (int k = 1; k < 9; ++k) acc = __builtin_fmaf(acc, v, H_POLY[k]);
        return acc * u;
    }
    const float s = __builtin_amdgcn_sqrtf(__builtin_fmaf(u, u, 1.0f));
    const float ash = __logf(u + s);
    return (u * s - ash) * __builtin_amdgcn_rcpf(2.0f * u * u);
}

// Hardware reciprocal and square root (about 1 ulp) are used throughout the
// rasterizer; forward and backward share this code, so both take the same
// decisions from the same values.

// Intersection state of one (pixel, primitive) pair.
struct Hit {
    float dxp, dyp, mx, my;
    float m0, m1, m2, e0, e1, e2;
    float A, B, C;
    float s, x, y, Q, rho2, h, u, g, E;
    bool linear;
};

// Ray-paraboloid intersection with the near/far selection and the k_sigma
// geodesic cut-off (Sec. 3.2.1), from the pixel offsets of conic_offsets.
// Returns true with the accepted hit in H.
__device__ inline bool ray_hit(const Prim &p, const PixelRay &r, const RasterParams &P, float dxp, float dyp, Hit &H)
{
    H.dxp = dxp;
    H.dyp = dyp;
    H.mx = p.kx * H.dxp;
    H.my = p.ky * H.dyp;
    H.m0 = __builtin_fmaf(p.R[0], H.mx, __builtin_fmaf(p.R[3], H.my, p.mz[0]));
    H.m1 = __builtin_fmaf(p.R[1], H.mx, __builtin_fmaf(p.R[4], H.my, p.mz[1]));
    H.m2 = __builtin_fmaf(p.R[2], H.mx, __builtin_fmaf(p.R[5], H.my, p.mz[2]));
    H.e0 = __builtin_fmaf(p.R[0], r.xn, __builtin_fmaf(p.R[3], r.yn, p.R[6]));
    H.e1 = __builtin_fmaf(p.R[1], r.xn, __builtin_fmaf(p.R[4], r.yn, p.R[7]));
    H.e2 = __builtin_fmaf(p.R[2], r.xn, __builtin_fmaf(p.R[5], r.yn, p.R[8]));
    const float l1e0 = p.l1 * H.e0, l2e1 = p.l2 * H.e1;
    H.A = __builtin_fmaf(l1e0, H.e0, l2e1 * H.e1);
    H.B = 2.0f * __builtin_fmaf(l1e0, H.m0, l2e1 * H.m1) - H.e2;
    H.C = __builtin_fmaf(p.l1 * H.m0, H.m0, __builtin_fmaf(p.l2 * H.m1, H.m1, -H.m2));

    // roots q / A and C / q with q = -(B + sgn(B) sqrt(D)) / 2; for |A| <
    // A_eps (the paper's nearly flat case) the root q / A, which diverges as A
    // -> 0, is dropped and C / q -- the tangent-plane intersection at A = 0 --
    // is the one candidate.  Evaluated relative to the centre, C / q needs no
    // cancellation of A terms, so the hit stays exact to rounding where A is
    // small only through cancellation (saddles seen along an asymptote).
    float cand0, cand1;
    int nc = 0;
    H.linear = __builtin_fabsf(H.A) < P.A_eps * r.e2;
    const float D = __builtin_fmaf(H.B, H.B, -4.0f * H.A * H.C);
    if (D >= 0.0f) {
        const float sq = __builtin_amdgcn_sqrtf(D);
        const float q = -0.5f * (H.B + (H.B >= 0.0f ? sq : -sq));
        if (q == 0.0f) {
            cand0 = cand1 = 0.0f;
            nc = H.linear ? 0 : 2;
        } else {
            const float r2 = H.C * __builtin_amdgcn_rcpf(q);
            if (H.linear) {
                cand0 = r2;
                nc = 1;
            } else {
                const float r1 = q * __builtin_amdgcn_rcpf(H.A);
                cand0 = fminf(r1, r2);
                cand1 = fmaxf(r1, r2);
                nc = 2;
            }
        }
    }
    // unrolled: a loop over the two candidates costs selects and branches per step
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (k >= nc) break;
        const float s = k == 0 ? cand0 : cand1;
        const float z = p.Zc + s;
        if (!(z > P.near_plane)) continue;
        const float x = __builtin_fmaf(s, H.e0, H.m0);
        const float y = __builtin_fmaf(s, H.e1, H.m1);
        const float xx = x * x, yy = y * y;
        const float Q = __builtin_fmaf(p.k1, xx, p.k2 * yy);
        if (!(Q <= P.k2)) continue;  // g >= 1, so E >= Q
        const float rho2 = xx + yy;
        const float h = __builtin_fmaf(p.l1, xx, p.l2 * yy);
        const float u = rho2 > 0.0f ? 2.0f * __builtin_fabsf(h) * __builtin_amdgcn_rsqf(rho2) : 0.0f;
        const float g = gfun(u);
        const float E = g * g * Q;
        if (E <= P.k2) {
            H.s = s; H.x = x; H.y = y; H.Q = Q; H.rho2 = rho2; H.h = h; H.u = u; H.g = g; H.E = E;
            return true;
        }
    }
    return false;
}

// Unit normal of the paraboloid at the hit, (-2 l1 x, -2 l2 y, 1) normalised,
// flipped to face the camera (n . ehat <= 0); returns the flip sign.
__device__ inline float hit_normal(const Prim &p, const Hit &H, float nl[3], float &inv_len)
{
    const float v0 = -2.0f * p.l1 * H.x, v1 = -2.0f * p.l2 * H.y;
    inv_len = __builtin_amdgcn_rsqf(__builtin_fmaf(v0, v0, __builtin_fmaf(v1, v1, 1.0f)));
    nl[0] = v0 * inv_len;
    nl[1] = v1 * inv_len;
    nl[2] = inv_len;
    const float dot = __builtin_fmaf(v0, H.e0, __builtin_fmaf(v1, H.e1, H.e2));
    return dot > 0.0f ? -1.0f : 1.0f;
}

// Gaussian curvature of the paraboloid at the hit (curvature equation,
// Sec. 3.2.1): 4 l1 l2 / (1 + 4 l1^2 x^2 + 4 l2^2 y^2)^2, where inv_len from
// hit_normal is 1 / sqrt of the bracket.
__device__ inline float hit_curvature(const Prim &p, float inv_len)
{
    const float i2 = inv_len * inv_len;
    return 4.0f * p.l1 * p.l2 * (i2 * i2);
}

}  // namespace qgs
