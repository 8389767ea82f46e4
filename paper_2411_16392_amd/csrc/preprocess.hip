// Per-primitive preprocess (projection, culling, conservative screen bounds)
// and its backward (record gradients -> scene parameter gradients).
//
// The forward runs in FP64 with a fixed operation order: its discrete outputs
// (cull flag, depth key, rectangles) must be reproducible bit for bit, and the
// projected centre is split into integer and fractional pixel parts at full
// precision for the rasterizer's centre-relative frame.  Contraction is off
// for this file; fma() appears only where the order of operations is specified.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "qgs_device.hpp"
#include "qgs_internal.hpp"
#include "qgs_keys.hpp"

#pragma clang fp contract(off)

namespace qgs {

__device__ inline bool finite_f(float v) { return __builtin_isfinite(v); }

// Real spherical harmonics of degree <= 3 at the unit direction (x, y, z)
// (normalisation sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!), Condon-Shortley phase,
// order l = 0..3, m = -l..l), and with dY their gradients; the colour model of
// 3DGS that the paper keeps (Sec. 3).
__device__ inline void sh_basis(int deg, double x, double y, double z, double *Y, double (*dY)[3])
{
    const double pi = 3.14159265358979323846;
    const double c0 = 0.5 * sqrt(1.0 / pi), c1 = sqrt(3.0 / (4.0 * pi));
    const double c2a = 0.5 * sqrt(15.0 / pi), c2b = 0.25 * sqrt(5.0 / pi), c2c = 0.25 * sqrt(15.0 / pi);
    const double c3a = 0.25 * sqrt(35.0 / (2.0 * pi)), c3b = 0.5 * sqrt(105.0 / pi);
    const double c3c = 0.25 * sqrt(21.0 / (2.0 * pi)), c3d = 0.25 * sqrt(7.0 / pi), c3e = 0.25 * sqrt(105.0 / pi);
    for (int k = 0; k < 16; ++k) {
        Y[k] = 0.0;
        if (dY) dY[k][0] = dY[k][1] = dY[k][2] = 0.0;
    }
    Y[0] = c0;
    if (deg >= 1) {
        Y[1] = -c1 * y;
        Y[2] = c1 * z;
        Y[3] = -c1 * x;
        if (dY) {
            dY[1][1] = -c1;
            dY[2][2] = c1;
            dY[3][0] = -c1;
        }
    }
    if (deg >= 2) {
        const double xx = x * x, yy = y * y, zz = z * z;
        Y[4] = c2a * x * y;
        Y[5] = -c2a * y * z;
        Y[6] = c2b * (2 * zz - xx - yy);
        Y[7] = -c2a * x * z;
        Y[8] = c2c * (xx - yy);
        if (dY) {
            dY[4][0] = c2a * y; dY[4][1] = c2a * x;
            dY[5][1] = -c2a * z; dY[5][2] = -c2a * y;
            dY[6][0] = -2 * c2b * x; dY[6][1] = -2 * c2b * y; dY[6][2] = 4 * c2b * z;
            dY[7][0] = -c2a * z; dY[7][2] = -c2a * x;
            dY[8][0] = 2 * c2c * x; dY[8][1] = -2 * c2c * y;
        }
    }
    if (deg >= 3) {
        const double xx = x * x, yy = y * y, zz = z * z;
        Y[9] = -c3a * y * (3 * xx - yy);
        Y[10] = c3b * x * y * z;
        Y[11] = -c3c * y * (4 * zz - xx - yy);
        Y[12] = c3d * z * (2 * zz - 3 * xx - 3 * yy);
        Y[13] = -c3c * x * (4 * zz - xx - yy);
        Y[14] = c3e * z * (xx - yy);
        Y[15] = -c3a * x * (xx - 3 * yy);
        if (dY) {
            dY[9][0] = -c3a * 6 * x * y; dY[9][1] = -c3a * (3 * xx - 3 * yy);
            dY[10][0] = c3b * y * z; dY[10][1] = c3b * x * z; dY[10][2] = c3b * x * y;
            dY[11][0] = c3c * 2 * x * y; dY[11][1] = -c3c * (4 * zz - xx - 3 * yy); dY[11][2] = -c3c * 8 * y * z;
            dY[12][0] = -c3d * 6 * x * z; dY[12][1] = -c3d * 6 * y * z; dY[12][2] = c3d * (6 * zz - 3 * xx - 3 * yy);
            dY[13][0] = -c3c * (4 * zz - 3 * xx - yy); dY[13][1] = c3c * 2 * x * y; dY[13][2] = -c3c * 8 * x * z;
            dY[14][0] = c3e * 2 * x * z; dY[14][1] = -c3e * 2 * y * z; dY[14][2] = c3e * (xx - yy);
            dY[15][0] = -c3a * (3 * xx - 3 * yy); dY[15][1] = c3a * 6 * x * y;
        }
    }
}

// unit direction from the camera centre -R^T t to the world point c, and its length
__device__ inline void view_dir(const qgs_camera &cam, const float *c, double d[3], double &r)
{
    double v[3];
    for (int j = 0; j < 3; ++j)
        v[j] = (double)c[j] + ((double)cam.R[j] * cam.t[0] + (double)cam.R[3 + j] * cam.t[1] + (double)cam.R[6 + j] * cam.t[2]);
    r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int j = 0; j < 3; ++j) d[j] = v[j] / r;
}

// Local box [-hx, hx] x [-hy, hy] x [zlo, zhi] holding every point of the
// support (accepted hits, l <= k sigma(theta)), inflated by 2^-10 (and z by a
// further k max(sigma) / 1024).  FP64, fixed operation order, no contraction.
//  default: the arc-length factor is >= 1, so Q <= k^2: |x| <= k s1,
//           |y| <= k s2; the height lambda1 x^2 + lambda2 y^2 lies between
//           the extremes of {0, k^2 lambda_i s_i^2} and |z| <= l <= k max(s).
//  tight:   the arc is at least its chord, so rho^2 + z^2 <= k^2 sigma(theta)^2,
//           hence Q + z^2 / sm^2 <= k^2 (sm = max(s1, s2)).  |x|'s bound is the
//           largest X = x^2 with min over Y = y^2 >= 0 of
//           X/s1^2 + Y/s2^2 + (l1 X + l2 Y)^2 / sm^2 <= k^2: at Y = 0 (root of a
//           quadratic) unless the curvatures have opposite signs and that root
//           passes the point Xc beyond which a Y > 0 lowers the height, where
//           the minimum is linear in X.  The height solves rho^2 (1 + a^2 rho^2)
//           <= k^2 sigma^2 with a sigma^2 between the lambda_i s_i^2.
__device__ inline double chord_axis_sq(double sa, double sb, double la, double lb, double sm, double k2)
{
    const double ra = ((la * sa) * sa) / sm;
    const double Xe = ((2.0 * k2) * (sa * sa)) / (1.0 + sqrt(1.0 + (4.0 * k2) * (ra * ra)));
    if (la * lb < 0.0) {
        const double rb = (fabs(lb) * sb) * sb;
        const double Xc = (sm * sm) / ((2.0 * fabs(la)) * rb);
        if (Xe > Xc) return (k2 + (sm * sm) / (4.0 * (rb * rb))) / (1.0 / (sa * sa) + fabs(la) / rb);
    }
    return Xe;
}

__device__ inline double chord_height(double m, double sm, double k2)
{
    const double r = m / sm;
    return ((2.0 * k2) * m) / (1.0 + sqrt(1.0 + (4.0 * k2) * (r * r)));
}

// Cut-off for the bounds of a primitive that blends only where alpha =
// min(alpha_max, o G) >= alpha_min, i.e. G >= alpha_min / o, i.e.
// E <= 2 ln(o / alpha_min): the smaller of k and sqrt(2 ln x), x = o /
// alpha_min, with ln x bounded from above by 64 (x^(1/64) - 1) (ln y <= y - 1
// at y = x^(1/64); six correctly rounded square roots) and a relative margin
// of 2^-20.  k itself when alpha_min is not positive or x <= 1.
__device__ inline double blend_k(float op, float alpha_min, float k_sigma)
{
    const double k = k_sigma;
    if (!(alpha_min > 0.0f)) return k;
    const double x = (double)op / (double)alpha_min;
    if (!(x > 1.0)) return k;
    double r = x;
    for (int i = 0; i < 6; ++i) r = sqrt(r);
    const double e2 = (128.0 * (r - 1.0)) * (1.0 + 1.0 / 1048576.0);
    return e2 < k * k ? sqrt(e2) : k;
}

__device__ inline void local_box(double s1, double s2, double l1, double l2, double k, bool tight, double &hx,
                                 double &hy, double &zlo, double &zhi)
{
    const double infl = 1.0 + 1.0 / 1024.0;
    const double k2 = k * k;
    const double smax = s1 > s2 ? s1 : s2;
    const double zcap = k * smax;
    const double m1 = (l1 * s1) * s1, m2 = (l2 * s2) * s2;
    double lo = 0.0, hi = 0.0;
    lo = m1 < lo ? m1 : lo; lo = m2 < lo ? m2 : lo;
    hi = m1 > hi ? m1 : hi; hi = m2 > hi ? m2 : hi;
    double ex = k * s1, ey = k * s2;
    if (tight) {
        const double bx = sqrt(chord_axis_sq(s1, s2, l1, l2, smax, k2));
        const double by = sqrt(chord_axis_sq(s2, s1, l2, l1, smax, k2));
        ex = bx < ex ? bx : ex;
        ey = by < ey ? by : ey;
        zlo = -chord_height(-lo, smax, k2);
        zhi = chord_height(hi, smax, k2);
    } else {
        zlo = k2 * lo;
        zhi = k2 * hi;
    }
    if (zlo < -zcap) zlo = -zcap;
    if (zhi > zcap) zhi = zcap;
    const double zpad = zcap / 1024.0;
    hx = ex * infl;
    hy = ey * infl;
    zlo = zlo * infl - zpad;
    zhi = zhi * infl + zpad;
}

// Everything of one primitive except its tile count: the record, depth key,
// rectangle and conic; `cl` receives the tile rectangle and conic for the
// tile tests (nx = 0 when it covers no tile).
__device__ inline void preprocess_one(const PreprocessArgs &a, int64_t p, ConicLane &cl)
{
    float4 *rec = reinterpret_cast<float4 *>(reinterpret_cast<char *>(a.records) + p * 128);
    int32_t *rt = a.rect + 4 * p;
    const float4 empty_rect = make_float4(__int_as_float(0), __int_as_float(-1), __int_as_float(0), __int_as_float(-1));

    const float cf0 = a.center[3 * p], cf1 = a.center[3 * p + 1], cf2 = a.center[3 * p + 2];
    const float qw = a.quat[4 * p], qx = a.quat[4 * p + 1], qy = a.quat[4 * p + 2], qz = a.quat[4 * p + 3];
    const float sf1 = a.scale[2 * p], sf2 = a.scale[2 * p + 1];
    const float lf1 = a.curv[2 * p], lf2 = a.curv[2 * p + 1];
    const float op = a.opacity[p];
    float r0, r1, r2;
    if (a.sh) {
        // view-dependent colour: max(0, sum_k sh[k] Y_k(d) + 1/2)
        double d[3], r, Y[16];
        view_dir(a.cam, a.center + 3 * p, d, r);
        sh_basis(a.sh_degree, d[0], d[1], d[2], Y, nullptr);
        const int K = (a.sh_degree + 1) * (a.sh_degree + 1);
        const float *cf = a.sh + (size_t)3 * K * p;
        double acc[3] = {0.5, 0.5, 0.5};
        for (int k = 0; k < K; ++k)
            for (int ch = 0; ch < 3; ++ch) acc[ch] += (double)cf[3 * k + ch] * Y[k];
        r0 = (float)(acc[0] > 0.0 ? acc[0] : 0.0);
        r1 = (float)(acc[1] > 0.0 ? acc[1] : 0.0);
        r2 = (float)(acc[2] > 0.0 ? acc[2] : 0.0);
    } else {
        r0 = a.rgb[3 * p];
        r1 = a.rgb[3 * p + 1];
        r2 = a.rgb[3 * p + 2];
    }

    bool ok = finite_f(cf0) && finite_f(cf1) && finite_f(cf2) && finite_f(qw) && finite_f(qx) && finite_f(qy) &&
              finite_f(qz) && finite_f(sf1) && finite_f(sf2) && finite_f(lf1) && finite_f(lf2) && finite_f(op) &&
              finite_f(r0) && finite_f(r1) && finite_f(r2) && sf1 > 0.0f && sf2 > 0.0f;
    const double w = qw, x = qx, y = qy, z = qz;
    const double ww = w * w, xx = x * x, yy = y * y, zz = z * z;
    const double qn = (ww + xx) + (yy + zz);
    ok = ok && qn > 0.0;

    double cc[3] = {0.0, 0.0, 0.0};
    float zf = 0.0f;
    if (ok) {
        for (int i = 0; i < 3; ++i)
            cc[i] = fma((double)a.cam.R[3 * i], (double)cf0,
                        fma((double)a.cam.R[3 * i + 1], (double)cf1, fma((double)a.cam.R[3 * i + 2], (double)cf2, (double)a.cam.t[i])));
        zf = (float)cc[2];
        ok = zf > a.near_plane;
    }
    if (!ok) {
        rec[0] = empty_rect;
        a.depth_key[p] = 0u;
        rt[0] = 0; rt[1] = 0; rt[2] = -1; rt[3] = -1;
        return;
    }

    // rotation of q / |q| from the unnormalised quaternion
    const double s = 2.0 / qn;
    const double xy = x * y, xz = x * z, yz = y * z, wx = w * x, wy = w * y, wz = w * z;
    double Rm[9];
    Rm[0] = 1.0 - s * (yy + zz); Rm[1] = s * (xy - wz);        Rm[2] = s * (xz + wy);
    Rm[3] = s * (xy + wz);       Rm[4] = 1.0 - s * (xx + zz);  Rm[5] = s * (yz - wx);
    Rm[6] = s * (xz - wy);       Rm[7] = s * (yz + wx);        Rm[8] = 1.0 - s * (xx + yy);
    double Rc[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            Rc[3 * i + j] = fma((double)a.cam.R[3 * i], Rm[j],
                                fma((double)a.cam.R[3 * i + 1], Rm[3 + j], (double)a.cam.R[3 * i + 2] * Rm[6 + j]));

    // local box of the support (see qgs_preprocess in qgs.h)
    const double s1 = sf1, s2 = sf2, l1 = lf1, l2 = lf2;
    double hx, hy, zlo, zhi;
    local_box(s1, s2, l1, l2, a.tight ? blend_k(op, a.alpha_min, a.k_sigma) : (double)a.k_sigma, a.tight != 0, hx, hy,
              zlo, zhi);

    const double fx = a.cam.fx, fy = a.cam.fy, cxp = a.cam.cx, cyp = a.cam.cy;
    const double near_d = a.near_plane;
    // the box's corners in camera space; the rectangle bounds the projection
    // of the part of the box in front of the near plane (hits need a camera
    // depth above it): the corners in front and, where an edge crosses the
    // plane, the crossing point
    double Pc[8][3];
    uint32_t front = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const double X = (c & 1) ? hx : -hx, Y = (c & 2) ? hy : -hy, Z = (c & 4) ? zhi : zlo;
        for (int i = 0; i < 3; ++i) Pc[c][i] = fma(Rc[3 * i], X, fma(Rc[3 * i + 1], Y, fma(Rc[3 * i + 2], Z, cc[i])));
        if (Pc[c][2] > near_d) front |= 1u << c;
    }
    const bool behind = front != 0xFFu;
    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (!((front >> c) & 1u)) continue;
        const double u = fma(fx, Pc[c][0] / Pc[c][2], cxp), v = fma(fy, Pc[c][1] / Pc[c][2], cyp);
        umin = u < umin ? u : umin;
        umax = u > umax ? u : umax;
        vmin = v < vmin ? v : vmin;
        vmax = v > vmax ? v : vmax;
    }
    if (behind && front != 0u) {
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            // edge e joins corner c and c | bit, c without that bit
            const int bit = 1 << (e >> 2), low = e & 3;
            const int c0 = bit == 1 ? (low << 1) : (bit == 2 ? ((low & 2) << 1) | (low & 1) : low);
            const int c1 = c0 | bit;
            const bool f0 = (front >> c0) & 1u, f1 = (front >> c1) & 1u;
            if (f0 == f1) continue;
            const double *F = f0 ? Pc[c0] : Pc[c1], *B = f0 ? Pc[c1] : Pc[c0];
            const double sc = (F[2] - near_d) / (F[2] - B[2]);
            const double xq = F[0] + sc * (B[0] - F[0]), yq = F[1] + sc * (B[1] - F[1]);
            const double u = fma(fx, xq / near_d, cxp), v = fma(fy, yq / near_d, cyp);
            umin = u < umin ? u : umin;
            umax = u > umax ? u : umax;
            vmin = v < vmin ? v : vmin;
            vmax = v > vmax ? v : vmax;
        }
    }
    const int W = a.cam.width, H = a.cam.height;
    int px0, px1, py0, py1;
    bool empty = false;
    if (front == 0u) {
        // the whole box is behind the near plane
        empty = true;
        px0 = py0 = 0;
        px1 = py1 = -1;
    } else {
        const double pad_px = 1.0 / 64.0;
        const double a0 = (umin - 0.5) - pad_px, a1 = (umax - 0.5) + pad_px;
        const double b0 = (vmin - 0.5) - pad_px, b1 = (vmax - 0.5) + pad_px;
        if (a1 < 0.0 || a0 > (double)(W - 1) || b1 < 0.0 || b0 > (double)(H - 1)) {
            empty = true;
            px0 = py0 = 0;
            px1 = py1 = -1;
        } else {
            px0 = a0 <= 0.0 ? 0 : (int)ceil(a0);
            px1 = a1 >= (double)(W - 1) ? W - 1 : (int)floor(a1);
            py0 = b0 <= 0.0 ? 0 : (int)ceil(b0);
            py1 = b1 >= (double)(H - 1) ? H - 1 : (int)floor(b1);
            empty = px0 > px1 || py0 > py1;
        }
    }
    a.depth_key[p] = __float_as_uint(zf);
    if (empty) {
        rec[0] = empty_rect;
        rt[0] = 0; rt[1] = 0; rt[2] = -1; rt[3] = -1;
        return;
    }
    const int tx0 = px0 / TILE, tx1 = px1 / TILE, ty0 = py0 / TILE, ty1 = py1 / TILE;
    rt[0] = tx0; rt[1] = ty0; rt[2] = tx1; rt[3] = ty1;
    if (a.frame) {
        // camera frame for the per-tile sort depth (projected vertex as for the record)
        double *F = a.frame + 16 * p;
        for (int i = 0; i < 3; ++i) F[i] = cc[i];
        for (int i = 0; i < 9; ++i) F[3 + i] = Rc[i];
        F[12] = fma(fx, cc[0] / cc[2], cxp);
        F[13] = fma(fy, cc[1] / cc[2], cyp);
        F[14] = l1;
        F[15] = l2;
    }

    // Ellipsoid enclosing the box's elliptic cylinder {x^2/hx^2 + y^2/hy^2 <= 1,
    // z in [zlo, zhi]}: squared semi-axes hx^2/(1-t), hy^2/(1-t), hz^2/t about
    // the mid-height, t = hz / (hz + min(hx, hy)); its image in the camera is
    // the conic (gamma - 1) A - w w^T with A = Rc diag(1/q) Rc^T, w = A c_e,
    // gamma = c_e^T w.
    double C[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    bool cok = false;
    if (!behind) {
        const double hz = 0.5 * (zhi - zlo), zm = 0.5 * (zlo + zhi);
        const double mxy = hx < hy ? hx : hy;
        const double t = hz / (hz + mxy);
        const double q[3] = {(hx * hx) / (1.0 - t), (hy * hy) / (1.0 - t), (hz * hz) / t};
        const double iq[3] = {1.0 / q[0], 1.0 / q[1], 1.0 / q[2]};
        double ce[3];
        for (int i = 0; i < 3; ++i) ce[i] = fma(Rc[3 * i + 2], zm, cc[i]);
        double A[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                A[i][j] = fma(Rc[3 * i] * iq[0], Rc[3 * j],
                              fma(Rc[3 * i + 1] * iq[1], Rc[3 * j + 1], (Rc[3 * i + 2] * iq[2]) * Rc[3 * j + 2]));
        double w3[3];
        for (int i = 0; i < 3; ++i) w3[i] = fma(A[i][0], ce[0], fma(A[i][1], ce[1], A[i][2] * ce[2]));
        const double gm1 = fma(ce[0], w3[0], fma(ce[1], w3[1], ce[2] * w3[2])) - 1.0;
        const int ii[6] = {0, 0, 1, 0, 1, 2}, jj[6] = {0, 1, 1, 2, 2, 2};
        for (int k = 0; k < 6; ++k) C[k] = fma(gm1, A[ii[k]][jj[k]], -(w3[ii[k]] * w3[jj[k]]));
        const double S33 = fma(q[0] * Rc[6], Rc[6], fma(q[1] * Rc[7], Rc[7], (q[2] * Rc[8]) * Rc[8]));
        const double dz = ce[2] - near_d;
        cok = dz > 0.0 && dz * dz > S33;
    }
    for (int i = 0; i < 6; ++i) cl.C[i] = C[i];
    if (cok) conic_center(C, cl.mx, cl.my, cl.ia, cl.ic);
    cl.cok = cok ? 1u : 0u;
    cl.tx0 = tx0;
    cl.ty0 = ty0;
    cl.nx = tx1 - tx0 + 1;
    cl.ny = ty1 - ty0 + 1;

    // projected centre split into integer + fraction, and the record.  The
    // record's centre depth zf is FP32; the centre is projected at that depth,
    // so that (u_c, v_c, zf) describe the point P0 = (Xc, Yc, zf) exactly, and
    // the rounding residual zl = Zc - zf (the true centre is P0 + zl z) goes
    // into the record as well: the rasterizers then measure offsets from the
    // true centre, where an FP32 depth alone would move the primitive by up to
    // half an ulp of Zc -- at grazing incidence enough to shift its hits by
    // 1e-3 of sigma.
    const double zl = cc[2] - (double)zf;
    const double uc = fma(fx, cc[0] / (double)zf, cxp), vc = fma(fy, cc[1] / (double)zf, cyp);
    const double U = floor(uc), V = floor(vc);
    const float hu = (float)(0.5 - (uc - U)), hv = (float)(0.5 - (vc - V));
    // the conic in pixels relative to the projected centre, scaled so that
    // f = -1 at the centre (which is inside: the local origin is in the box)
    float cA = 0.0f, cB = 0.0f, cC = 0.0f, cD = 0.0f, cE = 0.0f;
    if (cok) {
        const double xi = (uc - cxp) / fx, eta = (vc - cyp) / fy;
        const double f0 = conic_eval(C, xi, eta);
        if (f0 < 0.0) {
            const double sc = -1.0 / f0, ifx = 1.0 / fx, ify = 1.0 / fy;
            cA = (float)(C[0] * ifx * ifx * sc);
            cB = (float)(2.0 * C[1] * ifx * ify * sc);
            cC = (float)(C[2] * ify * ify * sc);
            cD = (float)(2.0 * (C[0] * xi + C[1] * eta + C[3]) * ifx * sc);
            cE = (float)(2.0 * (C[1] * xi + C[2] * eta + C[4]) * ify * sc);
        }
    }
    rec[0] = make_float4(__int_as_float(px0), __int_as_float(px1), __int_as_float(py0), __int_as_float(py1));
    rec[1] = make_float4((float)U, hu, (float)V, hv);
    rec[2] = make_float4(zf, lf1, lf2, op);
    rec[3] = make_float4((float)(1.0 / (s1 * s1)), (float)(1.0 / (s2 * s2)), cA, cB);
    rec[4] = make_float4((float)Rc[0], (float)Rc[1], (float)Rc[2], (float)Rc[3]);
    rec[5] = make_float4((float)Rc[4], (float)Rc[5], (float)Rc[6], (float)Rc[7]);
    rec[6] = make_float4((float)Rc[8], r0, r1, r2);
    rec[7] = make_float4(cC, cD, cE, (float)zl);
}

// One-wave workgroups; 4 waves per SIMD requested (128 VGPRs, 40 bytes of
// spills per lane) runs 3% faster than the 3 the unconstrained 144 VGPRs allow.
__global__ __launch_bounds__(64, 4) void k_preprocess(PreprocessArgs a)
{
    __shared__ ConicLane s_cl[64];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    ConicLane cl = {};
    if (p < a.n) preprocess_one(a, p, cl);
    // every thread of the workgroup takes part in the tile tests
    uint64_t mask = 0ull;
    const uint32_t cnt = wave_conic_tiles<false>(s_cl + (threadIdx.x & ~63u), cl, a.cam, 0, nullptr, nullptr, nullptr,
                                                 nullptr, nullptr, 0.0, &mask);
    if (p < a.n) {
        a.tiles[p] = cnt;
        // the conic, its validity and the decisions for the emission (the bits
        // of a 64-bit integer), the whole 64-byte row in one go (zeros for a
        // culled primitive)
        double *cq = a.conic + 8 * p;
        for (int i = 0; i < 6; ++i) cq[i] = cl.C[i];
        cq[6] = (cl.cok & 1u) ? 1.0 : 0.0;
        reinterpret_cast<uint64_t *>(cq)[7] = mask;
    }
}

// Chain rule from the record gradients (rotation as a right perturbation
// Rc exp([phi]x), centre depth, projected centre, curvatures, inverse variances,
// opacity, colour) to the scene parameters.
__global__ __launch_bounds__(256) void k_preprocess_bwd(PreprocessBwdArgs a)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const float *g = a.grad_rec + 16 * p;
    double gc[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, gs[2] = {0, 0};
    const bool active = a.tiles[p] != 0u;
    if (active) {
        const float cf0 = a.center[3 * p], cf1 = a.center[3 * p + 1], cf2 = a.center[3 * p + 2];
        double cc[3];
        for (int i = 0; i < 3; ++i)
            cc[i] = fma((double)a.cam.R[3 * i], (double)cf0,
                        fma((double)a.cam.R[3 * i + 1], (double)cf1, fma((double)a.cam.R[3 * i + 2], (double)cf2, (double)a.cam.t[i])));
        const double gZ = g[G_ZC], guc = g[G_UC], gvc = g[G_VC];
        // u_c = fx Xc / Zc + cx, v_c = fy Yc / Zc + cy
        const double iz = 1.0 / cc[2];
        const double dX = guc * a.cam.fx * iz;
        const double dY = gvc * a.cam.fy * iz;
        const double dZ = gZ - (guc * a.cam.fx * cc[0] + gvc * a.cam.fy * cc[1]) * iz * iz;
        // c_cam = W c + t
        for (int j = 0; j < 3; ++j)
            gc[j] = (double)a.cam.R[j] * dX + (double)a.cam.R[3 + j] * dY + (double)a.cam.R[6 + j] * dZ;
        if (a.sh) {
            // rgb_c = max(0, sum_k sh[k][c] Y_k(d) + 1/2), d = (c - o) / |c - o|:
            // coefficient gradients, and the view direction's share of the centre's
            double d[3], r, Y[16], dYd[16][3];
            view_dir(a.cam, a.center + 3 * p, d, r);
            sh_basis(a.sh_degree, d[0], d[1], d[2], Y, dYd);
            const int K = (a.sh_degree + 1) * (a.sh_degree + 1);
            const float *cf = a.sh + (size_t)3 * K * p;
            float *gsh = a.out.sh + (size_t)3 * K * p;
            double gd[3] = {0, 0, 0};
            for (int ch = 0; ch < 3; ++ch) {
                double acc = 0.5;
                for (int k = 0; k < K; ++k) acc += (double)cf[3 * k + ch] * Y[k];
                const double gch = acc > 0.0 ? (double)g[G_R + ch] : 0.0;
                for (int k = 0; k < K; ++k) {
                    const float v = (float)(Y[k] * gch);
                    if (a.accumulate) gsh[3 * k + ch] += v;
                    else gsh[3 * k + ch] = v;
                    for (int j = 0; j < 3; ++j) gd[j] += gch * (double)cf[3 * k + ch] * dYd[k][j];
                }
            }
            const double dg = d[0] * gd[0] + d[1] * gd[1] + d[2] * gd[2];
            for (int j = 0; j < 3; ++j) gc[j] += (gd[j] - d[j] * dg) / r;
        }
        if (a.out.screen_grad) {
            // the centre gradient in camera axes, as a gradient of its image
            // position in normalised device units
            double gcam[3];
            for (int i = 0; i < 3; ++i)
                gcam[i] = (double)a.cam.R[3 * i] * gc[0] + (double)a.cam.R[3 * i + 1] * gc[1] + (double)a.cam.R[3 * i + 2] * gc[2];
            const double su = 0.5 * a.cam.width * cc[2] / a.cam.fx * gcam[0];
            const double sv = 0.5 * a.cam.height * cc[2] / a.cam.fy * gcam[1];
            a.out.screen_grad[p] += (float)sqrt(su * su + sv * sv);
            a.out.visible[p] += 1.0f;
        }
        // rotation: Rm(qhat) -> Rm(qhat (1, phi/2)), so dL/dqhat = (-2 g.v, 2 (w g + v x g))
        const double q0 = a.quat[4 * p], q1 = a.quat[4 * p + 1], q2 = a.quat[4 * p + 2], q3 = a.quat[4 * p + 3];
        const double len = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
        const double w = q0 / len, vx = q1 / len, vy = q2 / len, vz = q3 / len;
        const double f0 = g[G_PHI0], f1 = g[G_PHI1], f2 = g[G_PHI2];
        gq[0] = -2.0 * (f0 * vx + f1 * vy + f2 * vz) / len;
        gq[1] = 2.0 * (w * f0 + (vy * f2 - vz * f1)) / len;
        gq[2] = 2.0 * (w * f1 + (vz * f0 - vx * f2)) / len;
        gq[3] = 2.0 * (w * f2 + (vx * f1 - vy * f0)) / len;
        // k_i = 1 / sigma_i^2
        const double s1 = a.scale[2 * p], s2 = a.scale[2 * p + 1];
        gs[0] = -2.0 * g[G_K1] / (s1 * s1 * s1);
        gs[1] = -2.0 * g[G_K2] / (s2 * s2 * s2);
    }
    const float vals[15] = {(float)gc[0], (float)gc[1], (float)gc[2], (float)gq[0], (float)gq[1], (float)gq[2],
                            (float)gq[3], (float)gs[0], (float)gs[1], active ? g[G_L1] : 0.0f, active ? g[G_L2] : 0.0f,
                            active ? g[G_OP] : 0.0f, active ? g[G_R] : 0.0f, active ? g[G_G] : 0.0f,
                            active ? g[G_B] : 0.0f};
    float *dst[15] = {a.out.center + 3 * p, a.out.center + 3 * p + 1, a.out.center + 3 * p + 2,
                      a.out.quat + 4 * p, a.out.quat + 4 * p + 1, a.out.quat + 4 * p + 2, a.out.quat + 4 * p + 3,
                      a.out.scale + 2 * p, a.out.scale + 2 * p + 1, a.out.curv + 2 * p, a.out.curv + 2 * p + 1,
                      a.out.opacity + p, a.out.rgb + 3 * p, a.out.rgb + 3 * p + 1, a.out.rgb + 3 * p + 2};
    if (a.accumulate) {
        for (int i = 0; i < 15; ++i) *dst[i] += vals[i];
    } else {
        for (int i = 0; i < 15; ++i) *dst[i] = vals[i];
        if (a.sh && !active) {
            const int K = (a.sh_degree + 1) * (a.sh_degree + 1);
            for (int k = 0; k < 3 * K; ++k) a.out.sh[(size_t)3 * K * p + k] = 0.0f;
        }
    }
}

hipError_t launch_preprocess(const PreprocessArgs &a, hipStream_t stream)
{
    if (a.n == 0) return hipSuccess;
    // one-wave workgroups (the tile tests are cooperative within a wave only)
    hipLaunchKernelGGL(k_preprocess, dim3((unsigned)((a.n + 63) / 64)), dim3(64), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_preprocess_bwd(const PreprocessBwdArgs &a, hipStream_t stream)
{
    if (a.n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((a.n + 255) / 256);
    hipLaunchKernelGGL(k_preprocess_bwd, dim3(blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace qgs
