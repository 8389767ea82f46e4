/*
 * FP64 CPU oracle for the quadric Gaussian splatting rasterizer
 * (Quadratic Gaussian Splatting, arXiv 2411.16392).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or constant generator with
 * the HIP library.
 *
 * Two parts:
 *
 *  A. Key stage (oracle_keys, oracle_bin_sort).  The discrete, order-defining
 *     outputs of preprocessing -- the cull flag, the depth key, the screen
 *     rectangle and the tile|depth key list -- written out as a fixed sequence
 *     of IEEE double operations on the FP32 inputs (round to nearest, no
 *     contraction, fma() only where written), then a plain comparison sort.
 *     This is a bit-exact reference for the GPU's discrete outputs.
 *
 *  B. Renderer (oracle_render).  Everything continuous, in FP64, as the plain
 *     per-pixel definition: for each pixel, every active primitive whose
 *     ray-splat hit passes the rules is composited front to back in global
 *     key order (depth key, then primitive index).  Binning here uses the
 *     oracle's own conservative bound (a projected ball), which does not
 *     change the result.  The backward pass is reverse-mode differentiation of
 *     the same sequence with the same discrete decisions.
 *
 * Notation follows the paper:
 *   local frame        x = R xhat + c                    (Sec. 3.2, congruent transform)
 *   paraboloid         zhat = lambda1 xhat^2 + lambda2 yhat^2
 *                      (explicit form, Sec. 3.2; lambda_i = sign(s_i) s_3 / s_i^2)
 *   ray                phat = ohat + t dhat, |dhat| = 1  (supplement, ray-splat intersection)
 *   quadratic          A t^2 + B t + C = 0              (supplement, intersection equation)
 *   small |A|          |A| < 1e-6: the root that diverges as A -> 0 is dropped; the
 *                      other tends to the tangent-plane intersection t = -C/B
 *   arc length         l = rho g(u), u = 2|a| rho, g(u) = (asinh u + u sqrt(1+u^2)) / (2u)
 *                      (geodesic equation, Sec. 3.2, and its derivation in the supplement)
 *   density            G = exp(-l^2 / (2 sigma(theta)^2)), and l^2/sigma^2 = g^2 Q with
 *                      Q = xhat^2/s1^2 + yhat^2/s2^2  (sigma(theta) equation, Sec. 3.2)
 *   root selection     near root if l <= 3 sigma, else far root if l <= 3 sigma,
 *                      else no hit (Sec. 3.2.1, ray-splat intersection)
 *   normal             gradient of the implicit function (Sec. 3.2.1, normal equation)
 *   compositing        X = sum alpha_i G_i T_i X_i, T_i = prod_{j<i}(1 - alpha_j G_j)
 *                      (Eq. 1 and the N/K render equation, Sec. 3)
 *   adjoint            dX/dabar_i = (X_i - sum_{j>i} X_j abar_j T_j / T_{i+1}) T_i
 *                      (supplement, per-tile sorting and per-pixel resorting)
 *
 * Readings where the paper is silent or garbled (near plane 0.2, alpha clamp
 * 0.99, alpha skip 1/255, stop before blending once T < 1e-4, inclusive 3-sigma
 * test, camera-space normals flipped to face the camera, depth = sum w t along
 * the unit ray, roots ordered t_n <= t_f and computed in the cancellation-free
 * form) are inputs or fixed below and listed in the design notes.
 *
 * Parity of whole images on random scenes is pinned only through the pins of
 * its parts (arc length vs quadrature, planar reduction, surface residual,
 * compositing invariants, symmetries, finite differences).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OT 16 /* tile edge in pixels (16 x 16 tiles, supplement: per-tile sorting) */

/* ======================================================================== */
/* A. key stage                                                             */
/* ======================================================================== */

static int finite_f(const float *v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

static double min3(double a, double b, double c) { double m = a < b ? a : b; return m < c ? m : c; }
static double max3(double a, double b, double c) { double m = a > b ? a : b; return m > c ? m : c; }

/*
 * Per primitive: cull flag, FP32 depth key, pixel rectangle and tile rectangle.
 * cam = {R[9] (world->camera, row-major), t[3], fx, fy, cx, cy} as FP32.
 * rect_px / rect_tile: {x0, y0, x1, y1} inclusive; empty = {0, 0, -1, -1}.
 */
/*
 * Conic test of one tile.  C = {c00, c01, c11, c02, c12, c22} is the image of
 * the enclosing ellipsoid in normalised camera coordinates (x, y) =
 * ((u - cx) / fx, (v - cy) / fy): f(x, y) = c00 x^2 + 2 c01 x y + c11 y^2 +
 * 2 c02 x + 2 c12 y + c22 <= 0 inside.  The tile's pixel centres, widened by
 * 1/64 pixel, span a rectangle; f is a convex quadratic, so it meets the
 * interior iff f's minimiser lies in the rectangle or the minimum of f along
 * one of its edges is <= 0.
 */
static double conic_f(const double *C, double x, double y)
{
    return ((C[0] * x + 2.0 * C[1] * y + 2.0 * C[3]) * x + (C[2] * y + 2.0 * C[4]) * y) + C[5];
}

static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Does tile (tx, ty) -- its pixel centres widened by 1/64 pixel -- meet the
   interior f <= 0 of the convex conic C?  Yes iff the conic's centre lies in
   the rectangle or f's minimum along one of the four edges is <= 0 (the edge
   minimiser clamped to the edge).  The divisions are written as products with
   reciprocals (1/fx, 1/fy, 1/det, 1/a, 1/c), each rounded once; the GPU
   evaluates the same sequence. */
static int oracle_tile_hit(const double *C, int tx, int ty, const float *cam, int width, int height)
{
    const double fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15];
    const double ifx = 1.0 / fx, ify = 1.0 / fy;
    const double pad_px = 1.0 / 64.0;
    const int ux0 = tx * OT, ux1 = (tx * OT + OT - 1) < width - 1 ? tx * OT + OT - 1 : width - 1;
    const int vy0 = ty * OT, vy1 = (ty * OT + OT - 1) < height - 1 ? ty * OT + OT - 1 : height - 1;
    const double x0 = ((((double)ux0 + 0.5) - pad_px) - cx) * ifx, x1 = ((((double)ux1 + 0.5) + pad_px) - cx) * ifx;
    const double y0 = ((((double)vy0 + 0.5) - pad_px) - cy) * ify, y1 = ((((double)vy1 + 0.5) + pad_px) - cy) * ify;
    const double a = C[0], b = C[1], c = C[2], d = C[3], e = C[4];
    const double inv_det = 1.0 / (a * c - b * b);
    const double mx = (b * e - c * d) * inv_det, my = (b * d - a * e) * inv_det;
    const double inv_a = 1.0 / a, inv_c = 1.0 / c;
    if (mx >= x0 && mx <= x1 && my >= y0 && my <= y1) return 1;
    const double xs[2] = {x0, x1}, ys[2] = {y0, y1};
    for (int k = 0; k < 2; ++k) {
        const double y = clampd(-(b * xs[k] + e) * inv_c, y0, y1);
        if (conic_f(C, xs[k], y) <= 0.0) return 1;
        const double x = clampd(-(b * ys[k] + d) * inv_a, x0, x1);
        if (conic_f(C, x, ys[k]) <= 0.0) return 1;
    }
    return 0;
}

/*
 * Local box of the support, [-hx, hx] x [-hy, hy] x [zlo, zhi], out = {hx, hy,
 * zlo, zhi}, inflated by 2^-10 (z also padded by k max(s) / 1024).  A support
 * point (x, y, z = lambda1 x^2 + lambda2 y^2) has arc length l = rho g(u) <=
 * k sigma(theta) with rho^2 = x^2 + y^2 and sigma(theta)^2 = rho^2 / Q
 * (Sec. 3.2, geodesic and sigma(theta) equations).
 *  tight == 0: g >= 1 gives Q <= k^2, so |x| <= k s1, |y| <= k s2; z lies
 *    between the extremes of {0, k^2 lambda_i s_i^2} and |z| <= l <= k max(s).
 *  tight != 0: the arc from the vertex is at least its chord, l^2 >= rho^2 +
 *    z^2, so (rho^2 + z^2) Q / rho^2 <= k^2 and, as Q / rho^2 >= 1/sm^2
 *    (sm = max(s1, s2)), Q + z^2 / sm^2 <= k^2.  With X = x^2, Y = y^2 the
 *    largest admissible X solves min_{Y>=0} [X/s1^2 + Y/s2^2 +
 *    (lambda1 X + lambda2 Y)^2 / sm^2] = k^2.  For lambda1 lambda2 >= 0 the
 *    minimum is at Y = 0: lambda1^2 X^2 / sm^2 + X / s1^2 = k^2.  For opposite
 *    signs Y = 0 is optimal up to Xc = sm^2 / (2 |lambda1 lambda2| s2^2);
 *    beyond it the minimum is X (1/s1^2 + |lambda1| / (|lambda2| s2^2)) -
 *    sm^2 / (4 lambda2^2 s2^4).  The height: per direction rho^2 (1 + a^2
 *    rho^2) <= k^2 sigma^2, so |z| = |a| rho^2 <= 2 k^2 m / (1 + sqrt(1 + 4 k^2
 *    m^2 / sigma^2)) with m = |a| sigma^2, increasing in m and sigma; a sigma^2
 *    is a weighted mean of lambda1 s1^2 and lambda2 s2^2, and sigma <= sm.
 * FP64, the operation order as written (the GPU follows the same sequence).
 */
static double chord_x2(double sa, double sb, double la, double lb, double sm, double k2)
{
    double ra = ((la * sa) * sa) / sm;
    double x_root = ((2.0 * k2) * (sa * sa)) / (1.0 + sqrt(1.0 + (4.0 * k2) * (ra * ra)));
    if (la * lb < 0.0) {
        double rb = (fabs(lb) * sb) * sb;
        double x_c = (sm * sm) / ((2.0 * fabs(la)) * rb);
        if (x_root > x_c) return (k2 + (sm * sm) / (4.0 * (rb * rb))) / (1.0 / (sa * sa) + fabs(la) / rb);
    }
    return x_root;
}

static double chord_z(double m, double sm, double k2)
{
    double r = m / sm;
    return ((2.0 * k2) * m) / (1.0 + sqrt(1.0 + (4.0 * k2) * (r * r)));
}

/*
 * The cut-off the tight bounds use for a primitive of opacity o.  It blends
 * only where alpha = min(alpha_max, o G) >= alpha_min (R7), so G >=
 * alpha_min / o and E <= 2 ln x with x = o / alpha_min.  ln x = 64 ln x^(1/64)
 * <= 64 (x^(1/64) - 1) (ln y <= y - 1); x^(1/64) by six correctly rounded
 * square roots; a relative margin of 2^-20 covers their rounding.  Returns
 * min(k, sqrt(that bound)), or k when alpha_min <= 0 or x <= 1.
 */
double oracle_blend_k(float o, float alpha_min, float k_sigma)
{
    const double k = k_sigma;
    if (!(alpha_min > 0.0f)) return k;
    const double x = (double)o / (double)alpha_min;
    if (!(x > 1.0)) return k;
    double r = x;
    for (int i = 0; i < 6; ++i) r = sqrt(r);
    const double e2 = (128.0 * (r - 1.0)) * (1.0 + 1.0 / 1048576.0);
    return e2 < k * k ? sqrt(e2) : k;
}

void oracle_local_box(double s1, double s2, double l1, double l2, double k, int32_t tight, double *out)
{
    const double infl = 1.0 + 1.0 / 1024.0;
    const double k2 = k * k;
    const double smax = s1 > s2 ? s1 : s2;
    const double zcap = k * smax;
    const double m1 = (l1 * s1) * s1, m2 = (l2 * s2) * s2;
    double ex = k * s1, ey = k * s2, zlo, zhi;
    if (tight) {
        double bx = sqrt(chord_x2(s1, s2, l1, l2, smax, k2)), by = sqrt(chord_x2(s2, s1, l2, l1, smax, k2));
        if (bx < ex) ex = bx;
        if (by < ey) ey = by;
        zlo = -chord_z(-min3(0.0, m1, m2), smax, k2);
        zhi = chord_z(max3(0.0, m1, m2), smax, k2);
    } else {
        zlo = k2 * min3(0.0, m1, m2);
        zhi = k2 * max3(0.0, m1, m2);
    }
    if (zlo < -zcap) zlo = -zcap;
    if (zhi > zcap) zhi = zcap;
    const double zpad = zcap / 1024.0;
    out[0] = ex * infl;
    out[1] = ey * infl;
    out[2] = zlo * infl - zpad;
    out[3] = zhi * infl + zpad;
}

/*
 * The paper's tangent-plane box (supplement, bounding box calculation), for
 * measurement only: it is not conservative.  Reading of the garbled passage:
 *  - the arc length is replaced by lhat(a, rho) = (4 |a| rho^2 + 6 rho) / 7 and
 *    rho_i is the positive root of lhat(lambda_i, rho) = k s_i along each
 *    principal axis (the k-sigma cut-off), in the cancellation-free form
 *    rho = 14 k s / (6 + sqrt(36 + 112 |a| k s)); 7 k s / 6 for a = 0;
 *  - the four points (+-rho1, 0, lambda1 rho1^2), (0, +-rho2, lambda2 rho2^2);
 *    the tangent plane of z = lambda x^2 at x0 meets z = 0 at x0 / 2, so the
 *    bottom half-widths are rho_i / 2 (rho_i when lambda_i = 0: the tangent
 *    plane is z = 0);
 *  - the frustum has its bottom face [+-x1] x [+-x2] at z = 0 and its top face
 *    [+-rho1] x [+-rho2] at the height h = lambda_j rho_j^2 of larger magnitude.
 * out = {rho1, rho2, x1, x2, h}.
 */
void oracle_tb_frustum(double s1, double s2, double l1, double l2, double k, double *out)
{
    const double sg[2] = {s1, s2}, lm[2] = {l1, l2};
    double rho[2], h[2];
    for (int i = 0; i < 2; ++i) {
        rho[i] = 14.0 * k * sg[i] / (6.0 + sqrt(36.0 + 112.0 * fabs(lm[i]) * k * sg[i]));
        out[2 + i] = lm[i] == 0.0 ? rho[i] : 0.5 * rho[i];
        h[i] = lm[i] * rho[i] * rho[i];
    }
    out[0] = rho[0];
    out[1] = rho[1];
    out[4] = fabs(h[0]) >= fabs(h[1]) ? h[0] : h[1];
}

void oracle_keys(int64_t n, const float *center, const float *quat, const float *scale,
                 const float *curv, const float *opac, const float *rgb,
                 const float *cam, int32_t width, int32_t height, float near_f, float k_sigma,
                 uint8_t *culled, uint32_t *depth_bits, int32_t *rect_px, int32_t *rect_tile,
                 uint32_t *tiles, double *conic, uint8_t *conic_ok, double *frame, int32_t tight, float alpha_min)
{
    double W[9], T[3];
    for (int i = 0; i < 9; ++i) W[i] = cam[i];
    for (int i = 0; i < 3; ++i) T[i] = cam[9 + i];
    const double fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15];
    const double near_d = near_f;
        const double pad_px = 1.0 / 64.0;

    for (int64_t p = 0; p < n; ++p) {
        int32_t *rp = rect_px + 4 * p, *rt = rect_tile + 4 * p;
        rp[0] = rp[1] = 0; rp[2] = rp[3] = -1;
        rt[0] = rt[1] = 0; rt[2] = rt[3] = -1;
        tiles[p] = 0;
        depth_bits[p] = 0;
        culled[p] = 1;
        conic_ok[p] = 0;
        for (int i = 0; i < 6; ++i) conic[6 * p + i] = 0.0;
        if (frame) for (int i = 0; i < 16; ++i) frame[16 * p + i] = 0.0;

        const float *cf = center + 3 * p, *qf = quat + 4 * p, *sf = scale + 2 * p, *lf = curv + 2 * p;
        if (!finite_f(cf, 3) || !finite_f(qf, 4) || !finite_f(sf, 2) || !finite_f(lf, 2) ||
            !finite_f(opac + p, 1) || !finite_f(rgb + 3 * p, 3))
            continue;
        const double s1 = sf[0], s2 = sf[1], l1 = lf[0], l2 = lf[1];
        if (!(s1 > 0.0) || !(s2 > 0.0)) continue;
        const double w = qf[0], x = qf[1], y = qf[2], z = qf[3];
        const double ww = w * w, xx = x * x, yy = y * y, zz = z * z;
        const double qn = (ww + xx) + (yy + zz);
        if (!(qn > 0.0)) continue;

        double cc[3];
        for (int i = 0; i < 3; ++i)
            cc[i] = fma(W[3 * i + 0], (double)cf[0], fma(W[3 * i + 1], (double)cf[1], fma(W[3 * i + 2], (double)cf[2], T[i])));
        const float zf = (float)cc[2];
        if (!(zf > near_f)) continue;

        /* rotation from the (unnormalised) quaternion: R = rot(q / |q|) */
        const double s = 2.0 / qn;
        const double xy = x * y, xz = x * z, yz = y * z, wx = w * x, wy = w * y, wz = w * z;
        double Rm[9];
        Rm[0] = 1.0 - s * (yy + zz); Rm[1] = s * (xy - wz);        Rm[2] = s * (xz + wy);
        Rm[3] = s * (xy + wz);       Rm[4] = 1.0 - s * (xx + zz);  Rm[5] = s * (yz - wx);
        Rm[6] = s * (xz - wy);       Rm[7] = s * (yz + wx);        Rm[8] = 1.0 - s * (xx + yy);
        double Rc[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                Rc[3 * i + j] = fma(W[3 * i + 0], Rm[j], fma(W[3 * i + 1], Rm[3 + j], W[3 * i + 2] * Rm[6 + j]));

        /* conservative local box of the support (oracle_local_box) */
        double box[4];
        oracle_local_box(s1, s2, l1, l2, tight == 1 ? oracle_blend_k(opac[p], alpha_min, k_sigma) : (double)k_sigma,
                         tight == 1, box);
        const double hx = box[0], hy = box[1], zlo = box[2], zhi = box[3];
        double tb[5];
        if (tight == 2) oracle_tb_frustum(s1, s2, l1, l2, (double)k_sigma, tb);

        /* The rectangle bounds the projection of the part of the box in front
           of the near plane (a hit needs a camera depth above it).  That part
           is a convex polytope whose vertices are the corners in front and the
           points where edges cross the plane; a central projection maps it to
           the convex hull of the vertices' images. */
        double P8[8][3];
        int in_front[8], n_front = 0;
        for (int c = 0; c < 8; ++c) {
            double X = (c & 1) ? hx : -hx, Y = (c & 2) ? hy : -hy, Z = (c & 4) ? zhi : zlo;
            if (tight == 2) {
                /* frustum: bottom face at z = 0, top face at the height h */
                const int top = (c & 4) != 0;
                X = ((c & 1) ? 1.0 : -1.0) * (top ? tb[0] : tb[2]);
                Y = ((c & 2) ? 1.0 : -1.0) * (top ? tb[1] : tb[3]);
                Z = top ? tb[4] : 0.0;
            }
            for (int i = 0; i < 3; ++i)
                P8[c][i] = fma(Rc[3 * i + 0], X, fma(Rc[3 * i + 1], Y, fma(Rc[3 * i + 2], Z, cc[i])));
            in_front[c] = P8[c][2] > near_d;
            n_front += in_front[c];
        }
        const int behind = n_front < 8;
        double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
        double pts[20][2];
        int npts = 0;
        for (int c = 0; c < 8; ++c) {
            if (!in_front[c]) continue;
            pts[npts][0] = fma(fx, P8[c][0] / P8[c][2], cx);
            pts[npts][1] = fma(fy, P8[c][1] / P8[c][2], cy);
            ++npts;
        }
        for (int a = 0; a < 8; ++a)
            for (int b = a + 1; b < 8; ++b) {
                const int d = a ^ b;
                if ((d & (d - 1)) != 0) continue; /* not an edge: corners differ in more than one axis */
                if (in_front[a] == in_front[b]) continue;
                const double *F = in_front[a] ? P8[a] : P8[b], *Bk = in_front[a] ? P8[b] : P8[a];
                const double s_cut = (F[2] - near_d) / (F[2] - Bk[2]);
                const double xq = F[0] + s_cut * (Bk[0] - F[0]), yq = F[1] + s_cut * (Bk[1] - F[1]);
                pts[npts][0] = fma(fx, xq / near_d, cx);
                pts[npts][1] = fma(fy, yq / near_d, cy);
                ++npts;
            }
        for (int i = 0; i < npts; ++i) {
            if (pts[i][0] < umin) umin = pts[i][0];
            if (pts[i][0] > umax) umax = pts[i][0];
            if (pts[i][1] < vmin) vmin = pts[i][1];
            if (pts[i][1] > vmax) vmax = pts[i][1];
        }
        int px0, px1, py0, py1;
        {
            const double a0 = (umin - 0.5) - pad_px, a1 = (umax - 0.5) + pad_px;
            const double b0 = (vmin - 0.5) - pad_px, b1 = (vmax - 0.5) + pad_px;
            if (n_front == 0 || a1 < 0.0 || a0 > (double)(width - 1) || b1 < 0.0 || b0 > (double)(height - 1)) {
                /* nothing in front of the near plane, or off screen */
                culled[p] = 0;
                depth_bits[p] = 0;
                memcpy(&depth_bits[p], &zf, 4);
                continue;
            }
            px0 = a0 <= 0.0 ? 0 : (int)ceil(a0);
            px1 = a1 >= (double)(width - 1) ? width - 1 : (int)floor(a1);
            py0 = b0 <= 0.0 ? 0 : (int)ceil(b0);
            py1 = b1 >= (double)(height - 1) ? height - 1 : (int)floor(b1);
        }
        culled[p] = 0;
        memcpy(&depth_bits[p], &zf, 4);
        if (frame) {
            /* camera frame of the primitive for the per-tile sort depth */
            double *F = frame + 16 * p;
            for (int i = 0; i < 3; ++i) F[i] = cc[i];
            for (int i = 0; i < 9; ++i) F[3 + i] = Rc[i];
            F[12] = fma(fx, cc[0] / cc[2], cx);
            F[13] = fma(fy, cc[1] / cc[2], cy);
            F[14] = l1;
            F[15] = l2;
        }
        if (px0 > px1 || py0 > py1) continue;
        rp[0] = px0; rp[1] = py0; rp[2] = px1; rp[3] = py1;
        rt[0] = px0 / OT; rt[1] = py0 / OT; rt[2] = px1 / OT; rt[3] = py1 / OT;

        /* Ellipsoid enclosing the box's elliptic cylinder {x^2/hx^2 + y^2/hy^2
           <= 1, z in [zlo, zhi]}: squared semi-axes hx^2/(1-t), hy^2/(1-t),
           hz^2/t about the mid-height zm (a point of the cylinder satisfies
           (1-t) + t = 1), with t = hz / (hz + min(hx, hy)). */
        double *Cq = conic + 6 * p;
        if (!behind && tight != 2) {
            const double hz = 0.5 * (zhi - zlo), zm = 0.5 * (zlo + zhi);
            const double mxy = hx < hy ? hx : hy;
            const double t = hz / (hz + mxy);
            const double q[3] = {(hx * hx) / (1.0 - t), (hy * hy) / (1.0 - t), (hz * hz) / t};
            const double iq[3] = {1.0 / q[0], 1.0 / q[1], 1.0 / q[2]};
            double ce[3];
            for (int i = 0; i < 3; ++i) ce[i] = fma(Rc[3 * i + 2], zm, cc[i]);
            /* A = Rc diag(1/q) Rc^T, symmetric: A[i][j] */
            double A[3][3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    A[i][j] = fma(Rc[3 * i] * iq[0], Rc[3 * j],
                                  fma(Rc[3 * i + 1] * iq[1], Rc[3 * j + 1], (Rc[3 * i + 2] * iq[2]) * Rc[3 * j + 2]));
            double w[3];
            for (int i = 0; i < 3; ++i) w[i] = fma(A[i][0], ce[0], fma(A[i][1], ce[1], A[i][2] * ce[2]));
            const double gm1 = fma(ce[0], w[0], fma(ce[1], w[1], ce[2] * w[2])) - 1.0;
            /* ray d = (x, y, 1) meets the ellipsoid iff d^T [(gamma-1) A - w w^T] d <= 0 */
            const int ii[6] = {0, 0, 1, 0, 1, 2}, jj[6] = {0, 1, 1, 2, 2, 2};
            for (int k = 0; k < 6; ++k) Cq[k] = fma(gm1, A[ii[k]][jj[k]], -(w[ii[k]] * w[jj[k]]));
            /* the conic is a bounded ellipse when the ellipsoid lies in front of the near plane */
            const double S33 = fma(q[0] * Rc[6], Rc[6], fma(q[1] * Rc[7], Rc[7], (q[2] * Rc[8]) * Rc[8]));
            const double dz = ce[2] - near_d;
            conic_ok[p] = (dz > 0.0 && dz * dz > S33) ? 1 : 0;
        }
        uint32_t cnt = 0;
        for (int ty = rt[1]; ty <= rt[3]; ++ty)
            for (int tx = rt[0]; tx <= rt[2]; ++tx)
                cnt += (!conic_ok[p] || oracle_tile_hit(Cq, tx, ty, cam, width, height)) ? 1u : 0u;
        tiles[p] = cnt;
    }
}

/*
 * Per-tile sort depth (supplement, per-tile sorting): for tile (tx, ty), the
 * camera depth at which the ray through the tile's pixel nearest the
 * projected vertex meets the paraboloid.  The pixel is the one containing the
 * projected vertex, clamped to the tile.  The ray d = (x_n, y_n, 1) makes the
 * ray parameter the camera depth; in the local frame p = o + s e with
 * o = -Rc^T c_cam and e = Rc^T d, and A s^2 + B s + C = 0 as for shading.  The
 * depth is the smallest root beyond the near plane (the small-|A| root -C/B
 * when |A| <= 1e-12 |e|^2), or the centre depth if there is none.  F is the
 * frame written by oracle_keys: c_cam[3], Rc[9], projected vertex (u, v),
 * lambda1, lambda2.  FP64, no contraction, the operation order as written.
 */
static uint32_t tile_depth_bits(const double *F, int tx, int ty, const double *cam, int width, int height,
                                double near_d)
{
    const double fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15];
    const int ux0 = tx * OT, ux1 = tx * OT + OT - 1 < width - 1 ? tx * OT + OT - 1 : width - 1;
    const int vy0 = ty * OT, vy1 = ty * OT + OT - 1 < height - 1 ? ty * OT + OT - 1 : height - 1;
    const double fu = floor(F[12]), fv = floor(F[13]);
    const int px = fu < (double)ux0 ? ux0 : (fu > (double)ux1 ? ux1 : (int)fu);
    const int py = fv < (double)vy0 ? vy0 : (fv > (double)vy1 ? vy1 : (int)fv);
    const double dx = (((double)px + 0.5) - cx) / fx, dy = (((double)py + 0.5) - cy) / fy;
    double o[3], e[3];
    for (int k = 0; k < 3; ++k) {
        o[k] = -((F[3 + k] * F[0] + F[6 + k] * F[1]) + F[9 + k] * F[2]);
        e[k] = (F[3 + k] * dx + F[6 + k] * dy) + F[9 + k];
    }
    const double l1 = F[14], l2 = F[15];
    const double A = (l1 * e[0]) * e[0] + (l2 * e[1]) * e[1];
    const double B = 2.0 * ((l1 * o[0]) * e[0] + (l2 * o[1]) * e[1]) - e[2];
    const double C = ((l1 * o[0]) * o[0] + (l2 * o[1]) * o[1]) - o[2];
    double r[2];
    int nr = 0;
    if (fabs(A) <= 1e-12 * ((e[0] * e[0] + e[1] * e[1]) + e[2] * e[2])) {
        if (B != 0.0) r[nr++] = -C / B;
    } else {
        const double D = B * B - 4.0 * (A * C);
        if (D >= 0.0) {
            const double sq = sqrt(D);
            const double q = -0.5 * (B + (B >= 0.0 ? sq : -sq));
            if (q != 0.0) {
                r[nr++] = q / A;
                r[nr++] = C / q;
            }
        }
    }
    double z = F[2];
    int found = 0;
    for (int i = 0; i < nr; ++i)
        if (r[i] > near_d && (!found || r[i] < z)) {
            z = r[i];
            found = 1;
        }
    const float zf = (float)z;
    uint32_t bits;
    memcpy(&bits, &zf, 4);
    return bits;
}

typedef struct {
    uint64_t key; /* tile << 32 | depth bits (centre depth, or the per-tile depth) */
    uint64_t tie; /* centre depth bits << 32 | primitive: the emission order of equal keys */
    uint64_t seq; /* emission index: primitive-major, tiles row-major in its rect */
    uint32_t prim;
} opair;

static int cmp_pair(const void *a, const void *b)
{
    const opair *x = (const opair *)a, *y = (const opair *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->tie != y->tie) return x->tie < y->tie ? -1 : 1;
    return 0;
}

/*
 * Emits one (key, primitive) pair per tile of every rectangle that passes the
 * conic test, in primitive order and row-major within a rectangle, and sorts
 * by key; equal keys are ordered by (centre depth key, primitive index).  The
 * key's depth is the primitive's centre depth, or with frame != NULL the
 * per-tile depth of tile_depth_bits.  Returns the pair count; writes outputs
 * only if it fits cap.  ranges[2t], ranges[2t+1] = [start, end) of tile t in
 * the sorted list; out_seq = emission index of each sorted pair.
 */
int64_t oracle_bin_sort(int64_t n, const uint8_t *culled, const uint32_t *depth_bits,
                        const int32_t *rect_tile, const double *conic, const uint8_t *conic_ok,
                        const float *cam, int32_t width, int32_t height, int32_t tiles_x, int32_t tiles_y,
                        int64_t cap, uint64_t *out_keys, uint32_t *out_prim, uint32_t *out_seq, uint32_t *ranges,
                        const double *frame, float near_f)
{
    double camd[16];
    for (int i = 0; i < 16; ++i) camd[i] = cam[i];
    int64_t total = 0;
    for (int64_t p = 0; p < n; ++p) {
        const int32_t *r = rect_tile + 4 * p;
        if (culled[p] || r[2] < r[0] || r[3] < r[1]) continue;
        for (int ty = r[1]; ty <= r[3]; ++ty)
            for (int tx = r[0]; tx <= r[2]; ++tx)
                total += (!conic_ok[p] || oracle_tile_hit(conic + 6 * p, tx, ty, cam, width, height)) ? 1 : 0;
    }
    if (total > cap) return total;
    opair *pairs = (opair *)malloc(sizeof(opair) * (size_t)(total > 0 ? total : 1));
    int64_t k = 0;
    for (int64_t p = 0; p < n; ++p) {
        const int32_t *r = rect_tile + 4 * p;
        if (culled[p] || r[2] < r[0] || r[3] < r[1]) continue;
        for (int ty = r[1]; ty <= r[3]; ++ty)
            for (int tx = r[0]; tx <= r[2]; ++tx) {
                if (conic_ok[p] && !oracle_tile_hit(conic + 6 * p, tx, ty, cam, width, height)) continue;
                const uint32_t db = frame ? tile_depth_bits(frame + 16 * p, tx, ty, camd, width, height, near_f)
                                          : depth_bits[p];
                pairs[k].key = ((uint64_t)(uint32_t)(ty * tiles_x + tx) << 32) | db;
                pairs[k].tie = ((uint64_t)depth_bits[p] << 32) | (uint64_t)p;
                pairs[k].seq = (uint64_t)k;
                pairs[k].prim = (uint32_t)p;
                ++k;
            }
    }
    qsort(pairs, (size_t)total, sizeof(opair), cmp_pair);
    const int64_t nt = (int64_t)tiles_x * tiles_y;
    for (int64_t t = 0; t < 2 * nt; ++t) ranges[t] = 0;
    for (int64_t i = 0; i < total; ++i) {
        out_keys[i] = pairs[i].key;
        out_prim[i] = pairs[i].prim;
        out_seq[i] = (uint32_t)pairs[i].seq;
        const uint32_t t = (uint32_t)(pairs[i].key >> 32);
        if (i == 0 || (uint32_t)(pairs[i - 1].key >> 32) != t) ranges[2 * t] = (uint32_t)i;
        if (i == total - 1 || (uint32_t)(pairs[i + 1].key >> 32) != t) ranges[2 * t + 1] = (uint32_t)(i + 1);
    }
    free(pairs);
    return total;
}

uint32_t oracle_tile_depth_bits(const double *F, int32_t tx, int32_t ty, const double *cam, int32_t width,
                                int32_t height, double near_d)
{
    return tile_depth_bits(F, tx, ty, cam, width, height, near_d);
}

double oracle_gfun(double u);

/* ======================================================================== */
/* B. FP64 renderer                                                         */
/* ======================================================================== */

/* options: near, k_sigma, alpha_min, alpha_max, T_eps, A_eps, bg[3] */
enum { O_NEAR = 0, O_K, O_AMIN, O_AMAX, O_TEPS, O_AEPS, O_BG, O_RESORT = O_BG + 3, O_NOPTS };
/* Discrete decisions of the per-pixel sequence, each with a margin scale in
   delta[]: |A| vs A_eps, the sign of D, the near test, E vs k^2, alpha vs
   alpha_min, T' vs T_eps, the normal's facing, the alpha clamp, the median's
   choices, the resort buffer's choice of the nearest.  M_DCOND is no decision
   but the conditioning of an accepted root's derivative, 1 / (2 A t + B) =
   1 / sqrt(D): the ratio of D to the change rounding its terms makes in it
   (ray_hit), relative to its scale (FP32 carries the derivative with a
   relative error of about 1e-7 / that ratio). */
enum { M_A = 0, M_D, M_NEAR, M_E, M_AMIN, M_T, M_N, M_CLAMP, M_MED, M_SORT, M_DCOND, M_COUNT };

/* per-pixel channels: colour[3], depth, normal[3], curvature, median depth,
   depth distortion */
enum { CH_DEPTH = 3, CH_N = 4, CH_K = 7, CH_MED = 8, CH_DIST = 9, NCH = 10 };

typedef struct {
    double Rc[9];  /* camera-from-local rotation: columns are the local axes */
    double cc[3];  /* centre in camera space */
    double o[3];   /* camera centre in the local frame, ohat = -Rc^T cc */
    double C;      /* constant term of the quadratic: lambda1 o1^2 + lambda2 o2^2 - o3 */
    double s1, s2, l1, l2, op, rgb[3];
    double qn[4], qlen;
} oprim;

/*
 * Spherical-harmonics colour (the 3DGS colour model the paper keeps, Sec. 3):
 * rgb_c = max(0, sum_k sh[k][c] Y_k(d) + 1/2) for the unit direction d from
 * the camera centre to the primitive centre, with the real spherical harmonics
 * of degree <= 3 written out from their definitions (normalisation
 * sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!), Condon-Shortley phase), in the order
 * l = 0..3, m = -l..l.
 */
static void sh_basis(int deg, double x, double y, double z, double Y[16], double dY[16][3])
{
    const double pi = 3.14159265358979323846;
    const double c0 = 0.5 * sqrt(1.0 / pi), c1 = sqrt(3.0 / (4.0 * pi));
    const double c2a = 0.5 * sqrt(15.0 / pi), c2b = 0.25 * sqrt(5.0 / pi), c2c = 0.25 * sqrt(15.0 / pi);
    const double c3a = 0.25 * sqrt(35.0 / (2.0 * pi)), c3b = 0.5 * sqrt(105.0 / pi);
    const double c3c = 0.25 * sqrt(21.0 / (2.0 * pi)), c3d = 0.25 * sqrt(7.0 / pi), c3e = 0.25 * sqrt(105.0 / pi);
    for (int k = 0; k < 16; ++k) {
        Y[k] = 0.0;
        dY[k][0] = dY[k][1] = dY[k][2] = 0.0;
    }
    Y[0] = c0;
    if (deg < 1) return;
    Y[1] = -c1 * y; dY[1][1] = -c1;
    Y[2] = c1 * z;  dY[2][2] = c1;
    Y[3] = -c1 * x; dY[3][0] = -c1;
    if (deg < 2) return;
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[4] = c2a * x * y;             dY[4][0] = c2a * y;  dY[4][1] = c2a * x;
    Y[5] = -c2a * y * z;            dY[5][1] = -c2a * z; dY[5][2] = -c2a * y;
    Y[6] = c2b * (2 * zz - xx - yy); dY[6][0] = -2 * c2b * x; dY[6][1] = -2 * c2b * y; dY[6][2] = 4 * c2b * z;
    Y[7] = -c2a * x * z;            dY[7][0] = -c2a * z; dY[7][2] = -c2a * x;
    Y[8] = c2c * (xx - yy);         dY[8][0] = 2 * c2c * x; dY[8][1] = -2 * c2c * y;
    if (deg < 3) return;
    Y[9] = -c3a * y * (3 * xx - yy);
    dY[9][0] = -c3a * 6 * x * y; dY[9][1] = -c3a * (3 * xx - 3 * yy);
    Y[10] = c3b * x * y * z;
    dY[10][0] = c3b * y * z; dY[10][1] = c3b * x * z; dY[10][2] = c3b * x * y;
    Y[11] = -c3c * y * (4 * zz - xx - yy);
    dY[11][0] = c3c * 2 * x * y; dY[11][1] = -c3c * (4 * zz - xx - 3 * yy); dY[11][2] = -c3c * 8 * y * z;
    Y[12] = c3d * z * (2 * zz - 3 * xx - 3 * yy);
    dY[12][0] = -c3d * 6 * x * z; dY[12][1] = -c3d * 6 * y * z; dY[12][2] = c3d * (6 * zz - 3 * xx - 3 * yy);
    Y[13] = -c3c * x * (4 * zz - xx - yy);
    dY[13][0] = -c3c * (4 * zz - 3 * xx - yy); dY[13][1] = c3c * 2 * x * y; dY[13][2] = -c3c * 8 * x * z;
    Y[14] = c3e * z * (xx - yy);
    dY[14][0] = c3e * 2 * x * z; dY[14][1] = -c3e * 2 * y * z; dY[14][2] = c3e * (xx - yy);
    Y[15] = -c3a * x * (xx - 3 * yy);
    dY[15][0] = -c3a * (3 * xx - 3 * yy); dY[15][1] = c3a * 6 * x * y;
}

void oracle_sh_basis(int32_t deg, const double *d, double *Y, double *dY)
{
    double yy[16], dd[16][3];
    sh_basis(deg, d[0], d[1], d[2], yy, dd);
    for (int k = 0; k < 16; ++k) {
        Y[k] = yy[k];
        for (int j = 0; j < 3; ++j) dY[3 * k + j] = dd[k][j];
    }
}

/* colour from SH coefficients sh[K][3] at the primitive centre c (world);
   also the unit direction, its length and which channels are not clamped */
static void sh_colour(int deg, const double *sh, const double *c, const double *W, const double *T, double rgb[3],
                      double dir[3], double *dist, int live[3])
{
    /* camera centre o = -W^T t */
    double v[3];
    for (int j = 0; j < 3; ++j) v[j] = c[j] + (W[j] * T[0] + W[3 + j] * T[1] + W[6 + j] * T[2]);
    const double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int j = 0; j < 3; ++j) dir[j] = v[j] / r;
    *dist = r;
    double Y[16], dY[16][3];
    sh_basis(deg, dir[0], dir[1], dir[2], Y, dY);
    const int K = (deg + 1) * (deg + 1);
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.5;
        for (int k = 0; k < K; ++k) acc += sh[3 * k + ch] * Y[k];
        live[ch] = acc > 0.0;
        rgb[ch] = acc > 0.0 ? acc : 0.0;
    }
}

static void setup_prim(const double *c, const double *q, const double *s, const double *l,
                       double op, const double *rgb, const double *W, const double *T, oprim *P)
{
    const double len = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double w = q[0] / len, x = q[1] / len, y = q[2] / len, z = q[3] / len;
    double Rm[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                    2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                    2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            P->Rc[3 * i + j] = W[3 * i] * Rm[j] + W[3 * i + 1] * Rm[3 + j] + W[3 * i + 2] * Rm[6 + j];
    for (int i = 0; i < 3; ++i) P->cc[i] = W[3 * i] * c[0] + W[3 * i + 1] * c[1] + W[3 * i + 2] * c[2] + T[i];
    for (int j = 0; j < 3; ++j)
        P->o[j] = -(P->Rc[j] * P->cc[0] + P->Rc[3 + j] * P->cc[1] + P->Rc[6 + j] * P->cc[2]);
    P->s1 = s[0]; P->s2 = s[1]; P->l1 = l[0]; P->l2 = l[1];
    P->op = op;
    P->rgb[0] = rgb[0]; P->rgb[1] = rgb[1]; P->rgb[2] = rgb[2];
    P->C = P->l1 * P->o[0] * P->o[0] + P->l2 * P->o[1] * P->o[1] - P->o[2];
    P->qn[0] = w; P->qn[1] = x; P->qn[2] = y; P->qn[3] = z;
    P->qlen = len;
}

/* arc-length factor g(u) = l / rho and its derivative.  Below u = 0.1 the
   closed forms lose digits (g' subtracts nearly equal terms), so the binomial
   series of the integrand is used: sqrt(1 + u^2 s^2) = sum_k C(1/2, k) u^2k s^2k
   integrated over s in [0, 1] gives g = sum_k C(1/2, k) u^2k / (2k + 1). */
static const double G_SERIES[9] = {1.0, 1.0 / 6, -1.0 / 40, 1.0 / 112, -5.0 / 1152, 7.0 / 2816,
                                   -21.0 / 13312, 11.0 / 10240, -429.0 / 557056};

double oracle_gfun(double u)
{
    if (u < 0.1) {
        const double v = u * u;
        double acc = 0.0;
        for (int k = 8; k >= 0; --k) acc = acc * v + G_SERIES[k];
        return acc;
    }
    return (asinh(u) + u * sqrt(1.0 + u * u)) / (2.0 * u);
}

double oracle_gprime(double u)
{
    if (u < 0.1) {
        const double v = u * u;
        double acc = 0.0;
        for (int k = 8; k >= 1; --k) acc = acc * v + 2.0 * k * G_SERIES[k];
        return acc * u;
    }
    return (u * sqrt(1.0 + u * u) - asinh(u)) / (2.0 * u * u);
}

/* arc length l(a, rho) of the normal section z = a r^2 from 0 to rho */
double oracle_arc_length(double a, double rho)
{
    return rho * oracle_gfun(2.0 * fabs(a) * rho);
}

typedef struct {
    int ok;
    int linear;     /* 1: |A| < A_eps, the diverging root dropped */
    double d[3];    /* dhat */
    double A, B, F1;/* F1 = dF/dt = 2 A t + B at the root */
    double t, x, y, Q, rho, h, u, g, E;
} ohit;

/*
 * Near-ties of the discrete decisions.  FP32 and FP64 may decide differently
 * where a quantity lies within its margin scale of a decision boundary, so
 * both outcomes are correct results there.  Every decision records its scaled
 * margin (distance to the boundary over the scale) per kind.  A decision of a
 * kind in `branch` whose margin is below 1 is a branch point: the first `len`
 * branch points met take the outcome `path` gives (1 = the other side of the
 * boundary), later ones their own side.  Enumerating paths gives every result
 * a correct implementation of the same arithmetic may produce.
 */
#define OPATH_MAX 24
typedef struct {
    unsigned branch;        /* kinds (bit k = kind k) that branch */
    const uint8_t *path;
    int len;
    int seen;               /* branch points met so far */
    double kmin[M_COUNT];   /* smallest scaled margin per kind */
} octl;

static void ctl_init(octl *c, unsigned branch, const uint8_t *path, int len)
{
    c->branch = branch;
    c->path = path;
    c->len = len;
    c->seen = 0;
    for (int k = 0; k < M_COUNT; ++k) c->kmin[k] = INFINITY;
}

/* record a decision's margin m (already scaled); 1 if it takes the other side */
static int ctl_flip(octl *c, double m, int kind)
{
    if (m < c->kmin[kind]) c->kmin[kind] = m;
    if (!((c->branch >> kind) & 1u) || !(m < 1.0)) return 0;
    const int j = c->seen++;
    return j < c->len && j < OPATH_MAX && c->path[j] != 0;
}

static double ctl_margin(const octl *c, unsigned kinds)
{
    double m = INFINITY;
    for (int k = 0; k < M_COUNT; ++k)
        if (((kinds >> k) & 1u) && c->kmin[k] < m) m = c->kmin[k];
    return m;
}

static inline double mscale(double v, const double *delta, int k) { return v / delta[k]; }

/* kinds whose near-ties leave the forward (nearly) unchanged but not its
   derivative: the alpha clamp, the small-|A| branch, and an accepted root's
   conditioning */
#define GRAD_KINDS ((1u << M_CLAMP) | (1u << M_DCOND) | (1u << M_A))

/* l^2 / sigma^2 at ray parameter t (used only to decide which margins matter) */
static double support_E(const oprim *P, double t, const double dcam[3])
{
    double d[3];
    for (int j = 0; j < 3; ++j) d[j] = P->Rc[j] * dcam[0] + P->Rc[3 + j] * dcam[1] + P->Rc[6 + j] * dcam[2];
    const double x = P->o[0] + t * d[0], y = P->o[1] + t * d[1];
    const double Q = x * x / (P->s1 * P->s1) + y * y / (P->s2 * P->s2);
    const double rho = sqrt(x * x + y * y);
    const double h = P->l1 * x * x + P->l2 * y * y;
    const double u = rho > 0.0 ? 2.0 * fabs(h) / rho : 0.0;
    const double g = oracle_gfun(u);
    return g * g * Q;
}

/* ray-splat intersection with root selection (Sec. 3.2.1 and supplement) */
static void ray_hit(const oprim *P, const double dcam[3], const double *opts, const double *delta, octl *ctl,
                    ohit *H)
{
    double *d = H->d;
    for (int j = 0; j < 3; ++j) d[j] = P->Rc[j] * dcam[0] + P->Rc[3 + j] * dcam[1] + P->Rc[6 + j] * dcam[2];
    const double l1 = P->l1, l2 = P->l2, *o = P->o;
    const double A = l1 * d[0] * d[0] + l2 * d[1] * d[1];
    const double B = 2.0 * (l1 * o[0] * d[0] + l2 * o[1] * d[1]) - d[2];
    const double C = P->C;
    const double near_ = opts[O_NEAR], k2 = opts[O_K] * opts[O_K], Aeps = opts[O_AEPS];
    H->A = A; H->B = B; H->ok = 0;

    /* Roots in the cancellation-free form (Press et al., Numerical Recipes,
       5.6): q = -(B + sgn(B) sqrt(D)) / 2, roots q / A and C / q.  As A -> 0
       the root q / A runs off to infinity while C / q tends to the
       tangent-plane intersection -C / B (exactly that at A = 0).  Reading of
       the supplement's small-|A| case: for |A| < A_eps the diverging root is
       dropped and C / q is the one candidate. */
    const double D = B * B - 4.0 * A * C;
    /* D relative to its sensitivity to rounding in the quadratic re-centred
       where the ray reaches the centre's depth, t = t0 + s (D does not change
       under the shift): the form a renderer working relative to the
       primitive's centre evaluates.  The camera-origin coefficients carry the
       whole distance to the camera and would overstate the cancellation by
       |ohat| / sigma and more.  Rounding moves D = Bs^2 - 4 A Cs by about
       eps (2 |Bs| SB + 4 |Cs| SA + 4 |A| SC), where SA, SB, SC bound the
       rounding of A, Bs and Cs in units of eps: each local component of the
       ray and of the offset p0 carries an error of about eps times the whole
       vector's length (it comes out of a rotation), even when the component
       itself is small, as for a ray grazing the surface. */
    const double t0 = P->cc[2] / dcam[2];
    const double p0x = o[0] + t0 * d[0], p0y = o[1] + t0 * d[1], p0z = o[2] + t0 * d[2];
    const double Bs = 2.0 * (l1 * p0x * d[0] + l2 * p0y * d[1]) - d[2];
    const double Cs = l1 * p0x * p0x + l2 * p0y * p0y - p0z;
    const double pn = sqrt(p0x * p0x + p0y * p0y + p0z * p0z);  /* |d| = 1 */
    const double SA = 2.0 * (fabs(l1 * d[0]) + fabs(l2 * d[1]));
    const double SB = 2.0 * (fabs(l1) * (fabs(p0x) + fabs(d[0]) * pn) + fabs(l2) * (fabs(p0y) + fabs(d[1]) * pn)) + 1.0;
    const double SC = 2.0 * (fabs(l1 * p0x) + fabs(l2 * p0y)) * pn + pn;
    const double Drel =
        fabs(Bs * Bs - 4.0 * A * Cs) / (2.0 * fabs(Bs) * SB + 4.0 * fabs(Cs) * SA + 4.0 * fabs(A) * SC);
    /* the sign of D only matters where the double root t* = -B/(2A) would be
       inside (or at the edge of) the support */
    int hit = D >= 0.0;
    if (A != 0.0 && support_E(P, -B / (2.0 * A), dcam) <= 1.01 * k2)
        hit ^= ctl_flip(ctl, mscale(Drel, delta, M_D), M_D);
    double cand[2];
    int nc = 0;
    H->linear = fabs(A) < Aeps;
    if (hit) {
        /* a hit taken on the other side of D = 0 is the double root */
        const double sq = D > 0.0 ? sqrt(D) : 0.0;
        const double qq = -0.5 * (B + (B >= 0.0 ? sq : -sq));
        if (qq != 0.0) {
            const double rfin = C / qq;
            cand[nc++] = rfin;
            if (A != 0.0) {
                /* dropping the diverging root only matters where it could be
                   accepted */
                const double rdiv = qq / A;
                int keep = !H->linear;
                if (support_E(P, rdiv, dcam) <= 1.01 * k2)
                    keep ^= ctl_flip(ctl, mscale(fabs(fabs(A) - Aeps) / Aeps, delta, M_A), M_A);
                if (keep) {
                    cand[nc++] = rdiv;
                    if (rdiv < rfin) { cand[0] = rdiv; cand[1] = rfin; }
                }
            }
        } else if (A != 0.0) {
            cand[nc++] = 0.0;  /* B = D = 0: the double root at t = 0 */
        }
    }
    for (int ci = 0; ci < nc; ++ci) {
        const double t = cand[ci];
        const double zc = t * dcam[2];
        int front = zc > near_;
        if (support_E(P, t, dcam) <= 1.01 * k2)
            front ^= ctl_flip(ctl, mscale(fabs(zc - near_) / near_, delta, M_NEAR), M_NEAR);
        if (!front) continue;
        const double x = o[0] + t * d[0], y = o[1] + t * d[1];
        const double Q = x * x / (P->s1 * P->s1) + y * y / (P->s2 * P->s2);
        const double r2 = x * x + y * y;
        const double rho = sqrt(r2);
        const double h = l1 * x * x + l2 * y * y;
        const double u = rho > 0.0 ? 2.0 * fabs(h) / rho : 0.0;
        const double g = oracle_gfun(u);
        const double E = g * g * Q;
        const int inside = (E <= k2) ^ ctl_flip(ctl, mscale(fabs(E - k2) / k2, delta, M_E), M_E);
        if (inside) {
            H->ok = 1;
            H->t = t; H->x = x; H->y = y; H->Q = Q; H->rho = rho; H->h = h; H->u = u; H->g = g; H->E = E;
            H->F1 = 2.0 * A * t + B;
            ctl_flip(ctl, mscale(Drel, delta, M_DCOND), M_DCOND);
            break;
        }
    }
}

/* unit normal of the paraboloid at the hit, flipped to face the camera */
static void hit_normal(const oprim *P, const ohit *H, double nl[3], double *flip, double *vlen)
{
    const double v[3] = {-2.0 * P->l1 * H->x, -2.0 * P->l2 * H->y, 1.0};
    const double L = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    *vlen = L;
    for (int j = 0; j < 3; ++j) nl[j] = v[j] / L;
    const double nd = nl[0] * H->d[0] + nl[1] * H->d[1] + nl[2] * H->d[2];
    *flip = nd > 0.0 ? -1.0 : 1.0;
}

/* per-primitive backward accumulator in the primitive's own variables */
typedef struct {
    double dRc[9], dcc[3], dl[2], ds[2], dop, drgb[3];
} ograd;

typedef struct {
    int32_t list;   /* index into the active order */
    double alpha, T;
    double flip;    /* the normal's facing sign the forward took */
    ohit H;         /* the hit the forward took */
} oentry;

typedef struct {
    const oprim *prims;     /* compact: active primitives in window order */
    const int64_t *ids;     /* compact index -> original primitive index */
    int32_t *cell_start, *cell_items; /* CSR over cells of OT x OT pixels */
    int32_t cells_x, cells_y;
    /* per-tile order (frame != NULL): key-stage frames, centre depth keys and
       the key-stage camera */
    const double *frame;
    const uint32_t *dbits;
    const double *keycam;
    int32_t width, height;
    double near_key;
} obins;

/* an accepted hit waiting in the per-pixel resort buffer */
typedef struct {
    int32_t list;
    int32_t seq;  /* arrival order, for equal depths */
    double alpha;
    ohit H;
} opending;

typedef struct {
    uint64_t key, tie;
    int32_t item;
} ocand;

static int cmp_cand(const void *a, const void *b)
{
    const ocand *x = (const ocand *)a, *y = (const ocand *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->tie != y->tie) return x->tie < y->tie ? -1 : 1;
    return 0;
}

static void pixel_ray(const double *cam, int px, int py, double d[3])
{
    const double xn = ((px + 0.5) - cam[14]) / cam[12];
    const double yn = ((py + 0.5) - cam[15]) / cam[13];
    const double L = sqrt(xn * xn + yn * yn + 1.0);
    d[0] = xn / L; d[1] = yn / L; d[2] = 1.0 / L;
}

/* backward of one blended entry: dalpha plus direct output gradients */
/* Gaussian curvature of z = l1 x^2 + l2 y^2 at (x, y) (curvature equation,
   Sec. 3.2.1 and its derivation in the supplement) */
static double curvature_K(double l1, double l2, double x, double y)
{
    const double den = 1.0 + 4.0 * l1 * l1 * x * x + 4.0 * l2 * l2 * y * y;
    return 4.0 * l1 * l2 / (den * den);
}

static void entry_backward(const oprim *P, const ohit *H, double flip, const double *dcam, const double *opts,
                           double dalpha, double w, const double gc[3], double dt_direct, const double gn[3],
                           double dK, ograd *G)
{
    /* direct colour, depth (and the depth terms of median and distortion),
       normal (facing sign `flip` as the forward took it) and curvature terms */
    for (int c = 0; c < 3; ++c) G->drgb[c] += gc[c] * w;
    double dt = dt_direct;
    double nl[3], flip_natural, vlen;
    hit_normal(P, H, nl, &flip_natural, &vlen);
    double dncam[3] = {gn[0] * w, gn[1] * w, gn[2] * w};
    double dx = 0.0, dy = 0.0;
    /* n_cam = flip * Rc nl */
    double dnl[3];
    for (int j = 0; j < 3; ++j) {
        dnl[j] = flip * (P->Rc[j] * dncam[0] + P->Rc[3 + j] * dncam[1] + P->Rc[6 + j] * dncam[2]);
        for (int i = 0; i < 3; ++i) G->dRc[3 * i + j] += flip * dncam[i] * nl[j];
    }
    const double ndot = nl[0] * dnl[0] + nl[1] * dnl[1] + nl[2] * dnl[2];
    double dv[3];
    for (int j = 0; j < 3; ++j) dv[j] = (dnl[j] - nl[j] * ndot) / vlen;
    /* v = (-2 l1 x, -2 l2 y, 1) */
    G->dl[0] += -2.0 * H->x * dv[0];
    G->dl[1] += -2.0 * H->y * dv[1];
    dx += -2.0 * P->l1 * dv[0];
    dy += -2.0 * P->l2 * dv[1];
    /* K = 4 l1 l2 / den^2, den = 1 + 4 l1^2 x^2 + 4 l2^2 y^2 */
    if (dK != 0.0) {
        const double l1 = P->l1, l2 = P->l2, x = H->x, y = H->y;
        const double den = 1.0 + 4.0 * l1 * l1 * x * x + 4.0 * l2 * l2 * y * y;
        const double K = 4.0 * l1 * l2 / (den * den);
        const double dden = -2.0 * K / den * dK;  /* dK/dden = -2 K / den */
        G->dl[0] += 4.0 * l2 / (den * den) * dK + 8.0 * l1 * x * x * dden;
        G->dl[1] += 4.0 * l1 / (den * den) * dK + 8.0 * l2 * y * y * dden;
        dx += 8.0 * l1 * l1 * x * dden;
        dy += 8.0 * l2 * l2 * y * dden;
    }

    /* opacity and density: alpha = min(alpha_max, op G), G = exp(-E/2) */
    const double Gv = exp(-0.5 * H->E);
    double dG = 0.0;
    if (P->op * Gv < opts[O_AMAX]) {
        G->dop += dalpha * Gv;
        dG = dalpha * P->op;
    }
    const double dE = -0.5 * Gv * dG;
    /* E = g(u)^2 Q */
    const double dQ = H->g * H->g * dE;
    const double du = 2.0 * H->g * oracle_gprime(H->u) * H->Q * dE;
    /* Q = x^2/s1^2 + y^2/s2^2 */
    const double s1 = P->s1, s2 = P->s2;
    dx += 2.0 * H->x / (s1 * s1) * dQ;
    dy += 2.0 * H->y / (s2 * s2) * dQ;
    G->ds[0] += -2.0 * H->x * H->x / (s1 * s1 * s1) * dQ;
    G->ds[1] += -2.0 * H->y * H->y / (s2 * s2 * s2) * dQ;
    /* u = 2 |h| / rho, h = l1 x^2 + l2 y^2, rho = sqrt(x^2 + y^2) */
    if (H->rho > 0.0 && du != 0.0) {
        const double sg = H->h > 0.0 ? 1.0 : (H->h < 0.0 ? -1.0 : 0.0);
        const double dh = du * 2.0 * sg / H->rho;
        const double drho = -du * 2.0 * fabs(H->h) / (H->rho * H->rho);
        G->dl[0] += H->x * H->x * dh;
        G->dl[1] += H->y * H->y * dh;
        dx += 2.0 * P->l1 * H->x * dh + H->x / H->rho * drho;
        dy += 2.0 * P->l2 * H->y * dh + H->y / H->rho * drho;
    }
    /* phat = ohat + t dhat (only x, y are used) */
    const double *d = H->d;
    double dO[3] = {dx, dy, 0.0};
    double dD[3] = {H->t * dx, H->t * dy, 0.0};
    dt += d[0] * dx + d[1] * dy;
    /* root of A t^2 + B t + C = 0 (implicit differentiation) */
    const double dA = -H->t * H->t / H->F1 * dt;
    const double dB = -H->t / H->F1 * dt;
    const double dC = -1.0 / H->F1 * dt;
    const double *o = P->o, l1 = P->l1, l2 = P->l2;
    /* A = l1 d1^2 + l2 d2^2 */
    G->dl[0] += d[0] * d[0] * dA;
    G->dl[1] += d[1] * d[1] * dA;
    dD[0] += 2.0 * l1 * d[0] * dA;
    dD[1] += 2.0 * l2 * d[1] * dA;
    /* B = 2 (l1 o1 d1 + l2 o2 d2) - d3 */
    G->dl[0] += 2.0 * o[0] * d[0] * dB;
    G->dl[1] += 2.0 * o[1] * d[1] * dB;
    dO[0] += 2.0 * l1 * d[0] * dB;
    dO[1] += 2.0 * l2 * d[1] * dB;
    dD[0] += 2.0 * l1 * o[0] * dB;
    dD[1] += 2.0 * l2 * o[1] * dB;
    dD[2] += -dB;
    /* C = l1 o1^2 + l2 o2^2 - o3 */
    G->dl[0] += o[0] * o[0] * dC;
    G->dl[1] += o[1] * o[1] * dC;
    dO[0] += 2.0 * l1 * o[0] * dC;
    dO[1] += 2.0 * l2 * o[1] * dC;
    dO[2] += -dC;
    /* dhat = Rc^T dcam ; ohat = -Rc^T cc */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            G->dRc[3 * i + j] += dcam[i] * dD[j] - P->cc[i] * dO[j];
            G->dcc[i] += -P->Rc[3 * i + j] * dO[j];
        }
}

/* the whole per-pixel sequence; with g != NULL also its backward.  ctl holds
   the forced outcomes of near-tied decisions and receives every margin. */
static void render_pixel(const obins *B, const double *cam, const double *opts, const double *delta, octl *ctl,
                         int px, int py, int cell, double out[NCH], double *T_out, int32_t *nb_out,
                         int64_t *stop_out, int64_t *evals, const double g[NCH], int grad_skip, ograd *grads,
                         oentry **scratch, int *scratch_cap)
{
    double dcam[3];
    pixel_ray(cam, px, py, dcam);
    double T = 1.0, acc[NCH] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    int nb = 0, med_k = -1, med2_k = -1;
    double med = 0.0, med2 = -INFINITY;
    /* blended (w, t) for the depth distortion, kept for its plain double sum */
    double *wt = NULL;
    int wt_cap = 0;
    const int32_t s = B->cell_start[cell], e = B->cell_start[cell + 1];
    /* candidate order: the global (centre depth, index) order of the cell, or
       the order of the pixel's tile list by per-tile depth */
    ocand *order = NULL;
    if (B->frame && e > s) {
        order = (ocand *)malloc(sizeof(ocand) * (size_t)(e - s));
        for (int32_t it = s; it < e; ++it) {
            const int32_t li = B->cell_items[it];
            const int64_t p = B->ids[li];
            order[it - s].key = tile_depth_bits(B->frame + 16 * p, px / OT, py / OT, B->keycam, B->width, B->height,
                                                B->near_key);
            order[it - s].tie = ((uint64_t)B->dbits[p] << 32) | (uint64_t)p;
            order[it - s].item = li;
        }
        qsort(order, (size_t)(e - s), sizeof(ocand), cmp_cand);
    }
    /* the backward runs only if some upstream gradient of the pixel is non-zero */
    int do_bwd = 0;
    if (g)
        for (int c = 0; c < NCH; ++c) do_bwd |= g[c] != 0.0;
    if (stop_out) *stop_out = -1;
    /* per-pixel resort (supplement, per-pixel resorting): accepted hits wait in
       a buffer of K entries; whenever it is full the nearest (smallest t, the
       earliest arrival among equal t) is blended, and at the end of the list
       the rest in the same way.  K <= 1 blends in list order. */
    const int K = opts[O_RESORT] > 1.0 ? (int)opts[O_RESORT] : 1;
    opending *buf = (opending *)malloc(sizeof(opending) * (size_t)K);
    int nbuf = 0, nseq = 0, stopped = 0;
    for (int32_t it = s; it <= e && !stopped; ++it) {
        if (it < e) {
            const int32_t li = order ? order[it - s].item : B->cell_items[it];
            const oprim *P = &B->prims[li];
            ohit H;
            ++*evals;
            ray_hit(P, dcam, opts, delta, ctl, &H);
            if (!H.ok) continue;
            const double Gv = exp(-0.5 * H.E);
            const double aa = P->op * Gv;
            ctl_flip(ctl, mscale(fabs(aa - opts[O_AMAX]) / opts[O_AMAX], delta, M_CLAMP), M_CLAMP);
            const double alpha = aa < opts[O_AMAX] ? aa : opts[O_AMAX];
            const int skip = (alpha < opts[O_AMIN]) ^
                             ctl_flip(ctl, mscale(fabs(alpha - opts[O_AMIN]) / opts[O_AMIN], delta, M_AMIN), M_AMIN);
            if (skip) continue;
            buf[nbuf].list = li;
            buf[nbuf].seq = nseq++;
            buf[nbuf].alpha = alpha;
            buf[nbuf].H = H;
            ++nbuf;
            if (nbuf < K) continue;
        }
        /* blend: one entry when the buffer is full, all of them at the end */
        while (nbuf > 0 && !stopped) {
            int best = 0;
            for (int b = 1; b < nbuf; ++b)
                if (buf[b].H.t < buf[best].H.t || (buf[b].H.t == buf[best].H.t && buf[b].seq < buf[best].seq))
                    best = b;
            if (nbuf > 1) {
                /* choosing the nearest of two close depths is a discrete
                   decision; its other side takes the runner-up */
                int next = -1;
                for (int b = 0; b < nbuf; ++b)
                    if (b != best && (next < 0 || buf[b].H.t < buf[next].H.t ||
                                      (buf[b].H.t == buf[next].H.t && buf[b].seq < buf[next].seq)))
                        next = b;
                const double gap = buf[next].H.t - buf[best].H.t;
                if (ctl_flip(ctl, mscale(gap / fabs(buf[best].H.t), delta, M_SORT), M_SORT)) best = next;
            }
            const opending en = buf[best];
            buf[best] = buf[--nbuf];
            const oprim *P = &B->prims[en.list];
            const ohit H = en.H;
            const double alpha = en.alpha;
            const double Tn = T * (1.0 - alpha);
            const int stop = (Tn < opts[O_TEPS]) ^
                             ctl_flip(ctl, mscale(fabs(Tn - opts[O_TEPS]) / opts[O_TEPS], delta, M_T), M_T);
            if (stop) {
                stopped = 1;
                if (stop_out) *stop_out = B->ids[en.list];
                break;
            }
            const double w = alpha * T;
            double nl[3], flip, vlen;
            hit_normal(P, &H, nl, &flip, &vlen);
            if (ctl_flip(ctl, mscale(fabs(nl[0] * H.d[0] + nl[1] * H.d[1] + nl[2] * H.d[2]), delta, M_N), M_N))
                flip = -flip;
            for (int c = 0; c < 3; ++c) acc[c] += w * P->rgb[c];
            acc[CH_DEPTH] += w * H.t;
            for (int i = 0; i < 3; ++i)
                acc[CH_N + i] += w * flip * (P->Rc[3 * i] * nl[0] + P->Rc[3 * i + 1] * nl[1] + P->Rc[3 * i + 2] * nl[2]);
            acc[CH_K] += w * curvature_K(P->l1, P->l2, H.x, H.y);
            /* median depth (mesh extraction, Sec. 4.1): the largest hit depth among
               entries whose incoming transmittance exceeds 0.5 */
            const int qualifies = (T > 0.5) ^ ctl_flip(ctl, mscale(fabs(T - 0.5) / 0.5, delta, M_MED), M_MED);
            if (qualifies) {
                if (med_k < 0 || H.t > med) {
                    if (med_k >= 0) { med2 = med; med2_k = med_k; }
                    med = H.t;
                    med_k = nb;
                } else if (H.t > med2) {
                    med2 = H.t;
                    med2_k = nb;
                }
            }
            if (nb >= wt_cap) {
                wt_cap = wt_cap ? 2 * wt_cap : 64;
                wt = (double *)realloc(wt, sizeof(double) * 2 * (size_t)wt_cap);
            }
            wt[2 * nb] = w;
            wt[2 * nb + 1] = H.t;
            if (do_bwd) {
                if (nb >= *scratch_cap) {
                    *scratch_cap = *scratch_cap ? 2 * *scratch_cap : 256;
                    *scratch = (oentry *)realloc(*scratch, sizeof(oentry) * (size_t)*scratch_cap);
                }
                (*scratch)[nb].list = en.list;
                (*scratch)[nb].alpha = alpha;
                (*scratch)[nb].T = T;
                (*scratch)[nb].flip = flip;
                (*scratch)[nb].H = H;
            }
            ++nb;
            T = Tn;
            if (it < e) break; /* one blend per arrival while the list lasts */
        }
    }
    free(buf);
    free(order);
    /* depth distortion (Sec. 3.3): sum_i sum_{j<i} w_i w_j (t_i - t_j)^2 */
    double dist = 0.0, W = 0.0;
    for (int i = 0; i < nb; ++i) {
        W += wt[2 * i];
        for (int j = 0; j < i; ++j) {
            const double d = wt[2 * i + 1] - wt[2 * j + 1];
            dist += wt[2 * i] * wt[2 * j] * d * d;
        }
    }
    /* the median's choice between two close hit depths is a discrete decision;
       its other side takes the second largest */
    if (med_k >= 0 && med2_k >= 0) {
        if (ctl_flip(ctl, mscale((med - med2) / fabs(med), delta, M_MED), M_MED)) {
            med = med2;
            med_k = med2_k;
        }
    }
    acc[CH_MED] = med;
    acc[CH_DIST] = dist;
    for (int c = 0; c < 3; ++c) acc[c] += T * opts[O_BG + c];
    for (int c = 0; c < NCH; ++c) out[c] = acc[c];
    *T_out = T;
    *nb_out = nb;

    /* grad_skip: a pixel whose derivative is ill-conditioned or ambiguous
       (a near-tie of GRAD_KINDS) contributes no gradient */
    if (grad_skip && ctl_margin(ctl, GRAD_KINDS) < 1.0) do_bwd = 0;
    if (!do_bwd) {
        free(wt);
        return;
    }
    /* back to front: S_c = sum_{j>i} w_j X_j,c (+ T_final bg for colour).
       Distortion: L = W B - A^2 over all blended entries (W = sum w, A = sum w t,
       B = sum w t^2), so dL/dw_i = L/W + W (t_i - A/W)^2 and
       dL/dt_i = 2 w_i W (t_i - A/W); the first is the distortion channel's X_i. */
    const double A = acc[CH_DEPTH], mean = W > 0.0 ? A / W : 0.0;
    enum { NX = 9 };  /* colour 3, depth, normal 3, curvature, distortion */
    double S[NX] = {T * opts[O_BG], T * opts[O_BG + 1], T * opts[O_BG + 2], 0, 0, 0, 0, 0, 0};
    double gx[NX];
    for (int c = 0; c < 8; ++c) gx[c] = g[c];
    gx[8] = g[CH_DIST];
    for (int k = nb - 1; k >= 0; --k) {
        const oentry *en = &(*scratch)[k];
        const oprim *P = &B->prims[en->list];
        const ohit *H = &en->H;
        double nl[3], flip_natural, vlen;
        hit_normal(P, H, nl, &flip_natural, &vlen);
        const double flip = en->flip;
        double X[NX];
        for (int c = 0; c < 3; ++c) X[c] = P->rgb[c];
        X[3] = H->t;
        for (int i = 0; i < 3; ++i)
            X[4 + i] = flip * (P->Rc[3 * i] * nl[0] + P->Rc[3 * i + 1] * nl[1] + P->Rc[3 * i + 2] * nl[2]);
        X[7] = curvature_K(P->l1, P->l2, H->x, H->y);
        X[8] = (W > 0.0 ? dist / W : 0.0) + W * (H->t - mean) * (H->t - mean);
        const double a = en->alpha, Ti = en->T, w = a * Ti;
        double dalpha = 0.0;
        for (int c = 0; c < NX; ++c) dalpha += gx[c] * (Ti * X[c] - S[c] / (1.0 - a));
        for (int c = 0; c < NX; ++c) S[c] += w * X[c];
        double dt = g[CH_DEPTH] * w + g[CH_DIST] * 2.0 * w * W * (H->t - mean);
        if (k == med_k) dt += g[CH_MED];
        entry_backward(P, H, flip, dcam, opts, dalpha, w, g, dt, g + CH_N, g[CH_K] * w, &grads[en->list]);
    }
    free(wt);
}

/* conservative pixel box of the ball |p - cc| <= r (oracle's own binning) */
static int ball_box(const double cc[3], double r, const double *cam, double near_, int width, int height,
                    int *px0, int *py0, int *px1, int *py1)
{
    if (cc[2] - r <= near_) {
        *px0 = 0; *py0 = 0; *px1 = width - 1; *py1 = height - 1;
        return 1;
    }
    const double za = cc[2] - r, zb = cc[2] + r;
    const double xl = fmin((cc[0] - r) / za, (cc[0] - r) / zb), xh = fmax((cc[0] + r) / za, (cc[0] + r) / zb);
    const double yl = fmin((cc[1] - r) / za, (cc[1] - r) / zb), yh = fmax((cc[1] + r) / za, (cc[1] + r) / zb);
    const double u0 = cam[12] * xl + cam[14] - 0.5 - 1.0, u1 = cam[12] * xh + cam[14] - 0.5 + 1.0;
    const double v0 = cam[13] * yl + cam[15] - 0.5 - 1.0, v1 = cam[13] * yh + cam[15] - 0.5 + 1.0;
    if (u1 < 0 || v1 < 0 || u0 > width - 1 || v0 > height - 1) return 0;
    *px0 = u0 < 0 ? 0 : (int)ceil(u0);
    *px1 = u1 > width - 1 ? width - 1 : (int)floor(u1);
    *py0 = v0 < 0 ? 0 : (int)ceil(v0);
    *py1 = v1 > height - 1 ? height - 1 : (int)floor(v1);
    return *px0 <= *px1 && *py0 <= *py1;
}

typedef struct { uint32_t key; int64_t id; } oorder;

static int cmp_order(const void *a, const void *b)
{
    const oorder *x = (const oorder *)a, *y = (const oorder *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->id < y->id ? -1 : (x->id > y->id);
}

/* active primitives of a window, in global order, binned into cells of
   OT x OT window pixels with the projected-ball bound */
typedef struct {
    obins B;
    oprim *tmp;
    int64_t *ids, nw;
    int32_t *cnt, *items, *box;
    oorder *ord;
} owin;

static void window_bins(owin *Wn, int64_t n, const double *center, const double *quat, const double *scale,
                        const double *curv, const double *opac, const double *rgb, const uint8_t *culled,
                        const uint32_t *depth_bits, const double *frame, const double *keycam, const double *cam,
                        int32_t width, int32_t height, const double *opts, int32_t x0, int32_t y0, int32_t w,
                        int32_t h, const double *sh, int32_t sh_deg)
{
    const double *W = cam, *T = cam + 9;
    /* active primitives in global order: depth key, then index */
    int64_t na = 0;
    for (int64_t p = 0; p < n; ++p) na += culled[p] ? 0 : 1;
    oorder *ord = (oorder *)malloc(sizeof(oorder) * (size_t)(na > 0 ? na : 1));
    na = 0;
    for (int64_t p = 0; p < n; ++p)
        if (!culled[p]) { ord[na].key = depth_bits[p]; ord[na].id = p; ++na; }
    qsort(ord, (size_t)na, sizeof(oorder), cmp_order);

    /* bin into window cells with the ball bound; keep only primitives that touch */
    const int cx_n = (w + OT - 1) / OT, cy_n = (h + OT - 1) / OT, ncell = cx_n * cy_n;
    int32_t *cnt = (int32_t *)calloc((size_t)ncell + 1, sizeof(int32_t));
    int32_t *box = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)(na > 0 ? na : 1));
    oprim *tmp = (oprim *)malloc(sizeof(oprim) * (size_t)(na > 0 ? na : 1));
    int64_t nw = 0;
    int64_t *ids = (int64_t *)malloc(sizeof(int64_t) * (size_t)(na > 0 ? na : 1));
    for (int64_t i = 0; i < na; ++i) {
        const int64_t p = ord[i].id;
        oprim P;
        double shrgb[3], sdir[3], sdist;
        int slive[3];
        if (sh)
            sh_colour(sh_deg, sh + 3 * (sh_deg + 1) * (sh_deg + 1) * p, center + 3 * p, W, T, shrgb, sdir, &sdist,
                      slive);
        setup_prim(center + 3 * p, quat + 4 * p, scale + 2 * p, curv + 2 * p, opac[p], sh ? shrgb : rgb + 3 * p, W, T,
                   &P);
        const double r = opts[O_K] * (P.s1 > P.s2 ? P.s1 : P.s2) * 1.01 + 1e-9;
        int a0, b0, a1, b1;
        if (!ball_box(P.cc, r, cam, opts[O_NEAR], width, height, &a0, &b0, &a1, &b1)) continue;
        /* intersect with window, to cell coordinates */
        if (a1 < x0 || b1 < y0 || a0 >= x0 + w || b0 >= y0 + h) continue;
        a0 = (a0 < x0 ? x0 : a0) - x0; a1 = (a1 >= x0 + w ? x0 + w - 1 : a1) - x0;
        b0 = (b0 < y0 ? y0 : b0) - y0; b1 = (b1 >= y0 + h ? y0 + h - 1 : b1) - y0;
        box[4 * nw] = a0 / OT; box[4 * nw + 1] = b0 / OT; box[4 * nw + 2] = a1 / OT; box[4 * nw + 3] = b1 / OT;
        tmp[nw] = P;
        ids[nw] = p;
        for (int cy = box[4 * nw + 1]; cy <= box[4 * nw + 3]; ++cy)
            for (int cx = box[4 * nw]; cx <= box[4 * nw + 2]; ++cx) cnt[cy * cx_n + cx + 1]++;
        ++nw;
    }
    for (int c = 0; c < ncell; ++c) cnt[c + 1] += cnt[c];
    int32_t *items = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cnt[ncell] > 0 ? cnt[ncell] : 1));
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncell > 0 ? ncell : 1));
    memcpy(fill, cnt, sizeof(int32_t) * (size_t)ncell);
    for (int64_t i = 0; i < nw; ++i)
        for (int cy = box[4 * i + 1]; cy <= box[4 * i + 3]; ++cy)
            for (int cx = box[4 * i]; cx <= box[4 * i + 2]; ++cx) items[fill[cy * cx_n + cx]++] = (int32_t)i;
    free(fill);
    obins Bn = {tmp, ids, cnt, items, cx_n, cy_n, frame, depth_bits, keycam, width, height, opts[O_NEAR]};
    Wn->B = Bn;
    Wn->tmp = tmp;
    Wn->ids = ids;
    Wn->nw = nw;
    Wn->cnt = cnt;
    Wn->items = items;
    Wn->box = box;
    Wn->ord = ord;
}

static void window_free(owin *Wn)
{
    free(Wn->items); free(Wn->cnt); free(Wn->box); free(Wn->tmp); free(Wn->ids); free(Wn->ord);
}

/* decision kinds that change the compared maps (colour, depth, normal, T and,
   with branch_median, the median depth) */
static unsigned forward_kinds(int branch_median)
{
    unsigned k = (1u << M_A) | (1u << M_D) | (1u << M_NEAR) | (1u << M_E) | (1u << M_AMIN) | (1u << M_T) |
                 (1u << M_N) | (1u << M_SORT);
    if (branch_median) k |= 1u << M_MED;
    return k;
}


/*
 * Render the pixel window [x0, x0+w) x [y0, y0+h) of a width x height view.
 * Parameters are FP64 (exact copies of FP32 inputs, or perturbed for finite
 * differences).  culled/depth_bits come from oracle_keys and fix the active set
 * and the order; with frame != NULL (oracle_keys' frames, and keycam the
 * key-stage camera) each pixel takes its tile's per-tile-depth order instead.
 * opts[O_RESORT] > 1 enables the per-pixel resort buffer of that size.
 * cam = {R[9], t[3], fx, fy, cx, cy}.
 * Outputs (window-sized, planar): color[3][h][w], depth, normal[3][h][w],
 * T_final, n_blend (entries blended), margin (min over the decisions of the
 * kinds forward_kinds(branch_median) selects of the scaled distance to the
 * boundary), optional gmargin (the same over GRAD_KINDS), kind_bits (bit k
 * set where kind k has a margin below 1) and stop_id (the primitive at which
 * the pixel stopped, -1 if it did not).
 * Near-tied decisions of the window pixels forced[i] (row-major index in the
 * window, i < n_forced) take the outcomes forced_path[i * OPATH_MAX ...] of
 * their first forced_len[i] branch points (see octl).
 * If dL_color != NULL the backward runs and parameter gradients are written
 * (full [n] arrays, zero for inactive primitives); with grad_skip, pixels
 * whose gmargin is below 1 contribute none.
 * Returns the number of (pixel, candidate) evaluations, or -1 on error.
 */
int64_t oracle_render(int64_t n, const double *center, const double *quat, const double *scale,
                      const double *curv, const double *opac, const double *rgb,
                      const uint8_t *culled, const uint32_t *depth_bits, const double *frame,
                      const double *keycam, const double *cam, int32_t width, int32_t height,
                      const double *opts, const double *delta,
                      int32_t x0, int32_t y0, int32_t w, int32_t h, int32_t nthreads,
                      double *color, double *depth, double *normal, double *T_final,
                      int32_t *n_blend, double *margin, double *curvature, double *median_depth,
                      double *distortion,
                      const double *dL_color, const double *dL_depth, const double *dL_normal,
                      const double *dL_curv, const double *dL_median, const double *dL_dist,
                      double *g_center, double *g_quat, double *g_scale, double *g_curv,
                      double *g_opac, double *g_rgb, const double *sh, int32_t sh_deg, double *g_sh,
                      int32_t branch_median, int64_t n_forced, const int32_t *forced, const uint8_t *forced_path,
                      const int32_t *forced_len, double *gmargin, uint16_t *kind_bits, int32_t grad_skip,
                      int64_t *stop_id)
{
    if (w <= 0 || h <= 0 || x0 < 0 || y0 < 0 || x0 + w > width || y0 + h > height) return -1;
    const double *W = cam, *T = cam + 9;
    owin Wn;
    window_bins(&Wn, n, center, quat, scale, curv, opac, rgb, culled, depth_bits, frame, keycam, cam, width, height,
                opts, x0, y0, w, h, sh, sh_deg);
    const obins Bn = Wn.B;
    const int64_t nw = Wn.nw;
    const int64_t *ids = Wn.ids;
    const oprim *tmp = Wn.tmp;
    const int cx_n = Bn.cells_x;
    const unsigned fkinds = forward_kinds(branch_median);
    /* window pixel -> forced path */
    int32_t *fmap = NULL;
    if (n_forced > 0) {
        fmap = (int32_t *)malloc(sizeof(int32_t) * (size_t)w * (size_t)h);
        for (size_t i = 0; i < (size_t)w * (size_t)h; ++i) fmap[i] = -1;
        for (int64_t i = 0; i < n_forced; ++i)
            if (forced[i] >= 0 && (int64_t)forced[i] < (int64_t)w * h) fmap[forced[i]] = (int32_t)i;
    }

    int nthr = nthreads > 0 ? nthreads : 1;
#ifdef _OPENMP
    omp_set_num_threads(nthr);
#else
    nthr = 1;
#endif
    const int do_bwd = dL_color != NULL;
    ograd *grads = NULL;
    if (do_bwd) grads = (ograd *)calloc((size_t)nthr * (size_t)(nw > 0 ? nw : 1), sizeof(ograd));
    int64_t evals_total = 0;
    const size_t npx = (size_t)w * h;

#pragma omp parallel num_threads(nthr) reduction(+ : evals_total)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        oentry *scratch = NULL;
        int cap = 0;
        int64_t ev = 0;
        ograd *mine = do_bwd ? grads + (size_t)tid * (size_t)(nw > 0 ? nw : 1) : NULL;
#pragma omp for schedule(static, 1)
        for (int j = 0; j < h; ++j) {
            for (int i = 0; i < w; ++i) {
                const size_t pix = (size_t)j * w + i;
                const int cell = (j / OT) * cx_n + (i / OT);
                double out[NCH], Tf, mg;
                int32_t nb;
                double gg[NCH] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
                if (do_bwd) {
                    for (int c = 0; c < 3; ++c) gg[c] = dL_color[c * npx + pix];
                    gg[CH_DEPTH] = dL_depth[pix];
                    for (int c = 0; c < 3; ++c) gg[CH_N + c] = dL_normal[c * npx + pix];
                    if (dL_curv) gg[CH_K] = dL_curv[pix];
                    if (dL_median) gg[CH_MED] = dL_median[pix];
                    if (dL_dist) gg[CH_DIST] = dL_dist[pix];
                }
                octl ctl;
                const int32_t fi = fmap ? fmap[pix] : -1;
                if (fi >= 0)
                    ctl_init(&ctl, fkinds, forced_path + (size_t)fi * OPATH_MAX,
                             forced_len[fi] < OPATH_MAX ? forced_len[fi] : OPATH_MAX);
                else
                    ctl_init(&ctl, fkinds, NULL, 0);
                render_pixel(&Bn, cam, opts, delta, &ctl, x0 + i, y0 + j, cell, out, &Tf, &nb,
                             stop_id ? stop_id + pix : NULL, &ev, do_bwd ? gg : NULL, grad_skip, mine, &scratch,
                             &cap);
                mg = ctl_margin(&ctl, fkinds);
                if (gmargin) gmargin[pix] = ctl_margin(&ctl, GRAD_KINDS);
                if (kind_bits) {
                    uint16_t bits = 0;
                    for (int k = 0; k < M_COUNT; ++k)
                        if (ctl.kmin[k] < 1.0) bits |= (uint16_t)(1u << k);
                    kind_bits[pix] = bits;
                }
                for (int c = 0; c < 3; ++c) color[c * npx + pix] = out[c];
                depth[pix] = out[CH_DEPTH];
                for (int c = 0; c < 3; ++c) normal[c * npx + pix] = out[CH_N + c];
                if (curvature) curvature[pix] = out[CH_K];
                if (median_depth) median_depth[pix] = out[CH_MED];
                if (distortion) distortion[pix] = out[CH_DIST];
                T_final[pix] = Tf;
                n_blend[pix] = nb;
                margin[pix] = mg;
            }
        }
        free(scratch);
        evals_total += ev;
    }

    if (do_bwd) {
        memset(g_center, 0, sizeof(double) * 3 * (size_t)n);
        memset(g_quat, 0, sizeof(double) * 4 * (size_t)n);
        memset(g_scale, 0, sizeof(double) * 2 * (size_t)n);
        memset(g_curv, 0, sizeof(double) * 2 * (size_t)n);
        memset(g_opac, 0, sizeof(double) * (size_t)n);
        memset(g_rgb, 0, sizeof(double) * 3 * (size_t)n);
        if (sh) memset(g_sh, 0, sizeof(double) * 3 * (size_t)((sh_deg + 1) * (sh_deg + 1)) * (size_t)n);
        for (int64_t i = 0; i < nw; ++i) {
            ograd S;
            memset(&S, 0, sizeof S);
            for (int t = 0; t < nthr; ++t) {
                const ograd *gt = &grads[(size_t)t * (size_t)nw + (size_t)i];
                for (int k = 0; k < 9; ++k) S.dRc[k] += gt->dRc[k];
                for (int k = 0; k < 3; ++k) { S.dcc[k] += gt->dcc[k]; S.drgb[k] += gt->drgb[k]; }
                for (int k = 0; k < 2; ++k) { S.dl[k] += gt->dl[k]; S.ds[k] += gt->ds[k]; }
                S.dop += gt->dop;
            }
            const int64_t p = ids[i];
            const oprim *P = &tmp[i];
            /* cc = W c + t  ->  dc = W^T dcc */
            for (int j = 0; j < 3; ++j)
                g_center[3 * p + j] = W[j] * S.dcc[0] + W[3 + j] * S.dcc[1] + W[6 + j] * S.dcc[2];
            /* Rc = W Rm  ->  dRm = W^T dRc */
            double dRm[9];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    dRm[3 * a + b] = W[a] * S.dRc[b] + W[3 + a] * S.dRc[3 + b] + W[6 + a] * S.dRc[6 + b];
            /* Rm(qhat) entry derivatives, qhat = (w, x, y, z) */
            const double qw = P->qn[0], qx = P->qn[1], qy = P->qn[2], qz = P->qn[3];
            double dq[4] = {0, 0, 0, 0};
            /* R00 = 1 - 2(y^2 + z^2) */
            dq[2] += -4 * qy * dRm[0]; dq[3] += -4 * qz * dRm[0];
            /* R01 = 2(xy - wz) */
            dq[0] += -2 * qz * dRm[1]; dq[1] += 2 * qy * dRm[1]; dq[2] += 2 * qx * dRm[1]; dq[3] += -2 * qw * dRm[1];
            /* R02 = 2(xz + wy) */
            dq[0] += 2 * qy * dRm[2]; dq[1] += 2 * qz * dRm[2]; dq[2] += 2 * qw * dRm[2]; dq[3] += 2 * qx * dRm[2];
            /* R10 = 2(xy + wz) */
            dq[0] += 2 * qz * dRm[3]; dq[1] += 2 * qy * dRm[3]; dq[2] += 2 * qx * dRm[3]; dq[3] += 2 * qw * dRm[3];
            /* R11 = 1 - 2(x^2 + z^2) */
            dq[1] += -4 * qx * dRm[4]; dq[3] += -4 * qz * dRm[4];
            /* R12 = 2(yz - wx) */
            dq[0] += -2 * qx * dRm[5]; dq[1] += -2 * qw * dRm[5]; dq[2] += 2 * qz * dRm[5]; dq[3] += 2 * qy * dRm[5];
            /* R20 = 2(xz - wy) */
            dq[0] += -2 * qy * dRm[6]; dq[1] += 2 * qz * dRm[6]; dq[2] += -2 * qw * dRm[6]; dq[3] += 2 * qx * dRm[6];
            /* R21 = 2(yz + wx) */
            dq[0] += 2 * qx * dRm[7]; dq[1] += 2 * qw * dRm[7]; dq[2] += 2 * qz * dRm[7]; dq[3] += 2 * qy * dRm[7];
            /* R22 = 1 - 2(x^2 + y^2) */
            dq[1] += -4 * qx * dRm[8]; dq[2] += -4 * qy * dRm[8];
            /* qhat = q / |q| */
            const double dotq = qw * dq[0] + qx * dq[1] + qy * dq[2] + qz * dq[3];
            for (int k = 0; k < 4; ++k) g_quat[4 * p + k] = (dq[k] - P->qn[k] * dotq) / P->qlen;
            g_scale[2 * p] = S.ds[0];
            g_scale[2 * p + 1] = S.ds[1];
            g_curv[2 * p] = S.dl[0];
            g_curv[2 * p + 1] = S.dl[1];
            g_opac[p] = S.dop;
            for (int k = 0; k < 3; ++k) g_rgb[3 * p + k] = S.drgb[k];
            if (sh) {
                /* rgb_c = max(0, sum_k sh[k][c] Y_k(d) + 1/2), d = (c - o) / |c - o| */
                const int K = (sh_deg + 1) * (sh_deg + 1);
                const double *cf = sh + 3 * K * p;
                double rgb_[3], d[3], r;
                int live[3];
                sh_colour(sh_deg, cf, center + 3 * p, W, T, rgb_, d, &r, live);
                double Y[16], dY[16][3];
                sh_basis(sh_deg, d[0], d[1], d[2], Y, dY);
                double gd[3] = {0, 0, 0};
                for (int ch = 0; ch < 3; ++ch) {
                    const double gch = live[ch] ? S.drgb[ch] : 0.0;
                    for (int k = 0; k < K; ++k) {
                        g_sh[3 * K * p + 3 * k + ch] = Y[k] * gch;
                        for (int j = 0; j < 3; ++j) gd[j] += gch * cf[3 * k + ch] * dY[k][j];
                    }
                }
                const double dg = d[0] * gd[0] + d[1] * gd[1] + d[2] * gd[2];
                for (int j = 0; j < 3; ++j) g_center[3 * p + j] += (gd[j] - d[j] * dg) / r;
            }
        }
        free(grads);
    }
    free(fmap);
    window_free(&Wn);
    return evals_total;
}

/*
 * Every result the window pixels pix[i] (row-major index in the window) may
 * take when their near-tied decisions (kinds forward_kinds(branch_median)) go
 * either way: a depth-first walk over the branch points (octl) with at most
 * max_leaves results per pixel.  The outputs per pixel are n_leaves[i] and
 * overflow[i] (1 if the walk stopped at max_leaves or met more than OPATH_MAX
 * branch points); per result j of pixel i, at r = i * max_leaves + j:
 * vals[r * (NCH + 1) + c] = colour 0-2, depth, normal 4-6, curvature, median
 * depth, distortion, then T_final; paths[r * OPATH_MAX + k] the outcome of its
 * k-th branch point (1 = the other side) and plen[r] their number.  Result 0
 * is the one every decision takes on its own side.  Returns the number of
 * evaluations, or -1 on error.
 */
int64_t oracle_render_alts(int64_t n, const double *center, const double *quat, const double *scale,
                           const double *curv, const double *opac, const double *rgb,
                           const uint8_t *culled, const uint32_t *depth_bits, const double *frame,
                           const double *keycam, const double *cam, int32_t width, int32_t height,
                           const double *opts, const double *delta,
                           int32_t x0, int32_t y0, int32_t w, int32_t h, int32_t nthreads,
                           const double *sh, int32_t sh_deg, int32_t branch_median,
                           int64_t npix, const int32_t *pix, int32_t max_leaves,
                           int32_t *n_leaves, uint8_t *overflow, double *vals, uint8_t *paths, int32_t *plen)
{
    if (w <= 0 || h <= 0 || x0 < 0 || y0 < 0 || x0 + w > width || y0 + h > height || max_leaves < 1) return -1;
    for (int64_t i = 0; i < npix; ++i)
        if (pix[i] < 0 || (int64_t)pix[i] >= (int64_t)w * h) return -1;
    owin Wn;
    window_bins(&Wn, n, center, quat, scale, curv, opac, rgb, culled, depth_bits, frame, keycam, cam, width, height,
                opts, x0, y0, w, h, sh, sh_deg);
    const unsigned fkinds = forward_kinds(branch_median);
    const int cx_n = Wn.B.cells_x;
    int nthr = nthreads > 0 ? nthreads : 1;
#ifdef _OPENMP
    omp_set_num_threads(nthr);
#else
    nthr = 1;
#endif
    int64_t evals_total = 0;
#pragma omp parallel num_threads(nthr) reduction(+ : evals_total)
    {
        /* stack of paths still to walk: their outcomes and lengths */
        int cap = 64, top = 0;
        uint8_t *stk = (uint8_t *)malloc((size_t)cap * OPATH_MAX);
        int32_t *stk_len = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
        int64_t ev = 0;
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < npix; ++i) {
            const int px = x0 + pix[i] % w, py = y0 + pix[i] / w;
            const int cell = ((py - y0) / OT) * cx_n + (px - x0) / OT;
            int leaves = 0;
            uint8_t ovf = 0;
            top = 0;
            memset(stk, 0, OPATH_MAX);
            stk_len[0] = 0;
            top = 1;
            while (top > 0) {
                --top;
                uint8_t node[OPATH_MAX];
                memcpy(node, stk + (size_t)top * OPATH_MAX, OPATH_MAX);
                const int L = stk_len[top];
                if (leaves == max_leaves) { ovf = 1; break; }
                octl ctl;
                ctl_init(&ctl, fkinds, node, L);
                double out[NCH], Tf;
                int32_t nb;
                render_pixel(&Wn.B, cam, opts, delta, &ctl, px, py, cell, out, &Tf, &nb, NULL, &ev, NULL, 0, NULL,
                             NULL, NULL);
                int m = ctl.seen;
                if (m > OPATH_MAX) { ovf = 1; m = OPATH_MAX; }
                const size_t r = (size_t)i * (size_t)max_leaves + (size_t)leaves;
                for (int c = 0; c < NCH; ++c) vals[r * (NCH + 1) + c] = out[c];
                vals[r * (NCH + 1) + NCH] = Tf;
                memset(paths + r * OPATH_MAX, 0, OPATH_MAX);
                memcpy(paths + r * OPATH_MAX, node, (size_t)L);
                plen[r] = m;
                ++leaves;
                /* children: the natural outcomes up to branch point j, then the other side at j */
                for (int j = m - 1; j >= L; --j) {
                    if (top == cap) {
                        cap *= 2;
                        stk = (uint8_t *)realloc(stk, (size_t)cap * OPATH_MAX);
                        stk_len = (int32_t *)realloc(stk_len, sizeof(int32_t) * (size_t)cap);
                    }
                    uint8_t *c = stk + (size_t)top * OPATH_MAX;
                    memset(c, 0, OPATH_MAX);
                    memcpy(c, node, (size_t)L);
                    c[j] = 1;
                    stk_len[top] = j + 1;
                    ++top;
                }
            }
            n_leaves[i] = leaves;
            overflow[i] = ovf;
        }
        free(stk);
        free(stk_len);
        evals_total += ev;
    }
    window_free(&Wn);
    return evals_total;
}

/*
 * Single ray against a single primitive (FP64), for pin tests.
 * out = {ok, linear, t, x, y, z_on_surface, E, G, A, B, C, n_cam[3] (flipped), K}.
 */
void oracle_ray_hit(const double *c, const double *q, const double *s, const double *l,
                    const double *cam, const double *dcam, const double *opts, double *out)
{
    const double delta[M_COUNT] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
    oprim P;
    setup_prim(c, q, s, l, 1.0, (const double[3]){0, 0, 0}, cam, cam + 9, &P);
    ohit H;
    octl ctl;
    ctl_init(&ctl, 0u, NULL, 0);
    ray_hit(&P, dcam, opts, delta, &ctl, &H);
    for (int i = 0; i < 15; ++i) out[i] = 0.0;
    out[0] = H.ok;
    out[1] = H.linear;
    out[8] = H.A;
    out[9] = H.B;
    out[10] = P.C;
    if (!H.ok) return;
    out[2] = H.t; out[3] = H.x; out[4] = H.y;
    out[5] = P.o[2] + H.t * H.d[2];
    out[6] = H.E;
    out[7] = exp(-0.5 * H.E);
    double nl[3], flip, vlen;
    hit_normal(&P, &H, nl, &flip, &vlen);
    for (int i = 0; i < 3; ++i)
        out[11 + i] = flip * (P.Rc[3 * i] * nl[0] + P.Rc[3 * i + 1] * nl[1] + P.Rc[3 * i + 2] * nl[2]);
    out[14] = curvature_K(P.l1, P.l2, H.x, H.y);
}
