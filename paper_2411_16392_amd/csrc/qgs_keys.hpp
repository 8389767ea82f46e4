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
// edges is <= 0.  FP64, fixed operation order, no contraction.
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

__device__ inline bool conic_tile_hit(const double *C, int tx, int ty, const qgs_camera &cam)
{
#pragma clang fp contract(off)
    const double fx = cam.fx, fy = cam.fy, cx = cam.cx, cy = cam.cy;
    const double pad_px = 1.0 / 64.0;
    const int ux0 = tx * 16, ux1 = (tx * 16 + 15) < cam.width - 1 ? tx * 16 + 15 : cam.width - 1;
    const int vy0 = ty * 16, vy1 = (ty * 16 + 15) < cam.height - 1 ? ty * 16 + 15 : cam.height - 1;
    const double x0 = ((((double)ux0 + 0.5) - pad_px) - cx) / fx, x1 = ((((double)ux1 + 0.5) + pad_px) - cx) / fx;
    const double y0 = ((((double)vy0 + 0.5) - pad_px) - cy) / fy, y1 = ((((double)vy1 + 0.5) + pad_px) - cy) / fy;
    const double a = C[0], b = C[1], c = C[2], d = C[3], e = C[4];
    const double det = a * c - b * b;
    const double mx = (b * e - c * d) / det, my = (b * d - a * e) / det;
    if (mx >= x0 && mx <= x1 && my >= y0 && my <= y1) return true;
    const double xs[2] = {x0, x1}, ys[2] = {y0, y1};
    for (int k = 0; k < 2; ++k) {
        const double y = clamp_d(-(b * xs[k] + e) / c, y0, y1);
        if (conic_eval(C, xs[k], y) <= 0.0) return true;
        const double x = clamp_d(-(b * ys[k] + d) / a, x0, x1);
        if (conic_eval(C, x, ys[k]) <= 0.0) return true;
    }
    return false;
}

}  // namespace qgs
