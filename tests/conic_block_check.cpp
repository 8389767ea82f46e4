// Host check of the rasterizers' block filter: conic_meets_block may say
// false for an 8 x 8 pixel block only if conic_offsets rejects every pixel of
// the block.  Random pre-test conics (ellipses in pixel space of radii 0.2 to
// 400 px, elongation up to 2000, centres offset inside the ellipse from the
// projected centre, projected centres anywhere in a 4096 px frame), blocks
// placed around them; prints "blocks kept_by_pixels kept_by_filter missed".
// Compiled for the host only (no GPU): both functions are host-callable.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>

#include "qgs_device.hpp"

using namespace qgs;

int main(int argc, char **argv)
{
    const long trials = argc > 1 ? atol(argv[1]) : 200000;
    std::mt19937_64 rng(12345);
    std::uniform_real_distribution<double> U01(0.0, 1.0);
    long kept_pix = 0, kept_filter = 0, missed = 0, blocks = 0, far_rejected = 0, far_blocks = 0;
    for (long t = 0; t < trials; ++t) {
        // ellipse: radii log-uniform in [0.2, 400], angle uniform
        const double r1 = 0.2 * std::pow(2000.0, U01(rng)), r2 = (t % 7 == 0) ? r1 : 0.2 * std::pow(2000.0, U01(rng));
        const double th = U01(rng) * M_PI;
        const double cs = std::cos(th), sn = std::sin(th);
        // A = R^T diag(1 / r1^2, 1 / r2^2) R
        const double i1 = 1.0 / (r1 * r1), i2 = 1.0 / (r2 * r2);
        const double A00 = cs * cs * i1 + sn * sn * i2, A11 = sn * sn * i1 + cs * cs * i2, A01 = cs * sn * (i1 - i2);
        // conic centre offset from the projected centre, inside the ellipse
        const double rr = 0.9 * std::sqrt(U01(rng)), ph = U01(rng) * 2 * M_PI;
        const double ux = rr * std::cos(ph) * r1, uy = rr * std::sin(ph) * r2;
        const double ccx = cs * ux - sn * uy, ccy = sn * ux + cs * uy;
        // f(p) = p^T A p - 2 c^T A p - 1: -1 at the projected centre
        const double a = A00, b = 2 * A01, c = A11;
        const double d = -2 * (A00 * ccx + A01 * ccy), e = -2 * (A01 * ccx + A11 * ccy);
        // projected centre anywhere in the frame, split as the record stores it
        const double uc = U01(rng) * 4096.0, vc = U01(rng) * 4096.0;
        float w[32] = {0};
        w[4] = (float)std::floor(uc);
        w[5] = (float)(0.5 - (uc - std::floor(uc)));
        w[6] = (float)std::floor(vc);
        w[7] = (float)(0.5 - (vc - std::floor(vc)));
        w[14] = (float)a;
        w[15] = (float)b;
        w[28] = (float)c;
        w[29] = (float)d;
        w[30] = (float)e;
        float4 rec[8];
        std::memcpy(rec, w, sizeof(w));
        // blocks around the ellipse: within 1.5 extents, plus some farther out
        const double ext = std::max(r1, r2) + std::sqrt(ccx * ccx + ccy * ccy) + 8.0;
        for (int k = 0; k < 4; ++k) {
            const double span = (k == 3 ? 4.0 : 1.5) * ext;
            const int bx = (int)std::floor(uc + (2 * U01(rng) - 1) * span) - 4;
            const int by = (int)std::floor(vc + (2 * U01(rng) - 1) * span) - 4;
            bool any = false;
            for (int j = 0; j < 64 && !any; ++j) {
                PixelRay ray{};
                ray.fpx = (float)(bx + (j & 7));
                ray.fpy = (float)(by + (j >> 3));
                float dxp, dyp;
                any = conic_offsets(w, ray, dxp, dyp);
            }
            const bool keep = conic_meets_block(rec, (float)bx, (float)by);
            ++blocks;
            kept_pix += any;
            kept_filter += keep;
            if (any && !keep) {
                ++missed;
                if (missed <= 5)
                    printf("MISS a=%g b=%g c=%g d=%g e=%g U=%g hu=%g V=%g hv=%g block=(%d,%d)\n", w[14], w[15], w[28],
                           w[29], w[30], w[4], w[5], w[6], w[7], bx, by);
            }
            if (k == 3) {
                ++far_blocks;
                far_rejected += !keep && !any;
            }
        }
    }
    printf("%ld %ld %ld %ld %ld %ld\n", blocks, kept_pix, kept_filter, missed, far_blocks, far_rejected);
    return 0;
}
