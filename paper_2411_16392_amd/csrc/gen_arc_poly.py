"""Coefficients of the polynomial forms of the arc-length factor used by the
rasterizers for u <= 1 (qgs_device.hpp, gfun and gprime).

g(u) = (asinh u + u sqrt(1 + u^2)) / (2u) and h(u) = g'(u) / u are analytic
functions of v = u^2 with their nearest singularity at v = -1, so Chebyshev
interpolation in v on [0, 1] converges fast: degree 6 for g and 8 for h reach
the FP32 rounding level (max relative error of the FP32 Horner evaluation:
9.5e-8 and 1.3e-7, printed below).  Node values come from 40-digit mpmath.

    python paper_2411_16392_amd/csrc/gen_arc_poly.py
"""
import mpmath
import numpy as np
from numpy.polynomial import chebyshev as C

mpmath.mp.dps = 40


def g_exact(u):
    u = mpmath.mpf(u)
    return (mpmath.asinh(u) + u * mpmath.sqrt(1 + u * u)) / (2 * u) if u != 0 else mpmath.mpf(1)


def h_exact(u):
    u = mpmath.mpf(u)
    return (u * mpmath.sqrt(1 + u * u) - mpmath.asinh(u)) / (2 * u ** 3) if u != 0 else mpmath.mpf(1) / 3


def fit(f, deg):
    n = deg + 1
    x = np.cos(np.pi * (np.arange(n) + 0.5) / n)     # Chebyshev nodes on [-1, 1]
    v = (x + 1) / 2                                   # -> v in [0, 1]
    y = np.array([float(f(mpmath.sqrt(vi))) for vi in v])
    p = np.polynomial.Polynomial(C.cheb2poly(C.chebfit(x, y, deg)))
    return p(np.polynomial.Polynomial([-1.0, 2.0])).coef   # monomial coefficients in v


def fp32_error(f, coef):
    u = np.linspace(0.0, 1.0, 4001)
    v = (u * u).astype(np.float32)
    acc = np.float32(coef[-1])
    for c in coef[-2::-1]:
        acc = (acc * v + np.float32(c)).astype(np.float32)
    ref = np.array([float(f(x)) for x in u])
    return float((np.abs(acc - ref) / ref).max())


if __name__ == "__main__":
    for name, f, deg in (("G_POLY", g_exact, 6), ("H_POLY", h_exact, 8)):
        c = fit(f, deg)
        body = ", ".join(f"{float(np.float32(x))!r}f" for x in c[::-1])
        print(f"// highest degree first; max relative error of the FP32 evaluation {fp32_error(f, c):.2e}")
        print(f"constexpr float {name}[{deg + 1}] = {{{body}}};")
