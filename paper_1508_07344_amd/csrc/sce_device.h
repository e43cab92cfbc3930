// Device helpers shared by the direct and matrix-core kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace sce {

__device__ inline double frac(double t) { return t - floor(t); }

// frac(k t) with the product formed exactly (two-product) before reduction.
__device__ inline double frac_mul(int k, double t)
{
    const double hi = (double)k * t;
    const double lo = fma((double)k, t, -hi);
    const double u = (hi - floor(hi)) + lo;
    return u - floor(u);
}

// frac(a ta + b tb), each product exact before reduction.
__device__ inline double frac_lin(int a, double ta, int b, double tb)
{
    const double h1 = (double)a * ta, l1 = fma((double)a, ta, -h1);
    const double h2 = (double)b * tb, l2 = fma((double)b, tb, -h2);
    const double u = (h1 - floor(h1)) + (h2 - floor(h2)) + (l1 + l2);
    return u - floor(u);
}

// (cos, sin)(2 pi u)
__device__ inline void cis_turns(double u, double &c, double &s) { sincospi(2.0 * u, &s, &c); }

// x wrapped into [0, L): x - L floor(x / L), and a result that rounds to L
// (or a non-finite one) becomes 0.
__device__ inline double wrap_box(double x, double L, double invL)
{
    double w = x - L * floor(x * invL);
    if (w >= L || w < 0.0) w = 0.0;
    return w;
}

}  // namespace sce
