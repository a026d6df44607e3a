// Point terms of the lower bounds shared by the bound kernels: FP64 from
// float32 inputs, each rounding as in a sequential evaluation.
#pragma once

#include "common.hpp"

namespace nndtw {

__device__ __forceinline__ double sqd(float x, float y)
{
    double d = (double)x - (double)y;
    return d * d;
}

// Distance of a to the interval [lo, u], squared (0 inside).  a - clamp(a)
// is exactly a - u above, a - lo below and 0 inside.
__device__ __forceinline__ double keogh_term(double a, double u, double lo)
{
    double c = __builtin_fmin(__builtin_fmax(a, lo), u);
    double t = a - c;
    return t * t;
}

// Smallest point cost over one band of links around the corner cell (c, c):
// the corner link itself and the pairs (c, x), (x, c) for x0 <= x <= x1
// (0-based).  The left band L^W_k (Section 3) has c = k and x ranging over
// the W positions before it; the right band, its mirror image at (L, L), has
// x ranging over the W positions after c.  min is exact, so the result does
// not depend on the order the links are visited in.
template <typename FA, typename FB>
__device__ __forceinline__ double band_min(FA av, FB bv, int c, int x0, int x1)
{
    const float ac = av(c), bc = bv(c);
    double m = sqd(ac, bc);
    for (int x = x0; x <= x1; ++x) {
        m = __builtin_fmin(m, sqd(ac, bv(x)));
        m = __builtin_fmin(m, sqd(av(x), bc));
    }
    return m;
}

// Bands part of LB_Enhanced^V (Equation 7) for nb = min(floor(L/2), V) band
// indices at each end: the single corner links (0, 0) and (L-1, L-1), then
// per band index k = 1..nb-1 the left band around (k, k) and the right band
// around (L-1-k, L-1-k), summed as res <- (res + left) + right (the
// accumulation order of the paper's algorithm, which the oracle follows too).
// av(i) / bv(j) fetch A_i and B_j (0-based).
template <typename FA, typename FB>
__device__ __forceinline__ double enh_bands(FA av, FB bv, int L, int W, int nb)
{
    double res = sqd(av(0), bv(0)) + sqd(av(L - 1), bv(L - 1));
    for (int k = 1; k < nb; ++k) {
        const double left = band_min(av, bv, k, max(0, k - W), k - 1);
        const int p = L - 1 - k;
        const double right = band_min(av, bv, p, p + 1, min(L - 1, p + W));
        res = res + left + right;
    }
    return res;
}

}  // namespace nndtw
