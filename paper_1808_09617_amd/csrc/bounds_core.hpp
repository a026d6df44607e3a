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

// Bands part of Algorithm 1 (corners and band indices 2..nb, 1-based).
// av(i) / bv(j) fetch A_i and B_j (0-based).
template <typename FA, typename FB>
__device__ __forceinline__ double enh_bands(FA av, FB bv, int L, int W, int nb)
{
    double res = sqd(av(0), bv(0)) + sqd(av(L - 1), bv(L - 1));
    for (int i = 1; i < nb; ++i) {
        const int r = L - 1 - i;
        const float ai = av(i), bi = bv(i), ar = av(r), br = bv(r);
        double mL = sqd(ai, bi), mR = sqd(ar, br);
        for (int j = max(0, i - W); j < i; ++j) {
            const int rj = L - 1 - j;
            mL = __builtin_fmin(mL, sqd(ai, bv(j)));
            mL = __builtin_fmin(mL, sqd(av(j), bi));
            mR = __builtin_fmin(mR, sqd(ar, bv(rj)));
            mR = __builtin_fmin(mR, sqd(av(rj), br));
        }
        res = res + mL + mR;
    }
    return res;
}

}  // namespace nndtw
