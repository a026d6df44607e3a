// Comparison lower bounds: the existing bounds the paper reviews
// (Section 2.2) and measures LB_Enhanced against (Section 4), and the
// symmetric LB_Enhanced its conclusion suggests.  All in FP64 from float32
// inputs; every sum is accumulated in ascending point order by one lane, so
// the values are reproducible bit for bit.
//
//  * LB_Kim, sum form of the experiments: corner costs, then the cost of the
//    two minima and of the two maxima, each extreme counted only when
//    neither series takes it at its first or last point ("without
//    repetitions"; with that rule every feature is paid by a different link
//    of every warping path).
//  * LB_Improved: LB_Keogh(A, B) + LB_Keogh(B, A'), A' the projection of A
//    on B's envelope (Equation 5) and the second term taken against the
//    envelope of A' for the same window.
//  * LB_New: corner costs plus, for every interior point A_i, the cost of
//    the nearest value of B inside its window.
//  * max(LB_Enhanced^V(A, B), LB_Enhanced^V(B, A)).
//
// One wave (a workgroup of 64 lanes) per pair: the lanes compute the point
// terms of the pair in parallel into LDS, and one lane sums them in order
// (two lanes when a bound has two independent sums).  Window envelopes of a
// row held in LDS (A' for LB_Improved, A for the reverse LB_Enhanced) come
// from a doubling scheme over the row padded with -inf / +inf: with F_1 the
// padded row and F_2s(t) = max(F_s(t), F_s(t + s)), the maximum over the
// window of point i (padded positions i .. i + 2w) is
// max(F_K(i), F_K(i + 2w + 1 - K)) for K the largest power of two <= 2w+1.
// Minima and maxima are exact, so the envelopes equal a direct evaluation.
#include "bounds_core.hpp"

namespace nndtw {

enum { CMP_KIM = 0, CMP_IMPROVED = 1, CMP_NEW = 2, CMP_ENH_SYM = 3 };

// LDS layout of one wave (byte offsets; sizes in elements):
//   xa, xb, xu, xl, xp   float[L] each  (A, B, an envelope pair, A')
//   t1                   double[L]      first term array
//   r                    max(float[2 (L + 2w)], double[L]): the doubling
//                        buffers, reused afterwards for the second term array
struct CmpLds {
    size_t xa, xb, xu, xl, xp, t1, r, total;
};

__host__ __device__ inline CmpLds cmp_lds(int L, int w)
{
    CmpLds m;
    size_t o = 0;
    m.xa = o; o += (size_t)L * 4;
    m.xb = o; o += (size_t)L * 4;
    m.xu = o; o += (size_t)L * 4;
    m.xl = o; o += (size_t)L * 4;
    m.xp = o; o += (size_t)L * 4;
    o = (o + 15) & ~(size_t)15;
    m.t1 = o; o += (size_t)L * 8;
    m.r = o;
    const size_t dbl = (size_t)2 * (L + 2 * w) * 4, term = (size_t)L * 8;
    o += dbl > term ? dbl : term;
    m.total = o;
    return m;
}

__device__ __forceinline__ float wave_maxf(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = __builtin_fmaxf(v, __shfl_xor(v, off));
    return v;
}
__device__ __forceinline__ float wave_minf(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = __builtin_fminf(v, __shfl_xor(v, off));
    return v;
}

// Envelope of x (LDS float[L]) for half-width w (<= L-1) into U, Lo (LDS
// float[L]); buf: LDS float[2 (L + 2w)].  Whole-wave call.
__device__ void window_envelope(const float *x, int L, int w, float *U, float *Lo, float *buf, int lane)
{
    if (w >= L - 1) {
        float mx = -__builtin_inff(), mn = __builtin_inff();
        for (int i = lane; i < L; i += WAVE) {
            mx = __builtin_fmaxf(mx, x[i]);
            mn = __builtin_fminf(mn, x[i]);
        }
        mx = wave_maxf(mx);
        mn = wave_minf(mn);
        for (int i = lane; i < L; i += WAVE) {
            U[i] = mx;
            Lo[i] = mn;
        }
        __syncthreads();
        return;
    }
    const int Lp = L + 2 * w, span = 2 * w + 1;
    for (int pass = 0; pass < 2; ++pass) {            // 0: maxima, 1: minima
        const bool mx = pass == 0;
        const float pad = mx ? -__builtin_inff() : __builtin_inff();
        float *cur = buf, *nxt = buf + Lp;
        for (int t = lane; t < Lp; t += WAVE) cur[t] = (t >= w && t < w + L) ? x[t - w] : pad;
        __syncthreads();
        int K = 1;
        while (2 * K <= span) {
            // F_2K(t) for t in [0, Lp - 2K]
            for (int t = lane; t <= Lp - 2 * K; t += WAVE) {
                const float a = cur[t], b = cur[t + K];
                nxt[t] = mx ? __builtin_fmaxf(a, b) : __builtin_fminf(a, b);
            }
            __syncthreads();
            float *s = cur; cur = nxt; nxt = s;
            K *= 2;
        }
        float *dst = mx ? U : Lo;
        for (int i = lane; i < L; i += WAVE) {
            const float a = cur[i], b = cur[i + span - K];
            dst[i] = mx ? __builtin_fmaxf(a, b) : __builtin_fminf(a, b);
        }
        __syncthreads();
    }
}

// In-order sum of t[lo .. hi) onto s (one lane).  The LDS loads of a block
// of 16 terms are issued before its adds, so the load latency is paid once
// per block instead of once per term; the additions keep their order.
__device__ __forceinline__ double ordered_sum(double s, const double *t, int lo, int hi)
{
    int i = lo;
    for (; i + 16 <= hi; i += 16) {
        double v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = t[i + k];
#pragma unroll
        for (int k = 0; k < 16; ++k) s += v[k];
    }
    for (; i < hi; ++i) s += t[i];
    return s;
}

__global__ void __launch_bounds__(WAVE)
compare_bounds_kernel(int what, const float *__restrict__ A, int64_t nA, const float *__restrict__ B,
                      const float *__restrict__ U, const float *__restrict__ Lo, int64_t nB, int L, int W, int nb,
                      const double *__restrict__ cutoff, int pairing, double *__restrict__ out)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x;
    const int w = W < L - 1 ? W : L - 1;
    const CmpLds m = cmp_lds(L, w);
    float *xa = reinterpret_cast<float *>(smem + m.xa), *xb = reinterpret_cast<float *>(smem + m.xb);
    float *xu = reinterpret_cast<float *>(smem + m.xu), *xl = reinterpret_cast<float *>(smem + m.xl);
    float *xp = reinterpret_cast<float *>(smem + m.xp);
    double *t1 = reinterpret_cast<double *>(smem + m.t1);
    float *buf = reinterpret_cast<float *>(smem + m.r);
    double *t2 = reinterpret_cast<double *>(smem + m.r);
    const int64_t np = pairing ? nA : nA * nB;

    for (int64_t p = blockIdx.x; p < np; p += gridDim.x) {
        const int64_t ia = pairing ? p : p / nB, ib = pairing ? p : p % nB;
        const float *a = A + ia * L, *b = B + ib * L;
        double res = 0.0;
        if (what == CMP_KIM) {
            float amin = __builtin_inff(), amax = -__builtin_inff(), bmin = amin, bmax = amax;
            for (int i = lane; i < L; i += WAVE) {
                const float x = a[i], y = b[i];
                amin = __builtin_fminf(amin, x);
                amax = __builtin_fmaxf(amax, x);
                bmin = __builtin_fminf(bmin, y);
                bmax = __builtin_fmaxf(bmax, y);
            }
            amin = wave_minf(amin);
            amax = wave_maxf(amax);
            bmin = wave_minf(bmin);
            bmax = wave_maxf(bmax);
            const float a0 = a[0], aL = a[L - 1], b0 = b[0], bL = b[L - 1];
            res = sqd(a0, b0) + sqd(aL, bL);
            const bool min_end = a0 == amin || aL == amin || b0 == bmin || bL == bmin;
            const bool max_end = a0 == amax || aL == amax || b0 == bmax || bL == bmax;
            if (!min_end) res += sqd(amin, bmin);
            if (!max_end) res += sqd(amax, bmax);
        } else if (what == CMP_NEW) {
            for (int i = lane; i < L; i += WAVE) xb[i] = b[i];
            __syncthreads();
            // min over the window of (A_i - B_j)^2 is the square of the
            // smallest |A_i - B_j| (both roundings are monotone)
            for (int i = 1 + lane; i < L - 1; i += WAVE) {
                const double x = (double)a[i];
                const int j0 = i - w > 0 ? i - w : 0, j1 = i + w < L - 1 ? i + w : L - 1;
                double md = __builtin_inf();
                for (int j = j0; j <= j1; ++j) md = __builtin_fmin(md, __builtin_fabs(x - (double)xb[j]));
                t1[i] = md * md;
            }
            __syncthreads();
            if (lane == 0) res = ordered_sum(sqd(a[0], xb[0]) + sqd(a[L - 1], xb[L - 1]), t1, 1, L - 1);
        } else if (what == CMP_IMPROVED) {
            const float *u = U + ib * L, *lo = Lo + ib * L;
            for (int i = lane; i < L; i += WAVE) {
                const float x = a[i], uu = u[i], ll = lo[i];
                t1[i] = keogh_term((double)x, (double)uu, (double)ll);
                xp[i] = x > uu ? uu : (x < ll ? ll : x);
            }
            __syncthreads();
            bool skip = false;
            double k1 = 0.0;
            if (cutoff) {                       // second pass only if the first does not exceed the cutoff
                k1 = ordered_sum(0.0, t1, 0, L);  // every lane (LDS broadcast reads): no lane branch
                skip = k1 > cutoff[ia];
            }
            if (skip) {
                res = __builtin_inf();
            } else {
                window_envelope(xp, L, w, xu, xl, buf, lane);
                for (int j = lane; j < L; j += WAVE) t2[j] = keogh_term((double)b[j], (double)xu[j], (double)xl[j]);
                __syncthreads();
                // lane 0: LB_Keogh(A, B) (unless already summed); lane 1: LB_Keogh(B, A')
                double s = 0.0;
                if (lane < 2 && !(cutoff && lane == 0)) s = ordered_sum(0.0, lane == 0 ? t1 : t2, 0, L);
                if (cutoff && lane == 0) s = k1;
                const double k2 = __shfl(s, 1);
                res = s + k2;
            }
        } else {                                // CMP_ENH_SYM
            const float *u = U + ib * L, *lo = Lo + ib * L;
            for (int i = lane; i < L; i += WAVE) {
                xa[i] = a[i];
                xb[i] = b[i];
            }
            __syncthreads();
            window_envelope(xa, L, w, xu, xl, buf, lane);
            for (int i = nb + lane; i < L - nb; i += WAVE) {
                t1[i] = keogh_term((double)xa[i], (double)u[i], (double)lo[i]);    // A against B's envelope
                t2[i] = keogh_term((double)xb[i], (double)xu[i], (double)xl[i]);   // B against A's envelope
            }
            __syncthreads();
            // lane 0: LB_Enhanced(A, B); lane 1: LB_Enhanced(B, A)
            double s = 0.0;
            if (lane < 2) {
                const float *p0 = lane == 0 ? xa : xb, *q0 = lane == 0 ? xb : xa;
                s = enh_bands([&](int i) { return p0[i]; }, [&](int j) { return q0[j]; }, L, w, nb);
                s = ordered_sum(s, lane == 0 ? t1 : t2, nb, L - nb);
            }
            const double ba = __shfl(s, 1);
            res = s > ba ? s : ba;
        }
        if (lane == 0) out[p] = res;
        __syncthreads();                        // LDS is reused by the next pair
    }
}

size_t compare_lds_bytes(int L, int W)
{
    const int w = W < L - 1 ? W : L - 1;
    return cmp_lds(L, w).total;
}

int launch_compare_bounds(int what, const float *A, int64_t nA, const float *B, const float *U, const float *Lo,
                          int64_t nB, int L, int W, int V, const double *cutoff, int pairing, double *out,
                          hipStream_t st)
{
    const int64_t np = pairing ? nA : nA * nB;
    if (np == 0) return NNDTW_OK;
    const int nb = V < L / 2 ? V : L / 2;
    const size_t lds = compare_lds_bytes(L, W);
    if (lds > 160 * 1024) return fail(NNDTW_EUNSUP, "series length %d too long for the comparison bounds", L);
    const int64_t blocks = np < 256 * 64 ? np : 256 * 64;
    hipLaunchKernelGGL(compare_bounds_kernel, dim3((unsigned)blocks), dim3(WAVE), lds, st, what, A, nA, B, U, Lo,
                       nB, L, W, nb, cutoff, pairing, out);
    NNDTW_LAUNCH_CHECK("comparison bounds kernel launch");
    return NNDTW_OK;
}

}  // namespace nndtw
