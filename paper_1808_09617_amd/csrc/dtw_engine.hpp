// Anti-diagonal wavefront engine for DTW_W on gfx950 (wave64).
//
// The cost-matrix recurrence of Equation (1),
//   D(i,j) = delta(A_i, B_j) + min(D(i-1,j-1), D(i,j-1), D(i-1,j)),
// is evaluated one anti-diagonal s = i + j at a time: every cell of
// anti-diagonal s depends only on anti-diagonals s-1 and s-2, so all cells of
// one anti-diagonal are independent.  Inside the Sakoe-Chiba window the cells
// lie on the 2W'+1 diagonals k = i - j in [-W', W'] (W' = min(W, L-1)), and a
// diagonal carries a cell only on every other anti-diagonal.  Diagonals are
// therefore handled in adjacent pairs (k, k+1): pair p = (-W'+2p, -W'+2p+1),
// p = 0..W'.  On each "super-step" the bottom diagonals of all pairs advance
// (anti-diagonal s), then the top ones (s+1); each pair updates exactly one
// cell per step, so no lane idles on parity.
//
// Lane layout: a group of G lanes computes one pair of series; a lane owns C
// consecutive diagonal pairs (G*C >= W'+1).  Lane 0 of the wave is a
// sentinel and group g occupies lanes 1 + g*G .. g*G + G, so P = 63 / G
// pairs of series run in one wave.  The only cross-lane values are the
// neighbour diagonals at a lane's two ends, moved with the GFX9 wave-wide
// DPP shifts (wave_shr:1 / wave_shl:1).  The diagonal W'+1 (top of the last
// pair) lies outside the window; it is forced to +inf after every step, which
// also isolates consecutive groups from each other.
//
// Boundaries without branches: the staged series are padded with a huge
// value PAD on both sides.  A cell with both indices in the padding costs
// (PAD - PAD)^2 = 0, a cell with exactly one index in the padding costs
// (PAD - x)^2 = +inf (overflow).  Starting the sweep far enough before the
// matrix with every register at 0 therefore reproduces D(0,0) = delta(A_1,B_1)
// exactly (the virtual predecessor is 0, the others +inf), and cells past the
// matrix never feed D(L-1, L-1).
//
// Series values: the a-value of a bottom cell of pair m equals the a-value of
// the top cell of pair m-1 and the b-value is shared by both cells of a pair,
// so a lane keeps windows of C+1 consecutive a and b values that slide by one
// element per super-step.  The windows live in registers whose roles rotate
// with period C+1 (the loop is unrolled by C+1 super-steps), so each
// super-step costs two LDS reads and no register moves.
//
// Early abandon: every warping path crosses every pair of consecutive
// anti-diagonals and costs only grow along a path, so once all cells of
// anti-diagonals s and s+1 exceed the cutoff the result exceeds it too.
#pragma once

#include "common.hpp"

namespace nndtw {

// ---------------------------------------------------------------- DPP moves
// Lane i receives lane i-1's value (lane 0 receives 0).
__device__ __forceinline__ float from_lower(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x138, 0xF, 0xF, true));
}
// Lane i receives lane i+1's value (lane 63 receives 0).
__device__ __forceinline__ float from_upper(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ double from_lower(double x)
{
    unsigned long long v = (unsigned long long)__double_as_longlong(x);
    unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)v, 0x138, 0xF, 0xF, true);
    unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(v >> 32), 0x138, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double from_upper(double x)
{
    unsigned long long v = (unsigned long long)__double_as_longlong(x);
    unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)v, 0x130, 0xF, 0xF, true);
    unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(v >> 32), 0x130, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ float min3(float a, float b, float c) { return __builtin_fminf(__builtin_fminf(a, b), c); }
__device__ __forceinline__ double min3(double a, double b, double c) { return __builtin_fmin(__builtin_fmin(a, b), c); }
__device__ __forceinline__ float vmax(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ double vmax(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ float vmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double vmin(double a, double b) { return __builtin_fmin(a, b); }

// One cell: FP32 uses a fused multiply-add; FP64 rounds the product and the
// sum separately, exactly as a sequential evaluation of the recurrence.
__device__ __forceinline__ float cell(float d, float m) { return __builtin_fmaf(d, d, m); }
__device__ __forceinline__ double cell(double d, double m) { return d * d + m; }

// Smallest float >= x (so that "float > result" implies "value > x").
__device__ __forceinline__ float round_up_f32(double x)
{
    float f = (float)x;
    if ((double)f < x) {
        int b = __float_as_int(f);
        f = __int_as_float(f >= 0.0f ? b + 1 : b - 1);
    }
    return f;
}

template <typename T> __device__ __forceinline__ T inf_of();
template <> __device__ __forceinline__ float inf_of<float>() { return __builtin_inff(); }
template <> __device__ __forceinline__ double inf_of<double>() { return __builtin_inf(); }

// Padding left of the first series element inside a staged LDS row (elements).
template <int C> struct Stage { static constexpr int PADL = C; };

// Stage series `src` (float[L], global) into LDS row `dst` of geo.LEN
// elements with PAD outside [0, L).  Whole-wave cooperative.
template <typename T, int C>
__device__ __forceinline__ void stage_row(T *dst, const float *__restrict__ src, const EngineGeom &geo, int lane)
{
    const int first = geo.base0 - Stage<C>::PADL;
    for (int e = lane; e < geo.LEN; e += WAVE) {
        int idx = first + e;
        dst[e] = (idx >= 0 && idx < geo.L) ? (T)src[idx] : Pad<T>::big();
    }
}

// Result of one pass, per group (written to LDS by the group's result lane).
template <typename T> struct PassOut {
    T *res;    // DTW_W, or +inf if abandoned
    int *trun; // super-steps executed
};

// One pass: groups 0..nact-1 each compute DTW_W of the pair staged at
// aRow(g) / bRow(g).  thr: abandon threshold (+inf: never).  Must be called
// by the whole wave with uniform arguments.
template <typename T, int C, bool EXACT>
__device__ __forceinline__ void engine_pass(const EngineGeom &geo, const T *aRows, int aStride,
                                            const T *bRows, int bStride, int nact, T thr,
                                            PassOut<T> out)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int G = geo.G, Wp = geo.Wp;
    const int gi = lane >= 1 ? (lane - 1) / G : 0;
    const int gl = lane >= 1 ? (lane - 1) - gi * G : 0;
    const bool in_group = lane >= 1 && gi < geo.P;
    const bool has_task = in_group && gi < nact;
    const int g = in_group ? gi : 0;                 // sentinel / idle lanes shadow group 0
    const int glc = in_group ? gl * C : 0;
    const T INF = inf_of<T>();

    const T *aP = aRows + (size_t)g * aStride + Stage<C>::PADL + glc;
    const T *bP = bRows + (size_t)g * bStride + Stage<C>::PADL + Wp - glc;

    T X0[C], X1[C], Aw[C + 1], Bw[C + 1];
    // Forced-infinite slots: the out-of-window diagonal W'+1 and the last
    // top diagonal of each group (and the sentinel's, which lane 1 reads).
    bool force_last = (lane == 0) || (in_group && gl == G - 1);
    T tm[EXACT ? 1 : C];
#pragma unroll
    for (int m = 0; m < C; ++m) {
        const int p = glc + m;                       // global pair index
        X0[m] = (!EXACT && in_group && p > Wp) ? INF : (T)0;
        X1[m] = (!EXACT && in_group && p >= Wp) ? INF : (T)0;
        if (!EXACT) tm[m] = ((m == C - 1 && force_last) || (in_group && p == Wp)) ? INF : (T)0;
    }
    if (EXACT && force_last) X1[C - 1] = INF;
#pragma unroll
    for (int m = 0; m <= C; ++m) Aw[m] = aP[m];
    Bw[1 % (C + 1)] = (T)0;                          // b-slot C: unused until refilled
#pragma unroll
    for (int m = 0; m < C; ++m) Bw[(C + 1 - m) % (C + 1)] = bP[-m];

    bool dead = !has_task;
    int trun = geo.T;
    for (int t0 = 0; t0 < geo.T; t0 += C + 1) {
#pragma unroll
        for (int u = 0; u <= C; ++u) {
            const int t = t0 + u;
            // bottom diagonals: anti-diagonal s_b(t)
            T nb = from_lower(X1[C - 1]);
#pragma unroll
            for (int m = 0; m < C; ++m) {
                T lo = (m == 0) ? nb : X1[m - 1];
                T d = Aw[(u + m) % (C + 1)] - Bw[(u - m + C + 1) % (C + 1)];
                X0[m] = cell(d, min3(X0[m], lo, X1[m]));
            }
            // top diagonals: anti-diagonal s_b(t) + 1
            T nt = from_upper(X0[0]);
#pragma unroll
            for (int m = 0; m < C; ++m) {
                T hi = (m == C - 1) ? nt : X0[m + 1];
                T d = Aw[(u + m + 1) % (C + 1)] - Bw[(u - m + C + 1) % (C + 1)];
                X1[m] = cell(d, min3(X1[m], X0[m], hi));
            }
            if (EXACT) {
                X1[C - 1] = force_last ? INF : X1[C - 1];
            } else {
#pragma unroll
                for (int m = 0; m < C; ++m) X1[m] = vmax(X1[m], tm[m]);
            }
            // windows for super-step t+1
            Aw[u] = aP[t + 1 + C];
            Bw[(u + 1) % (C + 1)] = bP[t + 1];
        }
        // early abandon on the frontier (two consecutive anti-diagonals)
        T lm = vmin(X0[0], X1[0]);
#pragma unroll
        for (int m = 1; m < C; ++m) lm = min3(lm, X0[m], X1[m]);
        unsigned long long ok = __ballot(lm <= thr);
        unsigned long long gmask = (G >= 64) ? ~0ull : ((1ull << G) - 1ull);
        bool alive = ((ok >> (1 + g * G)) & gmask) != 0ull;
        if (!dead && !alive) {
            dead = true;
            trun = t0 + C + 1;
        }
        if (__ballot(!dead) == 0ull) break;
    }
    // D(L-1, L-1) lies on diagonal 0: pair W'/2, bottom if W' is even.
    const int p0 = Wp >> 1;
    const int rlane = 1 + g * G + p0 / C;
    if (has_task && lane == rlane) {
        const int m0 = p0 % C;
        T r = INF;
#pragma unroll
        for (int m = 0; m < C; ++m)
            if (m == m0) r = (Wp & 1) ? X1[m] : X0[m];
        out.res[gi] = dead ? INF : r;
        out.trun[gi] = trun;
    }
}

}  // namespace nndtw
