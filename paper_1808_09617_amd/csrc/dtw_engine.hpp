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
// (PAD - x)^2 = +inf (overflow).  A sweep started far enough before the
// matrix with every register at 0 therefore reproduces D(0,0) = delta(A_1,B_1)
// exactly (the virtual predecessor is 0, the others +inf), and cells past the
// matrix never feed D(L-1, L-1).  The state that such a sweep reaches before
// the matrix is known in closed form (0 where both indices are in the
// padding, +inf elsewhere), so a task loads it directly at super-step t0,
// just before the matrix, and skips the steps before; blocks of M super-steps
// (and the register rotation of the windows) count from t0.
//
// Series values: the a-value of a bottom cell of pair m equals the a-value of
// the top cell of pair m-1 and the b-value is shared by both cells of a pair,
// so a lane keeps windows of C+1 consecutive a and b values that slide by one
// element per super-step.  The windows live in M >= C + D registers whose
// roles rotate with period M (the loop is unrolled by M super-steps, a
// "block"), and the values super-step t+D needs are read at the end of
// super-step t (from LDS or from global memory), so each super-step costs
// two reads and no register moves.
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

// Stage `nrows` series (row r is src + krow(r) * L) into consecutive LDS rows
// of geo.LEN elements.  Flattened over all rows, each thread keeps U global
// loads in flight before its LDS stores.  Cooperative over `nthreads`
// threads (tid = 0 .. nthreads-1).
template <typename T, int C, typename KF>
__device__ __forceinline__ void stage_rows(T *dst, const float *__restrict__ src, KF krow, int nrows,
                                           const EngineGeom &geo, int tid, int nthreads = WAVE)
{
    constexpr int U = 16;
    const int LEN = geo.LEN, L = geo.L;
    const int first = geo.base0 - Stage<C>::PADL;
    const int total = nrows * LEN;
    int g = 0, x = tid;
    while (x >= LEN) { x -= LEN; ++g; }
    for (int e0 = 0; e0 < total; e0 += nthreads * U) {
        T v[U];
        int gg[U], xx[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            gg[u] = g;
            xx[u] = x;
            const int idx = first + x;
            v[u] = Pad<T>::big();
            if (g < nrows && idx >= 0 && idx < L) v[u] = (T)src[(int64_t)krow(g) * L + idx];
            x += nthreads;
            while (x >= LEN) { x -= LEN; ++g; }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (gg[u] < nrows) dst[(size_t)gg[u] * LEN + xx[u]] = v[u];
    }
}

// Per-task outputs (LDS), written by the result lane of the group that ran
// the task.
template <typename T> struct TaskOut {
    T *res;     // DTW_W, or +inf if abandoned
    int *trun;  // super-steps executed
    // Optional shared abandon threshold (FP32 engine only): the bits of a
    // non-negative float in LDS.  A task that completes with result r lowers
    // it to round_up(r * slack), and every task abandons against
    // min(its own threshold, that value).
    unsigned *run_thr = nullptr;
    double slack = 1.0;
    // Optional wave-priority rotation (>= 0: on, the workgroup's phase 0..3;
    // see rotate_priority), checked once per block of M super-steps.
    int rot_phase = -1;
    // Optional shared batch (several workgroups, see search.hip): tasks are
    // dealt from the global word *deal64 = (tag << 32) | next index instead
    // of the LDS counter, only while its tag is `tag`, and res / trun are
    // global memory written with device-scope atomic stores, each task then
    // counted in *done.
    unsigned long long *deal64 = nullptr;
    uint32_t tag = 0;
    unsigned *done = nullptr;
};

// The next `n` task indices of a shared batch (see TaskOut::deal64), or
// `ntasks` once the batch has moved on (another tag) or is exhausted.  Whole
// wave, uniform arguments; lane 0 runs the compare-and-swap loop and the
// result is its value as a scalar.  The lane test goes through an empty asm
// statement, so that the compiler cannot relate it to the engines' lane-0
// result stores: with both plain `lane == 0` tests in one task loop it once
// merged them across the loop's back edge and sent lanes 1-63 round the task
// loop without lane 0, re-reading task 0 forever.  (Every lane issuing the
// compare-and-swap avoids the branch but made each deal 64 atomics on one
// word: the search ran several times slower.)
__device__ __forceinline__ int shared_deal(unsigned long long *deal64, uint32_t tag, int ntasks, int n, int lane)
{
    int first = lane == 0;
    asm volatile("" : "+v"(first));
    unsigned long long got = 0ull;
    if (first) {
        unsigned long long cur = __hip_atomic_load(deal64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while (true) {
            if ((uint32_t)(cur >> 32) != tag || (uint32_t)cur >= (uint32_t)ntasks) {
                got = (unsigned long long)ntasks;
                break;
            }
            if (__hip_atomic_compare_exchange_strong(deal64, &cur, cur + (unsigned long long)n, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                got = cur & 0xFFFFFFFFull;
                break;
            }
        }
    }
    return __builtin_amdgcn_readfirstlane((int)got);
}

// Optional per-cell record of the minimising predecessor (for the argmin
// warping path): codes(task) is the task's word array [T/8][W'+1]; word
// (t/8, p) holds pair p's cells of the 8 super-steps 8(t/8) .. 8(t/8)+7,
// four bits each, the first super-step in the top bits.  For super-step u
// of the word: bit 31-4u is set when the bottom cell's predecessor
// (i-1, j-1) is above the smaller of the other two, bit 30-4u when (i-1, j)
// is above (i, j-1); bits 29-4u and 28-4u the same for the top cell.  The
// path takes (i-1, j-1) if the first bit is clear, else (i-1, j) if the
// second is, else (i, j-1): the first of the three that attains the minimum.
// Needs M % 8 == 0 (then T % 8 == 0 too).
struct NoCodes {
    static constexpr bool on = false;
    __device__ uint32_t *operator()(int) const { return nullptr; }
};

// Shifts into the bottom of cw whether x > ref.  DTW values are
// non-negative floats or +inf, whose bit patterns order like the values and
// lie below 2^31, so the sign bit of the 32-bit difference ref - x is set
// exactly when x > ref: one subtract and one funnel shift, no lane mask
// (whose write and read would need wait states between them).  A cell's
// bits compare its predecessors with each other, not with their minimum,
// which then need not outlive the cell's update.
__device__ __forceinline__ uint32_t push_code(uint32_t cw, float x, float ref)
{
    return __builtin_amdgcn_alignbit(cw, __float_as_uint(ref) - __float_as_uint(x), 31);
}
__device__ __forceinline__ uint32_t push_code(uint32_t cw, double x, double ref)
{
    return (cw << 1) | (x > ref ? 1u : 0u);
}

// Run `ntasks` DTW tasks on the P groups of each calling wave.  Tasks are
// dealt from the LDS counter *next_task (0 before the call, shared by every
// wave of the workgroup that takes part).  Task i compares the rows arow(i)
// and brow(i) (geo.LEN elements each, in LDS or global memory; elements of
// any type that converts exactly to T, e.g. float rows for an FP64 sweep) and is
// abandoned once its frontier exceeds thr_of(i).  A group takes the next
// task as soon as its current one ends (completed or abandoned), at the next
// block boundary (every M super-steps), so abandoned candidates free their
// lanes early.  Every task starts at super-step geo.t0 of its own sweep and
// runs whole blocks from there, so block boundaries fall on the same
// super-steps modulo M in every group, which keeps the register rotation of
// the windows the same in all groups.  Whole-wave call with uniform
// arguments; ntasks >= 1.
template <typename T, int C, int D, int M, bool EXACT, typename ARow, typename BRow, typename Thr,
          typename Codes = NoCodes>
__device__ __forceinline__ void engine_run(const EngineGeom &geo, int ntasks, int *next_task, ARow arow, BRow brow,
                                           Thr thr_of, TaskOut<T> out, Codes codes_of = Codes())
{
    static_assert(M >= C + D, "window smaller than the live values");
    const int lane = threadIdx.x & (WAVE - 1);
    const int G = geo.G, Wp = geo.Wp, T_ = geo.T, t0 = geo.t0;
    const int gi = lane >= 1 ? (lane - 1) / G : 0;
    const int gl = lane >= 1 ? (lane - 1) - gi * G : 0;
    const bool in_group = lane >= 1 && gi < geo.P;
    const int g = in_group ? gi : 0;                 // sentinel / idle lanes shadow group 0
    const int glc = in_group ? gl * C : 0;
    const int lane0 = 1 + g * G;                     // first lane of the group
    const T INF = inf_of<T>();
    const unsigned long long gmask = (1ull << G) - 1ull;
    // D(L-1, L-1) lies on diagonal 0: pair W'/2, bottom diagonal if W' is even.
    const int p0 = Wp >> 1, m0 = p0 % C;
    const bool rlane = in_group && gl == p0 / C;

    // Forced-infinite slots: the out-of-window diagonal W'+1 and the last
    // top diagonal of each group (and the sentinel's, which lane 1 reads).
    const bool force_last = (lane == 0) || (in_group && gl == G - 1);
    T tm[EXACT ? 1 : C];
#pragma unroll
    for (int m = 0; m < C; ++m)
        if (!EXACT) tm[m] = ((m == C - 1 && force_last) || (in_group && glc + m == Wp)) ? INF : (T)0;

    T X0[C], X1[C], Aw[M], Bw[M];
    auto aP = arow(0) + Stage<C>::PADL + glc;
    auto bP = brow(0) + Stage<C>::PADL + Wp - glc;
#pragma unroll
    for (int m = 0; m < C; ++m) { X0[m] = (T)0; X1[m] = (T)0; }
#pragma unroll
    for (int m = 0; m < M; ++m) { Aw[m] = (T)0; Bw[m] = (T)0; }
    if (force_last) X1[C - 1] = INF;

    // State of this lane's cells before super-step t0 (all of it before the
    // matrix), bit m for pair glc+m: pair p's bottom cell there is
    // (i, j) = (t0+p-W'-2, t0-p-2) and its top cell (i+1, j); a cell inside
    // the window is 0 with both indices in the padding (so is its path from
    // the start), +inf with one index in it; outside the window +inf.
    unsigned z0 = 0u, z1 = 0u;
#pragma unroll
    for (int m = 0; m < C; ++m) {
        const int p = glc + m;
        const int ib = t0 + p - Wp - 2, jb = t0 - p - 2;
        z0 |= (p <= Wp && ib < 0 && jb < 0) ? (1u << m) : 0u;
        z1 |= (p < Wp && ib + 1 < 0 && jb < 0) ? (1u << m) : 0u;
    }
    int task = -1, tl = 0;
    bool dead = true, exhausted = false;
    static_assert(!Codes::on || M % 8 == 0, "codes need blocks of whole words");
    uint32_t *cb = nullptr;                          // this lane's code words (Codes::on)
    const int cpitch = Wp + 1;
    uint32_t cw[C];
#pragma unroll
    for (int m = 0; m < C; ++m) cw[m] = 0u;
    T thr = INF;
    while (true) {
        if (out.rot_phase >= 0) rotate_priority(out.rot_phase);
        // retire the tasks that ended
        if (__ballot(task >= 0 && (dead || tl >= T_)) != 0ull && task >= 0 && (dead || tl >= T_)) {
            if (rlane) {
                T r = INF;
#pragma unroll
                for (int m = 0; m < C; ++m)
                    if (m == m0) r = (Wp & 1) ? X1[m] : X0[m];
                if constexpr (sizeof(T) == 4) {
                    if (out.deal64 != nullptr) {
                        // shared batch: device-scope stores, complete before
                        // the task is counted
                        __hip_atomic_store(reinterpret_cast<unsigned *>(out.res) + task,
                                           __float_as_uint(dead ? INF : r), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_store(out.trun + task, dead ? tl : T_, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                        __builtin_amdgcn_s_waitcnt(0);
                        __hip_atomic_fetch_add(out.done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    } else {
                        out.res[task] = dead ? INF : r;
                        out.trun[task] = dead ? tl : T_;
                    }
                } else {
                    out.res[task] = dead ? INF : r;
                    out.trun[task] = dead ? tl : T_;
                }
                if constexpr (sizeof(T) == 4) {
                    if (out.run_thr != nullptr && !dead)
                        atomicMin(out.run_thr, __float_as_uint(round_up_f32((double)r * out.slack)));
                }
            }
            task = -1;
            tl = 0;
        }
        // hand the next tasks to free groups, in group order
        const unsigned long long freem = __ballot(in_group && gl == 0 && task < 0);
        const int nfree = __popcll(freem);
        if (nfree > 0 && !exhausted) {
            // whole-wave fetch (lane 0 adds nfree, the others 0), lane 0's
            // result as a scalar: no lane-dependent branch around the deal
            const int base = out.deal64 != nullptr
                                 ? shared_deal(out.deal64, out.tag, ntasks, nfree, lane)
                                 : __builtin_amdgcn_readfirstlane(atomicAdd(next_task, lane == 0 ? nfree : 0));
            const int left = ntasks - base;
            const int nassign = left < nfree ? (left > 0 ? left : 0) : nfree;
            exhausted = left <= nfree;
            const int rank = __popcll(freem & ((1ull << lane0) - 1ull));
            if (in_group && task < 0 && rank < nassign) {
                task = base + rank;
                thr = thr_of(task);
                dead = false;
                tl = t0;
                aP = arow(task) + Stage<C>::PADL + glc;
                bP = brow(task) + Stage<C>::PADL + Wp - glc;
                if constexpr (Codes::on) cb = codes_of(task) + glc;
#pragma unroll
                for (int m = 0; m < C; ++m) {
                    X0[m] = ((z0 >> m) & 1u) ? (T)0 : INF;
                    X1[m] = ((z1 >> m) & 1u) ? (T)0 : INF;
                }
                if (EXACT && force_last) X1[C - 1] = INF;
                // a-slot m at super-step t is aP[t + m] in Aw[(t - t0 + m) % M];
                // b-slot m is bP[t - m] in Bw[(t - t0 - m) mod M]: preload
                // what super-steps t0..t0+D-1 read.
#pragma unroll
                for (int r = 0; r < C + D; ++r) Aw[r % M] = (T)aP[t0 + r];
#pragma unroll
                for (int r = 1 - C; r <= D - 1; ++r) Bw[((r % M) + M) % M] = (T)bP[t0 + r];
            }
        }
        if (__ballot(task >= 0) == 0ull) break;

        const auto aC = aP + tl, bC = bP + tl;
#pragma unroll
        for (int u = 0; u < M; ++u) {
            // bottom diagonals: anti-diagonal s_b(t)
            const T nb = from_lower(X1[C - 1]);
#pragma unroll
            for (int m = 0; m < C; ++m) {
                const T lo = (m == 0) ? nb : X1[m - 1];
                const T d = Aw[(u + m) % M] - Bw[(u - m + M) % M];
                // predecessors: (i-1,j-1) = X0[m], (i-1,j) = lo, (i,j-1) = X1[m]
                if constexpr (Codes::on)
                    cw[m] = push_code(push_code(cw[m], X0[m], vmin(lo, X1[m])), lo, X1[m]);
                X0[m] = cell(d, min3(X0[m], lo, X1[m]));
            }
            // top diagonals: anti-diagonal s_b(t) + 1
            const T nt = from_upper(X0[0]);
#pragma unroll
            for (int m = 0; m < C; ++m) {
                const T hi = (m == C - 1) ? nt : X0[m + 1];
                const T d = Aw[(u + m + 1) % M] - Bw[(u - m + M) % M];
                // predecessors: (i-1,j-1) = X1[m], (i-1,j) = X0[m], (i,j-1) = hi
                if constexpr (Codes::on)
                    cw[m] = push_code(push_code(cw[m], X1[m], vmin(X0[m], hi)), X0[m], hi);
                X1[m] = cell(d, min3(X1[m], X0[m], hi));
            }
            // a word holds 8 super-steps (32 bits); cleared once stored, so
            // that no code word is live outside this loop
            if constexpr (Codes::on) {
                if (u % 8 == 7) {
                    if (task >= 0) {
#pragma unroll
                        for (int m = 0; m < C; ++m)
                            if (glc + m <= Wp) cb[(int64_t)((tl + u) / 8) * cpitch + m] = cw[m];
                    }
#pragma unroll
                    for (int m = 0; m < C; ++m) cw[m] = 0u;
                }
            }
            if (EXACT) {
                X1[C - 1] = force_last ? INF : X1[C - 1];
            } else {
#pragma unroll
                for (int m = 0; m < C; ++m) X1[m] = vmax(X1[m], tm[m]);
            }
            // windows for super-step t+D
            Aw[(u + D + C) % M] = (T)aC[u + D + C];
            Bw[(u + D) % M] = (T)bC[u + D];
        }
        if (task >= 0) tl += M;
        // early abandon on the frontier (two consecutive anti-diagonals)
        T lm = vmin(X0[0], X1[0]);
#pragma unroll
        for (int m = 1; m < C; ++m) lm = min3(lm, X0[m], X1[m]);
        T thr_now = thr;
        if constexpr (sizeof(T) == 4) {
            if (out.run_thr != nullptr)
                thr_now = __builtin_fminf(thr, __uint_as_float(__hip_atomic_load(
                                                   out.run_thr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)));
        }
        const unsigned long long ok = __ballot(lm <= thr_now);
        if (task >= 0 && ((ok >> lane0) & gmask) == 0ull) dead = true;
    }
}

}  // namespace nndtw
