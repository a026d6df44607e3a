// Row-strip wavefront engine for DTW_W with wide windows (gfx950, wave64).
//
// The diagonal-pair engine (dtw_engine.hpp) sweeps the 2W'+1 window
// diagonals; when the window covers most of the matrix (W' close to L-1)
// that sweep spans a parallelogram of up to twice the matrix, and windows of
// more than 63 x 16 diagonal pairs do not fit a wave at all.  This engine
// instead gives each lane of a wave a strip of S consecutive columns of the
// L x L cost matrix of Equation (1) (lane k: columns kS .. kS+S-1, 64 S >= L)
// and pipelines the rows across lanes: at step t lane k computes row
// i = t - k of its strip, left to right,
//   D(i,c) = (A_i - B_c)^2 + min(D(i-1,c-1), D(i-1,c), D(i,c-1)),
// from its own previous row (registers), the value of column kS-1 at rows i
// and i-1 that lane k-1 computed at steps t-1 and t-2 (one DPP shift per
// step), and A_i.  Cells outside the window |i - c| <= W' are +inf.  One
// pair of series per wave; L + (L-1)/S steps per pair.
//
// Early abandon: after step t the cells computed so far form a staircase
// (lane k's columns up to row min(t-k, L-1)).  A warping path leaves it
// through the top cell of some column, or, stepping right across a strip
// boundary, through the cell one row below the top of the strip's last
// column; both are held by the lanes (the row just computed, and the
// previous row's last value), and costs only grow along a path, so once all
// of them exceed the cutoff the result does too.
#pragma once

#include "dtw_engine.hpp"

namespace nndtw {

// Column strip width (columns per lane) for length L.
__host__ __device__ constexpr int strip_width(int L)
{
    return L <= 64 * 4 ? 4 : (L <= 64 * 8 ? 8 : (L <= 64 * 12 ? 12 : (L <= 64 * 16 ? 16 : (L <= 64 * 24 ? 24 : 32))));
}

// Band cells of column c in rows 0 .. rows-1 (|i - c| <= Wp).
__device__ __forceinline__ int band_rows(int c, int rows, int Wp)
{
    const int lo = c - Wp > 0 ? c - Wp : 0;
    const int hi = (c + Wp < rows - 1) ? c + Wp : rows - 1;
    return hi >= lo ? hi - lo + 1 : 0;
}

// Windows need 2 W' + 2 >= S (strip_fits).
__host__ __device__ constexpr bool strip_fits(int L, int Wp) { return Wp >= L - 1 || 2 * Wp + 2 >= strip_width(L); }

// Run `ntasks` pair tasks, one per wave at a time, dealt from the LDS counter
// *next_task (0 before the call, shared by the workgroup's waves).  The loop
// over tasks is wave-uniform by construction (the task index is a scalar).  Task i
// compares the unpadded float rows arow(i) and brow(i) (L elements, LDS or
// global) and is abandoned (+inf) once the staircase frontier exceeds
// thr_of(i) (or the shared run_thr, FP32 only, as in the diagonal engine).
// res[i]: DTW_W or +inf; cells[i]: band cells evaluated.  WIN: the window
// constrains (W' < L - 1).  Whole-wave call.
// deal64 != nullptr: a shared batch (several workgroups, see search.hip):
// tasks are dealt from the tagged global word as in the diagonal engine
// (shared_deal), and res / cells are global memory written with
// device-scope atomic stores, each task then counted in *done.
template <typename T, int S, bool WIN, typename ARow, typename BRow, typename Thr>
__device__ __forceinline__ void strip_run(int L, int Wp, int ntasks, int *next_task, ARow arow, BRow brow, Thr thr_of,
                                          T *res, int *cells, unsigned *run_thr = nullptr, double slack = 1.0,
                                          int rot_phase = -1, unsigned long long *deal64 = nullptr,
                                          uint32_t tag = 0, unsigned *done = nullptr)
{
    constexpr int BLK = 8;                    // steps between abandon tests (even: ping-pong rows)
    const int lane = threadIdx.x & (WAVE - 1);
    const T INF = inf_of<T>();
    const int c0 = lane * S;                  // first column of this lane's strip
    const int kend = (L - 1) / S;             // lane holding column L-1
    const int jend = (L - 1) - kend * S;
    const int steps = L + kend;               // rows 0..L-1 through lanes 0..kend
    while (true) {
        // the whole wave takes part in the fetch (lane 0 adds 1, the others
        // 0) and the task is lane 0's result: no branch on the lane, so no
        // lane can re-enter the loop apart from the others
        const int task = deal64 != nullptr
                             ? shared_deal(deal64, tag, ntasks, 1, lane)
                             : __builtin_amdgcn_readfirstlane(atomicAdd(next_task, lane == 0 ? 1 : 0));
        if (task >= ntasks) break;
        const auto a = arow(task);
        const auto b = brow(task);
        T bc[S], P0[S], P1[S];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            bc[j] = (c0 + j < L) ? (T)b[c0 + j] : Pad<T>::big();
            P0[j] = INF;
        }
        T thr = thr_of(task);
        T send = INF;                         // this lane's last column, for lane + 1
        T lcur = INF;                         // D(i, c0 - 1) for the row being computed
        T lastp = INF;                        // D(i - 1, c0 + S - 1): the previous row's last value
        bool dead = false;
        int t = 0;
        // one step: row i = t - lane from row src into row dst
        auto step = [&](const T (&src)[S], T (&dst)[S]) {
            const T lprev = lcur;             // D(i-1, c0-1)
            T recv = from_lower(send);
            const int i = t - lane;
            lcur = lane == 0 ? INF : recv;
            const T dg0 = lane == 0 ? (i == 0 ? (T)0 : INF) : lprev;
            const bool act = i >= 0 && i < L && c0 < L;
            if (act) {
                lastp = src[S - 1];
                const T ai = (T)a[i];
                T dg = dg0, lf = lcur;
                // window: only the two diagonals next to the band, c = i -
                // W' - 1 and c = i + W' + 1, are set to +inf; every cell
                // further out then has only +inf inputs and stays +inf (rows
                // start at +inf).  With 2 W' + 2 >= S at most one of them
                // crosses a strip in a row: its strip column is jm.
                const int jl = i - Wp - 1 - c0;
                const int jm = (unsigned)jl < (unsigned)S ? jl : jl + 2 * Wp + 2;
#pragma unroll
                for (int j = 0; j < S; ++j) {
                    const T up = src[j];
                    const T d = ai - bc[j];
                    T v = cell(d, min3(dg, up, lf));
                    if (WIN) v = j == jm ? INF : v;
                    dst[j] = v;
                    dg = up;
                    lf = v;
                }
            } else {
#pragma unroll
                for (int j = 0; j < S; ++j) dst[j] = src[j];
            }
            send = dst[S - 1];
            ++t;
        };
        while (t < steps) {
            if (rot_phase >= 0) rotate_priority(rot_phase);
#pragma unroll
            for (int u = 0; u < BLK; u += 2) {
                step(P0, P1);
                step(P1, P0);
            }
            // frontier: rows computed so far (after an even number of steps
            // the current rows are in P0)
            T lm = INF;
            const int i = t - 1 - lane;       // last row this lane computed (clamped below)
            if (i >= 0 && c0 < L) {
#pragma unroll
                for (int j = 0; j < S; ++j) lm = vmin(lm, P0[j]);
                lm = vmin(lm, lastp);
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) lm = vmin(lm, __shfl_xor(lm, off));
            T thr_now = thr;
            if constexpr (sizeof(T) == 4) {
                if (run_thr != nullptr)
                    thr_now = vmin(thr, __uint_as_float(__hip_atomic_load(run_thr, __ATOMIC_RELAXED,
                                                                         __HIP_MEMORY_SCOPE_WORKGROUP)));
            }
            if (lm > thr_now) {
                dead = true;
                break;
            }
        }
        // D(L-1, L-1) sits in lane kend, column jend (the steps ran past it:
        // a lane's rows stay at L-1 once done)
        T r = INF;
#pragma unroll
        for (int j = 0; j < S; ++j)
            if (j == jend) r = P0[j];
        r = __shfl(r, kend);
        // band cells evaluated: lane k's rows 0 .. min(t - 1 - k, L - 1)
        int rows = t - lane;
        rows = rows < 0 ? 0 : (rows > L ? L : rows);
        int nc = 0;
        if (c0 < L) {
#pragma unroll
            for (int j = 0; j < S; ++j)
                if (c0 + j < L) nc += band_rows(c0 + j, rows, Wp);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) nc += __shfl_xor(nc, off);
        if (lane == 0) {
            if constexpr (sizeof(T) == 4) {
                if (deal64 != nullptr) {
                    __hip_atomic_store(reinterpret_cast<unsigned *>(res) + task, __float_as_uint(dead ? INF : r),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(cells + task, nc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __builtin_amdgcn_s_waitcnt(0);
                    __hip_atomic_fetch_add(done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    res[task] = dead ? INF : r;
                    cells[task] = nc;
                }
            } else {
                res[task] = dead ? INF : r;
                cells[task] = nc;
            }
            if constexpr (sizeof(T) == 4) {
                if (run_thr != nullptr && !dead) atomicMin(run_thr, __float_as_uint(round_up_f32((double)r * slack)));
            }
        }
    }
}

}  // namespace nndtw
