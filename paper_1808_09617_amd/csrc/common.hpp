// Internal definitions shared by the HIP translation units of libnndtw.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nndtw.h"

namespace nndtw {

// Status plumbing (host side, api.hip).
int fail(int status, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);

#define NNDTW_LAUNCH_CHECK(what)                                  \
    do {                                                          \
        hipError_t e_ = hipGetLastError();                        \
        if (e_ != hipSuccess) return ::nndtw::hip_fail(e_, what); \
    } while (0)

// Padding value outside a series: its square overflows to +inf, and the
// difference of two pads is exactly 0 (see the DTW engine).
template <typename T> struct Pad;
template <> struct Pad<float> { static __host__ __device__ constexpr float big() { return 1e30f; } };
template <> struct Pad<double> { static __host__ __device__ constexpr double big() { return 1e200; } };

// Wave-priority rotation for kernels whose workgroups share the SIMDs for
// their whole run.  The SIMD issues the oldest ready wave first, so of
// several co-resident workgroups the last dispatched would run mostly in the
// gaps of the others and end far behind them, alone on an otherwise idle
// SIMD.  With the rotation each wave's priority cycles through 0..3, one step
// every 20.48 us of the 100 MHz real-time clock, offset by the workgroup's
// phase, so co-resident workgroups with different phases take turns at the
// top.  Workgroups are dispatched to successive compute units, so those that
// share a unit are ncu apart in dispatch order and rotation_phase gives them
// different phases; ncu <= 0 turns the rotation off (phase -1).
__device__ __forceinline__ int rotation_phase(int ncu)
{
    if (ncu <= 0) return -1;
    const unsigned b = blockIdx.z * gridDim.y * gridDim.x + blockIdx.y * gridDim.x + blockIdx.x;
    return (int)((b / (unsigned)ncu) & 3u);
}

__device__ __forceinline__ void rotate_priority(int phase)
{
    const unsigned pr = ((unsigned)(__builtin_amdgcn_s_memrealtime() >> 11) + (unsigned)phase) & 3u;
    if (pr == 0) __builtin_amdgcn_s_setprio(0);
    else if (pr == 1) __builtin_amdgcn_s_setprio(1);
    else if (pr == 2) __builtin_amdgcn_s_setprio(2);
    else __builtin_amdgcn_s_setprio(3);
}

constexpr int WAVE = 64;

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------- launchers
// Margins of the padded rows of a reference set (elements): wide enough for
// the DTW engine at every supported shape (C <= 16 pairs per lane, prefetch
// distance <= 8).
inline int padded_row_margin_left(int Wp) { return (Wp + 48 + 3) / 4 * 4; }
inline int padded_row_margin_right(int Wp) { return Wp / 2 + 40; }

// envelopes.hip
int launch_envelopes(const float *B, int64_t n, int L, int W, float *U, float *Lo, hipStream_t s);
// The envelopes plus, from the same read of B, its row-major copy Bc and its
// padded rows Bp (a reference-set build).
int launch_envelopes_build(const float *B, int64_t n, int L, int W, float *U, float *Lo, float *Bc, float *Bp,
                           int padl, int64_t ppitch, hipStream_t s);
int launch_transpose3(const float *B, const float *U, const float *Lo, int64_t n, int L,
                      int64_t pitch, float *Bt, float *Ut, float *Lt, hipStream_t s);
int launch_pad_rows(const float *B, int64_t n, int L, int padl, int64_t ppitch, float *Bp, hipStream_t s);
// bounds.hip
int launch_pair_bounds(int what, const float *A, int64_t nA, const float *B, const float *U,
                       const float *Lo, int64_t nB, int L, int W, int V, const double *cutoff,
                       int pairing, double *out, hipStream_t s);
int launch_cascade_bounds(const nndtw_refset *rs, const float *Q, int64_t nQ, int V,
                          double *ed2, double *lbk, double *lbeb, double *lbe, hipStream_t s);
struct BatchSet;
struct BatchHdr;
struct QueryShare;
struct EngineGeom;
// Also clears the helper headers share[0 .. nshare) of the batch's items.
int launch_batch_bounds(const BatchSet *sets, int nsets, const int64_t *tile_start, int64_t tiles,
                        BatchHdr *hdr, QueryShare *share, int64_t nshare, hipStream_t s);
// compare.hip: what = 0 LB_Kim, 1 LB_Improved, 2 LB_New, 3 symmetric LB_Enhanced
int launch_compare_bounds(int what, const float *A, int64_t nA, const float *B, const float *U,
                          const float *Lo, int64_t nB, int L, int W, int V, const double *cutoff,
                          int pairing, double *out, hipStream_t s);
size_t compare_lds_bytes(int L, int W);
// dtw.hip
// Whether the row-strip engine (strip_engine.hpp) serves window Wp at length L.
bool strip_preferred(int L, int Wp);
int launch_dtw_pairs(bool f64, const float *A, int64_t nA, const float *B, int64_t nB, int L,
                     int W, const double *cutoff, int pairing, void *out, hipStream_t s);
// grad.hip
size_t dtw_codes_bytes(int64_t nA, int64_t nB, int L, int W, int pairing);
int launch_dtw_codes(bool f64, const float *A, int64_t nA, const float *B, int64_t nB, int L, int W, int pairing,
                     void *out, uint8_t *codes, hipStream_t s);
int launch_dtw_backward(bool f64, const float *A, int64_t nA, const float *B, int64_t nB, int L, int W, int pairing,
                        const void *gout, const uint8_t *codes, void *gA, hipStream_t s);
// search.hip
struct SearchPlan {
    int Wp, C, G, P, PD, SLOTS, NW, exact, T, LEN;
    int S;          // row-strip engine: columns per lane (0: anti-diagonal engine)
    int helpers;    // helper workgroups per query
    int64_t R;
    double eps;
    size_t lds_bytes;
};
// batched: plan one set of a batched search, whose kernels cover 1-4 pairs
// per lane only (it rejects sets that need more).
int plan_search(const nndtw_refset *rs, const nndtw_search_opts *o, SearchPlan *plan, bool batched = false);
size_t search_ws_bytes(int64_t nQ, int64_t n, int L);
int launch_search(const nndtw_refset *rs, const float *Q, int64_t nQ, const nndtw_search_opts *o,
                  const SearchPlan &plan, int64_t *nn_idx, double *nn_dist, int64_t *counts,
                  void *ws, hipStream_t s);
struct WsLayout {
    size_t ed2, lbk, lbeb, lbe, sk, slbk, slbeb, slbe, prefix, share, total;
};
// share: with the per-query shared batches of helper workgroups (single-set search)
WsLayout ws_layout(int64_t nQ, int64_t n, int L, bool share = true);
int launch_cells_prefix(int L, int Wp, uint32_t *prefix, hipStream_t s);
int order_width(int64_t n);     // visiting-order sort size class: npow = 256 * width
int launch_batch_order(int E, const BatchSet *sets, const int64_t *items, int64_t nitems, hipStream_t s);
int launch_batch_rank(const BatchSet *sets, const int64_t *items, int64_t nitems, int64_t nmax, hipStream_t s);
int order_by_rank(int order, double work, int64_t nmax, int64_t nitems, bool *rank);
// helpers > 0: the kernel lends idle workgroups to running queries, at most
// `helpers` per query (their QueryShare headers cleared by the bound pass)
int launch_batch_search(int C, bool exact, const BatchSet *sets, const int64_t *items, int64_t nitems,
                        unsigned *counter, unsigned *running, int waves, int grid, size_t lds, int helpers,
                        hipStream_t s);
size_t search_lds_bytes(const EngineGeom &g, const EngineGeom &gd, int SLOTS, int PD);
// Compute units of the current device (0 if it cannot be queried).
int device_cu_count();
// batch.hip
size_t batch_ws_bytes(const nndtw_batch_set *sets, int nsets, const nndtw_search_opts *o);
int batch_prepare(nndtw_batch_set *sets, int nsets, const nndtw_search_opts *o, void *ws, size_t ws_bytes,
                  nndtw_batch_plan *plan, hipStream_t s);
int batch_launch(const nndtw_batch_plan *plan, void *ws, hipStream_t s);

// Prefetch distance (super-steps) of the DTW engine for C diagonal pairs per
// lane, enough to cover the read latency: when a row is read from LDS ...
__host__ __device__ constexpr int prefetch_lds(int C) { return C == 1 ? 4 : (C <= 6 ? 2 : 1); }
// ... and when it is streamed from global memory (L2 latency).
__host__ __device__ constexpr int prefetch_global(int C)
{
    return C == 1 ? 8 : (C <= 3 ? 6 : (C <= 4 ? 4 : (C <= 6 ? 3 : (C <= 12 ? 2 : 1))));
}

// Window registers per series of the engine (M >= C + D): C + D values are
// live at a super-step; spare slots let the compiler issue the window loads
// early without register copies (for C = 3 the block of 15 super-steps
// measured fastest: 3.76 VALU instructions per cell against 4.20 at M = 9).
__host__ __device__ constexpr int window_lds(int C) { return C + prefetch_lds(C); }
__host__ __device__ constexpr int window_global(int C) { return C == 3 ? 15 : C + prefetch_global(C); }
// FP64 recheck of the search: float rows from the same places, short
// prefetch and no spare slots (double windows cost two registers per value
// and must not raise the kernel's register count above the FP32 engine's).
__host__ __device__ constexpr int recheck_prefetch(int C) { return prefetch_lds(C); }
__host__ __device__ constexpr int recheck_window(int C) { return C + recheck_prefetch(C); }
// Diagonal pairs per lane of the FP64 recheck: one when all of the window's
// pairs fit in one wave, else the FP32 engine's C.  A recheck runs while the
// query's other groups wait, so its latency (super-steps x instructions per
// super-step) is on the query's critical path, and one pair per lane has the
// shortest super-step.
__host__ __device__ constexpr int recheck_cpl(int Wp, int C) { return Wp + 1 <= 63 ? 1 : C; }

// Engine geometry shared by the DTW kernels (see dtw_engine.hpp).
struct EngineGeom {
    int L, Wp, C, G, P, exact;
    int D;      // prefetch distance (super-steps)
    int M;      // window registers (super-steps per unrolled block)
    int T;      // super-steps (multiple of M)
    int t0;     // first super-step a task executes (multiple of M, before the matrix)
    int base0;  // series index of the first super-step's base
    int LEN;    // elements per staged series in LDS (with padding)
};
// The FP32 batch of one query that helper workgroups share (search.hip):
// every field is read and written with device-scope atomics only.
constexpr int SHARE_SLOTS = 256;
struct QueryShare {
    unsigned long long deal;  // (tag << 32) | next task index; tag = (epoch << 12) | batch
    unsigned done;            // tasks of the current batch finished (by any workgroup)
    unsigned nt;              // tasks in the current batch
    unsigned thrF;            // the batch's FP32 threshold (bits)
    unsigned helpers;         // (epoch << 12) | helper workgroups that joined in that call
    unsigned finished;        // epoch of the last call in which the query finished
    unsigned started;         // epoch of the last call in which the query's owner started
    unsigned pad[8];
    uint32_t cand[SHARE_SLOTS];
    unsigned res[SHARE_SLOTS];
    int trun[SHARE_SLOTS];
};
// Clears the header words of a QueryShare (before a launch whose epoch may
// repeat an earlier one); the slots need no clearing.
__device__ __forceinline__ void share_clear(QueryShare &s)
{
    s.deal = 0ull;
    s.done = 0u;
    s.nt = 0u;
    s.helpers = 0u;
    s.finished = 0u;
    s.started = 0u;
}

// Arguments of the per-query search (search.hip): one query against one
// reference set, with the workspace of that set.
struct SearchArgs {
    EngineGeom geo;    // FP32 engine (rows streamed from global memory)
    EngineGeom geoD;   // FP64 recheck engine (the same float rows, converted)
    int PD;        // FP64 rechecks per engine call (<= 64)
    int SLOTS;     // candidates per FP32 batch (<= 256)
    const float *B;
    const float *Bp;   // padded rows of the reference set
    int64_t ppitch;
    int padl;
    int64_t n;
    const float *Q;
    const uint32_t *sk;
    const double *slbk, *slbeb, *slbe, *ed2;
    const uint32_t *prefix;
    int cascade;
    int64_t R;
    double eps;
    int init_ub;
    int64_t *nn_idx;
    double *nn_dist;
    int64_t *counts;
    int ncu;           // compute units of the device (> 0: rotate the FP32
                       // engine's wave priority, see TaskOut)
    QueryShare *share; // per query, or nullptr (no helper workgroups)
    int64_t nq;        // queries (workgroups from nq on are helpers)
    uint32_t epoch;    // this call's tag (1 .. 2^20 - 1)
};

// One reference set of a batched search: the search arguments plus what the
// bound pass and the ordering of the batch need (batch.hip).
struct BatchSet {
    SearchArgs a;
    int C, exact;               // engine shape of the set
    const float *Bt, *Ut, *Lt;  // point-major copies of the reference set
    int64_t pitch, nQ;
    int L, W, nb;               // length, window, LB_Enhanced band count
    int64_t nrt;                // reference tiles of the bound pass
    double *ed2w, *lbk, *lbeb, *lbe;
    uint32_t *skw;
    double *slbkw, *slbebw, *slbew;
};
constexpr int BATCH_SHAPES = 8;  // engine shapes (C, EXACT), C = 1..4
constexpr int BATCH_MAX_GRID = 4096;  // persistent search workgroups at most
struct BatchHdr {
    unsigned counter[BATCH_SHAPES];   // next search item per shape (reset by the bound pass)
    // item + 1 that each persistent search workgroup runs (0: none; values
    // left by an earlier kernel name items that have been taken as well)
    unsigned running[BATCH_MAX_GRID];
};

// Choose the diagonal-pairs-per-lane C for a window (cmax bounds latency).
int choose_cpl(int Wp, int cmax, int prefer, int chard = 16, bool widen_single = false);
EngineGeom make_geom(int L, int W, int C, int D, int M);
// Geometry of the search's FP64 recheck for an FP32 engine of C pairs per lane.
inline EngineGeom recheck_geom(int L, int W, int C)
{
    const int Wp = W < L - 1 ? W : L - 1;
    const int CD = recheck_cpl(Wp, C);
    return make_geom(L, W, CD, recheck_prefetch(CD), recheck_window(CD));
}
// Elements of the query row the search stages for both engines: the
// recheck's rows start C - CD elements after the FP32 engine's (its left
// padding is CD instead of C elements).
__host__ __device__ inline int staged_len(const EngineGeom &g, const EngineGeom &gd)
{
    const int ld = gd.LEN + g.C - gd.C;
    return g.LEN > ld ? g.LEN : ld;
}
bool cpl_supported(int C);

}  // namespace nndtw
