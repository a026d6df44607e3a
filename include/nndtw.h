/*
 * nndtw.h -- C ABI of the MI355X (gfx950) library for nearest-neighbour search
 * under window-constrained dynamic time warping with the LB_Keogh /
 * LB_Enhanced lower-bound cascade of Tan, Petitjean & Webb, "Elastic bands
 * across the path: A new framework and method to lower bound DTW" (SDM 2019).
 *
 * Conventions for every entry point
 *  - Returns an int status: NNDTW_OK (0) or a negative NNDTW_E* code; the
 *    text of the last error of the calling thread is nndtw_last_error().
 *    Nothing throws, nothing aborts.
 *  - All arguments are validated on the host before anything is enqueued;
 *    an invalid call enqueues nothing.
 *  - Work is enqueued asynchronously on the caller's HIP stream (a
 *    hipStream_t passed as void*; NULL is the default stream).  Results are
 *    valid after the caller synchronises that stream.  The library never
 *    synchronises, never allocates device memory and never normalises data.
 *  - Array arguments are caller-owned DEVICE pointers unless stated
 *    otherwise, row-major and contiguous: a set of n series of length L is
 *    float[n][L].  Pointers must be 4-byte aligned (8 for doubles).
 *  - Series values must be finite with magnitude below 1e15.  Lengths must
 *    satisfy 2 <= L <= NNDTW_MAX_L.
 *  - W is the integer half-width of the Sakoe-Chiba window (Section 2.1):
 *    A_i may be aligned with B_j only if |i - j| <= W.  W >= 0; any
 *    W >= L-1 means unconstrained (W = L is accepted).
 *  - Distances and lower bounds are un-rooted sums of point costs
 *    delta(x, y) = (x - y)^2 (Section 2.1, Equation 2 without the root, as in
 *    the proofs of Theorems 1 and 2).
 *  - V (Section 3.1) is the number of left and right bands; V >= 1, and it is
 *    clamped to floor(L/2) as in Algorithm 1.
 *  - pairing: NNDTW_CROSS computes out[a][b] for every a < nA, b < nB;
 *    NNDTW_ZIP requires nA == nB and computes out[p] for the pair (A_p, B_p).
 */
#ifndef NNDTW_H
#define NNDTW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NNDTW_VERSION_MAJOR 0
#define NNDTW_VERSION_MINOR 1

#define NNDTW_OK      0
#define NNDTW_EINVAL (-1)   /* invalid argument                        */
#define NNDTW_EHIP   (-2)   /* a HIP runtime call failed               */
#define NNDTW_EUNSUP (-3)   /* valid but unsupported size or option    */

#define NNDTW_CROSS 0
#define NNDTW_ZIP   1

#define NNDTW_MAX_L 2048
/* Largest reference set of one set of the batched search (its visiting
 * order is sorted on chip).  nndtw_search takes any reference set. */
#define NNDTW_BATCH_MAX_N 8192
/* Largest number of waves (workgroup of 64-lane waves) one query may use.
 * Above 8 waves only engine shapes that fit 128 registers per lane qualify
 * (windows of up to 63 diagonal pairs with up to 6 pairs per lane);
 * nndtw_search_plan / nndtw_search return EUNSUP for the others. */
#define NNDTW_SEARCH_MAX_WAVES 16
/* Largest number of helper workgroups per query (nndtw_search_opts.helpers). */
#define NNDTW_SEARCH_MAX_HELPERS 7

/* Lower-bound cascades for nndtw_search. */
#define NNDTW_CASCADE_NONE      0  /* DTW_W of every candidate (with abandon)        */
#define NNDTW_CASCADE_KEOGH     1  /* LB_Keogh                                        */
#define NNDTW_CASCADE_KEOGH_ENH 2  /* LB_Keogh, then LB_Enhanced^V bands, then full   */
#define NNDTW_CASCADE_ENH       3  /* LB_Enhanced^V bands, then full                  */
/* Comparison cascades (the bounds the paper measures LB_Enhanced against,
 * Section 4, and the symmetric variant of its conclusion); nndtw_search only,
 * the batched search rejects them with NNDTW_EUNSUP. */
#define NNDTW_CASCADE_KIM       4  /* LB_Kim (sum form)                               */
#define NNDTW_CASCADE_IMPROVED  5  /* LB_Keogh (first pass), then LB_Improved         */
#define NNDTW_CASCADE_NEW       6  /* LB_New                                          */
#define NNDTW_CASCADE_ENH_SYM   7  /* LB_Enhanced^V(A,B) bands, then
                                      max(LB_Enhanced^V(A,B), LB_Enhanced^V(B,A))     */

/* Layout of the per-query counts written by nndtw_search (int64 each). */
#define NNDTW_COUNT_N              0  /* references visited (= n)                        */
#define NNDTW_COUNT_PRUNED_KEOGH   1  /* pruned by LB_Keogh (LB_Kim, LB_New in their
                                         cascades)                                       */
#define NNDTW_COUNT_PRUNED_BANDS   2  /* pruned by the band part of LB_Enhanced          */
#define NNDTW_COUNT_PRUNED_ENH     3  /* pruned by full LB_Enhanced (LB_Improved, the
                                         symmetric LB_Enhanced in their cascades)        */
#define NNDTW_COUNT_DTW_STARTED    4  /* DTW_W started (not pruned)                      */
#define NNDTW_COUNT_DTW_ABANDONED  5  /* implementation-defined: DTWs stopped early      */
#define NNDTW_COUNT_CELLS          6  /* implementation-defined: band cells evaluated    */
#define NNDTW_COUNT_RECHECKS       7  /* implementation-defined: FP64 recomputations     */
#define NNDTW_NCOUNTS              8

/* ---------------------------------------------------------------------------
 * Library information.
 */
/* Returns NNDTW_VERSION_MAJOR * 100 + NNDTW_VERSION_MINOR. */
int nndtw_version(void);
/* Static text for a status code (never NULL). */
const char *nndtw_status_string(int status);
/* Text of the last error raised by the calling thread ("" if none); the
 * pointer stays valid until the thread's next call into the library. */
const char *nndtw_last_error(void);

/* ---------------------------------------------------------------------------
 * Envelopes, Equations (3) and (4):
 *   U[s][i]  = max B[s][j],  Lo[s][i] = min B[s][j]
 *   over max(0, i-W) <= j <= min(L-1, i+W)   (0-based).
 * B: float[n][L]; U, Lo: float[n][L] outputs (exact: comparisons only).
 * n >= 0 (n = 0 enqueues nothing).  EINVAL for L, W or null pointers out of
 * range.
 */
int nndtw_envelopes(const float *B, int64_t n, int32_t L, int32_t W,
                    float *U, float *Lo, void *stream);

/* ---------------------------------------------------------------------------
 * Squared Euclidean distance sum_i (A_i - B_i)^2, accumulated in FP64 with i
 * ascending.  It equals DTW_0 (Section 2.1) and is the key of the visiting
 * order of the search (Section 4: candidates sorted by Euclidean distance).
 * A: float[nA][L], B: float[nB][L]; out: double[nA][nB] (CROSS) or [nA] (ZIP).
 */
int nndtw_ed2(const float *A, int64_t nA, const float *B, int64_t nB, int32_t L,
              int32_t pairing, double *out, void *stream);

/* ---------------------------------------------------------------------------
 * LB_Keogh (Section 2.2): sum over i of (A_i - U_i)^2 if A_i > U_i,
 * (A_i - Lo_i)^2 if A_i < Lo_i, else 0, with U/Lo the envelopes of B
 * (from nndtw_envelopes with the intended W).  FP64, i ascending.
 * A: float[nA][L]; U, Lo: float[nB][L]; out: double (CROSS [nA][nB] / ZIP [nA]).
 */
int nndtw_lb_keogh(const float *A, int64_t nA, const float *U, const float *Lo,
                   int64_t nB, int32_t L, int32_t pairing, double *out, void *stream);

/* ---------------------------------------------------------------------------
 * LB_Enhanced^V_W (Equation 7), evaluated as Algorithm 1: the point costs of
 * the two corners, then for band index i = 2..n_bands (n_bands =
 * min(floor(L/2), V)) the minimum over the left band L^W_i and over its
 * mirror image at (L, L), accumulated res <- (res + min_left) + min_right;
 * then the LB_Keogh terms of the points n_bands+1 .. L-n_bands added in
 * ascending order.  FP64 throughout.
 * cutoff: NULL, or a device double[nA]; when given, the result for a pair
 * whose band part already exceeds cutoff[a] (strictly) is +inf, the early
 * exit of Algorithm 1.
 * A: float[nA][L]; B, U, Lo: float[nB][L]; out: double (CROSS/ZIP).
 */
int nndtw_lb_enhanced(const float *A, int64_t nA, const float *B, const float *U,
                      const float *Lo, int64_t nB, int32_t L, int32_t W, int32_t V,
                      const double *cutoff, int32_t pairing, double *out, void *stream);

/* ---------------------------------------------------------------------------
 * Comparison lower bounds: the existing bounds reviewed in Section 2.2 and
 * measured against LB_Enhanced in Section 4, and the symmetric LB_Enhanced
 * of the conclusion.  FP64 from float32 inputs, sums in ascending point
 * order; each is at most DTW_W(A, B) for the same W.  Array and pairing
 * conventions as for nndtw_lb_enhanced; out: double (CROSS/ZIP).  Pointers
 * that a bound does not read may be NULL (U, Lo for nndtw_lb_kim).
 *
 * LB_Kim in the sum form of the experiments (Section 4): (A_1 - B_1)^2 +
 * (A_L - B_L)^2, plus (min A - min B)^2 unless either series takes its
 * minimum at its first or last point, plus (max A - max B)^2 under the same
 * rule for maxima ("without repetitions": each counted feature is then paid
 * by a different link of every warping path).  A, B: float[n][L].
 */
int nndtw_lb_kim(const float *A, int64_t nA, const float *B, int64_t nB, int32_t L,
                 int32_t pairing, double *out, void *stream);

/* LB_Improved (Section 2.2): LB_Keogh(A, B) + LB_Keogh(B, A'), where A' is
 * A projected on B's envelope (Equation 5: A_i clamped to [Lo_i, U_i]) and
 * the second LB_Keogh uses the envelope of A' for window W.  U, Lo: B's
 * envelopes for W (nndtw_envelopes).  cutoff: NULL, or device double[nA]:
 * where LB_Keogh(A, B) > cutoff[a] (strictly) the second pass is skipped
 * and the result is +inf. */
int nndtw_lb_improved(const float *A, int64_t nA, const float *B, const float *U,
                      const float *Lo, int64_t nB, int32_t L, int32_t W,
                      const double *cutoff, int32_t pairing, double *out, void *stream);

/* LB_New (Section 2.2): (A_1 - B_1)^2 + (A_L - B_L)^2 plus, for i = 2..L-1,
 * the smallest (A_i - B_j)^2 over max(1, i-W) <= j <= min(L, i+W). */
int nndtw_lb_new(const float *A, int64_t nA, const float *B, int64_t nB, int32_t L,
                 int32_t W, int32_t pairing, double *out, void *stream);

/* max(LB_Enhanced^V(A, B), LB_Enhanced^V(B, A)) (the conclusion: LB_Enhanced
 * is not symmetric), each direction as nndtw_lb_enhanced without cutoff.
 * U, Lo: B's envelopes for W; A's envelopes are computed internally. */
int nndtw_lb_enhanced_sym(const float *A, int64_t nA, const float *B, const float *U,
                          const float *Lo, int64_t nB, int32_t L, int32_t W, int32_t V,
                          int32_t pairing, double *out, void *stream);

/* ---------------------------------------------------------------------------
 * DTW_W (Equation 1 over the window of Section 2.1), FP32 cost matrix:
 *   D(i,j) = (A_i - B_j)^2 + min(D(i-1,j-1), D(i,j-1), D(i-1,j)),
 * result D(L,L) (un-rooted).  FP32 error is at most gamma_{2L+1} of float32
 * relative to the exact value.
 * Any window W >= 0 at any length up to NNDTW_MAX_L: windows of up to
 * 63 x 16 diagonal pairs covering less than 60 % of the L x L matrix run on
 * the anti-diagonal engine, the others on a row-strip engine (each lane a
 * strip of consecutive columns, rows pipelined across the lanes).
 * cutoff: NULL, or device double[nA]: the computation of a pair may stop
 * with +inf once every cell of a frontier that every warping path crosses
 * exceeds cutoff[a] (two consecutive anti-diagonals; on the row-strip
 * engine, the last computed row of every strip plus the cell that steps
 * right out of it), since costs only grow along a path; a finite result is
 * always the full DTW_W (possibly above the cutoff).
 * out: float (CROSS [nA][nB] / ZIP [nA]).
 */
int nndtw_dtw_w(const float *A, int64_t nA, const float *B, int64_t nB, int32_t L,
                int32_t W, const double *cutoff, int32_t pairing, float *out, void *stream);

/* As nndtw_dtw_w in FP64 with each cell computed as a product then a sum
 * (no fused multiply-add): bit-identical to a sequential FP64 evaluation of
 * the recurrence.  out: double. */
int nndtw_dtw_w_f64(const float *A, int64_t nA, const float *B, int64_t nB, int32_t L,
                    int32_t W, const double *cutoff, int32_t pairing, double *out,
                    void *stream);

/* ---------------------------------------------------------------------------
 * Reference sets.  A reference set is the training set of the search with
 * its envelopes for one window W, precomputed once ("at training time",
 * Section 4.1) in caller-provided device memory.  The descriptor below is a
 * plain host struct filled by nndtw_refset_build; it refers into `mem`,
 * which the caller keeps alive and unmodified while the set is used.
 */
#define NNDTW_REFSET_MAGIC 0x4E444157u
typedef struct nndtw_refset {
    uint32_t magic;      /* NNDTW_REFSET_MAGIC once built                  */
    int32_t  L;
    int64_t  n;
    int32_t  W;          /* window the envelopes were built for             */
    int32_t  reserved0;
    int64_t  pitch;      /* row pitch (elements) of the point-major arrays  */
    float   *B;          /* float[n][L]      the series                      */
    float   *U;          /* float[n][L]      upper envelopes                 */
    float   *Lo;         /* float[n][L]      lower envelopes                 */
    float   *Bt;         /* float[L][pitch]  point-major copies              */
    float   *Ut;
    float   *Lt;
    float   *Bp;         /* float[n][ppitch] the series inside a margin of
                          * 1e30 on both sides (rows the DTW engine streams) */
    int64_t  ppitch;     /* row pitch of Bp (elements)                       */
    int32_t  padl;       /* margin before the first value of a Bp row        */
    int32_t  reserved1;
} nndtw_refset;

/* Largest number of series in a reference set (row pitch of the
 * point-major arrays below 2^29 elements). */
#define NNDTW_REFSET_MAX_N ((int64_t)(1 << 29) - 64)
/* Device bytes needed for a reference set of n series of length L built
 * for window W.  1 <= n <= NNDTW_REFSET_MAX_N, else EINVAL. */
int nndtw_refset_bytes(int64_t n, int32_t L, int32_t W, size_t *bytes);
/* Copy B (device float[n][L]) into mem and build its envelopes and
 * point-major copies for window W.  1 <= n <= NNDTW_REFSET_MAX_N.  EINVAL
 * if bytes is too small. */
int nndtw_refset_build(const float *B, int64_t n, int32_t L, int32_t W, void *mem,
                       size_t bytes, nndtw_refset *out, void *stream);

/* ---------------------------------------------------------------------------
 * Nearest-neighbour search (Sections 1 and 4): for each query, the
 * references are visited in ascending (squared Euclidean distance, index)
 * order, cut into rounds of R consecutive candidates.  Every candidate of a
 * round is tested against
 *     thr = min(bsf, ub) * (1 + eps)
 * where bsf is the current nearest-neighbour distance (+inf at first) and ub
 * is +inf, or with init_ub the squared Euclidean distance of the first
 * visited candidate (an upper bound on its DTW_W).  A bound prunes iff it is
 * > thr; the cascade's bounds are tested in order and the first one that
 * prunes is counted.  Survivors get DTW_W (FP32, abandoned above thr); after
 * the round the record becomes the lexicographic minimum of (DTW_W, index)
 * over the round's DTWs that end <= thr (values decided in FP64).  R = 1 is
 * the paper's sequential search; with init_ub the results at R = 1 equal
 * those without it.  The nearest neighbour returned is always the
 * lexicographic argmin over all references of (DTW_W, index), i.e. ties go
 * to the lowest index, and its distance is the FP64 DTW_W.
 */
typedef struct nndtw_search_opts {
    int32_t V;        /* LB_Enhanced tightness parameter (>= 1)                      */
    int32_t cascade;  /* NNDTW_CASCADE_*                                              */
    int64_t R;        /* round size; 0 = library default; on return: the value used  */
    double  eps;      /* relative slack; <= 0 selects the floor 2 g / (1 - g) with
                       * g = (2L + 2) * 2^-24 (twice gamma_{2L+2} of float32, which
                       * covers the FP32 error of a path sum); 0 < eps < floor is
                       * EINVAL (a smaller slack could let FP32 rounding drop the
                       * nearest neighbour or a lower-index tie)                    */
    int32_t init_ub;  /* 1: bound the first round by the first candidate's ED^2      */
    int32_t cpl;      /* engine shape (diagonal pairs per lane); 0 = default; out    */
    void *const *events; /* optional hipEvent_t[5] (caller-created), recorded on the
                          * stream before the bound pass, after it (twice: the
                          * cells table is filled by the ordering kernel), after
                          * the ordering and after the search kernel; NULL
                          * records nothing                                           */
    int32_t waves;    /* waves per query (1..NNDTW_SEARCH_MAX_WAVES); 0 = default (8
                       * when the query count is at most twice the device's compute
                       * units, else 4); out                                          */
    int32_t engine;   /* DTW engine, NNDTW_ENGINE_*; 0 = library choice; out          */
    int64_t nq_hint;  /* nndtw_search_plan only: the query count to plan for (0 =
                       * many); nndtw_search plans for its own nQ                    */
    int32_t helpers;  /* helper workgroups per query (0 = default, -1 = none, at
                       * most NNDTW_SEARCH_MAX_HELPERS).  nndtw_search: default 3,
                       * launched after the queries' own workgroups (none at 3
                       * or 6 pairs per lane); a helper joins its query if it is
                       * still running and takes DTW tasks of its rounds through
                       * device-scope atomics.  Batch: default 7, the most that
                       * may join one query once a search kernel's items are all
                       * taken (idle persistent workgroups).  The result and the
                       * defined counts do not change; out (nndtw_search)     */
    int32_t order;    /* how the visiting order is found, NNDTW_ORDER_*; 0 = library
                       * choice                                                    */
} nndtw_search_opts;

/* DTW engines of the search (opts->engine).  DIAGONAL: anti-diagonal
 * sweep, groups of lanes per candidate, cpl diagonal pairs per lane, windows
 * with min(W, L-1) + 1 <= 567 (63 lanes x 9 pairs).  STRIP: one candidate per
 * wave, each lane a strip of consecutive columns with the rows pipelined
 * across the lanes; any window with 2 min(W, L-1) + 2 >= the strip width (4
 * columns for L <= 256, 8 to 512, 12 to 768, 16 to 1024, 24 to 1536, else
 * 32), or W >= L - 1; at most 8 waves per query (4 above 1024).  The
 * library's choice (AUTO): STRIP where the window is too wide for DIAGONAL,
 * and for unconstrained DTW (W >= L - 1) at L > 192; else DIAGONAL.  Both give the
 * same result and the same counts except the abandoned-DTW, cell and
 * recheck counts, which depend on where each engine tests its frontier.
 * The batched search runs DIAGONAL only. */
#define NNDTW_ENGINE_AUTO     0
#define NNDTW_ENGINE_DIAGONAL 1
#define NNDTW_ENGINE_STRIP    2

/* Visiting-order methods (opts->order).  SORT: one workgroup per query sorts
 * its (squared ED, index) pairs.  RANK: each reference's place is the count
 * of pairs that precede it, over many workgroups per query (n^2 comparisons
 * per query, but no step depends on another; at most 8192 references and
 * 2^20 workgroups of 64 references, else EUNSUP).  The library's choice
 * (AUTO): RANK while the sum of n^2 over the queries is at most 2^16 npow,
 * npow the power of two >= max(n, 256) (2^26 at 1000 references, 2^28 at
 * 4000), else SORT.  Both give the same order, so the same results and
 * counts; any other value is EINVAL. */
#define NNDTW_ORDER_AUTO 0
#define NNDTW_ORDER_SORT 1
#define NNDTW_ORDER_RANK 2

/* Workspace bytes nndtw_search needs for nQ queries against refset. */
int nndtw_search_workspace_bytes(const nndtw_refset *refset, int64_t nQ,
                                 const nndtw_search_opts *opts, size_t *bytes);

/* The launch plan nndtw_search would use for this reference set and these
 * options, decided on the host without enqueuing anything: writes opts->R
 * (round size, >= 1), opts->engine, opts->cpl (diagonal pairs per lane of
 * the DIAGONAL engine, 0 with STRIP) and opts->waves.  Every window runs on
 * one of the engines; a forced engine that cannot take the window is
 * EUNSUP. */
int nndtw_search_plan(const nndtw_refset *refset, nndtw_search_opts *opts);

/* Q: device float[nQ][L] (L of the reference set); outputs: nn_idx int64[nQ],
 * nn_dist double[nQ], counts int64[nQ][NNDTW_NCOUNTS] (NULL allowed).
 * ws: device workspace of at least nndtw_search_workspace_bytes() bytes
 * (60 bytes per (query, reference) pair, 3136 bytes per query for the
 * batches shared with helper workgroups, and a table of 8L bytes).  Any
 * reference-set size: above 8192 references the visiting order is sorted in
 * chunks of 8192 that are then merged in the workspace. */
int nndtw_search(const nndtw_refset *refset, const float *Q, int64_t nQ,
                 nndtw_search_opts *opts, int64_t *nn_idx, double *nn_dist,
                 int64_t *counts, void *ws, size_t ws_bytes, void *stream);

/* nndtw_search without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The workspace is a fixed device array of
 * NNDTW_SEARCH_SCRATCH_BYTES inside the library, one per GPU, held from the
 * device's first use until the process ends; the call allocates nothing and
 * otherwise behaves exactly as nndtw_search (same validation, kernels and
 * results).  EUNSUP when the workspace nndtw_search_workspace_bytes reports
 * exceeds NNDTW_SEARCH_SCRATCH_BYTES (60 bytes per (query, reference) pair
 * and 3136 per query: up to about 1.1 million pairs, e.g. 1000 queries x 1000
 * references; split
 * larger query sets into several calls).  Every call on one GPU uses that
 * GPU's single array: calls that overlap on the same GPU (other streams or
 * threads) race and corrupt each other's results; serialise them. */
#define NNDTW_SEARCH_SCRATCH_BYTES ((size_t)64 << 20)
/* Devices (ordinals 0 .. NNDTW_MAX_DEVICES-1) nndtw_search_noalloc serves. */
#define NNDTW_MAX_DEVICES 64
int nndtw_search_noalloc(const nndtw_refset *refset, const float *Q, int64_t nQ,
                         nndtw_search_opts *opts, int64_t *nn_idx, double *nn_dist,
                         int64_t *counts, void *stream);

/* The fused bound pass the search runs first, exposed on its own: for every
 * query q and reference k of the set, ed2 = squared Euclidean distance,
 * lbk = LB_Keogh, lbe_bands = Algorithm 1 bands part, lbe = LB_Enhanced^V
 * (values identical to nndtw_ed2 / nndtw_lb_keogh / nndtw_lb_enhanced).
 * Each output is a device double[nQ][n]; any of them may be NULL. */
int nndtw_cascade_bounds(const nndtw_refset *refset, const float *Q, int64_t nQ,
                         int32_t V, double *ed2, double *lbk, double *lbe_bands,
                         double *lbe, void *stream);

/* ------------------------------------------------------------------------
 * DTW_W backward: gradient with respect to the query along the minimising
 * warping path.  Equation (1) defines DTW_W as the minimum over warping paths
 * of the path cost; where the minimising path P* is unique the cost is
 * differentiable in A with dDTW/dA_i = sum over the cells (i, j) of P* of
 * 2 (A_i - B_j).  P* is recovered from (L-1, L-1) by taking at every cell the
 * first of (i-1,j-1), (i-1,j), (i,j-1) that attains the minimum (the order
 * that also resolves exact ties).  Arrays as for nndtw_dtw_w; f64 = 1 runs
 * the forward cells and the backward sums in FP64 (out, gout, gA double),
 * f64 = 0 in FP32 (float).  Near-ties can make FP32 choose another path than
 * FP64 with an equal cost up to FP32 rounding. */

/* Bytes of the buffer for the predecessor codes of np pairs (np = nA*nB
 * cross, nA zip): four bits per (anti-diagonal pair, window diagonal pair)
 * of each series pair and padded copies of A and B (codes: 256-byte
 * aligned device memory).  EUNSUP for
 * min(W, L-1) + 1 > 756; the FP64 calls take min(W, L-1) + 1 <= 567. */
int nndtw_dtw_codes_bytes(int64_t nA, int64_t nB, int32_t L, int32_t W, int32_t pairing,
                          size_t *bytes);

/* Forward: out = DTW_W per pair (no abandoning) and the predecessor codes
 * (device, >= nndtw_dtw_codes_bytes bytes, layout private to the library). */
int nndtw_dtw_w_codes(const float *A, int64_t nA, const float *B, int64_t nB, int32_t L,
                      int32_t W, int32_t pairing, int32_t f64, void *out, uint8_t *codes,
                      size_t codes_bytes, void *stream);

/* Backward: gA[a][i] = sum over the pairs (a, b) of gout[pair] * dDTW/dA_a[i]
 * (cross: gout [nA][nB]; zip: gout [nA]), from the codes of the forward call
 * with the same A, B, L, W, pairing and f64.  gA: device [nA][L].  Each
 * path's terms are summed per row i along the path, then the per-reference
 * row sums in ascending reference order, so results are the same from run
 * to run.  With cross pairing the backward writes the per-pair
 * row sums into the part of the codes buffer after the codes (L values per
 * series pair; the codes themselves are only read): backward calls on one
 * buffer must not overlap. */
int nndtw_dtw_w_backward(const float *A, int64_t nA, const float *B, int64_t nB, int32_t L,
                         int32_t W, int32_t pairing, int32_t f64, const void *gout,
                         const uint8_t *codes, size_t codes_bytes, void *gA, void *stream);

/* ------------------------------------------------------------------------
 * Batched search over many independent reference sets of different lengths
 * (the search of Sections 1 and 4, per set exactly as nndtw_search with the
 * same options, R and shape): every set's bound pass runs in one kernel, the
 * visiting orders in one kernel (ranking) or one per sort width, and the (set, query)
 * items in one persistent search kernel per engine shape that takes items
 * from a device counter, largest expected work first.  After nndtw_batch_prepare, the
 * launch nndtw_search_batch allocates, copies and synchronises nothing, so it
 * can be captured in a HIP graph and replayed.
 *
 * Per set: results equal nndtw_search on the same set, queries and options
 * with R and cpl as written back here (index, distance and the defined
 * counts; the implementation-defined counts depend on which DTW of a round
 * finishes first, in either call).  Sets may use
 * 1 to 4 diagonal pairs per lane, i.e. min(W, L-1) + 1 <= 252; larger windows
 * return EUNSUP. */
typedef struct nndtw_batch_set {
    const nndtw_refset *refset;  /* a built reference set (host descriptor)         */
    const float *Q;              /* device float[nQ][refset->L]                      */
    int64_t nQ;                  /* queries (>= 0)                                   */
    int64_t *nn_idx;             /* device int64[nQ]                                 */
    double *nn_dist;             /* device double[nQ]                                */
    int64_t *counts;             /* device int64[nQ][NNDTW_NCOUNTS], or NULL          */
    int64_t R;                   /* round size, 0 = default; on return: used         */
    int32_t cpl;                 /* pairs per lane, 0 = default; on return: used     */
    int32_t reserved;
} nndtw_batch_set;

/* Filled by nndtw_batch_prepare; passed unchanged to nndtw_search_batch. */
typedef struct nndtw_batch_plan {
    uint32_t magic;
    int32_t nsets;
    int64_t items;               /* (set, query) items                               */
    int64_t tiles;               /* bound-pass tiles                                  */
    int32_t waves;               /* waves per workgroup of the search kernel          */
    int32_t grid;                /* persistent search workgroups                     */
    int64_t lds;                 /* search kernel LDS bytes                          */
    int64_t ws_bytes;            /* workspace bytes the plan uses                    */
    int64_t order_off[6];        /* item-list offset and count per sort size class   */
    int64_t order_cnt[6];        /*   256, 512, ..., 8192 padded references          */
    int64_t search_off[8];       /* item-list offset and count per engine shape      */
    int64_t search_cnt[8];       /*   (C, exact) = (1,0), (1,1), ..., (4,1)          */
    int64_t reserved[4];
    int32_t helpers;             /* most helper workgroups per query (0: none)       */
    uint32_t share_shapes;       /* engine shapes whose kernel lends idle workgroups */
    int64_t share_off;           /* workspace offset of the items' helper headers    */
    int32_t order_rank;          /* 1: every visiting order by ranking, one launch   */
    int32_t order_nmax;          /* ... for sets of at most this many references     */
} nndtw_batch_plan;

/* Device workspace bytes for a batch (sets as passed to prepare, the same
 * opts): the per-set search workspaces, the item lists and, unless
 * opts->helpers is -1, a 3136-byte helper header per query. */
int nndtw_batch_workspace_bytes(const nndtw_batch_set *sets, int32_t nsets,
                                const nndtw_search_opts *opts, size_t *bytes);

/* Plan a batch into ws (device, >= nndtw_batch_workspace_bytes) and *plan:
 * validates every set, writes back each set's R and cpl, and enqueues on
 * `stream` the copy of the set descriptors and item lists into ws.  Returns
 * without waiting for the device (the host copy of that control block is
 * released by the stream once copied); run nndtw_search_batch on the same
 * stream, or ordered after it.  Options (V, cascade, eps, init_ub, waves,
 * helpers, order) are common to all sets, opts->order deciding for the
 * batch as a whole (AUTO as above, n the largest set's); opts->R and opts->cpl are ignored (per set
 * instead); opts->engine must be AUTO or DIAGONAL; opts->events must be
 * NULL. */
int nndtw_batch_prepare(nndtw_batch_set *sets, int32_t nsets, const nndtw_search_opts *opts,
                        void *ws, size_t ws_bytes, nndtw_batch_plan *plan, void *stream);

/* Run a prepared batch: 1 + (1 if plan->order_rank, else the sort widths
 * used) + (engine shapes used) kernels on `stream` (the first, the bound pass, also clears the helper
 * headers when plan->helpers > 0).  The
 * sets' reference sets, queries, outputs and ws must be those of prepare. */
int nndtw_search_batch(const nndtw_batch_plan *plan, void *ws, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* NNDTW_H */
