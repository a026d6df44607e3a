/*
 * nndtw_oracle.c -- plain, slow FP64 CPU oracle for nearest-neighbour search
 * under window-constrained DTW with the LB_Keogh / LB_Enhanced cascade of
 * Tan, Petitjean & Webb, "Elastic bands across the path: A new framework and
 * method to lower bound DTW" (SDM 2019, arXiv 1808.09617).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The GPU library shares
 * no code, header or table with it, and nothing in the product path calls it.
 *
 * Conventions (readings of the paper, listed with reasons in the design notes):
 *   - inputs are float32 series, widened to double; all arithmetic is FP64,
 *     compiled with -ffp-contract=off so every product and sum rounds once;
 *   - point cost delta(x, y) = (x - y)^2 (Section 2.1: the L2 cost of two
 *     points; squared so that DTW_0 is the squared Euclidean distance);
 *   - DTW distances and lower bounds are un-rooted sums of point costs (the
 *     proofs of Theorems 1 and 2 sum delta along the path without a root);
 *   - W is an integer half-width >= 0; W >= L-1 means unconstrained;
 *   - indices are 0-based here; comments give the paper's 1-based form;
 *   - V >= 1 and L >= 2; the number of bands is min(floor(L/2), V)
 *     (Algorithm 1, the n_bands assignment).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OINF INFINITY

enum { CASCADE_NONE = 0, CASCADE_KEOGH = 1, CASCADE_KEOGH_ENH = 2, CASCADE_ENH = 3,
       CASCADE_KIM = 4, CASCADE_IMPROVED = 5, CASCADE_NEW = 6, CASCADE_ENH_SYM = 7 };
enum { C_N = 0, C_PRUNED_KEOGH, C_PRUNED_ENH_BANDS, C_PRUNED_ENH, C_DTW_STARTED,
       C_DTW_ABANDONED, C_CELLS, C_RECHECKS, C_NCOUNTS };

/* Point cost of Section 2.1 (squared difference). */
static double delta(float x, float y)
{
    double d = (double)x - (double)y;
    return d * d;
}

static double dmin(double a, double b) { return b < a ? b : a; }
static int imin(int a, int b) { return a < b ? a : b; }
static int imax(int a, int b) { return a > b ? a : b; }

/* Effective half-width: a window wider than L-1 constrains nothing. */
static int eff_window(int L, int W) { return W < L - 1 ? W : L - 1; }

static int n_bands_of(int L, int V) { return imin(L / 2, V); }

/* Relative slack for every prune/abandon test: twice gamma_{2L+2} of float32,
 * gamma_n = n u / (1 - n u) with u = 2^-24.  An FP32 warping-path sum has at
 * most 2L-1 cells; its first term is rounded once by the difference (twice
 * after squaring) and once by every fused multiply-add after it, so every
 * FP32 path cost is within a factor 1 +- gamma_{2L+1} of the exact one, and
 * twice gamma_{2L+2} exceeds twice gamma_{2L+1} at every length.  (The
 * approximation 2 (2L+2) u falls just short of 2 gamma_{2L+1} at L = 2048.) */
double oracle_slack(int L)
{
    double nu = (double)(2 * L + 2) * ldexp(1.0, -24);
    return 2.0 * nu / (1.0 - nu);
}

/* ------------------------------------------------------------------------ */
/* Envelopes, Equations (3) and (4): U_i = max and Lo_i = min of B_j over
 * max(1, i-W) <= j <= min(L, i+W).  Direct O(L W) evaluation.             */
void oracle_envelopes(const float *B, int64_t n, int L, int W, float *U, float *Lo)
{
    int w = eff_window(L, W);
    for (int64_t s = 0; s < n; ++s) {
        const float *b = B + s * L;
        for (int i = 0; i < L; ++i) {
            int lo = imax(0, i - w), hi = imin(L - 1, i + w);
            float u = b[lo], l = b[lo];
            for (int j = lo; j <= hi; ++j) {
                if (b[j] > u) u = b[j];
                if (b[j] < l) l = b[j];
            }
            U[s * L + i] = u;
            Lo[s * L + i] = l;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Squared Euclidean distance, sum_i delta(A_i, B_i), i ascending.  Equals
 * DTW_0 (Section 2.1) and is the visiting-order key of Section 4.          */
double oracle_ed2(const float *A, const float *B, int L)
{
    double s = 0.0;
    for (int i = 0; i < L; ++i) s += delta(A[i], B[i]);
    return s;
}

/* Keogh term for point i: distance of A_i to the envelope [Lo_i, U_i],
 * zero inside it (LB_Keogh definition, Section 2.2).                        */
static double keogh_term(float a, float u, float l)
{
    if (a > u) return delta(a, u);
    if (a < l) return delta(a, l);
    return 0.0;
}

/* LB_Keogh_W(A, B) = sum_{i=1}^{L} Keogh term (the sum's upper limit "m" is
 * read as L).  Accumulated with i ascending.                                */
double oracle_lb_keogh(const float *A, const float *U, const float *Lo, int L)
{
    double s = 0.0;
    for (int i = 0; i < L; ++i) s += keogh_term(A[i], U[i], Lo[i]);
    return s;
}

/* ------------------------------------------------------------------------ */
/* Band sets of Section 3, as explicit lists of links (j, k) meaning that
 * A_j is aligned with B_k (0-based).
 *
 * Left band  L^W_i = {(i,i)} u {(i,j), (j,i) : max(1, i-W) <= j < i}
 * Right band R^W_p = {(p,p)} u {(p,q), (q,p) : p < q <= min(L, p+W)}
 * The right-band set as printed is garbled; this reading is the mirror image
 * of the left band at (L, L), which is what Algorithm 1 evaluates.
 * side: 0 = left, 1 = right, 2 = the vertical band V_i of Theorem 2's proof,
 * V_i = {(i, j) : max(1, i-W) <= j <= min(L, i+W)}.
 * Returns the number of links written (at most 2W+1).                      */
int oracle_band_cells(int L, int W, int side, int i, int *rows, int *cols)
{
    int w = eff_window(L, W), n = 0;
    if (i < 0 || i >= L) return 0;
    if (side == 2) {
        for (int j = imax(0, i - w); j <= imin(L - 1, i + w); ++j) { rows[n] = i; cols[n] = j; ++n; }
        return n;
    }
    rows[n] = i; cols[n] = i; ++n;
    if (side == 0) {
        for (int j = imax(0, i - w); j < i; ++j) {
            rows[n] = i; cols[n] = j; ++n;
            rows[n] = j; cols[n] = i; ++n;
        }
    } else {
        for (int q = i + 1; q <= imin(L - 1, i + w); ++q) {
            rows[n] = i; cols[n] = q; ++n;
            rows[n] = q; cols[n] = i; ++n;
        }
    }
    return n;
}

/* min over a band of delta(A_j, B_k), by enumerating the band's links.     */
static double band_min(const float *A, const float *B, int L, int W, int side, int i)
{
    int rows[2 * 4096 + 2], cols[2 * 4096 + 2];
    int n = oracle_band_cells(L, imin(W, 4096), side, i, rows, cols);
    double m = OINF;
    for (int c = 0; c < n; ++c) m = dmin(m, delta(A[rows[c]], B[cols[c]]));
    return m;
}

/* Theorem 1: sum_{i=1}^{L} min over L^W_i is a lower bound on DTW_W.       */
double oracle_left_bands_sum(const float *A, const float *B, int L, int W)
{
    double s = 0.0;
    for (int i = 0; i < L; ++i) s += band_min(A, B, L, W, 0, i);
    return s;
}

/* Equation (6): the right-band analogue.                                    */
double oracle_right_bands_sum(const float *A, const float *B, int L, int W)
{
    double s = 0.0;
    for (int i = 0; i < L; ++i) s += band_min(A, B, L, W, 1, i);
    return s;
}

/* LB_Enhanced^V_W from its definition, Equation (7): for i = 1..L (ascending)
 * add the left-band minimum if i <= V, the right-band minimum if i > L - V,
 * and the Keogh term otherwise.  V is clamped to floor(L/2).              */
double oracle_lb_enhanced_eq7(const float *A, const float *B, const float *U,
                              const float *Lo, int L, int W, int V)
{
    int nb = n_bands_of(L, V);
    double s = 0.0;
    for (int i = 0; i < L; ++i) {
        if (i < nb)            s += band_min(A, B, L, W, 0, i);
        else if (i >= L - nb)  s += band_min(A, B, L, W, 1, i);
        else                   s += keogh_term(A[i], U[i], Lo[i]);
    }
    return s;
}

/* Bands part of LB_Enhanced^V_W (Equation 7): the band minima at both ends
 * of the series, from the explicit band sets above.  Band index k = 1 is the
 * single link (1, 1) on the left and (L, L) on the right; for k = 2..n_bands
 * the left band L^W_k and the right band R^W_{L-k+1} (the mirror image of
 * L^W_k at (L, L)).  Summation order (a convention shared with the GPU path,
 * the order Algorithm 1 accumulates in): the two corner links first, then
 * per band index the left minimum and then the right one.                  */
double oracle_lb_enhanced_bands(const float *A, const float *B, int L, int W, int V)
{
    int nb = n_bands_of(L, V);
    double res = band_min(A, B, L, W, 0, 0) + band_min(A, B, L, W, 1, L - 1);
    for (int k = 1; k < nb; ++k) {
        double left = band_min(A, B, L, W, 0, k);
        double right = band_min(A, B, L, W, 1, L - 1 - k);
        res = res + left + right;
    }
    return res;
}

/* LB_Enhanced^V_W with the early exit of the paper's search: the bands part;
 * if it already exceeds the current nearest-neighbour distance D the bound is
 * +inf (strict comparison: a bound equal to D cannot exclude a tie),
 * otherwise the LB_Keogh terms of the middle points n_bands+1 .. L-n_bands
 * (1-based) are added in ascending order.  With D = +inf this is Equation 7
 * summed in the order above.                                               */
double oracle_lb_enhanced_alg1(const float *A, const float *B, const float *U,
                               const float *Lo, int L, int W, int V, double D)
{
    int nb = n_bands_of(L, V);
    double res = oracle_lb_enhanced_bands(A, B, L, W, V);
    if (res > D) return OINF;
    for (int i = nb; i < L - nb; ++i) res += keogh_term(A[i], U[i], Lo[i]);
    return res;
}

/* ------------------------------------------------------------------------ */
/* Comparison bounds: the existing lower bounds the paper reviews (Section
 * 2.2) and measures against (Section 4), and the symmetric variant its
 * conclusion suggests.                                                      */

/* LB_Kim in the sum form of the experiments (Section 4): the point costs of
 * the first points, of the last points, of the two minima and of the two
 * maxima, summed "without repetitions".  Reading: the min feature
 * delta(min A, min B) is added only when neither series takes its minimum
 * value at its first or last point, and likewise the max feature; the sum
 * runs first, last, min, max (the order of the feature list).  With that
 * rule each feature is paid by a different link of every warping path (the
 * corners, a link in an interior row or column holding an extreme), so the
 * sum is a lower bound on DTW_W for every W.                               */
double oracle_lb_kim(const float *A, const float *B, int L)
{
    float amin = A[0], amax = A[0], bmin = B[0], bmax = B[0];
    for (int i = 1; i < L; ++i) {
        if (A[i] < amin) amin = A[i];
        if (A[i] > amax) amax = A[i];
        if (B[i] < bmin) bmin = B[i];
        if (B[i] > bmax) bmax = B[i];
    }
    double s = delta(A[0], B[0]) + delta(A[L - 1], B[L - 1]);
    int min_at_end = A[0] == amin || A[L - 1] == amin || B[0] == bmin || B[L - 1] == bmin;
    int max_at_end = A[0] == amax || A[L - 1] == amax || B[0] == bmax || B[L - 1] == bmax;
    if (!min_at_end) s += delta(amin, bmin);
    if (!max_at_end) s += delta(amax, bmax);
    return s;
}

/* LB_Improved (Section 2.2): LB_Keogh(A, B), then the projection A' of A on
 * B's envelope (Equation 5: A_i clamped to [Lo_i, U_i]), the envelope of A'
 * for the same W, and LB_Keogh(B, A') against it; the result is the sum of
 * the two.  Second-pass skip: when the first pass already exceeds cutoff
 * (strictly) the second is not computed and the result is +inf.          */
double oracle_lb_improved(const float *A, const float *B, const float *U, const float *Lo,
                          int L, int W, double cutoff)
{
    double k1 = oracle_lb_keogh(A, U, Lo, L);
    if (k1 > cutoff) return OINF;
    float *P = (float *)malloc(sizeof(float) * (size_t)L * 3);
    float *UP = P + L, *LP = P + 2 * L;
    for (int i = 0; i < L; ++i) {
        if (A[i] > U[i])       P[i] = U[i];
        else if (A[i] < Lo[i]) P[i] = Lo[i];
        else                   P[i] = A[i];
    }
    oracle_envelopes(P, 1, L, W, UP, LP);
    double k2 = oracle_lb_keogh(B, UP, LP, L);
    free(P);
    return k1 + k2;
}

/* LB_New (Section 2.2): the two corner costs, then for every interior point
 * i = 2..L-1 (ascending) the smallest cost of A_i against a point of B
 * inside its window, max(1, i-W) <= j <= min(L, i+W).                      */
double oracle_lb_new(const float *A, const float *B, int L, int W)
{
    int w = eff_window(L, W);
    double s = delta(A[0], B[0]) + delta(A[L - 1], B[L - 1]);
    for (int i = 1; i < L - 1; ++i) {
        double m = OINF;
        for (int j = imax(0, i - w); j <= imin(L - 1, i + w); ++j) m = dmin(m, delta(A[i], B[j]));
        s += m;
    }
    return s;
}

/* max(LB_Enhanced^V(A, B), LB_Enhanced^V(B, A)) (the conclusion: LB_Enhanced
 * is not symmetric, so the larger of the two directions is also a bound).
 * UA/LoA and UB/LoB are the envelopes of A and B for window W; each
 * direction is Algorithm 1 without early exit.                            */
double oracle_lb_enhanced_sym(const float *A, const float *UA, const float *LoA, const float *B,
                              const float *UB, const float *LoB, int L, int W, int V)
{
    double ab = oracle_lb_enhanced_alg1(A, B, UB, LoB, L, W, V, OINF);
    double ba = oracle_lb_enhanced_alg1(B, A, UA, LoA, L, W, V, OINF);
    return ab > ba ? ab : ba;
}

/* ------------------------------------------------------------------------ */
/* DTW_W by the cost-matrix recurrence, Equation (1):
 *   D(i,j) = delta(A_i, B_j) + min(D(i-1,j-1), D(i,j-1), D(i-1,j))
 * for |i - j| <= W, +inf outside the window, D(0,0) = 0 before the first
 * cell.  Rows i ascending, each row recomputed from scratch: cells outside
 * the window are +inf.  With thr finite, the computation stops with +inf as
 * soon as a whole row exceeds thr (every warping path visits every row, and
 * costs only grow along a path).  *cells receives the cells evaluated.     */
static double dtw_rows(const float *A, const float *B, int L, int W, double thr, int64_t *cells)
{
    int w = eff_window(L, W);
    double *prev = (double *)malloc(sizeof(double) * (size_t)(L + 1));
    double *cur = (double *)malloc(sizeof(double) * (size_t)(L + 1));
    int64_t nc = 0;
    /* column/row 0 are the virtual origin: D(0,0) = 0, D(0,j>0) = +inf */
    prev[0] = 0.0;
    for (int j = 1; j <= L; ++j) prev[j] = OINF;
    double result = OINF;
    int abandoned = 0;
    for (int i = 1; i <= L; ++i) {
        for (int j = 0; j <= L; ++j) cur[j] = OINF;
        int lo = imax(1, i - w), hi = imin(L, i + w);
        double rowmin = OINF;
        for (int j = lo; j <= hi; ++j) {
            double m = dmin(dmin(prev[j - 1], cur[j - 1]), prev[j]);
            cur[j] = delta(A[i - 1], B[j - 1]) + m;
            rowmin = dmin(rowmin, cur[j]);
        }
        nc += hi - lo + 1;
        if (rowmin > thr) { abandoned = 1; break; }
        double *t = prev; prev = cur; cur = t;
    }
    if (!abandoned) result = prev[L];
    free(prev);
    free(cur);
    if (cells) *cells = nc;
    return result;
}

double oracle_dtw(const float *A, const float *B, int L, int W)
{
    return dtw_rows(A, B, L, W, OINF, NULL);
}

double oracle_dtw_abandon(const float *A, const float *B, int L, int W, double thr)
{
    return dtw_rows(A, B, L, W, thr, NULL);
}

/* ------------------------------------------------------------------------ */
/* Batch drivers.  pairing 0 = cross (out[a*nB + b]), 1 = zip (out[a]).      */
void oracle_ed2_batch(const float *A, int64_t nA, const float *B, int64_t nB, int L,
                      int pairing, double *out)
{
    int64_t np = pairing ? nA : nA * nB;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < np; ++p) {
        int64_t a = pairing ? p : p / nB, b = pairing ? p : p % nB;
        out[p] = oracle_ed2(A + a * L, B + b * L, L);
    }
}

void oracle_lb_keogh_batch(const float *A, int64_t nA, const float *U, const float *Lo,
                           int64_t nB, int L, int pairing, double *out)
{
    int64_t np = pairing ? nA : nA * nB;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < np; ++p) {
        int64_t a = pairing ? p : p / nB, b = pairing ? p : p % nB;
        out[p] = oracle_lb_keogh(A + a * L, U + b * L, Lo + b * L, L);
    }
}

/* variant: 0 = Equation (7), 1 = Algorithm 1 (with cutoff[a] or +inf when
 * cutoff is NULL), 2 = Algorithm 1 bands part only.                         */
void oracle_lb_enhanced_batch(const float *A, int64_t nA, const float *B, const float *U,
                              const float *Lo, int64_t nB, int L, int W, int V,
                              const double *cutoff, int pairing, int variant, double *out)
{
    int64_t np = pairing ? nA : nA * nB;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < np; ++p) {
        int64_t a = pairing ? p : p / nB, b = pairing ? p : p % nB;
        const float *x = A + a * L, *y = B + b * L, *u = U + b * L, *l = Lo + b * L;
        if (variant == 0)      out[p] = oracle_lb_enhanced_eq7(x, y, u, l, L, W, V);
        else if (variant == 1) out[p] = oracle_lb_enhanced_alg1(x, y, u, l, L, W, V, cutoff ? cutoff[a] : OINF);
        else                   out[p] = oracle_lb_enhanced_bands(x, y, L, W, V);
    }
}

/* Comparison bounds over pairs.  what: 0 LB_Kim, 1 LB_Improved (second pass
 * skipped above cutoff[a] when cutoff is given), 2 LB_New, 3 the symmetric
 * LB_Enhanced^V.  U/Lo are the envelopes of B; UA/LoA those of A (what = 3
 * only).                                                                   */
void oracle_lb_compare_batch(int what, const float *A, const float *UA, const float *LoA, int64_t nA,
                             const float *B, const float *U, const float *Lo, int64_t nB, int L,
                             int W, int V, const double *cutoff, int pairing, double *out)
{
    int64_t np = pairing ? nA : nA * nB;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < np; ++p) {
        int64_t a = pairing ? p : p / nB, b = pairing ? p : p % nB;
        const float *x = A + a * L, *y = B + b * L;
        if (what == 0)      out[p] = oracle_lb_kim(x, y, L);
        else if (what == 1) out[p] = oracle_lb_improved(x, y, U + b * L, Lo + b * L, L, W,
                                                        cutoff ? cutoff[a] : OINF);
        else if (what == 2) out[p] = oracle_lb_new(x, y, L, W);
        else                out[p] = oracle_lb_enhanced_sym(x, UA + a * L, LoA + a * L, y, U + b * L,
                                                            Lo + b * L, L, W, V);
    }
}

void oracle_dtw_batch(const float *A, int64_t nA, const float *B, int64_t nB, int L, int W,
                      const double *cutoff, int pairing, double *out)
{
    int64_t np = pairing ? nA : nA * nB;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < np; ++p) {
        int64_t a = pairing ? p : p / nB, b = pairing ? p : p % nB;
        double thr = cutoff ? cutoff[a] : OINF;
        out[p] = dtw_rows(A + a * L, B + b * L, L, W, thr, NULL);
    }
}

/* ------------------------------------------------------------------------ */
/* Nearest-neighbour search.
 *
 * Brute force: NN(q) = lexicographic argmin over k of (DTW_W(q, b_k), k).  */
void oracle_brute_nn(const float *refs, int64_t N, const float *queries, int64_t Q, int L, int W,
                     int64_t *nn_idx, double *nn_dist)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < Q; ++q) {
        double best = OINF;
        int64_t bi = -1;
        for (int64_t k = 0; k < N; ++k) {
            double d = oracle_dtw(queries + q * L, refs + k * L, L, W);
            if (bi < 0 || d < best) { best = d; bi = k; }
        }
        nn_idx[q] = bi;
        nn_dist[q] = best;
    }
}

typedef struct { double key; int64_t idx; } okey;

static int okey_cmp(const void *x, const void *y)
{
    const okey *a = (const okey *)x, *b = (const okey *)y;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

/* (d, k) lexicographically smaller than (bd, bk); bk < 0 means "none yet". */
static int lexless(double d, int64_t k, double bd, int64_t bk)
{
    if (bk < 0) return 1;
    return d < bd || (d == bd && k < bk);
}

/* Lower-bound search (Section 1 and Section 4): visit the references in
 * ascending (squared Euclidean distance to the query, index) order; for each
 * one, apply the cascade against the current threshold and compute DTW_W
 * (abandoning above the threshold) only if no bound exceeds it.
 *
 * The visit is cut into rounds of R consecutive candidates: all candidates of
 * a round are tested against the threshold in force at the round's start,
 * and the nearest-neighbour record is updated after the round with the
 * lexicographic minimum of (DTW, index) over the round's completed DTWs.
 * R = 1 is the paper's sequential loop.  Threshold of a round:
 *     thr = min(bsf, ub) * (1 + slack)
 * where bsf is the current nearest-neighbour distance (+inf before the first
 * completed DTW) and ub = +inf, or with init_ub = 1 the squared Euclidean
 * distance of the first visited candidate (an upper bound on its DTW_W and so
 * on the answer; with R = 1 both choices give identical results).  A bound
 * prunes iff bound > thr (strict).  The stage of the first bound that prunes
 * is counted.  Cascades: 0 none, 1 LB_Keogh, 2 LB_Keogh then LB_Enhanced^V
 * (bands part, then full), 3 LB_Enhanced^V only (bands, then full); the
 * comparison cascades 4 LB_Kim, 5 LB_Improved (LB_Keogh as its first pass,
 * then the full bound), 6 LB_New, 7 the symmetric LB_Enhanced^V (bands part
 * of LB_Enhanced^V(A, B), then the larger of both directions).
 * counts[q*8 + .] = {N, pruned by stage 1, 2, 3, dtw_started, dtw_abandoned,
 * cells, fp64_rechecks}; stage 1 is LB_Keogh (cascades 1, 2, 5), LB_Kim (4)
 * or LB_New (6); stage 2 the bands part of LB_Enhanced (2, 3, 7); stage 3
 * the full LB_Enhanced (2, 3), LB_Improved (5) or the symmetric bound (7). */
void oracle_search(const float *refs, int64_t N, const float *queries, int64_t Q, int L,
                   int W, int V, int cascade, int64_t R, int init_ub,
                   int64_t *nn_idx, double *nn_dist, int64_t *counts)
{
    float *U = (float *)malloc(sizeof(float) * (size_t)(N * L));
    float *Lo = (float *)malloc(sizeof(float) * (size_t)(N * L));
    oracle_envelopes(refs, N, L, W, U, Lo);
    double slack = oracle_slack(L);
    if (R < 1) R = 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < Q; ++q) {
        const float *A = queries + q * L;
        float *UA = (float *)malloc(sizeof(float) * (size_t)L * 2), *LoA = UA + L;
        oracle_envelopes(A, 1, L, W, UA, LoA);
        okey *order = (okey *)malloc(sizeof(okey) * (size_t)N);
        double *rd = (double *)malloc(sizeof(double) * (size_t)R);
        int64_t *rk = (int64_t *)malloc(sizeof(int64_t) * (size_t)R);
        int64_t *c = counts + q * C_NCOUNTS;
        for (int t = 0; t < C_NCOUNTS; ++t) c[t] = 0;
        c[C_N] = N;
        for (int64_t k = 0; k < N; ++k) {
            order[k].key = oracle_ed2(A, refs + k * L, L);
            order[k].idx = k;
        }
        qsort(order, (size_t)N, sizeof(okey), okey_cmp);
        double ub = (init_ub && N > 0) ? order[0].key : OINF;
        double bsf = OINF;
        int64_t bk = -1;
        for (int64_t r0 = 0; r0 < N; r0 += R) {
            double thr = dmin(bsf, ub) * (1.0 + slack);
            int64_t nr = 0;
            for (int64_t pos = r0; pos < N && pos < r0 + R; ++pos) {
                int64_t k = order[pos].idx;
                const float *Bk = refs + k * L, *Uk = U + k * L, *Lk = Lo + k * L;
                if (cascade == CASCADE_KEOGH || cascade == CASCADE_KEOGH_ENH) {
                    if (oracle_lb_keogh(A, Uk, Lk, L) > thr) { c[C_PRUNED_KEOGH]++; continue; }
                }
                if (cascade == CASCADE_KEOGH_ENH || cascade == CASCADE_ENH) {
                    if (oracle_lb_enhanced_bands(A, Bk, L, W, V) > thr) { c[C_PRUNED_ENH_BANDS]++; continue; }
                    if (oracle_lb_enhanced_alg1(A, Bk, Uk, Lk, L, W, V, OINF) > thr) { c[C_PRUNED_ENH]++; continue; }
                }
                if (cascade == CASCADE_KIM && oracle_lb_kim(A, Bk, L) > thr) { c[C_PRUNED_KEOGH]++; continue; }
                if (cascade == CASCADE_IMPROVED) {
                    if (oracle_lb_keogh(A, Uk, Lk, L) > thr) { c[C_PRUNED_KEOGH]++; continue; }
                    if (oracle_lb_improved(A, Bk, Uk, Lk, L, W, OINF) > thr) { c[C_PRUNED_ENH]++; continue; }
                }
                if (cascade == CASCADE_NEW && oracle_lb_new(A, Bk, L, W) > thr) { c[C_PRUNED_KEOGH]++; continue; }
                if (cascade == CASCADE_ENH_SYM) {
                    if (oracle_lb_enhanced_bands(A, Bk, L, W, V) > thr) { c[C_PRUNED_ENH_BANDS]++; continue; }
                    if (oracle_lb_enhanced_sym(A, UA, LoA, Bk, Uk, Lk, L, W, V) > thr) { c[C_PRUNED_ENH]++; continue; }
                }
                c[C_DTW_STARTED]++;
                int64_t nc = 0;
                double d = dtw_rows(A, Bk, L, W, thr, &nc);
                c[C_CELLS] += nc;
                if (d == OINF && thr < OINF) { c[C_DTW_ABANDONED]++; continue; }
                if (d > thr) continue;        /* completed above the threshold: cannot be the NN */
                rd[nr] = d;
                rk[nr] = k;
                ++nr;
            }
            for (int64_t t = 0; t < nr; ++t)
                if (lexless(rd[t], rk[t], bsf, bk)) { bsf = rd[t]; bk = rk[t]; }
        }
        nn_idx[q] = bk;
        nn_dist[q] = bsf;
        free(order);
        free(UA);
        free(rd);
        free(rk);
    }
    free(U);
    free(Lo);
}

/* ------------------------------------------------------------------------ */
/* DTW_W gradient with respect to the query along the argmin warping path.    */
/* The paper defines DTW_W (Equation 1) but no gradient.  With the point cost */
/* delta(a_i, b_j) = (a_i - b_j)^2, DTW_W(A, B) is the minimum over warping   */
/* paths of the path cost; where the minimising path P* is unique, the cost   */
/* is differentiable in A with                                               */
/*   dDTW/da_i = sum over the cells (i, j) of P* of 2 (a_i - b_j).           */
/* P* is recovered by walking back from (L-1, L-1): at each cell the         */
/* predecessor is the first of (i-1, j-1), (i-1, j), (i, j-1) whose D equals */
/* their minimum (the fixed order that also resolves exact ties).            */

/* Full FP64 cost matrix D[i*L + j] (+inf outside the window); returns D(L-1,L-1). */
static double dtw_full(const float *A, const float *B, int L, int W, double *D)
{
    int w = eff_window(L, W);
    for (int i = 0; i < L; ++i) {
        for (int j = 0; j < L; ++j) {
            double v = OINF;
            if (abs(i - j) <= w) {
                double m;
                if (i == 0 && j == 0) m = 0.0;
                else {
                    double dg = (i > 0 && j > 0) ? D[(i - 1) * L + j - 1] : OINF;
                    double up = i > 0 ? D[(i - 1) * L + j] : OINF;
                    double lf = j > 0 ? D[i * L + j - 1] : OINF;
                    m = dmin(dmin(dg, up), lf);
                }
                v = delta(A[i], B[j]) + m;
            }
            D[i * L + j] = v;
        }
    }
    return D[L * L - 1];
}

/* The argmin path, (0,0) first; returns its number of cells (<= 2L-1). */
static int backtrack(const double *D, int L, int *pi, int *pj)
{
    int i = L - 1, j = L - 1, n = 0;
    int ri[4096], rj[4096];
    for (;;) {
        ri[n] = i;
        rj[n] = j;
        ++n;
        if (i == 0 && j == 0) break;
        double dg = (i > 0 && j > 0) ? D[(i - 1) * L + j - 1] : OINF;
        double up = i > 0 ? D[(i - 1) * L + j] : OINF;
        double lf = j > 0 ? D[i * L + j - 1] : OINF;
        double m = dmin(dmin(dg, up), lf);
        if (dg == m) { --i; --j; }
        else if (up == m) { --i; }
        else { --j; }
    }
    for (int k = 0; k < n; ++k) {
        pi[k] = ri[n - 1 - k];
        pj[k] = rj[n - 1 - k];
    }
    return n;
}

/* DTW_W(A, B) and its argmin path (capacity 2L-1 cells each in pi, pj). */
double oracle_dtw_path(const float *A, const float *B, int L, int W, int *pi, int *pj, int *len)
{
    double *D = (double *)malloc(sizeof(double) * (size_t)L * L);
    double d = dtw_full(A, B, L, W, D);
    *len = backtrack(D, L, pi, pj);
    free(D);
    return d;
}

/* gA[i] += g * dDTW_W(A, B)/dA_i along the argmin path; returns DTW_W. */
static double dtw_grad_add(const float *A, const float *B, int L, int W, double g, double *gA)
{
    int *pi = (int *)malloc(sizeof(int) * (size_t)(2 * L));
    int *pj = (int *)malloc(sizeof(int) * (size_t)(2 * L));
    int n = 0;
    double d = oracle_dtw_path(A, B, L, W, pi, pj, &n);
    for (int k = 0; k < n; ++k)
        gA[pi[k]] += g * (2.0 * ((double)A[pi[k]] - (double)B[pj[k]]));
    free(pi);
    free(pj);
    return d;
}

/* Batched: gA[a][i] = sum over the pairs (a, b) of gout[pair] * dDTW/dA_a[i]
 * (pairing 0 cross: pair a*nB + b; 1 zip: pair a, b = a); dist[pair] = DTW_W. */
void oracle_dtw_grad_batch(const float *A, int64_t nA, const float *B, int64_t nB, int L, int W,
                           int pairing, const double *gout, double *gA, double *dist)
{
#pragma omp parallel for schedule(dynamic)
    for (int64_t a = 0; a < nA; ++a) {
        double *g = gA + a * L;
        for (int i = 0; i < L; ++i) g[i] = 0.0;
        int64_t b0 = pairing ? a : 0, b1 = pairing ? a + 1 : nB;
        for (int64_t b = b0; b < b1; ++b) {
            int64_t p = pairing ? a : a * nB + b;
            double d = dtw_grad_add(A + a * L, B + b * L, L, W, gout[p], g);
            if (dist) dist[p] = d;
        }
    }
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
