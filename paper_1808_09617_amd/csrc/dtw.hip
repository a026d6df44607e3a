// DTW_W over (A, B) pairs with the anti-diagonal engine, FP32 or FP64, and
// the engine geometry helpers shared with the search.
#include "strip_engine.hpp"

namespace nndtw {

// Diagonal pairs per lane that the kernels are instantiated for.
#define NNDTW_FOR_EACH_CPL(X) X(1) X(2) X(3) X(4) X(6) X(8) X(9) X(12) X(16)

bool cpl_supported(int C)
{
    switch (C) {
#define X(c) case c:
        NNDTW_FOR_EACH_CPL(X)
#undef X
        return true;
    default:
        return false;
    }
}

// Modelled VALU efficiency of a shape: lanes in use times useful operations
// per cell (3: sub, min3, fma) over issued ones.
static double cpl_score(int Wp, int C)
{
    const int G = (int)ceil_div(Wp + 1, C);
    if (G > 63) return -1.0;
    const bool exact = G * C == Wp + 1;
    const int P = 63 / G;
    const double ops = exact ? 3.0 + 1.5 / C : 3.5 + 1.0 / C;
    return (double)(P * G) / 64.0 * 3.0 / ops;
}

int choose_cpl(int Wp, int cmax, int prefer, int chard, bool widen_single)
{
    if (prefer > 0)
        return (cpl_supported(prefer) && prefer <= chard && cpl_score(Wp, prefer) > 0) ? prefer : -1;
    int best = -1;
    double bs = -1.0;
    const int cands[] = {1, 2, 3, 4, 6, 8, 9, 12, 16};
    // Shapes up to cmax pairs per lane first (fewer registers, more waves
    // per SIMD); the larger ones if none fits, or, with widen_single, if the
    // best of them leaves one group per wave (most lanes idle).
    auto single = [&](int C) { return C > 0 && 63 / (int)ceil_div(Wp + 1, C) < 2; };
    for (int pass = 0; pass < 2 && (best < 0 || (widen_single && single(best))); ++pass) {
        for (int C : cands) {
            if (C > chard || (pass == 0 && C > cmax)) continue;
            double s = cpl_score(Wp, C);
            if (s <= 0.0) continue;  // a group wider than the wave: no shape
            if (s > bs * 1.02) {     // a larger C must pay for its latency
                bs = s;
                best = C;
            }
        }
    }
    return best;
}

EngineGeom make_geom(int L, int W, int C, int D, int M)
{
    EngineGeom g;
    g.L = L;
    g.Wp = W < L - 1 ? W : L - 1;
    g.C = C;
    g.G = (int)ceil_div(g.Wp + 1, C);
    g.exact = g.G * C == g.Wp + 1;
    g.P = 63 / g.G;
    g.D = D;
    g.M = M;
    // The sweep is numbered from the first anti-diagonal pair outside the
    // matrix and reaches (L-1, L-1) after T0 super-steps.  Its first
    // (W'+2)/2 super-steps lie wholly before the matrix, where a cell costs 0
    // with both indices in the padding and +inf with one: a task starts at
    // t0 = (W'+2)/2 with that state loaded directly (see engine_run) and runs
    // whole blocks of M super-steps, so T = t0 + ceil((T0 - t0) / M) * M.
    // The super-steps after T0 run past the end: both series are padded there
    // with the same value, so every later cell of diagonal 0 keeps DTW_W
    // exactly (a pad pair costs 0, a pad against a value costs +inf); a DTW
    // that is abandoned never reaches them.
    const int T0 = L + (g.Wp + 2) / 2;
    g.t0 = (g.Wp + 2) / 2;
    g.T = g.t0 + (int)ceil_div(T0 - g.t0, M) * M;
    g.base0 = -g.Wp - 1;
    g.LEN = g.T + g.Wp + 2 * C + D + 2;
    return g;
}

template <typename T, int C, bool EXACT>
__global__ void __launch_bounds__(WAVE)
dtw_pairs_kernel(EngineGeom geo, int NB, const float *__restrict__ A, int64_t nA,
                 const float *__restrict__ B, int64_t nB, const double *__restrict__ cutoff,
                 int pairing, T *__restrict__ out)
{
    extern __shared__ __align__(16) unsigned char smem[];
    T *aR = reinterpret_cast<T *>(smem);
    T *bR = aR + (size_t)NB * geo.LEN;
    T *res = bR + (size_t)NB * geo.LEN;
    int *trun = reinterpret_cast<int *>(res + NB);
    int *next_task = trun + NB;
    const int lane = threadIdx.x;
    const int LEN = geo.LEN;
    const int64_t np = pairing ? nA : nA * nB;
    for (int64_t base = (int64_t)blockIdx.x * NB; base < np; base += (int64_t)gridDim.x * NB) {
        const int nt = (int)((np - base) < NB ? (np - base) : NB);
        stage_rows<T, C>(aR, A, [&](int i) { const int64_t p = base + i; return pairing ? p : p / nB; }, nt, geo,
                         lane);
        stage_rows<T, C>(bR, B, [&](int i) { const int64_t p = base + i; return pairing ? p : p % nB; }, nt, geo,
                         lane);
        if (lane == 0) *next_task = 0;
        __syncthreads();
        engine_run<T, C, prefetch_lds(C), window_lds(C), EXACT>(
            geo, nt, next_task, [&](int i) { return (const T *)(aR + (size_t)i * LEN); },
            [&](int i) { return (const T *)(bR + (size_t)i * LEN); },
            [&](int i) -> T {
                if (!cutoff) return inf_of<T>();
                const int64_t p = base + i;
                const double c = cutoff[pairing ? p : p / nB];
                return sizeof(T) == 4 ? (T)round_up_f32(c) : (T)c;
            },
            TaskOut<T>{res, trun});
        __syncthreads();
        if (lane < nt) out[base + lane] = res[lane];
        __syncthreads();
    }
}

// Pairs with the row-strip engine (wide windows): one pair per wave at a
// time, rows read from global memory (L2-resident), batches of sb <= STRIP_SB
// pairs per workgroup in a grid-stride loop.
constexpr int STRIP_WAVES = 4, STRIP_SB = 64;

template <typename T, int S, bool WIN>
__global__ void __launch_bounds__(WAVE * STRIP_WAVES)
dtw_strip_kernel(int L, int Wp, const float *__restrict__ A, int64_t nA, const float *__restrict__ B, int64_t nB,
                 const double *__restrict__ cutoff, int pairing, int sb, T *__restrict__ out)
{
    __shared__ int next_task;
    __shared__ int cells[STRIP_SB];
    const int64_t np = pairing ? nA : nA * nB;
    for (int64_t base = (int64_t)blockIdx.x * sb; base < np; base += (int64_t)gridDim.x * sb) {
        const int nt = (int)((np - base) < sb ? (np - base) : sb);
        __syncthreads();
        if (threadIdx.x == 0) next_task = 0;
        __syncthreads();
        strip_run<T, S, WIN>(
            L, Wp, nt, &next_task,
            [&](int i) {
                const int64_t p = base + i;
                return A + (pairing ? p : p / nB) * L;
            },
            [&](int i) {
                const int64_t p = base + i;
                return B + (pairing ? p : p % nB) * L;
            },
            [&](int i) -> T {
                if (!cutoff) return inf_of<T>();
                const int64_t p = base + i;
                const double c = cutoff[pairing ? p : p / nB];
                return sizeof(T) == 4 ? (T)round_up_f32(c) : (T)c;
            },
            out + base, cells);
    }
}

// Band cells of an L x L matrix within |i - j| <= Wp.
static int64_t band_cells(int L, int Wp) { return (int64_t)L * (2 * Wp + 1) - (int64_t)Wp * (Wp + 1); }

// Whether the row-strip engine serves window W' at length L: windows the
// diagonal-pair engine cannot hold (more than 63 x 16 pairs), and windows
// covering at least 60 % of the matrix, where the pair sweep's parallelogram
// wastes more than the strips' pipeline fill.
bool strip_preferred(int L, int Wp)
{
    if (!strip_fits(L, Wp)) return false;
    return Wp + 1 > 63 * 16 || (double)band_cells(L, Wp) >= 0.6 * (double)L * (double)L;
}

template <typename T>
static int launch_strip_t(const float *A, int64_t nA, const float *B, int64_t nB, int L, int Wp,
                          const double *cutoff, int pairing, T *out, hipStream_t st)
{
    const int64_t np = pairing ? nA : nA * nB;
    // pairs per workgroup batch: one per wave while that leaves fewer than
    // about 2048 workgroups (every wave of the chip busy), up to STRIP_SB
    int64_t sb = ceil_div(np, 256 * 8);
    sb = sb < STRIP_WAVES ? STRIP_WAVES : (sb > STRIP_SB ? STRIP_SB : sb);
    int64_t blocks = ceil_div(np, sb);
    if (blocks > 256 * 8) blocks = 256 * 8;
    const bool win = Wp < L - 1;
    switch (strip_width(L) * 2 + (win ? 1 : 0)) {
#define X(s)                                                                                                   \
    case s * 2:                                                                                                \
        hipLaunchKernelGGL((dtw_strip_kernel<T, s, false>), dim3((unsigned)blocks), dim3(WAVE * STRIP_WAVES), 0, st, \
                           L, Wp, A, nA, B, nB, cutoff, pairing, (int)sb, out);                                        \
        break;                                                                                                 \
    case s * 2 + 1:                                                                                            \
        hipLaunchKernelGGL((dtw_strip_kernel<T, s, true>), dim3((unsigned)blocks), dim3(WAVE * STRIP_WAVES), 0, st,  \
                           L, Wp, A, nA, B, nB, cutoff, pairing, (int)sb, out);                                        \
        break;
        X(4) X(8) X(12) X(16) X(24) X(32)
#undef X
    default:
        return fail(NNDTW_EUNSUP, "series length %d too long for the row-strip engine", L);
    }
    NNDTW_LAUNCH_CHECK("dtw strip kernel launch");
    return NNDTW_OK;
}

static size_t pairs_lds(const EngineGeom &g, int NB, size_t esz)
{
    return (size_t)2 * NB * g.LEN * esz + (size_t)NB * (esz + sizeof(int)) + 32;
}

template <typename T>
static int launch_pairs_t(const float *A, int64_t nA, const float *B, int64_t nB, int L, int W,
                          const double *cutoff, int pairing, T *out, hipStream_t st)
{
    const int64_t np = pairing ? nA : nA * nB;
    if (np == 0) return NNDTW_OK;
    const int Wp = W < L - 1 ? W : L - 1;
    if (strip_preferred(L, Wp)) return launch_strip_t<T>(A, nA, B, nB, L, Wp, cutoff, pairing, out, st);
    const int C = choose_cpl(Wp, 16, 0);
    if (C < 0) return fail(NNDTW_EUNSUP, "window %d too wide for the DTW engine", W);
    EngineGeom g = make_geom(L, W, C, prefetch_lds(C), window_lds(C));
    if (g.P < 1) return fail(NNDTW_EUNSUP, "window %d too wide for the DTW engine", W);
    // Tasks staged per batch: two per group so that groups refill, within
    // 64 KB of LDS (at least one).
    int NB = 2 * g.P < 64 ? 2 * g.P : 64;
    while (NB > 1 && pairs_lds(g, NB, sizeof(T)) > 64 * 1024) --NB;
    if (NB < g.P) g.P = NB;
    const size_t lds = pairs_lds(g, NB, sizeof(T));
    if (lds > 160 * 1024) return fail(NNDTW_EUNSUP, "series length %d too long for the DTW engine", L);
    int64_t blocks = ceil_div(np, NB);
    if (blocks > 256 * 16) blocks = 256 * 16;
    switch (C) {
#define X(c)                                                                                       \
    case c:                                                                                        \
        if (g.exact)                                                                               \
            hipLaunchKernelGGL((dtw_pairs_kernel<T, c, true>), dim3((unsigned)blocks), dim3(WAVE), lds, \
                               st, g, NB, A, nA, B, nB, cutoff, pairing, out);                     \
        else                                                                                       \
            hipLaunchKernelGGL((dtw_pairs_kernel<T, c, false>), dim3((unsigned)blocks), dim3(WAVE), lds, \
                               st, g, NB, A, nA, B, nB, cutoff, pairing, out);                     \
        break;
        NNDTW_FOR_EACH_CPL(X)
#undef X
    default:
        return fail(NNDTW_EUNSUP, "no DTW engine for %d pairs per lane", C);
    }
    NNDTW_LAUNCH_CHECK("dtw kernel launch");
    return NNDTW_OK;
}

int launch_dtw_pairs(bool f64, const float *A, int64_t nA, const float *B, int64_t nB, int L, int W,
                     const double *cutoff, int pairing, void *out, hipStream_t st)
{
    if (f64) return launch_pairs_t<double>(A, nA, B, nB, L, W, cutoff, pairing, (double *)out, st);
    return launch_pairs_t<float>(A, nA, B, nB, L, W, cutoff, pairing, (float *)out, st);
}

}  // namespace nndtw
