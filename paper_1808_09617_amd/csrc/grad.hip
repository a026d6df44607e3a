// DTW_W backward: the gradient of DTW_W(A, B) (Equation 1) with respect to
// the query A along the minimising warping path.  The paper defines DTW_W but
// no gradient; where the minimising path P* is unique the cost is
// differentiable in A with
//     dDTW/dA_i = sum over the cells (i, j) of P* of 2 (A_i - B_j).
//
// Two kernels:
//   1. forward: the DTW engine without abandoning, recording for every band
//      cell which predecessor attains the minimum (first of (i-1,j-1),
//      (i-1,j), (i,j-1), the order that also resolves exact ties), one byte
//      per (super-step, diagonal pair) and series pair;
//   2. backtrack: from (L-1, L-1) the recorded predecessors lead back to
//      (0, 0); every cell adds gout * 2 (A_i - B_j) to the query's gradient.
//      One workgroup per query (cross pairing): its threads walk the paths of
//      different references and accumulate into an LDS row with atomics.
#include "dtw_engine.hpp"

namespace nndtw {

namespace {

// Codes geometry: the engine shape of the forward pass (LDS-staged rows) and
// the bytes per series pair (T rows of W'+1 pairs, rounded up to 16).
struct CodesGeom {
    EngineGeom g;
    int64_t pitch;
};

int codes_geom(int L, int W, CodesGeom *cg)
{
    const int Wp = W < L - 1 ? W : L - 1;
    const int C = choose_cpl(Wp, 16, 0);
    if (C < 0) return fail(NNDTW_EUNSUP, "window %d too wide for the DTW engine", W);
    cg->g = make_geom(L, W, C, prefetch_lds(C), window_lds(C));
    cg->pitch = ((int64_t)cg->g.T * (Wp + 1) + 15) / 16 * 16;
    return NNDTW_OK;
}

struct CodesAt {
    static constexpr bool on = true;
    uint8_t *base;
    int64_t pitch, first;
    __device__ uint8_t *operator()(int i) const { return base + (first + i) * pitch; }
};

}  // namespace

template <typename T, int C, bool EXACT>
__global__ void __launch_bounds__(WAVE)
dtw_codes_kernel(EngineGeom geo, int NB, const float *__restrict__ A, int64_t nA, const float *__restrict__ B,
                 int64_t nB, int pairing, T *__restrict__ out, uint8_t *__restrict__ codes, int64_t cpitch)
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
            [&](int i) { return (const T *)(bR + (size_t)i * LEN); }, [&](int) { return inf_of<T>(); },
            TaskOut<T>{res, trun}, CodesAt{codes, cpitch, base});
        __syncthreads();
        if (lane < nt) out[base + lane] = res[lane];
        __syncthreads();
    }
}

// Walk back one pair's path, calling add(i, j) for every cell from (L-1,L-1)
// to (0,0).  The bounds tests only guard memory against corrupt codes.
template <typename Add>
__device__ __forceinline__ void walk_path(const EngineGeom &geo, const uint8_t *__restrict__ codes, Add add)
{
    const int L = geo.L, Wp = geo.Wp;
    const int s_start = 2 * geo.base0 + Wp;
    int i = L - 1, j = L - 1;
    for (int step = 0; step < 2 * L - 1; ++step) {
        add(i, j);
        if (i == 0 && j == 0) break;
        const int k = i - j + Wp;                // 0 .. 2W'
        const int p = k >> 1, top = k & 1;
        const int t = (i + j - top - s_start) >> 1;
        if (t < 0 || t >= geo.T || p > Wp) break;
        const unsigned c = (codes[(int64_t)t * (Wp + 1) + p] >> (top ? 2 : 0)) & 3u;
        if (c == 0) { --i; --j; }
        else if (c == 1) { --i; }
        else { --j; }
        if (i < 0 || j < 0 || i - j > Wp || j - i > Wp) break;
    }
}

constexpr int BT_THREADS = 256;

// Cross pairing: one workgroup per query a, gA[a] = sum over b of
// gout[a][b] * dDTW(a, b)/dA_a.  Zip pairing: one thread per pair.
template <typename T>
__global__ void __launch_bounds__(BT_THREADS)
dtw_backtrack_kernel(EngineGeom geo, const float *__restrict__ A, int64_t nA, const float *__restrict__ B,
                     int64_t nB, int pairing, const T *__restrict__ gout, const uint8_t *__restrict__ codes,
                     int64_t cpitch, T *__restrict__ gA)
{
    const int L = geo.L;
    if (pairing) {
        const int64_t k = (int64_t)blockIdx.x * BT_THREADS + threadIdx.x;
        if (k >= nA) return;
        const float *a = A + k * L, *b = B + k * L;
        T *g = gA + k * L;
        for (int i = 0; i < L; ++i) g[i] = (T)0;
        const T w = gout[k];
        walk_path(geo, codes + k * cpitch, [&](int i, int j) { g[i] += w * ((T)2 * ((T)a[i] - (T)b[j])); });
        return;
    }
    extern __shared__ __align__(16) unsigned char smem[];
    T *acc = reinterpret_cast<T *>(smem);
    const int64_t q = blockIdx.x;
    const float *a = A + q * L;
    for (int i = threadIdx.x; i < L; i += BT_THREADS) acc[i] = (T)0;
    __syncthreads();
    for (int64_t r = threadIdx.x; r < nB; r += BT_THREADS) {
        const float *b = B + r * L;
        const T w = gout[q * nB + r];
        walk_path(geo, codes + (q * nB + r) * cpitch,
                  [&](int i, int j) { atomicAdd(&acc[i], w * ((T)2 * ((T)a[i] - (T)b[j]))); });
    }
    __syncthreads();
    for (int i = threadIdx.x; i < L; i += BT_THREADS) gA[q * L + i] = acc[i];
}

size_t dtw_codes_bytes(int64_t np, int L, int W)
{
    CodesGeom cg;
    if (codes_geom(L, W, &cg)) return 0;
    return (size_t)(np * cg.pitch);
}

static size_t codes_lds(const EngineGeom &g, int NB, size_t esz)
{
    return (size_t)2 * NB * g.LEN * esz + (size_t)NB * (esz + sizeof(int)) + 32;
}

template <typename T>
static int launch_codes_t(const float *A, int64_t nA, const float *B, int64_t nB, int L, int W, int pairing, T *out,
                          uint8_t *codes, hipStream_t st)
{
    const int64_t np = pairing ? nA : nA * nB;
    if (np == 0) return NNDTW_OK;
    CodesGeom cg;
    if (int r = codes_geom(L, W, &cg)) return r;
    EngineGeom g = cg.g;
    int NB = 2 * g.P < 64 ? 2 * g.P : 64;
    while (NB > 1 && codes_lds(g, NB, sizeof(T)) > 64 * 1024) --NB;
    if (NB < g.P) g.P = NB;
    const size_t lds = codes_lds(g, NB, sizeof(T));
    if (lds > 160 * 1024) return fail(NNDTW_EUNSUP, "series length %d too long for the DTW engine", L);
    int64_t blocks = ceil_div(np, NB);
    if (blocks > 256 * 16) blocks = 256 * 16;
    switch (g.C) {
#define X(c)                                                                                                  \
    case c:                                                                                                   \
        if (g.exact)                                                                                          \
            hipLaunchKernelGGL((dtw_codes_kernel<T, c, true>), dim3((unsigned)blocks), dim3(WAVE), lds, st, g, NB, \
                               A, nA, B, nB, pairing, out, codes, cg.pitch);                                  \
        else                                                                                                  \
            hipLaunchKernelGGL((dtw_codes_kernel<T, c, false>), dim3((unsigned)blocks), dim3(WAVE), lds, st, g, NB, \
                               A, nA, B, nB, pairing, out, codes, cg.pitch);                                  \
        break;
        X(1) X(2) X(3) X(4) X(6) X(8) X(9) X(12) X(16)
#undef X
    default:
        return fail(NNDTW_EUNSUP, "no DTW engine for %d pairs per lane", g.C);
    }
    NNDTW_LAUNCH_CHECK("dtw codes kernel launch");
    return NNDTW_OK;
}

int launch_dtw_codes(bool f64, const float *A, int64_t nA, const float *B, int64_t nB, int L, int W, int pairing,
                     void *out, uint8_t *codes, hipStream_t st)
{
    if (f64) return launch_codes_t<double>(A, nA, B, nB, L, W, pairing, (double *)out, codes, st);
    return launch_codes_t<float>(A, nA, B, nB, L, W, pairing, (float *)out, codes, st);
}

int launch_dtw_backward(bool f64, const float *A, int64_t nA, const float *B, int64_t nB, int L, int W, int pairing,
                        const void *gout, const uint8_t *codes, void *gA, hipStream_t st)
{
    if (nA == 0 || (!pairing && nB == 0)) return NNDTW_OK;
    CodesGeom cg;
    if (int r = codes_geom(L, W, &cg)) return r;
    const unsigned blocks = (unsigned)(pairing ? ceil_div(nA, BT_THREADS) : nA);
    const size_t esz = f64 ? 8 : 4;
    const size_t lds = pairing ? 0 : (size_t)L * esz;
    if (f64)
        hipLaunchKernelGGL(dtw_backtrack_kernel<double>, dim3(blocks), dim3(BT_THREADS), lds, st, cg.g, A, nA, B, nB,
                           pairing, (const double *)gout, codes, cg.pitch, (double *)gA);
    else
        hipLaunchKernelGGL(dtw_backtrack_kernel<float>, dim3(blocks), dim3(BT_THREADS), lds, st, cg.g, A, nA, B, nB,
                           pairing, (const float *)gout, codes, cg.pitch, (float *)gA);
    NNDTW_LAUNCH_CHECK("dtw backtrack kernel launch");
    return NNDTW_OK;
}

}  // namespace nndtw
