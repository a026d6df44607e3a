// DTW_W backward: the gradient of DTW_W(A, B) (Equation 1) with respect to
// the query A along the minimising warping path.  The paper defines DTW_W but
// no gradient; where the minimising path P* is unique the cost is
// differentiable in A with
//     dDTW/dA_i = sum over the cells (i, j) of P* of 2 (A_i - B_j).
//
// Two kernels:
//   1. forward: the DTW engine of the search (rows streamed from padded
//      copies kept in the caller's code buffer) without abandoning, recording for every band
//      cell which predecessor attains the minimum (first of (i-1,j-1),
//      (i-1,j), (i,j-1), the order that also resolves exact ties), four bits
//      per (super-step, diagonal pair) and series pair, packed in 32-bit
//      words of 8 super-steps (one store per 8 super-steps and slot);
//   2. backtrack: from (L-1, L-1) the recorded predecessors lead back to
//      (0, 0); every cell adds gout * 2 (A_i - B_j) to the query's gradient.
//      One thread per pair sums its path's terms per row i (a path visits
//      the rows in order).  Cross pairing: the row sums are stored per pair
//      and a second kernel adds them per (query, i) in ascending reference
//      order, so the sums always run in the same order and the result is the
//      same from run to run.  Zip pairing: the row sums are the gradient.
#include <algorithm>

#include "dtw_engine.hpp"

namespace nndtw {

namespace {

// Forward geometry: the engine shape of the search (rows streamed from
// padded global copies, blocks of M super-steps rounded up to a multiple of
// 8 for whole code words) and the buffer layout: padded copies of A and B,
// then the code words, 32-bit words per series pair (T/8 rows of W'+1 pairs,
// rounded up to 4).
struct CodesGeom {
    EngineGeom g;
    int padl;
    int64_t ppitch;      // floats per padded row
    int64_t pitch;       // code words per series pair
    size_t offA, offB, offC, offP, total;
};

// Prefetch distance and block length (a multiple of 8): FP32 fills a block
// of 8 with prefetch for up to 6 pairs per lane; FP64 keeps the short
// prefetch (double windows cost two registers per value).
__host__ __device__ constexpr int codes_prefetch(bool f64, int C)
{
    return f64 ? prefetch_lds(C) : (C <= 6 ? 8 - C : prefetch_global(C));
}
__host__ __device__ constexpr int codes_window(bool f64, int C) { return (C + codes_prefetch(f64, C) + 7) / 8 * 8; }

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

int codes_geom(int64_t nA, int64_t nB, int L, int W, int pairing, bool f64, CodesGeom *cg)
{
    const int Wp = W < L - 1 ? W : L - 1;
    // FP64 cells need twice the registers: up to 9 pairs per lane (windows of
    // up to 567 diagonal pairs) fit without spilling to scratch memory, FP32
    // up to 12 (756)
    const int C = choose_cpl(Wp, 4, 0, f64 ? 9 : 12);
    if (C < 0) return fail(NNDTW_EUNSUP, "window %d too wide for the DTW engine", W);
    cg->g = make_geom(L, W, C, codes_prefetch(f64, C), codes_window(f64, C));
    if (cg->g.P < 1) return fail(NNDTW_EUNSUP, "window %d too wide for the DTW engine", W);
    // the code words cover every super-step from the first, in whole words
    cg->g.t0 = 0;
    cg->g.T = (int)ceil_div(cg->g.L + (cg->g.Wp + 2) / 2, cg->g.M) * cg->g.M;
    cg->g.LEN = cg->g.T + cg->g.Wp + 2 * C + cg->g.D + 2;
    cg->padl = padded_row_margin_left(Wp);
    cg->ppitch = ((int64_t)cg->padl + L + padded_row_margin_right(Wp) + 63) / 64 * 64;
    const int64_t boff = cg->padl + cg->g.base0 - C;
    if (boff < 0 || boff + cg->g.LEN > cg->ppitch)
        return fail(NNDTW_EUNSUP, "row margins too narrow for the DTW engine shape");
    cg->pitch = ((int64_t)(cg->g.T / 8) * (Wp + 1) + 3) / 4 * 4;
    const int64_t np = pairing ? nA : nA * nB;
    size_t o = 0;
    cg->offA = o; o = al256(o + (size_t)nA * cg->ppitch * 4);
    cg->offB = o; o = al256(o + (size_t)nB * cg->ppitch * 4);
    cg->offC = o; o = al256(o + (size_t)np * cg->pitch * 4);
    // cross backward: every pair's path sums per row, [nA][nB][L]
    cg->offP = o; o = al256(o + (pairing ? 0 : (size_t)np * L * (f64 ? 8 : 4)));
    cg->total = o;
    return NNDTW_OK;
}

struct CodesAt {
    static constexpr bool on = true;
    uint32_t *base;
    int64_t pitch, first;
    __device__ uint32_t *operator()(int i) const { return base + (first + i) * pitch; }
};

constexpr int CODES_WAVES = 4;

}  // namespace

// One workgroup of CODES_WAVES waves per K consecutive series pairs: the
// rows of both series are read from their padded copies (L2-resident), the
// pairs are dealt to the groups of all waves from an LDS counter, and every
// band cell's predecessor code is written to the pair's code words.
template <typename T, int C, bool EXACT>
__global__ void __launch_bounds__(WAVE * CODES_WAVES)
dtw_codes_kernel(EngineGeom geo, int K, int64_t np, int64_t nB, int pairing, const float *__restrict__ Ap,
                 const float *__restrict__ Bp, int64_t ppitch, int padl, T *__restrict__ out,
                 uint32_t *__restrict__ codes, int64_t cpitch)
{
    extern __shared__ __align__(16) unsigned char smem[];
    T *res = reinterpret_cast<T *>(smem);
    int *trun = reinterpret_cast<int *>(res + K);
    int *next_task = trun + K;
    const int64_t p0 = (int64_t)blockIdx.x * K;
    const int nt = (int)((np - p0) < K ? (np - p0) : K);
    // element e of a row the engine sees is series index base0 - PADL + e
    const int64_t off = padl + geo.base0 - Stage<C>::PADL;
    if (threadIdx.x == 0) *next_task = 0;
    __syncthreads();
    constexpr bool F64 = sizeof(T) == 8;
    engine_run<T, C, codes_prefetch(F64, C), codes_window(F64, C), EXACT>(
        geo, nt, next_task,
        [&](int i) {
            const int64_t p = p0 + i;
            return Ap + (pairing ? p : p / nB) * ppitch + off;
        },
        [&](int i) {
            const int64_t p = p0 + i;
            return Bp + (pairing ? p : p % nB) * ppitch + off;
        },
        [&](int) { return inf_of<T>(); }, TaskOut<T>{res, trun}, CodesAt{codes, cpitch, p0});
    __syncthreads();
    for (int i = threadIdx.x; i < nt; i += blockDim.x) out[p0 + i] = res[i];
}

// Walk back one pair's path, calling add(i, j) for every cell from (L-1,L-1)
// to (0,0) (i never increases).  The bounds tests only guard memory against
// corrupt codes.
template <typename Add>
__device__ __forceinline__ void walk_path(const EngineGeom &geo, const uint32_t *__restrict__ codes, Add add)
{
    const int L = geo.L, Wp = geo.Wp;
    const int s_start = 2 * geo.base0 + Wp;
    int i = L - 1, j = L - 1;
    int64_t widx = -1;                           // index of the code word held in `word`
    uint32_t word = 0u;
    for (int step = 0; step < 2 * L - 1; ++step) {
        add(i, j);
        if (i == 0 && j == 0) break;
        const int k = i - j + Wp;                // 0 .. 2W'
        const int p = k >> 1, top = k & 1;
        const int t = (i + j - top - s_start) >> 1;
        if (t < 0 || t >= geo.T || p > Wp) break;
        // consecutive steps mostly stay in one word (8 super-steps of a pair)
        const int64_t wi = (int64_t)(t >> 3) * (Wp + 1) + p;
        if (wi != widx) {
            widx = wi;
            word = codes[wi];
        }
        // the cell's two bits: bit 1 (i-1, j-1) above the smaller of the
        // other two predecessors, bit 0 (i-1, j) above (i, j-1)
        const unsigned nib = (word >> (28 - 4 * (t & 7))) & 0xFu;
        const unsigned c = top ? (nib & 3u) : (nib >> 2);
        if ((c & 2u) == 0u) { --i; --j; }
        else if ((c & 1u) == 0u) { --i; }
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
                     int64_t nB, int pairing, const T *__restrict__ gout, const uint32_t *__restrict__ codes,
                     int64_t cpitch, T *__restrict__ gA, T *__restrict__ rowsums)
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
    // cross pairing: one thread per (query, reference) pair sums its path's
    // terms per row i (a path visits the rows in order) and stores the row
    // sums rs[q][r][i]; the combine kernel adds them in reference order
    // (stored as rs[q][i][r]: the threads of a wave, walking neighbouring
    // references' paths at about the same row, store to neighbouring words)
    const int64_t p = (int64_t)blockIdx.x * BT_THREADS + threadIdx.x;
    if (p >= nA * nB) return;
    const int64_t q = p / nB, r = p - q * nB;
    const float *a = A + q * L, *b = B + r * L;
    const T w = gout[p];
    T *col = rowsums + q * L * nB + r;
    int cur = L - 1;
    T sum = (T)0;
    walk_path(geo, codes + p * cpitch, [&](int i, int j) {
        if (i != cur) {
            col[(int64_t)cur * nB] = sum;
            cur = i;
            sum = (T)0;
        }
        sum += w * ((T)2 * ((T)a[i] - (T)b[j]));
    });
    col[(int64_t)cur * nB] = sum;
}

// gA[q][i] = the pairs' row sums rs[q][i][r] added in ascending reference order.
template <typename T>
__global__ void __launch_bounds__(256)
dtw_backward_combine_kernel(int64_t nA, int64_t nB, int L, const T *__restrict__ rowsums, T *__restrict__ gA)
{
    const int64_t total = nA * L;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const T *src = rowsums + e * nB;       // rs[q][i][0 .. nB-1]
        T s = (T)0;
        for (int64_t r = 0; r < nB; ++r) s += src[r];
        gA[e] = s;
    }
}

size_t dtw_codes_bytes(int64_t nA, int64_t nB, int L, int W, int pairing)
{
    // the larger of the two precisions' layouts (they differ in T only); a
    // window wider than the FP64 kernels take is sized for FP32 (the FP64
    // calls return EUNSUP for it)
    CodesGeom cg, cd;
    if (codes_geom(nA, nB, L, W, pairing, false, &cg)) return 0;
    if (codes_geom(nA, nB, L, W, pairing, true, &cd)) return cg.total;
    return cg.total > cd.total ? cg.total : cd.total;
}


template <typename T>
static int launch_codes_t(const float *A, int64_t nA, const float *B, int64_t nB, int L, int W, int pairing, T *out,
                          uint8_t *buf, hipStream_t st)
{
    const int64_t np = pairing ? nA : nA * nB;
    if (np == 0) return NNDTW_OK;
    CodesGeom cg;
    if (int r = codes_geom(nA, nB, L, W, pairing, sizeof(T) == 8, &cg)) return r;
    const EngineGeom &g = cg.g;
    float *Ap = (float *)(buf + cg.offA), *Bp = (float *)(buf + cg.offB);
    uint32_t *codes = (uint32_t *)(buf + cg.offC);
    if (int r = launch_pad_rows(A, nA, L, cg.padl, cg.ppitch, Ap, st)) return r;
    if (int r = launch_pad_rows(B, nB, L, cg.padl, cg.ppitch, Bp, st)) return r;
    // two tasks per group of every wave: all pairs cost the same
    const int K = 2 * g.P * CODES_WAVES;
    const size_t lds = (size_t)K * (sizeof(T) + sizeof(int)) + 16;
    const unsigned blocks = (unsigned)ceil_div(np, K);
    switch (g.C * 2 + (g.exact ? 1 : 0)) {
#define X(c)                                                                                                   \
    case c * 2 + 1:                                                                                            \
        hipLaunchKernelGGL((dtw_codes_kernel<T, c, true>), dim3(blocks), dim3(WAVE * CODES_WAVES), lds, st, g, K, \
                           np, nB, pairing, Ap, Bp, cg.ppitch, cg.padl, out, codes, cg.pitch);                 \
        break;                                                                                                 \
    case c * 2:                                                                                                \
        hipLaunchKernelGGL((dtw_codes_kernel<T, c, false>), dim3(blocks), dim3(WAVE * CODES_WAVES), lds, st, g, K, \
                           np, nB, pairing, Ap, Bp, cg.ppitch, cg.padl, out, codes, cg.pitch);                 \
        break;
        X(1) X(2) X(3) X(4) X(6) X(8) X(9)
#undef X
    case 12 * 2 + 1:
        if (sizeof(T) == 8) return fail(NNDTW_EUNSUP, "FP64 codes: no engine for 12 pairs per lane");
        hipLaunchKernelGGL((dtw_codes_kernel<float, 12, true>), dim3(blocks), dim3(WAVE * CODES_WAVES), lds, st, g,
                           K, np, nB, pairing, Ap, Bp, cg.ppitch, cg.padl, (float *)out, codes, cg.pitch);
        break;
    case 12 * 2:
        if (sizeof(T) == 8) return fail(NNDTW_EUNSUP, "FP64 codes: no engine for 12 pairs per lane");
        hipLaunchKernelGGL((dtw_codes_kernel<float, 12, false>), dim3(blocks), dim3(WAVE * CODES_WAVES), lds, st, g,
                           K, np, nB, pairing, Ap, Bp, cg.ppitch, cg.padl, (float *)out, codes, cg.pitch);
        break;
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
    if (int r = codes_geom(nA, nB, L, W, pairing, f64, &cg)) return r;
    const uint32_t *cw = (const uint32_t *)(codes + cg.offC);
    const int64_t np = pairing ? nA : nA * nB;
    if (ceil_div(np, BT_THREADS) > 0x7FFFFFFFLL) return fail(NNDTW_EUNSUP, "backward: too many series pairs");
    const unsigned blocks = (unsigned)ceil_div(np, BT_THREADS);
    uint8_t *rs = const_cast<uint8_t *>(codes) + cg.offP;
    if (f64)
        hipLaunchKernelGGL(dtw_backtrack_kernel<double>, dim3(blocks), dim3(BT_THREADS), 0, st, cg.g, A, nA, B, nB,
                           pairing, (const double *)gout, cw, cg.pitch, (double *)gA, (double *)rs);
    else
        hipLaunchKernelGGL(dtw_backtrack_kernel<float>, dim3(blocks), dim3(BT_THREADS), 0, st, cg.g, A, nA, B, nB,
                           pairing, (const float *)gout, cw, cg.pitch, (float *)gA, (float *)rs);
    NNDTW_LAUNCH_CHECK("dtw backtrack kernel launch");
    if (!pairing) {
        const int64_t cb = std::min<int64_t>(ceil_div((int64_t)nA * L, 256), 65536);
        if (f64)
            hipLaunchKernelGGL(dtw_backward_combine_kernel<double>, dim3((unsigned)cb), dim3(256), 0, st, nA, nB, L,
                               (const double *)rs, (double *)gA);
        else
            hipLaunchKernelGGL(dtw_backward_combine_kernel<float>, dim3((unsigned)cb), dim3(256), 0, st, nA, nB, L,
                               (const float *)rs, (float *)gA);
        NNDTW_LAUNCH_CHECK("dtw backward combine kernel launch");
    }
    return NNDTW_OK;
}

}  // namespace nndtw
