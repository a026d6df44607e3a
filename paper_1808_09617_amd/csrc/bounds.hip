// Lower bounds of Sections 2.2 and 3 and the visiting-order key of Section 4,
// all in FP64 from float32 inputs, each sum accumulated in ascending point
// order so that the values are reproducible bit for bit.
//
//  * squared Euclidean distance  sum_i (A_i - B_i)^2
//  * LB_Keogh                    sum_i dist(A_i, [Lo_i, U_i])^2
//  * LB_Enhanced^V (Algorithm 1) corner costs, then per band index the left
//    band minimum and its mirror at (L, L), then the Keogh terms of the
//    middle points.
//
// Two kernels: a generic one over (A, B) pairs in row-major layout (one
// thread per pair, rows staged through LDS in coalesced chunks), and the
// fused pass of the search over a reference set,
// where lanes index references and read the point-major copies (coalesced),
// each thread carrying TQ queries so every reference value loaded from memory
// is reused TQ times.  The query values are staged in LDS as doubles.
#include "bounds_core.hpp"

namespace nndtw {

enum { PB_ED2 = 0, PB_KEOGH = 1, PB_ENH = 2 };

// Generic pairs: a workgroup of PB_THREADS threads takes PB_THREADS
// consecutive pairs, one per thread.  Rows are read in chunks of PB_CH
// points: the workgroup loads the chunk of every pair's rows with
// consecutive threads on consecutive points (64-byte row segments) into LDS,
// then each thread adds its pair's terms from LDS in ascending point order,
// as a sequential evaluation would.
constexpr int PB_THREADS = 256;
constexpr int PB_CH = 16;
constexpr int PB_PITCH = PB_CH + 1;      // odd pitch: a thread's row reads hit distinct banks

__global__ void __launch_bounds__(PB_THREADS)
pair_bounds_kernel(int what, const float *__restrict__ A, int64_t nA, const float *__restrict__ B,
                   const float *__restrict__ U, const float *__restrict__ Lo, int64_t nB, int L, int W,
                   int nb, const double *__restrict__ cutoff, int pairing, double *__restrict__ out)
{
    __shared__ float ta[PB_THREADS * PB_PITCH], t1[PB_THREADS * PB_PITCH], t2[PB_THREADS * PB_PITCH];
    const int64_t np = pairing ? nA : nA * nB;
    const int t = threadIdx.x;
    for (int64_t p0 = (int64_t)blockIdx.x * PB_THREADS; p0 < np; p0 += (int64_t)gridDim.x * PB_THREADS) {
        const int64_t p = p0 + t;
        const bool live = p < np;
        const int64_t ia = live ? (pairing ? p : p / nB) : 0, ib = live ? (pairing ? p : p % nB) : 0;
        const float *a = A + ia * L;
        // middle points of LB_Enhanced (its bands part is computed first)
        int lo = 0, hi = L;
        double s = 0.0;
        bool skip = false;
        if (what == PB_ENH) {
            lo = nb;
            hi = L - nb;
            if (live) {
                const float *b = B + ib * L;
                s = enh_bands([&](int i) { return a[i]; }, [&](int j) { return b[j]; }, L, W, nb);
                skip = cutoff && s > cutoff[ia];
            }
        }
        // the second and third arrays: B (squared ED) or the envelopes U, Lo
        const float *X1 = what == PB_ED2 ? B : U, *X2 = Lo;
        for (int c0 = 0; c0 < L; c0 += PB_CH) {
            const int cn = (L - c0) < PB_CH ? (L - c0) : PB_CH;
            __syncthreads();
            for (int e = t; e < PB_THREADS * PB_CH; e += PB_THREADS) {
                const int r = e / PB_CH, x = e % PB_CH;
                const int64_t q = p0 + r;
                if (q < np && x < cn) {
                    const int64_t qa = pairing ? q : q / nB, qb = pairing ? q : q % nB;
                    ta[r * PB_PITCH + x] = A[qa * L + c0 + x];
                    t1[r * PB_PITCH + x] = X1[qb * L + c0 + x];
                    if (what != PB_ED2) t2[r * PB_PITCH + x] = X2[qb * L + c0 + x];
                }
            }
            __syncthreads();
            if (!live) continue;
            const float *ra = ta + t * PB_PITCH, *r1 = t1 + t * PB_PITCH, *r2 = t2 + t * PB_PITCH;
            for (int x = 0; x < cn; ++x) {
                const int i = c0 + x;
                if (i < lo || i >= hi) continue;
                s += what == PB_ED2 ? sqd(ra[x], r1[x]) : keogh_term(ra[x], r1[x], r2[x]);
            }
        }
        if (live) out[p] = skip ? __builtin_inf() : s;
    }
}

int launch_pair_bounds(int what, const float *A, int64_t nA, const float *B, const float *U,
                       const float *Lo, int64_t nB, int L, int W, int V, const double *cutoff,
                       int pairing, double *out, hipStream_t st)
{
    const int64_t np = pairing ? nA : nA * nB;
    if (np == 0) return NNDTW_OK;
    const int nb = V < L / 2 ? V : L / 2;
    const int64_t blocks = ceil_div(np, PB_THREADS) < 65536 ? ceil_div(np, PB_THREADS) : 65536;
    hipLaunchKernelGGL(pair_bounds_kernel, dim3((unsigned)blocks), dim3(PB_THREADS), 0, st, what, A, nA, B, U,
                       Lo, nB, L, W, nb, cutoff, pairing, out);
    NNDTW_LAUNCH_CHECK("bounds kernel launch");
    return NNDTW_OK;
}

// ------------------------------------------------------------------ fused
constexpr int CB_THREADS = 256;
// Word 3 of a raw buffer resource on CDNA: 32-bit data format, no swizzle.
constexpr int BUF_DWORD3 = 0x00020000;
constexpr int CB_CHUNK = 128;   // points of the query tile staged per pass

// One tile: references rt*CB_THREADS .. +CB_THREADS-1 (one per thread)
// against queries qt*TQ .. qt*TQ+TQ-1.  Whole-workgroup call.
template <int TQ>
__device__ __forceinline__ void bounds_tile(int64_t rt, int64_t qt, const float *__restrict__ Bt,
                                            const float *__restrict__ Ut, const float *__restrict__ Lt,
                                            int64_t pitch, int64_t n, const float *__restrict__ Q, int64_t nQ,
                                            int L, int W, int nb, double *__restrict__ ed2,
                                            double *__restrict__ lbk, double *__restrict__ lbeb,
                                            double *__restrict__ lbe, int rot_phase)
{
    __shared__ double qa[CB_CHUNK][TQ];
    const int64_t k = rt * CB_THREADS + threadIdx.x;
    const int64_t q0 = qt * TQ;
    const bool live = k < n;
    const int64_t kk = live ? k : 0;
    const uint32_t kbytes = (uint32_t)kk * 4u;   // k < pitch < 2^29
    const int nq = (int)((nQ - q0) < TQ ? (nQ - q0) : TQ);

    double e[TQ], kg[TQ], en[TQ];
#pragma unroll
    for (int t = 0; t < TQ; ++t) {
        e[t] = 0.0;
        kg[t] = 0.0;
        en[t] = 0.0;
        if (t < nq) {
            const float *a = Q + (q0 + t) * L;
            en[t] = enh_bands([&](int i) { return a[i]; },
                              [&](int j) { return Bt[(int64_t)j * pitch + kk]; }, L, W, nb);
        }
    }
    const double *lbebv = en;   // bands part, kept before the middle terms are added
    double band[TQ];
#pragma unroll
    for (int t = 0; t < TQ; ++t) band[t] = lbebv[t];

    for (int c0 = 0; c0 < L; c0 += CB_CHUNK) {
        const int cn = (L - c0) < CB_CHUNK ? (L - c0) : CB_CHUNK;
        __syncthreads();
        for (int x = threadIdx.x; x < CB_CHUNK * TQ; x += CB_THREADS) {
            const int i = x / TQ, t = x % TQ;
            qa[i][t] = (i < cn && t < nq) ? (double)Q[(q0 + t) * L + c0 + i] : 0.0;
        }
        __syncthreads();
        // Middle points [nb, L - nb) also add their Keogh term to LB_Enhanced:
        // en = fma(kt, m, en) with m = 1 there rounds exactly like en + kt,
        // and with m = 0 leaves en unchanged, so the loop needs no branch.
        auto point = [&](int x, double b, double u, double lo) {
            const int i = c0 + x;
            const double m = (i >= nb && i < L - nb) ? 1.0 : 0.0;
#pragma unroll
            for (int t = 0; t < TQ; ++t) {
                const double a = qa[x][t];
                const double d = a - b;
                e[t] += d * d;
                const double kt = keogh_term(a, u, lo);
                kg[t] += kt;
                en[t] = __builtin_fma(kt, m, en[t]);
            }
        };
        // The reference values of point x + PF are loaded while point x is
        // processed (a ring of PF registers per array); loads past the chunk
        // re-read its last point, so every address stays in bounds.
        // Each point's row is read through a buffer resource built from the
        // wave-uniform row address (scalar work) and the lane's 32-bit byte
        // offset, so no per-load vector address arithmetic is needed.  The
        // resource covers the row (pitch floats); every offset is inside it.
        constexpr int PF = 8;
        float rb[PF], ru[PF], rl[PF];
        const int row_bytes = (int)(pitch * 4);
        auto at = [&](const float *rowp) {
            const __amdgpu_buffer_rsrc_t r =
                __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(rowp), 0, row_bytes, BUF_DWORD3);
            return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)kbytes, 0, 0));
        };
        auto fetch = [&](int x, int r) {
            const int64_t row = (int64_t)(c0 + (x < cn ? x : cn - 1)) * pitch;
            rb[r] = at(Bt + row);
            ru[r] = at(Ut + row);
            rl[r] = at(Lt + row);
        };
        const int cfull = cn - cn % PF;
#pragma unroll
        for (int r = 0; r < PF; ++r) fetch(r, r);
        for (int x0 = 0; x0 < cfull; x0 += PF) {
            if (rot_phase >= 0) rotate_priority(rot_phase);
#pragma unroll
            for (int r = 0; r < PF; ++r) {
                const double b = (double)rb[r], u = (double)ru[r], lo = (double)rl[r];
                fetch(x0 + r + PF, r);
                point(x0 + r, b, u, lo);
            }
        }
        for (int x = cfull; x < cn; ++x) {
            const int64_t o = (int64_t)(c0 + x) * pitch + kk;
            point(x, (double)Bt[o], (double)Ut[o], (double)Lt[o]);
        }
    }
    if (!live) return;
#pragma unroll
    for (int t = 0; t < TQ; ++t) {
        if (t < nq) {
            const int64_t o = (q0 + t) * n + k;
            if (ed2) ed2[o] = e[t];
            if (lbk) lbk[o] = kg[t];
            if (lbeb) lbeb[o] = band[t];
            if (lbe) lbe[o] = en[t];
        }
    }
}

template <int TQ>
__global__ void __launch_bounds__(CB_THREADS)
cascade_bounds_kernel(const float *__restrict__ Bt, const float *__restrict__ Ut,
                      const float *__restrict__ Lt, int64_t pitch, int64_t n,
                      const float *__restrict__ Q, int64_t nQ, int L, int W, int nb,
                      double *__restrict__ ed2, double *__restrict__ lbk,
                      double *__restrict__ lbeb, double *__restrict__ lbe, int ncu)
{
    bounds_tile<TQ>(blockIdx.x, blockIdx.y, Bt, Ut, Lt, pitch, n, Q, nQ, L, W, nb, ed2, lbk, lbeb, lbe,
                    rotation_phase(ncu));
}

// The bound pass of a batch: one workgroup per tile of any set; the set is
// found by binary search over the tiles' start indices.  Also resets the
// work counters of the batch's search kernels and clears the items' helper
// headers (those kernels run after it).  A tile with a single query (the
// usual case of a serving batch) runs the one-query body: the per-point
// chain of each thread is then a quarter as long.
template <int TQ>
__global__ void __launch_bounds__(CB_THREADS)
batch_bounds_kernel(const BatchSet *__restrict__ sets, int nsets, const int64_t *__restrict__ tile_start,
                    BatchHdr *hdr, QueryShare *share, int64_t nshare)
{
    const int64_t tile = blockIdx.x;
    if (tile == 0 && threadIdx.x < BATCH_SHAPES) hdr->counter[threadIdx.x] = 0u;
    for (int64_t i = tile * CB_THREADS + threadIdx.x; i < nshare; i += (int64_t)gridDim.x * CB_THREADS)
        share_clear(share[i]);
    int lo = 0, hi = nsets - 1;                 // last set with tile_start <= tile
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tile_start[mid] <= tile) lo = mid; else hi = mid - 1;
    }
    const int d = __builtin_amdgcn_readfirstlane(lo);
    const BatchSet &b = sets[d];
    const int64_t local = tile - tile_start[d];
    const int64_t rt = local % b.nrt, qt = local / b.nrt;
    if (b.nQ - qt * TQ == 1)
        bounds_tile<1>(rt, qt * TQ, b.Bt, b.Ut, b.Lt, b.pitch, b.a.n, b.a.Q, b.nQ, b.L, b.W, b.nb, b.ed2w, b.lbk,
                       b.lbeb, b.lbe, rotation_phase(b.a.ncu));
    else
        bounds_tile<TQ>(rt, qt, b.Bt, b.Ut, b.Lt, b.pitch, b.a.n, b.a.Q, b.nQ, b.L, b.W, b.nb, b.ed2w, b.lbk,
                        b.lbeb, b.lbe, rotation_phase(b.a.ncu));
}

constexpr int BATCH_TQ = 4;

int launch_batch_bounds(const BatchSet *sets, int nsets, const int64_t *tile_start, int64_t tiles, BatchHdr *hdr,
                        QueryShare *share, int64_t nshare, hipStream_t st)
{
    if (tiles == 0) return NNDTW_OK;
    hipLaunchKernelGGL(batch_bounds_kernel<BATCH_TQ>, dim3((unsigned)tiles), dim3(CB_THREADS), 0, st, sets, nsets,
                       tile_start, hdr, share, nshare);
    NNDTW_LAUNCH_CHECK("batch bound kernel launch");
    return NNDTW_OK;
}

int launch_cascade_bounds(const nndtw_refset *rs, const float *Q, int64_t nQ, int V, double *ed2,
                          double *lbk, double *lbeb, double *lbe, hipStream_t st)
{
    if (nQ == 0 || rs->n == 0) return NNDTW_OK;
    constexpr int TQ = 4;
    const int L = rs->L;
    const int nb = V < L / 2 ? V : L / 2;
    dim3 grid((unsigned)ceil_div(rs->n, CB_THREADS), (unsigned)ceil_div(nQ, TQ));
    hipLaunchKernelGGL(cascade_bounds_kernel<TQ>, grid, dim3(CB_THREADS), 0, st, rs->Bt, rs->Ut, rs->Lt,
                       rs->pitch, rs->n, Q, nQ, L, rs->W, nb, ed2, lbk, lbeb, lbe, device_cu_count());
    NNDTW_LAUNCH_CHECK("cascade bounds kernel launch");
    return NNDTW_OK;
}

}  // namespace nndtw
