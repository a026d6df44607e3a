// Envelopes of Equations (3) and (4) and the point-major copies of a
// reference set.
//
// U_i = max and Lo_i = min of B_j over the clipped window
// [max(0, i-W), min(L-1, i+W)].  One wave per series: the row is staged in
// LDS, the running max/min over every aligned block of p = 2^floor(log2(W'+1))
// elements is built by doubling (log2 p passes), and each output takes the
// max/min of at most four such blocks covering its window (max and min are
// exact, so the result equals a direct scan).  A wave touches only its own
// row, so it synchronises with itself only: each pass is done in place in
// ascending order, a group of chunks at a time, all reads of a group before
// its writes (a later position is never overwritten before it is read).
#include "common.hpp"

namespace nndtw {

constexpr int ENV_WAVES = 4;  // series per workgroup
constexpr int ENV_GROUP = 8;  // 64-element chunks read before they are written

// LDS accesses of one wave before this point complete before those after it
// (LDS executes a wave's instructions in order; this stops the compiler from
// moving them across).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Optional outputs of a reference-set build, written from the row this
// kernel reads anyway: the row itself (Bc, row-major) and the row inside its
// padding (Bp: ppitch elements, the series at padl, 1e30 around it).
struct RowCopies {
    float *Bc = nullptr;
    float *Bp = nullptr;
    int padl = 0;
    int64_t ppitch = 0;
};

__global__ void __launch_bounds__(WAVE *ENV_WAVES)
envelopes_kernel(const float *__restrict__ B, int64_t n, int L, int Wp, int p,
                 float *__restrict__ U, float *__restrict__ Lo, RowCopies rc)
{
    extern __shared__ float lds[];
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int64_t s = (int64_t)blockIdx.x * ENV_WAVES + w;
    if (s >= n) return;                      // waves never wait for each other
    float *mx = lds + (size_t)w * 2 * L;
    float *mn = mx + L;
    const float *b = B + s * (int64_t)L;
    for (int i = lane; i < L; i += WAVE) {
        const float v = b[i];
        mx[i] = v;
        mn[i] = v;
        if (rc.Bc) rc.Bc[s * (int64_t)L + i] = v;
    }
    if (rc.Bp) {
        float *row = rc.Bp + s * rc.ppitch;
        for (int64_t e = lane; e < rc.ppitch; e += WAVE) {
            const int64_t j = e - rc.padl;
            row[e] = (j >= 0 && j < L) ? b[j] : Pad<float>::big();
        }
    }
    wave_lds_sync();
    // mx[i] <- max over [i, min(i + 2h - 1, L - 1)] for h = 1, 2, ... < p
    for (int h = 1; h < p; h <<= 1) {
        for (int g0 = 0; g0 < L; g0 += WAVE * ENV_GROUP) {
            float a[ENV_GROUP], c[ENV_GROUP];
#pragma unroll
            for (int k = 0; k < ENV_GROUP; ++k) {
                const int i = g0 + k * WAVE + lane;
                const int j = min(i + h, L - 1);
                a[k] = 0.f;
                c[k] = 0.f;
                if (i < L) {
                    a[k] = fmaxf(mx[i], mx[j]);
                    c[k] = fminf(mn[i], mn[j]);
                }
            }
            wave_lds_sync();
#pragma unroll
            for (int k = 0; k < ENV_GROUP; ++k) {
                const int i = g0 + k * WAVE + lane;
                if (i < L) {
                    mx[i] = a[k];
                    mn[i] = c[k];
                }
            }
            wave_lds_sync();
        }
    }
    float *u = U + s * (int64_t)L, *l = Lo + s * (int64_t)L;
    for (int i = lane; i < L; i += WAVE) {
        int lo = max(0, i - Wp), hi = min(L - 1, i + Wp);
        // blocks [lo, lo+p), [lo+p, ...), ..., and the last one ending at hi
        float uu = mx[lo], ll = mn[lo];
        for (int k = lo + p; k + p - 1 < hi; k += p) { uu = fmaxf(uu, mx[k]); ll = fminf(ll, mn[k]); }
        int last = hi - p + 1;
        uu = fmaxf(uu, mx[last]);
        ll = fminf(ll, mn[last]);
        u[i] = uu;
        l[i] = ll;
    }
}

static int launch_envelopes_rc(const float *B, int64_t n, int L, int W, float *U, float *Lo, RowCopies rc,
                               hipStream_t st)
{
    if (n == 0) return NNDTW_OK;
    const int Wp = W < L - 1 ? W : L - 1;
    int p = 1;
    while (2 * p <= Wp + 1) p *= 2;
    const size_t lds = (size_t)ENV_WAVES * 2 * L * sizeof(float);
    const int64_t blocks = ceil_div(n, ENV_WAVES);
    hipLaunchKernelGGL(envelopes_kernel, dim3((unsigned)blocks), dim3(WAVE * ENV_WAVES), lds, st,
                       B, n, L, Wp, p, U, Lo, rc);
    NNDTW_LAUNCH_CHECK("envelopes kernel launch");
    return NNDTW_OK;
}

int launch_envelopes(const float *B, int64_t n, int L, int W, float *U, float *Lo, hipStream_t st)
{
    return launch_envelopes_rc(B, n, L, W, U, Lo, RowCopies{}, st);
}

int launch_envelopes_build(const float *B, int64_t n, int L, int W, float *U, float *Lo, float *Bc, float *Bp,
                           int padl, int64_t ppitch, hipStream_t st)
{
    RowCopies rc;
    rc.Bc = Bc;
    rc.Bp = Bp;
    rc.padl = padl;
    rc.ppitch = ppitch;
    return launch_envelopes_rc(B, n, L, W, U, Lo, rc, st);
}

// Point-major copies: Xt[i][k] = X[k][i] for B, U and Lo, via TT x TT LDS
// tiles (32 x 32: a set of a thousand series of length 256 is 256 tiles,
// enough workgroups to spread over the compute units).
constexpr int TT = 32;

__global__ void __launch_bounds__(256)
transpose3_kernel(const float *__restrict__ B, const float *__restrict__ U, const float *__restrict__ Lo,
                  int64_t n, int L, int64_t pitch, float *__restrict__ Bt, float *__restrict__ Ut,
                  float *__restrict__ Lt)
{
    __shared__ float tile[3][TT][TT + 1];
    const int64_t k0 = (int64_t)blockIdx.x * TT;
    const int i0 = blockIdx.y * TT;
    const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;     // ty in [0, 256 / TT)
    constexpr int RS = 256 / TT;
    for (int r = ty; r < TT; r += RS) {
        int64_t k = k0 + r;
        int i = i0 + tx;
        bool ok = k < n && i < L;
        tile[0][r][tx] = ok ? B[k * L + i] : 0.f;
        tile[1][r][tx] = ok ? U[k * L + i] : 0.f;
        tile[2][r][tx] = ok ? Lo[k * L + i] : 0.f;
    }
    __syncthreads();
    for (int r = ty; r < TT; r += RS) {
        int i = i0 + r;
        int64_t k = k0 + tx;
        if (i < L && k < pitch) {
            bool ok = k < n;
            Bt[(int64_t)i * pitch + k] = ok ? tile[0][tx][r] : 0.f;
            Ut[(int64_t)i * pitch + k] = ok ? tile[1][tx][r] : 0.f;
            Lt[(int64_t)i * pitch + k] = ok ? tile[2][tx][r] : 0.f;
        }
    }
}

int launch_transpose3(const float *B, const float *U, const float *Lo, int64_t n, int L, int64_t pitch,
                      float *Bt, float *Ut, float *Lt, hipStream_t st)
{
    dim3 grid((unsigned)ceil_div(pitch, TT), (unsigned)ceil_div(L, TT));
    hipLaunchKernelGGL(transpose3_kernel, grid, dim3(256), 0, st, B, U, Lo, n, L, pitch, Bt, Ut, Lt);
    NNDTW_LAUNCH_CHECK("transpose kernel launch");
    return NNDTW_OK;
}

// Padded rows: Bp[k][padl + j] = B[k][j], 1e30 in the margins.
__global__ void __launch_bounds__(256)
pad_rows_kernel(const float *__restrict__ B, int64_t n, int L, int padl, int64_t ppitch, float *__restrict__ Bp)
{
    const int64_t total = n * ppitch;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t k = e / ppitch;
        const int64_t j = e - k * ppitch - padl;
        Bp[e] = (j >= 0 && j < L) ? B[k * L + j] : Pad<float>::big();
    }
}

int launch_pad_rows(const float *B, int64_t n, int L, int padl, int64_t ppitch, float *Bp, hipStream_t st)
{
    int64_t blocks = ceil_div(n * ppitch, 256);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(pad_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, st, B, n, L, padl, ppitch, Bp);
    NNDTW_LAUNCH_CHECK("pad rows kernel launch");
    return NNDTW_OK;
}

}  // namespace nndtw
