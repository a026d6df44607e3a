// Envelopes of Equations (3) and (4) and the point-major copies of a
// reference set.
//
// U_i = max and Lo_i = min of B_j over the clipped window
// [max(0, i-W'), min(L-1, i+W')], W' = min(W, L-1), by the van Herk /
// Gil-Werman decomposition: cut the row into blocks of k = 2W'+1 elements
// starting at 0; P(x) is the maximum from the start of x's block to x, S(x)
// the maximum from x to the end of x's block (or to L-1).  A window [a, b]
// holds at most k elements, so it lies in one block or two adjacent ones:
//   two blocks:               max(S(a), P(b))
//   one block, a its start:   P(b)          (a clipped to 0)
//   one block, otherwise:     S(a)          (then b is the block's end or L-1)
// (an unclipped window is either two blocks' or exactly one whole block,
// where S(a) = P(b), so only the clipped ends need the one-block forms).
// About three comparisons per element whatever W is, and max/min are exact,
// so the result equals a direct scan bit for bit.
//
// One wave per series, streaming: lane t holds the E consecutive elements
// t*E .. t*E+E-1 in registers (16-byte loads and stores where the row allows),
// the block-segmented prefix and suffix scans run over the lane's elements
// and then across lanes with shuffles, and the two scans go to LDS once so
// that each output can read S(a) and P(b) at its window's ends.  The row is
// read from memory once and U, Lo (and in a reference-set build the
// row-major copy and the padded row) are written once.
#include <algorithm>

#include "common.hpp"

namespace nndtw {

constexpr int ENV_WAVES = 4;  // series per workgroup

// Optional outputs of a reference-set build, written from the row this
// kernel reads anyway: the row itself (Bc, row-major) and the row inside its
// padding (Bp: ppitch elements, the series at padl, 1e30 around it).
struct RowCopies {
    float *Bc = nullptr;
    float *Bp = nullptr;
    int padl = 0;
    int64_t ppitch = 0;
};

// LDS slot of element x of a scan array: one spare slot per E elements, so
// that the 64 lanes reading elements E apart hit 64 different banks.
template <int E> __device__ __forceinline__ int slot(int x) { return x + x / E; }

// Segmented inclusive scans of one wave for max and min together, blocks of
// k elements starting at multiples of k.  vx[r] / vn[r] is element t*E + r of
// the row (lane t), past L the identity of max / min.  On return Px[r] / Pn[r]
// hold the max / min from the start of the element's block and Sx[r] / Sn[r]
// those to the end of its block.  Branch-free: every lane runs the same
// instructions (selects, no divergent branches).
template <int E>
__device__ __forceinline__ void block_scans(const float (&vx)[E], const float (&vn)[E], float (&Px)[E], float (&Pn)[E],
                                            float (&Sx)[E], float (&Sn)[E], int k, int lane)
{
    const int base = lane * E;
    const int rem0 = base % k;                               // position of base inside its block
    const int first_start = rem0 == 0 ? base : base - rem0 + k;   // first block start >= base
    const int last_end_excl = (base + E) / k * k;            // last multiple of k <= base + E
    // positions inside the block (incremental: no division per element)
    int rem[E];
    rem[0] = rem0;
#pragma unroll
    for (int r = 1; r < E; ++r) rem[r] = rem[r - 1] + 1 == k ? 0 : rem[r - 1] + 1;
    // local scans: P restarts at a block start, S at a block end
    float ax = vx[0], an = vn[0];
    Px[0] = ax;
    Pn[0] = an;
#pragma unroll
    for (int r = 1; r < E; ++r) {
        const bool st = rem[r] == 0;
        ax = st ? vx[r] : __builtin_fmaxf(ax, vx[r]);
        an = st ? vn[r] : __builtin_fminf(an, vn[r]);
        Px[r] = ax;
        Pn[r] = an;
    }
    ax = vx[E - 1];
    an = vn[E - 1];
    Sx[E - 1] = ax;
    Sn[E - 1] = an;
#pragma unroll
    for (int r = E - 2; r >= 0; --r) {
        const bool en = rem[r] == k - 1;
        ax = en ? vx[r] : __builtin_fmaxf(ax, vx[r]);
        an = en ? vn[r] : __builtin_fminf(an, vn[r]);
        Sx[r] = ax;
        Sn[r] = an;
    }
    // across lanes: forward carry = the scan of the lanes before this one
    // since the last block start (a lane holding a block start ends the
    // segment); backward carry likewise from the lanes after it
    int ff = first_start < base + E;                         // a block starts in this lane
    int bf = last_end_excl > base;                           // a block ends in this lane
    float fx = Px[E - 1], fn = Pn[E - 1], bx = Sx[0], bn = Sn[0];
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        const float ux = __shfl_up(fx, off), un = __shfl_up(fn, off);
        const int uf = __shfl_up(ff, off);
        const float dx = __shfl_down(bx, off), dn = __shfl_down(bn, off);
        const int df = __shfl_down(bf, off);
        const bool take_f = lane >= off && !ff;
        const bool take_b = lane + off < WAVE && !bf;
        fx = take_f ? __builtin_fmaxf(fx, ux) : fx;
        fn = take_f ? __builtin_fminf(fn, un) : fn;
        ff = lane >= off ? (ff | uf) : ff;
        bx = take_b ? __builtin_fmaxf(bx, dx) : bx;
        bn = take_b ? __builtin_fminf(bn, dn) : bn;
        bf = lane + off < WAVE ? (bf | df) : bf;
    }
    const float cix = __shfl_up(fx, 1), cin = __shfl_up(fn, 1);      // inclusive scans of lane t-1
    const float cox = __shfl_down(bx, 1), con = __shfl_down(bn, 1);  // and of lane t+1 (reverse)
#pragma unroll
    for (int r = 0; r < E; ++r) {
        // no block start in [base, base + r]: the block began in an earlier lane
        const bool pf = lane > 0 && first_start > base + r;
        Px[r] = pf ? __builtin_fmaxf(Px[r], cix) : Px[r];
        Pn[r] = pf ? __builtin_fminf(Pn[r], cin) : Pn[r];
        // no block end in [base + r, base + E - 1]: the block ends in a later lane
        const bool sf = lane < WAVE - 1 && last_end_excl <= base + r;
        Sx[r] = sf ? __builtin_fmaxf(Sx[r], cox) : Sx[r];
        Sn[r] = sf ? __builtin_fminf(Sn[r], con) : Sn[r];
    }
}

// FULL: L is a multiple of E, so each lane's elements are all inside the row
// or all past its end (one predicate per lane instead of one per element).
template <int E, bool VEC, bool FULL>
__device__ __forceinline__ void load_row(float (&v)[E], const float *__restrict__ b, int base, int L)
{
    if (FULL) {
        if (base < L) {
            if (VEC) {
#pragma unroll
                for (int r = 0; r < E; r += 4) {
                    const float4 q = *reinterpret_cast<const float4 *>(b + base + r);
                    v[r] = q.x; v[r + 1] = q.y; v[r + 2] = q.z; v[r + 3] = q.w;
                }
            } else {
#pragma unroll
                for (int r = 0; r < E; ++r) v[r] = b[base + r];
            }
        } else {
#pragma unroll
            for (int r = 0; r < E; ++r) v[r] = 0.f;
        }
    } else {
#pragma unroll
        for (int r = 0; r < E; ++r) v[r] = base + r < L ? b[base + r] : 0.f;
    }
}

template <int E, bool VEC, bool FULL>
__device__ __forceinline__ void store_row(float *__restrict__ u, const float (&o)[E], int base, int L)
{
    if (FULL) {
        if (base < L) {
            if (VEC) {
#pragma unroll
                for (int r = 0; r < E; r += 4)
                    *reinterpret_cast<float4 *>(u + base + r) = make_float4(o[r], o[r + 1], o[r + 2], o[r + 3]);
            } else {
#pragma unroll
                for (int r = 0; r < E; ++r) u[base + r] = o[r];
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < E; ++r)
            if (base + r < L) u[base + r] = o[r];
    }
}

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Each wave streams rows s = wave, wave + nwaves, ...: the next row's loads
// are issued before the current row is scanned, so two rows per wave are in
// flight.  Per row: block scans of max and min, the four scans through the
// wave's LDS slots, then per element the window rule of the header.
template <int E, bool VEC, bool FULL>
__global__ void __launch_bounds__(WAVE *ENV_WAVES)
envelopes_kernel(const float *__restrict__ B, int64_t n, int L, int Wp, float *__restrict__ U,
                 float *__restrict__ Lo, RowCopies rc)
{
    constexpr int SLOTS = 64 * E + 64;                     // slot(64E - 1) < SLOTS
    __shared__ float lds[ENV_WAVES][4][SLOTS];
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int64_t stride = (int64_t)gridDim.x * ENV_WAVES;
    int64_t s = (int64_t)blockIdx.x * ENV_WAVES + w;
    if (s >= n) return;                      // waves never wait for each other
    const int base = lane * E;
    const int k = 2 * Wp + 1;
    float(*sc)[SLOTS] = lds[w];
    float v[E], vn[E];
    load_row<E, VEC, FULL>(v, B + s * (int64_t)L, base, L);
    for (; s < n; s += stride) {
        const bool more = s + stride < n;
        if (more) load_row<E, VEC, FULL>(vn, B + (s + stride) * (int64_t)L, base, L);
        // row copies of a reference-set build
        if (rc.Bc) store_row<E, VEC, FULL>(rc.Bc + s * (int64_t)L, v, base, L);
        if (rc.Bp) {
            float *row = rc.Bp + s * rc.ppitch;
            store_row<E, false, FULL>(row + rc.padl, v, base, L);
            for (int64_t e = lane; e < rc.padl; e += WAVE) row[e] = Pad<float>::big();
            for (int64_t e = (int64_t)rc.padl + L + lane; e < rc.ppitch; e += WAVE) row[e] = Pad<float>::big();
        }
        // The lane's block positions and masks do not change from row to
        // row; hidden from the compiler here so that it recomputes them per
        // row instead of keeping dozens of lane masks live across the loop
        // (which spilled scalar registers).
        int ln = lane;
        asm volatile("" : "+v"(ln));
        {
            float vx[E], vm[E], Px[E], Pn[E], Sx[E], Sn[E];
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const bool in = ln * E + r < L;
                vx[r] = in ? v[r] : -__builtin_inff();
                vm[r] = in ? v[r] : __builtin_inff();
            }
            block_scans<E>(vx, vm, Px, Pn, Sx, Sn, k, ln);
            wave_lds_sync();                   // the previous row's reads of the slots are done
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const int x = slot<E>(ln * E + r);
                sc[0][x] = Px[r];
                sc[1][x] = Sx[r];
                sc[2][x] = Pn[r];
                sc[3][x] = Sn[r];
            }
        }
        wave_lds_sync();
        float uo[E], lo[E];
        // The window [a, c] of i: unclipped it has k elements, so it spans
        // two blocks or is one whole block (where S(a) = P(c)): max(S(a),
        // P(c)) either way.  Clipped at 0 it lies in block 0 from its start:
        // P(c) alone.  Clipped at L-1 inside the last block (a at or after
        // that block's start): S(a) alone.  Otherwise clipped at L-1 it
        // spans the last two blocks: max(S(a), P(c)) again.
        const int lb = ln * E;
        const int last_start = (L - 1) / k * k;
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int i = lb + r;
            const int a = max(0, i - Wp), c = min(L - 1, i + Wp);
            const bool no_s = i - Wp < 0;
            const bool no_p = a >= last_start && c == L - 1 && !no_s;
            const int sa = slot<E>(a), sb = slot<E>(c);
            const float sx = sc[1][sa], px = sc[0][sb], sn = sc[3][sa], pn = sc[2][sb];
            uo[r] = __builtin_fmaxf(no_s ? -__builtin_inff() : sx, no_p ? -__builtin_inff() : px);
            lo[r] = __builtin_fminf(no_s ? __builtin_inff() : sn, no_p ? __builtin_inff() : pn);
        }
        store_row<E, VEC, FULL>(U + s * (int64_t)L, uo, base, L);
        store_row<E, VEC, FULL>(Lo + s * (int64_t)L, lo, base, L);
        if (more) {
#pragma unroll
            for (int r = 0; r < E; ++r) v[r] = vn[r];
        }
    }
}

static int launch_envelopes_rc(const float *B, int64_t n, int L, int W, float *U, float *Lo, RowCopies rc,
                               hipStream_t st)
{
    if (n == 0) return NNDTW_OK;
    const int Wp = W < L - 1 ? W : L - 1;
    int E = 1;
    while (64 * E < L) E *= 2;
    // 16-byte row accesses: every row (and every output row) 16-byte aligned
    auto al16 = [](const void *p) { return ((uintptr_t)p & 15u) == 0; };
    const bool vec = E >= 4 && L % 4 == 0 && al16(B) && al16(U) && al16(Lo) && (!rc.Bc || al16(rc.Bc));
    // enough workgroups for every compute unit several times over; each wave
    // then streams its share of the rows
    const int cu = device_cu_count() > 0 ? device_cu_count() : 256;
    const int64_t blocks = std::min<int64_t>(ceil_div(n, ENV_WAVES), (int64_t)cu * 8);
    const bool full = L % E == 0;
    switch (E * 4 + (vec ? 2 : 0) + (full ? 1 : 0)) {
#define NNDTW_ENV_CASE(e, v, f)                                                                               \
    case e * 4 + v * 2 + f:                                                                                 \
        hipLaunchKernelGGL((envelopes_kernel<e, v, f>), dim3((unsigned)blocks), dim3(WAVE * ENV_WAVES), 0, st, B, \
                           n, L, Wp, U, Lo, rc);                                                            \
        break;
        NNDTW_ENV_CASE(1, 0, 0)
        NNDTW_ENV_CASE(1, 0, 1)
        NNDTW_ENV_CASE(2, 0, 0)
        NNDTW_ENV_CASE(2, 0, 1)
        NNDTW_ENV_CASE(4, 0, 0)
        NNDTW_ENV_CASE(4, 0, 1)
        NNDTW_ENV_CASE(4, 1, 1)
        NNDTW_ENV_CASE(8, 0, 0)
        NNDTW_ENV_CASE(8, 0, 1)
        NNDTW_ENV_CASE(8, 1, 0)
        NNDTW_ENV_CASE(8, 1, 1)
        NNDTW_ENV_CASE(16, 0, 0)
        NNDTW_ENV_CASE(16, 0, 1)
        NNDTW_ENV_CASE(16, 1, 0)
        NNDTW_ENV_CASE(16, 1, 1)
        NNDTW_ENV_CASE(32, 0, 0)
        NNDTW_ENV_CASE(32, 0, 1)
        NNDTW_ENV_CASE(32, 1, 0)
        NNDTW_ENV_CASE(32, 1, 1)
#undef NNDTW_ENV_CASE
    default:
        return fail(NNDTW_EUNSUP, "series length %d too long for the envelope kernel", L);
    }
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
