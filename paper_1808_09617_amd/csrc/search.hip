// Nearest-neighbour lower-bound search (Sections 1 and 4) on one GPU.
//
// Enqueued as three kernels on the caller's stream (four with a comparison
// cascade, whose bound pass follows the fused one):
//   1. cascade bounds   squared ED, LB_Keogh, LB_Enhanced bands part and full
//                       bound for every (query, reference)       (bounds.hip)
//   2. order            per query, references sorted by (squared ED, index)
//                       in LDS, with the bounds gathered in that order; the
//                       first workgroup also fills the cells table (window
//                       cells on anti-diagonals 0..s, for the cell counts)
//   3. search           one workgroup per query: rounds of R candidates in visiting
//                       order are tested against the round's threshold; the
//                       survivors run through the DTW engine (FP32, abandoned
//                       above the threshold), groups of the wave computing
//                       different candidates at once; results that can decide
//                       the nearest neighbour are recomputed in FP64, and the
//                       record is updated with the lexicographic minimum of
//                       (distance, index) at the end of the round.
//
// Why the result and the stage counts do not depend on FP32 rounding: with
// u = 2^-24 and gamma = (2L+1)u / (1-(2L+1)u), an FP32 cell value is within a
// factor (1 +- gamma) of the exact one (each term of a path sum is rounded at
// most 2L+1 times).  Every test uses the slack eps >= 2 gamma (the default,
// also the smallest eps accepted, is twice gamma_{2L+2}):
//  * a bound prunes only if bound > thr = min(bsf, ub)(1 + eps), so the exact
//    DTW exceeds bsf and the candidate could not have changed the record;
//  * an FP32 frontier above thr means an exact value above thr / (1+gamma)
//    > bsf, likewise;
//  * the winner w of a round has an FP32 value within (1+gamma)/(1-gamma) of
//    the smallest FP32 value of the round and at most thr, so recomputing in
//    FP64 every completed result within the factor (1 + 2 eps) of the round's
//    FP32 minimum (and <= thr) always recomputes w.
// The bounds are FP64 sums in the same order as a sequential evaluation, and
// the recomputed distances are bit-identical to a sequential FP64 evaluation
// of the recurrence, so every decision is taken on the same values.
#include <algorithm>
#include <atomic>

#include "strip_engine.hpp"

namespace nndtw {

// Engine shapes of the search kernel: every one compiles within the
// register file at 8 waves per workgroup (no spill to scratch memory), so
// the search takes windows with min(W, L-1) + 1 <= 63 * SEARCH_MAX_CPL.
#define NNDTW_FOR_EACH_CPL(X) X(1) X(2) X(3) X(4) X(6) X(8) X(9)
constexpr int SEARCH_MAX_CPL = 9;

constexpr int QCAP = 512;        // survivor ring (>= the largest batch + one chunk of 64)
constexpr int SEARCH_MAX_WAVES = 8;        // workgroup size of the search kernels (waves)
constexpr int SEARCH_WIDE_WAVES = NNDTW_SEARCH_MAX_WAVES;   // ... of the wide ones
constexpr int SEARCH_DEFAULT_WAVES = 4;
constexpr int SEARCH_DEFAULT_HELPERS = 3;
// Engine shapes whose single-query search kernels hold the shared-batch code
// (helper workgroups): 3 and 6 pairs per lane fill the 128 registers those
// kernels are held to without it, and would spill with it.  (The batch's
// kernels are not held to 128 and share at every shape.)
__host__ __device__ constexpr bool share_ok(int C) { return C != 3 && C != 6; }
constexpr int ORDER_THREADS = 256;
constexpr int ORDER_LDS_PER_POSITION = 10;  // FP64 key + 16-bit index (order_query)

// ------------------------------------------------------------ workspace
static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
WsLayout ws_layout(int64_t nQ, int64_t n, int L, bool share)
{
    WsLayout w;
    const size_t m = (size_t)nQ * (size_t)n;
    size_t o = 0;
    w.ed2 = o;   o = al256(o + m * 8);
    w.lbk = o;   o = al256(o + m * 8);
    w.lbeb = o;  o = al256(o + m * 8);
    w.lbe = o;   o = al256(o + m * 8);
    w.sk = o;    o = al256(o + m * 4);
    w.slbk = o;  o = al256(o + m * 8);
    w.slbeb = o; o = al256(o + m * 8);
    w.slbe = o;  o = al256(o + m * 8);
    w.prefix = o; o = al256(o + (size_t)(2 * L) * 4);
    w.share = o;  o = al256(o + (share ? (size_t)nQ * sizeof(QueryShare) : 0));
    w.total = o;
    return w;
}
size_t search_ws_bytes(int64_t nQ, int64_t n, int L) { return ws_layout(nQ, n, L).total; }

// ------------------------------------------------------------ cells prefix
// prefix[s] = number of cells (i, j) of the L x L matrix with |i-j| <= W' and
// i + j <= s, for s = 0 .. 2L-2.
__global__ void __launch_bounds__(1024) cells_prefix_kernel(int L, int Wp, uint32_t *prefix)
{
    __shared__ uint32_t part[1024];
    const int S = 2 * L - 1;
    const int per = (S + 1023) / 1024;
    const int s0 = threadIdx.x * per;
    uint32_t loc[4];
    uint32_t acc = 0;
    for (int x = 0; x < per; ++x) {
        const int s = s0 + x;
        uint32_t c = 0;
        if (s < S) {
            int km = min(Wp, min(s, 2 * L - 2 - s));
            c = (uint32_t)(km + 1 - ((km + s) & 1));
        }
        acc += c;
        loc[x] = acc;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    const uint32_t before = threadIdx.x ? part[threadIdx.x - 1] : 0u;
    for (int x = 0; x < per; ++x)
        if (s0 + x < S) prefix[s0 + x] = before + loc[x];
}

// ------------------------------------------------------------ order
// Bitonic sort of (ed2, index) ascending, one workgroup per query.  Thread t
// of NT holds the E consecutive positions t*E .. t*E+E-1 (npow = NT * E), so a
// compare-exchange at stride s pairs two of its own registers when s < E,
// lanes t and t ^ (s / E) of one wave (a shuffle) when s < 64 E, and only
// larger strides go through LDS with a barrier.  Keys are unique (indices
// differ) except for the padding (+inf, 0xFFFFFFFF) entries.
__device__ __forceinline__ bool key_gt(double ka, uint32_t ia, double kb, uint32_t ib)
{
    return ka > kb || (ka == kb && ia > ib);
}

// (k, x) becomes the min (want_min) or max of itself and (ko, xo).
__device__ __forceinline__ void keep(double &k, uint32_t &x, double ko, uint32_t xo, bool want_min)
{
    const bool take = want_min ? key_gt(k, x, ko, xo) : key_gt(ko, xo, k, x);
    k = take ? ko : k;
    x = take ? xo : x;
}

// Bitonic sort of the (key, index) pairs held in registers: thread t of NT
// holds positions t*E .. t*E+E-1 before and after.  Whole-workgroup call.
// IX: the type the indices take in LDS (uint16_t when every index, padding
// included, is below 2^16: 10 bytes per position instead of 12, so that two
// 8192-position sorts fit a compute unit's LDS).
template <int E, int NT, typename IX = uint32_t>
__device__ __forceinline__ void sort_pairs(double (&k)[E], uint32_t (&x)[E], unsigned char *smem)
{
    constexpr int npow = NT * E;
    double *key = reinterpret_cast<double *>(smem);
    IX *idx = reinterpret_cast<IX *>(key + npow);
    const int t = threadIdx.x;
    for (int size = 2; size <= npow; size <<= 1) {
        int stride = size >> 1;
        for (; stride >= WAVE * E; stride >>= 1) {        // across waves
#pragma unroll
            for (int r = 0; r < E; ++r) {
                key[t * E + r] = k[r];
                idx[t * E + r] = (IX)x[r];
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const int e = t * E + r, p = e ^ stride;
                keep(k[r], x[r], key[p], (uint32_t)idx[p], ((e & stride) == 0) == ((e & size) == 0));
            }
            __syncthreads();
        }
        for (; stride >= E; stride >>= 1) {               // across lanes
            const int m = stride / E;
            const bool lo = (t & m) == 0;
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const double ko = __shfl_xor(k[r], m);
                const uint32_t xo = (uint32_t)__shfl_xor((int)x[r], m);
                keep(k[r], x[r], ko, xo, lo == (((t * E + r) & size) == 0));
            }
        }
#pragma unroll
        for (int s2 = E / 2; s2 >= 1; s2 >>= 1) {         // inside the thread
            if (s2 > stride) continue;
#pragma unroll
            for (int r = 0; r < E; ++r) {
                if (r & s2) continue;
                const bool up = ((t * E + r) & size) == 0;
                const double ka = k[r], kb = k[r | s2];
                const uint32_t ia = x[r], ib = x[r | s2];
                const bool sw = key_gt(ka, ia, kb, ib) == up;
                k[r] = sw ? kb : ka;
                x[r] = sw ? ib : ia;
                k[r | s2] = sw ? ka : kb;
                x[r | s2] = sw ? ia : ib;
            }
        }
    }
}

// Visiting order of one query of a set of n <= NT * E <= 8192 references,
// sorted on chip, with the bounds gathered in that order.  Indices (and the
// padding's 0xFFFF) fit 16 bits, which is how they are kept in LDS.
template <int E, int NT>
__device__ __forceinline__ void order_query(int64_t n, int64_t q, const double *__restrict__ ed2,
                                            const double *__restrict__ lbk, const double *__restrict__ lbeb,
                                            const double *__restrict__ lbe, uint32_t *__restrict__ sk,
                                            double *__restrict__ slbk, double *__restrict__ slbeb,
                                            double *__restrict__ slbe, unsigned char *smem)
{
    constexpr int npow = NT * E;
    static_assert(npow <= 0xFFFF, "16-bit indices");
    double *key = reinterpret_cast<double *>(smem);
    uint16_t *idx = reinterpret_cast<uint16_t *>(key + npow);
    const int t = threadIdx.x;
    const double *e2 = ed2 + q * n;
    double k[E];
    uint32_t x[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int e = t * E + r;
        k[r] = e < n ? e2[e] : __builtin_inf();
        x[r] = e < n ? (uint32_t)e : 0xFFFFu;
    }
    sort_pairs<E, NT, uint16_t>(k, x, smem);
#pragma unroll
    for (int r = 0; r < E; ++r) idx[t * E + r] = (uint16_t)x[r];
    __syncthreads();
    for (int i = t; i < n; i += NT) {
        const uint32_t kk = (uint32_t)idx[i];
        const int64_t o = q * n + i;
        sk[o] = kk;
        slbk[o] = lbk[q * n + kk];
        slbeb[o] = lbeb[q * n + kk];
        slbe[o] = lbe[q * n + kk];
    }
}

// ----------------------------------------------------- order by ranking
// With few queries the sort above leaves most of the chip idle: one
// workgroup per query, whose time is the latency of its dependent
// compare-exchange steps (78 of them at 4096 positions).  Ranking finds the
// same order with no dependent steps, spread over many workgroups: the place
// of reference i in the visiting order is the number of references whose
// (ED^2, index) pair precedes its own,
//     rank(i) = #{j : d_j < d_i} + #{j < i : d_j = d_i},
// at the price of n^2 comparisons per query.  The pairs are distinct, so the
// ranks are a permutation of 0 .. n-1 and the order is the sort's.  The
// distances are compared as FP64 bit patterns, which order non-negative
// values as the values do (-0 maps to +0, a NaN above +inf).
constexpr int RANK_BLOCK = 64;                // references per workgroup, one per lane
constexpr int RANK_WAVES = 16;                // waves per workgroup: wave w counts over the w-th slice of the keys
// The library's choice: rank while the sum of n^2 over the queries is at
// most RANK_WORK_PER_POSITION times the sort's padded size npow (the power of
// two >= max(n, 256)).  Measured at W = 6, L = 64 (order stage, us, sort /
// rank): n = 1000, 64 queries 27 / 20; n = 4000, 16 queries 79 / 43 and 32
// queries 80 / 76; n = 8192, 8 queries 161 / 74 and 16 queries 161 / 135.
// The sort's time grows with npow and hardly with the query count (its
// workgroups run side by side); ranking's with the comparisons.
constexpr int64_t RANK_WORK_PER_POSITION = 1ll << 16;
constexpr int64_t RANK_MAX_BLOCKS = 1ll << 20;
constexpr int RANK_MAX_N = 8192;              // references per query (all keys staged in LDS)

__device__ __forceinline__ uint64_t rank_key(double v)
{
    return v > 0.0 ? (uint64_t)__double_as_longlong(v) : (v == 0.0 ? 0ull : 0x7FF8000000000000ull);
}

// Places of references blk*RANK_BLOCK .. +RANK_BLOCK-1 of query q (n <=
// RANK_MAX_N references): every key of the query is staged in LDS, each
// wave counts the keys of its slice that precede each lane's reference, and
// the first wave adds the counts and writes the reference's index and bounds
// at its place.  Whole-workgroup call.
__device__ __forceinline__ void rank_block(int n, int64_t q, int blk, const double *__restrict__ ed2,
                                           const double *__restrict__ lbk, const double *__restrict__ lbeb,
                                           const double *__restrict__ lbe, uint32_t *__restrict__ sk,
                                           double *__restrict__ slbk, double *__restrict__ slbeb,
                                           double *__restrict__ slbe, unsigned char *smem)
{
    uint64_t *key = reinterpret_cast<uint64_t *>(smem);
    uint32_t *part = reinterpret_cast<uint32_t *>(key + n);   // [RANK_WAVES][RANK_BLOCK]
    const int t = threadIdx.x, lane = t % WAVE, w = t / WAVE;
    const double *e2 = ed2 + q * n;
    // every load in flight at once (n <= RANK_MAX_N): RANK_LOADS per thread
    constexpr int NT = RANK_WAVES * WAVE, RANK_LOADS = RANK_MAX_N / NT;
    double v[RANK_LOADS];
#pragma unroll
    for (int r = 0; r < RANK_LOADS; ++r) v[r] = t + r * NT < n ? e2[t + r * NT] : 0.0;
#pragma unroll
    for (int r = 0; r < RANK_LOADS; ++r)
        if (t + r * NT < n) key[t + r * NT] = rank_key(v[r]);
    __syncthreads();
    const int b0 = blk * RANK_BLOCK, i = b0 + lane;
    const uint64_t ki = i < n ? key[i] : 0ull;
    const uint64_t upto = ki + 1u;             // for j < i: d_j <= d_i precedes (no overflow: ki <= a NaN's)
    const int S = (n + RANK_WAVES - 1) / RANK_WAVES;
    const int lo = min(n, w * S), hi = min(n, lo + S);
    uint32_t c = 0;
    int j = lo;
    const int e1 = min(hi, max(lo, b0));       // keys before the block: j < i on every lane
#pragma unroll 8
    for (; j < e1; ++j) c += key[j] < upto ? 1u : 0u;
    const int e2x = min(hi, max(lo, b0 + RANK_BLOCK));
    for (; j < e2x; ++j) c += key[j] < (j < i ? upto : ki) ? 1u : 0u;
#pragma unroll 8
    for (; j < hi; ++j) c += key[j] < ki ? 1u : 0u;   // keys after the block: j > i on every lane
    part[w * RANK_BLOCK + lane] = c;
    __syncthreads();
    if (w == 0 && i < n) {
        uint32_t r = 0;
#pragma unroll
        for (int u = 0; u < RANK_WAVES; ++u) r += part[u * RANK_BLOCK + lane];
        const int64_t o = q * n + r, src = q * n + i;
        sk[o] = (uint32_t)i;
        slbk[o] = lbk[src];
        slbeb[o] = lbeb[src];
        slbe[o] = lbe[src];
    }
}

static size_t rank_lds(int64_t n) { return (size_t)n * 8 + (size_t)RANK_WAVES * RANK_BLOCK * 4; }

// ------------------------------------------------------- large reference sets
// Above the on-chip size (8192 references) the visiting order is sorted in
// chunks of 8192 on chip, then the sorted runs are merged pairwise in global
// memory: an element's place in the merged run is its place in its own run
// plus the number of elements of the other run that precede it, found by
// binary search (the (key, index) pairs are all distinct, so the order is
// total and every element lands on a distinct place).  Then the bounds are
// gathered in the final order.
constexpr int CHUNK_E = 8, CHUNK_NT = 1024, CHUNK = CHUNK_E * CHUNK_NT;

__global__ void __launch_bounds__(CHUNK_NT)
chunk_sort_kernel(int64_t n, int64_t nchunks, const double *__restrict__ ed2, double *__restrict__ kout,
                  uint32_t *__restrict__ xout)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t q = blockIdx.x / nchunks, c = blockIdx.x % nchunks;
    const int64_t c0 = c * CHUNK;
    const int64_t len = (n - c0) < CHUNK ? (n - c0) : CHUNK;
    const int t = threadIdx.x;
    double k[CHUNK_E];
    uint32_t x[CHUNK_E];
#pragma unroll
    for (int r = 0; r < CHUNK_E; ++r) {
        const int e = t * CHUNK_E + r;
        k[r] = e < len ? ed2[q * n + c0 + e] : __builtin_inf();
        x[r] = e < len ? (uint32_t)(c0 + e) : 0xFFFFFFFFu;
    }
    sort_pairs<CHUNK_E, CHUNK_NT>(k, x, smem);
#pragma unroll
    for (int r = 0; r < CHUNK_E; ++r) {
        const int e = t * CHUNK_E + r;
        if (e < len) {
            kout[q * n + c0 + e] = k[r];
            xout[q * n + c0 + e] = x[r];
        }
    }
}

// One merge pass over runs of w sorted elements per query: runs 2j and 2j+1
// become one sorted run of up to 2w.  One thread per element.
__global__ void __launch_bounds__(256)
merge_pass_kernel(int64_t nQ, int64_t n, int64_t w, const double *__restrict__ kin, const uint32_t *__restrict__ xin,
                  double *__restrict__ kout, uint32_t *__restrict__ xout)
{
    const int64_t total = nQ * n;
    for (int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x; id < total; id += (int64_t)gridDim.x * 256) {
        const int64_t q = id / n, g = id - q * n;
        const int64_t run = g / w, rs = run * w, ps = (run & ~(int64_t)1) * w;
        const bool first = (run & 1) == 0;
        const int64_t os = first ? ps + w : ps;                       // the other run
        const int64_t oe = first ? (ps + 2 * w < n ? ps + 2 * w : n) : ps + w;
        const double km = kin[id];
        const uint32_t xm = xin[id];
        int64_t lo = 0, hi = oe > os ? oe - os : 0;                   // count of the other run before (km, xm)
        const double *ko = kin + q * n + os;
        const uint32_t *xo = xin + q * n + os;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (key_gt(km, xm, ko[mid], xo[mid])) lo = mid + 1;
            else hi = mid;
        }
        const int64_t out = q * n + ps + (g - rs) + lo;
        kout[out] = km;
        xout[out] = xm;
    }
}

// The bounds in visiting order, from the sorted indices.
__global__ void __launch_bounds__(256)
gather_bounds_kernel(int64_t nQ, int64_t n, const uint32_t *__restrict__ sk, const double *__restrict__ lbk,
                     const double *__restrict__ lbeb, const double *__restrict__ lbe, double *__restrict__ slbk,
                     double *__restrict__ slbeb, double *__restrict__ slbe)
{
    const int64_t total = nQ * n;
    for (int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x; id < total; id += (int64_t)gridDim.x * 256) {
        const int64_t q = id / n;
        const int64_t src = q * n + sk[id];
        slbk[id] = lbk[src];
        slbeb[id] = lbeb[src];
        slbe[id] = lbe[src];
    }
}

// The cells table of the search (prefix[s] = window cells on anti-diagonals
// 0..s) by one wave: each lane counts a contiguous chunk of anti-diagonals,
// then the chunk totals are scanned across the wave.
__device__ void cells_prefix_wave(int L, int Wp, uint32_t *__restrict__ prefix, int lane)
{
    const int S = 2 * L - 1;
    const int per = (S + WAVE - 1) / WAVE;
    const int s0 = lane * per;
    auto count = [&](int s) {
        const int km = min(Wp, min(s, 2 * L - 2 - s));
        return (uint32_t)(km + 1 - ((km + s) & 1));
    };
    uint32_t tot = 0;
    for (int x = 0; x < per && s0 + x < S; ++x) tot += count(s0 + x);
    uint32_t inc = tot;
    for (int off = 1; off < WAVE; off <<= 1) {
        const uint32_t v = (uint32_t)__shfl_up((int)inc, off);
        if (lane >= off) inc += v;
    }
    uint32_t acc = inc - tot;
    for (int x = 0; x < per && s0 + x < S; ++x) {
        acc += count(s0 + x);
        prefix[s0 + x] = acc;
    }
}

// The 8192-position sort (512 threads of 16 positions, 80 KB of LDS) is held
// to 128 VGPRs so that two of its workgroups share a compute unit: each alone
// is bound by the latency of its barrier-separated steps (1024 threads of 8
// positions took 96 KB with 32-bit indices, one workgroup per unit, and
// spilled when held to the 64 VGPRs two such workgroups would need).
template <int E, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT * E >= 8192 ? 4 : 1)))
order_kernel(int64_t n, const double *__restrict__ ed2, const double *__restrict__ lbk,
             const double *__restrict__ lbeb, const double *__restrict__ lbe, uint32_t *__restrict__ sk,
             double *__restrict__ slbk, double *__restrict__ slbeb, double *__restrict__ slbe, int L, int Wp,
             uint32_t *__restrict__ prefix)
{
    extern __shared__ __align__(16) unsigned char smem[];
    order_query<E, NT>(n, blockIdx.x, ed2, lbk, lbeb, lbe, sk, slbk, slbeb, slbe, smem);
    // the first workgroup's first wave also fills the search's cells table
    if (blockIdx.x == 0 && threadIdx.x < WAVE) cells_prefix_wave(L, Wp, prefix, threadIdx.x);
}

// The ordering of a batch: one workgroup per (set, query) item of the sets
// whose sort width is E (items are (set << 32) | query).
template <int E, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT * E >= 8192 ? 4 : 1)))
batch_order_kernel(const BatchSet *__restrict__ sets, const int64_t *__restrict__ items)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t it = items[blockIdx.x];
    const int d = __builtin_amdgcn_readfirstlane((int)(it >> 32));
    const int64_t q = it & 0xFFFFFFFF;
    const BatchSet &b = sets[d];
    order_query<E, NT>(b.a.n, q, b.ed2w, b.lbk, b.lbeb, b.lbe, b.skw, b.slbkw, b.slbebw, b.slbew, smem);
    // the set's first query also fills the set's cells table (read only by
    // the search kernels, which follow on the stream)
    if (q == 0 && threadIdx.x < WAVE)
        cells_prefix_wave(b.a.geo.L, b.a.geo.Wp, const_cast<uint32_t *>(b.a.prefix), threadIdx.x);
}

// Ordering by ranking, one workgroup per RANK_BLOCK references of a query
// (workgroup x: query x / nblk, block x % nblk).
__global__ void __launch_bounds__(RANK_WAVES * WAVE)
rank_order_kernel(int n, int nblk, const double *__restrict__ ed2, const double *__restrict__ lbk,
                  const double *__restrict__ lbeb, const double *__restrict__ lbe, uint32_t *__restrict__ sk,
                  double *__restrict__ slbk, double *__restrict__ slbeb, double *__restrict__ slbe, int L, int Wp,
                  uint32_t *__restrict__ prefix)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t q = blockIdx.x / (unsigned)nblk;
    const int blk = (int)(blockIdx.x % (unsigned)nblk);
    rank_block(n, q, blk, ed2, lbk, lbeb, lbe, sk, slbk, slbeb, slbe, smem);
    if (blockIdx.x == 0 && threadIdx.x < WAVE) cells_prefix_wave(L, Wp, prefix, threadIdx.x);
}

// ... of a batch: nblk workgroups per item, the first ceil(n / RANK_BLOCK)
// of them work (the item's set decides n).
__global__ void __launch_bounds__(RANK_WAVES * WAVE)
batch_rank_kernel(const BatchSet *__restrict__ sets, const int64_t *__restrict__ items, int nblk)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t it = items[blockIdx.x / (unsigned)nblk];
    const int blk = (int)(blockIdx.x % (unsigned)nblk);
    const int d = __builtin_amdgcn_readfirstlane((int)(it >> 32));
    const int64_t q = it & 0xFFFFFFFF;
    const BatchSet &b = sets[d];
    const int n = (int)b.a.n;
    if (blk * RANK_BLOCK >= n) return;        // the whole workgroup, before any barrier
    rank_block(n, q, blk, b.ed2w, b.lbk, b.lbeb, b.lbe, b.skw, b.slbkw, b.slbebw, b.slbew, smem);
    if (q == 0 && blk == 0 && threadIdx.x < WAVE)
        cells_prefix_wave(b.a.geo.L, b.a.geo.Wp, const_cast<uint32_t *>(b.a.prefix), threadIdx.x);
}

int order_width(int64_t n)
{
    int E = 1;
    while ((int64_t)ORDER_THREADS * E < n) E <<= 1;
    return E;
}

// Sort shapes by padded size npow = 256 * W (W = order_width): up to 4096
// positions at most 8 per thread, 8192 as 512 threads of 16 (two workgroups
// per compute unit, see order_kernel).
#define NNDTW_FOR_EACH_SORT(X) X(1, 1, 256) X(2, 2, 256) X(4, 4, 256) X(8, 8, 256) X(16, 8, 512) X(32, 16, 512)

int launch_batch_order(int Wd, const BatchSet *sets, const int64_t *items, int64_t nitems, hipStream_t st)
{
    if (nitems == 0) return NNDTW_OK;
    const size_t lds = (size_t)ORDER_THREADS * Wd * ORDER_LDS_PER_POSITION;
    switch (Wd) {
#define NNDTW_BORDER_CASE(WW, EE, NT)                                                                \
    case WW:                                                                                         \
        hipLaunchKernelGGL((batch_order_kernel<EE, NT>), dim3((unsigned)nitems), dim3(NT), lds, st, \
                           sets, items);                                                             \
        break;
        NNDTW_FOR_EACH_SORT(NNDTW_BORDER_CASE)
#undef NNDTW_BORDER_CASE
    default:
        return fail(NNDTW_EUNSUP, "order: sort width %d not supported", Wd);
    }
    NNDTW_LAUNCH_CHECK("batch order kernel launch");
    return NNDTW_OK;
}

// The ordering of a batch by ranking (one launch for every item; oitems as
// for launch_batch_order, nmax the largest n of their sets).
int launch_batch_rank(const BatchSet *sets, const int64_t *items, int64_t nitems, int64_t nmax, hipStream_t st)
{
    if (nitems == 0) return NNDTW_OK;
    const int64_t nblk = ceil_div(nmax, RANK_BLOCK);
    if (nmax > RANK_MAX_N || nitems * nblk > RANK_MAX_BLOCKS)
        return fail(NNDTW_EUNSUP, "ordering by ranking: %lld items of up to %lld references", (long long)nitems,
                    (long long)nmax);
    hipLaunchKernelGGL(batch_rank_kernel, dim3((unsigned)(nitems * nblk)), dim3(RANK_WAVES * WAVE), rank_lds(nmax),
                       st, sets, items, (int)nblk);
    NNDTW_LAUNCH_CHECK("batch rank kernel launch");
    return NNDTW_OK;
}

// Ranking (rather than the per-query sort) for nitems queries of at most
// nmax references, sum of n^2 over the queries `work`: the option's choice,
// else while work <= RANK_WORK_PER_POSITION * npow.  EUNSUP when ranking is
// asked for beyond RANK_MAX_N references or RANK_MAX_BLOCKS workgroups.
int order_by_rank(int order, double work, int64_t nmax, int64_t nitems, bool *rank)
{
    if (order < NNDTW_ORDER_AUTO || order > NNDTW_ORDER_RANK)
        return fail(NNDTW_EINVAL, "order=%d is not an NNDTW_ORDER_* value", order);
    const bool fits = nmax <= RANK_MAX_N && nitems * ceil_div(nmax, RANK_BLOCK) <= RANK_MAX_BLOCKS;
    if (order == NNDTW_ORDER_RANK && !fits)
        return fail(NNDTW_EUNSUP, "ordering by ranking: %lld queries of up to %lld references",
                    (long long)nitems, (long long)nmax);
    int64_t npow = ORDER_THREADS;
    while (npow < nmax) npow <<= 1;
    *rank = order == NNDTW_ORDER_RANK ||
            (order == NNDTW_ORDER_AUTO && fits && work <= (double)RANK_WORK_PER_POSITION * (double)npow);
    return NNDTW_OK;
}

int launch_cells_prefix(int L, int Wp, uint32_t *prefix, hipStream_t st)
{
    hipLaunchKernelGGL(cells_prefix_kernel, dim3(1), dim3(1024), 0, st, L, Wp, prefix);
    NNDTW_LAUNCH_CHECK("cells prefix kernel launch");
    return NNDTW_OK;
}

// Visiting order of more than CHUNK references: sorted chunks, merge passes
// and the gather.  The key and index runs ping-pong between (slbk, sk) and
// (slbeb, slbe viewed as uint32): both are rewritten by the gather at the
// end, which reads the final indices from sk (so the chunks are sorted into
// the buffer that the last merge pass leaves in sk).
static int launch_order_large(int64_t n, int64_t nQ, const double *ed2, const double *lbk, const double *lbeb,
                              const double *lbe, uint32_t *sk, double *slbk, double *slbeb, double *slbe, int L,
                              int Wp, uint32_t *prefix, hipStream_t st)
{
    const int64_t nchunks = ceil_div(n, CHUNK);
    int passes = 0;
    while (((int64_t)CHUNK << passes) < n) ++passes;
    double *kb[2] = {slbk, slbeb};
    uint32_t *xb[2] = {sk, reinterpret_cast<uint32_t *>(slbe)};
    int cur = passes & 1;                                    // after `passes` swaps the runs are in buffer 0
    if (nchunks * nQ > 0x7FFFFFFFLL) return fail(NNDTW_EUNSUP, "visiting-order sort: too many chunks");
    const size_t lds = (size_t)CHUNK * 12;
    hipLaunchKernelGGL(chunk_sort_kernel, dim3((unsigned)(nchunks * nQ)), dim3(CHUNK_NT), lds, st, n, nchunks, ed2,
                       kb[cur], xb[cur]);
    NNDTW_LAUNCH_CHECK("chunk sort kernel launch");
    const int64_t blocks = std::min<int64_t>(ceil_div(nQ * n, 256), 256 * 64);
    for (int p = 0; p < passes; ++p) {
        hipLaunchKernelGGL(merge_pass_kernel, dim3((unsigned)blocks), dim3(256), 0, st, nQ, n, (int64_t)CHUNK << p,
                           kb[cur], xb[cur], kb[cur ^ 1], xb[cur ^ 1]);
        NNDTW_LAUNCH_CHECK("merge pass kernel launch");
        cur ^= 1;
    }
    hipLaunchKernelGGL(gather_bounds_kernel, dim3((unsigned)blocks), dim3(256), 0, st, nQ, n, sk, lbk, lbeb, lbe,
                       slbk, slbeb, slbe);
    NNDTW_LAUNCH_CHECK("gather kernel launch");
    return launch_cells_prefix(L, Wp, prefix, st);
}

static int launch_order(bool rank, int64_t n, int64_t nQ, const double *ed2, const double *lbk,
                        const double *lbeb, const double *lbe, uint32_t *sk, double *slbk, double *slbeb,
                        double *slbe, int L, int Wp, uint32_t *prefix, hipStream_t st)
{
    if (rank) {
        const int64_t nblk = ceil_div(n, RANK_BLOCK);
        hipLaunchKernelGGL(rank_order_kernel, dim3((unsigned)(nQ * nblk)), dim3(RANK_WAVES * WAVE), rank_lds(n), st,
                           (int)n, (int)nblk, ed2, lbk, lbeb, lbe, sk, slbk, slbeb, slbe, L, Wp, prefix);
        NNDTW_LAUNCH_CHECK("rank order kernel launch");
        return NNDTW_OK;
    }
    if (n > CHUNK) return launch_order_large(n, nQ, ed2, lbk, lbeb, lbe, sk, slbk, slbeb, slbe, L, Wp, prefix, st);
    const int Wd = order_width(n);
    const size_t lds = (size_t)ORDER_THREADS * Wd * ORDER_LDS_PER_POSITION;
    switch (Wd) {
#define NNDTW_ORDER_CASE(WW, EE, NT)                                                                     \
    case WW:                                                                                             \
        hipLaunchKernelGGL((order_kernel<EE, NT>), dim3((unsigned)nQ), dim3(NT), lds, st, n, ed2, lbk, lbeb, \
                           lbe, sk, slbk, slbeb, slbe, L, Wp, prefix);                                   \
        break;
        NNDTW_FOR_EACH_SORT(NNDTW_ORDER_CASE)
#undef NNDTW_ORDER_CASE
    default:
        return fail(NNDTW_EUNSUP, "order: %lld references exceed the supported maximum", (long long)n);
    }
    NNDTW_LAUNCH_CHECK("order kernel launch");
    return NNDTW_OK;
}

// ------------------------------------------------------------ search


__device__ __forceinline__ bool lexless(double d, int64_t k, double bd, int64_t bk)
{
    return bk < 0 || d < bd || (d == bd && k < bk);
}

__device__ __forceinline__ int64_t wave_sum(int64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// The stage whose bound prunes (0: the candidate survives).  b1, b2, b3 are
// the cascade's bounds in the order they are tested: LB_Keogh, LB_Enhanced
// bands part, full LB_Enhanced for the paper's cascades; for the comparison
// cascades b1 holds LB_Kim / LB_New / LB_Keogh (LB_Improved's first pass) and
// b3 LB_Improved / the symmetric LB_Enhanced.
__device__ __forceinline__ int stage_of(int cascade, double b1, double b2, double b3, double thr)
{
    switch (cascade) {
    case NNDTW_CASCADE_KEOGH:
    case NNDTW_CASCADE_KIM:
    case NNDTW_CASCADE_NEW:
        return b1 > thr ? 1 : 0;
    case NNDTW_CASCADE_KEOGH_ENH:
        return b1 > thr ? 1 : (b2 > thr ? 2 : (b3 > thr ? 3 : 0));
    case NNDTW_CASCADE_ENH:
    case NNDTW_CASCADE_ENH_SYM:
        return b2 > thr ? 2 : (b3 > thr ? 3 : 0);
    case NNDTW_CASCADE_IMPROVED:
        return b1 > thr ? 1 : (b3 > thr ? 3 : 0);
    default:
        return 0;
    }
}

// One workgroup of NW waves per query.  All waves run the same control flow
// on identical values (the scan, the thresholds, the record); only wave 0
// writes shared LDS state and counts.  Staging and DTW tasks are spread over
// all waves (tasks dealt from an LDS counter).
// RK: which FP64 recheck engine the code holds: 1 one diagonal pair per lane
// (windows of up to 63 pairs), 2 the FP32 engine's C pairs per lane, 0 both
// (chosen at run time).  A kernel holding one of them needs fewer registers.
// S > 0: the row-strip engine (strip_engine.hpp, S columns per lane, one
// candidate per wave) runs both the FP32 DTWs and the FP64 rechecks instead
// (C, EXACT and RK are then unused); WIN: the window constrains.
// SHARE: the code of shared batches (helper workgroups) is compiled in.
template <int C, bool EXACT, int RK = 0, int S = 0, bool WIN = true, bool SHARE = true>
__device__ __forceinline__ void search_query(const SearchArgs &a, const int64_t q, unsigned char *smem)
{
    const EngineGeom &geo = a.geo, &geoD = a.geoD;
    const int PD = a.PD, SLOTS = a.SLOTS;
    // the query row serves both engines: stage the longer of their rows
    const int LENA = S > 0 ? geo.L : staged_len(geo, geoD);
    constexpr int DG = prefetch_global(C), MG = window_global(C), DD = recheck_prefetch(C), MD = recheck_window(C);
    float *aF = reinterpret_cast<float *>(smem);
    double *resD = reinterpret_cast<double *>(aF + ((LENA + 1) & ~1));
    float *resF = reinterpret_cast<float *>(resD + PD);
    int *trunF = reinterpret_cast<int *>(resF + SLOTS);
    int *trunD = trunF + SLOTS;
    uint32_t *ring = reinterpret_cast<uint32_t *>(trunD + PD);
    uint32_t *rq = ring + QCAP;      // qualifying candidates of a batch
    int *next_task = reinterpret_cast<int *>(rq + SLOTS);
    unsigned *run_thr = reinterpret_cast<unsigned *>(next_task + 1);
    int *flags = reinterpret_cast<int *>(run_thr + 1);    // [0] shared batch, [1] wait timed out

    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & (WAVE - 1);
    const bool w0 = tid < WAVE;
    const int64_t N = a.n;
    const int L = geo.L;
    const int64_t qo = q * N;
    constexpr bool SH = SHARE;
    QueryShare *const sh = (SH && a.share != nullptr) ? a.share + q : nullptr;
    uint32_t seq = 0;                    // shared batches of this query so far
    // A candidate's FP32 row is read straight from the padded copy: element e
    // of the row the engines see is series index base0 - PADL + e (base0 is
    // the same in both geometries).
    const float *Bp = a.Bp + (a.padl + geo.base0 - Stage<C>::PADL);
    const double INF = __builtin_inf();
    const unsigned long long lt_mask = (1ull << lane) - 1ull;
    const int rot_phase = rotation_phase(a.ncu);

    if constexpr (S > 0) {
        for (int e = tid; e < L; e += nthr) aF[e] = a.Q[q * L + e];
    } else {
        EngineGeom ga = geo;
        ga.LEN = LENA;
        stage_rows<float, C>(aF, a.Q, [&](int) { return q; }, 1, ga, tid, nthr);
    }
    // Smallest completed FP32 result so far, widened by the FP32 error slack
    // (see the recheck rule below): a DTW whose frontier exceeds it cannot tie
    // or beat that result, so it is abandoned.  Pruning still uses thr.
    if (tid == 0) {
        *run_thr = __float_as_uint(__builtin_inff());
        flags[1] = 0;
        if (sh != nullptr)
            __hip_atomic_store(&sh->started, a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();

    const double ub = a.init_ub ? a.ed2[qo + a.sk[qo]] : INF;
    double bsf = INF;
    int64_t bk = -1;
    int64_t c_pk = 0, c_peb = 0, c_pe = 0, c_st = 0, c_ab = 0, c_rc = 0, c_cells = 0;
    int qh = 0, qt = 0;
    int64_t cached = -1;                 // chunk start whose bounds the lanes hold
    uint32_t ck = 0;
    double cbk = 0.0, cbb = 0.0, cbe = 0.0;
    const int s_start = 2 * geo.base0 + geo.Wp;

    int64_t pos = 0;
    while (pos < N) {
        const double thr = __builtin_fmin(bsf, ub) * (1.0 + a.eps);
        const float thrF = round_up_f32(thr);
        double rb = INF;
        int64_t rk = -1;

        // Run up to SLOTS queued survivors through the FP32 engine (groups
        // refill as candidates end), then recompute in FP64 the completed
        // results that can decide the round.
        auto run_batch = [&](int nt) {
            const int h0 = qh;
            // A batch is shared with the query's helper workgroups (see
            // help_query) once one has joined; until then it stays in LDS.
            if (sh != nullptr) {
                if (tid == 0) {
                    const unsigned hv = __hip_atomic_load(&sh->helpers, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    flags[0] = ((hv >> 12) == a.epoch && (hv & 0xFFFu) != 0u) ? 1 : 0;
                }
            }
            if (tid == 0) *next_task = 0;
            __syncthreads();
            bool shared = false;
            if constexpr (SH) shared = sh != nullptr && __builtin_amdgcn_readfirstlane(flags[0]) != 0;
            uint32_t tag = 0u;
            if (shared) {
                // publish the batch (candidates, size, threshold, a zero
                // count), then its tag: the stores are complete before the
                // tag is, so a workgroup that sees the tag reads this batch
                ++seq;
                tag = (a.epoch << 12) | (seq & 0xFFFu);
                for (int i = tid; i < nt; i += nthr)
                    __hip_atomic_store(&sh->cand[i], ring[(h0 + i) % QCAP], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (tid == 0) {
                    __hip_atomic_store(&sh->nt, (unsigned)nt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&sh->thrF, __float_as_uint(thrF), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&sh->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                if (tid == 0) {
                    __hip_atomic_store(&sh->deal, (unsigned long long)tag << 32, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    __builtin_amdgcn_s_waitcnt(0);
                }
                __syncthreads();
            }
            // candidate row of task i (a shared batch reads the published list)
            auto cand_of = [&](int i) -> uint32_t {
                return shared ? __hip_atomic_load(&sh->cand[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                              : ring[(h0 + i) % QCAP];
            };
            if constexpr (S > 0) {
                // trunF receives the band cells each task evaluated
                strip_run<float, S, WIN>(
                    L, geo.Wp, nt, next_task, [&](int) { return (const float *)aF; },
                    [&](int i) { return a.B + (int64_t)cand_of(i) * L; }, [&](int) { return thrF; },
                    shared ? reinterpret_cast<float *>(sh->res) : resF, shared ? sh->trun : trunF, run_thr,
                    1.0 + 2.0 * a.eps, rot_phase, shared ? &sh->deal : nullptr, tag, shared ? &sh->done : nullptr);
            } else {
                TaskOut<float> to{resF, trunF, run_thr, 1.0 + 2.0 * a.eps, rot_phase};
                if (shared) {
                    to.res = reinterpret_cast<float *>(sh->res);
                    to.trun = sh->trun;
                    to.deal64 = &sh->deal;
                    to.tag = tag;
                    to.done = &sh->done;
                }
                engine_run<float, C, DG, MG, EXACT>(
                    geo, nt, next_task, [&](int) { return (const float *)aF; },
                    [&](int i) { return Bp + (int64_t)cand_of(i) * a.ppitch; }, [&](int) { return thrF; }, to);
            }
            if (shared) {
                // every task dealt has been taken by a running workgroup:
                // wait until all are counted (bounded; a time-out is
                // reported as index -2)
                if (tid == 0) {
                    int spins = 0;
                    while (__hip_atomic_load(&sh->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)nt) {
                        __builtin_amdgcn_s_sleep(2);
                        if (++spins > (1 << 22)) {
                            flags[1] = 1;
                            break;
                        }
                    }
                }
                __syncthreads();
                for (int i = tid; i < nt; i += nthr) {
                    resF[i] = __uint_as_float(__hip_atomic_load(&sh->res[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                    trunF[i] = __hip_atomic_load(&sh->trun[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            __syncthreads();
            // the batch's results, 64 tasks per pass: counts and the
            // smallest completed FP32 result
            float mn = __builtin_inff();
            for (int j0 = 0; j0 < nt; j0 += WAVE) {
                const int j = j0 + lane;
                if (j < nt) {
                    const float d32 = resF[j];
                    const int tr = trunF[j];
                    const bool ab = __builtin_isinf(d32);
                    c_ab += ab;
                    if constexpr (S > 0) {
                        c_cells += tr;
                    } else {
                        int s_last = s_start + 2 * (tr - 1) + 1;
                        if (s_last > 2 * L - 2) s_last = 2 * L - 2;
                        c_cells += s_last >= 0 ? (int64_t)a.prefix[s_last] : 0;
                    }
                    if (!ab && (double)d32 <= thr) mn = __builtin_fminf(mn, d32);
                }
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) mn = __builtin_fminf(mn, __shfl_xor(mn, off));
            // the completed results that can decide the round, in batch order
            int nq = 0;
            for (int j0 = 0; j0 < nt; j0 += WAVE) {
                const int j = j0 + lane;
                bool qual = false;
                uint32_t kg = 0;
                if (j < nt) {
                    const float d32 = resF[j];
                    qual = !__builtin_isinf(d32) && (double)d32 <= thr &&
                           (double)d32 <= (double)mn * (1.0 + 2.0 * a.eps);
                    kg = ring[(h0 + j) % QCAP];
                }
                const unsigned long long qm = __ballot(qual);
                if (w0 && qual) rq[nq + __popcll(qm & lt_mask)] = kg;
                nq += __popcll(qm);
            }
            qh += nt;
            __syncthreads();                 // every wave has read the batch results
            // FP64 recheck: the same float rows, widened exactly at load (the
            // pad 1e30 squares to 1e60 in FP64, still far above any path sum
            // of finite inputs below 1e15, so every min and sum is unchanged)
            for (int b0 = 0; b0 < nq; b0 += PD) {
                const int nd = (nq - b0) < PD ? (nq - b0) : PD;
                __syncthreads();
                if (tid == 0) *next_task = 0;
                __syncthreads();
                // every wave of the workgroup waits for these few FP64
                // sweeps: run them at the top wave priority, so that the
                // waves of other workgroups sharing the SIMD do not stretch
                // this query's critical path
                __builtin_amdgcn_s_setprio(3);
                if constexpr (S > 0) {
                    strip_run<double, S, WIN>(
                        L, geo.Wp, nd, next_task, [&](int) { return (const float *)aF; },
                        [&](int i) { return a.B + (int64_t)rq[b0 + i] * L; }, [&](int) { return thr; }, resD,
                        trunD);
                } else if (RK == 1 || (RK == 0 && C > 1 && geoD.C == 1)) {
                    // one pair per lane: rows start C - 1 elements later
                    constexpr int D1 = recheck_prefetch(1), M1 = recheck_window(1);
                    engine_run<double, 1, D1, M1, true>(
                        geoD, nd, next_task, [&](int) { return (const float *)aF + (C - 1); },
                        [&](int i) { return Bp + (C - 1) + (int64_t)rq[b0 + i] * a.ppitch; },
                        [&](int) { return thr; }, TaskOut<double>{resD, trunD});
                } else {
                    engine_run<double, C, DD, MD, EXACT>(
                        geoD, nd, next_task, [&](int) { return (const float *)aF; },
                        [&](int i) { return Bp + (int64_t)rq[b0 + i] * a.ppitch; }, [&](int) { return thr; },
                        TaskOut<double>{resD, trunD});
                }
                __builtin_amdgcn_s_setprio(0);
                __syncthreads();
                for (int i = 0; i < nd; ++i) {
                    const double d = resD[i];
                    const int64_t k = rq[b0 + i];
                    if (!__builtin_isinf(d) && d <= thr && lexless(d, k, rb, rk)) { rb = d; rk = k; }
                }
                c_rc += (lane == 0) ? nd : 0;
            }
            __syncthreads();
        };

        // Scan the visiting order in aligned chunks of 64 positions (bounds
        // cached in registers across rounds) for the first round that has a
        // survivor; rounds before it are wholly pruned.
        int64_t scan = pos, re = -1;
        while (scan < N) {
            const int64_t c0 = scan & ~(int64_t)(WAVE - 1);
            const int64_t p = c0 + lane;
            if (c0 != cached) {
                cached = c0;
                if (p < N) {
                    ck = a.sk[qo + p];
                    cbk = a.slbk[qo + p];
                    cbb = a.slbeb[qo + p];
                    cbe = a.slbe[qo + p];
                }
            }
            const int st = (p >= scan && p < N) ? stage_of(a.cascade, cbk, cbb, cbe, thr) : 4;
            const unsigned long long sm = __ballot(st == 0);
            int64_t lim;
            if (re < 0) {
                if (sm == 0ull) {
                    lim = c0 + WAVE;
                } else {
                    const int64_t f = c0 + __ffsll((long long)sm) - 1;
                    const int64_t rs = (f / a.R) * a.R;
                    re = (rs + a.R) < N ? (rs + a.R) : N;
                    lim = re < c0 + WAVE ? re : c0 + WAVE;
                }
            } else {
                lim = re < c0 + WAVE ? re : c0 + WAVE;
            }
            const bool use = st != 4 && p < lim;
            if (use) {
                c_pk += st == 1;
                c_peb += st == 2;
                c_pe += st == 3;
            }
            const unsigned long long em = __ballot(use && st == 0);
            if (w0 && use && st == 0) ring[(qt + __popcll(em & lt_mask)) % QCAP] = ck;
            c_st += use && st == 0;
            qt += __popcll(em);
            __syncthreads();
            while (qt - qh >= SLOTS) run_batch(SLOTS);
            scan = c0 + WAVE;
            if (re >= 0 && scan >= re) break;
        }
        if (re < 0) break;     // every remaining candidate was pruned
        while (qt > qh) run_batch((qt - qh) < SLOTS ? (qt - qh) : SLOTS);
        if (rk >= 0 && lexless(rb, rk, bsf, bk)) { bsf = rb; bk = rk; }
        pos = re;
    }

    if (sh != nullptr && tid == 0)
        __hip_atomic_store(&sh->finished, a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!w0) return;
    c_pk = wave_sum(c_pk);
    c_peb = wave_sum(c_peb);
    c_pe = wave_sum(c_pe);
    c_st = wave_sum(c_st);
    c_ab = wave_sum(c_ab);
    c_rc = wave_sum(c_rc);
    c_cells = wave_sum(c_cells);
    if (lane == 0) {
        a.nn_idx[q] = flags[1] ? -2 : bk;
        a.nn_dist[q] = bsf;
        if (a.counts) {
            int64_t *c = a.counts + q * NNDTW_NCOUNTS;
            c[NNDTW_COUNT_N] = N;
            c[NNDTW_COUNT_PRUNED_KEOGH] = c_pk;
            c[NNDTW_COUNT_PRUNED_BANDS] = c_peb;
            c[NNDTW_COUNT_PRUNED_ENH] = c_pe;
            c[NNDTW_COUNT_DTW_STARTED] = c_st;
            c[NNDTW_COUNT_DTW_ABANDONED] = c_ab;
            c[NNDTW_COUNT_CELLS] = c_cells;
            c[NNDTW_COUNT_RECHECKS] = c_rc;
        }
    }
}

// A helper workgroup of query q: it takes DTW tasks of the query's shared
// FP32 batches (QueryShare) until the query finishes.  The owner never waits
// for a helper: it shares a batch only once a helper has joined, and then
// waits only for tasks that a running workgroup has taken.  A helper that
// finds its query finished, or not started, or `cap` helpers already joined,
// leaves at once.
template <int C, bool EXACT, int S = 0, bool WIN = true>
__device__ __forceinline__ void help_query(const SearchArgs &a, const int64_t q, unsigned char *smem,
                                           unsigned cap = 0xFFFu)
{
    const EngineGeom &geo = a.geo, &geoD = a.geoD;
    const int LENA = S > 0 ? geo.L : staged_len(geo, geoD);
    constexpr int DG = prefetch_global(C), MG = window_global(C);
    float *aF = reinterpret_cast<float *>(smem);
    int *ctl = reinterpret_cast<int *>(aF + ((LENA + 1) & ~1));   // next task, go, nt, threshold, tag
    const int tid = threadIdx.x, nthr = blockDim.x;
    QueryShare *const sh = a.share + q;
    if (tid == 0) {
        int go = 0;
        // the owner may be starting at the same time: wait for it briefly
        // (a few hundred microseconds), but never for an owner that is not
        // running yet
        bool started = false;
        for (int k = 0; k < 256 && !started; ++k) {
            started = __hip_atomic_load(&sh->started, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == a.epoch;
            if (!started) __builtin_amdgcn_s_sleep(16);
        }
        if (started && __hip_atomic_load(&sh->finished, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != a.epoch) {
            unsigned cur = __hip_atomic_load(&sh->helpers, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            go = 1;
            while (true) {
                const bool mine = (cur >> 12) == a.epoch;
                if (mine && (cur & 0xFFFu) >= cap) {
                    go = 0;
                    break;
                }
                const unsigned want = mine ? cur + 1u : ((a.epoch << 12) | 1u);
                if (__hip_atomic_compare_exchange_strong(&sh->helpers, &cur, want, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    break;
            }
        }
        ctl[1] = go;
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(ctl[1]) == 0) return;
    if constexpr (S > 0) {
        for (int e = tid; e < geo.L; e += nthr) aF[e] = a.Q[q * geo.L + e];
    } else {
        EngineGeom ga = geo;
        ga.LEN = LENA;
        stage_rows<float, C>(aF, a.Q, [&](int) { return q; }, 1, ga, tid, nthr);
    }
    const float *Bp = a.Bp + (a.padl + geo.base0 - Stage<C>::PADL);
    const int64_t N = a.n;
    uint32_t last = 0u;
    int idle = 0;
    while (true) {
        __syncthreads();
        if (tid == 0) {
            int go = 0;
            const unsigned long long d = __hip_atomic_load(&sh->deal, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t tag = (uint32_t)(d >> 32);
            if (__hip_atomic_load(&sh->finished, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == a.epoch) {
                go = -1;
            } else if ((tag >> 12) == a.epoch && tag != last) {
                const unsigned nt = __hip_atomic_load(&sh->nt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((uint32_t)d < nt && nt <= (unsigned)SHARE_SLOTS) {
                    go = 1;
                    ctl[2] = (int)nt;
                    ctl[3] = (int)__hip_atomic_load(&sh->thrF, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ctl[4] = (int)tag;
                }
            }
            ctl[1] = go;
            ctl[0] = 0;
        }
        __syncthreads();
        const int go = __builtin_amdgcn_readfirstlane(ctl[1]);
        if (go < 0) break;
        if (go > 0) {
            const uint32_t tag = (uint32_t)__builtin_amdgcn_readfirstlane(ctl[4]);
            const float thrF = __uint_as_float((unsigned)__builtin_amdgcn_readfirstlane(ctl[3]));
            const int nt = __builtin_amdgcn_readfirstlane(ctl[2]);
            auto cand_of = [&](int i) -> int64_t {
                uint32_t k = __hip_atomic_load(&sh->cand[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return k < (uint32_t)N ? k : 0;       // an index of the set (the owner writes only such)
            };
            if constexpr (S > 0) {
                strip_run<float, S, WIN>(geo.L, geo.Wp, nt, ctl, [&](int) { return (const float *)aF; },
                                         [&](int i) { return a.B + cand_of(i) * geo.L; }, [&](int) { return thrF; },
                                         reinterpret_cast<float *>(sh->res), sh->trun, nullptr, 1.0, -1, &sh->deal,
                                         tag, &sh->done);
            } else {
                engine_run<float, C, DG, MG, EXACT>(
                    geo, nt, ctl, [&](int) { return (const float *)aF; },
                    [&](int i) { return Bp + cand_of(i) * a.ppitch; }, [&](int) { return thrF; },
                    TaskOut<float>{reinterpret_cast<float *>(sh->res), sh->trun, nullptr, 1.0, -1, &sh->deal, tag,
                                   &sh->done});
            }
            last = tag;
            idle = 0;
        } else {
            if (++idle > (1 << 20)) break;
            __builtin_amdgcn_s_sleep(8);
        }
    }
}

// Kernels whose registers allow it (no scratch spill) are held to 128 VGPRs,
// so that two workgroups of 8 waves (a query each) share a compute unit:
// 512 queries run at once instead of 256, and a query with much more work
// than the others does not start late.  With the one-pair FP64 recheck
// (windows of up to 63 pairs) that holds up to 6 pairs per lane.
template <int C, bool EXACT, int RK>
__global__ void __launch_bounds__(WAVE * SEARCH_MAX_WAVES)
    __attribute__((amdgpu_waves_per_eu((C <= 3 || (RK == 1 && C <= 6)) ? 4 : 1)))
search_kernel(SearchArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    if constexpr (share_ok(C)) {
        if (a.share != nullptr && (int64_t)blockIdx.x >= a.nq) {
            help_query<C, EXACT>(a, ((int64_t)blockIdx.x - a.nq) % a.nq, smem);
            return;
        }
    }
    search_query<C, EXACT, RK, 0, true, share_ok(C)>(a, blockIdx.x, smem);
}

// Up to 16 waves per query for the shapes with the one-pair FP64 recheck
// and at most 6 pairs per lane (128 VGPRs): an expensive query's rounds run
// on twice the groups of lanes.
template <int C, bool EXACT>
__global__ void __launch_bounds__(WAVE * SEARCH_WIDE_WAVES) __attribute__((amdgpu_waves_per_eu(4)))
search_kernel_wide(SearchArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    if constexpr (share_ok(C)) {
        if (a.share != nullptr && (int64_t)blockIdx.x >= a.nq) {
            help_query<C, EXACT>(a, ((int64_t)blockIdx.x - a.nq) % a.nq, smem);
            return;
        }
    }
    search_query<C, EXACT, C == 1 ? 2 : 1, 0, true, share_ok(C)>(a, blockIdx.x, smem);
}

// Resets the shared-batch headers of nq queries (before a search with
// helper workgroups, so that nothing left in the workspace matches the call).
__global__ void __launch_bounds__(256) share_reset_kernel(QueryShare *share, int64_t nq)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nq) share_clear(share[q]);
}

// Whether a plan may use more than SEARCH_MAX_WAVES waves (search_kernel_wide).
static bool wide_ok(int C, int Wp) { return C <= 6 && recheck_cpl(Wp, C) == 1; }

// The search with the row-strip engine (wide windows): one candidate per
// wave.  Up to 8 waves per query for strips of up to 16 columns; wider
// strips hold up to 256 registers per lane in FP64, one wave per SIMD, so
// their workgroups have at most 4 waves.
__host__ __device__ constexpr int strip_search_waves(int S) { return S <= 16 ? SEARCH_MAX_WAVES : 4; }

template <int S, bool WIN>
__global__ void __launch_bounds__(WAVE * strip_search_waves(S))
search_kernel_strip(SearchArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    if (a.share != nullptr && (int64_t)blockIdx.x >= a.nq) {
        help_query<1, false, S, WIN>(a, ((int64_t)blockIdx.x - a.nq) % a.nq, smem);
        return;
    }
    search_query<1, false, 2, S, WIN>(a, blockIdx.x, smem);
}

// The search of a batch: persistent workgroups take (set, query) items of
// one engine shape (C, EXACT) from that shape's counter in the batch header,
// in the order of the item list (largest expected work first).  One launch
// per shape present: a kernel with several engine bodies would need the
// register count of their union.  The counters are reset by the batch's
// bound pass.
// SHARE: once the items are all taken, a workgroup lends itself to the
// queries still running (help_query, at most `cap` helpers per query).
// Every workgroup records the item it runs in running[blockIdx.x]; an idle
// one keeps drawing from the counter, and draw h past the end names the item
// of workgroup h mod gridDim.x, until it finds a query not finished and
// below the cap, or `probes` draws past the end have been made in all.  Each
// item's helper header (QueryShare) is reset before the launch.
template <int C, bool EXACT, bool SHARE>
__global__ void __launch_bounds__(WAVE * SEARCH_MAX_WAVES)
batch_search_kernel(const BatchSet *__restrict__ sets, const int64_t *__restrict__ items, int64_t nitems,
                    unsigned *counter, unsigned *running, unsigned cap, unsigned probes)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int64_t cur;
    while (true) {
        __syncthreads();                 // the previous item is finished by every wave
        if (threadIdx.x == 0) {
            cur = (int64_t)atomicAdd(counter, 1u);
            if constexpr (SHARE)
                __hip_atomic_store(&running[blockIdx.x], cur < nitems ? (unsigned)cur + 1u : 0u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        const int64_t i = cur;
        if (i >= nitems) break;
        const int64_t it = items[i];
        const int d = __builtin_amdgcn_readfirstlane((int)(it >> 32));
        search_query<C, EXACT, 0, 0, true, SHARE>(sets[d].a, it & 0xFFFFFFFF, smem);
    }
    if constexpr (SHARE) {
        const unsigned G = gridDim.x;
        while (true) {
            __syncthreads();
            if (threadIdx.x == 0) {
                int64_t found = -1;
                for (unsigned k = 0; k < G; ++k) {
                    const unsigned drawn = atomicAdd(counter, 1u);
                    if ((int64_t)drawn < nitems) break;          // not reached: the items are all taken
                    const unsigned h = drawn - (unsigned)nitems;
                    if (h >= probes) break;
                    const unsigned r =
                        __hip_atomic_load(&running[h % G], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (r == 0u || (int64_t)r > nitems) continue;
                    const int64_t j = (int64_t)r - 1;
                    const int64_t it = items[j];
                    const SearchArgs &aj = sets[(int)(it >> 32)].a;
                    const QueryShare *sh = aj.share + (it & 0xFFFFFFFF);
                    // not finished and not at the cap (a query whose owner
                    // has not written `started` yet is about to: every item
                    // has been taken by a running workgroup)
                    const unsigned hv = __hip_atomic_load(&sh->helpers, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (__hip_atomic_load(&sh->finished, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != aj.epoch &&
                        !((hv >> 12) == aj.epoch && (hv & 0xFFFu) >= cap)) {
                        found = j;
                        break;
                    }
                }
                cur = found;
            }
            __syncthreads();
            const int64_t j = cur;
            if (j < 0) break;
            const int64_t it = items[j];
            const int d = __builtin_amdgcn_readfirstlane((int)(it >> 32));
            help_query<C, EXACT>(sets[d].a, it & 0xFFFFFFFF, smem, cap);
        }
    }
}

int launch_batch_search(int C, bool exact, const BatchSet *sets, const int64_t *items, int64_t nitems,
                        unsigned *counter, unsigned *running, int waves, int grid, size_t lds, int helpers,
                        hipStream_t st)
{
    if (nitems == 0) return NNDTW_OK;
    if (grid > BATCH_MAX_GRID) return fail(NNDTW_EINVAL, "batch search: grid %d above %d", grid, BATCH_MAX_GRID);
    const unsigned cap = helpers > 0 ? (unsigned)helpers : 0u;
    // draws past the end in all: every workgroup's slot probed 64 times over
    const unsigned probes = 64u * (unsigned)grid;
    switch (C * 4 + (exact ? 2 : 0) + (helpers > 0 ? 1 : 0)) {
#define NNDTW_BSEARCH_CASE(c, e, h)                                                                            \
    case c * 4 + e * 2 + h:                                                                                   \
        hipLaunchKernelGGL((batch_search_kernel<c, e, h>), dim3((unsigned)grid), dim3(WAVE * waves), lds, st, sets, \
                           items, nitems, counter, running, cap, probes);                                     \
        break;
        NNDTW_BSEARCH_CASE(1, 0, 0)
        NNDTW_BSEARCH_CASE(1, 0, 1)
        NNDTW_BSEARCH_CASE(1, 1, 0)
        NNDTW_BSEARCH_CASE(1, 1, 1)
        NNDTW_BSEARCH_CASE(2, 0, 0)
        NNDTW_BSEARCH_CASE(2, 0, 1)
        NNDTW_BSEARCH_CASE(2, 1, 0)
        NNDTW_BSEARCH_CASE(2, 1, 1)
        NNDTW_BSEARCH_CASE(3, 0, 0)
        NNDTW_BSEARCH_CASE(3, 0, 1)
        NNDTW_BSEARCH_CASE(3, 1, 0)
        NNDTW_BSEARCH_CASE(3, 1, 1)
        NNDTW_BSEARCH_CASE(4, 0, 0)
        NNDTW_BSEARCH_CASE(4, 0, 1)
        NNDTW_BSEARCH_CASE(4, 1, 0)
        NNDTW_BSEARCH_CASE(4, 1, 1)
#undef NNDTW_BSEARCH_CASE
    default:
        return fail(NNDTW_EUNSUP, "batch search: %d pairs per lane not supported", C);
    }
    NNDTW_LAUNCH_CHECK("batch search kernel launch");
    return NNDTW_OK;
}

int device_cu_count()
{
    static int cached[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (cached[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) return 0;
        cached[dev] = v;
    }
    return cached[dev];
}

size_t search_lds_bytes(const EngineGeom &g, const EngineGeom &gd, int SLOTS, int PD)
{
    const int LENA = staged_len(g, gd);
    return (size_t)((LENA + 1) & ~1) * 4 + (size_t)PD * 12 + (size_t)SLOTS * 12 + QCAP * 4 + 32;
}

// Plan of the search with the row-strip engine.
static int plan_search_strip(const nndtw_refset *rs, const nndtw_search_opts *o, SearchPlan *plan)
{
    const int L = rs->L;
    const int Wp = rs->W < L - 1 ? rs->W : L - 1;
    if (o->cpl > 0) return fail(NNDTW_EINVAL, "cpl=%d: pairs per lane apply to the diagonal engine only", o->cpl);
    if (!strip_fits(L, Wp))
        return fail(NNDTW_EUNSUP, "window W=%d too narrow for the row-strip engine at L=%d (2 min(W, L-1) + 2 >= %d)",
                    rs->W, L, strip_width(L));
    const int S = strip_width(L);
    const int maxw = strip_search_waves(S);
    int NW = o->waves;
    if (NW <= 0) {
        const int cu = device_cu_count() > 0 ? device_cu_count() : 256;
        const bool few = o->nq_hint > 0 && o->nq_hint <= 2 * (int64_t)cu;
        NW = few ? maxw : (SEARCH_DEFAULT_WAVES < maxw ? SEARCH_DEFAULT_WAVES : maxw);
    }
    if (NW > maxw)
        return fail(NNDTW_EUNSUP, "waves=%d: the row-strip search takes at most %d waves per query at L=%d", NW, maxw,
                    L);
    // one candidate per wave: the same default round as the diagonal engine
    const int64_t R = o->R > 0 ? o->R : (2 * NW > 256 ? 2 * NW : 256);
    const int SLOTS = 256, PD = 64;
    const size_t lds = (size_t)((L + 1) & ~1) * 4 + (size_t)PD * 12 + (size_t)SLOTS * 12 + QCAP * 4 + 32;
    *plan = SearchPlan{};
    plan->Wp = Wp;
    plan->C = 0;
    plan->S = S;
    plan->G = WAVE;
    plan->P = 1;
    plan->PD = PD;
    plan->SLOTS = SLOTS;
    plan->NW = NW;
    plan->T = L + (L - 1) / S;
    plan->LEN = L;
    plan->R = R;
    plan->lds_bytes = lds;
    plan->helpers = o->helpers > 0 ? o->helpers : (o->helpers < 0 ? 0 : SEARCH_DEFAULT_HELPERS);
    return NNDTW_OK;
}

// The FP32 error floor of the slack (see the header): eps >= 2 gamma, with
// gamma = gamma_{2L+1} of float32.  The default and the smallest value
// accepted is twice gamma_{2L+2} = 2 n u / (1 - n u), n = 2L + 2.
static int plan_eps(int L, const nndtw_search_opts *o, SearchPlan *plan)
{
    const double nu = (double)(2 * L + 2) * 0x1p-24;
    const double eps_min = 2.0 * nu / (1.0 - nu);
    if (o->eps > 0 && o->eps < eps_min)
        return fail(NNDTW_EINVAL, "eps=%g below the FP32 error floor %.9g for L=%d (2 gamma_{2L+2})", o->eps,
                    eps_min, L);
    plan->eps = o->eps > 0 ? o->eps : eps_min;
    return NNDTW_OK;
}

int plan_search(const nndtw_refset *rs, const nndtw_search_opts *o, SearchPlan *plan, bool batched)
{
    if (o->order < NNDTW_ORDER_AUTO || o->order > NNDTW_ORDER_RANK)
        return fail(NNDTW_EINVAL, "order=%d is not an NNDTW_ORDER_* value", o->order);
    const int L = rs->L;
    const int Wp = rs->W < L - 1 ? rs->W : L - 1;
    int engine = o->engine;
    // The library's choice: strips where the diagonal shapes compiled for the
    // search cannot hold the window, and for unconstrained DTW (W' = L - 1)
    // when the strips keep at least 48 lanes busy (L > 192).  Elsewhere the
    // diagonal engine measured faster in the search, although strips do less
    // work per complete DTW from 60 % band coverage on (5000 x 500, L=512,
    // V=5, 8 waves per query: W=256 21 ms diagonal / 47 ms strips, W=450
    // 40 / 51, W=511 44 / 39): most candidates are abandoned after a third
    // of their rows, where the strips' pipeline fill and full-width rows
    // (window cells marked, not skipped) cost most, and a query's work runs
    // on one compute unit either way.
    if (engine == NNDTW_ENGINE_AUTO)
        engine = !batched && o->cpl <= 0 && strip_fits(L, Wp) &&
                         (Wp + 1 > 63 * SEARCH_MAX_CPL || (Wp >= L - 1 && L > 192))
                     ? NNDTW_ENGINE_STRIP
                     : NNDTW_ENGINE_DIAGONAL;
    if (engine == NNDTW_ENGINE_STRIP) {
        if (batched) return fail(NNDTW_EUNSUP, "the batched search runs the diagonal engine only");
        const int r = plan_search_strip(rs, o, plan);
        return r ? r : plan_eps(L, o, plan);
    }
    // Only shapes up to SEARCH_MAX_CPL pairs per lane are compiled for the
    // search: it takes windows with min(W, L-1) + 1 <= 63 * SEARCH_MAX_CPL.
    // The batched search keeps the narrow shapes even where one group fills
    // a wave (it has kernels for 1-4 pairs per lane and rejects wider ones).
    const int C = choose_cpl(Wp, 4, o->cpl, SEARCH_MAX_CPL, !batched);
    if (C < 0 && o->cpl <= 0)
        return fail(NNDTW_EUNSUP, "window W=%d too wide for the %s (min(W, L-1) + 1 <= %d)", rs->W,
                    batched ? "batched search" : "diagonal engine", 63 * SEARCH_MAX_CPL);
    if (C < 0) return fail(NNDTW_EINVAL, "no search engine shape with cpl=%d for W=%d", o->cpl, rs->W);
    EngineGeom g = make_geom(L, rs->W, C, prefetch_global(C), window_global(C));
    const EngineGeom gd = recheck_geom(L, rs->W, C);
    const int P = g.P;
    // at least one pair of series per wave, hence a round of at least one
    // candidate (the search divides positions by R)
    if (P < 1) return fail(NNDTW_EUNSUP, "no DTW engine shape for W=%d with %d pairs per lane", rs->W, C);
    // Waves per query: a query's rounds are a chain of dependent steps, so the
    // kernel lasts as long as its most expensive query (on the 5000 x 500,
    // L=512 workload one query does 3.7 times the mean work).  When the
    // queries do not fill the device at 4 waves each, each gets 8,
    // or 16 where the shape fits 128 VGPRs (5000 x 500, L=512, W=51: search
    // kernel 5.1 ms at 4 waves, 3.3 ms at 8, 2.5 ms at 16).
    int NW = o->waves;
    if (NW <= 0) {
        const int cu = device_cu_count() > 0 ? device_cu_count() : 256;
        const bool few = o->nq_hint > 0 && o->nq_hint <= 2 * (int64_t)cu;
        NW = few ? (!batched && wide_ok(C, Wp) ? SEARCH_WIDE_WAVES : 8) : SEARCH_DEFAULT_WAVES;
    }
    if (NW > SEARCH_MAX_WAVES && (batched || !wide_ok(C, Wp)))
        return fail(NNDTW_EUNSUP, "waves=%d: more than %d waves per query need a window of at most 63 diagonal "
                                  "pairs and at most 6 pairs per lane (W=%d, %d pairs per lane)%s",
                    NW, SEARCH_MAX_WAVES, rs->W, C, batched ? "; the batched search takes at most 8" : "");
    // Default round: two candidates per group, so that groups whose
    // candidate is abandoned early take another one within the round, and
    // at least 256: each round is a serial step of the query (threshold,
    // DTWs, FP64 recheck), and below that the chain of rounds cost more
    // than the extra DTWs a larger round starts on the measured workloads.
    // (With more than 8 waves a round of 512 measured faster: 3.40 -> 3.29 ms
    // for the search on the workload above.)
    int64_t R = o->R > 0 ? o->R : (2 * P * NW > 256 ? 2 * P * NW : 256);
    if (o->R <= 0 && NW > SEARCH_MAX_WAVES && R < 512) R = 512;
    // Candidates per FP32 batch: the round, up to 256, so that a round of
    // the default size is one batch (every batch ends waiting for its
    // longest DTW); up to 64 FP64 rechecks per engine call.  Only the query
    // row and bookkeeping live in LDS.
    const int SLOTS = 256;
    const int PD = 64;
    const size_t lds = search_lds_bytes(g, gd, SLOTS, PD);
    if (lds > 160 * 1024) return fail(NNDTW_EUNSUP, "series length %d too long for the search", L);
    // the engines read padded rows [base0 - PADL, base0 - PADL + LEN) of Bp
    const int64_t boff = rs->padl + g.base0 - C;
    const int LENA = staged_len(g, gd);
    if (g.base0 != gd.base0 || boff < 0 || boff + LENA > rs->ppitch)
        return fail(NNDTW_EUNSUP, "reference set margins too narrow for the DTW engine shape");
    plan->Wp = Wp;
    plan->C = C;
    plan->G = g.G;
    plan->P = P;
    plan->PD = PD;
    plan->SLOTS = SLOTS;
    plan->NW = NW;
    plan->exact = g.exact;
    plan->T = g.T;
    plan->LEN = g.LEN;
    plan->R = R;
    plan->S = 0;
    // Helper workgroups per query (help_query): they start once the owners
    // have been dispatched, so they serve the queries still running then,
    // which are the heavy ones (the kernel lasts as long as its heaviest
    // query).  Not in the batched search (persistent workgroups).
    plan->helpers = (batched || !share_ok(C)) ? 0
                                               : (o->helpers > 0 ? o->helpers
                                                                 : (o->helpers < 0 ? 0 : SEARCH_DEFAULT_HELPERS));
    plan->lds_bytes = lds;
    return plan_eps(L, o, plan);
}

int launch_search(const nndtw_refset *rs, const float *Qy, int64_t nQ, const nndtw_search_opts *o,
                  const SearchPlan &plan, int64_t *nn_idx, double *nn_dist, int64_t *counts, void *ws,
                  hipStream_t st)
{
    if (nQ == 0) return NNDTW_OK;
    const int64_t n = rs->n;
    const int L = rs->L;
    const WsLayout w = ws_layout(nQ, n, L);
    unsigned char *base = (unsigned char *)ws;
    double *ed2 = (double *)(base + w.ed2), *lbk = (double *)(base + w.lbk);
    double *lbeb = (double *)(base + w.lbeb), *lbe = (double *)(base + w.lbe);
    uint32_t *sk = (uint32_t *)(base + w.sk);
    double *slbk = (double *)(base + w.slbk), *slbeb = (double *)(base + w.slbeb);
    double *slbe = (double *)(base + w.slbe);
    uint32_t *prefix = (uint32_t *)(base + w.prefix);

    bool rank = false;                        // decided before anything is enqueued
    if (int r = order_by_rank(o->order, (double)nQ * (double)n * (double)n, n, nQ, &rank)) return r;
    hipEvent_t *ev = o->events ? (hipEvent_t *)o->events : nullptr;
    auto mark = [&](int i) -> int {
        if (!ev) return NNDTW_OK;
        hipError_t e = hipEventRecord(ev[i], st);
        return e == hipSuccess ? NNDTW_OK : hip_fail(e, "stage event record");
    };
    int r = mark(0);
    if (r) return r;
    r = launch_cascade_bounds(rs, Qy, nQ, o->V, ed2, lbk, lbeb, lbe, st);
    if (r) return r;
    // comparison cascades: their bound replaces b1 or b3 (see stage_of)
    switch (o->cascade) {
    case NNDTW_CASCADE_KIM: r = launch_compare_bounds(0, Qy, nQ, rs->B, rs->U, rs->Lo, n, L, rs->W, o->V, nullptr,
                                                      NNDTW_CROSS, lbk, st); break;
    case NNDTW_CASCADE_IMPROVED: r = launch_compare_bounds(1, Qy, nQ, rs->B, rs->U, rs->Lo, n, L, rs->W, o->V,
                                                           nullptr, NNDTW_CROSS, lbe, st); break;
    case NNDTW_CASCADE_NEW: r = launch_compare_bounds(2, Qy, nQ, rs->B, rs->U, rs->Lo, n, L, rs->W, o->V, nullptr,
                                                      NNDTW_CROSS, lbk, st); break;
    case NNDTW_CASCADE_ENH_SYM: r = launch_compare_bounds(3, Qy, nQ, rs->B, rs->U, rs->Lo, n, L, rs->W, o->V,
                                                          nullptr, NNDTW_CROSS, lbe, st); break;
    default: break;
    }
    if (r) return r;
    if ((r = mark(1))) return r;
    // (the cells table is filled by the ordering kernel: events 1 and 2 mark the same point)
    if ((r = mark(2))) return r;
    if ((r = launch_order(rank, n, nQ, ed2, lbk, lbeb, lbe, sk, slbk, slbeb, slbe, L, plan.Wp, prefix, st))) return r;
    if ((r = mark(3))) return r;

    SearchArgs a;
    if (plan.S > 0) {
        a.geo = EngineGeom{};
        a.geo.L = L;
        a.geo.Wp = plan.Wp;
        a.geoD = a.geo;
    } else {
        a.geo = make_geom(L, rs->W, plan.C, prefetch_global(plan.C), window_global(plan.C));
        a.geoD = recheck_geom(L, rs->W, plan.C);
    }
    a.PD = plan.PD;
    a.SLOTS = plan.SLOTS;
    a.B = rs->B;
    a.Bp = rs->Bp;
    a.ppitch = rs->ppitch;
    a.padl = rs->padl;
    a.n = n;
    a.Q = Qy;
    a.sk = sk;
    a.slbk = slbk;
    a.slbeb = slbeb;
    a.slbe = slbe;
    a.ed2 = ed2;
    a.prefix = prefix;
    a.cascade = o->cascade;
    a.R = plan.R;
    a.eps = plan.eps;
    a.init_ub = o->init_ub;
    a.nn_idx = nn_idx;
    a.nn_dist = nn_dist;
    a.counts = counts;
    a.ncu = device_cu_count();
    a.share = nullptr;
    a.nq = nQ;
    a.epoch = 0;
    int64_t grid = nQ;
    if (plan.helpers > 0) {
        // helper workgroups (help_query) follow the nQ owners in dispatch order
        static std::atomic<uint32_t> g_epoch{0};
        a.epoch = (g_epoch.fetch_add(1u) % 0xFFFFFu) + 1u;
        a.share = (QueryShare *)(base + w.share);
        grid = nQ * (1 + plan.helpers);
        if (grid > 0x7FFFFFFF) grid = nQ;
        hipLaunchKernelGGL(share_reset_kernel, dim3((unsigned)ceil_div(nQ, 256)), dim3(256), 0, st, a.share, nQ);
        NNDTW_LAUNCH_CHECK("share reset kernel launch");
        if (grid == nQ) a.share = nullptr;
    }
    const size_t lds = plan.lds_bytes;
    if (plan.S > 0) {
        const bool win = plan.Wp < L - 1;
        switch (plan.S * 2 + (win ? 1 : 0)) {
#define X(s)                                                                                                    \
    case s * 2:                                                                                                 \
        hipLaunchKernelGGL((search_kernel_strip<s, false>), dim3((unsigned)grid), dim3(WAVE * plan.NW), lds, st, a); \
        break;                                                                                                  \
    case s * 2 + 1:                                                                                             \
        hipLaunchKernelGGL((search_kernel_strip<s, true>), dim3((unsigned)grid), dim3(WAVE * plan.NW), lds, st, a);  \
        break;
            X(4) X(8) X(12) X(16) X(24) X(32)
#undef X
        default:
            return fail(NNDTW_EUNSUP, "no row-strip search kernel for %d columns per lane", plan.S);
        }
        NNDTW_LAUNCH_CHECK("search kernel launch");
        return mark(4);
    }
    if (plan.NW > SEARCH_MAX_WAVES) {
        switch (plan.C * 2 + (plan.exact ? 1 : 0)) {
#define X(c)                                                                                                    \
    case c * 2:                                                                                                 \
        hipLaunchKernelGGL((search_kernel_wide<c, false>), dim3((unsigned)grid), dim3(WAVE * plan.NW), lds, st, a); \
        break;                                                                                                  \
    case c * 2 + 1:                                                                                             \
        hipLaunchKernelGGL((search_kernel_wide<c, true>), dim3((unsigned)grid), dim3(WAVE * plan.NW), lds, st, a);  \
        break;
            X(1) X(2) X(3) X(4) X(6)
#undef X
        default:
            return fail(NNDTW_EUNSUP, "no wide search kernel for %d pairs per lane", plan.C);
        }
        NNDTW_LAUNCH_CHECK("search kernel launch");
        return mark(4);
    }
    // the FP64 recheck engine the kernel holds (see search_query)
    const bool rk1 = plan.C > 1 && a.geoD.C == 1;
    switch (plan.C * 4 + (plan.exact ? 2 : 0) + (rk1 ? 1 : 0)) {
#define X(c)                                                                                                       \
    case c * 4 + 0:                                                                                                \
        hipLaunchKernelGGL((search_kernel<c, false, 2>), dim3((unsigned)grid), dim3(WAVE * plan.NW), lds, st, a);   \
        break;                                                                                                     \
    case c * 4 + 1:                                                                                                \
        hipLaunchKernelGGL((search_kernel<c, false, 1>), dim3((unsigned)grid), dim3(WAVE * plan.NW), lds, st, a);   \
        break;                                                                                                     \
    case c * 4 + 2:                                                                                                \
        hipLaunchKernelGGL((search_kernel<c, true, 2>), dim3((unsigned)grid), dim3(WAVE * plan.NW), lds, st, a);    \
        break;                                                                                                     \
    case c * 4 + 3:                                                                                                \
        hipLaunchKernelGGL((search_kernel<c, true, 1>), dim3((unsigned)grid), dim3(WAVE * plan.NW), lds, st, a);    \
        break;
        NNDTW_FOR_EACH_CPL(X)
#undef X
    default:
        return fail(NNDTW_EUNSUP, "no search kernel for %d pairs per lane", plan.C);
    }
    NNDTW_LAUNCH_CHECK("search kernel launch");
    return mark(4);
}

}  // namespace nndtw
