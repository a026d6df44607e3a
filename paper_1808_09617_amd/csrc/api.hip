// extern "C" entry points of libnndtw: argument validation on the host, then
// asynchronous launches on the caller's stream.  Nothing here allocates
// device memory; only nndtw_batch_prepare waits (for its own copies).
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "common.hpp"

namespace nndtw {

static thread_local char g_err[512];

int fail(int status, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return status;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(NNDTW_EHIP, "%s: %s", what, hipGetErrorString(e));
}

static bool bad_len(int L) { return L < 2 || L > NNDTW_MAX_L; }
static bool misaligned(const void *p, size_t a) { return ((uintptr_t)p % a) != 0; }

#define REQUIRE(cond, ...)                                       \
    do {                                                         \
        if (!(cond)) return ::nndtw::fail(NNDTW_EINVAL, __VA_ARGS__); \
    } while (0)

static int check_len_w(int L, int W)
{
    if (bad_len(L)) {
        if (L > NNDTW_MAX_L) return fail(NNDTW_EUNSUP, "L=%d exceeds NNDTW_MAX_L=%d", L, NNDTW_MAX_L);
        return fail(NNDTW_EINVAL, "L=%d: series length must be >= 2", L);
    }
    REQUIRE(W >= 0, "W=%d: window must be >= 0", W);
    return NNDTW_OK;
}

static int check_pairing(int pairing, int64_t nA, int64_t nB)
{
    REQUIRE(pairing == NNDTW_CROSS || pairing == NNDTW_ZIP, "pairing=%d: expected NNDTW_CROSS or NNDTW_ZIP", pairing);
    REQUIRE(nA >= 0 && nB >= 0, "negative series count (nA=%lld, nB=%lld)", (long long)nA, (long long)nB);
    REQUIRE(pairing != NNDTW_ZIP || nA == nB, "zip pairing needs nA == nB (nA=%lld, nB=%lld)", (long long)nA,
            (long long)nB);
    return NNDTW_OK;
}

static int check_ptr(const void *p, size_t align, const char *name, bool needed)
{
    if (!needed) return NNDTW_OK;
    REQUIRE(p != nullptr, "%s is NULL", name);
    REQUIRE(!misaligned(p, align), "%s is not %zu-byte aligned", name, align);
    return NNDTW_OK;
}

#define TRY(x)                    \
    do {                          \
        int r_ = (x);             \
        if (r_ != NNDTW_OK) return r_; \
    } while (0)

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace nndtw

using namespace nndtw;

extern "C" {

int nndtw_version(void) { return NNDTW_VERSION_MAJOR * 100 + NNDTW_VERSION_MINOR; }

const char *nndtw_status_string(int status)
{
    switch (status) {
    case NNDTW_OK: return "ok";
    case NNDTW_EINVAL: return "invalid argument";
    case NNDTW_EHIP: return "HIP runtime error";
    case NNDTW_EUNSUP: return "unsupported size or option";
    default: return "unknown status";
    }
}

const char *nndtw_last_error(void) { return g_err; }

int nndtw_envelopes(const float *B, int64_t n, int32_t L, int32_t W, float *U, float *Lo, void *stream)
{
    g_err[0] = 0;
    TRY(check_len_w(L, W));
    REQUIRE(n >= 0, "n=%lld must be >= 0", (long long)n);
    TRY(check_ptr(B, 4, "B", n > 0));
    TRY(check_ptr(U, 4, "U", n > 0));
    TRY(check_ptr(Lo, 4, "Lo", n > 0));
    return launch_envelopes(B, n, L, W, U, Lo, (hipStream_t)stream);
}

int nndtw_ed2(const float *A, int64_t nA, const float *B, int64_t nB, int32_t L, int32_t pairing, double *out,
              void *stream)
{
    g_err[0] = 0;
    TRY(check_len_w(L, 0));
    TRY(check_pairing(pairing, nA, nB));
    const bool any = nA > 0 && nB > 0;
    TRY(check_ptr(A, 4, "A", any));
    TRY(check_ptr(B, 4, "B", any));
    TRY(check_ptr(out, 8, "out", any));
    return launch_pair_bounds(0, A, nA, B, nullptr, nullptr, nB, L, 0, 1, nullptr, pairing, out,
                              (hipStream_t)stream);
}

int nndtw_lb_keogh(const float *A, int64_t nA, const float *U, const float *Lo, int64_t nB, int32_t L,
                   int32_t pairing, double *out, void *stream)
{
    g_err[0] = 0;
    TRY(check_len_w(L, 0));
    TRY(check_pairing(pairing, nA, nB));
    const bool any = nA > 0 && nB > 0;
    TRY(check_ptr(A, 4, "A", any));
    TRY(check_ptr(U, 4, "U", any));
    TRY(check_ptr(Lo, 4, "Lo", any));
    TRY(check_ptr(out, 8, "out", any));
    return launch_pair_bounds(1, A, nA, nullptr, U, Lo, nB, L, 0, 1, nullptr, pairing, out, (hipStream_t)stream);
}

int nndtw_lb_enhanced(const float *A, int64_t nA, const float *B, const float *U, const float *Lo, int64_t nB,
                      int32_t L, int32_t W, int32_t V, const double *cutoff, int32_t pairing, double *out,
                      void *stream)
{
    g_err[0] = 0;
    TRY(check_len_w(L, W));
    REQUIRE(V >= 1, "V=%d: the number of bands must be >= 1", V);
    TRY(check_pairing(pairing, nA, nB));
    const bool any = nA > 0 && nB > 0;
    TRY(check_ptr(A, 4, "A", any));
    TRY(check_ptr(B, 4, "B", any));
    TRY(check_ptr(U, 4, "U", any));
    TRY(check_ptr(Lo, 4, "Lo", any));
    TRY(check_ptr(out, 8, "out", any));
    if (cutoff) TRY(check_ptr(cutoff, 8, "cutoff", any));
    return launch_pair_bounds(2, A, nA, B, U, Lo, nB, L, W, V, cutoff, pairing, out, (hipStream_t)stream);
}

// Comparison bounds: what = 0 LB_Kim, 1 LB_Improved, 2 LB_New, 3 symmetric LB_Enhanced.
static int compare_common(int what, const float *A, int64_t nA, const float *B, const float *U, const float *Lo,
                          int64_t nB, int32_t L, int32_t W, int32_t V, const double *cutoff, int32_t pairing,
                          double *out, void *stream)
{
    g_err[0] = 0;
    TRY(check_len_w(L, W));
    REQUIRE(V >= 1, "V=%d: the number of bands must be >= 1", V);
    TRY(check_pairing(pairing, nA, nB));
    const bool any = nA > 0 && nB > 0;
    const bool env = what == 1 || what == 3;
    TRY(check_ptr(A, 4, "A", any));
    TRY(check_ptr(B, 4, "B", any));
    TRY(check_ptr(U, 4, "U", any && env));
    TRY(check_ptr(Lo, 4, "Lo", any && env));
    TRY(check_ptr(out, 8, "out", any));
    if (cutoff) TRY(check_ptr(cutoff, 8, "cutoff", any));
    if (compare_lds_bytes(L, W) > 160 * 1024)
        return fail(NNDTW_EUNSUP, "series length %d too long for the comparison bounds", L);
    return launch_compare_bounds(what, A, nA, B, U, Lo, nB, L, W, V, cutoff, pairing, out, (hipStream_t)stream);
}

int nndtw_lb_kim(const float *A, int64_t nA, const float *B, int64_t nB, int32_t L, int32_t pairing, double *out,
                 void *stream)
{
    return compare_common(0, A, nA, B, nullptr, nullptr, nB, L, 0, 1, nullptr, pairing, out, stream);
}

int nndtw_lb_improved(const float *A, int64_t nA, const float *B, const float *U, const float *Lo, int64_t nB,
                      int32_t L, int32_t W, const double *cutoff, int32_t pairing, double *out, void *stream)
{
    return compare_common(1, A, nA, B, U, Lo, nB, L, W, 1, cutoff, pairing, out, stream);
}

int nndtw_lb_new(const float *A, int64_t nA, const float *B, int64_t nB, int32_t L, int32_t W, int32_t pairing,
                 double *out, void *stream)
{
    return compare_common(2, A, nA, B, nullptr, nullptr, nB, L, W, 1, nullptr, pairing, out, stream);
}

int nndtw_lb_enhanced_sym(const float *A, int64_t nA, const float *B, const float *U, const float *Lo, int64_t nB,
                          int32_t L, int32_t W, int32_t V, int32_t pairing, double *out, void *stream)
{
    return compare_common(3, A, nA, B, U, Lo, nB, L, W, V, nullptr, pairing, out, stream);
}

static int dtw_common(bool f64, const float *A, int64_t nA, const float *B, int64_t nB, int32_t L, int32_t W,
                      const double *cutoff, int32_t pairing, void *out, void *stream)
{
    g_err[0] = 0;
    TRY(check_len_w(L, W));
    TRY(check_pairing(pairing, nA, nB));
    const bool any = nA > 0 && nB > 0;
    TRY(check_ptr(A, 4, "A", any));
    TRY(check_ptr(B, 4, "B", any));
    TRY(check_ptr(out, f64 ? 8 : 4, "out", any));
    if (cutoff) TRY(check_ptr(cutoff, 8, "cutoff", any));
    return launch_dtw_pairs(f64, A, nA, B, nB, L, W, cutoff, pairing, out, (hipStream_t)stream);
}

int nndtw_dtw_w(const float *A, int64_t nA, const float *B, int64_t nB, int32_t L, int32_t W,
                const double *cutoff, int32_t pairing, float *out, void *stream)
{
    return dtw_common(false, A, nA, B, nB, L, W, cutoff, pairing, out, stream);
}

int nndtw_dtw_w_f64(const float *A, int64_t nA, const float *B, int64_t nB, int32_t L, int32_t W,
                    const double *cutoff, int32_t pairing, double *out, void *stream)
{
    return dtw_common(true, A, nA, B, nB, L, W, cutoff, pairing, out, stream);
}

// ----------------------------------------------------------- reference sets
struct RefsetLayout {
    int64_t pitch, ppitch;
    int padl;
    size_t off[7], total;
};

static RefsetLayout refset_layout(int64_t n, int L, int W)
{
    RefsetLayout r;
    const int Wp = W < L - 1 ? W : L - 1;
    r.pitch = (n + 63) / 64 * 64;
    r.padl = padded_row_margin_left(Wp);
    r.ppitch = ((int64_t)r.padl + L + padded_row_margin_right(Wp) + 63) / 64 * 64;
    const size_t rowb = (size_t)n * L * sizeof(float);
    const size_t colb = (size_t)L * r.pitch * sizeof(float);
    size_t o = 0;
    for (int i = 0; i < 3; ++i) { r.off[i] = o; o = al256(o + rowb); }
    for (int i = 3; i < 6; ++i) { r.off[i] = o; o = al256(o + colb); }
    r.off[6] = o;
    o = al256(o + (size_t)n * r.ppitch * sizeof(float));
    r.total = o;
    return r;
}

int nndtw_refset_bytes(int64_t n, int32_t L, int32_t W, size_t *bytes)
{
    g_err[0] = 0;
    TRY(check_len_w(L, W));
    REQUIRE(n >= 1, "n=%lld: a reference set needs at least one series", (long long)n);
    REQUIRE(n <= NNDTW_REFSET_MAX_N, "n=%lld: more than %lld series in a reference set", (long long)n,
            (long long)NNDTW_REFSET_MAX_N);
    REQUIRE(bytes != nullptr, "bytes is NULL");
    *bytes = refset_layout(n, L, W).total;
    return NNDTW_OK;
}

int nndtw_refset_build(const float *B, int64_t n, int32_t L, int32_t W, void *mem, size_t bytes,
                       nndtw_refset *out, void *stream)
{
    g_err[0] = 0;
    TRY(check_len_w(L, W));
    REQUIRE(n >= 1, "n=%lld: a reference set needs at least one series", (long long)n);
    REQUIRE(n <= NNDTW_REFSET_MAX_N, "n=%lld: more than %lld series in a reference set", (long long)n,
            (long long)NNDTW_REFSET_MAX_N);
    TRY(check_ptr(B, 4, "B", true));
    TRY(check_ptr(mem, 256, "mem", true));
    REQUIRE(out != nullptr, "out is NULL");
    const RefsetLayout lay = refset_layout(n, L, W);
    const size_t need = lay.total;
    const int64_t pitch = lay.pitch;
    const size_t *off = lay.off;
    REQUIRE(bytes >= need, "refset memory too small: %zu bytes given, %zu needed", bytes, need);
    hipStream_t st = (hipStream_t)stream;
    unsigned char *m = (unsigned char *)mem;
    nndtw_refset r;
    memset(&r, 0, sizeof r);
    r.L = L;
    r.n = n;
    r.W = W;
    r.pitch = pitch;
    r.B = (float *)(m + off[0]);
    r.U = (float *)(m + off[1]);
    r.Lo = (float *)(m + off[2]);
    r.Bt = (float *)(m + off[3]);
    r.Ut = (float *)(m + off[4]);
    r.Lt = (float *)(m + off[5]);
    r.Bp = (float *)(m + off[6]);
    r.ppitch = lay.ppitch;
    r.padl = lay.padl;
    // one pass over B: envelopes, the row-major copy and the padded rows;
    // then the point-major copies
    TRY(launch_envelopes_build(B, n, L, W, r.U, r.Lo, r.B, r.Bp, r.padl, r.ppitch, st));
    TRY(launch_transpose3(r.B, r.U, r.Lo, n, L, pitch, r.Bt, r.Ut, r.Lt, st));
    r.magic = NNDTW_REFSET_MAGIC;
    *out = r;
    return NNDTW_OK;
}

static int check_refset(const nndtw_refset *rs)
{
    REQUIRE(rs != nullptr, "refset is NULL");
    REQUIRE(rs->magic == NNDTW_REFSET_MAGIC, "refset was not built by nndtw_refset_build");
    TRY(check_len_w(rs->L, rs->W));
    REQUIRE(rs->n >= 1, "refset has no series");
    return NNDTW_OK;
}

static int check_opts(const nndtw_search_opts *o)
{
    REQUIRE(o != nullptr, "opts is NULL");
    REQUIRE(o->V >= 1, "V=%d: the number of bands must be >= 1", o->V);
    REQUIRE(o->cascade >= NNDTW_CASCADE_NONE && o->cascade <= NNDTW_CASCADE_ENH_SYM, "cascade=%d unknown",
            o->cascade);
    REQUIRE(o->R >= 0, "R=%lld must be >= 0", (long long)o->R);
    REQUIRE(o->cpl >= 0, "cpl=%d must be >= 0", o->cpl);
    REQUIRE(o->waves >= 0 && o->waves <= NNDTW_SEARCH_MAX_WAVES, "waves=%d must be in 0..%d", o->waves,
            NNDTW_SEARCH_MAX_WAVES);
    REQUIRE(o->nq_hint >= 0, "nq_hint=%lld must be >= 0", (long long)o->nq_hint);
    REQUIRE(o->engine >= NNDTW_ENGINE_AUTO && o->engine <= NNDTW_ENGINE_STRIP, "engine=%d unknown", o->engine);
    REQUIRE(o->helpers >= -1 && o->helpers <= NNDTW_SEARCH_MAX_HELPERS, "helpers=%d must be in -1..%d", o->helpers,
            NNDTW_SEARCH_MAX_HELPERS);
    REQUIRE(o->order >= NNDTW_ORDER_AUTO && o->order <= NNDTW_ORDER_RANK, "order=%d is not an NNDTW_ORDER_* value",
            o->order);
    return NNDTW_OK;
}

int nndtw_search_workspace_bytes(const nndtw_refset *refset, int64_t nQ, const nndtw_search_opts *opts,
                                 size_t *bytes)
{
    g_err[0] = 0;
    TRY(check_refset(refset));
    TRY(check_opts(opts));
    REQUIRE(nQ >= 0, "nQ=%lld must be >= 0", (long long)nQ);
    REQUIRE(bytes != nullptr, "bytes is NULL");
    *bytes = search_ws_bytes(nQ, refset->n, refset->L);
    return NNDTW_OK;
}

int nndtw_search_plan(const nndtw_refset *refset, nndtw_search_opts *opts)
{
    g_err[0] = 0;
    TRY(check_refset(refset));
    TRY(check_opts(opts));
    SearchPlan plan;
    TRY(plan_search(refset, opts, &plan));
    opts->R = plan.R;
    opts->cpl = plan.C;
    opts->waves = plan.NW;
    opts->engine = plan.S > 0 ? NNDTW_ENGINE_STRIP : NNDTW_ENGINE_DIAGONAL;
    opts->helpers = plan.helpers > 0 ? plan.helpers : -1;
    return NNDTW_OK;
}

int nndtw_search(const nndtw_refset *refset, const float *Q, int64_t nQ, nndtw_search_opts *opts,
                 int64_t *nn_idx, double *nn_dist, int64_t *counts, void *ws, size_t ws_bytes, void *stream)
{
    g_err[0] = 0;
    TRY(check_refset(refset));
    TRY(check_opts(opts));
    REQUIRE(nQ >= 0, "nQ=%lld must be >= 0", (long long)nQ);
    const bool any = nQ > 0;
    TRY(check_ptr(Q, 4, "Q", any));
    TRY(check_ptr(nn_idx, 8, "nn_idx", any));
    TRY(check_ptr(nn_dist, 8, "nn_dist", any));
    if (counts) TRY(check_ptr(counts, 8, "counts", any));
    TRY(check_ptr(ws, 256, "ws", any));
    const size_t need = search_ws_bytes(nQ, refset->n, refset->L);
    REQUIRE(!any || ws_bytes >= need, "workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
    if (opts->cascade > NNDTW_CASCADE_ENH && compare_lds_bytes(refset->L, refset->W) > 160 * 1024)
        return fail(NNDTW_EUNSUP, "series length %d too long for the comparison bounds", refset->L);
    SearchPlan plan;
    nndtw_search_opts po = *opts;
    po.nq_hint = nQ;
    TRY(plan_search(refset, &po, &plan));
    opts->R = plan.R;
    opts->cpl = plan.C;
    opts->waves = plan.NW;
    opts->engine = plan.S > 0 ? NNDTW_ENGINE_STRIP : NNDTW_ENGINE_DIAGONAL;
    opts->helpers = plan.helpers > 0 ? plan.helpers : -1;
    return launch_search(refset, Q, nQ, opts, plan, nn_idx, nn_dist, counts, ws, (hipStream_t)stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Search without a workspace argument: the workspace of nndtw_search lives in
// a fixed device array of this file, which every GPU the library runs on
// holds until the process ends.  In host code `scratch` is only a stand-in
// for the device address: kernels are given the address that
// hipGetSymbolAddress returns for the current device, taken once per device.
static __device__ __align__(256) unsigned char scratch[NNDTW_SEARCH_SCRATCH_BYTES];

namespace nndtw {
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[NNDTW_MAX_DEVICES];

// Device address of `scratch` on the current device (looked up on the
// device's first call).
static int scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= NNDTW_MAX_DEVICES)
        return fail(NNDTW_EUNSUP, "device %d: the scratch array is tracked for %d devices", dev, NNDTW_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (ptr == nullptr || ((uintptr_t)ptr & 255u) != 0)
            return fail(NNDTW_EHIP, "scratch array at an unexpected address %p", ptr);
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return NNDTW_OK;
}
}  // namespace nndtw

extern "C" {

int nndtw_search_noalloc(const nndtw_refset *refset, const float *Q, int64_t nQ, nndtw_search_opts *opts,
                         int64_t *nn_idx, double *nn_dist, int64_t *counts, void *stream)
{
    g_err[0] = 0;
    TRY(check_refset(refset));
    TRY(check_opts(opts));
    REQUIRE(nQ >= 0, "nQ=%lld must be >= 0", (long long)nQ);
    const size_t need = search_ws_bytes(nQ, refset->n, refset->L);
    if (nQ > 0 && need > (size_t)NNDTW_SEARCH_SCRATCH_BYTES)
        return fail(NNDTW_EUNSUP,
                    "search of %lld queries against %lld references needs %zu workspace bytes, above the %zu of "
                    "the fixed scratch array (NNDTW_SEARCH_SCRATCH_BYTES): split the queries or use nndtw_search",
                    (long long)nQ, (long long)refset->n, need, (size_t)NNDTW_SEARCH_SCRATCH_BYTES);
    void *ws = nullptr;
    if (nQ > 0) TRY(scratch_address(&ws));
    // nndtw_search validates everything else and enqueues the same kernels;
    // nothing in the workspace needs clearing (every array is written before
    // it is read within the call)
    return nndtw_search(refset, Q, nQ, opts, nn_idx, nn_dist, counts, ws, NNDTW_SEARCH_SCRATCH_BYTES, stream);
}

int nndtw_cascade_bounds(const nndtw_refset *refset, const float *Q, int64_t nQ, int32_t V, double *ed2,
                         double *lbk, double *lbe_bands, double *lbe, void *stream)
{
    g_err[0] = 0;
    TRY(check_refset(refset));
    REQUIRE(V >= 1, "V=%d: the number of bands must be >= 1", V);
    REQUIRE(nQ >= 0, "nQ=%lld must be >= 0", (long long)nQ);
    const bool any = nQ > 0;
    TRY(check_ptr(Q, 4, "Q", any));
    if (ed2) TRY(check_ptr(ed2, 8, "ed2", any));
    if (lbk) TRY(check_ptr(lbk, 8, "lbk", any));
    if (lbe_bands) TRY(check_ptr(lbe_bands, 8, "lbe_bands", any));
    if (lbe) TRY(check_ptr(lbe, 8, "lbe", any));
    return launch_cascade_bounds(refset, Q, nQ, V, ed2, lbk, lbe_bands, lbe, (hipStream_t)stream);
}

int nndtw_dtw_codes_bytes(int64_t nA, int64_t nB, int32_t L, int32_t W, int32_t pairing, size_t *bytes)
{
    g_err[0] = 0;
    TRY(check_len_w(L, W));
    TRY(check_pairing(pairing, nA, nB));
    REQUIRE(bytes != nullptr, "bytes is NULL");
    const int64_t np = pairing ? nA : nA * nB;
    *bytes = np ? dtw_codes_bytes(nA, nB, L, W, pairing) : 0;
    if (np && *bytes == 0) return fail(NNDTW_EUNSUP, "window %d too wide for the DTW engine", W);
    return NNDTW_OK;
}

static int grad_common(const float *A, int64_t nA, const float *B, int64_t nB, int32_t L, int32_t W,
                       int32_t pairing, int32_t f64, const void *p, const char *pname, const void *codes,
                       size_t codes_bytes)
{
    TRY(check_len_w(L, W));
    TRY(check_pairing(pairing, nA, nB));
    REQUIRE(f64 == 0 || f64 == 1, "f64=%d must be 0 or 1", f64);
    const int64_t np = pairing ? nA : nA * nB;
    const bool any = np > 0;
    TRY(check_ptr(A, 4, "A", any));
    TRY(check_ptr(B, 4, "B", any));
    TRY(check_ptr(p, f64 ? 8 : 4, pname, any));
    TRY(check_ptr(codes, 256, "codes", any));
    const size_t need = any ? dtw_codes_bytes(nA, nB, L, W, pairing) : 0;
    REQUIRE(!any || need > 0, "window %d too wide for the DTW engine", W);
    REQUIRE(codes_bytes >= need, "codes buffer too small: %zu bytes given, %zu needed", codes_bytes, need);
    return NNDTW_OK;
}

int nndtw_dtw_w_codes(const float *A, int64_t nA, const float *B, int64_t nB, int32_t L, int32_t W,
                      int32_t pairing, int32_t f64, void *out, uint8_t *codes, size_t codes_bytes, void *stream)
{
    g_err[0] = 0;
    TRY(grad_common(A, nA, B, nB, L, W, pairing, f64, out, "out", codes, codes_bytes));
    return launch_dtw_codes(f64 != 0, A, nA, B, nB, L, W, pairing, out, codes, (hipStream_t)stream);
}

int nndtw_dtw_w_backward(const float *A, int64_t nA, const float *B, int64_t nB, int32_t L, int32_t W,
                         int32_t pairing, int32_t f64, const void *gout, const uint8_t *codes, size_t codes_bytes,
                         void *gA, void *stream)
{
    g_err[0] = 0;
    TRY(grad_common(A, nA, B, nB, L, W, pairing, f64, gout, "gout", codes, codes_bytes));
    TRY(check_ptr(gA, f64 ? 8 : 4, "gA", nA > 0));
    return launch_dtw_backward(f64 != 0, A, nA, B, nB, L, W, pairing, gout, codes, gA, (hipStream_t)stream);
}

// Prefix the current error text with the set it concerns.
static int set_error(int status, int d)
{
    char tmp[sizeof g_err];
    std::snprintf(tmp, sizeof tmp, "%s", g_err);
    return fail(status, "set %d: %s", d, tmp);
}

static int check_batch(const nndtw_batch_set *sets, int32_t nsets, const nndtw_search_opts *opts, bool ptrs)
{
    REQUIRE(sets != nullptr, "sets is NULL");
    REQUIRE(nsets >= 1, "nsets=%d must be >= 1", nsets);
    TRY(check_opts(opts));
    REQUIRE(opts->events == nullptr, "opts->events must be NULL for a batch");
    if (opts->cascade > NNDTW_CASCADE_ENH)
        return fail(NNDTW_EUNSUP, "cascade=%d: the batched search runs the paper's cascades only", opts->cascade);
    for (int d = 0; d < nsets; ++d) {
        const nndtw_batch_set &s = sets[d];
        if (int r = check_refset(s.refset)) return set_error(r, d);
        REQUIRE(s.nQ >= 0, "set %d: nQ=%lld must be >= 0", d, (long long)s.nQ);
        REQUIRE(s.nQ <= 0xFFFFFFFFLL, "set %d: too many queries", d);
        REQUIRE(s.R >= 0 && s.cpl >= 0, "set %d: R and cpl must be >= 0", d);
        if (s.refset->n > NNDTW_BATCH_MAX_N)
            return fail(NNDTW_EUNSUP, "set %d: reference set of %lld series exceeds NNDTW_BATCH_MAX_N=%d", d,
                        (long long)s.refset->n, NNDTW_BATCH_MAX_N);
        if (!ptrs) continue;
        const bool any = s.nQ > 0;
        if (int r = check_ptr(s.Q, 4, "Q", any)) return set_error(r, d);
        if (int r = check_ptr(s.nn_idx, 8, "nn_idx", any)) return set_error(r, d);
        if (int r = check_ptr(s.nn_dist, 8, "nn_dist", any)) return set_error(r, d);
        if (s.counts)
            if (int r = check_ptr(s.counts, 8, "counts", any)) return set_error(r, d);
    }
    return NNDTW_OK;
}

int nndtw_batch_workspace_bytes(const nndtw_batch_set *sets, int32_t nsets, const nndtw_search_opts *opts,
                                size_t *bytes)
{
    g_err[0] = 0;
    TRY(check_batch(sets, nsets, opts, false));
    REQUIRE(bytes != nullptr, "bytes is NULL");
    *bytes = batch_ws_bytes(sets, nsets, opts);
    return NNDTW_OK;
}

int nndtw_batch_prepare(nndtw_batch_set *sets, int32_t nsets, const nndtw_search_opts *opts, void *ws,
                        size_t ws_bytes, nndtw_batch_plan *plan, void *stream)
{
    g_err[0] = 0;
    TRY(check_batch(sets, nsets, opts, true));
    REQUIRE(plan != nullptr, "plan is NULL");
    TRY(check_ptr(ws, 256, "ws", true));
    return batch_prepare(sets, nsets, opts, ws, ws_bytes, plan, (hipStream_t)stream);
}

int nndtw_search_batch(const nndtw_batch_plan *plan, void *ws, void *stream)
{
    g_err[0] = 0;
    REQUIRE(plan != nullptr, "plan is NULL");
    TRY(check_ptr(ws, 256, "ws", plan->items > 0));
    return batch_launch(plan, ws, (hipStream_t)stream);
}

}  // extern "C"
