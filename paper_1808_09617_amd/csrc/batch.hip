// Batched search over many reference sets (ragged lengths): planning and the
// launch sequence.  The per-set work is exactly that of nndtw_search (same
// bound pass, same ordering, same per-query search); only the schedule
// differs:
//   1. one bound-pass kernel over the tiles of every set (and the reset of
//      the search work counter);
//   2. one ordering kernel per sort width, over the (set, query) items whose
//      set has that width;
//   3. per engine shape (C, EXACT), one persistent search kernel whose
//      workgroups take (set, query) items from the shape's counter, largest
//      expected work (n * L * (2W'+1)) first; once the items are all taken,
//      idle workgroups help the queries still running (shared FP32 batches,
//      as the single-query search's helper workgroups; the bound pass clears
//      the items' helper headers).
// Everything the kernels need (set descriptors, item lists, tile starts) is
// copied into the caller's workspace once, at planning time (enqueued on the
// stream, without waiting), so the launch sequence allocates and copies
// nothing and can be captured in a graph.  The ordering kernel of each set's
// first query also writes the set's cells table.
#include <algorithm>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace nndtw {

namespace {

constexpr uint32_t BATCH_PLAN_MAGIC = 0x4E444242u;   // "NDBB"
constexpr int BATCH_TQ = 4;                           // queries per bound-pass tile
constexpr int BATCH_CB_THREADS = 256;                 // references per bound-pass tile
constexpr int N_WIDTHS = 6;                           // sort widths 1, 2, 4, ..., 32
constexpr int BATCH_DEFAULT_HELPERS = 7;              // helpers per query in a search's tail
constexpr int64_t BATCH_FEW_ITEMS = 32;               // items of a shape that get helpers at launch

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t hdr, sets, items, oitems, tstart, share;
    std::vector<size_t> set_off;                      // per-set search workspace
    size_t total;
};

// share: room for a helper header (QueryShare) per item.
Layout layout(const nndtw_batch_set *sets, int nsets, bool share)
{
    Layout y;
    int64_t items = 0;
    for (int d = 0; d < nsets; ++d) items += sets[d].nQ;
    size_t o = 0;
    y.hdr = o;    o = al256(o + sizeof(BatchHdr));
    y.sets = o;   o = al256(o + sizeof(BatchSet) * (size_t)nsets);
    y.items = o;  o = al256(o + 8 * (size_t)items);
    y.oitems = o; o = al256(o + 8 * (size_t)items);
    y.tstart = o; o = al256(o + 8 * (size_t)(nsets + 1));
    y.share = o;  o = al256(o + (share ? sizeof(QueryShare) * (size_t)items : 0));
    y.set_off.resize(nsets);
    for (int d = 0; d < nsets; ++d) {
        y.set_off[d] = o;
        o = al256(o + ws_layout(sets[d].nQ, sets[d].refset->n, sets[d].refset->L, false).total);
    }
    y.total = o;
    return y;
}

int width_slot(int E)
{
    int s = 0;
    while ((1 << s) < E) ++s;
    return s;
}

}  // namespace

// Helper workgroups per query in a search's tail: opts->helpers < 0 none,
// 0 the default, else at most that many.
int batch_helpers(const nndtw_search_opts *o)
{
    return o->helpers < 0 ? 0 : o->helpers == 0 ? BATCH_DEFAULT_HELPERS : o->helpers;
}

size_t batch_ws_bytes(const nndtw_batch_set *sets, int nsets, const nndtw_search_opts *o)
{
    return layout(sets, nsets, batch_helpers(o) > 0).total;
}

int batch_prepare(nndtw_batch_set *sets, int nsets, const nndtw_search_opts *o, void *ws, size_t ws_bytes,
                  nndtw_batch_plan *plan, hipStream_t st)
{
    const int H = batch_helpers(o);
    const Layout y = layout(sets, nsets, H > 0);
    if (ws_bytes < y.total) return fail(NNDTW_EINVAL, "workspace too small: %zu bytes given, %zu needed", ws_bytes, y.total);
    unsigned char *base = (unsigned char *)ws;

    std::vector<BatchSet> bs(nsets);
    std::vector<int64_t> tstart(nsets + 1, 0);
    std::vector<double> cost(nsets);
    std::vector<int> width(nsets);
    int NW = 0;
    size_t lds = 0;
    // the waves per query follow the whole batch's query count (8 when the
    // batch's queries do not fill the device at 4 waves each)
    int64_t nitems = 0;
    for (int d = 0; d < nsets; ++d) nitems += sets[d].nQ;
    for (int d = 0; d < nsets; ++d) {
        const nndtw_refset *rs = sets[d].refset;
        nndtw_search_opts od = *o;
        od.R = sets[d].R;
        od.cpl = sets[d].cpl;
        od.nq_hint = nitems;
        SearchPlan sp;
        if (int r = plan_search(rs, &od, &sp, true)) return r;
        if (sp.C > 4)
            return fail(NNDTW_EUNSUP, "set %d: W=%d at L=%d needs %d pairs per lane; the batch supports up to 4", d,
                        rs->W, rs->L, sp.C);
        NW = sp.NW;
        lds = std::max(lds, sp.lds_bytes);
        sets[d].R = sp.R;
        sets[d].cpl = sp.C;

        const int L = rs->L;
        const int64_t n = rs->n, nQ = sets[d].nQ;
        const WsLayout w = ws_layout(nQ, n, L, false);
        unsigned char *sb = base + y.set_off[d];
        BatchSet &b = bs[d];
        std::memset(&b, 0, sizeof(b));
        SearchArgs &a = b.a;
        a.geo = make_geom(L, rs->W, sp.C, prefetch_global(sp.C), window_global(sp.C));
        a.geoD = recheck_geom(L, rs->W, sp.C);
        a.PD = sp.PD;
        a.SLOTS = sp.SLOTS;
        a.B = rs->B;
        a.Bp = rs->Bp;
        a.ppitch = rs->ppitch;
        a.padl = rs->padl;
        a.n = n;
        a.Q = sets[d].Q;
        a.sk = (const uint32_t *)(sb + w.sk);
        a.slbk = (const double *)(sb + w.slbk);
        a.slbeb = (const double *)(sb + w.slbeb);
        a.slbe = (const double *)(sb + w.slbe);
        a.ed2 = (const double *)(sb + w.ed2);
        a.prefix = (const uint32_t *)(sb + w.prefix);
        a.cascade = o->cascade;
        a.R = sp.R;
        a.eps = sp.eps;
        a.init_ub = o->init_ub;
        a.nn_idx = sets[d].nn_idx;
        a.nn_dist = sets[d].nn_dist;
        a.counts = sets[d].counts;
        a.ncu = device_cu_count();
        b.C = sp.C;
        b.exact = sp.exact;
        b.Bt = rs->Bt;
        b.Ut = rs->Ut;
        b.Lt = rs->Lt;
        b.pitch = rs->pitch;
        b.nQ = nQ;
        b.L = L;
        b.W = rs->W;
        b.nb = o->V < L / 2 ? o->V : L / 2;
        b.nrt = (n + BATCH_CB_THREADS - 1) / BATCH_CB_THREADS;
        b.ed2w = (double *)(sb + w.ed2);
        b.lbk = (double *)(sb + w.lbk);
        b.lbeb = (double *)(sb + w.lbeb);
        b.lbe = (double *)(sb + w.lbe);
        b.skw = (uint32_t *)(sb + w.sk);
        b.slbkw = (double *)(sb + w.slbk);
        b.slbebw = (double *)(sb + w.slbeb);
        b.slbew = (double *)(sb + w.slbe);
        tstart[d + 1] = tstart[d] + (nQ > 0 ? b.nrt * ((nQ + BATCH_TQ - 1) / BATCH_TQ) : 0);
        cost[d] = (double)n * L * (2.0 * sp.Wp + 1.0);
        width[d] = order_width(n);
        if (width[d] > 32) return fail(NNDTW_EUNSUP, "set %d: %lld references exceed the sort", d, (long long)n);
    }
    if (NW == 0) NW = o->waves > 0 ? o->waves : 4;

    // search items per engine shape, largest expected work first (stable:
    // then set, query)
    std::vector<int> order(nsets);
    for (int d = 0; d < nsets; ++d) order[d] = d;
    std::stable_sort(order.begin(), order.end(), [&](int x, int z) { return cost[x] > cost[z]; });
    std::vector<int64_t> items, oitems;
    int64_t soff[BATCH_SHAPES] = {0}, scnt[BATCH_SHAPES] = {0};
    QueryShare *share = H > 0 ? (QueryShare *)(base + y.share) : nullptr;
    for (int sh = 0; sh < BATCH_SHAPES; ++sh) {
        soff[sh] = (int64_t)items.size();
        for (int d : order)
            if ((bs[d].C - 1) * 2 + bs[d].exact == sh) {
                // the set's queries are consecutive items: header of query q
                // at the set's first item + q
                if (share != nullptr) {
                    bs[d].a.share = share + items.size();
                    bs[d].a.nq = sets[d].nQ;
                    bs[d].a.epoch = 1u;          // the headers are reset before every launch
                }
                for (int64_t q = 0; q < sets[d].nQ; ++q) items.push_back(((int64_t)d << 32) | q);
            }
        scnt[sh] = (int64_t)items.size() - soff[sh];
    }
    // ordering: by ranking in one launch, or items grouped by sort width
    double rank_work = 0.0;
    int64_t nmax = 0;
    for (int d = 0; d < nsets; ++d)
        if (sets[d].nQ > 0) {
            const double n = (double)sets[d].refset->n;
            rank_work += (double)sets[d].nQ * n * n;
            nmax = std::max<int64_t>(nmax, sets[d].refset->n);
        }
    bool rank = false;
    if (int r = order_by_rank(o->order, rank_work, nmax, (int64_t)items.size(), &rank)) return r;
    int64_t ooff[N_WIDTHS] = {0}, ocnt[N_WIDTHS] = {0};
    for (int s = 0; s < N_WIDTHS; ++s) {
        ooff[s] = (int64_t)oitems.size();
        for (int d = 0; d < nsets; ++d)
            if (width_slot(width[d]) == s)
                for (int64_t q = 0; q < sets[d].nQ; ++q) oitems.push_back(((int64_t)d << 32) | q);
        ocnt[s] = (int64_t)oitems.size() - ooff[s];
    }

    // one host image of the control block, copied once.  The copy is only
    // enqueued: the image lives until a host function that follows the copy
    // on the stream releases it, so prepare does not wait for the device.
    auto *img = new std::vector<unsigned char>(y.set_off.empty() ? y.tstart + 8 * (size_t)(nsets + 1)
                                                                 : y.set_off[0], 0);
    BatchHdr hdr{};
    std::memcpy(img->data() + y.hdr, &hdr, sizeof(hdr));
    std::memcpy(img->data() + y.sets, bs.data(), sizeof(BatchSet) * bs.size());
    if (!items.empty()) {
        std::memcpy(img->data() + y.items, items.data(), 8 * items.size());
        std::memcpy(img->data() + y.oitems, oitems.data(), 8 * oitems.size());
    }
    std::memcpy(img->data() + y.tstart, tstart.data(), 8 * tstart.size());
    hipError_t e = hipMemcpyAsync(ws, img->data(), img->size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        delete img;
        return hip_fail(e, "batch control block copy");
    }
    e = hipLaunchHostFunc(
        st, [](void *p) { delete static_cast<std::vector<unsigned char> *>(p); }, img);
    if (e != hipSuccess) {
        // the copy is enqueued: wait for it before releasing its source
        (void)hipStreamSynchronize(st);
        delete img;
        return hip_fail(e, "batch control block release");
    }

    std::memset(plan, 0, sizeof(*plan));
    plan->magic = BATCH_PLAN_MAGIC;
    plan->nsets = nsets;
    plan->items = (int64_t)items.size();
    plan->tiles = tstart[nsets];
    plan->waves = NW;
    plan->grid = 4096 / NW;                           // workgroups resident at up to 4 waves per SIMD
    plan->lds = (int64_t)lds;
    plan->ws_bytes = (int64_t)y.total;
    for (int s = 0; s < N_WIDTHS; ++s) {
        plan->order_off[s] = ooff[s];
        plan->order_cnt[s] = ocnt[s];
    }
    for (int sh = 0; sh < BATCH_SHAPES; ++sh) {
        plan->search_off[sh] = soff[sh];
        plan->search_cnt[sh] = scnt[sh];
    }
    plan->reserved[0] = (int64_t)y.sets;
    plan->reserved[1] = (int64_t)y.items;
    plan->reserved[2] = (int64_t)y.oitems;
    plan->reserved[3] = (int64_t)y.tstart;
    plan->helpers = H;
    plan->share_shapes = 0u;
    if (H > 0)
        for (int sh = 0; sh < BATCH_SHAPES; ++sh)
            if (scnt[sh] > 0) plan->share_shapes |= 1u << sh;
    plan->share_off = H > 0 ? (int64_t)y.share : 0;
    plan->order_rank = rank ? 1 : 0;
    plan->order_nmax = (int32_t)nmax;
    return NNDTW_OK;
}

int batch_launch(const nndtw_batch_plan *plan, void *ws, hipStream_t st)
{
    if (plan->magic != BATCH_PLAN_MAGIC) return fail(NNDTW_EINVAL, "plan was not made by nndtw_batch_prepare");
    if (plan->items == 0) return NNDTW_OK;
    unsigned char *base = (unsigned char *)ws;
    const BatchSet *sets = (const BatchSet *)(base + plan->reserved[0]);
    const int64_t *items = (const int64_t *)(base + plan->reserved[1]);
    const int64_t *oitems = (const int64_t *)(base + plan->reserved[2]);
    const int64_t *tstart = (const int64_t *)(base + plan->reserved[3]);
    BatchHdr *hdr = (BatchHdr *)base;
    QueryShare *share = plan->share_shapes != 0u ? (QueryShare *)(base + plan->share_off) : nullptr;
    if (int r = launch_batch_bounds(sets, plan->nsets, tstart, plan->tiles, hdr, share, share ? plan->items : 0, st))
        return r;
    if (plan->order_rank) {
        // oitems holds every item (the width groups are consecutive from 0)
        if (int r = launch_batch_rank(sets, oitems, plan->items, plan->order_nmax, st)) return r;
    } else {
        for (int s = 0; s < N_WIDTHS; ++s)
            if (plan->order_cnt[s] > 0)
                if (int r = launch_batch_order(1 << s, sets, oitems + plan->order_off[s], plan->order_cnt[s], st))
                    return r;
    }
    for (int sh = 0; sh < BATCH_SHAPES; ++sh) {
        const int64_t cnt = plan->search_cnt[sh];
        if (cnt == 0) continue;
        // a sharing shape with few items (a serving batch) launches up to
        // `helpers` more workgroups per item; with more, the workgroups that
        // run out of items help (extra ones would take compute units from
        // the kernels of other streams)
        const int H = (plan->share_shapes >> sh) & 1u ? plan->helpers : 0;
        const int64_t want = cnt <= BATCH_FEW_ITEMS ? cnt * (1 + H) : cnt;
        const int grid = (int)std::min<int64_t>(want, plan->grid);
        if (int r = launch_batch_search(sh / 2 + 1, sh & 1, sets, items + plan->search_off[sh], cnt,
                                        &hdr->counter[sh], hdr->running, plan->waves, grid, (size_t)plan->lds, H,
                                        st))
            return r;
    }
    return NNDTW_OK;
}

}  // namespace nndtw
