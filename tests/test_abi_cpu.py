"""The C-ABI library loads, exports every function include/nndtw.h declares,
and rejects invalid arguments on the host (no GPU needed: every call below
fails validation before anything is enqueued)."""
import ctypes
import os
import re

import pytest

import paper_1808_09617_amd as nd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nndtw.h")

NULL = ctypes.c_void_p(0)
FAKE = ctypes.c_void_p(0x100000)      # never dereferenced: validation fails first


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nndtw_\w+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = nd.lib()
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(nd.SIGNATURES), "binding signatures out of sync with the header"


def test_header_constants_match_binding():
    text = open(HEADER).read()
    defs = dict(re.findall(r"#define\s+(NNDTW_\w+)\s+(\S+)", text))
    assert int(defs["NNDTW_MAX_L"]) == nd.MAX_L
    assert int(defs["NNDTW_BATCH_MAX_N"]) == nd.BATCH_MAX_N
    assert int(defs["NNDTW_SEARCH_MAX_WAVES"]) == nd.SEARCH_MAX_WAVES
    for name, v in nd.CASCADES.items():
        assert int(defs["NNDTW_CASCADE_" + name.upper()]) == v
    assert int(defs["NNDTW_NCOUNTS"]) == len(nd.COUNT_NAMES)


def test_version_and_status_strings():
    lib = nd.lib()
    assert lib.nndtw_version() == 1
    assert lib.nndtw_status_string(0) == b"ok"
    assert lib.nndtw_status_string(-1) == b"invalid argument"
    assert lib.nndtw_status_string(-3) == b"unsupported size or option"
    assert lib.nndtw_status_string(12345) == b"unknown status"


def test_struct_layouts():
    assert ctypes.sizeof(nd._Refset) == 104
    assert nd._Refset.B.offset == 32
    assert ctypes.sizeof(nd._SearchOpts) == 64
    assert nd._SearchOpts.eps.offset == 16 and nd._SearchOpts.events.offset == 32
    assert nd._SearchOpts.waves.offset == 40 and nd._SearchOpts.engine.offset == 44
    assert nd._SearchOpts.nq_hint.offset == 48
    assert nd._SearchOpts.helpers.offset == 56 and nd._SearchOpts.order.offset == 60


def _err(status, fragment):
    assert status != 0
    msg = nd.last_error()
    assert fragment in msg, msg
    return status


def test_envelope_validation():
    lib = nd.lib()
    assert _err(lib.nndtw_envelopes(NULL, 4, 64, 3, FAKE, FAKE, NULL), "B is NULL") == nd.EINVAL
    assert _err(lib.nndtw_envelopes(FAKE, 4, 1, 3, FAKE, FAKE, NULL), "L=1") == nd.EINVAL
    assert _err(lib.nndtw_envelopes(FAKE, 4, 4096, 3, FAKE, FAKE, NULL), "NNDTW_MAX_L") == nd.EUNSUP
    assert _err(lib.nndtw_envelopes(FAKE, 4, 64, -1, FAKE, FAKE, NULL), "W=-1") == nd.EINVAL
    assert _err(lib.nndtw_envelopes(FAKE, -4, 64, 3, FAKE, FAKE, NULL), "n=-4") == nd.EINVAL
    assert _err(lib.nndtw_envelopes(ctypes.c_void_p(0x100002), 4, 64, 3, FAKE, FAKE, NULL), "aligned") == nd.EINVAL
    # n = 0 is a valid empty call: nothing is enqueued
    assert lib.nndtw_envelopes(NULL, 0, 64, 3, NULL, NULL, NULL) == 0


def test_pairwise_validation():
    lib = nd.lib()
    assert _err(lib.nndtw_ed2(FAKE, 3, FAKE, 4, 64, nd.ZIP, FAKE, NULL), "nA == nB") == nd.EINVAL
    assert _err(lib.nndtw_ed2(FAKE, 3, FAKE, 4, 64, 7, FAKE, NULL), "pairing=7") == nd.EINVAL
    assert _err(lib.nndtw_lb_keogh(FAKE, 3, NULL, FAKE, 4, 64, 0, FAKE, NULL), "U is NULL") == nd.EINVAL
    assert _err(lib.nndtw_lb_enhanced(FAKE, 3, FAKE, FAKE, FAKE, 4, 64, 3, 0, NULL, 0, FAKE, NULL),
                "V=0") == nd.EINVAL
    assert _err(lib.nndtw_lb_enhanced(FAKE, 3, FAKE, FAKE, FAKE, 4, 64, 3, 1, ctypes.c_void_p(0x100004), 0,
                                      FAKE, NULL), "cutoff is not 8-byte aligned") == nd.EINVAL
    assert _err(lib.nndtw_dtw_w(FAKE, 3, FAKE, 4, 64, -2, NULL, 0, FAKE, NULL), "W=-2") == nd.EINVAL
    assert _err(lib.nndtw_dtw_w_f64(FAKE, 3, FAKE, 4, 64, 2, NULL, 0, ctypes.c_void_p(0x100004), NULL),
                "out is not 8-byte aligned") == nd.EINVAL
    assert lib.nndtw_dtw_w(NULL, 0, NULL, 5, 64, 2, NULL, 0, NULL, NULL) == 0      # empty


def test_comparison_bounds_validation():
    lib = nd.lib()
    assert _err(lib.nndtw_lb_kim(FAKE, 3, FAKE, 4, 1, 0, FAKE, NULL), "L=1") == nd.EINVAL
    assert _err(lib.nndtw_lb_kim(FAKE, 3, NULL, 4, 64, 0, FAKE, NULL), "B is NULL") == nd.EINVAL
    assert lib.nndtw_lb_kim(NULL, 0, NULL, 4, 64, 0, NULL, NULL) == 0                  # empty
    assert _err(lib.nndtw_lb_improved(FAKE, 3, FAKE, NULL, FAKE, 4, 64, 3, NULL, 0, FAKE, NULL),
                "U is NULL") == nd.EINVAL
    assert _err(lib.nndtw_lb_improved(FAKE, 3, FAKE, FAKE, FAKE, 4, 64, -1, NULL, 0, FAKE, NULL),
                "W=-1") == nd.EINVAL
    assert _err(lib.nndtw_lb_new(FAKE, 3, FAKE, 4, 64, 3, nd.ZIP, FAKE, NULL), "nA == nB") == nd.EINVAL
    assert _err(lib.nndtw_lb_new(FAKE, 3, FAKE, 3, 4096, 3, nd.ZIP, FAKE, NULL), "exceeds") == nd.EUNSUP
    assert _err(lib.nndtw_lb_enhanced_sym(FAKE, 3, FAKE, FAKE, FAKE, 4, 64, 3, 0, 0, FAKE, NULL),
                "V=0") == nd.EINVAL
    assert _err(lib.nndtw_lb_enhanced_sym(FAKE, 3, FAKE, FAKE, FAKE, 4, 64, 3, 2, 0, ctypes.c_void_p(0x100004),
                                          NULL), "out is not 8-byte aligned") == nd.EINVAL


def test_refset_and_search_validation():
    lib = nd.lib()
    nbytes = ctypes.c_size_t(0)
    assert lib.nndtw_refset_bytes(100, 64, 6, ctypes.byref(nbytes)) == 0
    assert nbytes.value >= 7 * 100 * 64 * 4
    assert _err(lib.nndtw_refset_bytes(0, 64, 6, ctypes.byref(nbytes)), "at least one series") == nd.EINVAL
    max_n = (1 << 29) - 64                       # NNDTW_REFSET_MAX_N
    assert lib.nndtw_refset_bytes(max_n, 2, 1, ctypes.byref(nbytes)) == 0
    assert _err(lib.nndtw_refset_bytes(max_n + 1, 2, 1, ctypes.byref(nbytes)), "series in a reference set") \
        == nd.EINVAL
    desc = nd._Refset()
    assert lib.nndtw_refset_bytes(100, 64, 3, ctypes.byref(nbytes)) == 0
    assert _err(lib.nndtw_refset_build(FAKE, 100, 64, 3, FAKE, nbytes.value - 1, ctypes.byref(desc), NULL),
                "too small") == nd.EINVAL
    assert _err(lib.nndtw_refset_build(FAKE, 100, 64, 3, ctypes.c_void_p(0x100010), nbytes.value,
                                       ctypes.byref(desc), NULL), "mem is not 256-byte aligned") == nd.EINVAL
    opts = nd._opts(5, "keogh_enh", 0, 0.0, True, 0)
    # a descriptor that was never built
    assert _err(lib.nndtw_search_workspace_bytes(ctypes.byref(desc), 10, ctypes.byref(opts),
                                                 ctypes.byref(nbytes)), "not built") == nd.EINVAL
    desc.magic, desc.L, desc.n, desc.W = nd.REFSET_MAGIC, 64, 100, 6
    assert lib.nndtw_search_workspace_bytes(ctypes.byref(desc), 10, ctypes.byref(opts), ctypes.byref(nbytes)) == 0
    bad = nd._opts(0, "keogh_enh", 0, 0.0, True, 0)
    assert _err(lib.nndtw_search_workspace_bytes(ctypes.byref(desc), 10, ctypes.byref(bad),
                                                 ctypes.byref(nbytes)), "V=0") == nd.EINVAL
    bad = nd._opts(5, "keogh_enh", 0, 0.0, True, 0, order=-1)
    assert _err(lib.nndtw_search_workspace_bytes(ctypes.byref(desc), 10, ctypes.byref(bad),
                                                 ctypes.byref(nbytes)), "order=-1") == nd.EINVAL
    # ranking asked for beyond its 8192 references: refused before anything is enqueued
    big = nd._Refset()
    big.magic, big.L, big.n, big.W = nd.REFSET_MAGIC, 64, 9000, 6
    big.pitch, big.padl, big.ppitch = 9024, 1024, 2112
    rank = nd._opts(5, "keogh_enh", 0, 0.0, True, 0, order="rank")
    nb_big = ctypes.c_size_t(0)
    assert lib.nndtw_search_workspace_bytes(ctypes.byref(big), 2, ctypes.byref(rank), ctypes.byref(nb_big)) == 0
    assert _err(lib.nndtw_search(ctypes.byref(big), FAKE, 2, ctypes.byref(rank), FAKE, FAKE, NULL, FAKE,
                                 nb_big.value, NULL), "ordering by ranking") == nd.EUNSUP
    bad = nd._opts(2, "keogh_enh", -1, 0.0, True, 0)
    assert _err(lib.nndtw_search(ctypes.byref(desc), FAKE, 10, ctypes.byref(bad), FAKE, FAKE, NULL, FAKE,
                                 nbytes.value, NULL), "R=-1") == nd.EINVAL
    assert _err(lib.nndtw_search(ctypes.byref(desc), FAKE, 10, ctypes.byref(opts), FAKE, FAKE, NULL, FAKE,
                                 nbytes.value - 1, NULL), "workspace too small") == nd.EINVAL
    assert _err(lib.nndtw_cascade_bounds(ctypes.byref(desc), NULL, 10, 2, NULL, NULL, NULL, NULL, NULL),
                "Q is NULL") == nd.EINVAL


def test_batch_struct_layouts():
    assert ctypes.sizeof(nd._BatchSet) == 64
    assert nd._BatchSet.R.offset == 48 and nd._BatchSet.cpl.offset == 56
    assert ctypes.sizeof(nd._BatchPlan) == 328
    assert nd._BatchPlan.order_off.offset == 48 and nd._BatchPlan.search_off.offset == 144
    assert nd._BatchPlan.reserved.offset == 272
    assert nd._BatchPlan.helpers.offset == 304 and nd._BatchPlan.share_shapes.offset == 308
    assert nd._BatchPlan.share_off.offset == 312
    assert nd._BatchPlan.order_rank.offset == 320 and nd._BatchPlan.order_nmax.offset == 324


def test_batch_validation_and_workspace_size():
    lib = nd.lib()
    opts = nd._opts(5, "keogh_enh", 0, 0.0, True, 0)
    nbytes = ctypes.c_size_t(0)
    descs = []
    for L, n, W in ((24, 50, 2), (300, 700, 30), (1839, 200, 184)):
        d = nd._Refset()
        d.magic, d.L, d.n, d.W = nd.REFSET_MAGIC, L, n, W
        descs.append(d)
    sets = (nd._BatchSet * 3)()
    for i, d in enumerate(descs):
        sets[i].refset = ctypes.addressof(d)
        sets[i].Q, sets[i].nQ, sets[i].nn_idx, sets[i].nn_dist = FAKE, 5 + i, FAKE, FAKE
    assert lib.nndtw_batch_workspace_bytes(sets, 3, ctypes.byref(opts), ctypes.byref(nbytes)) == 0
    # at least the three sets' search workspaces (bounds, order, gathered bounds)
    assert nbytes.value >= sum(8 * 7 * (5 + i) * d.n for i, d in enumerate(descs))
    # without helper workgroups: no helper header per query (18 queries)
    no_help = nd._opts(5, "keogh_enh", 0, 0.0, True, 0, helpers=-1)
    nb2 = ctypes.c_size_t(0)
    assert lib.nndtw_batch_workspace_bytes(sets, 3, ctypes.byref(no_help), ctypes.byref(nb2)) == 0
    assert nbytes.value - nb2.value == (18 * 3136 + 255) // 256 * 256
    bad = nd._opts(5, "keogh_enh", 0, 0.0, True, 0, helpers=8)
    assert _err(lib.nndtw_batch_workspace_bytes(sets, 3, ctypes.byref(bad), ctypes.byref(nb2)),
                "helpers=8") == nd.EINVAL
    bad = nd._opts(5, "keogh_enh", 0, 0.0, True, 0, order=3)
    assert _err(lib.nndtw_batch_workspace_bytes(sets, 3, ctypes.byref(bad), ctypes.byref(nb2)),
                "order=3") == nd.EINVAL
    assert _err(lib.nndtw_batch_workspace_bytes(sets, 0, ctypes.byref(opts), ctypes.byref(nbytes)),
                "nsets=0") == nd.EINVAL
    assert _err(lib.nndtw_batch_workspace_bytes(None, 3, ctypes.byref(opts), ctypes.byref(nbytes)),
                "sets is NULL") == nd.EINVAL
    plan = nd._BatchPlan()
    assert _err(lib.nndtw_batch_prepare(sets, 3, ctypes.byref(opts), ctypes.c_void_p(0x100000), 1,
                                        ctypes.byref(plan), NULL), "workspace too small") == nd.EINVAL
    sets[1].nQ = -1
    assert _err(lib.nndtw_batch_workspace_bytes(sets, 3, ctypes.byref(opts), ctypes.byref(nbytes)),
                "set 1: nQ=-1") == nd.EINVAL
    sets[1].nQ = 6
    sets[2].nn_dist = NULL
    assert _err(lib.nndtw_batch_prepare(sets, 3, ctypes.byref(opts), FAKE, 1 << 40, ctypes.byref(plan), NULL),
                "set 2: nn_dist is NULL") == nd.EINVAL
    bad = nd._Refset()
    sets[0].refset = ctypes.addressof(bad)
    assert _err(lib.nndtw_batch_workspace_bytes(sets, 3, ctypes.byref(opts), ctypes.byref(nbytes)),
                "set 0: refset was not built") == nd.EINVAL
    sets[0].refset = ctypes.addressof(descs[0])
    ev = nd._opts(5, "keogh_enh", 0, 0.0, True, 0)
    ev.events = FAKE
    assert _err(lib.nndtw_batch_workspace_bytes(sets, 3, ctypes.byref(ev), ctypes.byref(nbytes)),
                "events must be NULL") == nd.EINVAL
    cmp = nd._opts(5, "improved", 0, 0.0, True, 0)
    assert _err(lib.nndtw_batch_workspace_bytes(sets, 3, ctypes.byref(cmp), ctypes.byref(nbytes)),
                "paper's cascades only") == nd.EUNSUP
    assert _err(lib.nndtw_search_batch(None, FAKE, NULL), "plan is NULL") == nd.EINVAL
    assert _err(lib.nndtw_search_batch(ctypes.byref(plan), FAKE, NULL), "not made by") == nd.EINVAL


def test_python_binding_rejects_cpu_tensors():
    import torch
    with pytest.raises(TypeError):
        nd.envelopes(torch.zeros(3, 8), 2)


def _strip_width(L):
    return 4 if L <= 256 else 8 if L <= 512 else 12 if L <= 768 else 16 if L <= 1024 else 24 if L <= 1536 else 32


def _strip_chosen(L, Wp):
    """The search's engine choice: row strips where the window is too wide
    for its diagonal shapes (63 lanes x 9 pairs), and for unconstrained DTW
    at L > 192."""
    return Wp + 1 > 63 * 9 or (Wp >= L - 1 and L > 192)


def test_search_plan_has_a_shape_for_every_window():
    """For every window the host plan is either the row-strip engine (one
    candidate per wave) or a diagonal shape whose groups fit a wave (at least
    one pair of series per wave, so a round of at least one candidate).  (A
    plan with zero groups per wave once gave a round size of 0, which the
    kernel divides by.)  Forcing the diagonal engine beyond 63 lanes x 9
    pairs, or the strip engine on a window narrower than its strips, is
    EUNSUP."""
    lib = nd.lib()
    for L in (2, 3, 64, 300, 512, 2048):
        d = nd._Refset()
        d.magic, d.L, d.n = nd.REFSET_MAGIC, L, 100
        d.padl, d.ppitch = 4096, 16384                      # margins wide enough for any shape
        for W in sorted(set(range(0, min(L, 600) + 1)) | {L // 2, L - 2, L - 1, L, 2 * L} - {-1}):
            d.W = W
            Wp = min(W, L - 1)
            opts = nd._opts(5, "keogh_enh", 0, 0.0, True, 0)
            st = lib.nndtw_search_plan(ctypes.byref(d), ctypes.byref(opts))
            assert st == 0, (L, W, nd.last_error())
            if _strip_chosen(L, Wp):
                assert opts.engine == nd.ENGINES["strip"] and opts.cpl == 0, (L, W)
                assert opts.waves == 4 and opts.R == 256, (L, W, opts.waves, opts.R)
                assert opts.helpers == 3                           # helper workgroups, as on the diagonal shapes
            else:
                assert opts.engine == nd.ENGINES["diagonal"], (L, W)
                # 3 helper workgroups per query, except for the shapes whose
                # kernels hold no shared-batch code (3 and 6 pairs per lane)
                assert opts.helpers == (-1 if opts.cpl in (3, 6) else 3), (L, W, opts.cpl, opts.helpers)
                C = opts.cpl
                G = -(-(Wp + 1) // C)
                assert C in (1, 2, 3, 4, 6, 8, 9) and G <= 63, (L, W, C, G)
                # default round: two candidates per group, at least 256
                assert opts.R == max(2 * (63 // G) * opts.waves, 256), (L, W, opts.R)
            forced = nd._opts(5, "keogh_enh", 0, 0.0, True, 0, engine="diagonal")
            st = lib.nndtw_search_plan(ctypes.byref(d), ctypes.byref(forced))
            if Wp + 1 > 63 * 9:
                assert _err(st, "too wide for the diagonal engine") == nd.EUNSUP
            else:
                assert st == 0 and forced.engine == nd.ENGINES["diagonal"], (L, W, nd.last_error())
            forced = nd._opts(5, "keogh_enh", 0, 0.0, True, 0, engine="strip")
            st = lib.nndtw_search_plan(ctypes.byref(d), ctypes.byref(forced))
            if Wp >= L - 1 or 2 * Wp + 2 >= _strip_width(L):
                assert st == 0 and forced.engine == nd.ENGINES["strip"], (L, W, nd.last_error())
            else:
                assert _err(st, "too narrow for the row-strip engine") == nd.EUNSUP
    # where the narrow shapes (<= 4 pairs per lane) leave one group per wave
    # with lanes idle, a wider shape is taken: W=128 at L=512 (129 diagonal
    # pairs) runs 4 groups of 15 lanes at 9 pairs per lane, not one group of
    # 43 lanes at 3
    d.L, d.W = 512, 128
    opts = nd._opts(5, "keogh_enh", 0, 0.0, True, 0)
    assert lib.nndtw_search_plan(ctypes.byref(d), ctypes.byref(opts)) == 0 and opts.cpl == 9
    d.L = 2048
    d.W = 251
    opts = nd._opts(5, "keogh_enh", 0, 0.0, True, 2)              # 126 lanes per group: no fit
    assert _err(lib.nndtw_search_plan(ctypes.byref(d), ctypes.byref(opts)), "cpl=2") == nd.EINVAL
    # pairs per lane are a diagonal-engine option; strips take up to 4 waves above L = 1024
    d.W = 2047
    opts = nd._opts(5, "keogh_enh", 0, 0.0, True, 3, engine="strip")
    assert _err(lib.nndtw_search_plan(ctypes.byref(d), ctypes.byref(opts)), "diagonal engine only") == nd.EINVAL
    opts = nd._opts(5, "keogh_enh", 0, 0.0, True, 0, waves=8)
    assert _err(lib.nndtw_search_plan(ctypes.byref(d), ctypes.byref(opts)), "at most 4 waves") == nd.EUNSUP
    opts = nd._opts(5, "keogh_enh", 0, 0.0, True, 0)
    opts.engine = 3
    assert _err(lib.nndtw_search_plan(ctypes.byref(d), ctypes.byref(opts)), "engine=3") == nd.EINVAL
    for bad in (-2, nd.SEARCH_MAX_HELPERS + 1):
        opts = nd._opts(5, "keogh_enh", 0, 0.0, True, 0, helpers=bad)
        assert _err(lib.nndtw_search_plan(ctypes.byref(d), ctypes.byref(opts)), f"helpers={bad}") == nd.EINVAL
    d.L, d.W = 512, 51                                             # 4 pairs per lane
    for h, want in ((-1, -1), (0, 3), (5, 5)):
        opts = nd._opts(5, "keogh_enh", 0, 0.0, True, 0, helpers=h)
        assert lib.nndtw_search_plan(ctypes.byref(d), ctypes.byref(opts)) == 0 and opts.helpers == want


def test_search_kernels_fit_the_register_file():
    """Every search kernel shape compiles without spilling to scratch memory
    (the resource report the build writes from the compiler's remarks)."""
    from paper_1808_09617_amd import build as hipbuild
    if not os.path.exists(hipbuild.RESOURCES):
        hipbuild.build()
    rows = [l.split() for l in open(hipbuild.RESOURCES) if l.strip() and not l.startswith("#")]
    search = [r for r in rows if "search_kernel" in r[0]]
    assert len(search) >= 2 * 4 + 2 * 4 + 2 * 6             # single-set and batched shapes, strips
    for name, v, a, scratch in search:
        assert int(scratch) == 0, (name, v, a, scratch)
        # strips of 24 and 32 columns run one wave per SIMD (4-wave
        # workgroups) and may use accumulation registers as well
        wide_strip = "search_kernel_strip" in name and ("ILi24E" in name or "ILi32E" in name)
        assert int(v) <= 256 and (int(v) + int(a) <= 512 if wide_strip else int(a) == 0), (name, v, a)


def test_search_eps_floor():
    """The slack must cover the FP32 error of a path sum: eps <= 0 selects the
    floor 2 g / (1 - g), g = (2L + 2) 2^-24, and 0 < eps < floor is rejected
    (a smaller slack could let FP32 rounding drop the nearest neighbour or a
    lower-index tie).  The floor equals the oracle's slack."""
    import oracle
    lib = nd.lib()
    for L in (2, 64, 256, 512, 2048):
        d = nd._Refset()
        d.magic, d.L, d.n, d.W = nd.REFSET_MAGIC, L, 100, max(1, L // 10)
        d.padl, d.ppitch = 4096, 16384
        floor = oracle.slack(L)
        g = (2 * L + 2) * 2.0 ** -24
        assert floor == 2.0 * g / (1.0 - g)
        # twice gamma_{2L+1}, the FP32 error bound of a path sum, is covered
        n1 = (2 * L + 1) * 2.0 ** -24
        assert floor >= 2.0 * n1 / (1.0 - n1)
        for eps in (floor * (1 - 1e-9), floor / 2, 1e-12):
            opts = nd._opts(5, "keogh_enh", 0, eps, True, 0)
            assert _err(lib.nndtw_search_plan(ctypes.byref(d), ctypes.byref(opts)), "FP32 error floor") == nd.EINVAL
        for eps in (0.0, -1.0, floor, 2 * floor, 0.5):
            opts = nd._opts(5, "keogh_enh", 0, eps, True, 0)
            assert lib.nndtw_search_plan(ctypes.byref(d), ctypes.byref(opts)) == 0, (L, eps, nd.last_error())


def test_search_plan_waves_default_follows_query_count():
    """Default waves per query: when the queries would not fill the device at
    4 waves each (at most twice the compute units; 256 when the device cannot
    be queried) 16 for shapes that fit 128 VGPRs (at most 63 diagonal pairs,
    at most 6 pairs per lane), else 8; with more queries 4.  More than 8 waves
    take a default round of at least 512.  An explicit value is kept, and
    more than 8 waves for a shape that does not fit is EUNSUP."""
    lib = nd.lib()
    d = nd._Refset()
    d.magic, d.L, d.n, d.W = nd.REFSET_MAGIC, 512, 5000, 51
    d.padl, d.ppitch = 4096, 16384
    for hint, want in ((0, 4), (1, 16), (500, 16), (512, 16), (513, 4), (100000, 4)):
        opts = nd._opts(5, "keogh_enh", 0, 0.0, True, 0)
        opts.nq_hint = hint
        assert lib.nndtw_search_plan(ctypes.byref(d), ctypes.byref(opts)) == 0
        assert opts.waves == want, (hint, opts.waves)
        assert opts.R == (512 if want == 16 else 256), (hint, opts.R)
    d.W = 128                                   # 129 diagonal pairs: the 8-wave kernels
    opts = nd._opts(5, "keogh_enh", 0, 0.0, True, 0)
    opts.nq_hint = 500
    assert lib.nndtw_search_plan(ctypes.byref(d), ctypes.byref(opts)) == 0 and opts.waves == 8
    opts = nd._opts(5, "keogh_enh", 0, 0.0, True, 0, 12)
    assert _err(lib.nndtw_search_plan(ctypes.byref(d), ctypes.byref(opts)), "more than 8 waves") == nd.EUNSUP
    opts = nd._opts(5, "keogh_enh", 0, 0.0, True, 0, 2)
    opts.nq_hint = 10
    assert lib.nndtw_search_plan(ctypes.byref(d), ctypes.byref(opts)) == 0 and opts.waves == 2
