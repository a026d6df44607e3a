"""GPU parity: every hot-path step through the C ABI against the CPU oracle.

Bars: envelopes, squared ED and both lower bounds bit-exact (FP64 sums in the
same order); FP64 DTW bit-exact; FP32 DTW within 1e-5 relative of the FP64
oracle at every length; search nearest-neighbour indices, FP64 distances and
stage counts bit-exact at the same round size R.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1808_09617_amd as nd  # noqa: E402

DEV = torch.device("cuda:0")
U32 = 2.0 ** -24


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def gamma(n):
    return n * U32 / (1 - n * U32)


def series(n, L, seed, kind="rw"):
    return synth.random_series(n, L, seed, kind)


# ------------------------------------------------------------------ a1
@pytest.mark.parametrize("L", [2, 3, 17, 64, 129, 256, 511, 1000, 1024, 2048])
def test_envelopes_bit_exact(L):
    B = series(37, L, seed=L)
    for W in sorted({0, 1, 2, 5, L // 10, L // 3, L - 2, L - 1, L, 4 * L}):
        say("envelopes", L, W)
        U, Lo = nd.envelopes(dev(B), W)
        ou, ol = oracle.envelopes(B, W)
        assert np.array_equal(host(U), ou) and np.array_equal(host(Lo), ol), (L, W)


def test_refset_build_arrays():
    wl = synth.workload("nndtw-sin256", n_refs=300, n_queries=1)
    W = 26
    say("refset", wl.refs.shape, W)
    rs = nd.RefSet(dev(wl.refs), W)
    ou, ol = oracle.envelopes(wl.refs, W)
    assert np.array_equal(host(rs.B), wl.refs)
    assert np.array_equal(host(rs.U), ou) and np.array_equal(host(rs.Lo), ol)
    assert np.array_equal(host(rs.transposed("Bt")), wl.refs.T)
    assert np.array_equal(host(rs.transposed("Ut")), ou.T)
    assert np.array_equal(host(rs.transposed("Lt")), ol.T)


# ------------------------------------------------------------------ a2 / a3
@pytest.mark.parametrize("L", [2, 5, 64, 300])
def test_pairwise_bounds_bit_exact(L):
    A = series(23, L, seed=2 * L + 1)
    B = series(29, L, seed=2 * L + 2)
    say("ed2", L)
    assert np.array_equal(host(nd.ed2(dev(A), dev(B))), oracle.ed2(A, B))
    assert np.array_equal(host(nd.ed2(dev(A), dev(B[:23]), zip_=True)), oracle.ed2(A, B[:23], zip_=True))
    for W in sorted({0, 1, 4, L // 4, L - 1}):
        U, Lo = oracle.envelopes(B, W)
        say("lb_keogh", L, W)
        assert np.array_equal(host(nd.lb_keogh(dev(A), dev(U), dev(Lo))), oracle.lb_keogh(A, U, Lo))
        for V in sorted({1, 2, 5, L // 2 + 1}):
            say("lb_enhanced", L, W, V)
            got = host(nd.lb_enhanced(dev(A), dev(B), dev(U), dev(Lo), W, V))
            assert np.array_equal(got, oracle.lb_enhanced(A, B, U, Lo, W, V)), (L, W, V)
            gz = host(nd.lb_enhanced(dev(A), dev(B[:23]), dev(U[:23]), dev(Lo[:23]), W, V, zip_=True))
            assert np.array_equal(gz, oracle.lb_enhanced(A, B[:23], U[:23], Lo[:23], W, V, zip_=True))
            bands = oracle.lb_enhanced(A, B, U, Lo, W, V, variant="bands")
            cut = np.median(bands, axis=1)
            gc = host(nd.lb_enhanced(dev(A), dev(B), dev(U), dev(Lo), W, V, cutoff=dev(cut)))
            assert np.array_equal(gc, oracle.lb_enhanced(A, B, U, Lo, W, V, cutoff=cut)), (L, W, V)


@pytest.mark.parametrize("name,W,V", [("nndtw-small", 6, 1), ("nndtw-sin256", 26, 5), ("nndtw-mix512", 51, 5),
                                      ("nndtw-mix512", 511, 1)])
def test_cascade_bounds_bit_exact(name, W, V):
    wl = synth.workload(name, n_refs=333, n_queries=21)
    say("cascade_bounds", name, W, V)
    rs = nd.RefSet(dev(wl.refs), W)
    e, k, b, f = (host(x) for x in nd.cascade_bounds(rs, dev(wl.queries), V))
    U, Lo = oracle.envelopes(wl.refs, W)
    assert np.array_equal(e, oracle.ed2(wl.queries, wl.refs))
    assert np.array_equal(k, oracle.lb_keogh(wl.queries, U, Lo))
    assert np.array_equal(b, oracle.lb_enhanced(wl.queries, wl.refs, U, Lo, W, V, variant="bands"))
    assert np.array_equal(f, oracle.lb_enhanced(wl.queries, wl.refs, U, Lo, W, V))


@pytest.mark.parametrize("L,W,V", [(2, 1, 1), (5, 2, 2), (17, 3, 5), (128, 13, 5), (129, 13, 5), (300, 30, 5),
                                   (1024, 102, 5)])
def test_cascade_bounds_one_query_bit_exact(L, W, V):
    """One query across lengths around the 8-point prefetch ring and the
    128-point staging chunk, and reference counts around the 256-reference
    tile."""
    for n in (1, 255, 257):
        refs = series(n, L, seed=1500 + L + n)
        q = series(1, L, seed=1600 + L)
        say("cascade_bounds one query", L, W, V, n)
        rs = nd.RefSet(dev(refs), W)
        e, k, b, f = (host(x) for x in nd.cascade_bounds(rs, dev(q), V))
        U, Lo = oracle.envelopes(refs, W)
        assert np.array_equal(e, oracle.ed2(q, refs))
        assert np.array_equal(k, oracle.lb_keogh(q, U, Lo))
        assert np.array_equal(b, oracle.lb_enhanced(q, refs, U, Lo, W, V, variant="bands"))
        assert np.array_equal(f, oracle.lb_enhanced(q, refs, U, Lo, W, V))


# ------------------------------------------------------------------ a5
DTW_CASES = [(2, 0), (2, 1), (3, 1), (3, 5), (8, 0), (8, 3), (8, 7), (24, 2), (64, 6), (64, 63), (97, 13),
             (256, 26), (256, 255), (512, 5), (512, 51), (512, 128), (512, 256), (512, 511), (1000, 100),
             (2048, 205), (2048, 1000), (700, 699), (1500, 1499), (2048, 1500), (2048, 2047)]


@pytest.mark.parametrize("L,W", DTW_CASES)
def test_dtw_fp64_bit_exact_and_fp32_tolerance(L, W):
    nA, nB = (5, 7) if L >= 1000 else (9, 11)
    A = series(nA, L, seed=L + 7 * W)
    B = series(nB, L, seed=L + 7 * W + 1)
    say("dtw", L, W)
    ref = oracle.dtw(A, B, W)
    d64 = host(nd.dtw_w(dev(A), dev(B), W, f64=True))
    assert np.array_equal(d64, ref), (L, W, np.max(np.abs(d64 - ref)))
    d32 = host(nd.dtw_w(dev(A), dev(B), W)).astype(np.float64)
    rel = np.abs(d32 - ref) / np.maximum(ref, 1e-30)
    say("dtw", L, W, "fp32 max relative error", float(rel.max()))
    assert rel.max() <= 1e-5, (L, W, rel.max())
    z64 = host(nd.dtw_w(dev(A[:5]), dev(B[:5]), W, zip_=True, f64=True))
    assert np.array_equal(z64, oracle.dtw(A[:5], B[:5], W, zip_=True))


@pytest.mark.parametrize("L,W", [(1000, 100), (1000, 999), (2048, 205), (2048, 1007), (2048, 2047)])
def test_dtw_fp32_long_series(L, W):
    """FP32 DTW_W at the longest lengths against the FP64 oracle at 1e-5
    relative (the error of an FP32 path sum is typically sqrt(2L) u, far below
    its worst-case bound gamma_{2L+1}); the observed maximum is printed."""
    A = series(16, L, seed=5 * L + W, kind="rw")
    B = np.concatenate([series(8, L, seed=5 * L + W + 1, kind="rw"),
                        series(8, L, seed=5 * L + W + 2, kind="sin5")], 0)
    say("dtw fp32 long", L, W)
    ref = oracle.dtw(A, B, W)
    d32 = host(nd.dtw_w(dev(A), dev(B), W)).astype(np.float64)
    rel = np.abs(d32 - ref) / np.maximum(ref, 1e-30)
    say("dtw fp32 long", L, W, "max relative error", float(rel.max()))
    assert rel.max() <= 1e-5, (L, W, rel.max())


def test_dtw_special_inputs():
    L = 40
    A = series(6, L, seed=3)
    const = np.zeros((2, L), np.float32)
    B = np.concatenate([A[:2], const, -A[2:4]], 0)
    for W in (0, 3, 39):
        say("dtw special", W)
        ref = oracle.dtw(A, B, W)
        assert np.array_equal(host(nd.dtw_w(dev(A), dev(B), W, f64=True)), ref)
        d32 = host(nd.dtw_w(dev(A), dev(B), W))
        assert np.all(d32[np.arange(2), np.arange(2)] == 0.0)         # DTW(A, A) = 0
        assert np.allclose(d32, ref, rtol=1e-5, atol=0)
    # W = 0 is the squared Euclidean distance
    assert np.array_equal(host(nd.dtw_w(dev(A), dev(B), 0, f64=True)), oracle.ed2(A, B))


@pytest.mark.parametrize("L,W", [(64, 6), (256, 26), (512, 128), (300, 299), (2048, 2047), (1200, 900)])
def test_dtw_cutoff_abandon(L, W):
    A = series(8, L, seed=50 + W)
    B = series(16, L, seed=51 + W)
    ref = oracle.dtw(A, B, W)
    for f in (0.5, 0.9, 1.0, 1.2):
        cut = np.quantile(ref, 0.5, axis=1) * f
        say("dtw cutoff", L, W, f)
        for f64 in (False, True):
            got = host(nd.dtw_w(dev(A), dev(B), W, cutoff=dev(cut), f64=f64)).astype(np.float64)
            ab = np.isinf(got)
            assert np.all(ref[ab] > cut[:, None].repeat(B.shape[0], 1)[ab] / (1 + gamma(2 * L + 1)))
            ok = ~ab
            if f64:
                assert np.array_equal(got[ok], ref[ok])
            else:
                assert np.allclose(got[ok], ref[ok], rtol=1e-5, atol=0)
            # never abandoned when the true value is below the cutoff
            assert not np.any(ab & (ref <= cut[:, None] / (1 + gamma(2 * L + 1))))


def test_dtw_tightness_pairs_zip():
    a, b = synth.tightness_pairs(4000)
    say("tightness zip", a.shape)
    d = host(nd.dtw_w(dev(a), dev(b), 26, zip_=True)).astype(np.float64)
    ref = oracle.dtw(a, b, 26, zip_=True)
    assert np.allclose(d, ref, rtol=1e-5, atol=0)


# ------------------------------------------------------------------ search
def run_search(refs, queries, W, V, cascade="keogh_enh", R=0, init_ub=True, cpl=0, waves=0, engine="auto",
               helpers=0, order="auto"):
    rs = nd.RefSet(dev(refs), W)
    idx, dist, counts, R_used = nd.search(rs, dev(queries), V=V, cascade=cascade, R=R, init_ub=init_ub, cpl=cpl,
                                          waves=waves, engine=engine, helpers=helpers, order=order)
    return host(idx), host(dist), host(counts), R_used


def check_search(refs, queries, W, V, cascade="keogh_enh", R=0, init_ub=True, cpl=0, brute=True, waves=0,
                 engine="auto", helpers=0, order="auto"):
    say("search", refs.shape, queries.shape, W, V, cascade, R, init_ub, cpl, waves, engine, helpers, order)
    gi, gd, gc, R_used = run_search(refs, queries, W, V, cascade, R, init_ub, cpl, waves, engine, helpers, order)
    oi, od, oc = oracle.search(refs, queries, W, V, cascade, R_used, init_ub)
    assert np.array_equal(gi, oi), ("nn_idx", np.nonzero(gi != oi))
    assert np.array_equal(gd, od), ("nn_dist", np.max(np.abs(gd - od)))
    assert np.array_equal(gc[:, :5], oc[:, :5]), ("counts", gc[:3], oc[:3])
    assert np.all(gc[:, 1:5].sum(1) == refs.shape[0])
    if brute:
        bi, bd = oracle.brute_nn(refs, queries, W)
        assert np.array_equal(gi, bi) and np.array_equal(gd, bd)
    return gc, R_used


def test_search_small_workload_all_cascades():
    wl = synth.workload("nndtw-small")
    for cascade in ("none", "keogh", "keogh_enh", "enh"):
        for R in (0, 1, 5, 64, 100):
            check_search(wl.refs, wl.queries, 6, 1, cascade, R)


def test_search_init_ub_and_v():
    wl = synth.workload("nndtw-small")
    for V in (1, 2, 5, 40):
        for init_ub in (False, True):
            check_search(wl.refs, wl.queries, 6, V, "keogh_enh", 7, init_ub)


@pytest.mark.parametrize("W", [0, 1, 3, 12, 31, 32, 100])
def test_search_windows_and_shapes(W):
    refs = series(150, 64, seed=300 + W, kind="sin5")
    queries = series(12, 64, seed=400 + W, kind="sin5")
    for cpl in (0, 1, 2, 4):
        Wp = min(W, 63)
        if -(-(Wp + 1) // cpl if cpl else 1) > 63:
            continue
        check_search(refs, queries, W, 3, "keogh_enh", 0, True, cpl)


def test_search_ties_duplicates_and_exact_matches():
    base = series(40, 48, seed=77)
    refs = np.concatenate([base[[5, 9]], base, base[[5, 9, 5]]], 0)
    queries = np.ascontiguousarray(base[[5, 9, 20]])
    for R in (1, 3, 64):
        gc, _ = check_search(refs, queries, 4, 2, "keogh_enh", R)
    gi, gd, _, _ = run_search(refs, queries, 4, 2)
    assert gi.tolist()[:2] == [0, 1] and np.all(gd == 0.0)
    same = np.repeat(base[:1], 9, 0)
    check_search(same, base[1:4], 3, 1, "keogh_enh", 2)
    check_search(same, base[:1], 3, 1, "keogh_enh", 2)      # every distance is 0


def test_search_tiny_lengths_and_constant_series():
    for L in (2, 3, 5):
        refs = series(30, L, seed=L + 90)
        queries = series(6, L, seed=L + 91)
        for W in range(0, L + 1):
            check_search(refs, queries, W, 1)
    refs = np.zeros((10, 16), np.float32)
    refs[3] = 1.0
    check_search(refs, series(3, 16, seed=5), 2, 2)


def test_search_sin256_subset():
    wl = synth.workload("nndtw-sin256", n_refs=1000, n_queries=60)
    for V in (1, 2, 5):
        check_search(wl.refs, wl.queries, 26, V, "keogh_enh", 0, True, 0, brute=False)
    check_search(wl.refs, wl.queries[:20], 26, 5, "keogh", 0, True, 0, brute=False)


@pytest.mark.parametrize("n", [1, 63, 256, 257, 300, 1024, 1025, 2049, 4096, 4100, 8192])
def test_search_reference_counts(n):
    """Reference-set sizes around every power of two the visiting-order sort
    handles (1 to 32 positions per thread), against the oracle."""
    refs = series(n, 24, seed=900 + n % 97, kind="sin5")
    queries = series(5, 24, seed=901, kind="sin5")
    check_search(refs, queries, 3, 2, "keogh_enh", 0, True, 0, brute=n <= 2049)


def _al256(x):
    return (x + 255) // 256 * 256


def _ordered_region(searcher, n):
    """The visiting order and the bounds gathered in it, as the search's
    workspace holds them after a call (squared ED, LB_Keogh, both LB_Enhanced
    parts, then the sorted indices and the three gathered bounds)."""
    m = searcher.nQ * n
    sk = 4 * _al256(m * 8)
    slbk = sk + _al256(m * 4)
    parts = [searcher.ws[sk:sk + m * 4]] + [searcher.ws[o:o + m * 8] for o in
                                            (slbk, slbk + _al256(m * 8), slbk + 2 * _al256(m * 8))]
    return host(torch.cat(parts))           # (the 256-byte alignment gaps between them hold nothing)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 127, 1000, 4100, 8192])
def test_search_order_by_rank_equals_sort(n):
    """The two ways of finding the visiting order give the same order and the
    same gathered bounds, byte for byte, and the same search result, which is
    the oracle's.  Duplicated references give equal squared distances (ties
    broken by index), and a query equal to a reference a distance of 0."""
    base = series(max(1, n // 3), 40, seed=1300 + n, kind="sin5")
    refs = np.ascontiguousarray(np.resize(base, (n, 40)))        # every row repeated about three times
    queries = np.ascontiguousarray(np.concatenate([refs[n // 2:n // 2 + 1], series(3, 40, seed=1301)], 0))
    rs = nd.RefSet(dev(refs), 4)
    region, results = [], []
    for order in ("sort", "rank"):
        say("order", order, "n", n)
        s = nd.Searcher(rs, queries.shape[0], V=2, order=order)
        idx, dist, counts = s(dev(queries))
        torch.cuda.synchronize()
        region.append(_ordered_region(s, n))
        results.append((host(idx), host(dist), host(counts)))
    assert np.array_equal(region[0], region[1])
    (i0, d0, c0), (i1, d1, c1) = results
    assert np.array_equal(i0, i1) and np.array_equal(d0, d1) and np.array_equal(c0[:, :5], c1[:, :5])
    sk = region[1][: queries.shape[0] * n * 4].view(np.uint32).reshape(queries.shape[0], n)
    assert np.array_equal(np.sort(sk, 1), np.tile(np.arange(n, dtype=np.uint32), (queries.shape[0], 1)))
    check_search(refs, queries, 4, 2, "keogh_enh", 0, True, 0, brute=n <= 1000, order="rank")


def test_search_order_choice_and_limits():
    """The library ranks while nQ n^2 <= 2^16 npow (the result is the same
    either way); ranking is refused above 8192 references."""
    refs = series(300, 24, seed=1400, kind="sin5")
    queries = series(4, 24, seed=1401, kind="sin5")
    for order in ("auto", "sort", "rank"):
        check_search(refs, queries, 3, 2, "keogh_enh", 0, True, 0, brute=True, order=order)
    big = nd.RefSet(dev(series(8193, 24, seed=1402, kind="sin5")), 3)
    with pytest.raises(RuntimeError, match="ordering by ranking"):
        nd.search(big, dev(queries[:1]), V=2, order="rank")


@pytest.mark.parametrize("n", [8193, 16384, 16385, 40000])
def test_search_large_reference_sets(n):
    """Reference sets above the on-chip sort (8192): the visiting order is
    sorted in chunks and merged; sizes around one, two and five chunks."""
    refs = series(n, 24, seed=700 + n % 89, kind="sin5")
    queries = series(6, 24, seed=701, kind="sin5")
    for R in (0, 1000):
        check_search(refs, queries, 3, 2, "keogh_enh", R, True, 0, brute=False)


def test_search_hbm512_sampled():
    """The 200,000 x 512 reference set (W=51, V=5) searched end to end: four
    queries against the oracle at the same R."""
    hb = synth.workload("nndtw-hbm512")
    qs = np.ascontiguousarray(hb.queries[:4])
    check_search(hb.refs, qs, 51, 5, "keogh_enh", 0, True, 0, brute=False)


@pytest.mark.parametrize("waves", [1, 2, 3, 5, 8, 12, 16])
def test_search_waves_per_query(waves):
    """Every workgroup size gives the oracle's result and counts (the waves of
    a query share its DTW tasks)."""
    wl = synth.workload("nndtw-sin256", n_refs=1000, n_queries=40)
    for R in (0, 1, 37, 300):
        check_search(wl.refs, wl.queries, 26, 5, "keogh_enh", R, True, 0, brute=False, waves=waves)
    refs = series(90, 64, seed=31)
    check_search(refs, series(5, 64, seed=32), 12, 2, "keogh_enh", 0, True, 1, waves=waves)


@pytest.mark.parametrize("W", [5, 51, 128, 256, 511])
def test_search_mix512_full(W):
    """The window-sweep workload (5000 x 500, L=512) in its benchmarked launch
    shape against the oracle at the same R, over the full reference set: every
    query at W = 5 and 51 (0.01 L and 0.1 L), 25 queries spread over the set
    at the wide windows (the oracle's DTWs cost up to L^2 cells each)."""
    wl = synth.workload("nndtw-mix512", n_refs=5000, n_queries=500)
    sel = np.arange(500) if W <= 51 else np.linspace(0, 499, 25).astype(int)
    for V in (1, 5):
        check_search(wl.refs, wl.queries[sel], W, V, "keogh_enh", 0, True, 0, brute=False)


@pytest.mark.parametrize("L,W", [(2048, 205), (2048, 566), (1200, 566), (560, 559)])
def test_search_long_series_and_widest_windows(L, W):
    """Maximum length and the widest windows the diagonal engine compiles for
    the search (9 pairs per lane, min(W, L-1) + 1 = 567), forced, and the
    library's choice, against the oracle at the same R."""
    refs = series(60, L, seed=L + W, kind="rw")
    queries = series(3, L, seed=L + W + 1, kind="rw")
    for V in (1, 5):
        for engine in ("diagonal", "auto"):
            check_search(refs, queries, W, V, "keogh_enh", 0, True, 0, brute=False, engine=engine)


@pytest.mark.parametrize("L,W", [(64, 63), (100, 60), (300, 299), (512, 300), (700, 650), (1100, 1099),
                                 (2048, 1000), (2048, 2047)])
def test_search_strip_engine(L, W):
    """The row-strip engine in the search (the library's choice for windows
    too wide for the diagonal shapes and for unconstrained DTW at L > 192,
    forced elsewhere), up to unconstrained DTW at the maximum length, against
    the oracle at the same R and against brute force."""
    refs = series(40, L, seed=3 * L + W, kind="rw")
    queries = series(3, L, seed=3 * L + W + 1, kind="rw")
    s = nd.Searcher(nd.RefSet(dev(refs), W), 3)
    s(dev(queries))
    Wp = min(W, L - 1)
    auto_strip = Wp + 1 > 567 or (Wp == L - 1 and L > 192)
    assert s.engine == ("strip" if auto_strip else "diagonal"), (L, W, s.engine)
    for V in (1, 5):
        check_search(refs, queries, W, V, "keogh_enh", 0, True, 0, brute=V == 1, engine="strip")
    check_search(refs, queries, W, 2, "keogh_enh", 7, False, 0, brute=False, engine="strip")


def _helpers_joined(searcher, n, L, nq):
    """Helper workgroups that joined each query in the last call, read from
    the workspace (the shared-batch headers follow the bound and order
    arrays and the cells table; QueryShare: 3136 bytes, helpers word at byte
    20 = (call tag << 12) | count)."""
    al = lambda x: (x + 255) // 256 * 256
    m = nq * n
    off = 4 * al(8 * m) + al(4 * m) + 3 * al(8 * m) + al(8 * L)
    raw = searcher.ws[off: off + nq * 3136].cpu().numpy().view(np.uint32).reshape(nq, 3136 // 4)
    say("share header of query 0 (deal lo/hi, done, nt, thrF, helpers, finished, started):", raw[0, :8].tolist())
    return raw[:, 5] & 0xFFF


@pytest.mark.parametrize("W,helpers", [(12, -1), (12, 1), (12, 3), (12, 7), (40, 7)])
def test_search_helper_workgroups(W, helpers):
    """Helper workgroups (launched after the queries' own, they take DTW tasks
    of the queries still running) change neither the result nor the defined
    counts: against the oracle at the same R, with few enough queries that
    the helpers start at once and join every query."""
    L = 128
    refs = series(3000, L, seed=810 + W, kind="rw")
    queries = series(24, L, seed=811 + W, kind="rw")
    check_search(refs, queries, W, 3, "keogh_enh", 0, True, 0, brute=False, helpers=helpers)
    if helpers <= 0:
        return
    rs = nd.RefSet(dev(refs), W)
    s = nd.Searcher(rs, 24, V=3, helpers=helpers)
    s(dev(queries))
    torch.cuda.synchronize()
    joined = _helpers_joined(s, 3000, L, 24)
    say("helpers", W, helpers, "engine", s.engine, "cpl", s.cpl, "joined", joined.tolist())
    assert s.cpl not in (3, 6) and s.helpers == helpers
    assert np.all(joined == helpers)              # every helper joined its query


@pytest.mark.parametrize("L,W", [(300, 299), (700, 650)])
def test_search_helper_workgroups_strips(L, W):
    """Helper workgroups on the row-strip engine: results and defined counts
    equal the oracle's, and every helper joined its query."""
    refs = series(600, L, seed=820 + W, kind="rw")
    queries = series(12, L, seed=821 + W, kind="rw")
    check_search(refs, queries, W, 3, "keogh_enh", 0, True, 0, brute=False, helpers=3)
    rs = nd.RefSet(dev(refs), W)
    s = nd.Searcher(rs, 12, V=3, helpers=3)
    s(dev(queries))
    torch.cuda.synchronize()
    joined = _helpers_joined(s, 600, L, 12)
    say("helpers strips", L, W, "engine", s.engine, "joined", joined.tolist())
    assert s.engine == "strip" and np.all(joined == 3)


def test_search_helpers_headline_shape():
    """The headline launch shape (5000 references, L=512, W=51, 16 waves per
    query, 4 pairs per lane) with 7 helpers per query for 40 queries: every
    query against the oracle."""
    wl = synth.workload("nndtw-mix512", n_refs=5000, n_queries=500)
    qs = np.ascontiguousarray(wl.queries[::12][:40])
    check_search(wl.refs, qs, 51, 5, "keogh_enh", 0, True, 0, brute=False, helpers=7)


@pytest.mark.parametrize("L,W", [(40, 15), (256, 100), (512, 128), (600, 566)])
def test_search_engines_agree(L, W):
    """Windows both engines take: the strip engine forced, the diagonal engine
    forced and the library's choice give the oracle's result and counts, with
    1 to 8 waves per query."""
    refs = series(120, L, seed=5 * L + W, kind="sin5")
    queries = series(4, L, seed=5 * L + W + 1, kind="sin5")
    for engine in ("strip", "diagonal", "auto"):
        for waves in (1, 3, 8):
            check_search(refs, queries, W, 3, "keogh_enh", 0, True, 0, brute=False, waves=waves, engine=engine)


@pytest.mark.parametrize("L,W", [(64, 6), (256, 26), (300, 299), (512, 128), (512, 400), (2048, 2047)])
def test_search_cell_counts_of_complete_dtws(L, W):
    """References identical to the query: every distance is 0, the threshold
    is 0 and no DTW is abandoned (the test is strict), so the cells the search
    reports (the units of the roofline figure) are N times the window's cell
    count L(2W'+1) - W'(W'+1)."""
    q = series(1, L, seed=L + W)
    refs = np.repeat(q, 37, 0)
    gi, gd, gc, _ = run_search(refs, q, W, 2)
    Wp = min(W, L - 1)
    assert gi[0] == 0 and gd[0] == 0.0
    assert gc[0, 4] == 37 and gc[0, 5] == 0
    assert gc[0, 6] == 37 * (L * (2 * Wp + 1) - Wp * (Wp + 1))


def test_search_full_sin256_all_queries():
    """Full-size benchmarked workload (1000 x 1000, L=256, W=26, V=5) in its
    launch shape: every query against the oracle at the same R (index, FP64
    distance, defined counts), plus properties that hold at any size."""
    wl = synth.workload("nndtw-sin256")
    say("search full sin256")
    gi, gd, gc, R = run_search(wl.refs, wl.queries, 26, 5)
    assert np.all(gc[:, 1:5].sum(1) == 1000)
    # the reported distance is the FP64 DTW of the reported neighbour
    assert np.array_equal(gd, oracle.dtw(wl.queries, wl.refs[gi], 26, zip_=True))
    oi, od, oc = oracle.search(wl.refs, wl.queries, 26, 5, "keogh_enh", R, True)
    assert np.array_equal(gi, oi), ("nn_idx", np.nonzero(gi != oi))
    assert np.array_equal(gd, od)
    assert np.array_equal(gc[:, :5], oc[:, :5]), ("counts", np.nonzero(np.any(gc[:, :5] != oc[:, :5], 1)))


def test_search_eps_floor_with_duplicates():
    """Duplicated references (exact ties of DTW and of the visiting key) at the
    smallest slack accepted, given explicitly: the lowest index wins, and the
    result and counts equal the oracle's (whose slack is that floor)."""
    base = series(60, 128, seed=8080, kind="sin5")
    refs = np.concatenate([base, base[::-1], base[:20]], 0)
    queries = np.ascontiguousarray(np.concatenate([base[[3, 17, 59]], series(5, 128, seed=8081, kind="sin5")]))
    floor = oracle.slack(128)
    rs = nd.RefSet(dev(refs), 13)
    for R in (0, 1, 16):
        say("eps floor", R)
        idx, dist, counts, R_used = nd.search(rs, dev(queries), V=3, R=R, eps=floor)
        gi, gd, gc = host(idx), host(dist), host(counts)
        oi, od, oc = oracle.search(refs, queries, 13, 3, "keogh_enh", R_used, True)
        assert np.array_equal(gi, oi) and np.array_equal(gd, od) and np.array_equal(gc[:, :5], oc[:, :5])
        assert gi[:3].tolist() == [3, 17, 59] and np.all(gd[:3] == 0.0)
    with pytest.raises(nd.NNDTWError):
        nd.search(rs, dev(queries), V=3, eps=floor / 2)


# ------------------------------------------------------------------ batching
def run_batch(datasets, V=5, R=None, cpl=None, waves=0, helpers=0, order="auto"):
    pairs = [(nd.RefSet(dev(ds.refs), ds.W), dev(ds.queries)) for ds in datasets]
    bsr = nd.BatchSearcher(pairs, V=V, R=R, cpl=cpl, waves=waves, helpers=helpers, order=order)
    out = bsr()
    return bsr, pairs, [(host(i), host(d), host(c)) for i, d, c in out]


@pytest.mark.parametrize("waves", [0, 2, 8])
def test_batch_matches_single_search_and_oracle(waves):
    """Every set of a ragged batch gives exactly the single-set search (index,
    distance, the five defined counts) at the R and shape the batch used, and
    the oracle on a sample of its queries.  The implementation-defined counts
    (abandoned, cells, rechecks) depend on which DTW of a round finishes first
    and are only checked for consistency."""
    sets = synth.batch_workload(n_sets=10, L_range=(24, 700), N_range=(50, 600), q_frac=0.05)
    say("batch", len(sets), "sets, waves", waves)
    bsr, pairs, res = run_batch(sets, waves=waves)
    for d, ds in enumerate(sets):
        say("batch set", d, ds.refs.shape, ds.queries.shape, ds.W, bsr.R[d], bsr.cpl[d])
        gi, gd, gc = res[d]
        si, sd, sc, _ = nd.search(pairs[d][0], pairs[d][1], V=5, R=bsr.R[d], cpl=bsr.cpl[d], waves=waves)
        assert np.array_equal(gi, host(si)) and np.array_equal(gd, host(sd))
        assert np.array_equal(gc[:, :5], host(sc)[:, :5])
        assert np.all(gc[:, 5] <= gc[:, 4]) and np.all(gc[:, 6] >= 0) and np.all(gc[:, 7] >= (gc[:, 4] > 0))
        oi, od, oc = oracle.search(ds.refs, ds.queries[:3], ds.W, 5, "keogh_enh", bsr.R[d], True)
        assert np.array_equal(gi[:3], oi) and np.array_equal(gd[:3], od)
        assert np.array_equal(gc[:3, :5], oc[:, :5])


@pytest.mark.parametrize("n_sets,q_frac,helpers", [(4, 0.002, 0), (8, 0.05, -1)])
def test_batch_order_by_rank_equals_sort(n_sets, q_frac, helpers):
    """A batch ordered by ranking (one launch for all its sets) and by the
    per-width sorts gives every set the same result; the library's choice
    ranks a batch of a few queries and sorts a large one."""
    sets = synth.batch_workload(n_sets=n_sets, L_range=(24, 700), N_range=(50, 3000), q_frac=q_frac)
    res, Rs = {}, {}
    for order in ("sort", "rank", "auto"):
        say("batch order", order, "queries", sum(ds.queries.shape[0] for ds in sets))
        bsr, _, res[order] = run_batch(sets, helpers=helpers, order=order)
        Rs[order] = bsr.R
        npow = 256
        while npow < max(ds.refs.shape[0] for ds in sets):
            npow *= 2
        assert bsr.order_rank == (order == "rank" or (order == "auto" and sum(
            ds.queries.shape[0] * ds.refs.shape[0] ** 2 for ds in sets) <= (1 << 16) * npow))
    for d, ds in enumerate(sets):
        for order in ("rank", "auto"):
            (gi, gd, gc), (si, sd, sc) = res[order][d], res["sort"][d]
            assert np.array_equal(gi, si) and np.array_equal(gd, sd) and np.array_equal(gc[:, :5], sc[:, :5])
    ds = sets[-1]
    nq = min(3, ds.queries.shape[0])
    if nq:
        assert Rs["rank"] == Rs["sort"]
        oi, od, oc = oracle.search(ds.refs, ds.queries[:nq], ds.W, 5, "keogh_enh", Rs["rank"][-1], True)
        gi, gd, gc = res["rank"][-1]
        assert np.array_equal(gi[:nq], oi) and np.array_equal(gd[:nq], od) and np.array_equal(gc[:nq, :5], oc[:, :5])


def test_batch_one_query_per_set():
    """A batch in which no set has more than one query (a serving batch: the
    bound pass runs its one-query body on every tile, the order is ranked);
    every set's result is the single search's and the oracle's."""
    sets = synth.batch_workload(n_sets=6, L_range=(24, 1100), N_range=(50, 2500), q_frac=0.1)
    sets = [synth.BatchDataset(ds.refs, ds.queries[:1], ds.W, ds.V) for ds in sets]
    sets[2] = synth.BatchDataset(sets[2].refs, sets[2].queries[:0], sets[2].W, sets[2].V)   # and one with none
    bsr, pairs, res = run_batch(sets)
    for d, ds in enumerate(sets):
        gi, gd, gc = res[d]
        if ds.queries.shape[0] == 0:
            assert gi.shape == (0,)
            continue
        si, sd, sc, _ = nd.search(pairs[d][0], pairs[d][1], V=5, R=bsr.R[d], cpl=bsr.cpl[d])
        assert np.array_equal(gi, host(si)) and np.array_equal(gd, host(sd))
        assert np.array_equal(gc[:, :5], host(sc)[:, :5])
        oi, od, oc = oracle.search(ds.refs, ds.queries, ds.W, 5, "keogh_enh", bsr.R[d], True)
        assert np.array_equal(gi, oi) and np.array_equal(gd, od) and np.array_equal(gc[:, :5], oc[:, :5])


def test_tuners_pick_valid_schedules():
    """Both tuners return, per set, a schedule from their candidates (the
    throughput tuner one per (L, W) bucket); a batch run with the tuned round
    sizes and shapes gives each set the oracle's result, and a single-query
    batch with the latency tuner's helper choice the same result."""
    from paper_1808_09617_amd import tune
    sets = synth.batch_workload(n_sets=3, L_range=(40, 400), N_range=(200, 600), q_frac=0.02)
    pairs = [(nd.RefSet(dev(ds.refs), ds.W), dev(ds.queries)) for ds in sets]
    R, cpl, report = tune.autotune(pairs, V=5, R_candidates=(64, 256), reps=1)
    assert all(r in (64, 256) for r in R) and all(1 <= c <= 4 for c in cpl)
    assert sum(v["sets"] for v in report.values()) == len(sets)
    R_lat, helpers, lat = tune.tune_latency(pairs, cpl, V=5, R_candidates=(128, 256), reps=2)
    assert all(r in (128, 256) for r in R_lat) and all(h in (-1, 0) for h in helpers) and len(lat) == len(sets)
    bsr = nd.BatchSearcher(pairs, V=5, R=R, cpl=cpl)
    out = bsr()
    for d, ds in enumerate(sets):
        gi, gd, gc = (host(x) for x in out[d])
        oi, od, oc = oracle.search(ds.refs, ds.queries, ds.W, 5, "keogh_enh", bsr.R[d], True)
        assert np.array_equal(gi, oi) and np.array_equal(gd, od) and np.array_equal(gc[:, :5], oc[:, :5])
        one = nd.BatchSearcher([(pairs[d][0], pairs[d][1][:1])], V=5, R=[R_lat[d]], cpl=[cpl[d]],
                               helpers=helpers[d])
        i1, d1, c1 = (host(x) for x in one()[0])
        oi, od, oc = oracle.search(ds.refs, ds.queries[:1], ds.W, 5, "keogh_enh", one.R[0], True)
        assert i1[0] == oi[0] and d1[0] == od[0] and np.array_equal(c1[:, :5], oc[:, :5])


def test_batch_rounds_and_shapes_per_set():
    """Per-set R and engine shape overrides (as an autotuner sets them)."""
    sets = synth.batch_workload(n_sets=5, L_range=(30, 200), N_range=(60, 300), q_frac=0.05)
    R = [1, 7, 64, 0, 300]
    cpl = [1, 2, 0, 4, 3]
    bsr, pairs, res = run_batch(sets, R=R, cpl=cpl)
    for d, ds in enumerate(sets):
        if R[d]:
            assert bsr.R[d] == R[d]
        if cpl[d]:
            assert bsr.cpl[d] == cpl[d]
        oi, od, oc = oracle.search(ds.refs, ds.queries, ds.W, 5, "keogh_enh", bsr.R[d], True)
        gi, gd, gc = res[d]
        assert np.array_equal(gi, oi) and np.array_equal(gd, od) and np.array_equal(gc[:, :5], oc[:, :5])


def test_batch_graph_replay():
    """The launch sequence captured in a graph: every replay, with eager work
    and synchronisation between replays, reproduces the eager result."""
    sets = synth.batch_workload(n_sets=6, L_range=(24, 300), N_range=(50, 400), q_frac=0.05)
    bsr, pairs, ref = run_batch(sets)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bsr()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bsr()
    for rep in range(3):
        say("graph replay", rep)
        for i, dd, c in bsr.out:
            i.fill_(-7)
            dd.fill_(-1.0)
            c.fill_(-3)
        x = torch.randn(4096, device=DEV)
        (x * x).sum().item()
        g.replay()
        torch.cuda.synchronize()
        for d, (i, dd, c) in enumerate(bsr.out):
            assert np.array_equal(host(i), ref[d][0]) and np.array_equal(host(dd), ref[d][1])
            assert np.array_equal(host(c)[:, :5], ref[d][2][:, :5])


def _batch_helper_counts(bsr):
    """Helper workgroups that joined each item's query in the last call: the
    helpers word of the items' headers in the workspace (3136-byte
    QueryShare at plan.share_off per item, byte 20 = (1 << 12) | count)."""
    n, off = int(bsr.plan.items), int(bsr.plan.share_off)
    raw = bsr.ws[off:off + n * 3136].view(n, 3136)[:, 20:24].contiguous().cpu().numpy().view(np.uint32).ravel()
    return np.where((raw >> 12) == 1, raw & 0xFFF, 0)


@pytest.mark.parametrize("helpers", [-1, 1, 3, 0])
def test_batch_helper_workgroups(helpers):
    """A batch of a few long queries (each search kernel is all tail): the
    idle persistent workgroups join the running queries, at most `helpers`
    per query (0: the default 7, -1: none), and every result and defined
    count equals the oracle's at the batch's R."""
    sets = synth.batch_workload(n_sets=3, L_range=(500, 900), N_range=(500, 700), q_frac=0.004)
    say("batch helpers", helpers, [ds.queries.shape for ds in sets])
    bsr, pairs, res = run_batch(sets, helpers=helpers)
    cap = {-1: 0, 0: 7}.get(helpers, helpers)
    assert bsr.helpers == cap
    if cap > 0:
        assert int(bsr.plan.share_shapes) != 0
        joined = _batch_helper_counts(bsr)
        say("batch helpers joined", joined.tolist())
        assert joined.max() >= 1 and joined.max() <= cap
    else:
        assert int(bsr.plan.share_shapes) == 0
    for d, ds in enumerate(sets):
        gi, gd, gc = res[d]
        oi, od, oc = oracle.search(ds.refs, ds.queries, ds.W, 5, "keogh_enh", bsr.R[d], True)
        assert np.array_equal(gi, oi) and np.array_equal(gd, od) and np.array_equal(gc[:, :5], oc[:, :5])


@pytest.mark.parametrize("name,W,V,helpers", [("nndtw-small", 6, 1, 0), ("nndtw-sin256", 26, 5, 3)])
def test_search_graph_replay(name, W, V, helpers):
    """The single search captured in a graph (one launch per call): every
    replay, with eager work and synchronisation between replays, reproduces
    the eager result (with helper workgroups too, whose headers the captured
    reset kernel clears on every replay)."""
    wl = synth.workload(name)
    nq = min(wl.queries.shape[0], 200)
    rs = nd.RefSet(dev(wl.refs), W)
    qs = dev(wl.queries[:nq])
    sr = nd.Searcher(rs, nq, V=V, helpers=helpers)
    ref = [host(x).copy() for x in sr(qs)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        sr(qs)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sr(qs)
    for rep in range(3):
        say("search graph replay", name, rep)
        sr.idx.fill_(-7)
        sr.dist.fill_(-1.0)
        sr.counts.fill_(-3)
        x = torch.randn(4096, device=DEV)
        (x * x).sum().item()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(sr.idx), ref[0]) and np.array_equal(host(sr.dist), ref[1])
        assert np.array_equal(host(sr.counts)[:, :5], ref[2][:, :5])
    oi, od, oc = oracle.search(wl.refs, wl.queries[:4], W, V, "keogh_enh", sr.R, True)
    assert np.array_equal(ref[0][:4], oi) and np.array_equal(ref[1][:4], od)


@pytest.mark.parametrize("seed", range(6))
def test_search_random_edge_shapes(seed):
    """Seeded random single searches over edge shapes: L from 2, windows from
    0 to unconstrained, one reference, round sizes 1, 7 and the default, both
    engines where they apply, helper workgroups off, default and at the
    maximum; index, distance and defined counts against the oracle."""
    rng = np.random.default_rng(7000 + seed)
    L = int(rng.choice([2, 3, 9, 64, 200, 513, 700]))
    n = int(rng.choice([1, 5, 100, 700]))
    W = int(rng.choice([0, 1, max(1, L // 10), L // 2, L - 1, L + 3]))
    nq = int(rng.choice([1, 3, 8]))
    V = int(rng.choice([1, 3, 5]))
    R = int(rng.choice([0, 1, 7]))
    helpers = int(rng.choice([-1, 0, 7]))
    engines = ["auto", "diagonal"] + (["strip"] if W >= L - 1 and L > 2 else [])
    refs = series(n, L, seed=30000 + seed, kind="sin5")
    qs = series(nq, L, seed=31000 + seed, kind="sin5")
    rs = nd.RefSet(dev(refs), W)
    for engine in engines:
        say("search random", seed, L, n, W, nq, V, R, helpers, engine)
        idx, dist, counts, R_used = nd.search(rs, dev(qs), V=V, R=R, engine=engine, helpers=helpers)
        oi, od, oc = oracle.search(refs, qs, W, V, "keogh_enh", R_used, True)
        gi, gd, gc = host(idx), host(dist), host(counts)
        assert np.array_equal(gi, oi), (engine, gi, oi)
        assert np.array_equal(gd, od) and np.array_equal(gc[:, :5], oc[:, :5])


@pytest.mark.parametrize("seed,helpers", [(1, -1), (2, 1), (3, 0), (4, 7)])
def test_batch_random_edge_shapes(seed, helpers):
    """Seeded random batches of edge shapes through the batched search: series
    of 2 to 300 points, windows from 0 to beyond L (unconstrained), single
    references, sets without queries, several V, with and without helper
    workgroups; every query of every set against the oracle at the batch's R."""
    rng = np.random.default_rng(9000 + seed)
    sets = []
    for d in range(7):
        L = int(rng.choice([2, 3, 5, 17, 64, 130, 300]))
        n = int(rng.choice([1, 2, 63, 257, 400]))
        W = int(rng.choice([0, 1, L // 10, L // 3, L - 1, L + 5]))
        W = min(W, 250)                                # the batch takes up to 252 diagonal pairs
        nq = int(rng.choice([0, 1, 3, 6]))
        refs = series(n, L, seed=10000 + 100 * seed + d, kind=("rw", "sin5")[d % 2])
        qs = series(max(nq, 1), L, seed=20000 + 100 * seed + d, kind="rw")[:nq]
        sets.append(synth.BatchDataset(refs, np.ascontiguousarray(qs.reshape(nq, L)), W, 5))
    V = int(rng.choice([1, 2, 5]))
    say("batch random", seed, helpers, V, [(ds.L, ds.refs.shape[0], ds.W, ds.queries.shape[0]) for ds in sets])
    bsr, pairs, res = run_batch(sets, V=V, helpers=helpers)
    for d, ds in enumerate(sets):
        gi, gd, gc = res[d]
        if ds.queries.shape[0] == 0:
            assert gi.shape == (0,)
            continue
        oi, od, oc = oracle.search(ds.refs, ds.queries, ds.W, V, "keogh_enh", bsr.R[d], True)
        assert np.array_equal(gi, oi), (d, gi, oi)
        assert np.array_equal(gd, od) and np.array_equal(gc[:, :5], oc[:, :5])


def test_batch_full_workload():
    """The full batching workload (64 sets, L 25..1839, 26,583 queries) in the
    benchmarked launch shape: every query against size-independent
    properties, and four queries of every one of the 64 sets (first, last and
    two between) against the oracle at the set's R."""
    sets = synth.batch_workload()
    say("batch full", len(sets), "sets")
    bsr, pairs, res = run_batch(sets)
    for d, ds in enumerate(sets):
        gi, gd, gc = res[d]
        assert np.all(gc[:, 1:5].sum(1) == ds.refs.shape[0])
        assert np.all((gi >= 0) & (gi < ds.refs.shape[0]))
        assert np.array_equal(gd, oracle.dtw(ds.queries, ds.refs[gi], ds.W, zip_=True))
    for d, ds in enumerate(sets):
        nq = ds.queries.shape[0]
        sel = np.unique(np.linspace(0, nq - 1, 4).astype(int))
        say("batch full oracle set", d, ds.refs.shape, ds.W, bsr.R[d], bsr.cpl[d], sel.tolist())
        oi, od, oc = oracle.search(ds.refs, ds.queries[sel], ds.W, 5, "keogh_enh", bsr.R[d], True)
        gi, gd, gc = res[d]
        assert np.array_equal(gi[sel], oi) and np.array_equal(gd[sel], od)
        assert np.array_equal(gc[sel, :5], oc[:, :5])


# ------------------------------------------------------------------ DTW backward
@pytest.mark.parametrize("L,W", [(2, 1), (17, 0), (17, 4), (64, 6), (64, 63), (256, 26), (300, 100), (600, 300)])
def test_dtw_backward_f64_matches_oracle(L, W):
    """FP64 forward with codes: distances bit-exact; the gradient with respect
    to the queries equal to the oracle's up to the order of its sums."""
    A = series(9, L, seed=1300 + L + W)
    B = series(7, L, seed=1400 + L + W)
    w = np.random.default_rng(L + W).standard_normal((9, 7))
    say("backward f64", L, W)
    out, codes = nd.dtw_w_codes(dev(A), dev(B), W, f64=True)
    assert np.array_equal(host(out), oracle.dtw(A, B, W))
    g = host(nd.dtw_w_backward(dev(A), dev(B), W, torch.from_numpy(w).to(DEV), codes, f64=True))
    og, od = oracle.dtw_grad(A, B, W, gout=w)
    assert np.allclose(g, og, rtol=1e-12, atol=1e-12 * np.abs(og).max())


def test_dtw_backward_tie_order_on_integer_series():
    """Exact ties between predecessors (integer-valued series) are broken in
    the oracle's order: (i-1,j-1), then (i-1,j), then (i,j-1)."""
    rng = np.random.default_rng(1500)
    for L, W in ((6, 2), (12, 4), (40, 7)):
        A = rng.integers(0, 3, (30, L)).astype(np.float32)
        B = rng.integers(0, 3, (30, L)).astype(np.float32)
        for f64 in (True, False):
            out, codes = nd.dtw_w_codes(dev(A), dev(B), W, zip_=True, f64=f64)
            g = host(nd.dtw_w_backward(dev(A), dev(B), W, torch.ones(30, device=DEV), codes, zip_=True, f64=f64))
            og, od = oracle.dtw_grad(A, B, W, zip_=True)
            assert np.array_equal(host(out).astype(np.float64), od)   # small integers: exact in FP32 too
            assert np.array_equal(g.astype(np.float64), og)


def test_dtw_backward_f32_against_f64():
    """FP32 codes follow the FP64 path except where two paths cost the same
    up to FP32 rounding; such pairs are rare and their costs are checked."""
    L, W = 256, 26
    A = series(400, L, seed=1600, kind="sin5")
    B = series(400, L, seed=1601, kind="sin5")
    ones = torch.ones(400, device=DEV)
    o32, c32 = nd.dtw_w_codes(dev(A), dev(B), W, zip_=True)
    g32 = host(nd.dtw_w_backward(dev(A), dev(B), W, ones, c32, zip_=True))
    og, od = oracle.dtw_grad(A, B, W, zip_=True)
    assert np.all(np.abs(host(o32) - od) <= 1e-5 * od)
    scale = np.abs(og).max(1, keepdims=True) + 1e-30
    same = np.all(np.abs(g32 - og) <= 1e-4 * scale, axis=1)
    assert same.mean() >= 0.98, same.mean()
    for k in np.nonzero(~same)[0]:
        # the FP32 path is another optimum: the gradient differs, the cost does not
        assert abs(float(host(o32)[k]) - od[k]) <= 4 * oracle.slack(L) * od[k]


def test_dtw_autograd_function():
    L, W = 64, 6
    A = series(5, L, seed=1700)
    B = series(3, L, seed=1701)
    w = np.random.default_rng(1702).standard_normal((5, 3))
    At = dev(A).requires_grad_(True)
    loss = (nd.dtw(At, dev(B), W, f64=True) * torch.from_numpy(w).to(DEV)).sum()
    loss.backward()
    og, _ = oracle.dtw_grad(A, B, W, gout=w)
    assert At.grad.dtype == torch.float32
    assert np.allclose(host(At.grad), og, rtol=1e-6, atol=1e-6 * np.abs(og).max())


def test_dtw_backward_finite_differences_on_gpu():
    """Central differences of the GPU's FP64 DTW_W with a step exact in
    float32 equal the GPU gradient wherever the path does not change."""
    rng = np.random.default_rng(1800)
    L, W = 48, 5
    A = (np.round(rng.standard_normal((4, L)) * 256) / 256).astype(np.float32)
    B = (np.round(rng.standard_normal((4, L)) * 256) / 256).astype(np.float32)
    h = np.float32(2.0 ** -8)
    _, codes = nd.dtw_w_codes(dev(A), dev(B), W, zip_=True, f64=True)
    g = host(nd.dtw_w_backward(dev(A), dev(B), W, torch.ones(4, device=DEV, dtype=torch.float64), codes,
                                zip_=True, f64=True))
    agree = 0
    for i in range(L):
        Ap, Am = A.copy(), A.copy()
        Ap[:, i] += h
        Am[:, i] -= h
        dp = host(nd.dtw_w(dev(Ap), dev(B), W, zip_=True, f64=True))
        dm = host(nd.dtw_w(dev(Am), dev(B), W, zip_=True, f64=True))
        fd = (dp - dm) / (2 * float(h))
        for k in range(4):
            _, p0 = oracle.dtw_path(A[k], B[k], W)
            _, pp = oracle.dtw_path(Ap[k], B[k], W)
            _, pm = oracle.dtw_path(Am[k], B[k], W)
            if np.array_equal(p0, pp) and np.array_equal(p0, pm):
                assert abs(fd[k] - g[k, i]) <= 1e-9 * (1 + abs(g[k, i]))
                agree += 1
    assert agree >= 0.8 * 4 * L


def test_dtw_backward_full_config():
    """256 queries x 256 references, L=256, W=26 (cross) in the benchmarked
    launch shape.  FP32: all distances within 1e-5 of FP64; per pair of the
    sampled queries, the gradient equals the oracle's or the FP32 path is
    another optimum up to FP32 rounding (a near-tie; at most 2 % of pairs).
    FP64: sampled queries' gradients equal the oracle's."""
    L, W = 256, 26
    A = series(256, L, seed=1900, kind="sin5")
    B = series(256, L, seed=1901, kind="sin5")
    w = np.random.default_rng(1902).standard_normal((256, 256))
    say("backward full 256x256")
    out, codes = nd.dtw_w_codes(dev(A), dev(B), W)
    nd.dtw_w_backward(dev(A), dev(B), W, torch.from_numpy(w).to(DEV), codes)
    d64 = oracle.dtw(A, B, W)
    assert np.all(np.abs(host(out) - d64) <= 1e-5 * d64)
    sel = np.arange(0, 256, 37)
    og, _ = oracle.dtw_grad(A[sel], B, W, gout=w[sel])
    out64, codes64 = nd.dtw_w_codes(dev(A), dev(B), W, f64=True)
    assert np.array_equal(host(out64), d64)
    g64 = host(nd.dtw_w_backward(dev(A), dev(B), W, torch.from_numpy(w).to(DEV), codes64, f64=True))
    assert np.allclose(g64[sel], og, rtol=1e-10, atol=1e-10 * np.abs(og).max())
    # per pair, FP32, the sampled queries against every reference
    Az, Bz = np.repeat(A[sel], 256, 0), np.tile(B, (len(sel), 1))
    oz, cz = nd.dtw_w_codes(dev(Az), dev(Bz), W, zip_=True)
    gz = host(nd.dtw_w_backward(dev(Az), dev(Bz), W, torch.ones(len(Az), device=DEV), cz, zip_=True))
    ogz, odz = oracle.dtw_grad(Az, Bz, W, zip_=True)
    same = np.all(np.abs(gz - ogz) <= 1e-4 * (np.abs(ogz).max(1, keepdims=True) + 1e-30), axis=1)
    assert same.mean() >= 0.98, same.mean()
    oz = host(oz)
    assert np.all(np.abs(oz[~same] - odz[~same]) <= 4 * oracle.slack(L) * odz[~same])


def test_dtw_backward_deterministic():
    """The cross backward sums in a fixed order: two runs (and a run with the
    codes recomputed) give bit-identical gradients, FP32 and FP64, and L=1000
    (chunks of fewer references than threads) matches the FP64 oracle."""
    L, W = 256, 26
    A = series(5, L, seed=4100, kind="sin5")
    B = series(300, L, seed=4101, kind="sin5")
    g = np.random.default_rng(9).standard_normal((5, 300))
    for f64 in (False, True):
        say("backward deterministic", f64)
        out, codes = nd.dtw_w_codes(dev(A), dev(B), W, f64=f64)
        gt = torch.from_numpy(g).to(DEV)
        g1 = host(nd.dtw_w_backward(dev(A), dev(B), W, gt, codes, f64=f64))
        g2 = host(nd.dtw_w_backward(dev(A), dev(B), W, gt, codes, f64=f64))
        _, codes2 = nd.dtw_w_codes(dev(A), dev(B), W, f64=f64)
        g3 = host(nd.dtw_w_backward(dev(A), dev(B), W, gt, codes2, f64=f64))
        assert np.array_equal(g1, g2) and np.array_equal(g1, g3)
    L, W = 1000, 100
    A = series(2, L, seed=4102)
    B = series(40, L, seed=4103)
    w = np.random.default_rng(10).standard_normal((2, 40))
    out, codes = nd.dtw_w_codes(dev(A), dev(B), W, f64=True)
    g64 = host(nd.dtw_w_backward(dev(A), dev(B), W, torch.from_numpy(w).to(DEV), codes, f64=True))
    og, _ = oracle.dtw_grad(A, B, W, gout=w)
    assert np.allclose(g64, og, rtol=1e-10, atol=1e-10 * np.abs(og).max())


# ------------------------------------------------------------------ serving
@pytest.mark.parametrize("helpers", [0, [-1, -1, 0, 3, -1, 7]])
def test_serving_results_equal_alone(helpers):
    """Requests served in the mix (continuous batching on several streams)
    give exactly the result of each query searched alone; a sample is also
    checked against the oracle.  With helper workgroups per set, batches
    whose sets all ask for none run without them."""
    from paper_1808_09617_amd import serve
    sets = synth.serving_sets(n_sets=6, n_refs=300, L_range=(48, 256))
    rss = [nd.RefSet(dev(refs), W) for refs, W in sets]
    Ls = [refs.shape[1] for refs, _ in sets]
    reqs = serve.poisson_requests(Ls, rate=4000.0, duration=0.1, seed=11, device=DEV,
                                  make_query=lambda s, L, k: synth.serving_query(s, L, k))
    torch.cuda.synchronize()
    say("serving", len(reqs), "requests")
    server = serve.Server(rss, n_streams=3, max_batch=64, helpers=helpers)
    done, summary = server.run(reqs)
    assert summary["batches"] > 1
    # every batch runs each set at the server's round size and shape (the
    # counts are defined per round size)
    for r in done:
        q = r.query[None]
        i, d, c, R = nd.search(rss[r.set_id], q, V=5, R=server.plan_R[r.set_id], cpl=server.plan_cpl[r.set_id])
        assert r.result[0] == int(host(i)[0]) and r.result[1] == float(host(d)[0])
        assert r.result[2][:5] == host(c)[0, :5].tolist()
    for r in done[::25]:
        refs, W = sets[r.set_id]
        q = host(r.query)[None]
        oi, od, oc = oracle.search(refs, q, W, 5, "keogh_enh", server.plan_R[r.set_id], True)
        assert r.result[0] == oi[0] and r.result[1] == od[0] and r.result[2][:5] == oc[0, :5].tolist()


def test_serving_budget_and_overlap():
    """All requests at once (a saturation run): batches overlap on the
    streams, the workspaces of the batches in flight never exceed the
    device-wide budget (which holds about two batches, so admissions wait for
    memory), and every result equals its query searched alone."""
    from paper_1808_09617_amd import serve
    sets = synth.serving_sets(n_sets=5, n_refs=250, L_range=(40, 200))
    rss = [nd.RefSet(dev(refs), W) for refs, W in sets]
    Ls = [refs.shape[1] for refs, _ in sets]
    reqs = serve.poisson_requests(Ls, rate=float("inf"), duration=240, seed=21, device=DEV,
                                  make_query=lambda s, L, k: synth.serving_query(s, L, 5000 + k))
    torch.cuda.synchronize()
    budget = int(2.5 * 16 * max(serve.batch_bytes([rs], [1]) for rs in rss))
    server = serve.Server(rss, n_streams=4, max_batch=16, budget_bytes=budget)
    done, summary = server.run(reqs)
    say("serving saturation", summary)
    assert summary["max_batches_in_flight"] >= 2
    assert summary["max_workspace_bytes"] <= budget
    assert summary["batches"] >= 240 // 16
    assert server.arena.used == 0 and server.arena.free_blocks == [(0, server.arena.size)]
    for r in done:
        i, d, c, _ = nd.search(rss[r.set_id], r.query[None], V=5, R=server.plan_R[r.set_id],
                               cpl=server.plan_cpl[r.set_id])
        assert r.result[0] == int(host(i)[0]) and r.result[1] == float(host(d)[0])
        assert r.result[2][:5] == host(c)[0, :5].tolist()


def test_serving_full_size():
    """Serving at the configured size: 8 resident sets of 4000 random walks,
    L_s = 64 .. 1024, W = 0.1 L_s, V = 5, a Poisson stream at 2000 requests/s.
    Every request's result equals its query searched alone (same set, R and
    engine shape), and a sample covering every set equals the oracle."""
    from paper_1808_09617_amd import serve
    sets = synth.serving_sets()
    rss = [nd.RefSet(dev(refs), W) for refs, W in sets]
    Ls = [refs.shape[1] for refs, _ in sets]
    reqs = serve.poisson_requests(Ls, rate=2000.0, duration=0.25, seed=12, device=DEV,
                                  make_query=lambda s, L, k: synth.serving_query(s, L, k))
    torch.cuda.synchronize()
    say("serving full", len(reqs), "requests")
    server = serve.Server(rss, n_streams=3)
    done, summary = server.run(reqs)
    say("serving full summary", summary)
    assert summary["batches"] > 1
    for r in done:
        q = r.query[None]
        R, cpl = server.plan_R[r.set_id], server.plan_cpl[r.set_id]
        i, d, c, _ = nd.search(rss[r.set_id], q, V=5, R=R, cpl=cpl)
        assert r.result[0] == int(host(i)[0]) and r.result[1] == float(host(d)[0])
        assert r.result[2][:5] == host(c)[0, :5].tolist()
    checked = set()
    for r in done:
        if r.set_id in checked and r.rid % 20:
            continue
        checked.add(r.set_id)
        refs, W = sets[r.set_id]
        q = host(r.query)[None]
        say("serving full oracle", r.rid, r.set_id, refs.shape)
        oi, od, oc = oracle.search(refs, q, W, 5, "keogh_enh", server.plan_R[r.set_id], True)
        assert r.result[0] == oi[0] and r.result[1] == od[0] and r.result[2][:5] == oc[0, :5].tolist()
    assert checked == set(range(len(sets)))


# ------------------------------------------------------------ comparison bounds
# LB_Kim, LB_Improved, LB_New and the symmetric LB_Enhanced: FP64 sums in
# ascending point order (one lane per sum), so bit-exact against the oracle.
CMP_CASES = [(2, 0), (2, 1), (3, 1), (5, 2), (17, 4), (64, 6), (64, 63), (97, 13), (256, 26), (300, 100),
             (512, 128), (512, 511), (1000, 37), (2048, 205), (2048, 2047)]


@pytest.mark.parametrize("L,W", CMP_CASES)
def test_comparison_bounds_bit_exact(L, W):
    nA, nB = (4, 5) if L >= 1000 else (7, 9)
    A = series(nA, L, seed=3 * L + W)
    B = series(nB, L, seed=3 * L + W + 1, kind="sin5")
    say("compare", L, W)
    dA, dB = dev(A), dev(B)
    U, Lo = nd.envelopes(dB, W)
    assert np.array_equal(host(nd.lb_kim(dA, dB)), oracle.lb_kim(A, B))
    assert np.array_equal(host(nd.lb_new(dA, dB, W)), oracle.lb_new(A, B, W))
    imp = oracle.lb_improved(A, B, W)
    assert np.array_equal(host(nd.lb_improved(dA, dB, U, Lo, W)), imp)
    for V in (1, 5):
        assert np.array_equal(host(nd.lb_enhanced_sym(dA, dB, U, Lo, W, V)), oracle.lb_enhanced_sym(A, B, W, V))
    # second-pass skip: +inf exactly where LB_Keogh(A, B) exceeds the cutoff
    ou, ol = oracle.envelopes(B, W)
    k = oracle.lb_keogh(A, ou, ol)
    cut = np.median(k, axis=1)
    got = host(nd.lb_improved(dA, dB, U, Lo, W, cutoff=torch.from_numpy(cut).to(DEV)))
    want = np.where(k > cut[:, None], np.inf, imp)
    assert np.array_equal(got, want)
    # zip pairing
    Z = B[:nA]
    dZ = dev(Z)
    Uz, Lz = nd.envelopes(dZ, W)
    assert np.array_equal(host(nd.lb_kim(dA, dZ, zip_=True)), oracle.lb_kim(A, Z, zip_=True))
    assert np.array_equal(host(nd.lb_new(dA, dZ, W, zip_=True)), oracle.lb_new(A, Z, W, zip_=True))
    assert np.array_equal(host(nd.lb_improved(dA, dZ, Uz, Lz, W, zip_=True)), oracle.lb_improved(A, Z, W, zip_=True))
    assert np.array_equal(host(nd.lb_enhanced_sym(dA, dZ, Uz, Lz, W, 3, zip_=True)),
                          oracle.lb_enhanced_sym(A, Z, W, 3, zip_=True))


def test_comparison_bounds_special_inputs():
    """Constant series (every point is an extreme: LB_Kim keeps only the
    corners), exact copies (all bounds 0) and extremes at the series' ends."""
    L = 40
    base = series(6, L, seed=4242)
    A = np.concatenate([np.zeros((1, L), np.float32), np.full((1, L), 3.0, np.float32), base])
    B = np.concatenate([np.full((1, L), -2.0, np.float32), base[:1], base])
    B[-1, 0] = B[-1].max() + 1.0                 # maximum at the first point
    B[-2, -1] = B[-2].min() - 1.0                # minimum at the last point
    A = np.ascontiguousarray(A)
    B = np.ascontiguousarray(B)
    for W in (0, 3, 39):
        say("compare special", W)
        dA, dB = dev(A), dev(B)
        U, Lo = nd.envelopes(dB, W)
        assert np.array_equal(host(nd.lb_kim(dA, dB)), oracle.lb_kim(A, B))
        assert np.array_equal(host(nd.lb_new(dA, dB, W)), oracle.lb_new(A, B, W))
        assert np.array_equal(host(nd.lb_improved(dA, dB, U, Lo, W)), oracle.lb_improved(A, B, W))
        assert np.array_equal(host(nd.lb_enhanced_sym(dA, dB, U, Lo, W, 2)), oracle.lb_enhanced_sym(A, B, W, 2))
        same = host(nd.lb_new(dev(base), dev(base), W, zip_=True))
        assert np.all(same == 0.0)


def test_comparison_bounds_tightness_pairs_zip():
    """The benchmarked tightness pairs (sin5, L=256, W=26), sampled."""
    a, b = synth.tightness_pairs(2000)
    say("compare tightness pairs", a.shape)
    da, db = dev(a), dev(b)
    U, Lo = nd.envelopes(db, 26)
    assert np.array_equal(host(nd.lb_kim(da, db, zip_=True)), oracle.lb_kim(a, b, zip_=True))
    assert np.array_equal(host(nd.lb_new(da, db, 26, zip_=True)), oracle.lb_new(a, b, 26, zip_=True))
    assert np.array_equal(host(nd.lb_improved(da, db, U, Lo, 26, zip_=True)), oracle.lb_improved(a, b, 26, zip_=True))
    assert np.array_equal(host(nd.lb_enhanced_sym(da, db, U, Lo, 26, 5, zip_=True)),
                          oracle.lb_enhanced_sym(a, b, 26, 5, zip_=True))


@pytest.mark.parametrize("cascade", ["kim", "improved", "new", "enh_sym"])
def test_search_comparison_cascades(cascade):
    wl = synth.workload("nndtw-small")
    for R in (0, 1, 7):
        check_search(wl.refs, wl.queries, 6, 2, cascade, R)
    sub = synth.workload("nndtw-sin256", n_refs=1000, n_queries=24)
    check_search(sub.refs, sub.queries, 26, 5, cascade, 0, True, 0, brute=False)
    mix = synth.workload("nndtw-mix512", n_refs=600, n_queries=6)
    check_search(mix.refs, mix.queries, 51, 5, cascade, 0, True, 0, brute=False)
