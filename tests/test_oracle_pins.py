"""Pins for the CPU oracle: checks against what the paper and mathematics fix.

None of these re-type the oracle's formulas: they compare it with brute-force
path enumeration, closed forms (Delannoy numbers, the W=0 and W>=L-1 special
cases), the theorems of the paper (Theorems 1 and 2, Equation 6), library
routines (numpy sliding windows) and a hand-derived worked example.
"""
import itertools
import math
import os

import numpy as np
import pytest

import synth
from oracle import paths

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _pairs(n, L, seed, kind="rw"):
    x = synth.random_series(2 * n, L, seed, kind)
    return x[:n], x[n:]


# ---------------------------------------------------------------- paths / DTW
def test_path_counts_delannoy():
    rows = [l.split() for l in open(os.path.join(GOLD, "delannoy.txt")) if l.strip() and l[0] != "#"]
    for L, cnt in rows:
        assert paths.count_paths(int(L)) == int(cnt)


def test_windowed_path_counts_small():
    # W = 0 leaves only the diagonal; a window never adds paths.
    for L in range(1, 8):
        assert paths.count_paths(L, 0) == 1
        counts = [paths.count_paths(L, w) for w in range(L)]
        assert counts == sorted(counts)
        assert counts[-1] == paths.count_paths(L)


@pytest.mark.parametrize("L", [2, 3, 4, 5, 6, 7])
def test_dtw_equals_min_over_enumerated_paths(orc, L):
    A, B = _pairs(3, L, seed=L)
    for a, b in zip(A, B):
        for W in range(L):
            want = paths.dtw_brute(a, b, W)
            got = orc.dtw(a, b, W)[0, 0]
            # The recurrence takes the min of left-to-right path sums; with
            # monotone rounding that is bit-identical to the brute force.
            assert got == want, (L, W, got, want)


def test_dtw_equals_min_over_enumerated_paths_L8(orc):
    a, b = _pairs(1, 8, seed=88, kind="normal")
    for W in (1, 3, 7):
        assert orc.dtw(a[0], b[0], W)[0, 0] == paths.dtw_brute(a[0], b[0], W)


def test_worked_example(orc):
    fx = {}
    for line in open(os.path.join(GOLD, "worked_example.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        parts = line.split()
        key = " ".join(p for p in parts if not _isnum(p))
        fx[key] = [float(p) for p in parts if _isnum(p)]
    a = np.array(fx["A"], np.float32)
    b = np.array(fx["B"], np.float32)
    assert orc.dtw(a, b, 10)[0, 0] == fx["dtw W=inf"][0]
    assert orc.dtw(a, b, 1)[0, 0] == fx["dtw W=1"][0]
    assert orc.dtw(a, b, 0)[0, 0] == fx["dtw W=0"][0]
    U, Lo = orc.envelopes(b, 1)
    assert U[0].tolist() == fx["U W=1"]
    assert Lo[0].tolist() == fx["Lo W=1"]
    assert orc.lb_keogh(a, U, Lo)[0, 0] == fx["lb_keogh W=1"][0]
    assert orc.lb_enhanced(a, b, U, Lo, 1, 1)[0, 0] == fx["lb_enhanced W=1 V=1"][0]
    assert orc.lb_enhanced(a, b, U, Lo, 1, 2)[0, 0] == fx["lb_enhanced W=1 V=2"][0]
    U0, L0 = orc.envelopes(b, 0)
    assert orc.lb_keogh(a, U0, L0)[0, 0] == fx["lb_keogh W=0"][0]
    assert orc.lb_enhanced(a, b, U0, L0, 0, 1)[0, 0] == fx["lb_enhanced W=0 V=1"][0]


def _isnum(s):
    try:
        float(s)
        return True
    except ValueError:
        return False


def test_dtw_special_cases(orc):
    A, B = _pairs(6, 37, seed=5)
    ed = orc.ed2(A, B, zip_=True)
    d0 = orc.dtw(A, B, 0, zip_=True)
    assert np.array_equal(d0, ed)                                   # DTW_0 = squared ED
    assert np.array_equal(ed, ((A.astype(np.float64) - B) ** 2).sum(1)) or np.allclose(
        ed, ((A.astype(np.float64) - B) ** 2).sum(1), rtol=1e-14)
    for W in (0, 2, 9, 36, 50):
        dab = orc.dtw(A, B, W, zip_=True)
        dba = orc.dtw(B, A, W, zip_=True)
        assert np.array_equal(dab, dba)                             # symmetric
        assert np.all(orc.dtw(A, A, W, zip_=True) == 0.0)           # DTW(A,A) = 0
        # exact scaling by powers of two
        assert np.array_equal(orc.dtw(2 * A, 2 * B, W, zip_=True), 4 * dab)
    full = orc.dtw(A, B, 36, zip_=True)
    assert np.array_equal(full, orc.dtw(A, B, 37, zip_=True))        # W >= L-1 unconstrained
    assert np.array_equal(full, orc.dtw(A, B, 10 ** 6, zip_=True))
    prev = None
    for W in range(0, 37):
        d = orc.dtw(A, B, W, zip_=True)
        if prev is not None:
            assert np.all(d <= prev)                                # nonincreasing in W
        prev = d


def test_dtw_abandon(orc):
    A, B = _pairs(20, 48, seed=6)
    full = orc.dtw(A, B, 5, zip_=True)
    for f in (0.3, 0.9, 1.0, 1.1):
        cut = full * f
        got = orc.dtw(A, B, 5, cutoff=cut, zip_=True)
        for g, d, c in zip(got, full, cut):
            if math.isinf(g):
                assert d > c                        # abandoned only when above the cutoff
            else:
                assert g == d


# ---------------------------------------------------------------- envelopes
def _np_envelopes(b, W):
    L = b.shape[-1]
    w = min(W, L - 1)
    hi = np.pad(b, (w, w), constant_values=-np.inf)
    lo = np.pad(b, (w, w), constant_values=np.inf)
    win_hi = np.lib.stride_tricks.sliding_window_view(hi, 2 * w + 1)
    win_lo = np.lib.stride_tricks.sliding_window_view(lo, 2 * w + 1)
    return win_hi.max(-1), win_lo.min(-1)


@pytest.mark.parametrize("L", [2, 3, 17, 64, 257])
def test_envelopes_vs_sliding_window(orc, L):
    B = synth.random_series(5, L, seed=L)
    for W in sorted({0, 1, 2, 5, L // 3, L - 2, L - 1, L, 3 * L}):
        if W < 0:
            continue
        U, Lo = orc.envelopes(B, W)
        for s in range(B.shape[0]):
            u, l = _np_envelopes(B[s], W)
            assert np.array_equal(U[s], u.astype(np.float32))
            assert np.array_equal(Lo[s], l.astype(np.float32))
        assert np.all(Lo <= B) and np.all(B <= U)
    U0, L0 = orc.envelopes(B, 0)
    assert np.array_equal(U0, B) and np.array_equal(L0, B)
    Uf, Lf = orc.envelopes(B, L - 1)
    assert np.array_equal(Uf, np.repeat(B.max(1, keepdims=True), L, 1))
    assert np.array_equal(Lf, np.repeat(B.min(1, keepdims=True), L, 1))


# ---------------------------------------------------------------- LB_Keogh
def test_lb_keogh_properties(orc):
    A, B = _pairs(40, 64, seed=11)
    ed = orc.ed2(A, B, zip_=True)
    prev = None
    for W in (0, 1, 3, 6, 12, 32, 63):
        U, Lo = orc.envelopes(B, W)
        lbk = orc.lb_keogh(A, U, Lo, zip_=True)
        d = orc.dtw(A, B, W, zip_=True)
        assert np.all(lbk <= d)                                     # lower bound
        assert np.all(lbk >= 0)
        assert np.all(orc.lb_keogh(B, U, Lo, zip_=True) == 0.0)      # B inside its own envelope
        if W == 0:
            assert np.array_equal(lbk, ed)                          # W=0: squared ED
        if prev is not None:
            assert np.all(lbk <= prev)                              # nonincreasing in W
        prev = lbk


# ---------------------------------------------------------------- band sets
@pytest.mark.parametrize("L", [2, 3, 4, 5, 6])
def test_bands_are_crossed_by_every_path(orc, L):
    """Theorem 1 (and its mirror for Equation 6): every warping path inside the
    window contains at least one link of every left band and every right band."""
    for W in range(L):
        P = [set(p) for p in paths.enumerate_paths(L, W)]
        for i in range(L):
            left = set(orc.band_cells(L, W, 0, i))
            right = set(orc.band_cells(L, W, 1, i))
            assert len(left) == 2 * min(i, W) + 1
            assert len(right) == 2 * min(L - 1 - i, W) + 1
            for p in P:
                assert p & left and p & right


@pytest.mark.parametrize("L", [2, 3, 4, 7, 10, 11])
def test_band_partition_is_disjoint(orc, L):
    """Proof of Theorem 2: L_1..L_V, V_{V+1}..V_{L-V} and R_{L-V+1}..R_L are
    mutually exclusive, and their union covers every link a path may use in
    the first V columns, the middle columns and the last V columns."""
    for W in range(L):
        for V in range(1, L // 2 + 1):
            sets = [set(orc.band_cells(L, W, 0, i)) for i in range(V)]
            sets += [set(orc.band_cells(L, W, 2, i)) for i in range(V, L - V)]
            sets += [set(orc.band_cells(L, W, 1, i)) for i in range(L - V, L)]
            for s, t in itertools.combinations(sets, 2):
                assert not (s & t)
            for i in range(L):
                vert = set(orc.band_cells(L, W, 2, i))
                assert len(vert) == min(L - 1, i + W) - max(0, i - W) + 1


def test_band_sums_are_lower_bounds(orc):
    A, B = _pairs(30, 40, seed=21)
    for W in (0, 1, 4, 10, 39):
        d = orc.dtw(A, B, W, zip_=True)
        for a, b, dd in zip(A, B, d):
            assert orc.left_bands_sum(a, b, W) <= dd * (1 + 1e-12)       # Theorem 1
            assert orc.right_bands_sum(a, b, W) <= dd * (1 + 1e-12)      # Equation 6


# ---------------------------------------------------------------- LB_Enhanced
@pytest.mark.parametrize("L", [2, 3, 8, 33, 64])
def test_lb_enhanced_properties(orc, L):
    A, B = _pairs(25, L, seed=100 + L)
    ed = orc.ed2(A, B, zip_=True)
    for W in sorted({0, 1, 2, 5, L // 2, L - 1}):
        U, Lo = orc.envelopes(B, W)
        d = orc.dtw(A, B, W, zip_=True)
        lbk = orc.lb_keogh(A, U, Lo, zip_=True)
        for V in sorted({1, 2, 3, 5, L // 2, L // 2 + 3}):
            eq7 = orc.lb_enhanced(A, B, U, Lo, W, V, zip_=True, variant="eq7")
            alg = orc.lb_enhanced(A, B, U, Lo, W, V, zip_=True, variant="alg1")
            bands = orc.lb_enhanced(A, B, U, Lo, W, V, zip_=True, variant="bands")
            np.testing.assert_allclose(alg, eq7, rtol=1e-12, atol=0)    # Eq 7 = Algorithm 1
            assert np.all(alg <= d * (1 + 1e-12))                       # Theorem 2
            assert np.all(bands <= alg)
            if W == 0:
                np.testing.assert_allclose(alg, ed, rtol=1e-12)         # W=0: squared ED
            if V == 1:
                assert np.all(alg >= lbk * (1 - 1e-12))                 # uniformly tighter than Keogh
            if V > L // 2:
                clamp = orc.lb_enhanced(A, B, U, Lo, W, L // 2, zip_=True)
                assert np.array_equal(alg, clamp)                      # V clamped to floor(L/2)


def test_lb_enhanced_cutoff(orc):
    A, B = _pairs(30, 50, seed=31)
    W, V = 5, 4
    U, Lo = orc.envelopes(B, W)
    full = orc.lb_enhanced(A, B, U, Lo, W, V, zip_=True)
    bands = orc.lb_enhanced(A, B, U, Lo, W, V, zip_=True, variant="bands")
    cut = np.median(bands)
    got = [orc.lb_enhanced(a, b, u, l, W, V, cutoff=cut)[0, 0] for a, b, u, l in zip(A, B, U, Lo)]
    for g, f, bd in zip(got, full, bands):
        assert (math.isinf(g) and bd > cut) or (g == f and bd <= cut)


def test_lb_enhanced_asymmetric(orc):
    A, B = _pairs(20, 32, seed=41)
    W, V = 4, 3
    Ub, Lb = orc.envelopes(B, W)
    Ua, La = orc.envelopes(A, W)
    ab = orc.lb_enhanced(A, B, Ub, Lb, W, V, zip_=True)
    ba = orc.lb_enhanced(B, A, Ua, La, W, V, zip_=True)
    assert np.any(ab != ba)


def test_lb_le_dtw_on_generated_workload_pairs(orc):
    """LB <= DTW_W on every pair of a generated workload (truncated sizes)."""
    wl = synth.workload("nndtw-small")
    W = wl.windows[0]
    U, Lo = orc.envelopes(wl.refs, W)
    d = orc.dtw(wl.queries, wl.refs, W)
    lbk = orc.lb_keogh(wl.queries, U, Lo)
    assert np.all(lbk <= d)
    for V in (1, 2, 5, 32):
        lbe = orc.lb_enhanced(wl.queries, wl.refs, U, Lo, W, V)
        assert np.all(lbe <= d * (1 + 1e-12))


# ---------------------------------------------------------------- search
def _closed_form_counts(orc, refs, queries, W, V, cascade, R, init_ub):
    """Stage counts from full matrices: the best-so-far after each round is the
    lexicographic min of (DTW, index) over the candidates visited so far."""
    L = refs.shape[1]
    eps = orc.slack(L)
    U, Lo = orc.envelopes(refs, W)
    ed = orc.ed2(queries, refs)
    d = orc.dtw(queries, refs, W)
    lbk = orc.lb_keogh(queries, U, Lo)
    lbb = orc.lb_enhanced(queries, refs, U, Lo, W, V, variant="bands")
    lbe = orc.lb_enhanced(queries, refs, U, Lo, W, V)
    out = []
    for q in range(queries.shape[0]):
        order = sorted(range(refs.shape[0]), key=lambda k: (ed[q, k], k))
        ub = ed[q, order[0]] if init_ub else math.inf
        best = (math.inf, -1)
        c = [refs.shape[0], 0, 0, 0, 0]
        for r0 in range(0, len(order), R):
            thr = min(best[0], ub) * (1.0 + eps)
            rnd = order[r0:r0 + R]
            for k in rnd:
                if cascade in ("keogh", "keogh_enh") and lbk[q, k] > thr:
                    c[1] += 1
                elif cascade in ("keogh_enh", "enh") and lbb[q, k] > thr:
                    c[2] += 1
                elif cascade in ("keogh_enh", "enh") and lbe[q, k] > thr:
                    c[3] += 1
                else:
                    c[4] += 1
            for k in rnd:
                if d[q, k] <= thr and (best[1] < 0 or (d[q, k], k) < best):
                    best = (d[q, k], k)
        out.append((best, c))
    return out


@pytest.mark.parametrize("cascade", ["none", "keogh", "keogh_enh", "enh"])
@pytest.mark.parametrize("R", [1, 3, 16])
def test_search_equals_brute_force(orc, cascade, R):
    refs = synth.random_series(60, 32, seed=7, kind="sin5")
    queries = synth.random_series(8, 32, seed=8, kind="sin5")
    for W in (0, 3, 31):
        bi, bd = orc.brute_nn(refs, queries, W)
        for V in (1, 3):
            for init_ub in (False, True):
                si, sd, cnt = orc.search(refs, queries, W, V, cascade, R, init_ub)
                assert np.array_equal(si, bi) and np.array_equal(sd, bd)
                assert np.all(cnt[:, 1:5].sum(1) == cnt[:, 0])              # stages sum to N
                cf = _closed_form_counts(orc, refs, queries, W, V, cascade, R, init_ub)
                for q, (best, c) in enumerate(cf):
                    assert best == (bd[q], bi[q])
                    assert cnt[q, :5].tolist() == c, (q, cnt[q], c)


def test_search_r1_independent_of_initial_bound(orc):
    refs = synth.random_series(80, 48, seed=9)
    queries = synth.random_series(10, 48, seed=10)
    a = orc.search(refs, queries, 5, 2, "keogh_enh", 1, False)
    b = orc.search(refs, queries, 5, 2, "keogh_enh", 1, True)
    for x, y in zip(a, b):
        assert np.array_equal(x[..., :5] if x.ndim == 2 else x, y[..., :5] if y.ndim == 2 else y)


def test_search_dominance_enh1_over_keogh(orc):
    wl = synth.workload("nndtw-small")
    W = wl.windows[0]
    for R in (1, 8):
        _, _, ck = orc.search(wl.refs, wl.queries, W, 1, "keogh", R)
        _, _, ce = orc.search(wl.refs, wl.queries, W, 1, "enh", R)
        assert np.all(ce[:, 4] <= ck[:, 4])


def test_search_ties_go_to_lowest_index(orc):
    base = synth.random_series(30, 24, seed=12)
    refs = np.concatenate([base, base[[3, 7, 3]]], 0)       # duplicates at 30, 31, 32
    refs = np.ascontiguousarray(refs[::-1])                 # now duplicates at low indices too
    queries = np.ascontiguousarray(base[[3, 7, 11]])        # exact copies: distance 0
    for R in (1, 4, 33):
        idx, dist, _ = orc.search(refs, queries, 4, 2, "keogh_enh", R)
        bi, bd = orc.brute_nn(refs, queries, 4)
        assert np.array_equal(idx, bi) and np.all(dist == 0.0)
        for q, i in zip(queries, idx):
            same = [k for k in range(refs.shape[0]) if np.array_equal(refs[k], q)]
            assert i == min(same)
    # all candidates identical
    refs = np.repeat(base[:1], 9, 0)
    idx, dist, cnt = orc.search(refs, base[1:3], 3, 1, "keogh_enh", 2)
    assert np.all(idx == 0)


def test_search_equal_ed_visited_by_index(orc):
    """Two references at the same squared ED (exact small integers) but with
    different DTW: the lower index is visited first (ascending (ED^2, index)),
    which decides whether the other one is pruned."""
    A = np.arange(8, dtype=np.float32)
    B1 = A.copy(); B1[0] = 3.0                  # ED^2 = 9; the forced (1,1) link costs 9
    B2 = A.copy(); B2[3] = 6.0                  # ED^2 = 9; warping absorbs most of it
    d1, d2 = orc.dtw(A, B1, 1)[0, 0], orc.dtw(A, B2, 1)[0, 0]
    assert d1 == 9.0 and d2 < d1
    assert orc.ed2(A, B1)[0, 0] == orc.ed2(A, B2)[0, 0] == 9.0
    U, Lo = orc.envelopes(B1, 1)
    assert orc.lb_enhanced(A, B1, U, Lo, 1, 1, variant="bands")[0, 0] > d2 * (1 + orc.slack(8))
    refs = np.stack([B2, B1])                   # B2 at index 0: visited first, B1 then pruned
    idx, dist, cnt = orc.search(refs, A, 1, 1, "enh", 1)
    assert idx[0] == 0 and dist[0] == d2
    assert cnt[0, 2] == 1 and cnt[0, 4] == 1
    refs = np.stack([B1, B2])                   # B1 first: both need DTW
    idx, dist, cnt = orc.search(refs, A, 1, 1, "enh", 1)
    assert idx[0] == 1 and cnt[0, 4] == 2


# ------------------------------------------------------------------ gradient
# DTW_W (Equation 1) is the minimum over warping paths of the path cost; the
# oracle's gradient with respect to the query follows the minimising path
# recovered by walking back from (L-1, L-1), ties broken in the order
# (i-1,j-1), (i-1,j), (i,j-1).  Pinned against path enumeration, closed forms
# and exact finite differences.

def _moves_from_end(path):
    """The walk back from (L-1,L-1) as a move sequence: 0 diagonal, 1 (i-1,j), 2 (i,j-1)."""
    out = []
    for (i0, j0), (i1, j1) in zip(path[::-1][1:], path[::-1][:-1]):
        out.append(0 if (i1 - i0, j1 - j0) == (1, 1) else (1 if (i1 - i0, j1 - j0) == (1, 0) else 2))
    return tuple(out)


def _brute_path(a, b, W):
    """Among all minimum-cost paths, the one whose walk back takes the first
    predecessor of the order diagonal, (i-1,j), (i,j-1) at every step, i.e.
    the lexicographically smallest move sequence from the end."""
    ps = paths.enumerate_paths(len(a), W)
    costs = [paths.path_cost(a, b, p) for p in ps]
    best = min(costs)
    opt = [p for p, c in zip(ps, costs) if c == best]
    return best, min(opt, key=_moves_from_end), sorted(costs)


@pytest.mark.parametrize("L", [2, 3, 5, 7])
def test_grad_path_is_the_unique_argmin(orc, L):
    rng = np.random.default_rng(700 + L)
    for W in range(0, L):
        for _ in range(4):
            a = rng.standard_normal(L).astype(np.float32)
            b = rng.standard_normal(L).astype(np.float32)
            best, p, costs = _brute_path(a, b, W)
            d, path = orc.dtw_path(a, b, W)
            assert d == best
            if len(costs) > 1:
                assert costs[1] > costs[0]          # continuous data: unique argmin
            assert [tuple(x) for x in path] == list(p)


@pytest.mark.parametrize("L", [3, 4, 5, 6])
def test_grad_path_tie_order_on_integer_series(orc, L):
    """Integer-valued series create exact ties between optimal paths; the
    path must be the one the fixed predecessor order selects."""
    rng = np.random.default_rng(800 + L)
    nties = 0
    for W in range(0, L):
        for _ in range(12):
            a = rng.integers(0, 3, L).astype(np.float32)
            b = rng.integers(0, 3, L).astype(np.float32)
            best, p, costs = _brute_path(a, b, W)
            nties += len(costs) > 1 and costs[1] == costs[0]
            d, path = orc.dtw_path(a, b, W)
            assert d == best and [tuple(x) for x in path] == list(p)
    assert nties > 0


def test_grad_w0_and_identical_series(orc):
    A = synth.random_series(6, 40, seed=81)
    B = synth.random_series(6, 40, seed=82)
    g, d = orc.dtw_grad(A, B, 0, zip_=True)
    assert np.array_equal(g, 2.0 * (A.astype(np.float64) - B.astype(np.float64)))
    assert np.array_equal(d, orc.ed2(A, B, zip_=True))
    g, d = orc.dtw_grad(A, A, 7, zip_=True)
    assert np.all(g == 0.0) and np.all(d == 0.0)


def test_grad_path_cost_is_dtw_and_path_is_valid(orc):
    A = synth.random_series(4, 64, seed=83)
    B = synth.random_series(4, 64, seed=84)
    for W in (3, 9, 63):
        for a, b in zip(A, B):
            d, path = orc.dtw_path(a, b, W)
            assert d == orc.dtw(a, b, W)[0, 0]
            assert d == paths.path_cost(a, b, [tuple(x) for x in path])
            assert tuple(path[0]) == (0, 0) and tuple(path[-1]) == (63, 63)
            steps = np.diff(path, axis=0)
            assert all(tuple(s) in ((1, 0), (0, 1), (1, 1)) for s in steps)
            assert np.all(np.abs(path[:, 0] - path[:, 1]) <= W)


def test_grad_exact_finite_differences(orc):
    """Along a fixed path the cost is a quadratic in each a_i, so the central
    difference with a step h that is exact in float32 equals the derivative;
    checked wherever perturbing a_i by +-h leaves the path unchanged."""
    rng = np.random.default_rng(85)
    h = 2.0 ** -8
    checked = 0
    for L, W in ((16, 3), (24, 6), (32, 31)):
        a = (np.round(rng.standard_normal(L) * 256) / 256).astype(np.float32)
        b = (np.round(rng.standard_normal(L) * 256) / 256).astype(np.float32)
        g, _ = orc.dtw_grad(a, b, W)
        _, p0 = orc.dtw_path(a, b, W)
        for i in range(L):
            ap, am = a.copy(), a.copy()
            ap[i] += np.float32(h)
            am[i] -= np.float32(h)
            dp, pp = orc.dtw_path(ap, b, W)
            dm, pm = orc.dtw_path(am, b, W)
            if np.array_equal(pp, p0) and np.array_equal(pm, p0):
                assert abs((dp - dm) / (2 * h) - g[0, i]) <= 1e-9 * (1 + abs(g[0, i]))
                checked += 1
    assert checked >= 40


def test_grad_is_linear_in_the_output_weights(orc):
    A = synth.random_series(3, 48, seed=86)
    B = synth.random_series(5, 48, seed=87)
    w = np.random.default_rng(88).standard_normal((3, 5))
    g, d = orc.dtw_grad(A, B, 5, gout=w)
    assert np.array_equal(d, orc.dtw(A, B, 5))
    for x in range(3):
        want = np.zeros(48)
        for y in range(5):
            gy, _ = orc.dtw_grad(A[x], B[y], 5)
            want += w[x, y] * gy[0]
        assert np.allclose(g[x], want, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------- comparison bounds
# LB_Kim (sum form), LB_Improved, LB_New (Section 2.2 and the experiments of
# Section 4) and the symmetric LB_Enhanced of the conclusion.  Pinned against
# a hand-derived fixture, path enumeration, dominance relations that follow
# from the definitions, the W = 0 and unconstrained special cases, and the
# brute-force nearest neighbour.

def _fixture(name):
    fx = {}
    for line in open(os.path.join(GOLD, name)):
        if not line.strip() or line.startswith("#"):
            continue
        parts = line.split()
        key = " ".join(p for p in parts if not _isnum(p))
        fx[key] = [float(p) for p in parts if _isnum(p)]
    return fx


def test_comparison_bounds_worked_example(orc):
    fx = _fixture("comparison_bounds.txt")
    s = {k: np.array(fx[k], np.float32) for k in "ABCDEF"}
    for x, y in ("AB", "CD", "EF"):
        assert orc.dtw(s[x], s[y], 1)[0, 0] == fx["dtw " + x + y][0]
        assert orc.lb_kim(s[x], s[y])[0, 0] == fx["kim " + x + y][0]
    for x, y in ("AB", "CD"):
        assert orc.lb_new(s[x], s[y], 1)[0, 0] == fx["new " + x + y][0]
        assert orc.lb_improved(s[x], s[y], 1)[0, 0] == fx["improved " + x + y][0]
        assert orc.lb_enhanced_sym(s[x], s[y], 1, 1)[0, 0] == fx["sym " + x + y][0]
        for p, q in ((x, y), (y, x)):
            U, Lo = orc.envelopes(s[q], 1)
            assert orc.lb_enhanced(s[p], s[q], U, Lo, 1, 1)[0, 0] == fx["enh1 " + p + q][0]


@pytest.mark.parametrize("L", [2, 3, 4, 5, 6, 7])
def test_comparison_bounds_below_every_path(orc, L):
    """Each bound is at most the cheapest enumerated warping path, at every W,
    on random series and on series shifted far apart (where counting an
    extreme feature twice would exceed the path cost)."""
    A, B = _pairs(4, L, seed=500 + L, kind="normal")
    A = np.concatenate([A, A[:2] + 10.0]).astype(np.float32)
    B = np.concatenate([B, B[:2] * 0.25]).astype(np.float32)
    for a, b in zip(A, B):
        for W in range(L):
            best = paths.dtw_brute(a, b, W)
            tol = best * 1e-12
            assert orc.lb_kim(a, b)[0, 0] <= best + tol
            assert orc.lb_new(a, b, W)[0, 0] <= best + tol
            assert orc.lb_improved(a, b, W)[0, 0] <= best + tol
            for V in (1, 2, 3):
                assert orc.lb_enhanced_sym(a, b, W, V)[0, 0] <= best + tol


def test_kim_without_repetitions_is_needed(orc):
    """Constant series 10 and 0: every point is both minimum and maximum, so
    both extreme features coincide with the corners.  The bound must equal
    the two corner costs (= DTW = 200); counting the extremes would give 400."""
    a = np.full(2, 10.0, np.float32)
    b = np.zeros(2, np.float32)
    assert orc.dtw(a, b, 1)[0, 0] == 200.0
    assert orc.lb_kim(a, b)[0, 0] == 200.0


def test_comparison_bounds_properties(orc):
    A, B = _pairs(12, 40, seed=611, kind="sin5")
    ed = orc.ed2(A, B, zip_=True)
    kim_ab, kim_ba = orc.lb_kim(A, B, zip_=True), orc.lb_kim(B, A, zip_=True)
    assert np.array_equal(kim_ab, kim_ba)                      # the definition is symmetric
    for W in (0, 1, 4, 13, 39, 60):
        d = orc.dtw(A, B, W, zip_=True)
        U, Lo = orc.envelopes(B, W)
        k = orc.lb_keogh(A, U, Lo, zip_=True)
        imp = orc.lb_improved(A, B, W, zip_=True)
        new = orc.lb_new(A, B, W, zip_=True)
        assert np.all(imp >= k)                                # LB_Keogh plus a non-negative pass
        assert np.all(new >= k * (1 - 1e-12))                  # every term dominates the Keogh term
        assert np.all(imp <= d * (1 + 1e-12)) and np.all(new <= d * (1 + 1e-12))
        Ua, La = orc.envelopes(A, W)
        for V in (1, 3, 20):
            ab = orc.lb_enhanced(A, B, U, Lo, W, V, zip_=True)
            ba = orc.lb_enhanced(B, A, Ua, La, W, V, zip_=True)
            sym = orc.lb_enhanced_sym(A, B, W, V, zip_=True)
            assert np.all(sym >= ab) and np.all(sym >= ba) and np.all((sym == ab) | (sym == ba))
            assert np.all(sym <= d * (1 + 1e-12))
        if W == 0:
            assert np.array_equal(imp, ed)                     # A' = B, second pass 0
            assert np.allclose(new, ed, rtol=1e-12, atol=0)
        if W >= 39:
            # unconstrained: nearest value of the whole of B (sorted search)
            for a, b, v in zip(A, B, new):
                sb = np.sort(b.astype(np.float64))
                want = (float(a[0]) - float(b[0])) ** 2 + (float(a[-1]) - float(b[-1])) ** 2
                for x in a[1:-1].astype(np.float64):
                    t = np.searchsorted(sb, x)
                    want += min((x - sb[max(t - 1, 0)]) ** 2, (x - sb[min(t, sb.size - 1)]) ** 2)
                assert abs(v - want) <= 1e-12 * want


def test_improved_cutoff_skips_the_second_pass(orc):
    A, B = _pairs(10, 33, seed=612)
    W = 3
    U, Lo = orc.envelopes(B, W)
    k = orc.lb_keogh(A, U, Lo, zip_=True)
    full = orc.lb_improved(A, B, W, zip_=True)
    cut = np.median(k)
    got = np.array([orc.lb_improved(A[i], B[i], W, cutoff=cut)[0, 0] for i in range(10)])
    assert np.all(np.isinf(got[k > cut]))
    assert np.array_equal(got[k <= cut], full[k <= cut])


def _compare_matrices(orc, refs, queries, W, V):
    U, Lo = orc.envelopes(refs, W)
    Ua, La = orc.envelopes(queries, W)
    return {
        "lbk": orc.lb_keogh(queries, U, Lo),
        "lbb": orc.lb_enhanced(queries, refs, U, Lo, W, V, variant="bands"),
        "kim": orc.lb_kim(queries, refs),
        "imp": orc.lb_improved(queries, refs, W),
        "new": orc.lb_new(queries, refs, W),
        "sym": np.maximum(orc.lb_enhanced(queries, refs, U, Lo, W, V),
                          np.stack([orc.lb_enhanced(refs, queries[q], Ua[q], La[q], W, V)[:, 0]
                                    for q in range(queries.shape[0])])),
    }


@pytest.mark.parametrize("cascade", ["kim", "improved", "new", "enh_sym"])
@pytest.mark.parametrize("R", [1, 5])
def test_search_comparison_cascades(orc, cascade, R):
    """The search with each comparison bound returns the brute-force nearest
    neighbour, and its stage counts equal the closed form recomputed from full
    bound matrices (bsf after each round = min over the visited DTWs)."""
    refs = synth.random_series(50, 28, seed=71, kind="sin5")
    queries = synth.random_series(6, 28, seed=72, kind="sin5")
    for W in (0, 3, 27):
        bi, bd = orc.brute_nn(refs, queries, W)
        V = 3
        m = _compare_matrices(orc, refs, queries, W, V)
        stages = {"kim": [("kim", 1)], "improved": [("lbk", 1), ("imp", 3)], "new": [("new", 1)],
                  "enh_sym": [("lbb", 2), ("sym", 3)]}[cascade]
        ed = orc.ed2(queries, refs)
        d = orc.dtw(queries, refs, W)
        eps = orc.slack(refs.shape[1])
        si, sd, cnt = orc.search(refs, queries, W, V, cascade, R, True)
        assert np.array_equal(si, bi) and np.array_equal(sd, bd)
        for q in range(queries.shape[0]):
            order = sorted(range(refs.shape[0]), key=lambda k: (ed[q, k], k))
            ub, best = ed[q, order[0]], (math.inf, -1)
            c = [refs.shape[0], 0, 0, 0, 0]
            for r0 in range(0, len(order), R):
                thr = min(best[0], ub) * (1.0 + eps)
                rnd = order[r0:r0 + R]
                for k in rnd:
                    hit = next((slot for name, slot in stages if m[name][q, k] > thr), 4)
                    c[hit] += 1
                for k in rnd:
                    if d[q, k] <= thr and (best[1] < 0 or (d[q, k], k) < best):
                        best = (d[q, k], k)
            assert cnt[q, :5].tolist() == c, (cascade, W, q, cnt[q], c)


def test_search_comparison_dominance(orc):
    """Pointwise dominance of the bounds gives fewer DTW calls at any R:
    LB_Improved and LB_New over LB_Keogh, the symmetric bound over LB_Enhanced."""
    wl = synth.workload("nndtw-small")
    W = wl.windows[0]
    for R in (1, 8):
        started = {c: orc.search(wl.refs, wl.queries, W, 2, c, R)[2][:, 4]
                   for c in ("keogh", "improved", "new", "enh", "enh_sym")}
        assert np.all(started["improved"] <= started["keogh"])
        assert np.all(started["new"] <= started["keogh"])
        assert np.all(started["enh_sym"] <= started["enh"])
