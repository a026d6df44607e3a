"""The oracle's pins have teeth: plant plausible mistakes in copies of the
oracle source (on the CPU), rebuild, and check that the pin suite fails for
every one of them.  Each mutation is (description, original text, mistake)."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "nndtw_oracle.c")

MUTATIONS = [
    ("keogh: lower branch measured to U", "if (a < l) return delta(a, l);", "if (a < l) return delta(a, u);"),
    ("keogh: upper branch measured to Lo", "if (a > u) return delta(a, u);", "if (a > u) return delta(a, l);"),
    ("envelope window one short", "hi = imin(L - 1, i + w);\n            float u", "hi = imin(L - 1, i + w - (w > 0));\n            float u"),
    ("dtw: diagonal predecessor dropped", "double m = dmin(dmin(prev[j - 1], cur[j - 1]), prev[j]);", "double m = dmin(cur[j - 1], prev[j]);"),
    ("dtw: band one too wide", "int lo = imax(1, i - w), hi = imin(L, i + w);", "int lo = imax(1, i - w - 1), hi = imin(L, i + w);"),
    ("band set: transposed link in the right band", "rows[n] = q; cols[n] = i; ++n;", "rows[n] = q; cols[n] = q; ++n;"),
    ("enh: right band at the wrong position", "double right = band_min(A, B, L, W, 1, L - 1 - k);",
     "double right = band_min(A, B, L, W, 1, L - 2 - k);"),
    ("enh: right corner dropped", "double res = band_min(A, B, L, W, 0, 0) + band_min(A, B, L, W, 1, L - 1);",
     "double res = band_min(A, B, L, W, 0, 0);"),
    ("enh: right band of the left position", "double right = band_min(A, B, L, W, 1, L - 1 - k);",
     "double right = band_min(A, B, L, W, 0, L - 1 - k);"),
    ("enh: n_bands not clamped", "static int n_bands_of(int L, int V) { return imin(L / 2, V); }", "static int n_bands_of(int L, int V) { return V; }"),
    ("enh: keogh middle starts one late", "for (int i = nb; i < L - nb; ++i) res += keogh_term", "for (int i = nb + 1; i < L - nb; ++i) res += keogh_term"),
    ("eq7: left/right switch point", "else if (i >= L - nb)  s += band_min", "else if (i > L - nb)  s += band_min"),
    ("band set: left band misses a mirrored link", "rows[n] = j; cols[n] = i; ++n;\n        }\n    } else {", "}\n    } else {"),
    ("search: prune on >=", "CASCADE_KEOGH_ENH) {\n                    if (oracle_lb_keogh(A, Uk, Lk, L) > thr)",
     "CASCADE_KEOGH_ENH) {\n                    if (oracle_lb_keogh(A, Uk, Lk, L) >= thr)"),
    ("search: ties to the highest index", "return d < bd || (d == bd && k < bk);", "return d < bd || (d == bd && k > bk);"),
    ("search: order ties by reversed index", "return (a->idx > b->idx) - (a->idx < b->idx);", "return (a->idx < b->idx) - (a->idx > b->idx);"),
    ("search: no slack", "double thr = dmin(bsf, ub) * (1.0 + slack);", "double thr = dmin(bsf, ub);"),
    ("brute nn: last index on ties", "if (bi < 0 || d < best)", "if (bi < 0 || d <= best)"),
    ("ed2 skips the last point", "for (int i = 0; i < L; ++i) s += delta(A[i], B[i]);", "for (int i = 0; i < L - 1; ++i) s += delta(A[i], B[i]);"),
    ("grad: (i,j-1) preferred to (i-1,j) on ties", "else if (up == m) { --i; }\n        else { --j; }", "else if (lf == m) { --j; }\n        else { --i; }"),
    ("grad: diagonal preferred last on ties", "if (dg == m) { --i; --j; }\n        else if (up == m) { --i; }", "if (up == m) { --i; }\n        else if (dg == m) { --i; --j; }"),
    ("grad: factor 2 dropped", "g * (2.0 * ((double)A[pi[k]] - (double)B[pj[k]]))", "g * (((double)A[pi[k]] - (double)B[pj[k]]))"),
    ("grad: accumulated at the reference index", "gA[pi[k]] += g * (2.0", "gA[pj[k]] += g * (2.0"),
    ("grad: output weight ignored", "gA[pi[k]] += g * (2.0", "gA[pi[k]] += 1.0 * (2.0"),
    ("kim: extremes counted with repetitions", "if (!min_at_end) s += delta(amin, bmin);", "s += delta(amin, bmin);"),
    ("kim: max feature against the other minimum", "if (!max_at_end) s += delta(amax, bmax);", "if (!max_at_end) s += delta(amax, bmin);"),
    ("improved: second pass without the projection", "if (A[i] > U[i])       P[i] = U[i];", "if (A[i] > U[i])       P[i] = A[i];"),
    ("new: first point also takes a window minimum", "for (int i = 1; i < L - 1; ++i) {\n        double m = OINF;", "for (int i = 0; i < L - 1; ++i) {\n        double m = OINF;"),
    ("new: window one short", "j <= imin(L - 1, i + w); ++j) m = dmin(m, delta(A[i], B[j]));", "j < imin(L - 1, i + w); ++j) m = dmin(m, delta(A[i], B[j]));"),
    ("sym: smaller direction", "return ab > ba ? ab : ba;", "return ab < ba ? ab : ba;"),
    ("search: improved second pass counted at stage 1", "if (oracle_lb_improved(A, Bk, Uk, Lk, L, W, OINF) > thr) { c[C_PRUNED_ENH]++;", "if (oracle_lb_improved(A, Bk, Uk, Lk, L, W, OINF) > thr) { c[C_PRUNED_KEOGH]++;"),
    ("grad: last path cell dropped", "    for (int k = 0; k < n; ++k)\n        gA[pi[k]]", "    for (int k = 0; k < n - 1; ++k)\n        gA[pi[k]]"),
]


@pytest.mark.parametrize("desc,orig,bad", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(desc, orig, bad):
    src = open(SRC).read()
    assert src.count(orig) == 1, "mutation anchor not found: " + desc
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "mut.c")
        so = os.path.join(td, "mut.so")
        open(c, "w").write(src.replace(orig, bad))
        subprocess.check_call(["gcc", "-O1", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC",
                               "-shared", "-w", "-o", so, c, "-lm"])
        env = dict(os.environ, NNDTW_ORACLE_LIB=so, OMP_NUM_THREADS="2")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
        assert r.returncode != 0, "planted mistake not caught: " + desc
