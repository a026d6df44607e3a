"""CPU oracle for LB_Enhanced-pruned NN-DTW (FP64, plain C via ctypes).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only code allowed to import this
package.  The GPU library shares no code with it.

Every function takes float32 numpy arrays (the same arrays the GPU path
consumes) and computes in float64; see ``nndtw_oracle.c`` for the paper
passage each routine follows.  ``paths.py`` adds a brute-force enumeration of
warping paths for tiny series.

Parity status: every routine here is pinned by ``tests/test_oracle_pins.py``
(closed forms, theorems of the paper, brute force and library routines).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nndtw_oracle.c")
LIB = os.path.join(HERE, "_nndtw_oracle.so")
# A planted-mistake build of the oracle (mutation tests only) may be loaded instead.
_ALT = os.environ.get("NNDTW_ORACLE_LIB")

CASCADE = {"none": 0, "keogh": 1, "keogh_enh": 2, "enh": 3,
           "kim": 4, "improved": 5, "new": 6, "enh_sym": 7}
COUNT_NAMES = ("n", "pruned_keogh", "pruned_enh_bands", "pruned_enh", "dtw_started",
               "dtw_abandoned", "cells", "fp64_rechecks")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, FP contraction off, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


SAN_LIB = os.path.join(HERE, "_nndtw_oracle_san.so")


def build_sanitized() -> str:
    """The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
    (gcc, every undefined-behaviour report fatal), for the CPU test that runs
    the pins against it.  Loading it needs the ASan runtime preloaded."""
    tmp = SAN_LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _ALT:
            L = ctypes.CDLL(_ALT)
        else:
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build(force=True)
            L = ctypes.CDLL(LIB)
        d, i32, i64, p = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
        sig = {
            "oracle_slack": (d, [i32]),
            "oracle_envelopes": (None, [p, i64, i32, i32, p, p]),
            "oracle_ed2": (d, [p, p, i32]),
            "oracle_lb_keogh": (d, [p, p, p, i32]),
            "oracle_band_cells": (i32, [i32, i32, i32, i32, p, p]),
            "oracle_left_bands_sum": (d, [p, p, i32, i32]),
            "oracle_right_bands_sum": (d, [p, p, i32, i32]),
            "oracle_lb_enhanced_eq7": (d, [p, p, p, p, i32, i32, i32]),
            "oracle_lb_enhanced_bands": (d, [p, p, i32, i32, i32]),
            "oracle_lb_enhanced_alg1": (d, [p, p, p, p, i32, i32, i32, d]),
            "oracle_dtw": (d, [p, p, i32, i32]),
            "oracle_dtw_abandon": (d, [p, p, i32, i32, d]),
            "oracle_ed2_batch": (None, [p, i64, p, i64, i32, i32, p]),
            "oracle_lb_keogh_batch": (None, [p, i64, p, p, i64, i32, i32, p]),
            "oracle_lb_enhanced_batch": (None, [p, i64, p, p, p, i64, i32, i32, i32, p, i32, i32, p]),
            "oracle_dtw_batch": (None, [p, i64, p, i64, i32, i32, p, i32, p]),
            "oracle_lb_kim": (d, [p, p, i32]),
            "oracle_lb_improved": (d, [p, p, p, p, i32, i32, d]),
            "oracle_lb_new": (d, [p, p, i32, i32]),
            "oracle_lb_enhanced_sym": (d, [p, p, p, p, p, p, i32, i32, i32]),
            "oracle_lb_compare_batch": (None, [i32, p, p, p, i64, p, p, p, i64, i32, i32, i32, p, i32, p]),
            "oracle_dtw_path": (ctypes.c_double, [p, p, i32, i32, p, p, p]),
            "oracle_dtw_grad_batch": (None, [p, i64, p, i64, i32, i32, i32, p, p, p]),
            "oracle_brute_nn": (None, [p, i64, p, i64, i32, i32, p, p]),
            "oracle_search": (None, [p, i64, p, i64, i32, i32, i32, i32, i64, i32, p, p, p]),
            "oracle_max_threads": (i32, []),
            "oracle_set_threads": (None, [i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _f32(x):
    return np.ascontiguousarray(x, dtype=np.float32)


def _ptr(x):
    return x.ctypes.data_as(ctypes.c_void_p) if x is not None else None


def _one(x):
    x = _f32(x)
    return x.reshape(1, -1) if x.ndim == 1 else x


def slack(L: int) -> float:
    return lib().oracle_slack(int(L))


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def max_threads() -> int:
    return lib().oracle_max_threads()


def envelopes(B, W):
    B = _one(B)
    n, L = B.shape
    U = np.empty_like(B)
    Lo = np.empty_like(B)
    lib().oracle_envelopes(_ptr(B), n, L, int(W), _ptr(U), _ptr(Lo))
    return U, Lo


def _pairing(A, B, zip_):
    if zip_ and A.shape[0] != B.shape[0]:
        raise ValueError("zip pairing needs equal counts")
    return (A.shape[0],) if zip_ else (A.shape[0], B.shape[0])


def ed2(A, B, zip_=False):
    A, B = _one(A), _one(B)
    out = np.empty(_pairing(A, B, zip_), np.float64)
    lib().oracle_ed2_batch(_ptr(A), A.shape[0], _ptr(B), B.shape[0], A.shape[1], int(zip_), _ptr(out))
    return out


def lb_keogh(A, U, Lo, zip_=False):
    A, U, Lo = _one(A), _one(U), _one(Lo)
    out = np.empty(_pairing(A, U, zip_), np.float64)
    lib().oracle_lb_keogh_batch(_ptr(A), A.shape[0], _ptr(U), _ptr(Lo), U.shape[0], A.shape[1],
                                int(zip_), _ptr(out))
    return out


def lb_enhanced(A, B, U, Lo, W, V, cutoff=None, zip_=False, variant="alg1"):
    """variant: 'eq7' (Equation 7), 'alg1' (Algorithm 1), 'bands' (Algorithm 1 bands part)."""
    A, B, U, Lo = _one(A), _one(B), _one(U), _one(Lo)
    out = np.empty(_pairing(A, B, zip_), np.float64)
    cut = None if cutoff is None else np.ascontiguousarray(np.broadcast_to(
        np.asarray(cutoff, np.float64), (A.shape[0],)))
    v = {"eq7": 0, "alg1": 1, "bands": 2}[variant]
    lib().oracle_lb_enhanced_batch(_ptr(A), A.shape[0], _ptr(B), _ptr(U), _ptr(Lo), B.shape[0],
                                   A.shape[1], int(W), int(V), _ptr(cut), int(zip_), v, _ptr(out))
    return out


def _compare(what, A, B, W=0, V=1, cutoff=None, zip_=False):
    A, B = _one(A), _one(B)
    out = np.empty(_pairing(A, B, zip_), np.float64)
    UA = LA = UB = LB = None
    if what == 3:
        UA, LA = envelopes(A, W)
    if what in (1, 3):
        UB, LB = envelopes(B, W)
    cut = None if cutoff is None else np.ascontiguousarray(np.broadcast_to(
        np.asarray(cutoff, np.float64), (A.shape[0],)))
    lib().oracle_lb_compare_batch(what, _ptr(A), _ptr(UA), _ptr(LA), A.shape[0], _ptr(B), _ptr(UB), _ptr(LB),
                                  B.shape[0], A.shape[1], int(W), int(V), _ptr(cut), int(zip_), _ptr(out))
    return out


def lb_kim(A, B, zip_=False):
    """LB_Kim, sum of the first, last, minimum and maximum features without repetitions."""
    return _compare(0, A, B, zip_=zip_)


def lb_improved(A, B, W, cutoff=None, zip_=False):
    """LB_Improved = LB_Keogh(A, B) + LB_Keogh(B, A'); +inf where LB_Keogh(A, B) > cutoff."""
    return _compare(1, A, B, W, cutoff=cutoff, zip_=zip_)


def lb_new(A, B, W, zip_=False):
    """LB_New: corner costs plus, per interior point, the nearest point of B in its window."""
    return _compare(2, A, B, W, zip_=zip_)


def lb_enhanced_sym(A, B, W, V, zip_=False):
    """max(LB_Enhanced^V(A, B), LB_Enhanced^V(B, A))."""
    return _compare(3, A, B, W, V, zip_=zip_)


def dtw(A, B, W, cutoff=None, zip_=False):
    A, B = _one(A), _one(B)
    out = np.empty(_pairing(A, B, zip_), np.float64)
    cut = None if cutoff is None else np.ascontiguousarray(np.broadcast_to(
        np.asarray(cutoff, np.float64), (A.shape[0],)))
    lib().oracle_dtw_batch(_ptr(A), A.shape[0], _ptr(B), B.shape[0], A.shape[1], int(W), _ptr(cut),
                           int(zip_), _ptr(out))
    return out


def dtw_path(a, b, W):
    """(DTW_W(a, b), argmin warping path as an int array [n][2] from (0,0) to
    (L-1,L-1)); ties resolved in the order (i-1,j-1), (i-1,j), (i,j-1)."""
    a, b = _f32(a), _f32(b)
    L = a.shape[0]
    pi = np.zeros(2 * L, np.int32)
    pj = np.zeros(2 * L, np.int32)
    n = ctypes.c_int(0)
    d = lib().oracle_dtw_path(_ptr(a), _ptr(b), L, int(W), _ptr(pi), _ptr(pj), ctypes.byref(n))
    return d, np.stack([pi[:n.value], pj[:n.value]], 1)


def dtw_grad(A, B, W, gout=None, zip_=False):
    """Gradient of DTW_W with respect to the query along the argmin path:
    returns (gA [nA][L], DTW_W per pair) with gA[a] = sum over the pairs
    (a, b) of gout[pair] * dDTW(a, b)/dA_a (gout defaults to ones)."""
    A, B = _one(A), _one(B)
    shape = _pairing(A, B, zip_)
    g = np.ones(shape, np.float64) if gout is None else np.ascontiguousarray(np.broadcast_to(
        np.asarray(gout, np.float64), shape))
    gA = np.zeros(A.shape, np.float64)
    dist = np.empty(shape, np.float64)
    lib().oracle_dtw_grad_batch(_ptr(A), A.shape[0], _ptr(B), B.shape[0], A.shape[1], int(W), int(zip_),
                                _ptr(g), _ptr(gA), _ptr(dist))
    return gA, dist


def left_bands_sum(a, b, W):
    a, b = _f32(a), _f32(b)
    return lib().oracle_left_bands_sum(_ptr(a), _ptr(b), a.shape[0], int(W))


def right_bands_sum(a, b, W):
    a, b = _f32(a), _f32(b)
    return lib().oracle_right_bands_sum(_ptr(a), _ptr(b), a.shape[0], int(W))


def band_cells(L, W, side, i):
    """Links (j, k) of the left (side 0), right (1) or vertical (2) band at i (0-based)."""
    rows = np.zeros(2 * L + 2, np.int32)
    cols = np.zeros(2 * L + 2, np.int32)
    n = lib().oracle_band_cells(int(L), int(W), int(side), int(i), _ptr(rows), _ptr(cols))
    return list(zip(rows[:n].tolist(), cols[:n].tolist()))


def brute_nn(refs, queries, W):
    refs, queries = _one(refs), _one(queries)
    Q = queries.shape[0]
    idx = np.empty(Q, np.int64)
    dist = np.empty(Q, np.float64)
    lib().oracle_brute_nn(_ptr(refs), refs.shape[0], _ptr(queries), Q, refs.shape[1], int(W),
                          _ptr(idx), _ptr(dist))
    return idx, dist


def search(refs, queries, W, V, cascade="keogh_enh", R=1, init_ub=True):
    """Round-based lower-bound search; returns (nn_idx, nn_dist, counts[Q][8])."""
    refs, queries = _one(refs), _one(queries)
    Q = queries.shape[0]
    idx = np.empty(Q, np.int64)
    dist = np.empty(Q, np.float64)
    counts = np.zeros((Q, 8), np.int64)
    lib().oracle_search(_ptr(refs), refs.shape[0], _ptr(queries), Q, refs.shape[1], int(W), int(V),
                        CASCADE[cascade], int(R), int(bool(init_ub)), _ptr(idx), _ptr(dist),
                        _ptr(counts))
    return idx, dist, counts
