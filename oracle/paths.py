"""Brute-force enumeration of warping paths for tiny series (L <= 8).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

A warping path (Section 2.1) starts at (1,1), ends at (L,L) and moves by one of
(1,0), (0,1), (1,1) at each step; under a window W every link satisfies
|i - j| <= W.  DTW_W is the minimum over those paths of the sum of point costs
delta(A_i, B_j) = (A_i - B_j)^2, summed from the first link to the last in
float64 (the order in which the cost-matrix recurrence accumulates a path).
"""
from __future__ import annotations

import functools


def enumerate_paths(L: int, W: int | None = None):
    """All warping paths as tuples of 0-based links (i, j)."""
    w = L - 1 if W is None else min(W, L - 1)
    out = []

    def rec(path):
        i, j = path[-1]
        if (i, j) == (L - 1, L - 1):
            out.append(tuple(path))
            return
        for di, dj in ((1, 0), (0, 1), (1, 1)):
            ni, nj = i + di, j + dj
            if ni < L and nj < L and abs(ni - nj) <= w:
                path.append((ni, nj))
                rec(path)
                path.pop()

    rec([(0, 0)])
    return out


@functools.lru_cache(maxsize=None)
def count_paths(L: int, W: int | None = None) -> int:
    return len(enumerate_paths(L, W))


def path_cost(a, b, path) -> float:
    s = 0.0
    for i, j in path:
        d = float(a[i]) - float(b[j])
        s = s + d * d
    return s


def dtw_brute(a, b, W: int | None = None) -> float:
    L = len(a)
    return min(path_cost(a, b, p) for p in enumerate_paths(L, W))
