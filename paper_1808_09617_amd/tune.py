"""Autotuner for batched searches: engine shape and round size per (L, W) bucket.

The search of one set has two free parameters that do not change its result
(only its schedule and its implementation-defined counts; the stage counts
are defined per round size R and the oracle takes the same R):

* cpl, the diagonal pairs per lane of the DTW engine (1 to 4 in a batch):
  small windows favour few pairs per lane (more groups per wave), large
  windows more pairs per lane (fewer lanes per group);
* R, the round size: small rounds keep the threshold tight, large rounds give
  the workgroup's groups enough candidates and fewer synchronised batches.

Sets are grouped into buckets of similar length and window (half-octaves of
L and of W'+1).  For each bucket the set with the most (query, reference)
pairs is searched on the GPU with every candidate (cpl, R), each timed with
events on the current stream (median of a few runs, after one warm-up run),
and the fastest pair is used for every set of the bucket.

``tune_latency`` tunes for the other regime, a request searched on its own
(a serving batch at low load): per set, the round size and whether idle
workgroups help the query, each timed on single-query batches.  Helpers pay
off where one DTW is long (their joining and the shared rounds cost a few
microseconds each) and cost time where it is short.
"""
from __future__ import annotations

import math

import torch

from . import BatchSearcher, Searcher

BATCH_MAX_CPL = 4


def shapes_for(W: int, L: int):
    """Engine shapes a batch can run for window W at length L (groups of at
    most 63 lanes)."""
    wp = min(W, L - 1)
    return [c for c in range(1, BATCH_MAX_CPL + 1) if -(-(wp + 1) // c) <= 63]


def bucket_of(L: int, W: int):
    wp = min(W, L - 1)
    return (round(2 * math.log2(L)), round(2 * math.log2(wp + 1)))


def _time_search(rs, Q, V, R, cpl, waves, reps):
    s = Searcher(rs, Q.shape[0], V=V, R=R, cpl=cpl, waves=waves)
    s(Q)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s(Q)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return sorted(times)[len(times) // 2], s.R, s.cpl


def autotune(pairs, V: int = 5, waves: int = 0, R_candidates=(64, 128, 256, 512), reps: int = 3):
    """pairs: list of (RefSet, queries).  Returns (R list, cpl list, report):
    per set the tuned round size and engine shape, and per bucket the timings
    of every candidate (ms) and the choice."""
    buckets = {}
    for d, (rs, Q) in enumerate(pairs):
        buckets.setdefault(bucket_of(rs.L, rs.W), []).append(d)
    R = [0] * len(pairs)
    cpl = [0] * len(pairs)
    report = {}
    for key, members in sorted(buckets.items()):
        rep = max(members, key=lambda d: pairs[d][0].n * pairs[d][1].shape[0])
        rs, Q = pairs[rep]
        trials = {}
        for c in shapes_for(rs.W, rs.L):
            for r in R_candidates:
                ms, r_used, c_used = _time_search(rs, Q, V, r, c, waves, reps)
                trials[(c_used, r_used)] = ms
        (c_best, r_best), ms_best = min(trials.items(), key=lambda kv: kv[1])
        for d in members:
            R[d], cpl[d] = r_best, c_best
        report[f"L{rs.L}_W{rs.W}"] = {"sets": len(members), "cpl": c_best, "R": r_best, "ms": ms_best,
                                      "trials": {f"C{c}_R{r}": round(t, 3) for (c, r), t in trials.items()}}
    return R, cpl, report


def tune_latency(pairs, cpl, V: int = 5, R_candidates=(128, 256, 512), helper_candidates=(-1, 0), reps: int = 8):
    """pairs: list of (RefSet, sample queries [k][L]); cpl: the engine shape
    per set.  Each set's (R, helpers) is the pair with the smallest mean GPU
    time over single-query batches of its first `reps` sample queries (the
    same queries for every pair, after one untimed batch per pair; queries
    differ in cost far more than the runs of one query do, so the mean over
    several of them, not one query's median, decides).  Returns (R list,
    helpers list, report)."""
    R, H, report = [], [], {}
    for d, (rs, Q) in enumerate(pairs):
        trials = {}
        for r in R_candidates:
            for h in helper_candidates:
                times = []
                for k in range(reps + 1):
                    q = Q[k % Q.shape[0]:k % Q.shape[0] + 1]
                    b = BatchSearcher([(rs, q)], V=V, R=[r], cpl=[cpl[d]], helpers=h)
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    b()
                    e1.record()
                    e1.synchronize()
                    if k > 0:
                        times.append(e0.elapsed_time(e1))
                trials[(r, h)] = sum(times) / len(times)
        (r_best, h_best), ms = min(trials.items(), key=lambda kv: kv[1])
        R.append(r_best)
        H.append(h_best)
        report[f"L{rs.L}_W{rs.W}"] = {"R": r_best, "helpers": h_best, "ms": round(ms, 3),
                                      "trials": {f"R{r}_h{h}": round(t, 3) for (r, h), t in trials.items()}}
    return R, H, report
