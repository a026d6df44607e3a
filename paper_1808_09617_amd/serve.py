"""Serving loop: NN-DTW queries against device-resident reference sets.

Requests (a query series for one of the resident sets) arrive over time.
The loop batches them continuously: whenever one of its streams is free it
admits the requests that have arrived, in arrival order, while the batch's
device workspace stays within a memory budget, and launches one batched
search (``BatchSearcher``: one bound pass, the sorts, the persistent
searches) on that stream.  Batches on different streams overlap on the
device; a request's latency runs from its arrival to the completion event of
its batch.  Each request's result is that of a search of its query alone
(same set, options, round size and engine shape): batching changes the
schedule, not the computation.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field

import torch

from . import BatchSearcher, RefSet, _BatchSet, _check, _opts, lib


@dataclass
class Request:
    rid: int
    set_id: int
    query: torch.Tensor          # device float32 [L_s]
    arrival: float               # seconds since the start of the session
    done: float = -1.0
    result: tuple = field(default=None)   # (nn index, nn distance, counts[8])


def batch_bytes(refsets, counts, V=5, cascade="keogh_enh", waves=0):
    """Device workspace of a batch with counts[s] queries for set s."""
    arr = (_BatchSet * len(refsets))()
    for d, (rs, c) in enumerate(zip(refsets, counts)):
        arr[d].refset = ctypes.addressof(rs.desc)
        arr[d].nQ = int(c)
    opts = _opts(V, cascade, 0, 0.0, True, 0, waves)
    nbytes = ctypes.c_size_t(0)
    _check(lib().nndtw_batch_workspace_bytes(arr, len(refsets), ctypes.byref(opts), ctypes.byref(nbytes)))
    return int(nbytes.value)


class Server:
    """Continuous batching over ``refsets`` (a list of RefSet) on
    ``n_streams`` streams, each batch at most ``max_batch`` requests and
    ``budget_bytes`` of workspace.  ``R`` and ``cpl`` (per set or None) are
    passed to every batch."""

    def __init__(self, refsets, n_streams: int = 3, max_batch: int = 512, budget_bytes: int = 1 << 30,
                 V: int = 5, R=None, cpl=None):
        self.refsets = list(refsets)
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.max_batch = max_batch
        self.budget = budget_bytes
        self.V, self.R, self.cpl = V, R, cpl
        # workspace of one query per set, for admission by footprint
        self.per_query = [batch_bytes([rs], [1], V) for rs in self.refsets]
        # the round size and engine shape every batch uses per set (given, or
        # the batched search's defaults): a request's result is that of its
        # query searched alone with these
        probe = BatchSearcher([(rs, torch.zeros((1, rs.L), dtype=torch.float32, device=rs.device))
                               for rs in self.refsets], V=V, R=R, cpl=cpl)
        self.plan_R, self.plan_cpl = list(probe.R), list(probe.cpl)
        del probe

    def _launch(self, reqs, stream):
        """One batched search over `reqs` on `stream`; returns (searcher,
        event, per-request (set, row) positions)."""
        by_set = {}
        for r in reqs:
            by_set.setdefault(r.set_id, []).append(r)
        sets = sorted(by_set)
        where = {}
        R = [self.plan_R[s] for s in sets]
        cpl = [self.plan_cpl[s] for s in sets]
        with torch.cuda.stream(stream):
            pairs = []
            for k, s in enumerate(sets):
                rows = by_set[s]
                pairs.append((self.refsets[s], torch.stack([r.query for r in rows])))
                for j, r in enumerate(rows):
                    where[r.rid] = (k, j)
            bs = BatchSearcher(pairs, V=self.V, R=R, cpl=cpl)
            bs()
            ev = torch.cuda.Event()
            ev.record(stream)
        return bs, ev, where

    def run(self, requests, poll_sleep: float = 0.0):
        """Serve `requests` (sorted by arrival time) in real time; returns
        them with completion times and results filled in, and a summary."""
        pending = list(requests)
        queue, inflight = [], []              # queue: arrived, not admitted
        free = list(range(len(self.streams)))
        t0 = time.perf_counter()
        nb = 0
        sizes = []
        while pending or queue or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.pop(0))
            # completions
            still = []
            for bs, ev, where, reqs, k in inflight:
                if ev.query():
                    tdone = time.perf_counter() - t0
                    outs = [(i.cpu(), d.cpu(), c.cpu()) for i, d, c in bs.out]
                    for r in reqs:
                        s, j = where[r.rid]
                        r.done = tdone
                        r.result = (int(outs[s][0][j]), float(outs[s][1][j]), outs[s][2][j].tolist())
                    free.append(k)
                else:
                    still.append((bs, ev, where, reqs, k))
            inflight = still
            # admissions: arrival order, within the batch size and the budget
            while queue and free:
                batch, used = [], 0
                while queue and len(batch) < self.max_batch:
                    need = self.per_query[queue[0].set_id]
                    if batch and used + need > self.budget:
                        break
                    used += need
                    batch.append(queue.pop(0))
                k = free.pop(0)
                bs, ev, where = self._launch(batch, self.streams[k])
                inflight.append((bs, ev, where, batch, k))
                nb += 1
                sizes.append(len(batch))
            if poll_sleep:
                time.sleep(poll_sleep)
        wall = time.perf_counter() - t0
        lat = sorted(r.done - r.arrival for r in requests)
        n = len(lat)
        summary = {
            "requests": n, "batches": nb, "mean_batch": sum(sizes) / max(1, nb), "wall_s": wall,
            "throughput_rps": n / wall,
            "latency_ms": {"p50": 1e3 * lat[n // 2], "p99": 1e3 * lat[min(n - 1, int(0.99 * n))],
                           "max": 1e3 * lat[-1]},
        }
        return requests, summary


def poisson_requests(sets_L, rate: float, duration: float, seed: int, device, make_query):
    """Requests of a seeded Poisson stream at `rate` per second over
    `duration` seconds; each picks a set uniformly; make_query(set, L, k)
    returns its float32 series (moved to `device` before the session)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        s = int(rng.integers(0, len(sets_L)))
        out.append(Request(len(out), s, torch.from_numpy(make_query(s, sets_L[s], len(out))).to(device), t))
    return out
