"""Serving loop: NN-DTW queries against device-resident reference sets.

Requests (a query series for one of the resident sets) arrive over time.
The loop batches them continuously: whenever one of its streams is free it
admits the requests that have arrived, in arrival order, as long as the
batch's device workspace fits in the free part of one device-wide arena of
``budget_bytes`` (shared by every batch in flight, released when a batch's
completion event fires), and launches one batched search (one bound pass,
the sorts, the persistent searches) on that stream.  Batches on different
streams overlap on the device; a request's latency runs from its arrival to
the completion event of its batch.

Nothing on the admission path allocates device memory or waits for the
device: the workspace is carved out of the arena, each stream owns
preallocated query, output and pinned host result buffers, and
``nndtw_batch_prepare`` only enqueues its copy.  Results come back by an
asynchronous copy into the stream's pinned buffers, read once the batch's
event has fired.

Each request's result is that of a search of its query alone (same set,
options, round size and engine shape): batching changes the schedule, not
the computation.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field

import torch

from . import BatchSearcher, RefSet, _BatchPlan, _BatchSet, _check, _opts, lib

ALIGN = 256


@dataclass
class Request:
    rid: int
    set_id: int
    query: torch.Tensor          # device float32 [L_s]
    arrival: float               # seconds since the start of the session
    done: float = -1.0
    result: tuple = field(default=None)   # (nn index, nn distance, counts[8])


def batch_bytes(refsets, counts, V=5, cascade="keogh_enh", waves=0, helpers=0):
    """Device workspace of a batch with counts[s] queries for set s."""
    arr = (_BatchSet * len(refsets))()
    for d, (rs, c) in enumerate(zip(refsets, counts)):
        arr[d].refset = ctypes.addressof(rs.desc)
        arr[d].nQ = int(c)
    opts = _opts(V, cascade, 0, 0.0, True, 0, waves, helpers=helpers)
    nbytes = ctypes.c_size_t(0)
    _check(lib().nndtw_batch_workspace_bytes(arr, len(refsets), ctypes.byref(opts), ctypes.byref(nbytes)))
    return int(nbytes.value)


class Arena:
    """First-fit suballocation of one device buffer (offsets aligned to 256
    bytes).  ``alloc`` returns an offset or None; ``free`` returns a block."""

    def __init__(self, nbytes: int, device):
        self.size = (int(nbytes) // ALIGN) * ALIGN
        self.buf = torch.empty(max(self.size, ALIGN), dtype=torch.uint8, device=device)
        self.free_blocks = [(0, self.size)]          # sorted, coalesced (offset, size)
        self.used = 0

    def alloc(self, n: int):
        n = -(-int(n) // ALIGN) * ALIGN
        for k, (off, sz) in enumerate(self.free_blocks):
            if sz >= n:
                if sz == n:
                    del self.free_blocks[k]
                else:
                    self.free_blocks[k] = (off + n, sz - n)
                self.used += n
                return off, n
        return None

    def free(self, block):
        off, n = block
        self.used -= n
        blocks = self.free_blocks
        k = 0
        while k < len(blocks) and blocks[k][0] < off:
            k += 1
        blocks.insert(k, (off, n))
        # coalesce with the neighbours
        if k + 1 < len(blocks) and blocks[k][0] + blocks[k][1] == blocks[k + 1][0]:
            blocks[k] = (blocks[k][0], blocks[k][1] + blocks[k + 1][1])
            del blocks[k + 1]
        if k > 0 and blocks[k - 1][0] + blocks[k - 1][1] == blocks[k][0]:
            blocks[k - 1] = (blocks[k - 1][0], blocks[k - 1][1] + blocks[k][1])
            del blocks[k]

    def ptr(self, off: int):
        return ctypes.c_void_p(self.buf.data_ptr() + off)


class _Slot:
    """One stream with its preallocated query staging, outputs and pinned
    host result buffers (``max_batch`` queries of up to ``Lmax`` points)."""

    def __init__(self, device, max_batch: int, Lmax: int):
        self.stream = torch.cuda.Stream(device=device)
        self.q = torch.empty(max_batch * Lmax, dtype=torch.float32, device=device)
        # one buffer [nn_idx | nn_dist | counts] (so that one copy returns a
        # batch's results), and its pinned host twin
        mb = max_batch
        self.out = torch.empty(10 * mb, dtype=torch.int64, device=device)
        self.h_out = torch.empty(10 * mb, dtype=torch.int64, pin_memory=True)
        self.idx, self.dist, self.counts = self._views(self.out, mb)
        self.h_idx, self.h_dist, self.h_counts = self._views(self.h_out, mb)
        self.plan = _BatchPlan()
        self.event = torch.cuda.Event()

    @staticmethod
    def _views(buf, mb):
        return buf[:mb], buf[mb:2 * mb].view(torch.float64), buf[2 * mb:].view(mb, 8)


class Server:
    """Continuous batching over ``refsets`` (a list of RefSet) on
    ``n_streams`` streams; each batch holds at most ``max_batch`` requests,
    and the workspaces of all batches in flight fit in ``budget_bytes``.
    ``R`` and ``cpl`` (per set or None) are passed to every batch.
    ``helpers`` (idle workgroups that join a batch's running queries: 0 the
    library default, -1 none, or a count) is one value or one per set; a
    batch runs without helpers when every set in it asks for none, else with
    the most any of its sets asks for (0 counting as the default 7)."""

    def __init__(self, refsets, n_streams: int = 3, max_batch: int = 512, budget_bytes: int = 1 << 30,
                 V: int = 5, R=None, cpl=None, helpers: int = 0):
        self.refsets = list(refsets)
        dev = self.refsets[0].device
        self.max_batch = max_batch
        self.V = V
        hs = list(helpers) if isinstance(helpers, (list, tuple)) else [helpers] * len(self.refsets)
        if len(hs) != len(self.refsets):
            raise ValueError(f"{len(hs)} helper counts for {len(self.refsets)} sets")
        self.set_helpers = [int(h) for h in hs]
        # workspace of one query per set: an upper bound of what each query
        # adds to a batch (it includes the batch's fixed part once more, and
        # the helper header whether or not its batch uses helpers)
        self.per_query = [batch_bytes([rs], [1], V, helpers=0) for rs in self.refsets]
        if max(self.per_query) > budget_bytes:
            raise ValueError(f"budget of {budget_bytes} bytes below one query's workspace {max(self.per_query)}")
        self.arena = Arena(budget_bytes, dev)
        Lmax = max(rs.L for rs in self.refsets)
        self.slots = [_Slot(dev, max_batch, Lmax) for _ in range(n_streams)]
        # the round size and engine shape every batch uses per set (given, or
        # the batched search's defaults): a request's result is that of its
        # query searched alone with these
        probe = BatchSearcher([(rs, torch.zeros((1, rs.L), dtype=torch.float32, device=dev))
                               for rs in self.refsets], V=V, R=R, cpl=cpl)
        self.plan_R, self.plan_cpl = list(probe.R), list(probe.cpl)
        del probe
        torch.cuda.synchronize(dev)
        self.opts = {h: _opts(V, "keogh_enh", 0, 0.0, True, 0, helpers=h) for h in set(self.set_helpers) | {0, -1}}
        self.stats = {}

    def _helpers(self, sets):
        """The helper count of a batch over `sets` (set ids)."""
        hs = [self.set_helpers[s] for s in sets]
        if all(h == -1 for h in hs):
            return -1
        hmax = max(h if h > 0 else 7 for h in hs if h != -1)
        return 0 if hmax == 7 else hmax

    def _launch(self, reqs, slot: _Slot, block):
        """Enqueue one batched search over `reqs` on the slot's stream, its
        workspace at arena block `block`; returns per-request result rows."""
        by_set = {}
        for r in reqs:
            by_set.setdefault(r.set_id, []).append(r)
        sets = sorted(by_set)
        arr = (_BatchSet * len(sets))()
        row_of = {}
        qoff = row = 0
        with torch.cuda.stream(slot.stream):
            for k, s in enumerate(sets):
                rows = by_set[s]
                rs = self.refsets[s]
                n = len(rows)
                qv = slot.q[qoff:qoff + n * rs.L].view(n, rs.L)
                torch.stack([r.query for r in rows], out=qv)
                b = arr[k]
                b.refset = ctypes.addressof(rs.desc)
                b.Q, b.nQ = qv.data_ptr(), n
                b.nn_idx = slot.idx[row:].data_ptr()
                b.nn_dist = slot.dist[row:].data_ptr()
                b.counts = slot.counts[row:].data_ptr()
                b.R, b.cpl = self.plan_R[s], self.plan_cpl[s]
                for j, r in enumerate(rows):
                    row_of[r.rid] = row + j
                qoff += n * rs.L
                row += n
            st = ctypes.c_void_p(slot.stream.cuda_stream)
            ws = self.arena.ptr(block[0])
            hb = self._helpers(sets)
            if hb not in self.opts:
                self.opts[hb] = _opts(self.V, "keogh_enh", 0, 0.0, True, 0, helpers=hb)
            opts = self.opts[hb]
            _check(lib().nndtw_batch_prepare(arr, len(sets), ctypes.byref(opts), ws, block[1],
                                             ctypes.byref(slot.plan), st))
            _check(lib().nndtw_search_batch(ctypes.byref(slot.plan), ws, st))
            end = 2 * self.max_batch + 8 * row      # through the batch's last counts row
            slot.h_out[:end].copy_(slot.out[:end], non_blocking=True)
            slot.event.record(slot.stream)
        return row_of

    def _need(self, reqs):
        counts = {}
        for r in reqs:
            counts[r.set_id] = counts.get(r.set_id, 0) + 1
        sets = sorted(counts)
        return batch_bytes([self.refsets[s] for s in sets], [counts[s] for s in sets], self.V,
                           helpers=self._helpers(sets))

    def run(self, requests, poll_sleep: float = 0.0):
        """Serve `requests` (sorted by arrival time) in real time; returns
        them with completion times and results filled in, and a summary."""
        pending = list(requests)
        queue, inflight = [], []              # queue: arrived, not admitted
        free = list(range(len(self.slots)))
        t0 = time.perf_counter()
        nb = 0
        sizes = []
        max_inflight = max_bytes = 0
        head = 0
        while head < len(pending) or queue or inflight:
            now = time.perf_counter() - t0
            while head < len(pending) and pending[head].arrival <= now:
                queue.append(pending[head])
                head += 1
            # completions
            still = []
            for k, block, row_of, reqs in inflight:
                slot = self.slots[k]
                if slot.event.query():
                    tdone = time.perf_counter() - t0
                    idx, dist, counts = slot.h_idx.numpy(), slot.h_dist.numpy(), slot.h_counts.numpy()
                    for r in reqs:
                        j = row_of[r.rid]
                        r.done = tdone
                        r.result = (int(idx[j]), float(dist[j]), counts[j].tolist())
                    self.arena.free(block)
                    free.append(k)
                else:
                    still.append((k, block, row_of, reqs))
            inflight = still
            # admissions: arrival order, within the batch size and the free
            # part of the device-wide budget
            while queue and free:
                avail = max((sz for _, sz in self.arena.free_blocks), default=0)
                batch, est = [], 0
                while queue and len(batch) < self.max_batch:
                    need = self.per_query[queue[0].set_id]
                    if est + need > avail:
                        break
                    est += need
                    batch.append(queue.pop(0))
                if not batch:
                    break                          # wait for memory to free up
                block = self.arena.alloc(self._need(batch))
                if block is None:                  # the estimate bounds the need: not reached
                    queue[:0] = batch
                    break
                k = free.pop(0)
                row_of = self._launch(batch, self.slots[k], block)
                inflight.append((k, block, row_of, batch))
                nb += 1
                sizes.append(len(batch))
                max_inflight = max(max_inflight, len(inflight))
                max_bytes = max(max_bytes, self.arena.used)
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
            "max_batches_in_flight": max_inflight, "max_workspace_bytes": max_bytes,
            "budget_bytes": self.arena.size,
        }
        return requests, summary


def poisson_requests(sets_L, rate: float, duration: float, seed: int, device, make_query):
    """Requests of a seeded Poisson stream at `rate` per second over
    `duration` seconds; each picks a set uniformly; make_query(set, L, k)
    returns its float32 series (moved to `device` before the session).
    rate = inf gives every request at time 0 (a saturation run of
    `duration` requests)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    n_sat = int(duration) if rate == float("inf") else -1
    while True:
        if n_sat >= 0:
            if len(out) >= n_sat:
                break
        else:
            t += rng.exponential(1.0 / rate)
            if t > duration:
                break
        s = int(rng.integers(0, len(sets_L)))
        out.append(Request(len(out), s, torch.from_numpy(make_query(s, sets_L[s], len(out))).to(device), t))
    return out
