#!/usr/bin/env python3
"""Benchmark of the NN-DTW hot path on one MI355X.

A step is one pass of the whole path over one batch: build the reference set
(copy, envelopes, point-major copies), then the search (fused bound pass,
visiting order, round-based pruned search with DTW_W).  The headline workload
is the largest plain NN-DTW configuration: 5000 references x 500 queries,
L=512, random walks mixed with class sinusoids, window W=51 (0.1 L, the
paper's recommended fraction) with V=5 and the LB_Keogh -> LB_Enhanced
cascade.  Inputs are resident in HBM before timing starts.  The 1000 x 1000,
L=256 class-sinusoid configuration, the whole window sweep, batching,
serving, the backward pass and the comparison bounds are reported beside it.

Prints ONE JSON line: the headline throughput (queries/s, whole step), the
step's latency and stage times, the search kernel's roofline (3 VALU lane
operations per band cell it evaluates, over its average duration from HIP
events and, when the committed rocprofv3 summary was taken from the same
device code, from that trace; HBM bytes per launch from the committed
FETCH_SIZE / WRITE_SIZE summary), the pruning rates and stage counts, the CPU
oracle's rate on a sample, and the extras above.
"""
import argparse
import ctypes
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

VALU_PEAK_OPS = 256 * 64 * 2.4e9      # non-packed VALU lane operations per second (fp32 or fp64)
HBM_PEAK = 8.0e12
METRIC = "NN-DTW queries/sec and DTW cells/sec (% VALU peak); pruning rate; p99 latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Hip:
    """Minimal HIP event API through ctypes (events on torch's current stream)."""

    def __init__(self):
        self.h = ctypes.CDLL("libamdhip64.so")
        self.h.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.h.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        self.h.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.h.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def events(self, n):
        arr = (ctypes.c_void_p * n)()
        for i in range(n):
            e = ctypes.c_void_p()
            assert self.h.hipEventCreate(ctypes.byref(e)) == 0
            arr[i] = e.value
        return arr

    def record(self, ev, stream):
        assert self.h.hipEventRecord(ev, stream) == 0

    def ms(self, a, b):
        f = ctypes.c_float(0)
        assert self.h.hipEventElapsedTime(ctypes.byref(f), a, b) == 0
        return float(f.value)


def device_code_fingerprint():
    """SHA-256 of the device code of the built library (its .hip_fatbin
    section, read from the ELF section table): it changes exactly when a
    kernel's code changes, not with comments or host code."""
    import hashlib
    import struct
    path = os.path.join(ROOT, "paper_1808_09617_amd", "libnndtw.so")
    if not os.path.exists(path):
        return None
    data = open(path, "rb").read()
    shoff = struct.unpack_from("<Q", data, 0x28)[0]
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", data, 0x3A)

    def section(i):
        return struct.unpack_from("<IIQQQQIIQQ", data, shoff + i * shentsize)

    names = section(shstrndx)[4]
    for i in range(shnum):
        name_off, _, _, _, off, size = section(i)[:6]
        end = data.index(b"\0", names + name_off)
        if data[names + name_off:end] == b".hip_fatbin":
            return hashlib.sha256(data[off:off + size]).hexdigest()
    return None


def profiled_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE
    summary, or None if the kernels changed since those counters were taken."""
    path = os.path.join(ROOT, "profiles", f"memory_counters_{workload}.txt")
    if not os.path.exists(path):
        return None
    fp, val = None, None
    for line in open(path):
        if line.startswith("# device code fingerprint"):
            fp = line.split(":", 1)[1].strip()
        # the kernel's family (search_kernel covers search_kernel_wide, ...)
        if line.startswith("# bytes_per_launch ") and kernel in line.split()[2] and "batch" not in line:
            val = int(line.split()[3])
    return val if fp is not None and fp == device_code_fingerprint() else None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, W, V, target_s, unit_scale=1.0):
    """The oracle's paper-mode search (R = 1, the paper's sequential loop) on
    the host's cores: all threads over a prefix of the queries sized to about
    target_s seconds, then one thread over a smaller prefix."""
    import oracle
    threads = oracle.max_threads()
    nq_all = wl.queries.shape[0]
    n = min(nq_all, max(4, threads))
    t = time.perf_counter()
    oracle.search(wl.refs, wl.queries[:n], W, V, "keogh_enh", 1, True)
    dt = time.perf_counter() - t
    want = int(min(nq_all, max(n, n * target_s / max(dt, 1e-3))))
    t = time.perf_counter()
    oracle.search(wl.refs, wl.queries[:want], W, V, "keogh_enh", 1, True)
    dt = time.perf_counter() - t
    # single thread, on a prefix of about target_s / 4 seconds
    one = int(min(want, max(1, want * (target_s / 4.0) / max(dt * threads, 1e-3))))
    oracle.set_threads(1)
    try:
        t = time.perf_counter()
        oracle.search(wl.refs, wl.queries[:one], W, V, "keogh_enh", 1, True)
        dt1 = time.perf_counter() - t
    finally:
        oracle.set_threads(threads)
    return {"value": want / dt, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "single_thread": {"value": one / dt1, "unit": "queries/s", "queries": one, "wall_s": dt1},
            "sample": f"first {want} of {nq_all} queries of {wl.name}, full reference set ({wl.refs.shape[0]}), "
                      f"W={W}, paper-mode sequential search (R=1), LB_Keogh->LB_Enhanced^{V}, FP64, "
                      f"{dt:.1f} s wall on {threads} threads; single thread: first {one} queries, {dt1:.1f} s"}


def hbm_streaming(nd, synth, torch, dev):
    """Bandwidth of the streaming kernels on a reference set far larger than
    the 256 MB MALL (200,000 x 512, mix, W=51, V=5): the envelope pass and the
    fused bound pass at 1 and 64 queries.  Algorithmic bytes: envelopes read B
    and write U, Lo (12 B per element); the bound pass streams the point-major
    B, U, Lo once per tile of 4 queries (12 B per reference point per tile),
    reads the queries and writes four float64 values per (query, reference)."""
    hb = synth.workload("nndtw-hbm512")
    W, V = hb.windows[0], 5
    n, L = hb.refs.shape
    B = torch.from_numpy(hb.refs).to(dev)
    Qall = torch.from_numpy(hb.queries).to(dev)
    rs = nd.RefSet(B, W)

    def timed(fn, reps=5):
        fn()
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3)
        return sorted(times)[len(times) // 2]

    out = {"workload": "nndtw-hbm512", "N": n, "L": L, "W": W, "V": V, "resident_refset_bytes": int(rs.mem.numel())}
    t = timed(lambda: nd.envelopes(B, W))
    out["envelopes"] = {"ms": t * 1e3, "gbps": 12.0 * n * L / t / 1e9}
    for nq in (1, 64):
        Qs = Qall[:nq].contiguous()
        t = timed(lambda: nd.cascade_bounds(rs, Qs, V))
        tiles = -(-nq // 4)
        byts = 12.0 * n * L * tiles + 4.0 * nq * L + 32.0 * nq * n
        out[f"bounds_q{nq}"] = {"ms": t * 1e3, "gbps": byts / t / 1e9, "fp64_gops": 10.0 * nq * n * L / t / 1e9}
    del rs, B
    torch.cuda.empty_cache()
    return out


def backward_bench(nd, synth, torch, dev, reps=5, cpu=True):
    """DTW_W forward with argmin codes and the backward (gradient with
    respect to the queries) for 256 queries x 256 references, L=256, W=26,
    FP32, inputs resident; the oracle's FP64 gradient timed on a sample."""
    L, W = 256, 26
    A = torch.from_numpy(synth.random_series(256, L, seed=1900, kind="sin5")).to(dev)
    B = torch.from_numpy(synth.random_series(256, L, seed=1901, kind="sin5")).to(dev)
    g = torch.randn(256, 256, device=dev)
    out, codes = nd.dtw_w_codes(A, B, W)
    nd.dtw_w_backward(A, B, W, g, codes)
    torch.cuda.synchronize()
    tf, tb = [], []
    for _ in range(reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        out, codes = nd.dtw_w_codes(A, B, W)
        e[1].record()
        nd.dtw_w_backward(A, B, W, g, codes)
        e[2].record()
        e[2].synchronize()
        tf.append(e[0].elapsed_time(e[1]) / 1e3)
        tb.append(e[1].elapsed_time(e[2]) / 1e3)
    tf, tb = sorted(tf)[reps // 2], sorted(tb)[reps // 2]
    cells = 256 * 256 * (L * (2 * W + 1) - W * (W + 1))
    res = {"config": "256 x 256 pairs, L=256, W=26, fp32", "forward_ms": tf * 1e3, "backward_ms": tb * 1e3,
           "pairs_per_s": 65536 / (tf + tb), "forward_cells_per_s": cells / tf,
           "forward_valu_frac": 3.0 * cells / tf / VALU_PEAK_OPS, "codes_bytes": int(codes.numel())}
    if cpu:
        import oracle
        a, b = A[:4].cpu().numpy(), B.cpu().numpy()
        t = time.perf_counter()
        oracle.dtw_grad(a, b, W, gout=g[:4].double().cpu().numpy())
        dt = time.perf_counter() - t
        res["cpu_oracle"] = {"pairs_per_s": 4 * 256 / dt, "cores": oracle.max_threads(),
                             "sample": "4 queries x 256 references, FP64 full matrix + backtrack"}
    del codes, out
    torch.cuda.empty_cache()
    return res


def one_request_latency(nd, synth, torch, dev, serve, rss, Ls, R, cpl, helpers=0, reps=30):
    """GPU time of a batch holding one request, per serving set (HIP events
    around the batch's launch on its stream; median and maximum over `reps`
    requests), with the server's own buffers and plan."""
    server = serve.Server(rss, n_streams=1, R=R, cpl=cpl, helpers=helpers)
    slot = server.slots[0]
    out = {}
    for s, L in enumerate(Ls):
        ms = []
        for k in range(-2, reps):                  # two untimed warm-up requests
            q = torch.from_numpy(synth.serving_query(s, L, 5 * 10 ** 6 + k)).to(dev)
            r = serve.Request(k, s, q, 0.0)
            torch.cuda.synchronize()
            blk = server.arena.alloc(server._need([r]))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(slot.stream)
            server._launch([r], slot, blk)
            e1.record(slot.stream)
            e1.synchronize()
            server.arena.free(blk)
            if k >= 0:
                ms.append(e0.elapsed_time(e1))
        ms.sort()
        out[str(L)] = {"median_ms": ms[len(ms) // 2], "max_ms": ms[-1]}
    del server
    return out


def serving_bench(nd, synth, torch, dev, rate=2000.0, duration=3.0):
    """A seeded Poisson stream of NN-DTW requests at `rate` per second for
    `duration` seconds against 8 resident reference sets of 4000 random walks
    (lengths 64 .. 1024, W = 0.1 L, V = 5), served by continuous batching on
    3 streams; queries resident on the device before the session."""
    from paper_1808_09617_amd import serve
    sets = synth.serving_sets()
    rss = [nd.RefSet(torch.from_numpy(refs).to(dev), W) for refs, W in sets]
    Ls = [refs.shape[1] for refs, _ in sets]
    warm = serve.poisson_requests(Ls, rate=rate, duration=0.2, seed=1, device=dev,
                                  make_query=lambda s, L, k: synth.serving_query(s, L, 10 ** 6 + k))
    reqs = serve.poisson_requests(Ls, rate=rate, duration=duration, seed=2, device=dev,
                                  make_query=lambda s, L, k: synth.serving_query(s, L, k))
    torch.cuda.synchronize()
    # per-set round size and engine shape, tuned on 16 sample queries per set
    from paper_1808_09617_amd import tune
    sample = [(rs, torch.stack([torch.from_numpy(synth.serving_query(s, Ls[s], 2 * 10 ** 6 + k)).to(dev)
                                for k in range(16)])) for s, rs in enumerate(rss)]
    R, cpl, _ = tune.autotune(sample, V=5)
    # at 2000 requests/s a batch holds one request or two: the round size and
    # the helper workgroups per set tuned for one request on its own
    R_lat, helpers, _ = tune.tune_latency(sample, cpl, V=5)
    # the same stream without helper workgroups, for comparison
    server = serve.Server(rss, n_streams=3, R=R_lat, cpl=cpl, helpers=-1)
    server.run(warm)
    _, nohelp = server.run(reqs)
    del server
    server = serve.Server(rss, n_streams=3, R=R_lat, cpl=cpl, helpers=helpers)
    server.run(warm)
    _, summary = server.run(reqs)
    del server
    summary.update({"offered_rps": rate, "sets": len(sets), "refs_per_set": sets[0][0].shape[0],
                    "lengths": Ls, "R": R_lat, "cpl": cpl, "helpers": helpers, "R_saturation": R,
                    "without_helpers": {"mean_batch": nohelp["mean_batch"], "latency_ms": nohelp["latency_ms"]}})
    # saturation runs with the round sizes tuned for batches of many queries
    server = serve.Server(rss, n_streams=3, R=R, cpl=cpl)
    # saturation: 4000 requests present at the start, served as fast as the
    # server admits them (batches of up to 512 within the 1 GiB budget)
    sat = serve.poisson_requests(Ls, rate=float("inf"), duration=4000, seed=3, device=dev,
                                 make_query=lambda s, L, k: synth.serving_query(s, L, 3 * 10 ** 6 + k))
    torch.cuda.synchronize()
    _, ssum = server.run(sat)
    summary["saturation"] = {k: ssum[k] for k in ("requests", "batches", "mean_batch", "wall_s", "throughput_rps",
                                                  "max_batches_in_flight", "max_workspace_bytes", "budget_bytes")}
    del server
    summary["one_request"] = one_request_latency(nd, synth, torch, dev, serve, rss, Ls, R_lat, cpl, helpers)
    del rss
    torch.cuda.empty_cache()
    return summary


def batch_bench(nd, synth, torch, dev, reps=3, tuned=None):
    """The batching workload (64 random-walk sets, L 25..1839, 26,583 queries,
    W = 0.1 L, V = 5) as one captured graph of the batched search, inputs
    resident; against the same sets searched one after another with the
    single-set entry point.  Reference-set builds and planning are untimed
    (the paper's training time)."""
    sets = synth.batch_workload()
    pairs = [(nd.RefSet(torch.from_numpy(ds.refs).to(dev), ds.W), torch.from_numpy(ds.queries).to(dev))
             for ds in sets]
    nq = sum(ds.queries.shape[0] for ds in sets)
    R = cpl = None
    report = None
    if tuned is not None:
        from paper_1808_09617_amd import tune
        t0 = time.perf_counter()
        R, cpl, report = tune.autotune(pairs, V=5)
        tune_s = time.perf_counter() - t0
    def graph_time(bsr):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            bsr()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            bsr()
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            g.replay()
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3)
        del g
        return sorted(times)[len(times) // 2]

    # without helper workgroups first (same plan otherwise), for comparison
    bsr = nd.BatchSearcher(pairs, V=5, R=R, cpl=cpl, helpers=-1)
    t_nohelp = graph_time(bsr)
    del bsr
    torch.cuda.empty_cache()
    bsr = nd.BatchSearcher(pairs, V=5, R=R, cpl=cpl)
    t = graph_time(bsr)
    cells = sum(int(c[:, 6].sum()) for _, _, c in bsr.out)
    started = sum(int(c[:, 4].sum()) for _, _, c in bsr.out)
    pairs_total = sum(ds.refs.shape[0] * ds.queries.shape[0] for ds in sets)
    out = {"workload": "batch64-rw", "sets": len(sets), "queries": nq, "pairs": pairs_total,
           "schedule": "autotuned" if tuned is not None else "library defaults",
           "ms": t * 1e3, "helpers": bsr.helpers, "ms_without_helpers": t_nohelp * 1e3,
           "queries_per_s": nq / t, "dtw_cells_per_s": cells / t,
           "valu_frac_dtw": 3.0 * cells / t / VALU_PEAK_OPS, "pruning_rate": 1.0 - started / pairs_total,
           "launches": 1 + sum(1 for c in bsr.plan.order_cnt if c) + sum(1 for c in bsr.plan.search_cnt if c),
           "shapes": {f"C{sh // 2 + 1}{'x' if sh & 1 else ''}": int(bsr.plan.search_cnt[sh])
                      for sh in range(8) if bsr.plan.search_cnt[sh]}}
    # the same sets one after another through the single-set entry point
    srs = [nd.Searcher(rs, Q.shape[0], V=5, R=bsr.R[d], cpl=bsr.cpl[d]) for d, (rs, Q) in enumerate(pairs)]
    for (rs, Q), sr in zip(pairs, srs):
        sr(Q)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for (rs, Q), sr in zip(pairs, srs):
        sr(Q)
    e1.record()
    e1.synchronize()
    t1 = e0.elapsed_time(e1) / 1e3
    out["per_set_loop_ms"] = t1 * 1e3
    out["speedup_vs_per_set_loop"] = t1 / t
    if report is not None:
        out["tuning_s"] = tune_s
        out["buckets"] = {k: {"sets": v["sets"], "cpl": v["cpl"], "R": v["R"]} for k, v in report.items()}
    del bsr, srs, pairs
    torch.cuda.empty_cache()
    return out


def _median_ms(torch, fn, reps):
    times = []
    out = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        out = fn()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return sorted(times)[len(times) // 2], out


def window_sweep(nd, synth, torch, dev, reps=3):
    """The window sweep: 5000 mixed references (random walks and class
    sinusoids) x 500 queries, L=512, W = round(f L) for f in {0.01, 0.1,
    0.25, 0.5, 1.0} (W = 5, 51, 128, 256, 511), V in {1, 5}, cascade
    LB_Keogh -> LB_Enhanced^V.  Per (W, V): the reference-set build, the
    search and their sum (end to end), pruning per stage, DTW cells/s."""
    wl = synth.workload("nndtw-mix512")
    refs = torch.from_numpy(wl.refs).to(dev)
    qs = torch.from_numpy(wl.queries).to(dev)
    N, Q = wl.refs.shape[0], wl.queries.shape[0]
    rows = []
    for W in wl.windows:
        rs = nd.RefSet(refs, W)
        t_build, _ = _median_ms(torch, lambda: rs.rebuild(refs), reps)
        for V in wl.vs:
            sr = nd.Searcher(rs, Q, V=V, cascade="keogh_enh")
            sr(qs)
            t_search, (_, _, c) = _median_ms(torch, lambda: sr(qs), reps)
            c = c.cpu().numpy()
            pairs = N * Q
            rows.append({"W": W, "V": V, "cpl": sr.cpl, "R": sr.R, "build_ms": t_build, "search_ms": t_search,
                         "end_to_end_ms": t_build + t_search, "queries_per_s": Q / ((t_build + t_search) / 1e3),
                         "pruning_rate": 1.0 - int(c[:, 4].sum()) / pairs,
                         "pruned": {"keogh": int(c[:, 1].sum()) / pairs, "enh_bands": int(c[:, 2].sum()) / pairs,
                                    "enh": int(c[:, 3].sum()) / pairs},
                         "dtw_cells_per_s": int(c[:, 6].sum()) / (t_search / 1e3)})
            del sr
        del rs
    torch.cuda.empty_cache()
    return {"workload": "nndtw-mix512", "N": N, "Q": Q, "L": wl.L, "rows": rows}


def small_latency(nd, synth, torch, dev, calls=1000):
    """The smallest instance (100 random-walk references x 20 queries, L=64,
    W=6, V=1): per-call latency of the search over `calls` calls (HIP events
    around each call; reference set built once), p50 and p99."""
    wl = synth.workload("nndtw-small")
    refs = torch.from_numpy(wl.refs).to(dev)
    qs = torch.from_numpy(wl.queries).to(dev)
    rs = nd.RefSet(refs, wl.windows[0])
    sr = nd.Searcher(rs, qs.shape[0], V=wl.vs[0], cascade="keogh_enh")
    for _ in range(10):
        sr(qs)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(calls)]
    torch.cuda.synchronize()
    for e0, e1 in ev:
        e0.record()
        sr(qs)
        e1.record()
    torch.cuda.synchronize()
    lat = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    # the same call captured once in a graph and replayed (one launch per call)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        sr(qs)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sr(qs)
    for _ in range(10):
        g.replay()
    torch.cuda.synchronize()
    for e0, e1 in ev:
        e0.record()
        g.replay()
        e1.record()
    torch.cuda.synchronize()
    glat = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    pct = lambda v: {"p50": v[calls // 2], "p99": v[int(math.ceil(0.99 * calls)) - 1], "max": v[-1]}
    return {"workload": "nndtw-small", "N": wl.refs.shape[0], "Q": wl.queries.shape[0], "L": wl.L,
            "W": wl.windows[0], "V": wl.vs[0], "calls": calls, "latency_ms": pct(lat),
            "graph_latency_ms": pct(glat),
            "queries_per_s_at_p50": wl.queries.shape[0] / (lat[calls // 2] / 1e3),
            "queries_per_s_at_p50_graph": wl.queries.shape[0] / (glat[calls // 2] / 1e3)}


def arms_2x2(nd, torch, rs, qs, V, nq_per_query=100, reps=3):
    """{per-query, batched} x {LB_Keogh, LB_Keogh -> LB_Enhanced^V} on the
    benchmarked set, search only (reference set built): batched = all queries
    in one call; per-query = one query per call (timed over nq_per_query calls)."""
    out = {}
    for cas in ("keogh", "keogh_enh"):
        sr = nd.Searcher(rs, qs.shape[0], V=V, cascade=cas)
        sr(qs)
        t, _ = _median_ms(torch, lambda: sr(qs), reps)
        one = nd.Searcher(rs, 1, V=V, cascade=cas)
        one(qs[:1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(nq_per_query):
            one(qs[i:i + 1])
        torch.cuda.synchronize()
        per = nq_per_query / (time.perf_counter() - t0)
        out[cas] = {"batched_queries_per_s": qs.shape[0] / (t / 1e3), "per_query_queries_per_s": per}
    out["factor_batching"] = {c: out[c]["batched_queries_per_s"] / out[c]["per_query_queries_per_s"]
                              for c in ("keogh", "keogh_enh")}
    out["factor_enhanced"] = {m: out["keogh_enh"][m] / out["keogh"][m]
                              for m in ("batched_queries_per_s", "per_query_queries_per_s")}
    return out


def per_v(nd, torch, rs, qs, reps=3):
    """The benchmarked set at V = 1, 2, 5 (search only): queries/s and pruning per stage."""
    out = {}
    N, Q = rs.n, qs.shape[0]
    for V in (1, 2, 5):
        sr = nd.Searcher(rs, Q, V=V, cascade="keogh_enh")
        sr(qs)
        t, (_, _, c) = _median_ms(torch, lambda: sr(qs), reps)
        c = c.cpu().numpy()
        out[str(V)] = {"search_ms": t, "queries_per_s": Q / (t / 1e3),
                       "pruning_rate": 1.0 - int(c[:, 4].sum()) / (N * Q),
                       "pruned": {"keogh": int(c[:, 1].sum()) / (N * Q), "enh_bands": int(c[:, 2].sum()) / (N * Q),
                                  "enh": int(c[:, 3].sum()) / (N * Q)}}
    return out


COMPARE_CASCADES = (("kim", "kim"), ("keogh", "keogh"), ("improved", "improved"), ("new", "new"),
                    ("enhanced5", "enh"), ("keogh_enhanced5", "keogh_enh"), ("enhanced5_sym", "enh_sym"))


def compare_bounds(nd, synth, torch, dev, a, b, W=26):
    """Synthetic analogues of the paper's comparisons (UCR is not available):
    tightness LB/DTW of every bound on the independent class-sinusoid pairs
    (L=256, W=26), and the NN-DTW search with each bound alone (plus the
    cascade and the symmetric variant) on the benchmarked 1000 x 1000 set and
    across the windows of the window sweep (V=5).  Search time includes the
    bound pass, the ordering and the DTWs."""
    A, B = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    U, Lo = nd.envelopes(B, W)
    d = nd.dtw_w(A, B, W, zip_=True).double()
    keep = d > 0
    bounds = {"kim": nd.lb_kim(A, B, zip_=True), "keogh": nd.lb_keogh(A, U, Lo, zip_=True),
              "improved": nd.lb_improved(A, B, U, Lo, W, zip_=True), "new": nd.lb_new(A, B, W, zip_=True),
              "enhanced5_sym": nd.lb_enhanced_sym(A, B, U, Lo, W, 5, zip_=True)}
    for v in (1, 2, 5):
        bounds[f"enhanced{v}"] = nd.lb_enhanced(A, B, U, Lo, W, v, zip_=True)
    tight = {k: float((x[keep] / d[keep]).mean()) for k, x in bounds.items()}
    ms = {}
    for k, x in bounds.items():
        if k.startswith("enhanced") and k != "enhanced5":
            continue
        fn = {"kim": lambda: nd.lb_kim(A, B, zip_=True), "keogh": lambda: nd.lb_keogh(A, U, Lo, zip_=True),
              "improved": lambda: nd.lb_improved(A, B, U, Lo, W, zip_=True),
              "new": lambda: nd.lb_new(A, B, W, zip_=True),
              "enhanced5": lambda: nd.lb_enhanced(A, B, U, Lo, W, 5, zip_=True),
              "enhanced5_sym": lambda: nd.lb_enhanced_sym(A, B, U, Lo, W, 5, zip_=True)}[k]
        fn()
        ms[k], _ = _median_ms(torch, fn, 3)
    del A, B, U, Lo, d, bounds

    def search_rows(refs, qs, W, reps):
        rs = nd.RefSet(refs, W)
        out = {}
        for name, cas in COMPARE_CASCADES:
            sr = nd.Searcher(rs, qs.shape[0], V=5, cascade=cas)
            sr(qs)
            t, (_, _, c) = _median_ms(torch, lambda: sr(qs), reps)
            c = c.cpu().numpy()
            pairs = refs.shape[0] * qs.shape[0]
            out[name] = {"search_ms": t, "queries_per_s": qs.shape[0] / (t / 1e3),
                         "pruning_rate": 1.0 - int(c[:, 4].sum()) / pairs}
            del sr
        del rs
        return out

    wl = synth.workload("nndtw-sin256")
    c2 = search_rows(torch.from_numpy(wl.refs).to(dev), torch.from_numpy(wl.queries).to(dev), W, 3)
    mx = synth.workload("nndtw-mix512")
    refs, qs = torch.from_numpy(mx.refs).to(dev), torch.from_numpy(mx.queries).to(dev)
    c3 = {str(w): search_rows(refs, qs, w, 1) for w in mx.windows}
    torch.cuda.empty_cache()
    return {"tightness_pairs": int(keep.sum()), "W": W, "tightness": tight, "pairwise_ms_250k": ms,
            "search_nndtw_sin256": c2, "search_nndtw_mix512_by_W": c3}


def profiled_kernel_us(kernel, workload):
    """Average duration (us) of `kernel` in the committed rocprofv3 kernel-trace
    summary of `workload`, if it was taken from the current device code."""
    path = os.path.join(ROOT, "profiles", f"kernel_stats_{workload}.txt")
    if not os.path.exists(path):
        return None
    fp, val = None, None
    for line in open(path):
        if line.startswith("# device code fingerprint"):
            fp = line.split(":", 1)[1].strip()
        parts = line.split()
        if not line.startswith("#") and len(parts) >= 6 and kernel in line:
            try:
                val = float(parts[-4])
            except ValueError:
                pass
    return val if fp is not None and fp == device_code_fingerprint() else None


def search_step_bench(nd, torch, hip, dev, wl, W, V, args, headline):
    """Time steps (reference-set build + full search) of one workload: K timed
    steps that enqueue nothing else, then K untimed steps with an event pair
    each (latency) and K with events between the stages (stage times, and the
    search kernel's average duration for the roofline)."""
    N, Q, L = wl.refs.shape[0], wl.queries.shape[0], wl.L
    refs = torch.from_numpy(wl.refs).to(dev)
    qs = torch.from_numpy(wl.queries).to(dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rs = nd.RefSet(refs, W)
    srch = nd.Searcher(rs, Q, V=V, cascade="keogh_enh", R=args.R, init_ub=True, cpl=args.cpl, waves=args.waves)

    def step(ev=None, stage_ev=None):
        if ev is not None:
            hip.record(ev[0], stream)
        rs.rebuild(refs)
        srch.set_events(stage_ev)
        out = srch(qs)
        if ev is not None:
            hip.record(ev[1], stream)
        return out

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    K = args.steps
    step_ev = [hip.events(2) for _ in range(K)]
    stage_ev = [hip.events(5) for _ in range(K)]
    torch.cuda.synchronize()
    # timed steps: nothing but the steps (an event recorded between kernels
    # costs the stream time of its own)
    t0 = time.perf_counter()
    for k in range(K):
        idx, dist, counts = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / K
    for k in range(K):
        step(step_ev[k])
    torch.cuda.synchronize()
    lat = sorted(hip.ms(e[0], e[1]) for e in step_ev)
    for k in range(K):
        step(None, stage_ev[k])
    torch.cuda.synchronize()
    st = {name: [hip.ms(e[i], e[i + 1]) for e in stage_ev] for i, name in
          enumerate(["bounds", "cells_prefix", "order", "search"])}
    st_avg = {k: sum(v) / len(v) for k, v in st.items()}

    c = counts.cpu().numpy()
    cells = int(c[:, 6].sum())
    started = int(c[:, 4].sum())
    pairs = N * Q
    # roofline of the dominant kernel: the search kernel, ALU-bound (3 useful
    # VALU lane operations per band cell it evaluates)
    cells_ops = 3.0 * cells
    t_search = st_avg["search"] / 1e3
    ach = cells_ops / t_search
    prof_us = profiled_kernel_us("search_kernel", wl.name)
    roof = {"kernel": "search_kernel", "bound": "alu", "achieved": ach / 1e12, "peak": VALU_PEAK_OPS / 1e12,
            "unit": "Tops/s", "frac": ach / VALU_PEAK_OPS,
            "traffic": profiled_traffic("search_kernel", wl.name),
            "kernel_avg_us_events": t_search * 1e6, "cells_per_launch": cells,
            "kernel_avg_us_rocprof": prof_us,
            "frac_rocprof": (cells_ops / (prof_us / 1e6) / VALU_PEAK_OPS) if prof_us else None}
    bytes_bounds = 12.0 * N * L * math.ceil(Q / 4) + 32.0 * Q * N
    res = {
        "metric": METRIC, "value": Q / (ms_step / 1e3), "unit": "queries/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "N": N, "Q": Q, "L": L, "W": W, "V": V, "cascade": "keogh_enh",
                   "R": srch.R, "cpl": srch.cpl, "waves_per_query": srch.waves, "init_ub": True},
        "roofline": roof,
        "dtw_cells_per_s": cells / (ms_step / 1e3),
        "search_kernel_cells_per_s": cells / t_search,
        "valu_frac_dtw": cells_ops / t_search / VALU_PEAK_OPS,
        "pruning_rate": 1.0 - started / pairs,
        "pruned": {"keogh": int(c[:, 1].sum()) / pairs, "enh_bands": int(c[:, 2].sum()) / pairs,
                   "enh": int(c[:, 3].sum()) / pairs},
        "dtw_started": started, "dtw_abandoned": int(c[:, 5].sum()), "fp64_rechecks": int(c[:, 7].sum()),
        "latency_ms": {"p50": lat[len(lat) // 2], "p99": lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)],
                       "max": lat[-1]},
        "stage_ms": st_avg,
        "bounds_kernel_gbps_algorithmic": bytes_bounds / (st_avg["bounds"] / 1e3) / 1e9,
    }
    if not headline:
        for k in ("metric", "n_gpus", "steps", "warmup", "higher_is_better", "scaling", "vs_baseline", "data"):
            res.pop(k)
    res["_refset"], res["_queries"] = rs, qs
    del srch
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--V", type=int, default=5)
    ap.add_argument("--R", type=int, default=0)
    ap.add_argument("--cpl", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the per-query arm and tightness")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the batching workload (defaults and autotuned), one JSON line each")
    ap.add_argument("--sweep-only", action="store_true",
                    help="only the window sweep and the comparison bounds, one JSON line")
    ap.add_argument("--windows-only", action="store_true", help="only the window sweep, one JSON line")
    ap.add_argument("--backward-only", action="store_true", help="only the DTW backward, one JSON line")
    ap.add_argument("--serving-only", action="store_true", help="only the serving loop, one JSON line")
    ap.add_argument("--one-request-only", action="store_true",
                    help="only the GPU time of one-request serving batches per set, one JSON line")
    ap.add_argument("--hbm-only", action="store_true",
                    help="only the streaming kernels on the 200,000 x 512 reference set, one JSON line")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="after timing, one plain device copy of this many MiB (memory-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(f"bench.py measures one GPU only (queries shard across GPUs with no exchange, reference sets "
              f"with one exchange of the per-shard minima per query); --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1808_09617_amd as nd
    import synth

    if args.batch_only:
        dev = torch.device("cuda:0")
        for tuned in (None, "auto"):
            print(json.dumps(batch_bench(nd, synth, torch, dev, tuned=tuned)), flush=True)
        return

    if args.windows_only:
        print(json.dumps({"window_sweep": window_sweep(nd, synth, torch, torch.device("cuda:0"))}), flush=True)
        return
    if args.one_request_only:
        from paper_1808_09617_amd import serve
        dev = torch.device("cuda:0")
        sets = synth.serving_sets()
        rss = [nd.RefSet(torch.from_numpy(refs).to(dev), W) for refs, W in sets]
        Ls = [refs.shape[1] for refs, _ in sets]
        # the round size, shape and helper workgroups the serving benchmark's
        # tuners pick on this workload
        R = [512, 512, 256, 256, 256, 256, 256, 256]
        cpl = [3, 3, 3, 2, 2, 2, 2, 2]
        helpers = [-1, -1, 0, 0, 0, 0, 0, 0]
        print(json.dumps({"one_request": one_request_latency(nd, synth, torch, dev, serve, rss, Ls, R, cpl,
                                                             helpers)}), flush=True)
        return
    if args.serving_only:
        print(json.dumps({"serving": serving_bench(nd, synth, torch, torch.device("cuda:0"))}), flush=True)
        return
    if args.backward_only:
        print(json.dumps({"backward": backward_bench(nd, synth, torch, torch.device("cuda:0"), cpu=False)}), flush=True)
        return

    if args.hbm_only:
        dev = torch.device("cuda:0")
        out = {"hbm_streaming": hbm_streaming(nd, synth, torch, dev)}
        if args.calib_copy_mb:
            src = torch.ones(args.calib_copy_mb * 2 ** 18, dtype=torch.float32, device=dev)
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
            out["calib_copy_bytes"] = src.numel() * 4
        print(json.dumps(out), flush=True)
        return

    if args.sweep_only:
        dev = torch.device("cuda:0")
        a, b = synth.tightness_pairs(250_000)
        print(json.dumps({"window_sweep": window_sweep(nd, synth, torch, dev),
                          "compare_bounds": compare_bounds(nd, synth, torch, dev, a, b)}), flush=True)
        return

    dev = torch.device("cuda:0")
    hip = Hip()
    wl = synth.workload("nndtw-mix512")
    W_head = int(math.floor(0.1 * wl.L + 0.5))           # W = round-half-up(0.1 L) = 51
    log(f"workload nndtw-mix512 W={W_head} V={args.V}")
    res = search_step_bench(nd, torch, hip, dev, wl, W_head, args.V, args, headline=True)
    log(f"timed {args.steps} steps")

    if not args.no_extras:
        V = args.V
        # the headline set searched one query per launch sequence (arm B:
        # plain per-query LB_Keogh -> DTW, no ED upper bound)
        rs, qs = res.pop("_refset"), res.pop("_queries")
        nq = 100
        one = nd.Searcher(rs, 1, V=V, cascade="keogh", R=0, init_ub=False)
        one(qs[:1])
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(nq):
            one(qs[i:i + 1])
        torch.cuda.synchronize()
        per_q = nq / (time.perf_counter() - t)
        res["per_query_keogh_qps"] = per_q
        res["speedup_vs_per_query_keogh"] = res["value"] / per_q
        res["arms_2x2"] = arms_2x2(nd, torch, rs, qs, V)
        del rs, qs, one
        torch.cuda.empty_cache()
        # the 1000 x 1000, L=256 class-sinusoid workload, measured as the headline
        c2 = synth.workload("nndtw-sin256")
        W = c2.windows[0]
        sub = search_step_bench(nd, torch, hip, dev, c2, W, V, args, headline=False)
        rs, qs = sub.pop("_refset"), sub.pop("_queries")
        sub["arms_2x2"] = arms_2x2(nd, torch, rs, qs, V)
        sub["per_v"] = per_v(nd, torch, rs, qs)
        res["nndtw_sin256"] = sub
        del rs, qs
        # LB tightness on independent class-sinusoid pairs (LB / DTW, un-rooted)
        a, b = synth.tightness_pairs(250_000)
        A, B = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
        U, Lo = nd.envelopes(B, W)
        d = nd.dtw_w(A, B, W, zip_=True).double()
        keep = d > 0
        tight = {"pairs": int(keep.sum()), "keogh": float((nd.lb_keogh(A, U, Lo, zip_=True)[keep] / d[keep]).mean())}
        for v in (1, 2, 5):
            tight[f"enhanced{v}"] = float((nd.lb_enhanced(A, B, U, Lo, W, v, zip_=True)[keep] / d[keep]).mean())
        res["tightness"] = tight
        res["small_latency"] = small_latency(nd, synth, torch, dev)
        log("arms, V and small-instance latency done")
        res["window_sweep"] = window_sweep(nd, synth, torch, dev)
        log("window sweep done")
        res["compare_bounds"] = compare_bounds(nd, synth, torch, dev, a, b, W)
        log("comparison bounds done")
        res["hbm_streaming"] = hbm_streaming(nd, synth, torch, dev)
        res["backward"] = backward_bench(nd, synth, torch, dev, cpu=not args.no_cpu)
        res["serving"] = serving_bench(nd, synth, torch, dev)
        res["batch"] = batch_bench(nd, synth, torch, dev)
        res["batch_tuned"] = batch_bench(nd, synth, torch, dev, tuned="auto")
        log("extras done")

    if args.calib_copy_mb:
        src = torch.ones(args.calib_copy_mb * 2 ** 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        res["calib_copy_bytes"] = src.numel() * 4

    res.pop("_refset", None)
    res.pop("_queries", None)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(wl, W_head, args.V, args.cpu_seconds)
        log("cpu baseline done")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
