"""nndtw_search_noalloc (the search with the library's fixed device
workspace) against nndtw_search with a caller workspace: identical results on
two calls in a row, the second one smaller, and the size limit enforced on
the host."""
import ctypes
import sys

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1808_09617_amd as nd  # noqa: E402

DEV = torch.device("cuda:0")


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _both(refs, queries, W, V, R=0):
    rs = nd.RefSet(torch.from_numpy(refs).to(DEV), W)
    Q = torch.from_numpy(queries).to(DEV)
    nq = Q.shape[0]
    idx = torch.full((nq,), -5, dtype=torch.int64, device=DEV)
    dist = torch.full((nq,), -5.0, dtype=torch.float64, device=DEV)
    counts = torch.full((nq, 8), -5, dtype=torch.int64, device=DEV)
    R_na = nd.search_noalloc(rs, Q, idx, dist, counts, V=V, R=R)
    gi, gd, gc = _host(idx), _host(dist), _host(counts)
    si, sd, sc, R_s = nd.search(rs, Q, V=V, R=R)
    si, sd, sc = _host(si), _host(sd), _host(sc)
    assert R_na == R_s
    assert np.array_equal(gi, si) and np.array_equal(gd, sd), ("results", np.nonzero(gi != si))
    assert np.array_equal(gc[:, :5], sc[:, :5])
    # implementation-defined counts: consistent (their values depend on which
    # DTW of a round ends first)
    assert np.all(gc[:, 5] <= gc[:, 4]) and np.all(gc[:, 6] >= 0) and np.all(gc[:, 7] >= (gc[:, 4] > 0))
    return rs


def test_search_noalloc_matches_search_twice():
    big = synth.workload("nndtw-sin256", n_refs=1000, n_queries=600)      # 36 MB of workspace
    say("noalloc call 1", big.refs.shape, big.queries.shape)
    _both(big.refs, big.queries, 26, 5)
    small = synth.workload("nndtw-small")                                 # 100 x 20, L=64
    say("noalloc call 2", small.refs.shape, small.queries.shape)
    rs = _both(small.refs, small.queries, 6, 1)
    say("noalloc call 3 (R=1)", small.refs.shape, small.queries[:7].shape)
    _both(small.refs, np.ascontiguousarray(small.queries[:7]), 6, 2, R=1)
    # beyond the fixed array: rejected on the host, nothing enqueued
    Q = torch.zeros((nd.SEARCH_SCRATCH_BYTES // (60 * rs.n) + 10, rs.L), dtype=torch.float32, device=DEV)
    out_i = torch.empty(Q.shape[0], dtype=torch.int64, device=DEV)
    out_d = torch.empty(Q.shape[0], dtype=torch.float64, device=DEV)
    with pytest.raises(nd.NNDTWError) as e:
        nd.search_noalloc(rs, Q, out_i, out_d, None, V=1)
    assert e.value.status == nd.EUNSUP and "NNDTW_SEARCH_SCRATCH_BYTES" in str(e.value)
    # an empty call is valid and enqueues nothing
    nd.search_noalloc(rs, Q[:0], out_i[:0], out_d[:0], None, V=1)
    torch.cuda.synchronize()
