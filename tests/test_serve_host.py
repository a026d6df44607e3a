"""Host logic of the serving loop (CPU): the device-wide workspace arena and
the seeded request stream.  The arena is exercised over a CPU buffer; the
serving loop itself (streams, events, batched searches) is covered by the
GPU tests."""
import numpy as np
import pytest
import torch

from paper_1808_09617_amd import serve


def test_arena_first_fit_alignment_and_coalescing():
    a = serve.Arena(10 * 256 + 100, "cpu")
    assert a.size == 10 * 256                      # whole 256-byte units only
    b1 = a.alloc(1)                                # rounded up to one unit
    b2 = a.alloc(257)                              # two units
    b3 = a.alloc(256)
    assert b1 == (0, 256) and b2 == (256, 512) and b3 == (768, 256)
    assert a.used == 1024
    a.free(b2)
    assert a.free_blocks == [(256, 512), (1024, 1536)]
    # first fit: a one-unit request takes the hole left by b2
    b4 = a.alloc(200)
    assert b4 == (256, 256)
    a.free(b1)
    a.free(b4)                                     # coalesces with b1's block and the rest of the hole
    assert a.free_blocks == [(0, 768), (1024, 1536)]
    a.free(b3)                                     # everything free again: one block
    assert a.free_blocks == [(0, 2560)] and a.used == 0
    assert a.alloc(2561) is None                   # larger than the arena
    assert a.alloc(2560) == (0, 2560) and a.alloc(1) is None


def test_arena_random_sequence_never_overlaps():
    rng = np.random.default_rng(7)
    a = serve.Arena(64 * 256, "cpu")
    live = []
    for _ in range(2000):
        if live and (rng.random() < 0.45 or len(live) > 40):
            blk = live.pop(int(rng.integers(len(live))))
            a.free(blk)
        else:
            blk = a.alloc(int(rng.integers(1, 6 * 256)))
            if blk is not None:
                live.append(blk)
        # invariants: aligned, inside the arena, disjoint, and the free list
        # sorted, coalesced and complementary to the live blocks
        spans = sorted(live + a.free_blocks)
        assert all(o % 256 == 0 and n % 256 == 0 and n > 0 for o, n in spans)
        pos = 0
        for o, n in spans:
            assert o == pos
            pos += n
        assert pos == a.size
        fb = a.free_blocks
        assert all(fb[k][0] + fb[k][1] < fb[k + 1][0] for k in range(len(fb) - 1))
        assert a.used == sum(n for _, n in live)


def test_arena_pointer_offsets():
    a = serve.Arena(4 * 256, "cpu")
    off, n = a.alloc(300)
    assert a.ptr(off).value == a.buf.data_ptr() + off


@pytest.mark.parametrize("rate", [500.0, 4000.0])
def test_poisson_requests_seeded_and_ordered(rate):
    Ls = [16, 32, 48]
    mk = lambda s, L, k: np.full(L, float(k), dtype=np.float32)
    r1 = serve.poisson_requests(Ls, rate=rate, duration=0.5, seed=3, device="cpu", make_query=mk)
    r2 = serve.poisson_requests(Ls, rate=rate, duration=0.5, seed=3, device="cpu", make_query=mk)
    t = np.array([r.arrival for r in r1])
    assert len(r1) == len(r2) and np.array_equal(t, [r.arrival for r in r2])
    assert np.all(np.diff(t) > 0) and t[-1] <= 0.5
    # a Poisson count over 0.5 s: mean rate / 2, within 5 standard deviations
    mean = rate * 0.5
    assert abs(len(r1) - mean) < 5 * mean ** 0.5
    for k, r in enumerate(r1):
        assert r.rid == k and 0 <= r.set_id < len(Ls)
        assert r.query.shape == (Ls[r.set_id],) and float(r.query[0]) == k
    assert {r.set_id for r in r1} == {0, 1, 2}


def test_poisson_requests_saturation_mode():
    mk = lambda s, L, k: np.zeros(L, dtype=np.float32)
    reqs = serve.poisson_requests([8, 8], rate=float("inf"), duration=37, seed=1, device="cpu", make_query=mk)
    assert len(reqs) == 37 and all(r.arrival == 0.0 for r in reqs)
    assert [r.rid for r in reqs] == list(range(37))


def test_server_helpers_per_batch():
    """A batch runs without helper workgroups only when every set in it asks
    for none; otherwise with the most any of its sets asks for (0, the
    library default, counting as 7)."""
    srv = serve.Server.__new__(serve.Server)          # the resolution only, no device state
    srv.set_helpers = [-1, -1, 0, 3, 5, -1]
    assert srv._helpers([0]) == -1 and srv._helpers([0, 1, 5]) == -1
    assert srv._helpers([3]) == 3 and srv._helpers([0, 3]) == 3 and srv._helpers([3, 4]) == 5
    assert srv._helpers([2]) == 0 and srv._helpers([2, 4]) == 0 and srv._helpers([1, 2, 3]) == 0
