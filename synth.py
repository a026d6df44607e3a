"""Seeded synthetic workloads for NN-DTW (stand-ins for the UCR archive).

The paper evaluates on the 85 UCR datasets (Section 4), which are not shipped
here; these generators produce series with the shapes, lengths and value
distributions of the evaluated workloads instead.  This module holds no part of
the method's arithmetic: it only draws numbers, z-normalises them and casts them
to float32 once.  Both the CPU oracle and the GPU path consume its arrays.

Families (all series z-normalised per series in float64, ddof=0, then float32):

* ``rw``   Gaussian random walk: x_1 ~ N(0,1), x_t = x_{t-1} + N(0,1).
* ``sin5`` five class prototypes, each the sum of three sinusoids with a
  frequency drawn uniformly in [1, 8] cycles per series and a phase uniform in
  [0, 2*pi); a series picks a class uniformly, adds N(0, 0.3^2) noise per point.
* ``mix``  exactly half ``rw`` and half ``sin5``, in a seeded permutation.

Seeds: ``numpy.random.SeedSequence([180809617, config_id, stream])`` with stream
0 = references, 1 = queries, 2 = tightness pairs, 3 = class prototypes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ROOT_SEED = 180809617
STREAM_REFS, STREAM_QUERIES, STREAM_PAIRS, STREAM_PROTOS = 0, 1, 2, 3


def rng_for(config_id: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([ROOT_SEED, config_id, stream]))


def znorm(x: np.ndarray) -> np.ndarray:
    """Per-row z-normalisation in float64 (ddof=0); constant rows become zeros."""
    x = np.asarray(x, dtype=np.float64)
    mu = x.mean(axis=-1, keepdims=True)
    sd = x.std(axis=-1, keepdims=True)
    out = np.zeros_like(x)
    np.divide(x - mu, sd, out=out, where=sd > 0)
    return out


def rw(n: int, L: int, rng: np.random.Generator) -> np.ndarray:
    steps = rng.standard_normal((n, L))
    return znorm(np.cumsum(steps, axis=1)).astype(np.float32)


def sin5_prototypes(L: int, rng: np.random.Generator, n_classes: int = 5) -> np.ndarray:
    t = np.arange(L, dtype=np.float64)
    freq = rng.uniform(1.0, 8.0, size=(n_classes, 3))
    phase = rng.uniform(0.0, 2.0 * math.pi, size=(n_classes, 3))
    arg = 2.0 * math.pi * freq[:, :, None] * t[None, None, :] / L + phase[:, :, None]
    return np.sin(arg).sum(axis=1)


def sin5(n: int, L: int, rng: np.random.Generator, protos: np.ndarray,
         noise: float = 0.3, return_labels: bool = False):
    labels = rng.integers(0, protos.shape[0], size=n)
    x = protos[labels] + noise * rng.standard_normal((n, L))
    out = znorm(x).astype(np.float32)
    return (out, labels) if return_labels else out


def mix(n: int, L: int, rng: np.random.Generator, protos: np.ndarray) -> np.ndarray:
    n_rw = n // 2
    parts = np.concatenate([rw(n_rw, L, rng), sin5(n - n_rw, L, rng, protos)], axis=0)
    return np.ascontiguousarray(parts[rng.permutation(n)])


def window_from_fraction(f: float, L: int) -> int:
    """W = round-half-up(f * L), clamped to L - 1 (W >= L - 1 is unconstrained)."""
    w = int(math.floor(f * L + 0.5))
    return min(w, L - 1)


@dataclass
class Workload:
    name: str
    refs: np.ndarray          # float32 [N][L]
    queries: np.ndarray       # float32 [Q][L]
    windows: list
    vs: list
    desc: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def L(self) -> int:
        return int(self.refs.shape[1])


def _family(kind: str, n: int, L: int, config_id: int, stream: int) -> np.ndarray:
    rng = rng_for(config_id, stream)
    if kind == "rw":
        return rw(n, L, rng)
    protos = sin5_prototypes(L, rng_for(config_id, STREAM_PROTOS))
    if kind == "sin5":
        return sin5(n, L, rng, protos)
    if kind == "mix":
        return mix(n, L, rng, protos)
    raise ValueError(kind)


def workload(name: str, n_refs: int | None = None, n_queries: int | None = None) -> Workload:
    """The evaluated configurations, optionally truncated to fewer series.

    nndtw-small   100 refs x 20 queries, L=64, random walks, W=6, V=1
    nndtw-sin256  1000 x 1000, L=256, sin5, W=26 (0.1 L), V in {1,2,5}
    nndtw-mix512  5000 x 500, L=512, mix, W in {0.01,0.1,0.25,0.5,1.0} L, V in {1,5}
    nndtw-hbm512  200000 refs, L=512, mix (streaming-kernel bandwidth only)
    """
    table = {
        "nndtw-small": (1, "rw", 100, 20, 64, [6], [1]),
        "nndtw-sin256": (2, "sin5", 1000, 1000, 256, [26], [1, 2, 5]),
        "nndtw-mix512": (3, "mix", 5000, 500, 512,
                         [window_from_fraction(f, 512) for f in (0.01, 0.1, 0.25, 0.5, 1.0)], [1, 5]),
        "nndtw-hbm512": (6, "mix", 200000, 64, 512, [51], [5]),
    }
    cid, kind, N, Q, L, ws, vs = table[name]
    N = N if n_refs is None else n_refs
    Q = Q if n_queries is None else n_queries
    refs = _family(kind, N, L, cid, STREAM_REFS)
    queries = _family(kind, Q, L, cid, STREAM_QUERIES)
    return Workload(name, refs, queries, ws, vs, desc=f"{kind} N={N} Q={Q} L={L}")


@dataclass
class BatchDataset:
    refs: np.ndarray          # float32 [N][L]
    queries: np.ndarray       # float32 [Q][L]
    W: int
    V: int

    @property
    def L(self) -> int:
        return self.refs.shape[1]


def batch_params(n_sets: int = 64, L_range=(24, 2048), N_range=(50, 8000), q_frac: float = 0.1,
                 w_frac: float = 0.1, config_id: int = 4):
    """(L, N, Q, W) of each dataset of the batching workload: L log-uniform in
    L_range (rounded), N uniform in N_range, Q = max(1, round(q_frac N)),
    W = round-half-up(w_frac L).  Drawn from stream 4 of the configuration."""
    rng = rng_for(config_id, 4)
    L = np.rint(np.exp(rng.uniform(math.log(L_range[0]), math.log(L_range[1]), n_sets))).astype(int)
    N = rng.integers(N_range[0], N_range[1] + 1, n_sets)
    Q = np.maximum(1, np.rint(q_frac * N)).astype(int)
    W = np.array([window_from_fraction(w_frac, int(l)) for l in L])
    return [(int(L[d]), int(N[d]), int(Q[d]), int(W[d])) for d in range(n_sets)]


def batch_workload(n_sets: int = 64, L_range=(24, 2048), N_range=(50, 8000), q_frac: float = 0.1,
                   w_frac: float = 0.1, V: int = 5, config_id: int = 4) -> list:
    """The batching workload: independent random-walk datasets of ragged
    lengths (64 sets, L log-uniform in [24, 2048], N uniform in [50, 8000],
    Q = 0.1 N, W = 0.1 L, V = 5 by default).  Dataset d draws its references
    and queries from SeedSequence([180809617, config_id, 100 + d, stream])."""
    out = []
    for d, (L, N, Q, W) in enumerate(batch_params(n_sets, L_range, N_range, q_frac, w_frac, config_id)):
        rr = np.random.default_rng(np.random.SeedSequence([ROOT_SEED, config_id, 100 + d, STREAM_REFS]))
        rq = np.random.default_rng(np.random.SeedSequence([ROOT_SEED, config_id, 100 + d, STREAM_QUERIES]))
        out.append(BatchDataset(rw(N, L, rr), rw(Q, L, rq), W, V))
    return out


def serving_sets(n_sets: int = 8, n_refs: int = 4000, L_range=(64, 1024), w_frac: float = 0.1,
                 config_id: int = 5):
    """Reference sets of the serving workload: set s has the fixed length
    L_s = round(L_lo + (L_hi - L_lo) s / (n_sets - 1)) (equal lengths within
    a set), n_refs random walks, W = round-half-up(w_frac L_s); drawn from
    SeedSequence([180809617, config_id, 200 + s, 0])."""
    out = []
    for s in range(n_sets):
        L = int(round(L_range[0] + (L_range[1] - L_range[0]) * s / max(1, n_sets - 1)))
        rng = np.random.default_rng(np.random.SeedSequence([ROOT_SEED, config_id, 200 + s, STREAM_REFS]))
        out.append((rw(n_refs, L, rng), window_from_fraction(w_frac, L)))
    return out


def serving_query(set_id: int, L: int, k: int, config_id: int = 5) -> np.ndarray:
    """Request k's query (a random walk of the set's length)."""
    rng = np.random.default_rng(np.random.SeedSequence([ROOT_SEED, config_id, 300 + k, set_id]))
    return rw(1, L, rng)[0]


def tightness_pairs(n_pairs: int = 250_000, L: int = 256, config_id: int = 2):
    """Independent sin5 pairs (A_k, B_k) for LB/DTW tightness (Figure 1 workload shape)."""
    rng = rng_for(config_id, STREAM_PAIRS)
    protos = sin5_prototypes(L, rng_for(config_id, STREAM_PROTOS))
    a = sin5(n_pairs, L, rng, protos)
    b = sin5(n_pairs, L, rng, protos)
    return a, b


def random_series(n: int, L: int, seed: int, kind: str = "rw") -> np.ndarray:
    """Small ad-hoc inputs for tests (seeded, z-normalised float32)."""
    rng = np.random.default_rng(np.random.SeedSequence([ROOT_SEED, 1000 + seed, L]))
    if kind == "rw":
        return rw(n, L, rng)
    if kind == "normal":
        return znorm(rng.standard_normal((n, L))).astype(np.float32)
    if kind == "sin5":
        protos = sin5_prototypes(L, rng)
        return sin5(n, L, rng, protos)
    raise ValueError(kind)
