"""MI355X (gfx950) nearest-neighbour search under window-constrained DTW with
the LB_Keogh / LB_Enhanced^V lower-bound cascade of Tan, Petitjean & Webb,
"Elastic bands across the path: A new framework and method to lower bound DTW".

This module is argument marshalling only: every computation runs in the HIP
kernels of ``libnndtw.so`` (C ABI declared in ``include/nndtw.h``).  Tensors
are torch CUDA tensors on the current device; work is enqueued on torch's
current stream.  If the library is missing, every call raises: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
# NNDTW_LIB selects another build of the same library (the host-sanitized
# build of the CPU sanitizer test); the default is the in-tree build.
LIB_PATH = os.environ.get("NNDTW_LIB") or os.path.join(PKG, "libnndtw.so")

OK, EINVAL, EHIP, EUNSUP = 0, -1, -2, -3
CROSS, ZIP = 0, 1
CASCADES = {"none": 0, "keogh": 1, "keogh_enh": 2, "enh": 3,
            "kim": 4, "improved": 5, "new": 6, "enh_sym": 7}
ENGINES = {"auto": 0, "diagonal": 1, "strip": 2}
ORDERS = {"auto": 0, "sort": 1, "rank": 2}
COUNT_NAMES = ("n", "pruned_keogh", "pruned_enh_bands", "pruned_enh", "dtw_started",
               "dtw_abandoned", "cells", "fp64_rechecks")
MAX_L = 2048
BATCH_MAX_N = 8192
SEARCH_MAX_WAVES = 16
SEARCH_MAX_HELPERS = 7
SEARCH_SCRATCH_BYTES = 64 << 20
REFSET_MAGIC = 0x4E444157


class NNDTWError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"nndtw status {status}: {msg}")
        self.status = status


class _Refset(ctypes.Structure):
    _fields_ = [("magic", ctypes.c_uint32), ("L", ctypes.c_int32), ("n", ctypes.c_int64),
                ("W", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("pitch", ctypes.c_int64),
                ("B", ctypes.c_void_p), ("U", ctypes.c_void_p), ("Lo", ctypes.c_void_p),
                ("Bt", ctypes.c_void_p), ("Ut", ctypes.c_void_p), ("Lt", ctypes.c_void_p),
                ("Bp", ctypes.c_void_p), ("ppitch", ctypes.c_int64), ("padl", ctypes.c_int32),
                ("reserved1", ctypes.c_int32)]


class _SearchOpts(ctypes.Structure):
    _fields_ = [("V", ctypes.c_int32), ("cascade", ctypes.c_int32), ("R", ctypes.c_int64),
                ("eps", ctypes.c_double), ("init_ub", ctypes.c_int32), ("cpl", ctypes.c_int32),
                ("events", ctypes.c_void_p), ("waves", ctypes.c_int32), ("engine", ctypes.c_int32),
                ("nq_hint", ctypes.c_int64), ("helpers", ctypes.c_int32), ("order", ctypes.c_int32)]


class _BatchSet(ctypes.Structure):
    _fields_ = [("refset", ctypes.c_void_p), ("Q", ctypes.c_void_p), ("nQ", ctypes.c_int64),
                ("nn_idx", ctypes.c_void_p), ("nn_dist", ctypes.c_void_p), ("counts", ctypes.c_void_p),
                ("R", ctypes.c_int64), ("cpl", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _BatchPlan(ctypes.Structure):
    _fields_ = [("magic", ctypes.c_uint32), ("nsets", ctypes.c_int32), ("items", ctypes.c_int64),
                ("tiles", ctypes.c_int64), ("waves", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("lds", ctypes.c_int64), ("ws_bytes", ctypes.c_int64), ("order_off", ctypes.c_int64 * 6),
                ("order_cnt", ctypes.c_int64 * 6), ("search_off", ctypes.c_int64 * 8),
                ("search_cnt", ctypes.c_int64 * 8), ("reserved", ctypes.c_int64 * 4),
                ("helpers", ctypes.c_int32), ("share_shapes", ctypes.c_uint32), ("share_off", ctypes.c_int64),
                ("order_rank", ctypes.c_int32), ("order_nmax", ctypes.c_int32)]


_P, _I32, _I64, _D, _SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
SIGNATURES = {
    "nndtw_version": (ctypes.c_int, []),
    "nndtw_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "nndtw_last_error": (ctypes.c_char_p, []),
    "nndtw_envelopes": (ctypes.c_int, [_P, _I64, _I32, _I32, _P, _P, _P]),
    "nndtw_ed2": (ctypes.c_int, [_P, _I64, _P, _I64, _I32, _I32, _P, _P]),
    "nndtw_lb_keogh": (ctypes.c_int, [_P, _I64, _P, _P, _I64, _I32, _I32, _P, _P]),
    "nndtw_lb_enhanced": (ctypes.c_int, [_P, _I64, _P, _P, _P, _I64, _I32, _I32, _I32, _P, _I32, _P, _P]),
    "nndtw_lb_kim": (ctypes.c_int, [_P, _I64, _P, _I64, _I32, _I32, _P, _P]),
    "nndtw_lb_improved": (ctypes.c_int, [_P, _I64, _P, _P, _P, _I64, _I32, _I32, _P, _I32, _P, _P]),
    "nndtw_lb_new": (ctypes.c_int, [_P, _I64, _P, _I64, _I32, _I32, _I32, _P, _P]),
    "nndtw_lb_enhanced_sym": (ctypes.c_int, [_P, _I64, _P, _P, _P, _I64, _I32, _I32, _I32, _I32, _P, _P]),
    "nndtw_dtw_w": (ctypes.c_int, [_P, _I64, _P, _I64, _I32, _I32, _P, _I32, _P, _P]),
    "nndtw_dtw_w_f64": (ctypes.c_int, [_P, _I64, _P, _I64, _I32, _I32, _P, _I32, _P, _P]),
    "nndtw_dtw_codes_bytes": (ctypes.c_int, [_I64, _I64, _I32, _I32, _I32, ctypes.POINTER(_SZ)]),
    "nndtw_dtw_w_codes": (ctypes.c_int, [_P, _I64, _P, _I64, _I32, _I32, _I32, _I32, _P, _P, _SZ, _P]),
    "nndtw_dtw_w_backward": (ctypes.c_int, [_P, _I64, _P, _I64, _I32, _I32, _I32, _I32, _P, _P, _SZ, _P, _P]),
    "nndtw_refset_bytes": (ctypes.c_int, [_I64, _I32, _I32, ctypes.POINTER(_SZ)]),
    "nndtw_refset_build": (ctypes.c_int, [_P, _I64, _I32, _I32, _P, _SZ, ctypes.POINTER(_Refset), _P]),
    "nndtw_search_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(_Refset), _I64,
                                                    ctypes.POINTER(_SearchOpts), ctypes.POINTER(_SZ)]),
    "nndtw_search": (ctypes.c_int, [ctypes.POINTER(_Refset), _P, _I64, ctypes.POINTER(_SearchOpts), _P, _P,
                                    _P, _P, _SZ, _P]),
    "nndtw_search_plan": (ctypes.c_int, [ctypes.POINTER(_Refset), ctypes.POINTER(_SearchOpts)]),
    "nndtw_search_noalloc": (ctypes.c_int, [ctypes.POINTER(_Refset), _P, _I64, ctypes.POINTER(_SearchOpts), _P, _P,
                                            _P, _P]),
    "nndtw_cascade_bounds": (ctypes.c_int, [ctypes.POINTER(_Refset), _P, _I64, _I32, _P, _P, _P, _P, _P]),
    "nndtw_batch_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(_BatchSet), _I32, ctypes.POINTER(_SearchOpts),
                                                   ctypes.POINTER(_SZ)]),
    "nndtw_batch_prepare": (ctypes.c_int, [ctypes.POINTER(_BatchSet), _I32, ctypes.POINTER(_SearchOpts), _P, _SZ,
                                           ctypes.POINTER(_BatchPlan), _P]),
    "nndtw_search_batch": (ctypes.c_int, [ctypes.POINTER(_BatchPlan), _P, _P]),
}

_lib = None


def lib():
    """Load libnndtw.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                              "g.build()'` (hipcc for gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().nndtw_last_error().decode()


def _check(status: int):
    if status != OK:
        raise NNDTWError(status, last_error())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _series(x: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if x.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if x.dim() == 1:
        x = x.unsqueeze(0)
    if x.dim() != 2:
        raise ValueError(f"{name} must be [n][L]")
    return x.contiguous()


def _ptr(x):
    return ctypes.c_void_p(x.data_ptr()) if x is not None and x.numel() > 0 else ctypes.c_void_p(0)


def _cutoff(cutoff, n, device):
    if cutoff is None:
        return None
    c = torch.as_tensor(cutoff, dtype=torch.float64, device=device)
    return c.expand(n).contiguous() if c.dim() == 0 else c.contiguous()


def _pair_shape(nA, nB, zip_):
    if zip_ and nA != nB:
        raise ValueError("zip pairing needs equal counts")
    return (nA,) if zip_ else (nA, nB)


def envelopes(B: torch.Tensor, W: int):
    """Equations (3)-(4): upper/lower envelopes of every row of B (float32)."""
    B = _series(B, "B")
    U, Lo = torch.empty_like(B), torch.empty_like(B)
    _check(lib().nndtw_envelopes(_ptr(B), B.shape[0], B.shape[1], int(W), _ptr(U), _ptr(Lo), _stream()))
    return U, Lo


def ed2(A, B, zip_: bool = False):
    A, B = _series(A, "A"), _series(B, "B")
    out = torch.empty(_pair_shape(A.shape[0], B.shape[0], zip_), dtype=torch.float64, device=A.device)
    _check(lib().nndtw_ed2(_ptr(A), A.shape[0], _ptr(B), B.shape[0], A.shape[1], int(zip_), _ptr(out), _stream()))
    return out


def lb_keogh(A, U, Lo, zip_: bool = False):
    A, U, Lo = _series(A, "A"), _series(U, "U"), _series(Lo, "Lo")
    out = torch.empty(_pair_shape(A.shape[0], U.shape[0], zip_), dtype=torch.float64, device=A.device)
    _check(lib().nndtw_lb_keogh(_ptr(A), A.shape[0], _ptr(U), _ptr(Lo), U.shape[0], A.shape[1], int(zip_),
                                _ptr(out), _stream()))
    return out


def lb_enhanced(A, B, U, Lo, W: int, V: int, cutoff=None, zip_: bool = False):
    A, B, U, Lo = _series(A, "A"), _series(B, "B"), _series(U, "U"), _series(Lo, "Lo")
    out = torch.empty(_pair_shape(A.shape[0], B.shape[0], zip_), dtype=torch.float64, device=A.device)
    cut = _cutoff(cutoff, A.shape[0], A.device)
    _check(lib().nndtw_lb_enhanced(_ptr(A), A.shape[0], _ptr(B), _ptr(U), _ptr(Lo), B.shape[0], A.shape[1],
                                   int(W), int(V), _ptr(cut), int(zip_), _ptr(out), _stream()))
    return out


def lb_kim(A, B, zip_: bool = False):
    """LB_Kim, sum of the corner, minimum and maximum features without repetitions."""
    A, B = _series(A, "A"), _series(B, "B")
    out = torch.empty(_pair_shape(A.shape[0], B.shape[0], zip_), dtype=torch.float64, device=A.device)
    _check(lib().nndtw_lb_kim(_ptr(A), A.shape[0], _ptr(B), B.shape[0], A.shape[1], int(zip_), _ptr(out),
                              _stream()))
    return out


def lb_improved(A, B, U, Lo, W: int, cutoff=None, zip_: bool = False):
    """LB_Improved = LB_Keogh(A, B) + LB_Keogh(B, A'); +inf where LB_Keogh(A, B) > cutoff."""
    A, B, U, Lo = _series(A, "A"), _series(B, "B"), _series(U, "U"), _series(Lo, "Lo")
    out = torch.empty(_pair_shape(A.shape[0], B.shape[0], zip_), dtype=torch.float64, device=A.device)
    cut = _cutoff(cutoff, A.shape[0], A.device)
    _check(lib().nndtw_lb_improved(_ptr(A), A.shape[0], _ptr(B), _ptr(U), _ptr(Lo), B.shape[0], A.shape[1],
                                   int(W), _ptr(cut), int(zip_), _ptr(out), _stream()))
    return out


def lb_new(A, B, W: int, zip_: bool = False):
    """LB_New: corner costs plus, per interior point, the nearest value of B in its window."""
    A, B = _series(A, "A"), _series(B, "B")
    out = torch.empty(_pair_shape(A.shape[0], B.shape[0], zip_), dtype=torch.float64, device=A.device)
    _check(lib().nndtw_lb_new(_ptr(A), A.shape[0], _ptr(B), B.shape[0], A.shape[1], int(W), int(zip_),
                              _ptr(out), _stream()))
    return out


def lb_enhanced_sym(A, B, U, Lo, W: int, V: int, zip_: bool = False):
    """max(LB_Enhanced^V(A, B), LB_Enhanced^V(B, A)); U, Lo are B's envelopes."""
    A, B, U, Lo = _series(A, "A"), _series(B, "B"), _series(U, "U"), _series(Lo, "Lo")
    out = torch.empty(_pair_shape(A.shape[0], B.shape[0], zip_), dtype=torch.float64, device=A.device)
    _check(lib().nndtw_lb_enhanced_sym(_ptr(A), A.shape[0], _ptr(B), _ptr(U), _ptr(Lo), B.shape[0], A.shape[1],
                                       int(W), int(V), int(zip_), _ptr(out), _stream()))
    return out


def dtw_w(A, B, W: int, cutoff=None, zip_: bool = False, f64: bool = False):
    """DTW_W (un-rooted), FP32 (default) or FP64; +inf where abandoned above cutoff."""
    A, B = _series(A, "A"), _series(B, "B")
    dt = torch.float64 if f64 else torch.float32
    out = torch.empty(_pair_shape(A.shape[0], B.shape[0], zip_), dtype=dt, device=A.device)
    cut = _cutoff(cutoff, A.shape[0], A.device)
    fn = lib().nndtw_dtw_w_f64 if f64 else lib().nndtw_dtw_w
    _check(fn(_ptr(A), A.shape[0], _ptr(B), B.shape[0], A.shape[1], int(W), _ptr(cut), int(zip_), _ptr(out),
              _stream()))
    return out


def dtw_w_codes(A, B, W: int, zip_: bool = False, f64: bool = False):
    """Forward DTW_W (no abandoning) plus the predecessor codes of every band
    cell, for dtw_w_backward.  Returns (distances, codes uint8 tensor)."""
    A, B = _series(A, "A"), _series(B, "B")
    nA, nB, L = A.shape[0], B.shape[0], A.shape[1]
    nbytes = ctypes.c_size_t(0)
    _check(lib().nndtw_dtw_codes_bytes(nA, nB, L, int(W), int(zip_), ctypes.byref(nbytes)))
    codes = torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=A.device)
    out = torch.empty(_pair_shape(nA, nB, zip_), dtype=torch.float64 if f64 else torch.float32, device=A.device)
    _check(lib().nndtw_dtw_w_codes(_ptr(A), nA, _ptr(B), nB, L, int(W), int(zip_), int(f64), _ptr(out),
                                   _ptr(codes), codes.numel(), _stream()))
    return out, codes


def dtw_w_backward(A, B, W: int, gout, codes, zip_: bool = False, f64: bool = False):
    """Gradient with respect to A: gA[a] = sum over pairs (a, b) of
    gout[pair] * dDTW_W(a, b)/dA_a along the minimising warping path."""
    A, B = _series(A, "A"), _series(B, "B")
    dt = torch.float64 if f64 else torch.float32
    g = gout.to(dt).contiguous()
    if tuple(g.shape) != _pair_shape(A.shape[0], B.shape[0], zip_):
        raise ValueError("gout has the wrong shape")
    gA = torch.empty(A.shape, dtype=dt, device=A.device)
    _check(lib().nndtw_dtw_w_backward(_ptr(A), A.shape[0], _ptr(B), B.shape[0], A.shape[1], int(W), int(zip_),
                                      int(f64), _ptr(g), _ptr(codes), codes.numel(), _ptr(gA), _stream()))
    return gA


class DTWFunction(torch.autograd.Function):
    """DTW_W(A, B) with its gradient with respect to the queries A (the
    references B get none).  ``dtw(A, B, W)`` = DTWFunction.apply(A, B, W, zip_, f64)."""

    @staticmethod
    def forward(ctx, A, B, W, zip_=False, f64=False):
        out, codes = dtw_w_codes(A.detach(), B.detach(), W, zip_, f64)
        ctx.save_for_backward(A, B)
        ctx.codes, ctx.W, ctx.zip_, ctx.f64 = codes, W, zip_, f64
        return out

    @staticmethod
    def backward(ctx, gout):
        A, B = ctx.saved_tensors
        gA = dtw_w_backward(A.detach(), B.detach(), ctx.W, gout, ctx.codes, ctx.zip_, ctx.f64)
        return gA.to(A.dtype), None, None, None, None


def dtw(A, B, W: int, zip_: bool = False, f64: bool = False):
    """Differentiable DTW_W (gradient with respect to A)."""
    return DTWFunction.apply(A, B, W, zip_, f64)


class RefSet:
    """A reference (training) set with envelopes for window W, resident in HBM."""

    def __init__(self, B: torch.Tensor, W: int):
        B = _series(B, "B")
        n, L = B.shape
        nbytes = ctypes.c_size_t(0)
        _check(lib().nndtw_refset_bytes(n, L, int(W), ctypes.byref(nbytes)))
        self.mem = torch.empty(int(nbytes.value), dtype=torch.uint8, device=B.device)
        self.desc = _Refset()
        _check(lib().nndtw_refset_build(_ptr(B), n, L, int(W), _ptr(self.mem), nbytes.value,
                                        ctypes.byref(self.desc), _stream()))
        self.n, self.L, self.W = n, L, int(W)
        self.device = B.device

    def rebuild(self, B: torch.Tensor):
        """Rebuild the set in place from new series of the same shape (no allocation)."""
        B = _series(B, "B")
        if tuple(B.shape) != (self.n, self.L):
            raise ValueError("rebuild needs the same [n][L] shape")
        _check(lib().nndtw_refset_build(_ptr(B), self.n, self.L, self.W, _ptr(self.mem), self.mem.numel(),
                                        ctypes.byref(self.desc), _stream()))

    def _view(self, attr, shape):
        """A tensor view of one array of the set (for tests)."""
        off = getattr(self.desc, attr) - self.mem.data_ptr()
        count = 1
        for s in shape:
            count *= s
        return self.mem[off:off + 4 * count].view(torch.float32).view(*shape)

    @property
    def U(self):
        return self._view("U", (self.n, self.L))

    @property
    def Lo(self):
        return self._view("Lo", (self.n, self.L))

    @property
    def B(self):
        return self._view("B", (self.n, self.L))

    def transposed(self, which: str):
        return self._view(which, (self.L, self.desc.pitch))[:, : self.n]


def _opts(V, cascade, R, eps, init_ub, cpl, waves=0, engine="auto", helpers=0, order="auto"):
    o = _SearchOpts()
    o.V, o.cascade, o.R, o.eps = int(V), CASCADES[cascade], int(R), float(eps)
    o.init_ub, o.cpl, o.waves, o.engine = int(bool(init_ub)), int(cpl), int(waves), ENGINES[engine]
    o.helpers = int(helpers)
    o.order = ORDERS[order] if isinstance(order, str) else int(order)
    return o


class Searcher:
    """Preallocated workspace for repeated nndtw_search calls on one RefSet."""

    def __init__(self, refset: RefSet, nQ: int, V: int = 5, cascade: str = "keogh_enh", R: int = 0,
                 eps: float = 0.0, init_ub: bool = True, cpl: int = 0, waves: int = 0, engine: str = "auto",
                 helpers: int = 0, order: str = "auto"):
        self.refset = refset
        self.nQ = int(nQ)
        self.opts = _opts(V, cascade, R, eps, init_ub, cpl, waves, engine, helpers, order)
        nbytes = ctypes.c_size_t(0)
        _check(lib().nndtw_search_workspace_bytes(ctypes.byref(refset.desc), self.nQ, ctypes.byref(self.opts),
                                                  ctypes.byref(nbytes)))
        dev = refset.device
        self.ws = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=dev)
        self.idx = torch.empty(self.nQ, dtype=torch.int64, device=dev)
        self.dist = torch.empty(self.nQ, dtype=torch.float64, device=dev)
        self.counts = torch.empty((self.nQ, 8), dtype=torch.int64, device=dev)

    def set_events(self, events_array):
        """Pass a ctypes array of 5 hipEvent_t recorded around the search stages (None: off)."""
        self._events = events_array
        self.opts.events = ctypes.cast(events_array, ctypes.c_void_p) if events_array is not None else None

    def __call__(self, Q: torch.Tensor):
        Q = _series(Q, "Q")
        if Q.shape[0] != self.nQ or Q.shape[1] != self.refset.L:
            raise ValueError(f"queries must be [{self.nQ}][{self.refset.L}]")
        _check(lib().nndtw_search(ctypes.byref(self.refset.desc), _ptr(Q), self.nQ, ctypes.byref(self.opts),
                                  _ptr(self.idx), _ptr(self.dist), _ptr(self.counts), _ptr(self.ws),
                                  self.ws.numel(), _stream()))
        return self.idx, self.dist, self.counts

    @property
    def R(self):
        return int(self.opts.R)

    @property
    def cpl(self):
        return int(self.opts.cpl)

    @property
    def waves(self):
        return int(self.opts.waves)

    @property
    def helpers(self):
        """Helper workgroups per query of the last call (0: none)."""
        return max(0, int(self.opts.helpers))

    @property
    def engine(self):
        """The DTW engine of the last call: "diagonal" or "strip"."""
        return {v: k for k, v in ENGINES.items()}[int(self.opts.engine)]


class BatchSearcher:
    """A prepared batched search over several reference sets (ragged lengths).

    ``sets`` is a list of (RefSet, queries) pairs; ``R`` and ``cpl`` are None
    (library defaults) or one value per set.  Calling the object runs the
    whole batch on the current stream (no allocation or copy, so it can be
    captured in a CUDA/HIP graph) and returns per set (nn_idx, nn_dist, counts).
    Each set's result equals ``search`` on that set with the R and cpl
    reported in ``self.R`` / ``self.cpl``.  ``helpers``: the most idle
    workgroups that may join one query at a search kernel's end (0 = the
    library default, -1 = none); ``order``: "auto", "sort" or "rank", how the
    visiting orders are found.  The result depends on neither."""

    def __init__(self, sets, V: int = 5, cascade: str = "keogh_enh", R=None, cpl=None, eps: float = 0.0,
                 init_ub: bool = True, waves: int = 0, helpers: int = 0, order: str = "auto"):
        n = len(sets)
        if n == 0:
            raise ValueError("empty batch")
        self.refsets = [rs for rs, _ in sets]
        self.Qs = [_series(Q, "Q") for _, Q in sets]
        dev = self.refsets[0].device
        self.out = []
        arr = (_BatchSet * n)()
        for d, (rs, Q) in enumerate(zip(self.refsets, self.Qs)):
            if Q.shape[1] != rs.L:
                raise ValueError(f"set {d}: queries of length {Q.shape[1]} against a reference set of length {rs.L}")
            nq = Q.shape[0]
            o = (torch.empty(nq, dtype=torch.int64, device=dev), torch.empty(nq, dtype=torch.float64, device=dev),
                 torch.empty((nq, 8), dtype=torch.int64, device=dev))
            self.out.append(o)
            b = arr[d]
            b.refset = ctypes.addressof(rs.desc)
            b.Q, b.nQ = _ptr(Q), nq
            b.nn_idx, b.nn_dist, b.counts = _ptr(o[0]), _ptr(o[1]), _ptr(o[2])
            b.R = 0 if R is None else int(R[d])
            b.cpl = 0 if cpl is None else int(cpl[d])
        self.sets = arr
        self.opts = _opts(V, cascade, 0, eps, init_ub, 0, waves, helpers=helpers, order=order)
        nbytes = ctypes.c_size_t(0)
        _check(lib().nndtw_batch_workspace_bytes(arr, n, ctypes.byref(self.opts), ctypes.byref(nbytes)))
        self.ws = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=dev)
        self.plan = _BatchPlan()
        _check(lib().nndtw_batch_prepare(arr, n, ctypes.byref(self.opts), _ptr(self.ws), self.ws.numel(),
                                         ctypes.byref(self.plan), _stream()))
        self.R = [int(arr[d].R) for d in range(n)]
        self.cpl = [int(arr[d].cpl) for d in range(n)]

    @property
    def helpers(self) -> int:
        """Most helper workgroups per query the plan allows (0: none)."""
        return int(self.plan.helpers)

    @property
    def order_rank(self) -> bool:
        """True when the plan finds the visiting orders by ranking."""
        return bool(self.plan.order_rank)

    def __call__(self):
        _check(lib().nndtw_search_batch(ctypes.byref(self.plan), _ptr(self.ws), _stream()))
        return self.out


def search(refset: RefSet, Q: torch.Tensor, V: int = 5, cascade: str = "keogh_enh", R: int = 0,
           eps: float = 0.0, init_ub: bool = True, cpl: int = 0, waves: int = 0, engine: str = "auto",
           helpers: int = 0, order: str = "auto"):
    """One-shot NN-DTW search: returns (nn_idx int64, nn_dist float64, counts int64[nQ][8], R used)."""
    Q = _series(Q, "Q")
    s = Searcher(refset, Q.shape[0], V, cascade, R, eps, init_ub, cpl, waves, engine, helpers, order)
    idx, dist, counts = s(Q)
    return idx.clone(), dist.clone(), counts.clone(), s.R


def search_noalloc(refset: RefSet, Q: torch.Tensor, idx: torch.Tensor, dist: torch.Tensor, counts=None,
                   V: int = 5, cascade: str = "keogh_enh", R: int = 0, eps: float = 0.0, init_ub: bool = True,
                   cpl: int = 0, waves: int = 0, engine: str = "auto", helpers: int = 0):
    """nndtw_search_noalloc: the search into caller-provided outputs (idx int64
    [nQ], dist float64 [nQ], counts int64 [nQ][8] or None) with the library's
    fixed device workspace; returns the R used."""
    Q = _series(Q, "Q")
    opts = _opts(V, cascade, R, eps, init_ub, cpl, waves, engine, helpers)
    _check(lib().nndtw_search_noalloc(ctypes.byref(refset.desc), _ptr(Q), Q.shape[0], ctypes.byref(opts), _ptr(idx),
                                      _ptr(dist), _ptr(counts), _stream()))
    return int(opts.R)


def cascade_bounds(refset: RefSet, Q: torch.Tensor, V: int):
    """(ed2, lb_keogh, lb_enhanced bands part, lb_enhanced) for all (query, reference), float64."""
    Q = _series(Q, "Q")
    shape = (Q.shape[0], refset.n)
    outs = [torch.empty(shape, dtype=torch.float64, device=Q.device) for _ in range(4)]
    _check(lib().nndtw_cascade_bounds(ctypes.byref(refset.desc), _ptr(Q), Q.shape[0], int(V),
                                      *[_ptr(o) for o in outs], _stream()))
    return tuple(outs)
