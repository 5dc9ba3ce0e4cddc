"""ctypes binding of libbnc.so (declarations in include/bnc.h).

Argument marshalling only: tensors must already live on the GPU in the
K-plane layout, a float64 tensor of shape (K, n, n) whose element [w, j, i]
is word w of matrix entry (i, j) (planes column-major), or (K, n) for
vectors.  Calls run on torch's current HIP stream.  There is no CPU path: if
the library cannot be loaded the import of this module fails.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libbnc.so")

BNC_CONVERGED, BNC_MAX_ITER, BNC_SINGULAR, BNC_NONFINITE, BNC_BAD_SIZE, BNC_STAGNATED = 0, 1, 2, 3, 4, 5
BNC_AUTO = 0
BNC_TIMED_OUT = 6
BNC_SPLIT_RANGE = 7
BNC_ERR_HIP, BNC_ERR_UNSUPPORTED, BNC_ERR_WORKSPACE, BNC_ERR_TIMEOUT = -100, -101, -102, -103
OP_FMS, OP_MUL, OP_ADD, OP_RECIP, OP_ROUND4 = 0, 1, 2, 3, 4
_SUFFIX = {1: "d", 2: "dd", 3: "td", 4: "qd"}


class BncError(RuntimeError):
    def __init__(self, msg: str, code: int = 0):
        super().__init__(msg)
        self.code = code


class RefineOpts(ctypes.Structure):
    _fields_ = [("factor_words", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("atol", ctypes.c_double), ("ctol", ctypes.c_double), ("ozaki_slices", ctypes.c_int32),
                ("escalate", ctypes.c_int32), ("stagnation_ratio", ctypes.c_double), ("batch_panel", ctypes.c_int32),
                ("batch_threads", ctypes.c_int32), ("long_words", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("selector_params", ctypes.c_void_p), ("selector_norm", ctypes.c_void_p)]


class RefineResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("info", ctypes.c_int64),
                ("resid_norm", ctypes.c_double), ("x_norm", ctypes.c_double), ("a_norm", ctypes.c_double),
                ("residual_inexact", ctypes.c_int32), ("final_words", ctypes.c_int32),
                ("escalations", ctypes.c_int32), ("first_words", ctypes.c_int32)]


class AdamOpts(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("step", ctypes.c_int64)]


class BatchResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("info", ctypes.c_int64),
                ("t_start", ctypes.c_uint64), ("t_end", ctypes.c_uint64), ("residual_inexact", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("t_factored", ctypes.c_uint64)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(lib_path):
        from . import build as _b
        _b.build()
    L = ctypes.CDLL(lib_path)
    I64, VP, D, I32 = ctypes.c_int64, ctypes.c_void_p, ctypes.c_double, ctypes.c_int32
    SZ = ctypes.c_size_t
    for s in _SUFFIX.values():
        f = getattr(L, f"bnc_getrf_{s}")
        f.argtypes = [I64, VP, I64, I64, VP, VP, VP, SZ, VP]
        f.restype = ctypes.c_int
        g = getattr(L, f"bnc_getrs_{s}")
        g.argtypes = [I64, I64, VP, I64, I64, VP, VP, I64, I64, VP, VP, SZ, VP]
        g.restype = ctypes.c_int
    L.bnc_getrf_ozaki.argtypes = [I32, I32, I64, VP, I64, I64, VP, VP, VP, SZ, VP]
    L.bnc_getrf_ozaki.restype = ctypes.c_int
    L.bnc_getrf_workspace_size.argtypes = [I32, I32, I64]
    L.bnc_getrf_workspace_size.restype = SZ
    L.bnc_getrs_workspace_size.argtypes = [I32, I64]
    L.bnc_getrs_workspace_size.restype = SZ
    L.bnc_residual_workspace_size.argtypes = [I64]
    L.bnc_residual_workspace_size.restype = SZ
    L.bnc_test_force_timeout.argtypes = [I32]
    L.bnc_test_force_timeout.restype = ctypes.c_int
    for s in _SUFFIX.values():
        gm = getattr(L, f"bnc_gemm_{s}")
        gm.argtypes = [I64, I64, I64, VP, I64, I64, VP, I64, I64, VP, I64, I64, VP]
        gm.restype = ctypes.c_int
    L.bnc_oz_beta.argtypes = [I32, I32]
    L.bnc_oz_beta.restype = ctypes.c_int
    L.bnc_features_workspace_size.argtypes = [I32]
    L.bnc_features_workspace_size.restype = ctypes.c_size_t
    L.bnc_features_default_slots.restype = I32
    L.bnc_features.argtypes = [I64, VP, VP, VP, VP, VP, VP, ctypes.c_size_t, I32, VP]
    L.bnc_features.restype = ctypes.c_int
    L.bnc_mlp_param_count.restype = I32
    L.bnc_mlp_workspace_size.argtypes = [I64]
    L.bnc_mlp_workspace_size.restype = ctypes.c_size_t
    L.bnc_mlp_forward.argtypes = [I64, VP, VP, VP, VP, VP]
    L.bnc_mlp_forward.restype = ctypes.c_int
    L.bnc_mlp_grad.argtypes = [I64, VP, VP, VP, VP, VP, VP, VP, VP, ctypes.c_size_t, VP]
    L.bnc_mlp_grad.restype = ctypes.c_int
    L.bnc_mlp_adam.argtypes = [VP, VP, VP, VP, ctypes.POINTER(AdamOpts), VP]
    L.bnc_mlp_adam.restype = ctypes.c_int
    L.bnc_refine_workspace_size.argtypes = [I64, I32]
    L.bnc_refine_workspace_size.restype = ctypes.c_size_t
    L.bnc_refine.argtypes = [I64, I32, VP, I64, I64, VP, I64, VP, I64, VP, ctypes.c_size_t,
                             ctypes.POINTER(RefineOpts), ctypes.POINTER(RefineResult), VP]
    L.bnc_refine.restype = ctypes.c_int
    L.bnc_refine_async.argtypes = [I64, I32, VP, I64, I64, VP, I64, VP, I64, VP, ctypes.c_size_t,
                                   ctypes.POINTER(RefineOpts), VP, VP]
    L.bnc_refine_async.restype = ctypes.c_int
    L.bnc_refine_batched_workspace_size.argtypes = [I32, I32, I32]
    L.bnc_refine_batched_workspace_size.restype = ctypes.c_size_t
    L.bnc_refine_batched_default_slots.argtypes = [I32, I32, I32]
    L.bnc_refine_batched_default_slots.restype = I32
    L.bnc_refine_batched.argtypes = [I64, VP, VP, VP, VP, VP, VP, VP, ctypes.c_size_t, ctypes.POINTER(RefineOpts),
                                     I32, VP, VP]
    L.bnc_refine_batched.restype = ctypes.c_int
    L.bnc_refine_batched_graph.argtypes = [I64, VP, VP, VP, VP, VP, VP, VP, ctypes.c_size_t,
                                           ctypes.POINTER(RefineOpts), I32, VP, VP, ctypes.POINTER(ctypes.c_void_p)]
    L.bnc_refine_batched_graph.restype = ctypes.c_int
    L.bnc_graph_destroy.argtypes = [VP]
    L.bnc_wall_clock_khz.restype = ctypes.c_int64
    L.bnc_residual.argtypes = [I64, I32, I32, VP, I64, I64, VP, I64, VP, I64, VP, I64, VP, VP, SZ, VP]
    L.bnc_residual.restype = ctypes.c_int
    L.bnc_mw_apply.argtypes = [I32, I32, I64, VP, VP, VP, VP, VP]
    L.bnc_mw_apply.restype = ctypes.c_int
    L.bnc_profile_enable.argtypes = [I32]
    L.bnc_profile_read.argtypes = [ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(I64)]
    for name in ("bnc_status_string", "bnc_last_error", "bnc_version"):
        getattr(L, name).restype = ctypes.c_char_p
    L.bnc_status_string.argtypes = [I32]
    return L


_lib = _load()


def lib() -> ctypes.CDLL:
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise BncError(f"{what}: code {rc}: {_lib.bnc_last_error().decode()}", rc)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, name: str, ndim: int):
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.dim() == ndim):
        raise BncError(f"{name}: expected a contiguous float64 CUDA tensor with {ndim} dims")
    return ctypes.c_void_p(t.data_ptr())


def _workspace(nbytes: int, device, work: torch.Tensor | None = None) -> torch.Tensor:
    if work is not None and work.numel() >= nbytes:
        return work
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def getrf_workspace_size(K: int, n: int, slices: int = 0) -> int:
    return int(_lib.bnc_getrf_workspace_size(K, slices, n))


def getrs_workspace_size(K: int, n: int) -> int:
    return int(_lib.bnc_getrs_workspace_size(K, n))


def residual_workspace_size(n: int) -> int:
    return int(_lib.bnc_residual_workspace_size(n))


def getrf(K: int, A: torch.Tensor, work: torch.Tensor | None = None):
    """In-place P A = L U of a (K, n, n) tensor; returns (ipiv, info) tensors."""
    n = A.shape[1]
    ipiv = torch.empty(max(n, 1), dtype=torch.int64, device=A.device)
    info = torch.empty(1, dtype=torch.int64, device=A.device)
    work = _workspace(getrf_workspace_size(K, n), A.device, work)
    f = getattr(_lib, f"bnc_getrf_{_SUFFIX[K]}")
    _check(f(n, _dev(A, "A", 3), n, n * n, ctypes.c_void_p(ipiv.data_ptr()), ctypes.c_void_p(info.data_ptr()),
             ctypes.c_void_p(work.data_ptr()), work.numel(), _stream()), "getrf")
    return ipiv[:n], info


def getrf_ozaki(K: int, slices: int, A: torch.Tensor, work: torch.Tensor | None = None):
    """bnc_getrf_ozaki: P A = L U with split trailing updates; returns (ipiv, info)."""
    n = A.shape[1]
    ipiv = torch.empty(max(n, 1), dtype=torch.int64, device=A.device)
    info = torch.empty(1, dtype=torch.int64, device=A.device)
    work = _workspace(getrf_workspace_size(K, n, slices) if 1 <= slices <= 12 else 0, A.device, work)
    _check(_lib.bnc_getrf_ozaki(K, slices, n, _dev(A, "A", 3), n, n * n, ctypes.c_void_p(ipiv.data_ptr()),
                                ctypes.c_void_p(info.data_ptr()), ctypes.c_void_p(work.data_ptr()), work.numel(),
                                _stream()), "getrf_ozaki")
    return ipiv[:n], info


def getrs(K: int, LU: torch.Tensor, ipiv: torch.Tensor, B: torch.Tensor, info: torch.Tensor | None = None,
          work: torch.Tensor | None = None) -> torch.Tensor:
    """Solve in place; B is (K, n) or (K, nrhs, n).  info (optional int64
    device tensor) gets 0, or -1 if the substitutions' bounded waits gave up."""
    n = LU.shape[1]
    nrhs = 1 if B.dim() == 2 else B.shape[1]
    f = getattr(_lib, f"bnc_getrs_{_SUFFIX[K]}")
    if not (B.is_cuda and B.dtype == torch.float64 and B.is_contiguous()):
        raise BncError("B: expected a contiguous float64 CUDA tensor")
    if not (ipiv.is_cuda and ipiv.dtype == torch.int64 and ipiv.is_contiguous() and ipiv.numel() >= n):
        raise BncError("ipiv: expected a contiguous int64 CUDA tensor of n entries")
    if info is not None and not (info.is_cuda and info.dtype == torch.int64):
        raise BncError("info: expected an int64 CUDA tensor")
    work = _workspace(getrs_workspace_size(K, n), LU.device, work)
    _check(f(n, nrhs, _dev(LU, "LU", 3), n, n * n, ctypes.c_void_p(ipiv.data_ptr()), ctypes.c_void_p(B.data_ptr()),
             n, n * nrhs, None if info is None else ctypes.c_void_p(info.data_ptr()),
             ctypes.c_void_p(work.data_ptr()), work.numel(), _stream()), "getrs")
    return B


def test_force_timeout(bits: int):
    """Timeout test hook of the library (bnc_test_force_timeout)."""
    _check(_lib.bnc_test_force_timeout(bits), "test_force_timeout")


def gemm(K: int, A: torch.Tensor, B: torch.Tensor, C: torch.Tensor) -> torch.Tensor:
    """C <- C - A B in K-word arithmetic, in place.  A (K, k, m), B (K, n, k)
    and C (K, n, m) are K-plane column-major tensors (column index first)."""
    for name, t in (("A", A), ("B", B), ("C", C)):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.dim() == 3 and t.shape[0] == K):
            raise BncError(f"{name}: expected a contiguous float64 CUDA tensor of shape (K, cols, rows)")
    _, k, m = A.shape
    n = B.shape[1]
    if B.shape[2] != k or C.shape[1] != n or C.shape[2] != m:
        raise BncError("gemm: shapes do not match")
    f = getattr(_lib, f"bnc_gemm_{_SUFFIX[K]}")
    vp = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    _check(f(m, n, k, vp(A), max(m, 1), max(m, 1) * k, vp(B), max(k, 1), max(k, 1) * n, vp(C), max(m, 1),
             max(m, 1) * n, _stream()), "gemm")
    return C


def oz_beta(K: int, slices: int) -> int:
    """Bits per slice of the split form for K-word values cut into `slices`
    slices (host query)."""
    b = int(_lib.bnc_oz_beta(K, slices))
    if b < 0:
        raise BncError("oz_beta: K or slices out of range")
    return b


def refine_workspace_size(n: int, K: int) -> int:
    return int(_lib.bnc_refine_workspace_size(n, K))


def refine(A: torch.Tensor, b: torch.Tensor, K: int, max_iter: int = 30, rtol: float = 0.0, atol: float = 0.0,
           ctol: float = 2.0 ** -208, x: torch.Tensor | None = None, work: torch.Tensor | None = None,
           ozaki: int = 0, escalate: bool = False, stagnation_ratio: float = 0.0, long_words: int = 4,
           selector: "MLP | None" = None) -> dict:
    """Listing 1 of the paper with a K-word factorisation and an L-word long
    precision, L = long_words (4: quad-double, 8: 424 bits).  A: (aw, n, n)
    with aw = 1 or 4; b: (L, n); ozaki = S > 0 factors with the split
    trailing update (S slices); escalate and stagnation_ratio as in
    bnc_refine_opts.  K = BNC_AUTO (0) with `selector` (an MLP) lets the
    library's features and network choose the first factor's words.
    Returns a dict with x (L, n) and the outcome fields."""
    aw, n = A.shape[0], A.shape[1]
    if x is None:
        x = torch.empty((long_words, n), dtype=torch.float64, device=A.device)
    need = refine_workspace_size(n, 0 if K == BNC_AUTO else (4 if escalate else K))
    if work is None or work.numel() < need:
        work = torch.empty(need, dtype=torch.uint8, device=A.device)
    o = RefineOpts(K, max_iter, rtol, atol, ctol, ozaki, 1 if escalate else 0, stagnation_ratio, 0, 0, long_words, 0,
                   None, None)
    if K == BNC_AUTO:
        if selector is None:
            raise BncError("refine: K = BNC_AUTO needs a selector network")
        o.selector_params = selector.params.data_ptr()
        o.selector_norm = selector.norm.data_ptr()
    r = RefineResult()
    _check(_lib.bnc_refine(n, aw, _dev(A, "A", 3), n, n * n, _dev(b, "b", 2), n, _dev(x, "x", 2), n,
                           ctypes.c_void_p(work.data_ptr()), work.numel(), ctypes.byref(o), ctypes.byref(r),
                           _stream()), "refine")
    return dict(x=x, status=r.status, iters=r.iters, info=r.info, resid_norm=r.resid_norm, x_norm=r.x_norm,
                a_norm=r.a_norm, residual_inexact=bool(r.residual_inexact), final_words=r.final_words,
                escalations=r.escalations, first_words=r.first_words)


def refine_async(A: torch.Tensor, b: torch.Tensor, K: int, result: torch.Tensor, x: torch.Tensor,
                 work: torch.Tensor, max_iter: int = 30, rtol: float = 0.0, atol: float = 0.0,
                 ctol: float = 2.0 ** -208, ozaki: int = 0, stagnation_ratio: float = 0.0, long_words: int = 4):
    """bnc_refine_async: the refinement with its loop driven on the device,
    enqueued on the current stream (capturable).  result: a uint8 CUDA
    tensor of sizeof(bnc_refine_result) bytes that receives the outcome;
    read it with refine_result() once the stream is through."""
    aw, n = A.shape[0], A.shape[1]
    if result.numel() < ctypes.sizeof(RefineResult) or result.dtype != torch.uint8 or not result.is_cuda:
        raise BncError("result: expected a CUDA uint8 tensor of sizeof(bnc_refine_result) bytes")
    o = RefineOpts(K, max_iter, rtol, atol, ctol, ozaki, 0, stagnation_ratio, 0, 0, long_words, 0, None, None)
    _check(_lib.bnc_refine_async(n, aw, _dev(A, "A", 3), n, n * n, _dev(b, "b", 2), n, _dev(x, "x", 2), n,
                                 ctypes.c_void_p(work.data_ptr()), work.numel(), ctypes.byref(o),
                                 ctypes.c_void_p(result.data_ptr()), _stream()), "refine_async")


def refine_result(result: torch.Tensor) -> dict:
    """Outcome fields from a device bnc_refine_result (synchronises)."""
    raw = result.cpu().numpy().tobytes()[:ctypes.sizeof(RefineResult)]
    r = RefineResult.from_buffer_copy(raw)
    return dict(status=r.status, iters=r.iters, info=r.info, resid_norm=r.resid_norm, x_norm=r.x_norm,
                a_norm=r.a_norm, residual_inexact=bool(r.residual_inexact), final_words=r.final_words,
                escalations=r.escalations, first_words=r.first_words)


def refine_result_bytes() -> int:
    return ctypes.sizeof(RefineResult)


class BatchSolver:
    """Batched refined solves (bnc_refine_batched) over a fixed set of
    systems: A_s (aw, n, n) planes (aw = 1 binary64 or 4 quad-double words)
    and b_s (4, n) CUDA tensors.  Device pointer arrays, the largest-first
    order, outputs and the workspace are set up once; run() launches
    (optionally through a captured HIP graph).  threads = 0 takes 256, or
    512 when some order is above 256."""

    def __init__(self, As, bs, K: int, max_iter: int = 30, rtol: float = 0.0, atol: float = 0.0,
                 ctol: float = 2.0 ** -208, slots: int = 0, order=None, stagnation_ratio: float = 0.0,
                 panel: int = 0, threads: int = 0):
        dev = As[0].device
        self.count = len(As)
        self.As = [a.contiguous() for a in As]
        self.bs = [b.contiguous() for b in bs]
        self.ns = [int(a.shape[-1]) for a in As]
        self.xs = [torch.empty((4, n), dtype=torch.float64, device=dev) for n in self.ns]
        self.n_dev = torch.tensor(self.ns, dtype=torch.int64, device=dev)
        self.aw_dev = torch.tensor([int(a.shape[0]) if a.dim() == 3 else 1 for a in self.As], dtype=torch.int32,
                                   device=dev)
        if threads == 0 and self.ns and max(self.ns) > 256:
            threads = 512
        self.A_dev = torch.tensor([a.data_ptr() for a in self.As], dtype=torch.int64, device=dev)
        self.b_dev = torch.tensor([b.data_ptr() for b in self.bs], dtype=torch.int64, device=dev)
        self.x_dev = torch.tensor([x.data_ptr() for x in self.xs], dtype=torch.int64, device=dev)
        if order is None:
            order = sorted(range(self.count), key=lambda i: -self.ns[i])
        self.order = torch.tensor(list(order), dtype=torch.int32, device=dev)
        self.res = torch.zeros((self.count, ctypes.sizeof(BatchResult)), dtype=torch.uint8, device=dev)
        if slots == 0:
            slots = int(_lib.bnc_refine_batched_default_slots(K, panel, threads))
            if slots <= 0:
                raise BncError(f"refine_batched_default_slots: {_lib.bnc_last_error().decode()}")
        self.slots = slots
        need = int(_lib.bnc_refine_batched_workspace_size(K, slots, threads))
        self.work = torch.empty(need, dtype=torch.uint8, device=dev)
        self.opts = RefineOpts(K, max_iter, rtol, atol, ctol, 0, 0, stagnation_ratio, panel, threads, 0, 0, None,
                               None)
        self.graph = ctypes.c_void_p(None)
        self.stream = None

    def _args(self):
        P = ctypes.c_void_p
        return (self.count, P(self.n_dev.data_ptr()), P(self.aw_dev.data_ptr()), P(self.A_dev.data_ptr()),
                P(self.b_dev.data_ptr()),
                P(self.x_dev.data_ptr()), P(self.order.data_ptr()), P(self.work.data_ptr()), self.work.numel(),
                ctypes.byref(self.opts), self.slots, P(self.res.data_ptr()))

    def run(self, graph: bool = False):
        if not graph:
            _check(_lib.bnc_refine_batched(*self._args(), _stream()), "refine_batched")
            return
        if self.stream is None:
            self.stream = torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            _check(_lib.bnc_refine_batched_graph(*self._args(), ctypes.c_void_p(self.stream.cuda_stream),
                                                 ctypes.byref(self.graph)), "refine_batched_graph")
        torch.cuda.current_stream().wait_stream(self.stream)

    def results(self):
        import numpy as np
        torch.cuda.synchronize()
        raw = self.res.cpu().numpy()
        dt = np.dtype([("status", "<i4"), ("iters", "<i4"), ("info", "<i8"), ("t_start", "<u8"), ("t_end", "<u8"),
                       ("residual_inexact", "<i4"), ("reserved", "<i4"), ("t_factored", "<u8")])
        return raw.view(dt).reshape(self.count)

    def close(self):
        if self.graph.value:
            _lib.bnc_graph_destroy(self.graph)
            self.graph = ctypes.c_void_p(None)


def wall_clock_khz() -> int:
    return int(_lib.bnc_wall_clock_khz())


def residual(A: torch.Tensor, x: torch.Tensor, b: torch.Tensor):
    """r = b - A x exactly, rounded to its canonical L-word form (L = the
    words of x and b, 4 or 8); returns (r, inexact)."""
    aw, n = A.shape[0], A.shape[1]
    lw = x.shape[0]
    if b.shape[0] != lw:
        raise BncError("residual: x and b must have the same number of words")
    r = torch.empty((lw, n), dtype=torch.float64, device=A.device)
    flag = torch.zeros(1, dtype=torch.int32, device=A.device)
    work = _workspace(residual_workspace_size(n), A.device)
    _check(_lib.bnc_residual(n, aw, lw, _dev(A, "A", 3), n, n * n, _dev(x, "x", 2), n, _dev(b, "b", 2), n,
                             ctypes.c_void_p(r.data_ptr()), n, ctypes.c_void_p(flag.data_ptr()),
                             ctypes.c_void_p(work.data_ptr()), work.numel(), _stream()), "residual")
    return r, flag


def mw_apply(op: int, K: int, a: torch.Tensor, b: torch.Tensor | None = None,
             c: torch.Tensor | None = None) -> torch.Tensor:
    """Element-wise K-word primitive on (K, n) tensors (a: (4, n) for OP_ROUND4)."""
    n = a.shape[1]
    out = torch.empty((K, n), dtype=torch.float64, device=a.device)

    def p(t):
        return None if t is None else ctypes.c_void_p(t.data_ptr())
    _check(_lib.bnc_mw_apply(op, K, n, p(c), p(a), p(b), p(out), _stream()), "mw_apply")
    return out


def profile_enable(on: bool = True):
    _lib.bnc_profile_enable(1 if on else 0)


def profile_read():
    ms, fl, nl = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    _check(_lib.bnc_profile_read(ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(nl)), "profile_read")
    return ms.value, fl.value, nl.value


# --------------------------------------------------------------------------
# learned choice of the factor precision
# --------------------------------------------------------------------------
NFEATURES = 24


def _vp(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def features(As, bs, slots: int = 0) -> torch.Tensor:
    """bnc_features over lists of (1, n, n) binary64 matrices and (4, n)
    right-hand sides (CUDA tensors); returns a (count, 24) float32 tensor."""
    dev = As[0].device
    count = len(As)
    As = [a.contiguous() for a in As]
    bs = [b.contiguous() for b in bs]
    ns = [int(a.shape[-1]) for a in As]
    n = torch.tensor(ns, dtype=torch.int64, device=dev)
    Ap = torch.tensor([a.data_ptr() for a in As], dtype=torch.int64, device=dev)
    bp = torch.tensor([b.data_ptr() for b in bs], dtype=torch.int64, device=dev)
    order = torch.tensor(sorted(range(count), key=lambda i: -ns[i]), dtype=torch.int32, device=dev)
    F = torch.empty((count, NFEATURES), dtype=torch.float32, device=dev)
    need = int(_lib.bnc_features_workspace_size(slots))
    work = torch.empty(need, dtype=torch.uint8, device=dev)
    _check(_lib.bnc_features(count, _vp(n), _vp(Ap), _vp(bp), _vp(order), _vp(F), _vp(work), need, slots,
                             _stream()), "features")
    return F


class MLP:
    """Parameters, input normalisation and Adam moments of the 24-64-64-5
    network on the device; every computation runs in the library's kernels
    (bnc_mlp_forward / bnc_mlp_grad / bnc_mlp_adam)."""

    def __init__(self, params: torch.Tensor, norm: torch.Tensor):
        self.nparam = int(_lib.bnc_mlp_param_count())
        if params.numel() != self.nparam or norm.numel() != 2 * NFEATURES:
            raise BncError("MLP: wrong parameter or normalisation size")
        self.params = params.to(torch.float32).contiguous()
        self.norm = norm.to(torch.float32).contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grads = torch.zeros_like(self.params)
        self.step = 0
        self._work = None

    def forward(self, X: torch.Tensor) -> torch.Tensor:
        X = X.to(torch.float32).contiguous()
        out = torch.empty((X.shape[0], 5), dtype=torch.float32, device=X.device)
        _check(_lib.bnc_mlp_forward(X.shape[0], _vp(X), _vp(self.norm), _vp(self.params), _vp(out), _stream()),
               "mlp_forward")
        return out

    def grad(self, X: torch.Tensor, cls: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
        """Fills self.grads; returns the mean loss as a 1-element tensor."""
        X = X.to(torch.float32).contiguous()
        cls = cls.to(torch.int32).contiguous()
        target = target.to(torch.float32).contiguous()
        B = X.shape[0]
        need = int(_lib.bnc_mlp_workspace_size(B))
        if self._work is None or self._work.numel() < need:
            self._work = torch.empty(need, dtype=torch.uint8, device=X.device)
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        _check(_lib.bnc_mlp_grad(B, _vp(X), _vp(self.norm), _vp(cls), _vp(target), _vp(self.params), _vp(self.grads),
                                 _vp(loss), _vp(self._work), self._work.numel(), _stream()), "mlp_grad")
        return loss

    def adam(self, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.step += 1
        o = AdamOpts(lr, beta1, beta2, eps, self.step)
        _check(_lib.bnc_mlp_adam(_vp(self.params), _vp(self.grads), _vp(self.m), _vp(self.v), ctypes.byref(o),
                                 _stream()), "mlp_adam")
