"""Python binding of librid (randomized interpolative decomposition on MI355X).

Thin ctypes marshalling over the C ABI in include/rid.h: the functions here
have the C names, take torch tensors that live on the GPU, pass their device
pointers, leading dimensions and the current HIP stream, and raise RidError
on a non-OK status.  Every step of the computation runs in librid's HIP
kernels; nothing here computes.  There is no CPU fallback: importing this
package works, but every call raises ImportError until librid.so is built.

Layouts (as in rid.h): A, Y, R, P are column-major, i.e. tensors of shape
(rows, cols) with stride (1, ld); ``colmajor()`` makes such a copy.  G is
row-major (an ordinary contiguous (l, m) tensor).  Indices are int64.

Method: Lucas, Stalzer & Feo, arXiv 1205.3830, Sec. 2 (sketch, pivoted QR,
R2 = R1 T, P = [I T]) and Table 5 (the error ||A - BP||_2).
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librid.so")

RID_OK = 0
RID_ERR_INVALID_ARG = 1
RID_ERR_UNSUPPORTED = 2
RID_ERR_NOMEM = 3
RID_ERR_HIP = 4
RID_ERR_RANK = 5

RID_C128 = 0
RID_C64 = 1
RID_FP64 = 0
RID_FP32 = 1
RID_BF16X2 = 2
RID_BF16X3 = 3

EXPORTED = ["rid_create", "rid_destroy", "rid_status_string", "rid_last_hip_error",
            "rid_reserve", "rid_gaussian", "rid_sketch", "rid_sketch_explicit", "rid_pivqr",
            "rid_pivqr_static", "rid_interp", "rid_residual", "rid_decompose", "rid_decompose_explicit",
            "rid_query_status", "rid_profile",
            "rid_profile_read", "rid_set_sketch", "rid_srft_operator", "rid_decompose_batched",
            "rid_server_create", "rid_server_submit", "rid_server_drain", "rid_server_stats",
            "rid_server_destroy", "rid_set_batch_plan", "rid_get_batch_plan", "rid_tune_batched",
            "rid_set_qr", "rid_set_residual", "rid_svd"]

RID_SKETCH_GAUSSIAN = 0
RID_SKETCH_SRFT = 1
RID_QR_HOUSEHOLDER = 0
RID_QR_CGS2 = 1
RID_RESIDUAL_AUTO = 0
RID_RESIDUAL_DOT2 = 1
RID_RESIDUAL_FP64 = 2
RID_RESIDUAL_FP32 = 3

RID_KERNEL_SKETCH = 0
RID_KERNEL_AX = 1
RID_KERNEL_AHZ = 2
RID_KERNEL_PIVQR = 3
RID_KERNEL_INTERP = 4
KERNEL_NAMES = {RID_KERNEL_SKETCH: "sketch", RID_KERNEL_AX: "residual_ax",
                RID_KERNEL_AHZ: "residual_ahz", RID_KERNEL_PIVQR: "pivqr",
                RID_KERNEL_INTERP: "interp"}

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_U64 = ctypes.c_uint64
_I = ctypes.c_int
_D = ctypes.c_double

_lib = None


class rid_job(ctypes.Structure):
    """Mirror of the C struct rid_job (one ID of a batch)."""
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
                ("l", ctypes.c_int64), ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("J", ctypes.c_void_p), ("P", ctypes.c_void_p),
                ("ldp", ctypes.c_int64), ("sigma", ctypes.c_void_p)]


class rid_server_config(ctypes.Structure):
    """Mirror of the C struct rid_server_config."""
    _fields_ = [("hbm_budget", ctypes.c_int64), ("big_bytes", ctypes.c_int64),
                ("big_lanes", ctypes.c_int), ("batch_lanes", ctypes.c_int),
                ("max_batch", ctypes.c_int)]


class rid_request(ctypes.Structure):
    """Mirror of the C struct rid_request (one served ID)."""
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
                ("l", ctypes.c_int64), ("dtype", ctypes.c_int), ("prec", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("q", ctypes.c_int), ("max_retries", ctypes.c_int),
                ("rank_tol", ctypes.c_double), ("fill_bytes", ctypes.c_int64)]


ADMIT_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                            ctypes.POINTER(rid_job))
DONE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64,
                           ctypes.POINTER(ctypes.c_double))

_sig = {
    "rid_create": ([ctypes.POINTER(_P), _I], _I),
    "rid_destroy": ([_P], _I),
    "rid_status_string": ([_I], ctypes.c_char_p),
    "rid_last_hip_error": ([_P], _I),
    "rid_reserve": ([_P, _I64, _I64, _I64, _I64], _I),
    "rid_gaussian": ([_P, _P, _I64, _I64, _U64, ctypes.c_uint32, _P, _I64], _I),
    "rid_sketch": ([_P, _P, _I, _I, _I64, _I64, _I64, _P, _I64, _U64, _P, _I64], _I),
    "rid_sketch_explicit": ([_P, _P, _I, _I, _I64, _I64, _I64, _P, _I64, _P, _I64, _P, _I64],
                            _I),
    "rid_pivqr": ([_P, _P, _I64, _I64, _I64, _P, _I64, _P, _P, _D], _I),
    "rid_pivqr_static": ([_P, _P, _I64, _I64, _I64, _P, _I64, _P, _P, _D], _I),
    "rid_interp": ([_P, _P, _I64, _I64, _P, _I64, _P, _P, _I64], _I),
    "rid_residual": ([_P, _P, _I, _I, _I64, _I64, _I64, _P, _I64, _P, _P, _I64, _I, _U64, _P,
                      _P], _I),
    "rid_decompose": ([_P, _P, _I, _I, _I64, _I64, _I64, _I64, _P, _I64, _U64, _I, _I, _D, _P,
                       _P, _I64, _P, ctypes.POINTER(_U64)], _I),
    "rid_decompose_explicit": ([_P, _P, _I, _I, _I64, _I64, _I64, _I64, _P, _I64, _P, _I64,
                                _U64, _I, _I, _D, _P, _P, _I64, _P, ctypes.POINTER(_U64)], _I),
    "rid_query_status": ([_P, _P], _I),
    "rid_profile": ([_P, _I], _I),
    "rid_set_sketch": ([_P, _I], _I),
    "rid_decompose_batched": ([_P, _P, _I, _I, ctypes.POINTER(rid_job), _I, _I, _I, _D,
                               ctypes.POINTER(_I), ctypes.POINTER(_U64)], _I),
    "rid_srft_operator": ([_P, _P, _I64, _I64, _U64, _P, _I64], _I),
    "rid_server_create": ([ctypes.POINTER(_P), _I, ctypes.POINTER(rid_server_config), ADMIT_FN,
                           DONE_FN, _P], _I),
    "rid_server_submit": ([_P, ctypes.POINTER(rid_request), ctypes.POINTER(_U64)], _I),
    "rid_server_drain": ([_P], _I),
    "rid_set_batch_plan": ([_P, _I64, _I64, _I], _I),
    "rid_set_qr": ([_P, _I], _I),
    "rid_set_residual": ([_P, _I], _I),
    "rid_svd": ([_P, _P, _I, _I64, _I64, _I64, _P, _I64, _P, _P, _I64, _P, _I64, _P, _P, _I64,
                 ctypes.POINTER(_I)], _I),
    "rid_get_batch_plan": ([_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I)],
                           _I),
    "rid_tune_batched": ([_P, _P, _I, _I, ctypes.POINTER(rid_job), _I, _I,
                          ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I)], _I),
    "rid_server_stats": ([_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I64)],
                         _I),
    "rid_server_destroy": ([_P], _I),
    "rid_profile_read": ([_P, _I, ctypes.POINTER(_D), ctypes.POINTER(_I64)], _I),
}


class _Lib:
    """librid.so, loaded on first use; raises if it has not been built."""

    def __getattr__(self, name):
        global _lib
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError("librid.so is not built (run __graft_entry__.build() or "
                                  "python -m paper_1205_3830_amd.build); there is no "
                                  "fallback")
            lib = ctypes.CDLL(LIB_PATH)
            for fname, (args, res) in _sig.items():
                f = getattr(lib, fname)
                f.argtypes = args
                f.restype = res
            _lib = lib
        return getattr(_lib, name)


_L = _Lib()


def load():
    """Load librid.so now (ImportError if it is missing); returns the CDLL."""
    _L.rid_status_string
    return _lib


class RidError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _L.rid_status_string(status).decode()
        super().__init__("%s failed: %s" % (where, msg))


def _check(st: int, where: str) -> None:
    if st != RID_OK:
        raise RidError(st, where)


def _torch():
    import torch
    return torch


def _stream(stream):
    if stream is None:
        return _P(_torch().cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return _P(stream)
    return _P(stream.cuda_stream)


def _ptr(t):
    return _P(t.data_ptr()) if t is not None else _P(0)


def colmajor(t):
    """A column-major (stride (1, rows)) copy of a 2-D tensor."""
    return t.t().contiguous().t()


def _ld_colmajor(t, name):
    if t.dim() != 2 or (t.stride(0) != 1 and t.shape[0] > 1) or not t.is_cuda:
        raise ValueError("%s must be a 2-D column-major CUDA tensor" % name)
    return max(t.stride(1), t.shape[0], 1)


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.complex128:
        return RID_C128
    if t.dtype == torch.complex64:
        return RID_C64
    raise ValueError("A must be complex128 or complex64")


# --------------------------------------------------------------------- handle
def rid_create(device: int = 0):
    h = _P()
    _check(_L.rid_create(ctypes.byref(h), device), "rid_create")
    return h


def rid_destroy(h) -> None:
    _check(_L.rid_destroy(h), "rid_destroy")


def rid_status_string(status: int) -> str:
    return _L.rid_status_string(status).decode()


def rid_last_hip_error(h) -> int:
    return _L.rid_last_hip_error(h)


def rid_reserve(h, max_m: int, max_n: int, max_l: int, max_k: int) -> None:
    _check(_L.rid_reserve(h, max_m, max_n, max_l, max_k), "rid_reserve")


# --------------------------------------------------------------------- steps
def rid_gaussian(h, rows: int, cols: int, seed: int, stream_id: int, out=None, stream=None):
    """rows x cols block of the Gaussian stream (row-major complex128)."""
    torch = _torch()
    if out is None:
        out = torch.empty((rows, cols), dtype=torch.complex128, device="cuda")
    ld = out.stride(0) if rows > 1 else max(cols, 1)
    _check(_L.rid_gaussian(h, _stream(stream), rows, cols, seed, stream_id, _ptr(out), ld),
           "rid_gaussian")
    return out


def rid_set_residual(h, kind: int) -> None:
    """Choose the accumulation of the residual's passes over A for later
    rid_residual / rid_decompose / batched calls (RID_RESIDUAL_*)."""
    _check(_L.rid_set_residual(h, kind), "rid_set_residual")


def rid_set_qr(h, kind: int) -> None:
    """Choose the pivoted-QR method (RID_QR_HOUSEHOLDER or RID_QR_CGS2) of
    later rid_pivqr / rid_decompose calls."""
    _check(_L.rid_set_qr(h, kind), "rid_set_qr")


def rid_set_sketch(h, kind: int) -> None:
    """Choose the random operator of later rid_sketch / rid_decompose calls."""
    _check(_L.rid_set_sketch(h, kind), "rid_set_sketch")


def rid_srft_operator(h, rows: int, m: int, seed: int, out=None, stream=None):
    """rows x m block of the S F D operator (row-major complex128)."""
    torch = _torch()
    if out is None:
        out = torch.empty((rows, m), dtype=torch.complex128, device="cuda")
    ld = out.stride(0) if rows > 1 else max(m, 1)
    _check(_L.rid_srft_operator(h, _stream(stream), rows, m, seed, _ptr(out), ld),
           "rid_srft_operator")
    return out


def _new_colmajor(rows, cols, dtype):
    torch = _torch()
    return torch.empty((cols, rows), dtype=dtype, device="cuda").t()


def rid_sketch(h, A, l: int, seed: int, Y=None, prec: int = RID_FP64, stream=None):
    """Y = G(seed) A (l x n complex128, column-major)."""
    torch = _torch()
    m, n = A.shape
    lda = _ld_colmajor(A, "A")
    if Y is None:
        Y = _new_colmajor(l, n, torch.complex128)
    ldy = _ld_colmajor(Y, "Y")
    _check(_L.rid_sketch(h, _stream(stream), _dtype_code(A), prec, m, n, l, _ptr(A), lda,
                           seed, _ptr(Y), ldy), "rid_sketch")
    return Y


def rid_sketch_explicit(h, A, G, Y=None, prec: int = RID_FP64, stream=None):
    """Y = G A with a caller-supplied row-major G (l x m complex128)."""
    torch = _torch()
    m, n = A.shape
    l = G.shape[0]
    lda = _ld_colmajor(A, "A")
    if G.dim() != 2 or G.shape[1] != m or (G.stride(1) != 1 and m > 1):
        raise ValueError("G must be a row-major (l, m) tensor")
    ldg = max(G.stride(0), m, 1)
    if Y is None:
        Y = _new_colmajor(l, n, torch.complex128)
    ldy = _ld_colmajor(Y, "Y")
    _check(_L.rid_sketch_explicit(h, _stream(stream), _dtype_code(A), prec, m, n, l,
                                    _ptr(A), lda, _ptr(G), ldg, _ptr(Y), ldy),
           "rid_sketch_explicit")
    return Y


def rid_pivqr(h, Y, k: int, perm=None, gaps=None, rank_tol: float = 1e-12, stream=None):
    """Pivoted QR of Y in place; returns (perm, gaps)."""
    torch = _torch()
    l, n = Y.shape
    ldy = _ld_colmajor(Y, "Y")
    if perm is None:
        perm = torch.empty(n, dtype=torch.int64, device="cuda")
    if gaps is None:
        gaps = torch.empty(k, dtype=torch.float64, device="cuda")
    _check(_L.rid_pivqr(h, _stream(stream), l, n, k, _ptr(Y), ldy, _ptr(perm), _ptr(gaps),
                          rank_tol), "rid_pivqr")
    return perm, gaps


def rid_pivqr_static(h, Y, k: int, perm=None, gaps=None, rank_tol: float = 1e-12, stream=None):
    """rid_pivqr with its scratch in the library's static device array (no
    device allocation inside the call); returns (perm, gaps)."""
    torch = _torch()
    l, n = Y.shape
    ldy = _ld_colmajor(Y, "Y")
    if perm is None:
        perm = torch.empty(n, dtype=torch.int64, device="cuda")
    if gaps is None:
        gaps = torch.empty(k, dtype=torch.float64, device="cuda")
    _check(_L.rid_pivqr_static(h, _stream(stream), l, n, k, _ptr(Y), ldy, _ptr(perm),
                                 _ptr(gaps), rank_tol), "rid_pivqr_static")
    return perm, gaps


def rid_interp(h, R, J, P=None, stream=None):
    """P = [I T] with R1 T = R2 (k x n complex128, original column order)."""
    torch = _torch()
    k = J.shape[0]
    n = R.shape[1]
    ldr = _ld_colmajor(R, "R")
    if P is None:
        P = _new_colmajor(k, n, torch.complex128)
    ldp = _ld_colmajor(P, "P")
    _check(_L.rid_interp(h, _stream(stream), n, k, _ptr(R), ldr, _ptr(J), _ptr(P), ldp),
           "rid_interp")
    return P


def rid_residual(h, A, J, P, q: int, seed: int, sigma=None, hist=None, prec: int = RID_FP64,
                 stream=None):
    """Power-iteration estimate of ||A - A(:,J) P||_2; returns (sigma, hist)."""
    torch = _torch()
    m, n = A.shape
    k = J.shape[0] if J is not None else 0
    lda = _ld_colmajor(A, "A")
    ldp = _ld_colmajor(P, "P") if k > 0 else 1
    if sigma is None:
        sigma = torch.zeros(1, dtype=torch.float64, device="cuda")
    if hist is None:
        hist = torch.zeros(q, dtype=torch.float64, device="cuda")
    _check(_L.rid_residual(h, _stream(stream), _dtype_code(A), prec, m, n, k, _ptr(A), lda,
                             _ptr(J) if k else _P(0), _ptr(P) if k else _P(0), ldp, q, seed,
                             _ptr(sigma), _ptr(hist)), "rid_residual")
    return sigma, hist


def rid_decompose(h, A, k: int, l: int, seed: int = 0, q: int = 10, max_retries: int = 3,
                  rank_tol: float = 1e-12, J=None, P=None, sigma=None, prec: int = RID_FP64,
                  stream=None):
    """The whole ID; returns (J, P, sigma, seed_used).  Synchronises."""
    torch = _torch()
    m, n = A.shape
    lda = _ld_colmajor(A, "A")
    if J is None:
        J = torch.empty(k, dtype=torch.int64, device="cuda")
    if P is None:
        P = _new_colmajor(k, n, torch.complex128)
    ldp = _ld_colmajor(P, "P")
    if sigma is None:
        sigma = torch.zeros(1, dtype=torch.float64, device="cuda")
    used = _U64(0)
    _check(_L.rid_decompose(h, _stream(stream), _dtype_code(A), prec, m, n, k, l, _ptr(A),
                              lda, seed, q, max_retries, rank_tol, _ptr(J), _ptr(P), ldp,
                              _ptr(sigma), ctypes.byref(used)), "rid_decompose")
    return J, P, sigma, int(used.value)


def rid_decompose_explicit(h, A, G0, k: int, seed: int = 0, q: int = 10,
                           max_retries: int = 3, rank_tol: float = 1e-12, J=None, P=None,
                           sigma=None, prec: int = RID_FP64, stream=None):
    """rid_decompose whose first draw uses the row-major (l, m) operator G0;
    redraws use the operators of seed + 1, ...  Returns (J, P, sigma,
    seed_used).  Synchronises."""
    torch = _torch()
    m, n = A.shape
    l = G0.shape[0]
    lda = _ld_colmajor(A, "A")
    if G0.dim() != 2 or G0.shape[1] != m or (G0.stride(1) != 1 and m > 1):
        raise ValueError("G0 must be a row-major (l, m) tensor")
    ldg = max(G0.stride(0), m, 1)
    if J is None:
        J = torch.empty(k, dtype=torch.int64, device="cuda")
    if P is None:
        P = _new_colmajor(k, n, torch.complex128)
    ldp = _ld_colmajor(P, "P")
    if sigma is None:
        sigma = torch.zeros(1, dtype=torch.float64, device="cuda")
    used = _U64(0)
    _check(_L.rid_decompose_explicit(h, _stream(stream), _dtype_code(A), prec, m, n, k, l,
                                       _ptr(A), lda, _ptr(G0), ldg, seed, q, max_retries,
                                       rank_tol, _ptr(J), _ptr(P), ldp, _ptr(sigma),
                                       ctypes.byref(used)), "rid_decompose_explicit")
    return J, P, sigma, int(used.value)


def rid_svd(h, A, J, P, U=None, S=None, V=None, stream=None):
    """Rank-k SVD of A(:,J) P; returns (U m x k, S k descending, V n x k,
    Jacobi sweeps).  Synchronises."""
    torch = _torch()
    m, n = A.shape
    k = J.shape[0]
    lda = _ld_colmajor(A, "A")
    ldp = _ld_colmajor(P, "P")
    if U is None:
        U = _new_colmajor(m, k, torch.complex128)
    if S is None:
        S = torch.zeros(k, dtype=torch.float64, device="cuda")
    if V is None:
        V = _new_colmajor(n, k, torch.complex128)
    ldu = _ld_colmajor(U, "U")
    ldv = _ld_colmajor(V, "V")
    sweeps = _I(0)
    _check(_L.rid_svd(h, _stream(stream), _dtype_code(A), m, n, k, _ptr(A), lda, _ptr(J),
                        _ptr(P), ldp, _ptr(U), ldu, _ptr(S), _ptr(V), ldv, ctypes.byref(sweeps)),
           "rid_svd")
    return U, S, V, int(sweeps.value)


def rid_query_status(h, stream=None) -> int:
    """Synchronise and read the handle's status word (RID_OK or RID_ERR_RANK)."""
    st = _L.rid_query_status(h, _stream(stream))
    if st not in (RID_OK, RID_ERR_RANK):
        raise RidError(st, "rid_query_status")
    return st


def rid_profile(h, enable: bool) -> None:
    """Start (and clear) or stop event timing of the hot kernels."""
    _check(_L.rid_profile(h, 1 if enable else 0), "rid_profile")


def rid_profile_read(h, kernel: int):
    """(total milliseconds, launches) recorded for one kernel family."""
    ms = _D(0.0)
    cnt = _I64(0)
    _check(_L.rid_profile_read(h, kernel, ctypes.byref(ms), ctypes.byref(cnt)),
           "rid_profile_read")
    return ms.value, cnt.value


class _Slices:
    """Per-job views into one output slab, made when indexed."""

    def __init__(self, base, spans, shape_of):
        self._base, self._spans, self._shape_of = base, spans, shape_of

    def __len__(self):
        return len(self._spans)

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [self[j] for j in range(*i.indices(len(self)))]
        off, size, shape = self._spans[i]
        return self._shape_of(self._base[off:off + size], shape)

    def __iter__(self):
        return (self[i] for i in range(len(self)))


def rid_decompose_batched(h, As, ks, ls, seeds, q: int = 10, max_retries: int = 3,
                          rank_tol: float = 1e-12, prec: int = RID_FP64, stream=None,
                          raise_on_rank: bool = True):
    """Many IDs in one call.  As: list of column-major device tensors (one
    dtype); ks, ls, seeds: per-job ints.  Returns (Js, Ps, sigmas, status,
    seeds_used): per-job device views (J: k int64, P: k x n complex128
    column-major, sigma: 1 float64) into three output slabs, and host lists."""
    tab, dt, Jall, Pall, sall, koff, poff, ks, ns = _batch_table(As, ks, ls, seeds)
    count = len(As)
    status = (_I * max(count, 1))()
    used = (_U64 * max(count, 1))()
    st = _L.rid_decompose_batched(h, _stream(stream), dt, prec,
                                  ctypes.cast(tab.ctypes.data, ctypes.POINTER(rid_job)),
                                  count, q, max_retries, rank_tol, status, used)
    if st != RID_OK and not (st == RID_ERR_RANK and not raise_on_rank):
        raise RidError(st, "rid_decompose_batched")
    Js = _Slices(Jall, [(int(koff[i]), ks[i], None) for i in range(count)], lambda v, s: v)
    Ps = _Slices(Pall, [(int(poff[i]), ks[i] * ns[i], (ns[i], ks[i])) for i in range(count)],
                 lambda v, s: v.view(s).t())
    sig = _Slices(sall, [(i, 1, None) for i in range(count)], lambda v, s: v)
    return Js, Ps, sig, [status[i] for i in range(count)], [int(used[i]) for i in range(count)]


def _batch_table(As, ks, ls, seeds):
    """The rid_job array of a batch (numpy, one row of 11 int64 per job) and
    the output slabs it points into."""
    import numpy as np
    torch = _torch()
    count = len(As)
    dts = {A.dtype for A in As}
    if len(dts) > 1:
        raise ValueError("all matrices of a batch must share one dtype")
    dt = _dtype_code(As[0]) if count else RID_C128
    ks = [int(x) for x in ks]
    ls = [int(x) for x in ls]
    ns = [int(A.shape[1]) for A in As]
    tab = np.zeros((max(count, 1), 11), dtype=np.int64)
    if count:
        tab[:count, 0] = [int(A.shape[0]) for A in As]
        tab[:count, 1] = ns
        tab[:count, 2] = ks
        tab[:count, 3] = ls
        tab[:count, 4] = [A.data_ptr() for A in As]
        tab[:count, 5] = [_ld_colmajor(A, "A") for A in As]
        tab[:count, 6] = np.array([int(x) for x in seeds], dtype=np.uint64).view(np.int64)
    koff = np.concatenate([[0], np.cumsum(ks)]).astype(np.int64)
    poff = np.concatenate([[0], np.cumsum(np.array(ks, dtype=np.int64) *
                                          np.array(ns, dtype=np.int64))]).astype(np.int64)
    Jall = torch.empty(max(int(koff[-1]), 1), dtype=torch.int64, device="cuda")
    Pall = torch.empty(max(int(poff[-1]), 1), dtype=torch.complex128, device="cuda")
    sall = torch.zeros(max(count, 1), dtype=torch.float64, device="cuda")
    if count:
        tab[:count, 7] = Jall.data_ptr() + 8 * koff[:-1]
        tab[:count, 8] = Pall.data_ptr() + 16 * poff[:-1]
        tab[:count, 9] = ks
        tab[:count, 10] = sall.data_ptr() + 8 * np.arange(count, dtype=np.int64)
    return tab, dt, Jall, Pall, sall, koff, poff, ks, ns


def rid_set_batch_plan(h, sketch_rows: int, res_block_bytes: int, ahz_cols: int = 8) -> None:
    _check(_L.rid_set_batch_plan(h, sketch_rows, res_block_bytes, ahz_cols),
           "rid_set_batch_plan")


def rid_get_batch_plan(h):
    """(sketch split rows, A-pass workgroup bytes, A^H z columns per wave) of
    the handle's batches."""
    a, b, c = _I64(0), _I64(0), _I(0)
    _check(_L.rid_get_batch_plan(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
           "rid_get_batch_plan")
    return a.value, b.value, c.value


def rid_tune_batched(h, As, ks, ls, seeds, q: int = 10, prec: int = RID_FP64, stream=None):
    """Autotune the handle's batch plan on this batch; returns the chosen
    (sketch split rows, A-pass workgroup bytes, A^H z columns per wave)."""
    tab, dt, Jall, Pall, sall, _, _, _, _ = _batch_table(As, ks, ls, seeds)
    a, b, c = _I64(0), _I64(0), _I(0)
    _check(_L.rid_tune_batched(h, _stream(stream), dt, prec,
                               ctypes.cast(tab.ctypes.data, ctypes.POINTER(rid_job)), len(As), q,
                               ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
           "rid_tune_batched")
    return a.value, b.value, c.value


def rid_server_create(device: int, cfg: rid_server_config, admit_cb, done_cb):
    """Start a server (admit_cb / done_cb: ADMIT_FN / DONE_FN objects the
    caller keeps alive); returns its handle."""
    h = _P()
    _check(_L.rid_server_create(ctypes.byref(h), device, ctypes.byref(cfg), admit_cb, done_cb,
                                None), "rid_server_create")
    return h


def rid_server_submit(s, req: rid_request) -> int:
    t = _U64(0)
    _check(_L.rid_server_submit(s, ctypes.byref(req), ctypes.byref(t)), "rid_server_submit")
    return t.value


def rid_server_drain(s) -> None:
    _check(_L.rid_server_drain(s), "rid_server_drain")


def rid_server_stats(s):
    peak, done, batches = _I64(0), _I64(0), _I64(0)
    _check(_L.rid_server_stats(s, ctypes.byref(peak), ctypes.byref(done), ctypes.byref(batches)),
           "rid_server_stats")
    return {"peak_bytes": peak.value, "completed": done.value, "batches": batches.value}


def rid_server_destroy(s) -> None:
    _check(_L.rid_server_destroy(s), "rid_server_destroy")


class RidServer:
    """Continuous-batching request loop on one device (rid_server_*).

    fill(ticket, req) -> A is called on a server lane once request `ticket`
    is admitted, with torch's current stream set to the lane's stream; it
    returns A as a column-major device tensor of the request's dtype
    (complex128 for RID_C128, complex64 for RID_C64).  The binding allocates
    J, P and sigma per request; result(ticket) returns them with the status,
    the seed of the last draw and the four times (arrival, admission, A in
    place, done; seconds since the server started).  A is released when the
    job is done.
    """

    def __init__(self, fill, device: int = 0, hbm_budget: int | None = None,
                 big_bytes: int = 1 << 30, big_lanes: int = 2, batch_lanes: int = 2,
                 max_batch: int = 512):
        import threading
        torch = _torch()
        if hbm_budget is None:
            free, total = torch.cuda.mem_get_info(device)
            hbm_budget = int(0.8 * free)
        self._fill = fill
        self._device = device
        self._lock = threading.Lock()
        self._reqs = {}
        self._live = {}
        self._results = {}
        self._errors = {}
        cfg = rid_server_config(hbm_budget, big_bytes, big_lanes, batch_lanes, max_batch)
        self._admit_cb = ADMIT_FN(self._admit)
        self._done_cb = DONE_FN(self._done)
        self._s = rid_server_create(device, cfg, self._admit_cb, self._done_cb)

    def _admit(self, ctx, ticket, stream, job_p):
        try:
            torch = _torch()
            with self._lock:
                req = self._reqs[ticket]
            with torch.cuda.device(self._device), \
                    torch.cuda.stream(torch.cuda.ExternalStream(stream)):
                A = self._fill(ticket, req)
                k, n = req["k"], req["n"]
                J = torch.empty(k, dtype=torch.int64, device="cuda")
                P = _new_colmajor(k, n, torch.complex128)
                sig = torch.zeros(1, dtype=torch.float64, device="cuda")
            want = torch.complex128 if req["dtype"] == RID_C128 else torch.complex64
            if tuple(A.shape) != (req["m"], n) or A.dtype != want:
                raise ValueError("fill returned %s %s for request %s" % (tuple(A.shape), A.dtype, req))
            job = job_p.contents
            job.A = A.data_ptr()
            job.lda = _ld_colmajor(A, "A")
            job.J = J.data_ptr()
            job.P = P.data_ptr()
            job.ldp = _ld_colmajor(P, "P")
            job.sigma = sig.data_ptr()
            with self._lock:
                self._live[ticket] = (A, J, P, sig)
            return 0
        except Exception as e:  # reported through result(ticket)
            with self._lock:
                self._errors[ticket] = repr(e)
            return 1

    def _done(self, ctx, ticket, status, seed_used, times):
        with self._lock:
            out = self._live.pop(ticket, None)
            self._results[ticket] = {
                "status": status, "seed_used": seed_used,
                "times": [times[i] for i in range(4)],
                "J": out[1] if out else None, "P": out[2] if out else None,
                "sigma": out[3] if out else None, "error": self._errors.pop(ticket, None)}

    def submit(self, m: int, n: int, k: int, l: int, dtype: int = RID_C128,
               prec: int = RID_FP64, seed: int = 0, q: int = 10, max_retries: int = 3,
               rank_tol: float = 1e-12, fill_bytes: int = 0, **meta) -> int:
        """Queue one ID; returns its ticket.  meta is handed to fill()."""
        req = rid_request(m, n, k, l, dtype, prec, seed, q, max_retries, rank_tol, fill_bytes)
        with self._lock:
            t = rid_server_submit(self._s, req)
            d = dict(m=m, n=n, k=k, l=l, dtype=dtype, prec=prec, seed=seed, q=q)
            d.update(meta)
            self._reqs[t] = d
        return t

    def drain(self) -> None:
        rid_server_drain(self._s)

    def result(self, ticket: int):
        with self._lock:
            return self._results.get(ticket)

    def request(self, ticket: int):
        with self._lock:
            return self._reqs.get(ticket)

    def stats(self):
        return rid_server_stats(self._s)

    def close(self) -> None:
        if getattr(self, "_s", None):
            rid_server_destroy(self._s)
            self._s = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
