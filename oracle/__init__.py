"""Reference CPU oracle for the randomized interpolative decomposition.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_1205_3830_amd``) and never imports it.

Source: Lucas, Stalzer & Feo, arXiv 1205.3830, Sec. 2 (the algorithm:
randomization Y = (random operator) A, approximate QR with a column
permutation, R2 = R1 T, P = [I T]) and Table 5 (the error ||A - BP||_2).
The randomization operator here is a complex Gaussian matrix, which Sec. 2
allows in place of the subsampled FFT when it is the faster choice.

The arithmetic lives in ``rid_oracle.c`` (plain loops, IEEE double; the power
iteration in binary128).  This module is the ctypes marshalling around it, plus
``decompose`` which chains the steps and redraws on a rank failure (Sec. 2),
and ``svd_from_id``, the SVD of the ID's approximation A(:,J) P (Sec. 1 lists
fast SVDs among the ID's uses), written as its definition over LAPACK's SVD.

Every function is pinned by a CPU test (tests/test_oracle_pins.py); none is
"parity unpinned".  Arrays are numpy complex128, column-major (Fortran order)
unless stated; index arrays are int64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rid_oracle.c")
_LIB = os.path.join(_HERE, "librid_oracle.so")

OK = 0
ERR_ARG = 1
ERR_RANK = 5


def build(force: bool = True) -> str:
    """Compile rid_oracle.c with gcc (no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp, "-lquadmath", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_philox4x32_10.argtypes = [P, P, P]
        lib.orc_gauss_entry.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_uint64, P]
        lib.orc_gaussian_rowmajor.argtypes = [I64, I64, ctypes.c_uint64, ctypes.c_uint32, P, I64]
        lib.orc_sketch.argtypes = [I64, I64, I64, P, I64, P, I64, P, I64]
        lib.orc_srft_operator.argtypes = [I64, I64, ctypes.c_uint64, P, I64]
        lib.orc_srft_row.argtypes = [ctypes.c_uint64, ctypes.c_uint64, I64]
        lib.orc_srft_row.restype = I64
        lib.orc_srft_phase.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.orc_srft_phase.restype = ctypes.c_double
        lib.orc_sketch_seeded.argtypes = [I64, I64, I64, P, I64, ctypes.c_uint64, P, I64]
        lib.orc_select.argtypes = [I64, I64, I64, P, I64, ctypes.c_double, P, P, I64, P]
        lib.orc_select.restype = ctypes.c_int
        lib.orc_select_forced.argtypes = [I64, I64, I64, P, I64, ctypes.c_double, P, P, P, I64,
                                          P, P, P]
        lib.orc_select_forced.restype = ctypes.c_int
        lib.orc_interp.argtypes = [I64, I64, P, I64, P, P, I64]
        lib.orc_interp.restype = ctypes.c_int
        lib.orc_residual.argtypes = [I64, I64, I64, P, I64, P, P, I64, P, ctypes.c_int, P, P]
        lib.orc_residual.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    """OpenMP threads the oracle's loops run on."""
    return int(_load().orc_num_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _cf(a) -> np.ndarray:
    """complex128, Fortran order."""
    return np.asfortranarray(np.asarray(a, dtype=np.complex128))


# --------------------------------------------------------------------------
# Random draws (the method's randomization, Sec. 2)
# --------------------------------------------------------------------------
def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block function: 4 counter words, 2 key words -> 4 words."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(4))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(2))
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def gaussian(rows: int, cols: int, seed: int, stream: int) -> np.ndarray:
    """rows x cols complex Gaussian, entry (i, j) from counter (j, i, stream)."""
    out = np.zeros((rows, cols), dtype=np.complex128)  # C order == row-major
    if rows and cols:
        _load().orc_gaussian_rowmajor(rows, cols, seed, stream, _ptr(out), cols)
    return out


def sketch_operator(l: int, m: int, seed: int) -> np.ndarray:
    """The l x m Gaussian sketch operator G (stream 0)."""
    return gaussian(l, m, seed, 0)


def srft_rows(l: int, m: int, seed: int) -> np.ndarray:
    """Rows s_0..s_{l-1} kept by S (eq. (5)), i.i.d. uniform on {0..m-1}."""
    return np.array([_load().orc_srft_row(seed, i, m) for i in range(l)], dtype=np.int64)


def srft_phases(m: int, seed: int) -> np.ndarray:
    """phi_0..phi_{m-1} of D (eq. (7)), uniform on (0, 1)."""
    return np.array([_load().orc_srft_phase(seed, p) for p in range(m)], dtype=np.float64)


def srft_operator(l: int, m: int, seed: int) -> np.ndarray:
    """G = S F D as an explicit l x m operator (Sec. 2, eqs. (4)-(7))."""
    out = np.zeros((l, m), dtype=np.complex128)
    if l and m:
        _load().orc_srft_operator(l, m, seed, _ptr(out), m)
    return out


def start_vector(n: int, seed: int) -> np.ndarray:
    """Power-iteration start vector x0 (stream 1), unnormalised, length n."""
    return gaussian(1, n, seed, 1).reshape(n)


# --------------------------------------------------------------------------
# The four steps
# --------------------------------------------------------------------------
def sketch(A, G) -> np.ndarray:
    """Y = G A (Sec. 2 randomization step with the Gaussian operator G)."""
    A = _cf(A)
    G = np.ascontiguousarray(np.asarray(G, dtype=np.complex128))
    m, n = A.shape
    l, mg = G.shape
    assert mg == m
    Y = np.zeros((l, n), dtype=np.complex128, order="F")
    if l and n and m:
        _load().orc_sketch(m, n, l, _ptr(A), m, _ptr(G), m, _ptr(Y), l)
    return Y


def sketch_seeded_columns(Acols, l: int, seed: int) -> np.ndarray:
    """G(seed) @ Acols for a few columns of A (G drawn inside the oracle)."""
    Acols = _cf(Acols)
    m, nc = Acols.shape
    Y = np.zeros((l, nc), dtype=np.complex128, order="F")
    _load().orc_sketch_seeded(m, nc, l, _ptr(Acols), m, seed, _ptr(Y), l)
    return Y


def select(Y, k: int, rank_tol: float = 1e-12):
    """Greedy pivoted column selection + R = Q^H Y (Sec. 2 QR, Sec. 3.2 CGS2).

    Returns (status, J[k] in pivot order, R k x n in original column order,
    gaps[k]).  On a rank failure J holds the steps reached and R is zero.
    """
    Y = _cf(Y)
    l, n = Y.shape
    J = np.full(k, -1, dtype=np.int64)
    R = np.zeros((k, n), dtype=np.complex128, order="F")
    gaps = np.zeros(k, dtype=np.float64)
    st = _load().orc_select(l, n, k, _ptr(Y), l, rank_tol, _ptr(J), _ptr(R), k, _ptr(gaps))
    return st, J, R, gaps


def select_forced(Y, forced, rank_tol: float = 1e-12):
    """The greedy selection re-synchronised onto given pivots.

    Step t takes column forced[t] (where >= 0) instead of its own argmax; the
    step's own choice, its pivot gap and the trailing norm of the column
    taken relative to the best are recorded first.  Sec. 2 only asks for a
    permutation that brings the most weighted columns to the front, so where
    two trailing norms nearly tie either pick is valid; forcing the other
    side's pick keeps every later step comparable.
    Returns a dict: status, J (the columns taken), R (k x n, original column
    order), gaps, argmax (the oracle's own pick per step), ratio.
    """
    Y = _cf(Y)
    l, n = Y.shape
    forced = np.ascontiguousarray(np.asarray(forced, dtype=np.int64))
    k = forced.shape[0]
    J = np.full(k, -1, dtype=np.int64)
    R = np.zeros((k, n), dtype=np.complex128, order="F")
    gaps = np.zeros(k, dtype=np.float64)
    argmax = np.full(k, -1, dtype=np.int64)
    ratio = np.zeros(k, dtype=np.float64)
    st = _load().orc_select_forced(l, n, k, _ptr(Y), l, rank_tol, _ptr(forced), _ptr(J),
                                   _ptr(R), k, _ptr(gaps), _ptr(argmax), _ptr(ratio))
    return dict(status=st, J=J, R=R, gaps=gaps, argmax=argmax, ratio=ratio)


def interp(R, J) -> np.ndarray:
    """P = [I T] with R1 T = R2 (Sec. 2), in original column order."""
    R = _cf(R)
    J = np.ascontiguousarray(np.asarray(J, dtype=np.int64))
    k, n = R.shape
    P = np.zeros((k, n), dtype=np.complex128, order="F")
    st = _load().orc_interp(n, k, _ptr(R), k, _ptr(J), _ptr(P), k)
    if st != OK:
        raise ValueError("oracle interp: invalid arguments")
    return P


def residual(A, J, P, x0, q: int):
    """Power-iteration estimate of ||A - A(:,J) P||_2 (Table 5's quantity).

    Returns (sigma_q, history[q]).
    """
    A = _cf(A)
    P = _cf(P)
    J = np.ascontiguousarray(np.asarray(J, dtype=np.int64))
    x0 = np.ascontiguousarray(np.asarray(x0, dtype=np.complex128))
    m, n = A.shape
    k = P.shape[0]
    sigma = np.zeros(1, dtype=np.float64)
    hist = np.zeros(q, dtype=np.float64)
    st = _load().orc_residual(m, n, k, _ptr(A), m, _ptr(J), _ptr(P), max(k, 1), _ptr(x0), q,
                              _ptr(sigma), _ptr(hist))
    if st != OK:
        raise ValueError("oracle residual: invalid arguments")
    return float(sigma[0]), hist


def decompose(A, k: int, l: int, seed: int = 0, q: int = 10, max_retries: int = 3,
              rank_tol: float = 1e-12, G=None, kind: str = "gaussian"):
    """Full ID: sketch, select, interp, residual; redraw with seed+1 on a
    rank failure, at most max_retries more times (Sec. 2 failure remedy).

    With an explicit G the seed only drives the start vector and no redraw
    of G is possible (a rank failure is returned as is).
    Returns a dict with status, J, P, sigma, hist, seed_used, Y, R, gaps.
    """
    A = _cf(A)
    m, n = A.shape
    s = seed
    attempts = 1 if G is not None else 1 + max_retries
    for _ in range(attempts):
        if G is not None:
            Gs = G
        elif kind == "srft":
            Gs = srft_operator(l, m, s)
        else:
            Gs = sketch_operator(l, m, s)
        Y = sketch(A, Gs)
        st, J, R, gaps = select(Y, k, rank_tol)
        if st == OK:
            P = interp(R, J)
            sigma, hist = residual(A, J, P, start_vector(n, s), q)
            return dict(status=OK, J=J, P=P, sigma=sigma, hist=hist, seed_used=s, Y=Y, R=R,
                        gaps=gaps)
        s += 1
    return dict(status=ERR_RANK, J=J, P=None, sigma=None, hist=None, seed_used=s - 1, Y=Y,
                R=None, gaps=gaps)


# --------------------------------------------------------------------------
# Downstream use: the SVD built on the ID
# --------------------------------------------------------------------------
def svd_from_id(A, J, P):
    """Rank-k SVD of the ID's approximation A(:, J) P (Sec. 1 names fast
    SVDs among the ID's uses).

    The plain definition: form the m x n product A(:, J) P and take its
    SVD with LAPACK (numpy's zgesdd), keeping the k leading triplets.
    Returns (U m x k, S k descending, V n x k) with A(:,J) P ~ U diag(S) V^H.
    """
    A = _cf(A)
    P = _cf(P)
    J = np.asarray(J, dtype=np.int64)
    k = P.shape[0]
    BP = A[:, J] @ P
    U, S, Vh = np.linalg.svd(BP, full_matrices=False)
    return np.asfortranarray(U[:, :k]), S[:k].copy(), np.asfortranarray(Vh[:k].conj().T)
