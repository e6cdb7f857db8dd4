"""Seeded synthetic inputs for the randomized ID.

This module holds none of the method's arithmetic: it only builds test
matrices.  Both the oracle side and the GPU side of every test and benchmark
take their inputs from here.

Recipe (after the benchmark matrices of arXiv 1205.3830, Sec. 3.3, which are
products of complex Gaussian factors of the right shapes, hence of exact
rank k up to rounding):

    A = X W + c N,   X m x k, W k x n, N m x n,

with every entry of X, W, N i.i.d. complex Gaussian, real and imaginary parts
each N(0, 1/2) (so E|x|^2 = 1).  c is the noise level that sets
sigma_{k+1}(A) ~ c (sqrt(m) + sqrt(n)).  Small inputs are generated on the
host with numpy's PCG64 (seeded per factor); large inputs are generated on the
GPU with torch's seeded device generator and never leave the device.
"""
from __future__ import annotations

import numpy as np


def _cgauss(rng: np.random.Generator, shape) -> np.ndarray:
    s = np.sqrt(0.5)
    return rng.normal(0.0, s, shape) + 1j * rng.normal(0.0, s, shape)


def lowrank(m: int, n: int, k: int, noise: float, seed: int = 0,
            dtype=np.complex128) -> np.ndarray:
    """Host A = X W + noise * N, Fortran order (column-major)."""
    ss = np.random.SeedSequence(seed)
    rx, rw, rn = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(3)]
    X = _cgauss(rx, (m, k))
    W = _cgauss(rw, (k, n))
    A = X @ W
    if noise != 0.0:
        A = A + noise * _cgauss(rn, (m, n))
    return np.asfortranarray(A.astype(dtype))


def lowrank_device(m: int, n: int, k: int, noise: float, seed: int = 0,
                   dtype=None, device="cuda", col_chunk: int = 2048):
    """Device A = X W + noise * N as a column-major torch tensor.

    Returns a tensor T of shape (n, m) (row j of T is column j of A, so T's
    memory is A in column-major order with lda = m).  Built in column chunks
    so that the peak extra memory is one chunk of N.
    """
    import torch
    if dtype is None:
        dtype = torch.complex128
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    rdt = torch.float64 if dtype == torch.complex128 else torch.float32
    s = 0.5 ** 0.5

    def cg(shape):
        re = torch.randn(shape, generator=g, device=device, dtype=rdt) * s
        im = torch.randn(shape, generator=g, device=device, dtype=rdt) * s
        return torch.complex(re, im)

    X = cg((m, k)).to(torch.complex128)
    W = cg((k, n)).to(torch.complex128)
    T = torch.empty((n, m), dtype=dtype, device=device)
    for j0 in range(0, n, col_chunk):
        j1 = min(n, j0 + col_chunk)
        blk = (W[:, j0:j1].transpose(0, 1).contiguous() @ X.transpose(0, 1).contiguous())
        if noise != 0.0:
            blk = blk + noise * cg((j1 - j0, m)).to(torch.complex128)
        T[j0:j1] = blk.to(dtype)
        del blk
    del X, W
    return T


def with_spectrum(m: int, n: int, s, seed: int = 0) -> np.ndarray:
    """Host A = U0 diag(s) V0^H, Fortran order, with U0 (m x r) and V0 (n x r)
    orthonormal (QR of complex Gaussian factors), r = len(s): the singular
    values of A are the entries of s (up to rounding)."""
    s = np.asarray(s, dtype=np.float64)
    r = s.shape[0]
    ss = np.random.SeedSequence(seed)
    ru, rv = [np.random.Generator(np.random.PCG64(x)) for x in ss.spawn(2)]
    U0, _ = np.linalg.qr(_cgauss(ru, (m, r)))
    V0, _ = np.linalg.qr(_cgauss(rv, (n, r)))
    return np.asfortranarray((U0 * s) @ V0.conj().T)


def hand_example():
    """The 2 x 3 integer matrix used as a worked example in the tests."""
    return np.asfortranarray(np.array([[2, 0, 1], [0, 1, 1]], dtype=np.complex128))
