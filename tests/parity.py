"""Shared parity checks of the GPU tests against the oracle.

Pivots (Sec. 2: the permutation brings the k most weighted independent
columns to the front; the reading here is greedy pivoting on exact trailing
norms, lowest index on an exact tie).  Two implementations that round
differently may break a near-tie differently, and every later step then
works on a different set of columns.  So the oracle is re-synchronised onto
the GPU's pivots: it takes the GPU's pick at every step, after recording its
own.  Each step is then checked:
  * where the oracle's pivot gap (best - second) / best exceeds tau, the
    GPU's pick must be the oracle's own pick, bit for bit;
  * at a near-tie (gap <= tau) the GPU's pick must be valid: its trailing
    norm within a factor (1 - tau) of the best.
The oracle's R on the GPU's pivots then gives the P that the GPU's P is
compared with, entry by entry, whether or not any near-tie occurred.
"""
import numpy as np

import oracle


def check_pivots(Y, Jg, tau, rank_tol=1e-12):
    """Check the GPU's pivots Jg on the sketch Y (see the module docstring).

    Returns the oracle's forced selection (dict of select_forced) with two
    more keys: near_ties (steps checked by validity) and P, the oracle's
    interpolation matrix on the GPU's pivots.
    """
    Jg = np.asarray(Jg, dtype=np.int64)
    k = Jg.shape[0]
    assert len(np.unique(Jg)) == k, "repeated pivot"
    r = oracle.select_forced(Y, Jg, rank_tol)
    assert r["status"] == oracle.OK, r["status"]
    ties = 0
    for t in range(k):
        if r["gaps"][t] > tau:
            assert Jg[t] == r["argmax"][t], (t, Jg[t], r["argmax"][t], r["gaps"][t])
        else:
            ties += 1
            assert r["ratio"][t] >= 1.0 - tau, (t, r["ratio"][t], r["gaps"][t])
    r["near_ties"] = ties
    r["P"] = oracle.interp(r["R"], Jg)
    return r


def check_P(P, Pref, tol):
    """max |P - Pref| <= tol max(1, max |Pref|), and P(:, J) = I exactly is
    checked by the caller."""
    scale = max(1.0, float(np.abs(Pref).max()))
    err = float(np.abs(np.asarray(P) - Pref).max())
    assert err <= tol * scale, (err, tol * scale)
    return err


def sigma_on_pivots(A, Jg, Pref, seed, q, ref=None):
    """The oracle's residual for the GPU's pivots and the oracle's own P on
    them.  When the pivots equal those of an oracle run `ref` (a dict of
    oracle.decompose), its sigma is that value already."""
    Jg = np.asarray(Jg, dtype=np.int64)
    if ref is not None and np.array_equal(Jg, ref["J"]):
        return ref["sigma"], ref["hist"]
    n = np.asarray(A).shape[1]
    return oracle.residual(A, Jg, Pref, oracle.start_vector(n, seed), q)


def check_decompose(A, Y, J, P, sigma, seed, q, tau=1e-10, ptol=1e-10, ref=None,
                    rank_tol=1e-12, sigma_factor=None):
    """End-to-end check of one ID against the oracle on the GPU's pivots.

    FP64 (sigma_factor None): |dsigma| <= 1e-10 sigma + 2 ||A(:,J)||_F ||dP||_F,
    since | ||E1|| - ||E2|| | <= ||A(:,J) (P1 - P2)||.  Reduced precision:
    sigma within sigma_factor of the oracle's, both ways.
    Returns the forced oracle selection (see check_pivots) with sigma_ref.
    """
    J = np.asarray(J, dtype=np.int64)
    k = J.shape[0]
    r = check_pivots(Y, J, tau, rank_tol)
    assert np.array_equal(np.asarray(P)[:, J], np.eye(k))
    check_P(P, r["P"], ptol)
    s_ref, _ = sigma_on_pivots(A, J, r["P"], seed, q, ref)
    if sigma_factor is None:
        dP = np.asarray(P) - r["P"]
        Ac = np.asarray(A).astype(np.complex128)
        tol = 1e-10 * s_ref + 2 * np.linalg.norm(Ac[:, J]) * np.linalg.norm(dP)
        assert abs(sigma - s_ref) <= tol + 1e-300, (sigma, s_ref, tol)
    else:
        assert s_ref / sigma_factor <= sigma <= sigma_factor * s_ref, (sigma, s_ref)
    r["sigma_ref"] = s_ref
    return r


# unit roundoff of the residual's sums over A, by accumulation kind
ACC_U = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24}


def plain_sigma_tol(A, P, acc):
    """Bound on |sigma_gpu - sigma_exact| for plain (uncompensated) sums over
    A: each entry of z = A x~ (and of u = A^H z) is a sum whose rounding error
    is about u sqrt(terms) |a_i| |x~|, so ||dz|| <~ u sqrt(m + n) ||A||_F
    ||x~||, with ||x~|| <= 1 + ||P||_2 for a unit x; a direction error of x
    moves the next sigma by the same order.  Factor 10 on top."""
    Ac = np.asarray(A).astype(np.complex128)
    m, n = Ac.shape
    p2 = np.linalg.norm(np.asarray(P), 2) if np.asarray(P).size else 0.0
    return 10 * ACC_U[acc] * np.sqrt(m + n) * np.linalg.norm(Ac) * (1 + p2)


def check_sigma_call_for_call(A, J, P, sigma, seed, q, acc="dot2", hist=None):
    """The GPU's sigma is the power estimate of ||A - A(:,J) P|| for its own
    J and P: the oracle's iteration (binary128) on the same (A, J, P, start
    vector, q).  Compensated sums ("dot2") agree to 1e-10 relative; plain
    double ("fp64") or single ("fp32") sums to plain_sigma_tol.  With hist,
    every step is checked.  Returns the oracle's sigma."""
    n = np.asarray(A).shape[1]
    s_ref, h_ref = oracle.residual(A, J, P, oracle.start_vector(n, seed), q)
    if acc == "dot2":
        tol = 1e-10 * s_ref + 1e-300
        htol = 1e-10 * h_ref
    else:
        tol = htol = plain_sigma_tol(A, P, acc)
    assert abs(sigma - s_ref) <= tol, (sigma, s_ref, tol)
    if hist is not None:
        assert np.all(np.abs(np.asarray(hist) - h_ref) <= htol), (hist, h_ref, htol)
    return s_ref
