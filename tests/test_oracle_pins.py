"""Pins for the CPU oracle: each test checks the oracle against something
other than itself (published test vectors, closed forms, LAPACK/BLAS special
cases, brute force, invariants the mathematics fixes).

Paper: Lucas, Stalzer & Feo, arXiv 1205.3830.  Sec. 2 defines the steps
(randomization, pivoted approximate QR, R2 = R1 T, P = [I T]) and the error
bound eq. (errorbound); Sec. 3.3 the test matrices and the precision floor;
Table 5 the error ||A - BP||_2.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sl

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- randomness
def _kat_rows():
    rows = []
    with open(os.path.join(GOLD, "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat_rows())
def test_philox_known_answers(ctr, key, out):
    assert [int(x) for x in oracle.philox4x32_10(ctr, key)] == out


def test_gaussian_moments():
    # Complex Gaussian with Re, Im ~ N(0, 1/2): |g|^2 ~ Exp(1), so
    # E g = 0, E|g|^2 = 1, E g^2 = 0 (circular), E|g|^4 = 2, E|g|^8 = 24.
    N = 400_000
    g = oracle.gaussian(4, N // 4, seed=12345, stream=0).ravel()
    a2 = np.abs(g) ** 2
    assert abs(g.mean()) < 5 * np.sqrt(1.0 / N)
    assert abs(a2.mean() - 1.0) < 5 * np.sqrt(1.0 / N)
    assert abs((g * g).mean()) < 5 * np.sqrt(2.0 / N)
    assert abs((a2 * a2).mean() - 2.0) < 5 * np.sqrt(20.0 / N)
    assert abs(np.mean(g.real * g.imag)) < 5 * np.sqrt(0.25 / N)
    assert abs(np.mean(g.real ** 2) - 0.5) < 5 * np.sqrt(0.5 / N)


def test_gaussian_streams_and_counters_distinct():
    a = oracle.gaussian(3, 50, seed=7, stream=0)
    b = oracle.gaussian(3, 50, seed=7, stream=1)
    c = oracle.gaussian(3, 50, seed=8, stream=0)
    assert len(np.unique(np.concatenate([a.ravel(), b.ravel(), c.ravel()]))) == 450
    # entry (i, j) does not depend on the matrix shape
    big = oracle.gaussian(5, 80, seed=7, stream=0)
    assert np.array_equal(big[:3, :50], a)


# ---------------------------------------------------------------- sketch
def test_sketch_identity_operator_is_exact():
    # G = I_m (l = m) reduces the randomization to Y = A, bit for bit.
    A = synth.lowrank(37, 23, 5, 1e-3, seed=3)
    Y = oracle.sketch(A, np.eye(37, dtype=np.complex128))
    assert np.array_equal(Y, A)


@pytest.mark.parametrize("m,n,l", [(1, 1, 1), (50, 17, 9), (300, 41, 30)])
def test_sketch_matches_blas(m, n, l):
    rng = np.random.default_rng(m * 100 + n)
    A = rng.normal(size=(m, n)) + 1j * rng.normal(size=(m, n))
    G = rng.normal(size=(l, m)) + 1j * rng.normal(size=(l, m))
    Y = oracle.sketch(A, G)
    ref = G @ A
    assert np.linalg.norm(Y - ref) <= 1e-14 * np.sqrt(m) * np.linalg.norm(ref)


def test_sketch_seeded_columns_match_explicit_operator():
    A = synth.lowrank(64, 9, 3, 1e-6, seed=1)
    G = oracle.sketch_operator(11, 64, seed=5)
    Y = oracle.sketch(A, G)
    Yc = oracle.sketch_seeded_columns(A[:, [2, 7]], 11, seed=5)
    assert np.array_equal(Yc, Y[:, [2, 7]])


# ---------------------------------------------------------------- selection
def _greedy_bruteforce(Y, k):
    """Step t: for every unselected column, the norm of its component
    orthogonal to the selected ones, by least squares (independent of QR)."""
    n = Y.shape[1]
    J = []
    for _ in range(k):
        best, bj = -1.0, -1
        for j in range(n):
            if j in J:
                continue
            if J:
                B = Y[:, J]
                c = np.linalg.lstsq(B, Y[:, j], rcond=None)[0]
                r = Y[:, j] - B @ c
            else:
                r = Y[:, j]
            nr = np.linalg.norm(r)
            if nr > best * (1 + 1e-12):
                best, bj = nr, j
        J.append(bj)
    return J


@pytest.mark.parametrize("seed", range(8))
def test_select_matches_bruteforce_tiny(seed):
    rng = np.random.default_rng(seed)
    l, n = rng.integers(3, 9), rng.integers(4, 12)
    k = int(rng.integers(1, min(l, n, 4) + 1))
    Y = rng.normal(size=(l, n)) + 1j * rng.normal(size=(l, n))
    st, J, R, gaps = oracle.select(Y, k)
    assert st == oracle.OK
    assert list(J) == _greedy_bruteforce(Y, k)


def test_select_forced_on_its_own_picks_is_the_plain_selection():
    Y = synth.lowrank(40, 300, 25, 1e-9, seed=21)
    st, J, R, gaps = oracle.select(Y, 25)
    r = oracle.select_forced(Y, J)
    assert st == r["status"] == oracle.OK
    assert np.array_equal(r["J"], J) and np.array_equal(r["argmax"], J)
    assert np.array_equal(r["R"], R) and np.array_equal(r["gaps"], gaps)
    assert np.all(r["ratio"] == 1.0)
    # -1 entries leave the step free: the same as no forcing at all
    r2 = oracle.select_forced(Y, np.full(25, -1))
    assert np.array_equal(r2["J"], J) and np.array_equal(r2["R"], R)


def test_select_forced_follows_the_forced_pivots():
    # forcing step 0 onto another column: that column is taken, and every
    # later step is the greedy choice among what is left, which equals the
    # plain selection of Y with the forced column moved out of the way first
    Y = synth.lowrank(30, 120, 12, 1e-9, seed=22)
    st, J, R, gaps = oracle.select(Y, 12)
    f = np.full(12, -1)
    f[0] = J[1]
    r = oracle.select_forced(Y, f)
    assert r["status"] == oracle.OK and r["J"][0] == J[1] and r["argmax"][0] == J[0]
    nrm = np.linalg.norm(Y, axis=0)
    assert r["ratio"][0] == pytest.approx(nrm[J[1]] / nrm[J[0]], rel=1e-14)
    # later picks are greedy on the projection orthogonal to Y(:, J[1])
    assert list(r["J"]) == [J[1]] + _greedy_bruteforce_after(Y, [int(J[1])], 11)
    # R is Q^H Y for the forced order: R1 upper triangular, T = lstsq
    R1 = r["R"][:, r["J"]]
    assert np.allclose(np.tril(R1, -1), 0, atol=1e-12 * np.abs(R1).max())
    P = oracle.interp(r["R"], r["J"])
    others = np.setdiff1d(np.arange(120), r["J"])
    T = np.linalg.lstsq(Y[:, r["J"]], Y[:, others], rcond=None)[0]
    assert np.abs(P[:, others] - T).max() <= 1e-10 * max(1, np.abs(T).max())
    bad = r["J"].copy()
    bad[3] = bad[2]
    assert oracle.select_forced(Y, bad)["status"] == oracle.ERR_ARG     # repeated column


def _greedy_bruteforce_after(Y, first, k):
    n = Y.shape[1]
    J = list(first)
    for _ in range(k):
        B = Y[:, J]
        best, bj = -1.0, -1
        for j in range(n):
            if j in J:
                continue
            r = Y[:, j] - B @ np.linalg.lstsq(B, Y[:, j], rcond=None)[0]
            if np.linalg.norm(r) > best * (1 + 1e-12):
                best, bj = np.linalg.norm(r), j
        J.append(bj)
    return J[len(first):]


def test_parity_checker_accepts_near_tie_swaps_and_rejects_wrong_picks():
    # the shared GPU-test check (tests/parity.py) on planted pivot lists: a
    # near-tie broken the other way passes, a wrong pick at a clear gap fails
    from parity import check_pivots
    rng = np.random.default_rng(4)
    l, n, k = 20, 80, 10
    Y = (rng.standard_normal((l, n)) + 1j * rng.standard_normal((l, n))) / np.sqrt(2)
    Y[:, 5] *= 4.0
    Y[:, 9] = Y[:, 5] * np.exp(0.7j)            # near-tie with column 5 at step 0
    Y = np.asfortranarray(Y)
    st, J, R, gaps = oracle.select(Y, k)
    assert gaps[0] <= 1e-10 and J[0] in (5, 9)
    other = 9 if J[0] == 5 else 5
    swapped = oracle.select_forced(Y, np.r_[other, np.full(k - 1, -1)])["J"]
    r = check_pivots(Y, swapped, 1e-10)
    assert r["near_ties"] >= 1
    assert np.array_equal(r["P"][:, swapped], np.eye(k))
    wrong = J.copy()
    wrong[3], wrong[4] = J[4], J[3]
    assert gaps[3] > 1e-6
    with pytest.raises(AssertionError):
        check_pivots(Y, wrong, 1e-10)


def test_id_error_against_the_best_column_subsets_tiny():
    # brute force over every k-subset J' on tiny inputs: the best column
    # subset's error min ||(I - Pi_J') A||_2 bounds the ID's error from below
    # (the ID's P is one choice of coefficients for its own J), and the ID's
    # error stays within eq. (3) (eps = 1e-10); the ratio to the optimum is
    # reported.  A plausible mistake in the selection or the solve (a wrong
    # pivot, a transposed or conjugated T) pushes the ID above the optimum
    # by orders of magnitude on these near-low-rank inputs.
    from itertools import combinations
    ratios = []
    for seed in range(6):
        rng = np.random.default_rng(100 + seed)
        m, n = int(rng.integers(6, 11)), int(rng.integers(6, 13))
        k = int(rng.integers(1, 4))
        A = synth.lowrank(m, n, k, 1e-6, seed=200 + seed)
        r = oracle.decompose(A, k, min(m, k + 3), seed=seed, q=30)
        assert r["status"] == oracle.OK
        err = np.linalg.norm(A - A[:, r["J"]] @ r["P"], 2)
        best = min(np.linalg.norm(A - A[:, list(c)] @ np.linalg.lstsq(A[:, list(c)], A,
                                                                       rcond=None)[0], 2)
                   for c in combinations(range(n), k))
        s = np.linalg.svd(A, compute_uv=False)
        assert s[k] <= best * (1 + 1e-9)            # Eckart-Young below the best subset
        assert best <= err * (1 + 1e-9)
        assert err <= 50 * np.sqrt(m * n) * (1e10) ** (1.0 / k) * s[k]
        assert r["sigma"] <= err * (1 + 1e-9)       # the power estimate is from below
        ratios.append(err / best)
    print("ID error / best-subset error: %s" % ", ".join("%.3f" % x for x in ratios))
    assert max(ratios) < 10.0


@pytest.mark.parametrize("l,n,k", [(30, 500, 20), (60, 200, 40), (12, 12, 12)])
def test_select_matches_lapack_zgeqp3(l, n, k):
    A = synth.lowrank(400, n, k, 1e-8, seed=l)
    Y = oracle.sketch(A, oracle.sketch_operator(l, 400, seed=1))
    st, J, R, gaps = oracle.select(Y, k)
    assert st == oracle.OK
    _, _, piv = sl.qr(Y, pivoting=True, mode="economic")
    assert np.array_equal(J, piv[:k])
    assert gaps.min() > 1e-8


def test_select_R_is_upper_triangular_with_decreasing_diagonal():
    A = synth.lowrank(300, 120, 15, 1e-9, seed=4)
    Y = oracle.sketch(A, oracle.sketch_operator(25, 300, seed=2))
    st, J, R, _ = oracle.select(Y, 15)
    R1 = R[:, J]
    assert np.abs(np.tril(R1, -1)).max() <= 1e-13 * np.abs(R1).max()
    d = np.abs(np.diag(R1))
    assert np.all(np.diff(d) <= 1e-12 * d[0])
    # R = Q^H Y with orthonormal Q: column norms of R1 match those of Y(:, J)
    assert np.allclose(np.linalg.norm(R1, axis=0), np.linalg.norm(Y[:, J], axis=0), rtol=1e-13)


def test_select_rank_one_closed_form():
    rng = np.random.default_rng(0)
    x = rng.normal(size=7) + 1j * rng.normal(size=7)
    y = rng.normal(size=20) + 1j * rng.normal(size=20)
    Y = np.outer(x, y.conj())
    st, J, R, _ = oracle.select(Y, 1)
    assert st == oracle.OK and J[0] == int(np.argmax(np.abs(y)))
    P = oracle.interp(R, J)
    assert np.allclose(P[0], np.conj(y / y[J[0]]), rtol=1e-13, atol=1e-15)
    assert np.abs(P).max() <= 1 + 1e-13


def test_select_rank_failure():
    # rank(Y) = 3 < k = 4: the Sec. 2 failure case.
    rng = np.random.default_rng(1)
    Y = (rng.normal(size=(10, 3)) + 1j * rng.normal(size=(10, 3))) @ (
        rng.normal(size=(3, 30)) + 1j * rng.normal(size=(3, 30)))
    st, J, R, gaps = oracle.select(Y, 4)
    assert st == oracle.ERR_RANK
    st, J, R, gaps = oracle.select(Y, 3)
    assert st == oracle.OK


def test_select_zero_matrix_is_rank_failure():
    st, _, _, _ = oracle.select(np.zeros((4, 5)), 1)
    assert st == oracle.ERR_RANK


def test_identity_operator_reduces_to_pivoted_qr_of_A():
    # With G = I the ID is the deterministic pivoted-QR ID of A itself.
    A = synth.lowrank(40, 60, 6, 1e-7, seed=9)
    Y = oracle.sketch(A, np.eye(40, dtype=np.complex128))
    st, J, R, _ = oracle.select(Y, 6)
    _, _, piv = sl.qr(A, pivoting=True, mode="economic")
    assert np.array_equal(J, piv[:6])


# ---------------------------------------------------------------- interpolation
@pytest.mark.parametrize("l,n,k", [(30, 500, 20), (9, 9, 9), (5, 40, 1)])
def test_interp_matches_least_squares(l, n, k):
    A = synth.lowrank(300, n, k, 1e-10, seed=n)
    Y = oracle.sketch(A, oracle.sketch_operator(l, 300, seed=3))
    st, J, R, _ = oracle.select(Y, k)
    P = oracle.interp(R, J)
    # P(:, J) = I exactly
    assert np.array_equal(P[:, J], np.eye(k))
    Jc = np.setdiff1d(np.arange(n), J)
    if len(Jc):
        T = sl.lstsq(Y[:, J], Y[:, Jc], lapack_driver="gelsd")[0]
        assert np.abs(P[:, Jc] - T).max() <= 1e-11 * max(1.0, np.abs(T).max())
    assert np.abs(P).max() <= 2.0


def test_interp_rejects_bad_pivots():
    R = np.eye(2, 4, dtype=np.complex128)
    with pytest.raises(ValueError):
        oracle.interp(R, [0, 0])
    with pytest.raises(ValueError):
        oracle.interp(R, [0, 9])


# ---------------------------------------------------------------- hand example
def _hand_rows():
    rows = []
    with open(os.path.join(GOLD, "hand_example.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, J, P, e = [s.strip() for s in line.split("|")]
            P = np.array([[float(v) for v in r.split()] for r in P.split(";")])
            rows.append((int(k), [int(v) for v in J.split()], P, float(e)))
    return rows


@pytest.mark.parametrize("k,J,P,normE", _hand_rows())
def test_hand_example(k, J, P, normE):
    A = synth.hand_example()
    r = oracle.decompose(A, k, 2, seed=0, q=4, G=np.eye(2, dtype=np.complex128))
    assert r["status"] == oracle.OK
    assert list(r["J"]) == J
    assert np.array_equal(r["P"], P.astype(np.complex128))
    if normE == 0:
        # E = 0 exactly; the binary128 iteration leaves only quad rounding
        assert r["sigma"] <= 1e-30
    else:
        assert abs(r["sigma"] - normE) <= 4e-16 * normE
        assert abs(r["hist"][1] - normE) <= 4e-16 * normE


# ---------------------------------------------------------------- residual
def _power_iteration_longdouble(A, J, P, x0, q):
    """Independent check of the power iteration: E formed explicitly in
    80-bit extended precision, then plain iteration x <- E^H E x."""
    Al = A.astype(np.clongdouble)
    E = Al - Al[:, J] @ P.astype(np.clongdouble)
    x = x0.astype(np.clongdouble)
    x = x / np.sqrt(np.sum(np.abs(x) ** 2))
    hist = []
    for t in range(q):
        z = E @ x
        hist.append(float(np.sqrt(np.sum(np.abs(z) ** 2))))
        w = E.conj().T @ z
        x = w / np.sqrt(np.sum(np.abs(w) ** 2))
    return np.array(hist)


def test_residual_matches_extended_precision_iteration():
    # noise 1e-6: E is ~1e-7 of A, so 80-bit E keeps ~12 digits.
    A = synth.lowrank(120, 80, 6, 1e-6, seed=2)
    r = oracle.decompose(A, 6, 12, seed=4, q=6)
    ref = _power_iteration_longdouble(A, r["J"], r["P"], oracle.start_vector(80, 4), 6)
    assert np.allclose(r["hist"], ref, rtol=1e-9, atol=0)


def test_residual_converges_to_spectral_norm_and_stays_below_it():
    # A rank-1 perturbation on top of the low-rank part gives E a dominant
    # singular value, so the iteration converges quickly to ||E||_2.
    rng = np.random.default_rng(5)
    A = synth.lowrank(200, 90, 8, 0.0, seed=5)
    u = rng.normal(size=200) + 1j * rng.normal(size=200)
    v = rng.normal(size=90) + 1j * rng.normal(size=90)
    A = np.asfortranarray(A + 1e-3 * np.outer(u, v.conj()) + 1e-9 * rng.normal(size=(200, 90)))
    r = oracle.decompose(A, 8, 16, seed=1, q=30)
    E = A - A[:, r["J"]] @ r["P"]
    nE = np.linalg.norm(E, 2)
    h = r["hist"]
    assert np.all(np.diff(h) >= -1e-14 * h[-1])          # non-decreasing
    assert np.all(h <= nE * (1 + 1e-10))                  # below ||E||_2
    assert abs(h[-1] - nE) <= 1e-10 * nE


def test_residual_error_bounds():
    # Eckart-Young lower bound and eq. (errorbound) upper bound with eps=1e-10.
    m, n, k = 300, 200, 10
    A = synth.lowrank(m, n, k, 1e-8, seed=6)
    r = oracle.decompose(A, k, k + 10, seed=0, q=12)
    s = np.linalg.svd(A, compute_uv=False)
    E = A - A[:, r["J"]] @ r["P"]
    nE = np.linalg.norm(E, 2)
    assert s[k] <= nE * (1 + 1e-8)
    bound = 50 * np.sqrt(m * n) * (1e10) ** (1.0 / k) * s[k]
    assert r["sigma"] <= bound
    assert r["sigma"] >= 0.5 * nE   # the iteration has (nearly) converged


def test_residual_exact_rank_k_is_at_rounding_level():
    # Noise-free rank-k A: ||A - BP|| is at the rounding floor (Sec. 3.3).
    m, n, k = 500, 300, 12
    A = synth.lowrank(m, n, k, 0.0, seed=8)
    r = oracle.decompose(A, k, k + 8, seed=0, q=8)
    nA = np.linalg.norm(A, 2)
    assert r["sigma"] <= 10 * np.sqrt(m + n) * np.finfo(float).eps * nA


def test_residual_zero_error_and_early_stop():
    # k = 2 on the hand example: E = 0, so the estimate is quad rounding only.
    A = synth.hand_example()
    s, hist = oracle.residual(A, [0, 1], np.array([[1, 0, 0.5], [0, 1, 1]]),
                              oracle.start_vector(3, 0), 5)
    assert s <= 1e-30 and np.all(hist <= 1e-30)
    # A = 0: E x = 0 exactly, E^H z = 0, the iteration stops and keeps 0.
    s, hist = oracle.residual(np.zeros((2, 3)), [0], np.array([[1, 0, 0.5]]),
                              oracle.start_vector(3, 0), 5)
    assert s == 0.0 and np.all(hist == 0.0)


# ---------------------------------------------------------------- metamorphic
def test_scaling_by_two_is_exact():
    A = synth.lowrank(150, 70, 7, 1e-9, seed=11)
    r1 = oracle.decompose(A, 7, 12, seed=2, q=5)
    r2 = oracle.decompose(2 * A, 7, 12, seed=2, q=5)
    assert np.array_equal(r1["J"], r2["J"])
    assert np.array_equal(r1["P"], r2["P"])
    assert r2["sigma"] == 2 * r1["sigma"]


def test_column_permutation_permutes_J_and_P():
    A = synth.lowrank(150, 70, 7, 1e-9, seed=12)
    pi = np.random.default_rng(3).permutation(70)
    G = oracle.sketch_operator(12, 150, seed=3)
    r1 = oracle.decompose(A, 7, 12, seed=3, q=5, G=G)
    Ap = np.asfortranarray(A[:, pi])
    r2 = oracle.decompose(Ap, 7, 12, seed=3, q=5, G=G)
    inv = np.argsort(pi)
    assert np.array_equal(pi[r2["J"]], r1["J"])
    assert np.array_equal(r2["P"], r1["P"][:, pi])
    # same start vector, permuted: same residual up to summation order
    x0 = oracle.start_vector(70, 3)
    s1, _ = oracle.residual(A, r1["J"], r1["P"], x0, 5)
    s2, _ = oracle.residual(Ap, r2["J"], r2["P"], x0[pi], 5)
    assert abs(s1 - s2) <= 1e-14 * s1
    assert inv.shape == (70,)


# ---------------------------------------------------------------- failure path
def test_decompose_rank_deficient_input_fails_every_draw():
    A = synth.lowrank(60, 40, 3, 0.0, seed=13)    # rank 3
    r = oracle.decompose(A, 4, 8, seed=0, q=3, max_retries=2)
    assert r["status"] == oracle.ERR_RANK and r["seed_used"] == 2


def test_decompose_rank_deficient_operator_then_fresh_draw_succeeds():
    A = synth.lowrank(60, 40, 4, 1e-9, seed=14)
    G = np.zeros((6, 60), dtype=np.complex128)
    G[:3] = oracle.sketch_operator(3, 60, seed=0)   # rank(G) = 3 < k
    assert oracle.decompose(A, 4, 6, seed=0, q=3, G=G)["status"] == oracle.ERR_RANK
    r = oracle.decompose(A, 4, 6, seed=0, q=3)
    assert r["status"] == oracle.OK


def test_precision_floor_of_noise_free_products():
    # Sec. 3.3: rounding of A = X W alone leaves sigma_{k+1} of order
    # sqrt(2 min(m,n)) * 1e-16 relative to the entries.
    A = synth.lowrank(256, 128, 8, 0.0, seed=15)
    s = np.linalg.svd(A, compute_uv=False)
    floor = np.sqrt(2 * 128) * 1e-16 * np.abs(A).max()
    assert s[8] < 100 * floor


# ---------------------------------------------------------------- S F D (eqs. (4)-(7))
@pytest.mark.parametrize("m,n,l", [(64, 5, 10), (1000, 7, 30), (97, 3, 40)])
def test_srft_operator_equals_sampled_fft(m, n, l):
    # Y = S F D A computed the long way: phases, a full FFT down each column
    # (numpy), then the sampled rows -- against the operator product.
    rng = np.random.default_rng(m)
    A = rng.normal(size=(m, n)) + 1j * rng.normal(size=(m, n))
    G = oracle.srft_operator(l, m, seed=3)
    s = oracle.srft_rows(l, m, seed=3)
    ph = oracle.srft_phases(m, seed=3)
    Yf = np.fft.fft(np.exp(2j * np.pi * ph)[:, None] * A, axis=0)[s, :]
    Y = oracle.sketch(A, G)
    assert np.abs(Y - Yf).max() <= 1e-13 * np.sqrt(m) * np.abs(Yf).max()
    assert np.allclose(np.abs(G), 1.0, rtol=0, atol=1e-15)


def test_srft_rows_and_phases_are_uniform():
    m, l = 10, 20000
    s = oracle.srft_rows(l, m, seed=1)
    counts = np.bincount(s, minlength=m)
    expected = l / m
    chi2 = np.sum((counts - expected) ** 2 / expected)
    assert chi2 < 40.0                                     # 9 dof, far tail
    assert len(np.unique(oracle.srft_rows(30, 40, seed=2))) < 30   # drawn with replacement
    ph = oracle.srft_phases(50000, seed=4)
    assert abs(ph.mean() - 0.5) < 5 * np.sqrt(1 / 12 / 50000)
    assert abs(ph.var() - 1 / 12) < 5e-3
    assert ph.min() > 0.0 and ph.max() < 1.0


def test_srft_decompose_matches_pivoted_qr_of_its_sketch():
    A = synth.lowrank(1000, 500, 20, 1e-10, seed=0)
    r = oracle.decompose(A, 20, 40, seed=0, q=6, kind="srft")
    assert r["status"] == oracle.OK
    _, _, piv = sl.qr(r["Y"], pivoting=True, mode="economic")
    assert np.array_equal(r["J"], piv[:20])
    E = A - A[:, r["J"]] @ r["P"]
    assert r["sigma"] <= np.linalg.norm(E, 2) * (1 + 1e-6)


# ---------------------------------------------------------------- SVD on the ID
def test_svd_from_id_rank_one_closed_form():
    # A = sigma x y^H with unit x, y: the ID of rank 1 is exact, so the one
    # singular triplet is (sigma, x, y) up to a common phase.
    rng = np.random.default_rng(11)
    x = rng.normal(size=40) + 1j * rng.normal(size=40)
    y = rng.normal(size=25) + 1j * rng.normal(size=25)
    x /= np.linalg.norm(x)
    y /= np.linalg.norm(y)
    sigma = 3.75
    A = np.asfortranarray(sigma * np.outer(x, y.conj()))
    r = oracle.decompose(A, 1, 4, seed=2, q=4)
    U, S, V = oracle.svd_from_id(A, r["J"], r["P"])
    assert U.shape == (40, 1) and S.shape == (1,) and V.shape == (25, 1)
    assert abs(S[0] - sigma) < 1e-13 * sigma
    assert abs(abs(np.vdot(x, U[:, 0])) - 1.0) < 1e-13
    assert abs(abs(np.vdot(y, V[:, 0])) - 1.0) < 1e-13
    # the phases of u and v agree: u S v^H reproduces A itself
    assert np.abs(U * S @ V.conj().T - A).max() < 1e-13 * sigma


@pytest.mark.parametrize("m,n,k", [(120, 90, 8), (60, 200, 13)])
def test_svd_from_id_recovers_a_prescribed_spectrum(m, n, k):
    # A = U0 diag(s0) V0^H has rank k exactly, so A(:,J) P = A up to
    # rounding: S must be s0 and every pair must satisfy A v_i = s_i u_i and
    # A^H u_i = s_i v_i for A itself.
    s0 = np.logspace(0, -6, k)
    A = synth.with_spectrum(m, n, s0, seed=k)
    r = oracle.decompose(A, k, k + 6, seed=5, q=4)
    U, S, V = oracle.svd_from_id(A, r["J"], r["P"])
    assert np.abs(S - s0).max() < 1e-12
    assert np.abs(A @ V - U * S).max() < 1e-12
    assert np.abs(A.conj().T @ U - V * S).max() < 1e-12


def test_svd_from_id_weyl_and_optimality_bounds():
    # With noise A is not of rank k: Weyl's inequality bounds each singular
    # value of A(:,J) P by the ID's error E, and no rank-k matrix beats
    # sigma_{k+1}(A) (Eckart-Young).
    m, n, k = 150, 110, 10
    A = synth.lowrank(m, n, k, noise=1e-6, seed=21)
    r = oracle.decompose(A, k, 2 * k, seed=3, q=4)
    U, S, V = oracle.svd_from_id(A, r["J"], r["P"])
    sA = np.linalg.svd(A, compute_uv=False)
    normE = np.linalg.norm(A - A[:, r["J"]] @ r["P"], 2)
    assert np.all(np.abs(S - sA[:k]) <= normE * (1 + 1e-9) + 1e-12 * sA[0])
    assert np.linalg.norm(A - U * S @ V.conj().T, 2) >= sA[k] * (1 - 1e-9)
    assert np.all(np.diff(S) <= 0) and S[-1] >= 0
    assert np.abs(U.conj().T @ U - np.eye(k)).max() < 1e-13
    assert np.abs(V.conj().T @ V - np.eye(k)).max() < 1e-13
