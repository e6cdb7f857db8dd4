"""Parity at the full benchmark sizes, in the launch configuration bench.py
times: A = X W + 1e-12 N, complex128, q = 10, at m = 131072, n = 16384,
k = 100, l = 108 (34.4 GB on the device), at the square case
m = n = 32768, k = 200, l = 208 (17.2 GB), and at the served workload's big
job m = 262144, n = 16384, k = 64, l = 72 (68.7 GB).

The oracle cannot redo a 34 GB ID in seconds, so this checks
  * sampled columns of Y against the oracle, one column at a time;
  * J and P against the oracle's selection and interpolation run on the
    library's own Y (108 x 16384 and 208 x 32768 take seconds on the host):
    J bit-exact at every step whose pivot gap exceeds 1e-10 (valid picks at
    near-ties, with the oracle forced onto the library's picks), P within
    1e-10 entry by entry;
  * P(:, J) = I exactly, |P| <= 2, and the least-squares normal equations
    Y(:,J)^H (Y(:,J) P(:,j) - Y(:,j)) = 0 on sampled columns;
  * sigma: non-decreasing power steps, Eckart-Young and eq. (3) bounds from
    the known noise level, and sigma >= the exact norm of sampled columns of
    E = A - A(:,J) P (80-bit arithmetic on the host).
"""
import numpy as np
import pytest

import oracle
import synth
from parity import check_P, check_pivots

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
rid = pytest.importorskip("paper_1205_3830_amd")

Q, NOISE = 10, 1e-12
# the two shapes of the large workload: 131072 x 16384, k = 100, l = 108, and
# the square case 32768 x 32768, k = 200, l = 208; and the served workload's
# big job, 262144 x 16384, k = 64, l = 72 (68.7 GB)
SHAPES = [(131072, 16384, 100, 108), (32768, 32768, 200, 208), (262144, 16384, 64, 72)]


@pytest.fixture(scope="module", params=SHAPES,
                ids=["131072x16384", "32768x32768", "262144x16384"])
def big(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    M, N, K, L = request.param
    free, _ = torch.cuda.mem_get_info()
    if free < 16.0 * M * N * 1.3 + 20e9:
        pytest.skip("needs %.0f GB of free device memory" % ((16.0 * M * N * 1.3 + 20e9) / 1e9))
    A = synth.lowrank_device(M, N, K, NOISE, seed=0).t()
    h = rid.rid_create(0)
    rid.rid_reserve(h, M, N, L, K)
    J, P, sigma, used = rid.rid_decompose(h, A, K, L, seed=0, q=Q)
    Y = rid.rid_sketch(h, A, L, used)
    sig, hist = rid.rid_residual(h, A, J, P, Q, used)
    torch.cuda.synchronize()
    out = dict(A=A, h=h, J=J.cpu().numpy(), P=P.cpu().numpy(), sigma=float(sigma.cpu()[0]),
               Y=Y.cpu().numpy(), hist=hist.cpu().numpy(), sigma2=float(sig.cpu()[0]), seed=used,
               shape=(M, N, K, L))
    yield out
    rid.rid_destroy(h)
    del out["A"]
    torch.cuda.empty_cache()


def test_fullsize_sampled_sketch_columns(big):
    M, N, K, L = big["shape"]
    cols = [0, 1, 63, 64, 8191, N - 1]
    Ah = big["A"][:, cols].t().contiguous().cpu().numpy().T
    ref = oracle.sketch_seeded_columns(Ah, L, big["seed"])
    Y = big["Y"][:, cols]
    for c in range(len(cols)):
        assert np.linalg.norm(Y[:, c] - ref[:, c]) <= 1e-12 * np.linalg.norm(ref[:, c])


def test_fullsize_pivots_and_P_match_oracle(big):
    # the library's own full-size sketch, re-selected and re-interpolated by
    # the oracle; the library's rid_pivqr on the same Y gives the same J
    M, N, K, L = big["shape"]
    Y, J, P = big["Y"], big["J"], big["P"]
    r = check_pivots(Y, J, 1e-10)
    assert np.array_equal(P[:, J], np.eye(K))
    err = check_P(P, r["P"], 1e-10)
    print("full size %dx%d: J equal on %d of %d steps (near-ties %d), max|dP| %.2e, "
          "min gap %.2e" % (M, N, K - r["near_ties"], K, r["near_ties"], err, r["gaps"].min()))
    Yd = torch.from_numpy(np.ascontiguousarray(Y.T)).cuda().t()
    perm, _ = rid.rid_pivqr(big["h"], Yd, K)
    assert np.array_equal(perm[:K].cpu().numpy(), J)


def test_fullsize_interpolation_matrix(big):
    M, N, K, L = big["shape"]
    P, J, Y = big["P"], big["J"], big["Y"]
    assert np.array_equal(P[:, J], np.eye(K))
    assert np.abs(P).max() <= 2.0
    YJ = Y[:, J]
    rng = np.random.default_rng(0)
    others = np.setdiff1d(np.arange(N), J)
    for j in rng.choice(others, 16, replace=False):
        r = YJ @ P[:, j] - Y[:, j]
        g = YJ.conj().T @ r
        scale = np.linalg.norm(YJ, 2) * (np.linalg.norm(YJ, 2) * np.linalg.norm(P[:, j]) +
                                         np.linalg.norm(Y[:, j]))
        assert np.linalg.norm(g) <= 1e-10 * scale


def test_fullsize_residual(big):
    M, N, K, L = big["shape"]
    s, hist = big["sigma"], big["hist"]
    assert s == big["sigma2"]                              # decompose == residual call
    assert np.all(np.diff(hist) >= -1e-12 * hist[-1])      # power steps do not decrease
    lo = NOISE * (np.sqrt(M) - np.sqrt(N))                 # sigma_min of the noise part
    hi = NOISE * (np.sqrt(M) + np.sqrt(N))
    assert s >= 0.5 * lo
    assert s <= 50 * np.sqrt(M * N) * (1e10) ** (1.0 / K) * 1.1 * hi   # eq. (3), eps = 1e-10
    # ||E||_2 >= ||E e_j|| for every column j; compute a few exactly on the host
    J, P = big["J"], big["P"]
    AJ = big["A"][:, J.tolist()].t().contiguous().cpu().numpy().T.astype(np.clongdouble)
    cols = [int(c) for c in np.setdiff1d(np.arange(N), J)[:: N // 6][:6]]
    Ac = big["A"][:, cols].t().contiguous().cpu().numpy().T.astype(np.clongdouble)
    col_norms = [float(np.sqrt(np.sum(np.abs(Ac[:, i] - AJ @ P[:, c].astype(np.clongdouble)) ** 2)))
                 for i, c in enumerate(cols)]
    assert s >= 0.9 * max(col_norms)


def test_fullsize_svd_on_the_id(big):
    M, N, K, L = big["shape"]
    # The SVD built on the ID at full size, by properties that hold at any
    # size: orthonormal U and V, descending S, U S V^H = A(:,J) P on sampled
    # columns, and, on sampled rows, A V - U S = E V with E = A - A(:,J) P,
    # so each row is at most ||E||_2 (~ sigma, the power estimate) long.
    A, J, P = big["A"], big["J"], big["P"]
    Pd = torch.from_numpy(np.ascontiguousarray(P.T)).cuda().t()
    U, S, V, sweeps = rid.rid_svd(big["h"], A, torch.from_numpy(J).cuda(), Pd)
    U, S, V = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
    assert 1 <= sweeps < 60
    assert np.all(np.diff(S) <= 0.0) and S[-1] > 0.0
    s0 = S[0]
    assert np.abs(U.conj().T @ U - np.eye(K)).max() <= 1e-11
    assert np.abs(V.conj().T @ V - np.eye(K)).max() <= 1e-11
    AJ = A[:, J.tolist()].t().contiguous().cpu().numpy().T
    for c in [0, 1, 4097, N - 1] + [int(J[0]), int(J[-1])]:
        rec = (U * S) @ V[c].conj()
        assert np.abs(rec - AJ @ P[:, c]).max() <= 1e-11 * s0, c
    rows = [0, 5, M // 2, M - 1]
    Ar = A[rows, :].cpu().numpy()
    for i, r in enumerate(rows):
        assert np.linalg.norm(Ar[i] @ V - U[r] * S) <= 4 * big["sigma"] + 1e-11 * s0, r
