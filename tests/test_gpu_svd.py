"""GPU parity of the SVD built on the ID (rid_svd) against the oracle's
definition, the LAPACK SVD of A(:,J) P (arXiv 1205.3830, Sec. 1 lists fast
SVDs among the ID's uses).  J and P come from the oracle's own ID of the same
A; both sides take them as inputs.

Tolerances (FP64, tau = 1e-12 relative to S_0 = ||A(:,J) P||_2):
  S       : |dS_i| <= tau S_0.  The GPU result is the exact SVD of
            A(:,J) P + F with ||F|| a modest multiple of u sqrt(m) k S_0
            (CholeskyQR3's and Jacobi's backward errors; u = 2^-53), so by
            Weyl each singular value moves by at most ||F||.
  vectors : after aligning the phase of each pair, ||du_i||, ||dv_i||
            <= 10 tau S_0 / gap_i (Wedin's sin-theta bound), gap_i the
            distance from S_i to the rest of the spectrum; pairs with
            gap_i < 1e3 tau S_0 are not determined that well and are
            checked through the reconstruction only.
  U S V^H : max entry difference from the oracle's <= 10 tau S_0 (unique).
  U, V    : ||U^H U - I||_max, ||V^H V - I||_max <= 1e-12.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
rid = pytest.importorskip("paper_1205_3830_amd")

TAU = 1e-12


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hd = rid.rid_create(0)
    yield hd
    rid.rid_destroy(hd)


def dev(A, dtype=np.complex128):
    A = np.asarray(A, dtype=dtype)
    return torch.from_numpy(np.ascontiguousarray(A.T)).to("cuda").t()


def host(t):
    return t.detach().cpu().numpy()


def _compare(A_ref, J, P, U, S, V):
    Ur, Sr, Vr = oracle.svd_from_id(A_ref, J, P)
    k = Sr.shape[0]
    s0 = max(Sr[0], 1e-300)
    assert S.shape == (k,)
    assert np.all(np.diff(S) <= 0.0) and S[-1] >= 0.0
    assert np.abs(S - Sr).max() <= TAU * s0
    assert np.abs(U.conj().T @ U - np.eye(k)).max() <= 1e-12
    assert np.abs(V.conj().T @ V - np.eye(k)).max() <= 1e-12
    rec = (U * S) @ V.conj().T
    ref = (Ur * Sr) @ Vr.conj().T
    assert np.abs(rec - ref).max() <= 10 * TAU * s0
    for i in range(k):
        others = np.delete(Sr, i)
        gap = np.min(np.abs(others - Sr[i])) if k > 1 else s0
        if gap < 1e3 * TAU * s0:
            continue
        ph = np.vdot(Ur[:, i], U[:, i])
        ph = ph / abs(ph)
        bound = 10 * TAU * s0 / gap
        assert np.linalg.norm(U[:, i] - ph * Ur[:, i]) <= bound, i
        assert np.linalg.norm(V[:, i] - ph * Vr[:, i]) <= bound, i


SVD_CASES = [
    # m, n, k, l, spectrum (None: X W + noise, else prescribed)
    (1000, 500, 20, 30, None),          # the 1000 x 500 parity workload
    (333, 257, 17, 27, None),           # ragged m, n; odd k (padded pairing)
    (50, 40, 1, 5, None),               # k = 1: no rotation at all
    (64, 64, 2, 8, None),
    (700, 400, 75, 85, None),           # odd k in (64, 100]: recorded rotations
    (2000, 300, 100, 108, None),        # k and l of the large workload
    (900, 500, 120, 130, None),         # k > 100: Jacobi and Cholesky in global memory
    (600, 400, 256, 266, None),         # largest k
    (800, 300, 30, 40, "1e-10"),        # cond(A(:,J)) ~ 1e10: needs the shifted pass
]


@pytest.mark.parametrize("m,n,k,l,spec", SVD_CASES)
def test_svd_matches_oracle(h, m, n, k, l, spec):
    if spec is None:
        A = synth.lowrank(m, n, k, 1e-8, seed=m + k)
    else:
        A = synth.with_spectrum(m, n, np.logspace(0, np.log10(float(spec)), k), seed=k)
    r = oracle.decompose(A, k, l, seed=4, q=4)
    assert r["status"] == oracle.OK
    J, P = r["J"], r["P"]
    U, S, V, sweeps = rid.rid_svd(h, dev(A), torch.from_numpy(J).cuda(), dev(P))
    assert 1 <= sweeps < 60 or k == 1
    _compare(A, J, P, host(U), host(S), host(V))


def test_svd_complex64_input_is_widened(h):
    m, n, k = 700, 350, 24
    A32 = synth.lowrank(m, n, k, 1e-5, seed=9).astype(np.complex64)
    A = A32.astype(np.complex128)                  # the values the library reads
    r = oracle.decompose(A, k, k + 10, seed=1, q=4)
    J, P = r["J"], r["P"]
    U, S, V, _ = rid.rid_svd(h, dev(A32, np.complex64), torch.from_numpy(J).cuda(), dev(P))
    _compare(A, J, P, host(U), host(S), host(V))


def test_svd_padded_leading_dimensions(h):
    m, n, k = 300, 200, 12
    A = synth.lowrank(m, n, k, 1e-8, seed=3)
    r = oracle.decompose(A, k, k + 8, seed=2, q=4)
    J, P = r["J"], r["P"]
    Ad = torch.zeros((n, m + 5), dtype=torch.complex128, device="cuda")
    Ad[:, :m] = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
    Pd = torch.zeros((n, k + 3), dtype=torch.complex128, device="cuda")
    Pd[:, :k] = torch.from_numpy(np.ascontiguousarray(P.T)).cuda()
    Ub = torch.full((k, m + 7), 7.0 + 0j, dtype=torch.complex128, device="cuda")
    Vb = torch.full((k, n + 2), 7.0 + 0j, dtype=torch.complex128, device="cuda")
    U, S, V, _ = rid.rid_svd(h, Ad[:, :m].t(), torch.from_numpy(J).cuda(), Pd[:, :k].t(),
                             U=Ub[:, :m].t(), V=Vb[:, :n].t())
    _compare(A, J, P, host(U), host(S), host(V))
    # the padding of the outputs is left alone
    assert torch.all(Ub[:, m:] == 7.0) and torch.all(Vb[:, n:] == 7.0)


def test_svd_of_an_exact_rank_k_matrix_is_its_svd(h):
    # exact rank k: A(:,J) P = A up to rounding, so S is the prescribed
    # spectrum and A v_i = s_i u_i for A itself
    m, n, k = 500, 380, 16
    s0 = np.logspace(0, -6, k)
    A = synth.with_spectrum(m, n, s0, seed=31)
    r = oracle.decompose(A, k, k + 6, seed=8, q=4)
    U, S, V, _ = rid.rid_svd(h, dev(A), torch.from_numpy(r["J"]).cuda(), dev(r["P"]))
    U, S, V = host(U), host(S), host(V)
    assert np.abs(S - s0).max() <= 1e-12
    assert np.abs(A @ V - U * S).max() <= 1e-12
    assert np.abs(A.conj().T @ U - V * S).max() <= 1e-12


@pytest.mark.parametrize("kind", ["out_of_range", "zero_column"])
def test_svd_breakdown_of_the_skeleton_qr_is_reported(h, kind):
    # a zero column of A(:,J) (or an index outside [0, n), read as one)
    # gives an exactly zero Cholesky pivot in the second pass of its QR
    m, n, k = 200, 150, 10
    A = synth.lowrank(m, n, k, 1e-8, seed=5)
    r = oracle.decompose(A, k, k + 6, seed=0, q=2)
    J = r["J"].copy()
    if kind == "out_of_range":
        J[-1] = n + 5
    else:
        A[:, J[2]] = 0.0
    with pytest.raises(rid.RidError) as ei:
        rid.rid_svd(h, dev(A), torch.from_numpy(J).cuda(), dev(r["P"]))
    assert ei.value.status == rid.RID_ERR_RANK


def test_svd_repeated_skeleton_index_reveals_the_rank(h):
    # A(:,J) with a repeated column has rank k-1: the shifted CholeskyQR3
    # still returns an orthonormal Q (cond(A(:,J)) = inf is past its 1/u
    # range, so the bound is 1e-11 S_0 here), and the last singular value
    # of A(:,J) P drops to rounding level
    m, n, k = 200, 150, 10
    A = synth.lowrank(m, n, k, 1e-8, seed=5)
    r = oracle.decompose(A, k, k + 6, seed=0, q=2)
    J = r["J"].copy()
    J[3] = J[1]
    U, S, V, _ = rid.rid_svd(h, dev(A), torch.from_numpy(J).cuda(), dev(r["P"]))
    U, S, V = host(U), host(S), host(V)
    Ur, Sr, Vr = oracle.svd_from_id(A, J, r["P"])
    assert S[-1] <= 1e-11 * S[0] and Sr[-1] <= 1e-11 * Sr[0]
    assert np.abs(S - Sr).max() <= 1e-11 * Sr[0]
    assert np.abs(U.conj().T @ U - np.eye(k)).max() <= 1e-12
    assert np.abs(V.conj().T @ V - np.eye(k)).max() <= 1e-12
    assert np.abs((U * S) @ V.conj().T - (Ur * Sr) @ Vr.conj().T).max() <= 1e-11 * Sr[0]


def test_svd_after_gpu_decompose(h):
    # the library's own ID followed by its SVD: S must lie within the ID's
    # error ||A - A(:,J) P||_2 of A's singular values (Weyl)
    m, n, k, l = 1000, 500, 20, 30
    A = synth.lowrank(m, n, k, 1e-8, seed=77)
    Ad = dev(A)
    J, P, sigma, _ = rid.rid_decompose(h, Ad, k, l, seed=3, q=10)
    U, S, V, _ = rid.rid_svd(h, Ad, J, P)
    Jh, Ph = host(J), host(P)
    E = A - A[:, Jh] @ Ph
    normE = np.linalg.norm(E, 2)
    sA = np.linalg.svd(A, compute_uv=False)
    assert np.all(np.abs(host(S) - sA[:k]) <= normE + TAU * sA[0])


def test_svd_invalid_arguments(h):
    A = dev(synth.lowrank(20, 10, 5, 0.0, seed=1))
    J = torch.arange(3, dtype=torch.int64, device="cuda")
    P = dev(np.zeros((3, 10)))
    with pytest.raises(rid.RidError) as ei:   # k > 256
        rid.rid_svd(h, dev(np.ones((300, 300))), torch.arange(257, device="cuda"),
                    dev(np.zeros((257, 300))))
    assert ei.value.status == rid.RID_ERR_UNSUPPORTED
    with pytest.raises(rid.RidError) as ei:   # k > m
        rid.rid_svd(h, dev(np.ones((2, 10))), J, P)
    assert ei.value.status == rid.RID_ERR_INVALID_ARG
    with pytest.raises(rid.RidError) as ei:   # P = 0: A(:,J) P has rank 0 < k
        rid.rid_svd(h, A, J, P)
    assert ei.value.status == rid.RID_ERR_RANK
    P1 = np.zeros((3, 10))
    P1[:, :3] = np.eye(3)                     # a valid call still works afterwards
    U, S, V, _ = rid.rid_svd(h, A, J, dev(P1))
    assert U.shape == (20, 3) and V.shape == (10, 3)
    sref = np.linalg.svd(host(A)[:, :3], compute_uv=False)
    assert np.abs(host(S) - sref).max() <= TAU * sref[0]
