"""GPU parity: every step of the HIP path against the CPU oracle, through the
C ABI, on seeded synthetic inputs (arXiv 1205.3830, Sec. 3.3 recipe: products
of complex Gaussian factors plus a small Gaussian noise).

Tolerances (double precision):
  G      : <= 1e-14 relative per entry (log/sin/cos of two math libraries).
  Y      : ||dY||_F <= 1e-12 ||Y||_F (summation order; ~u sqrt(m) expected).
  J      : bit-exact wherever the pivot gap exceeds 1e-10.
  P      : max|dP| <= 1e-10 max(1, max|P|)  (1e-12 with identical R).
  sigma  : call-for-call (same A, J, P, seed, q): |d sigma| <= 1e-10 sigma,
           possible because both sides accumulate the cancelling sums in
           better than double; end to end (each side its own P):
           |d sigma| <= 1e-10 sigma + 2 ||A(:,J)||_F ||dP||_F, since
           | ||E1|| - ||E2|| | <= ||A(:,J)(P1 - P2)||.
"""
import numpy as np
import pytest

import oracle
import synth
from parity import check_decompose, check_P, check_pivots

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
rid = pytest.importorskip("paper_1205_3830_amd")

TAU_J = 1e-10


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hd = rid.rid_create(0)
    yield hd
    rid.rid_destroy(hd)


def dev(A):
    """host complex array (m, n) -> column-major device tensor."""
    A = np.asarray(A)
    return torch.from_numpy(np.ascontiguousarray(A.T)).to("cuda").t()


def host(t):
    return t.detach().cpu().numpy()


def _lowrank(m, n, k, noise, seed):
    return synth.lowrank(m, n, k, noise, seed=seed)


# ------------------------------------------------------------------ a1: G
@pytest.mark.parametrize("rows,cols,seed,sid", [(7, 1000, 0, 0), (1, 513, 5, 1),
                                                (108, 300, 2**40 + 3, 0)])
def test_gaussian_matches_oracle(h, rows, cols, seed, sid):
    g = host(rid.rid_gaussian(h, rows, cols, seed, sid))
    ref = oracle.gaussian(rows, cols, seed, sid)
    assert np.max(np.abs(g - ref) / np.maximum(np.abs(ref), 1e-300)) <= 1e-14


# ------------------------------------------------------------------ a2: Y = G A
SKETCH_CASES = [
    (1000, 500, 30),   # 1000 x 500 parity workload, l = k + 10
    (1037, 131, 30),   # ragged m, n
    (257, 70, 108),    # l of the large workload (7 row tiles of Y)
    (64, 64, 1),
    (5, 3, 2),
    (1, 1, 1),
    (600, 97, 208),    # l of the square workload (13 row tiles)
    (300, 65, 250),    # 16 row tiles: split along the rows of Y (two z-slices)
    (4096, 40, 16),    # several K splits
]


def _check_Y(Y, ref, tol=1e-12):
    """||dY||_F <= tol ||Y||_F, and column by column ||dY(:,j)|| <= tol ||Y(:,j)||
    (the summation order of each column's l sums differs between the two)."""
    assert np.linalg.norm(Y - ref) <= tol * np.linalg.norm(ref)
    dcol = np.linalg.norm(Y - ref, axis=0)
    assert np.all(dcol <= tol * np.linalg.norm(ref, axis=0) + 1e-300), dcol.max()


@pytest.mark.parametrize("m,n,l", SKETCH_CASES)
def test_sketch_explicit_matches_oracle(h, m, n, l):
    A = _lowrank(m, n, min(8, m, n), 1e-6, seed=m + n)
    G = oracle.sketch_operator(l, m, seed=1)
    Y = host(rid.rid_sketch_explicit(h, dev(A), torch.from_numpy(G).cuda()))
    ref = oracle.sketch(A, G)
    _check_Y(Y, ref)


# Every row tiling of the FP64 sketch (1 to 14 tiles of 16 rows of Y, each
# full and ragged, then z-slices of 8 tiles beyond 224 rows), with complex128
# and complex64 storage; the grid spans two column blocks with a ragged tail
# and several K splits with a ragged last step.
SKETCH_TILING_LS = sorted({16 * r - d for r in range(1, 15) for d in (0, 7)} | {225, 300, 401})


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
@pytest.mark.parametrize("l", SKETCH_TILING_LS)
def test_sketch_every_row_tiling_matches_oracle(h, l, dt):
    m, n = 1100, 77
    A = _lowrank(m, n, 6, 1e-6, seed=l).astype(dt)
    G = oracle.sketch_operator(l, m, seed=l + 1)
    Y = host(rid.rid_sketch_explicit(h, dev(A), torch.from_numpy(G).cuda()))
    ref = oracle.sketch(A.astype(np.complex128), G)
    _check_Y(Y, ref)


@pytest.mark.parametrize("m,n,l,seed", [(1000, 500, 30, 0), (333, 77, 20, 9)])
def test_sketch_seeded_matches_oracle(h, m, n, l, seed):
    A = _lowrank(m, n, 10, 1e-8, seed=3)
    Y = host(rid.rid_sketch(h, dev(A), l, seed))
    ref = oracle.sketch(A, oracle.sketch_operator(l, m, seed))
    assert np.linalg.norm(Y - ref) <= 1e-12 * np.linalg.norm(ref)


def test_sketch_leading_dimensions(h):
    m, n, l = 300, 40, 12
    A = _lowrank(m, n, 5, 1e-6, seed=4)
    big = torch.zeros((n, m + 13), dtype=torch.complex128, device="cuda")
    big[:, :m] = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
    Ad = big.t()[:m]                      # lda = m + 13
    Yb = torch.full((n, l + 5), 7.0, dtype=torch.complex128, device="cuda")
    Yd = Yb.t()[:l]                        # ldy = l + 5
    G = oracle.sketch_operator(l, m, seed=2)
    rid.rid_sketch_explicit(h, Ad, torch.from_numpy(G).cuda(), Y=Yd)
    ref = oracle.sketch(A, G)
    Yh = host(Yb).T
    assert np.linalg.norm(Yh[:l] - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.all(Yh[l:] == 7.0)           # padding rows untouched


# ------------------------------------------------------------------ a3: pivoted QR
PIVQR_CASES = [(30, 500, 20), (108, 2000, 100), (12, 12, 12), (40, 9, 9), (8, 300, 1),
               (200, 700, 150), (65, 100, 64),
               # large l (16 and 32 rows per lane) and k > 256 (R1^-1 then one GEMM)
               (600, 700, 300), (2000, 400, 100), (1024, 1100, 1000),
               # the panel form through 28, 24 and 20 rows per lane
               (1700, 700, 600)]


# both forms of the Householder steps: "plain" rewrites the trailing rows every
# step; "panel" keeps up to 4 reflectors pending and writes every 4th step
# (chosen by size for a Y beyond the last-level cache, forced here).  The
# panel form's workgroups each take every G-th column block; "panel3" caps
# them at 3, so that each takes several blocks (as at the sweep's sizes).
QR_FORMS = ["plain", "panel", "panel3"]


@pytest.fixture
def qr_form(request, monkeypatch):
    monkeypatch.setenv("RID_QR_PANEL", "0" if request.param == "plain" else "1")
    if request.param == "panel3":
        monkeypatch.setenv("RID_QR_PANEL_GROUPS", "3")
    return request.param


@pytest.mark.parametrize("qr_form", QR_FORMS, indirect=True)
@pytest.mark.parametrize("l,n,k", PIVQR_CASES)
def test_pivqr_and_interp_match_oracle(h, qr_form, l, n, k):
    A = _lowrank(max(l, 400), n, k, 1e-9, seed=l * 7 + n)
    Y = oracle.sketch(A, oracle.sketch_operator(l, A.shape[0], seed=1))
    Yd = dev(Y)
    perm, gaps = rid.rid_pivqr(h, Yd, k)
    assert rid.rid_query_status(h) == rid.RID_OK
    perm = host(perm)
    J = perm[:k]
    r = check_pivots(Y, J, TAU_J)
    rest = np.setdiff1d(np.arange(n), J)
    assert np.array_equal(perm[k:], rest)
    assert np.allclose(host(gaps), r["gaps"], rtol=1e-6, atol=1e-12)
    R = host(Yd)[:k]
    # |diag R1| is the step's trailing norm: independent of the reflector convention
    assert np.allclose(np.abs(R[np.arange(k), J]), np.abs(r["R"][np.arange(k), J]),
                       rtol=1e-11)
    # R1 upper triangular in pivot order
    R1 = R[:, J]
    assert np.all(np.tril(R1, -1) == 0)
    P = host(rid.rid_interp(h, Yd[:k], torch.from_numpy(J).cuda()))
    assert np.array_equal(P[:, J], np.eye(k))
    check_P(P, r["P"], 1e-10)


def near_tie_sketch(l, n, pairs, seed):
    """A sketch with columns in pairs y_b = e^{i theta} y_a.  The two trailing
    norms of a pair agree up to rounding at every step, so the step that
    reaches a pair has a pivot gap at rounding level and two implementations
    may take either column (the other then drops to a rounding-level norm).
    The pairs are scaled so that they are reached at steps 0, 1, 2, ..."""
    rng = np.random.default_rng(seed)
    Y = (rng.standard_normal((l, n)) + 1j * rng.standard_normal((l, n))) / np.sqrt(2)
    for i, (a, b) in enumerate(pairs):
        Y[:, a] *= 4.0 - 0.4 * i
        Y[:, b] = Y[:, a] * np.exp(1j * rng.uniform(0, 2 * np.pi))
    return np.asfortranarray(Y)


NEAR_TIE_PAIRS = [(3, 40), (11, 10), (90, 25), (7, 150), (60, 61)]


@pytest.mark.parametrize("kind", ["householder", "panel", "panel3", "cgs2"])
def test_pivqr_near_ties_are_valid_picks(h, monkeypatch, kind):
    # every pair meets a near-tie; the oracle is forced onto the GPU's picks,
    # the picks are checked for validity there and for equality elsewhere,
    # and P is compared entry by entry on the GPU's pivots
    l, n, k = 30, 200, 20
    Y = near_tie_sketch(l, n, NEAR_TIE_PAIRS, seed=12)
    monkeypatch.setenv("RID_QR_PANEL", "1" if kind.startswith("panel") else "0")
    if kind == "panel3":
        monkeypatch.setenv("RID_QR_PANEL_GROUPS", "3")
    rid.rid_set_qr(h, rid.RID_QR_CGS2 if kind == "cgs2" else rid.RID_QR_HOUSEHOLDER)
    try:
        Yd = dev(Y)
        perm, gaps = rid.rid_pivqr(h, Yd, k)
        assert rid.rid_query_status(h) == rid.RID_OK
        J = host(perm)[:k]
        P = host(rid.rid_interp(h, Yd[:k], torch.from_numpy(J).cuda()))
    finally:
        rid.rid_set_qr(h, rid.RID_QR_HOUSEHOLDER)
    r = check_pivots(Y, J, TAU_J)
    assert r["near_ties"] >= len(NEAR_TIE_PAIRS)
    assert set(J[:len(NEAR_TIE_PAIRS)].tolist()) <= {c for p in NEAR_TIE_PAIRS for c in p}
    assert np.array_equal(P[:, J], np.eye(k))
    check_P(P, r["P"], 1e-10)


@pytest.mark.parametrize("qr_form", QR_FORMS, indirect=True)
def test_pivqr_rows_per_lane_shrink_over_the_steps(h, qr_form):
    # each step launches with the fewest rows per lane that cover the rows in
    # play: here 1600 -> 951 rows, so RR 32, 24 and 16 in turn (the panel form
    # changes RR only where it writes back)
    l, n, k = 1600, 1500, 650
    Y = synth.lowrank(l, n, k, 1e-9, seed=3100)
    Yd = dev(Y)
    perm, gaps = rid.rid_pivqr(h, Yd, k)
    assert rid.rid_query_status(h) == rid.RID_OK
    J = host(perm)[:k]
    r = check_pivots(Y, J, TAU_J)
    R = host(Yd)[:k]
    assert np.allclose(np.abs(R[np.arange(k), J]), np.abs(r["R"][np.arange(k), J]),
                       rtol=1e-11)
    assert np.all(np.tril(R[:, J], -1) == 0)
    P = host(rid.rid_interp(h, Yd[:k], torch.from_numpy(J).cuda()))
    assert np.array_equal(P[:, J], np.eye(k))
    check_P(P, r["P"], 1e-10)


@pytest.mark.parametrize("qr_form", QR_FORMS, indirect=True)
@pytest.mark.parametrize("l,n,k", [(64, 1 << 18, 48), (800, 1 << 17, 40)])
def test_pivqr_with_more_workgroups_than_fit_at_once(h, qr_form, l, n, k):
    # 4096 (2048) column workgroups per step launch: many start after others
    # finished, so a step must not overwrite what the same launch still reads
    Y = synth.lowrank(l, n, k, 1e-9, seed=n + l)
    Yd = dev(Y)
    perm, gaps = rid.rid_pivqr(h, Yd, k)
    assert rid.rid_query_status(h) == rid.RID_OK
    J = host(perm)[:k]
    r = check_pivots(Y, J, TAU_J)
    P = host(rid.rid_interp(h, Yd[:k], torch.from_numpy(J).cuda()))
    check_P(P, r["P"], 1e-10)


@pytest.mark.parametrize("m,n,k,l,q", [(1000, 500, 20, 30, 10), (2500, 900, 300, 600, 3)])
def test_decompose_with_panel_qr_matches_oracle(h, monkeypatch, m, n, k, l, q):
    monkeypatch.setenv("RID_QR_PANEL", "1")
    A = _lowrank(m, n, k, 1e-10, seed=1)
    r = oracle.decompose(A, k, l, seed=0, q=q)
    J, P, sigma, used = rid.rid_decompose(h, dev(A), k, l, seed=0, q=q)
    J, P, s = host(J), host(P), float(host(sigma)[0])
    check_decompose(A, r["Y"], J, P, s, 0, q, ref=r)


@pytest.mark.parametrize("l,n,k,tol", [(30, 500, 20, 1e-12), (108, 1000, 100, 1e-12),
                                       (250, 300, 250, 1e-12), (400, 900, 300, 1e-11)])
def test_interp_same_R_matches_oracle(h, l, n, k, tol):
    A = _lowrank(max(l, 300), n, k, 1e-8, seed=n)
    Y = oracle.sketch(A, oracle.sketch_operator(l, A.shape[0], seed=4))
    st, Jo, Ro, _ = oracle.select(Y, k)
    Po = oracle.interp(Ro, Jo)
    P = host(rid.rid_interp(h, dev(Ro), torch.from_numpy(Jo).cuda()))
    assert np.array_equal(P[:, Jo], np.eye(k))
    assert np.abs(P - Po).max() <= tol * max(1.0, np.abs(Po).max())


def test_pivqr_rank_failure_sets_status(h):
    A = _lowrank(200, 80, 5, 0.0, seed=11)          # rank 5 < k = 6
    Y = oracle.sketch(A, oracle.sketch_operator(10, 200, seed=0))
    rid.rid_pivqr(h, dev(Y), 6)
    assert rid.rid_query_status(h) == rid.RID_ERR_RANK
    rid.rid_pivqr(h, dev(Y), 5)
    assert rid.rid_query_status(h) == rid.RID_OK


def test_pivqr_exact_tie_goes_to_lowest_index(h):
    Y = synth.hand_example()
    perm, gaps = rid.rid_pivqr(h, dev(Y), 2)
    assert list(host(perm)) == [0, 1, 2]
    assert host(gaps)[1] == 0.0


# ------------------------------------------------------------------ a5: residual
# (700, 800, 300): u_J staged in two chunks of the w step, five row chunks
# of P in the P x sets; (300, 17000, 12): more columns than the P x step has
# sets (1024 sets of 17 columns, the last one short)
@pytest.mark.parametrize("m,n,k,l,noise,q", [(1000, 500, 20, 30, 1e-10, 10),
                                             (777, 333, 9, 17, 1e-7, 6),
                                             (300, 1100, 40, 48, 1e-9, 4),
                                             (64, 50, 50, 50, 0.0, 3),
                                             (700, 800, 300, 310, 1e-9, 3),
                                             (300, 17000, 12, 20, 1e-9, 3)])
def test_residual_call_for_call(h, m, n, k, l, noise, q):
    A = _lowrank(m, n, k, noise, seed=m)
    r = oracle.decompose(A, k, l, seed=3, q=q)
    assert r["status"] == oracle.OK
    sigma, hist = rid.rid_residual(h, dev(A), torch.from_numpy(r["J"]).cuda(),
                                   dev(r["P"]), q, 3)
    s, hi = float(host(sigma)[0]), host(hist)
    if r["sigma"] == 0.0 or noise == 0.0:
        # k = n: E = 0 up to rounding of P's identity columns
        assert s <= 1e-12 * np.linalg.norm(A, 2)
    else:
        assert abs(s - r["sigma"]) <= 1e-10 * r["sigma"]
        assert np.all(np.abs(hi - r["hist"]) <= 1e-10 * r["hist"])


def test_residual_zero_matrix_stops_early(h):
    A = np.zeros((20, 6), dtype=np.complex128)
    J = torch.tensor([0, 1], dtype=torch.int64, device="cuda")
    P = dev(np.eye(2, 6, dtype=np.complex128))
    sigma, hist = rid.rid_residual(h, dev(A), J, P, 4, 0)
    assert float(host(sigma)[0]) == 0.0 and np.all(host(hist) == 0.0)


# ------------------------------------------------------------------ end to end
DECOMP_CASES = [
    (1000, 500, 20, 30, 1e-10, 10),   # the 1000 x 500 parity workload, seed 0
    (1000, 500, 20, 30, 0.0, 10),     # exactly rank k
    (513, 257, 1, 1, 1e-10, 5),       # k = 1, l = k
    (300, 40, 40, 40, 1e-10, 4),      # k = n: no T at all
    (2048, 700, 100, 108, 1e-12, 6),  # l, k of the large workload
    (2500, 900, 300, 600, 1e-10, 3),  # l = 2k with k > 256 (the paper's l)
]


@pytest.mark.parametrize("m,n,k,l,noise,q", DECOMP_CASES)
def test_decompose_matches_oracle(h, m, n, k, l, noise, q):
    A = _lowrank(m, n, k, noise, seed=0)
    r = oracle.decompose(A, k, l, seed=0, q=q)
    assert r["status"] == oracle.OK
    J, P, sigma, used = rid.rid_decompose(h, dev(A), k, l, seed=0, q=q)
    J, P, s = host(J), host(P), float(host(sigma)[0])
    assert used == r["seed_used"]
    check_decompose(A, r["Y"], J, P, s, 0, q, ref=r)
    assert np.abs(P).max() <= 2.0


def test_decompose_rank_deficient_fails_every_draw(h):
    A = _lowrank(120, 60, 3, 0.0, seed=2)
    with pytest.raises(rid.RidError) as ei:
        rid.rid_decompose(h, dev(A), 4, 8, seed=0, q=2, max_retries=2)
    assert ei.value.status == rid.RID_ERR_RANK


def test_decompose_redraws_after_a_rank_deficient_first_operator(h):
    # Sec. 2: when rank(Y) < k the randomization is drawn again.  The first
    # operator G0 = B C has rank k - 1, so G0 A has rank k - 1 and the QR
    # stops at step k - 1; the redraw with seed + 1 succeeds and gives the
    # oracle's ID of that seed.
    m, n, k, l = 600, 300, 12, 20
    A = _lowrank(m, n, k, 1e-10, seed=31)
    rng = np.random.default_rng(5)
    B = rng.standard_normal((l, k - 1)) + 1j * rng.standard_normal((l, k - 1))
    C = rng.standard_normal((k - 1, m)) + 1j * rng.standard_normal((k - 1, m))
    G0 = np.ascontiguousarray(B @ C)
    r0 = oracle.decompose(A, k, l, seed=5, q=6, G=G0)
    assert r0["status"] == oracle.ERR_RANK                   # the oracle agrees G0 fails
    G0d = torch.from_numpy(G0).cuda()
    J, P, sigma, used = rid.rid_decompose_explicit(h, dev(A), G0d, k, seed=5, q=6)
    assert used == 6
    r = oracle.decompose(A, k, l, seed=6, q=6, max_retries=0)
    assert r["status"] == oracle.OK
    check_decompose(A, r["Y"], host(J), host(P), float(host(sigma)[0]), 6, 6, ref=r)
    with pytest.raises(rid.RidError) as ei:                   # no redraw allowed
        rid.rid_decompose_explicit(h, dev(A), G0d, k, seed=5, q=6, max_retries=0)
    assert ei.value.status == rid.RID_ERR_RANK
    # a full-rank explicit first operator is used as given
    G1 = oracle.sketch_operator(l, m, seed=77)
    J, P, sigma, used = rid.rid_decompose_explicit(h, dev(A), torch.from_numpy(G1).cuda(), k,
                                                   seed=5, q=6)
    assert used == 5
    r1 = oracle.decompose(A, k, l, seed=5, q=6, G=G1)
    check_decompose(A, r1["Y"], host(J), host(P), float(host(sigma)[0]), 5, 6, ref=r1)


def test_misaligned_pointers_and_short_leading_dimensions_rejected(h):
    # through the raw C entry points: argument errors come back before any
    # launch, so nothing is read through the bad pointers
    import ctypes
    lib = rid.load()
    Pv = ctypes.c_void_p
    m, n, k, l = 50, 20, 3, 5
    A = dev(_lowrank(m, n, k, 1e-10, seed=1))
    J = torch.zeros(k, dtype=torch.int64, device="cuda")
    P = torch.zeros((n, k), dtype=torch.complex128, device="cuda").t()
    Y = torch.zeros((n, l), dtype=torch.complex128, device="cuda").t()
    sig = torch.zeros(1, dtype=torch.float64, device="cuda")
    a, p = A.data_ptr(), P.data_ptr()
    C128, C64, F64 = rid.RID_C128, rid.RID_C64, rid.RID_FP64
    INV = rid.RID_ERR_INVALID_ARG

    def dec(Ap, lda, Pp, ldp, dt=C128):
        return lib.rid_decompose(h, None, dt, F64, m, n, k, l, Pv(Ap), lda, 0, 4, 1, 1e-12,
                                 Pv(J.data_ptr()), Pv(Pp), ldp, Pv(sig.data_ptr()), None)

    assert dec(a + 8, m, p, k) == INV           # complex128 A must be 16-byte aligned
    assert dec(a + 4, m, p, k, C64) == INV      # complex64 A 8-byte aligned
    assert dec(a, m - 1, p, k) == INV           # lda < m
    assert dec(a, m, p + 8, k) == INV           # P 16-byte aligned
    assert dec(a, m, p, k - 1) == INV           # ldp < k
    assert lib.rid_sketch(h, None, C128, F64, m, n, l, Pv(a + 8), m, 0, Pv(Y.data_ptr()),
                          l) == INV
    assert lib.rid_sketch(h, None, C128, F64, m, n, l, Pv(a), m - 1, 0, Pv(Y.data_ptr()),
                          l) == INV
    assert lib.rid_sketch(h, None, C128, F64, m, n, l, Pv(a), m, 0, Pv(Y.data_ptr() + 8),
                          l) == INV
    assert lib.rid_sketch(h, None, C128, F64, m, n, l, Pv(a), m, 0, Pv(Y.data_ptr()),
                          l - 1) == INV
    assert lib.rid_pivqr(h, None, l, n, k, Pv(Y.data_ptr() + 8), l, Pv(J.data_ptr()), None,
                         1e-12) == INV
    assert lib.rid_pivqr(h, None, l, n, k, Pv(Y.data_ptr()), l - 1, Pv(J.data_ptr()), None,
                         1e-12) == INV
    assert lib.rid_interp(h, None, n, k, Pv(Y.data_ptr()), k - 1, Pv(J.data_ptr()), Pv(p),
                          k) == INV
    assert lib.rid_interp(h, None, n, k, Pv(Y.data_ptr()), l, Pv(J.data_ptr()), Pv(p + 8),
                          k) == INV
    assert lib.rid_residual(h, None, C128, F64, m, n, k, Pv(a + 8), m, Pv(J.data_ptr()),
                            Pv(p), k, 4, 0, Pv(sig.data_ptr()), None) == INV
    assert lib.rid_residual(h, None, C128, F64, m, n, k, Pv(a), m - 1, Pv(J.data_ptr()),
                            Pv(p), k, 4, 0, Pv(sig.data_ptr()), None) == INV
    # the handle still works afterwards
    J2, P2, s2, _ = rid.rid_decompose(h, A, k, l, seed=0, q=4)
    assert rid.rid_query_status(h) == rid.RID_OK


def test_decompose_is_deterministic_and_scale_equivariant(h):
    A = _lowrank(700, 300, 15, 1e-9, seed=7)
    J1, P1, s1, _ = rid.rid_decompose(h, dev(A), 15, 25, seed=1, q=5)
    J2, P2, s2, _ = rid.rid_decompose(h, dev(A), 15, 25, seed=1, q=5)
    J3, P3, s3, _ = rid.rid_decompose(h, dev(2 * A), 15, 25, seed=1, q=5)
    assert torch.equal(J1, J2) and torch.equal(P1, P2) and torch.equal(s1, s2)
    assert torch.equal(J1, J3) and torch.equal(P1, P3)
    assert float(s3[0]) == 2 * float(s1[0])


def test_invalid_arguments_rejected(h):
    A = dev(_lowrank(50, 20, 3, 0.0, seed=1))
    with pytest.raises(rid.RidError) as ei:
        rid.rid_decompose(h, A, 5, 4, seed=0)          # l < k
    assert ei.value.status == rid.RID_ERR_INVALID_ARG
    with pytest.raises(rid.RidError) as ei:
        rid.rid_decompose(h, A, 3, 60, seed=0)         # l > m
    assert ei.value.status == rid.RID_ERR_INVALID_ARG
    with pytest.raises(rid.RidError) as ei:
        rid.rid_decompose(h, A, 3, 5, seed=0, q=0)     # q < 1
    assert ei.value.status == rid.RID_ERR_INVALID_ARG
    with pytest.raises(rid.RidError) as ei:
        rid.rid_decompose(h, A, 3, 5, seed=0, prec=7)  # no such product arithmetic
    assert ei.value.status == rid.RID_ERR_INVALID_ARG


# ------------------------------------------------------------------ S F D operator
@pytest.mark.parametrize("rows,m,seed", [(10, 64, 3), (108, 5000, 7), (1, 1, 0)])
def test_srft_operator_matches_oracle(h, rows, m, seed):
    g = host(rid.rid_srft_operator(h, rows, m, seed))
    ref = oracle.srft_operator(rows, m, seed)
    assert np.abs(g - ref).max() <= 1e-13


def test_decompose_with_srft_matches_oracle(h):
    m, n, k, l = 1000, 500, 20, 40
    A = _lowrank(m, n, k, 1e-10, seed=0)
    r = oracle.decompose(A, k, l, seed=0, q=8, kind="srft")
    rid.rid_set_sketch(h, rid.RID_SKETCH_SRFT)
    try:
        J, P, sigma, used = rid.rid_decompose(h, dev(A), k, l, seed=0, q=8)
        Y = host(rid.rid_sketch(h, dev(A), l, 0))
    finally:
        rid.rid_set_sketch(h, rid.RID_SKETCH_GAUSSIAN)
    assert np.linalg.norm(Y - r["Y"]) <= 1e-12 * np.linalg.norm(r["Y"])
    J, P, s = host(J), host(P), float(host(sigma)[0])
    check_decompose(A, r["Y"], J, P, s, 0, 8, ref=r)


SRFT_SKETCH_CASES = [
    # m, n, l, seed, storage; m % 8 == 0 takes the four-step DFT, else the explicit operator
    (4096, 300, 108, 7, np.complex128),
    (1048, 129, 30, 2, np.complex128),    # ragged n, m2 = 131
    (8, 3, 5, 1, np.complex128),          # m2 = 1
    (2000, 100, 30, 4, np.complex64),     # complex64 storage, FP64 products
    (1600, 64, 250, 5, np.complex128),    # large l: about 31 rows per residue group
    (512, 40, 1, 6, np.complex128),       # one row, one group
    (1001, 50, 20, 3, np.complex128),     # m not a multiple of 8: explicit operator
]


@pytest.mark.parametrize("m,n,l,seed,dt", SRFT_SKETCH_CASES)
def test_srft_sketch_matches_oracle(h, m, n, l, seed, dt):
    A = _lowrank(m, n, min(8, n), 1e-6, seed=m + n).astype(dt)
    ref = oracle.sketch(A.astype(np.complex128), oracle.srft_operator(l, m, seed))
    rid.rid_set_sketch(h, rid.RID_SKETCH_SRFT)
    try:
        Y = host(rid.rid_sketch(h, dev(A), l, seed))
    finally:
        rid.rid_set_sketch(h, rid.RID_SKETCH_GAUSSIAN)
    assert np.linalg.norm(Y - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("form", ["fused", "two_pass"])
@pytest.mark.parametrize("m,n,l,seed", [(4096, 300, 108, 7), (2048, 70, 30, 11),
                                         (1024, 65, 400, 12)])
def test_srft_sketch_forms_match_oracle(h, monkeypatch, form, m, n, l, seed):
    # The one-pass (fused) and two-pass four-step forms on the same input.
    # With l = 400 the residue groups exceed 32 rows, so both runs take the
    # two-pass form.
    if form == "two_pass":
        monkeypatch.setenv("RID_SRFT_TWO_PASS", "1")
    else:
        monkeypatch.delenv("RID_SRFT_TWO_PASS", raising=False)
    A = _lowrank(m, n, 8, 1e-6, seed=m + l)
    ref = oracle.sketch(A, oracle.srft_operator(l, m, seed))
    rid.rid_set_sketch(h, rid.RID_SKETCH_SRFT)
    try:
        Y = host(rid.rid_sketch(h, dev(A), l, seed))
    finally:
        rid.rid_set_sketch(h, rid.RID_SKETCH_GAUSSIAN)
    assert np.linalg.norm(Y - ref) <= 1e-12 * np.linalg.norm(ref)


def test_srft_sketch_column_blocks_match_numpy_fft(h):
    # 2^21 rows: the four-step form's Z buffer (2 GiB) holds 64 columns, so
    # 150 columns take three blocks.  Sampled columns against numpy's FFT of
    # D A(:, j), sampled at the rows s_i (eqs. (4)-(7)).
    m, n, l, seed = 1 << 21, 150, 40, 9
    Ad = synth.lowrank_device(m, n, 6, 1e-6, seed=3).t()
    rid.rid_set_sketch(h, rid.RID_SKETCH_SRFT)
    try:
        Y = host(rid.rid_sketch(h, Ad, l, seed))
    finally:
        rid.rid_set_sketch(h, rid.RID_SKETCH_GAUSSIAN)
    s = oracle.srft_rows(l, m, seed)
    d = np.exp(2j * np.pi * oracle.srft_phases(m, seed))
    for j in [0, 63, 64, 127, 128, 149]:
        col = Ad[:, j].cpu().numpy()
        ref = np.fft.fft(d * col)[s]
        assert np.linalg.norm(Y[:, j] - ref) <= 1e-12 * np.linalg.norm(ref), j


# ------------------------------------------------------------------ QR method: CGS2 (Sec. 3.2)
@pytest.fixture
def h_cgs2(h):
    rid.rid_set_qr(h, rid.RID_QR_CGS2)
    yield h
    rid.rid_set_qr(h, rid.RID_QR_HOUSEHOLDER)


# k > 65 takes the second pass spread over the device (one direction chunk
# at k = 100, two at k = 200, three at k = 300)
@pytest.mark.parametrize("l,n,k", [(30, 500, 20), (108, 2000, 100), (12, 12, 12), (8, 300, 1),
                                   (600, 700, 300), (64, 1 << 17, 30), (250, 3000, 200)])
def test_cgs2_pivqr_and_interp_match_oracle(h_cgs2, l, n, k):
    h = h_cgs2
    Y = synth.lowrank(l, n, k, 1e-9, seed=3 * l + n)
    Yd = dev(Y)
    perm, gaps = rid.rid_pivqr(h, Yd, k)
    assert rid.rid_query_status(h) == rid.RID_OK
    perm = host(perm)
    J = perm[:k]
    r = check_pivots(Y, J, TAU_J)
    assert np.array_equal(perm[k:], np.setdiff1d(np.arange(n), J))
    R = host(Yd)[:k]
    R1 = R[:, J]
    assert np.all(np.tril(R1, -1) == 0)
    # CGS2 gives a real positive diagonal: the exact trailing norms
    assert np.allclose(R1.diagonal().real, np.abs(r["R"][np.arange(k), J]), rtol=1e-11)
    assert np.all(R1.diagonal().imag == 0)
    P = host(rid.rid_interp(h, Yd[:k], torch.from_numpy(J).cuda()))
    check_P(P, r["P"], 1e-10)


def test_cgs2_and_householder_agree(h):
    Y = synth.lowrank(108, 3000, 100, 1e-10, seed=5)
    out = {}
    for kind in (rid.RID_QR_HOUSEHOLDER, rid.RID_QR_CGS2):
        rid.rid_set_qr(h, kind)
        Yd = dev(Y)
        perm, _ = rid.rid_pivqr(h, Yd, 100)
        P = rid.rid_interp(h, Yd[:100], perm[:100].clone())
        out[kind] = (host(perm), host(P))
    rid.rid_set_qr(h, rid.RID_QR_HOUSEHOLDER)
    (ph, Ph), (pc, Pc) = out[rid.RID_QR_HOUSEHOLDER], out[rid.RID_QR_CGS2]
    assert np.array_equal(ph, pc)
    assert np.abs(Ph - Pc).max() <= 1e-10 * max(1.0, np.abs(Ph).max())
    with pytest.raises(rid.RidError) as ei:
        rid.rid_set_qr(h, 7)
    assert ei.value.status == rid.RID_ERR_INVALID_ARG


@pytest.mark.parametrize("m,n,k,l,noise,q", [(1000, 500, 20, 30, 1e-10, 10),
                                             (2500, 900, 300, 600, 1e-10, 3)])
def test_cgs2_decompose_matches_oracle(h_cgs2, m, n, k, l, noise, q):
    h = h_cgs2
    A = _lowrank(m, n, k, noise, seed=0)
    r = oracle.decompose(A, k, l, seed=0, q=q)
    J, P, sigma, used = rid.rid_decompose(h, dev(A), k, l, seed=0, q=q)
    J, P, s = host(J), host(P), float(host(sigma)[0])
    check_decompose(A, r["Y"], J, P, s, 0, q, ref=r)
