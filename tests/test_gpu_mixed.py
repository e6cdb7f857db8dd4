"""GPU parity of the reduced-precision form: A stored complex64, sketch
products in FP32 or as two- or three-term bfloat16 splits (single-precision
accumulation within a K split in each case), QR, triangular solve and
residual sums in double.  The oracle runs in double on
exactly the same complex64 values (converted to complex128, which is exact).

Stated accuracy of the FP32 and BF16x3 sketches, against the double oracle:
  Y      : ||dY||_F <= 2e-5 ||Y||_F  (u32 sqrt(K) per split, splits summed in double)
  J      : equal at every step whose relative pivot gap exceeds 1e-4
  P      : max|dP| <= 1e-3 max(1, max|P|)   (kappa(R1) times the Y error)
  sigma  : within a factor 2 of the oracle's (the ID error is dominated by
           sigma_{k+1}, set to 1e-3 and 1e-6 of ||A||_2 here)
BF16x2 (two-term split, 16 significant bits per operand): Y within 2^-14,
J equal beyond a gap of 1e-3, P within 1e-2 max(1, max|P|), sigma within 2x.
Everything computed in double on complex64 storage (the residual, and the
sketch with RID_FP64 products) keeps the double-precision bars.
"""
import numpy as np
import pytest

import oracle
import synth
from parity import check_decompose, check_sigma_call_for_call

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
rid = pytest.importorskip("paper_1205_3830_amd")


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hd = rid.rid_create(0)
    yield hd
    rid.rid_destroy(hd)


def dev(A):
    A = np.asarray(A)
    return torch.from_numpy(np.ascontiguousarray(A.T)).to("cuda").t()


def host(t):
    return t.detach().cpu().numpy()


def lowrank64(m, n, k, rho, seed):
    """complex64 A with sigma_{k+1} ~ rho ||A||_2."""
    A = synth.lowrank(m, n, k, 0.0, seed=seed)
    nrm = np.linalg.norm(A, 2)
    c = rho * nrm / (np.sqrt(m) + np.sqrt(n))
    A = synth.lowrank(m, n, k, c, seed=seed)
    return np.asfortranarray(A.astype(np.complex64))


@pytest.mark.parametrize("m,n,l", [(1000, 500, 30), (1037, 131, 30), (600, 97, 108)])
def test_sketch_fp64_products_on_complex64(h, m, n, l):
    A = lowrank64(m, n, 8, 1e-3, seed=m)
    G = oracle.sketch_operator(l, m, seed=1)
    Y = host(rid.rid_sketch_explicit(h, dev(A), torch.from_numpy(G).cuda(), prec=rid.RID_FP64))
    ref = oracle.sketch(A.astype(np.complex128), G)
    assert np.linalg.norm(Y - ref) <= 1e-12 * np.linalg.norm(ref)


# ||dY||_F / ||Y||_F bars: u32 sqrt(K)-level for FP32 and BF16x3; for BF16x2
# each operand keeps 16 significant bits (representation error <= 2^-17
# relative) and the dropped a_l b_l term is below 2^-16 of |a b|, so 2^-14
# leaves a factor 4 over the rounding of random-signed terms
Y_TOL = {"RID_FP32": 2e-5, "RID_BF16X3": 2e-5, "RID_BF16X2": 2.0 ** -14}


@pytest.mark.parametrize("prec", ["RID_FP32", "RID_BF16X3", "RID_BF16X2"])
@pytest.mark.parametrize("dt", [np.complex64, np.complex128])
@pytest.mark.parametrize("m,n,l", [(1000, 500, 30), (4096, 300, 108), (333, 65, 208),
                                   (9, 40, 12), (2053, 129, 113)])
def test_sketch_reduced_precision_products(h, prec, dt, m, n, l):
    A = lowrank64(m, n, 8, 1e-3, seed=n).astype(dt)
    G = oracle.sketch_operator(l, m, seed=2)
    Y = host(rid.rid_sketch_explicit(h, dev(A), torch.from_numpy(G).cuda(),
                                     prec=getattr(rid, prec)))
    ref = oracle.sketch(A.astype(np.complex128), G)
    err = np.linalg.norm(Y - ref) / np.linalg.norm(ref)
    print("%s %s %dx%d l=%d: ||dY||/||Y|| = %.2e" % (prec, np.dtype(dt).name, m, n, l, err))
    assert err <= Y_TOL[prec], err
    assert err > 0.0          # the products really are of reduced precision


def test_bf16x2_error_is_the_two_term_split(h):
    # the two-term split is the coarser form: its error is well above the
    # three-term split's on the same input, and within its own bar
    m, n, l = 4096, 300, 108
    A = lowrank64(m, n, 8, 1e-3, seed=7)
    G = oracle.sketch_operator(l, m, seed=3)
    ref = oracle.sketch(A.astype(np.complex128), G)
    errs = {}
    for prec in ("RID_BF16X2", "RID_BF16X3"):
        Y = host(rid.rid_sketch_explicit(h, dev(A), torch.from_numpy(G).cuda(),
                                         prec=getattr(rid, prec)))
        errs[prec] = np.linalg.norm(Y - ref) / np.linalg.norm(ref)
    assert errs["RID_BF16X2"] >= 8 * errs["RID_BF16X3"], errs
    assert errs["RID_BF16X2"] <= Y_TOL["RID_BF16X2"], errs


# Every row tiling of the FP32 sketch: 1 to 14 tiles of 16 rows of Y, full and
# ragged, then z-slices of 8 tiles beyond 224 rows.
@pytest.mark.parametrize("l", sorted({16 * r - d for r in range(1, 15) for d in (0, 7)} | {225, 401}))
def test_sketch_fp32_every_row_tiling(h, l):
    m, n = 1100, 77
    A = lowrank64(m, n, 6, 1e-3, seed=l)
    G = oracle.sketch_operator(l, m, seed=l + 3)
    Y = host(rid.rid_sketch_explicit(h, dev(A), torch.from_numpy(G).cuda(), prec=rid.RID_FP32))
    ref = oracle.sketch(A.astype(np.complex128), G)
    err = np.linalg.norm(Y - ref) / np.linalg.norm(ref)
    assert 0.0 < err <= 2e-5, err


@pytest.mark.parametrize("m,n,k,l,q", [(1000, 500, 20, 30, 8), (777, 333, 9, 17, 6)])
def test_residual_complex64_call_for_call(h, m, n, k, l, q):
    A = lowrank64(m, n, k, 1e-3, seed=k)
    A128 = A.astype(np.complex128)
    r = oracle.decompose(A128, k, l, seed=3, q=q)
    sigma, hist = rid.rid_residual(h, dev(A), torch.from_numpy(r["J"]).cuda(), dev(r["P"]), q, 3)
    assert abs(float(host(sigma)[0]) - r["sigma"]) <= 1e-10 * r["sigma"]
    assert np.all(np.abs(host(hist) - r["hist"]) <= 1e-10 * r["hist"])


# The residual's accumulation kinds (rid_set_residual), call for call
# against the oracle's binary128 iteration on the same A, J, P, start vector
# and q: compensated sums within 1e-10, plain double and single sums within
# their derived bound (tests/parity.py: plain_sigma_tol).  Both storage
# types; the whole-slab fast path of the ax pass (1600 rows) and a ragged
# slab (1000 rows); rho 1e-3 and 1e-6.  Odd m (so odd lda): complex64
# columns alternate between 16-byte aligned and shifted pairs, with a ragged
# slab (1001), whole slabs and one row (1537), a second ahz chunk of one row
# (2049) and of 553 rows (2601).
@pytest.mark.parametrize("kind", ["RID_RESIDUAL_DOT2", "RID_RESIDUAL_FP64", "RID_RESIDUAL_FP32"])
@pytest.mark.parametrize("dt", [np.complex64, np.complex128])
@pytest.mark.parametrize("m,n,rho", [(1000, 500, 1e-3), (1600, 300, 1e-6), (1001, 301, 1e-3),
                                     (1537, 300, 1e-6), (2049, 200, 1e-3), (2601, 151, 1e-6)])
def test_residual_accumulation_kinds_call_for_call(h, kind, dt, m, n, rho):
    k, l, q = 20, 30, 6
    A = lowrank64(m, n, k, rho, seed=m + 1).astype(dt)
    A128 = A.astype(np.complex128)
    r = oracle.decompose(A128, k, l, seed=3, q=q)
    rid.rid_set_residual(h, getattr(rid, kind))
    try:
        sigma, hist = rid.rid_residual(h, dev(A), torch.from_numpy(r["J"]).cuda(), dev(r["P"]),
                                       q, 3)
    finally:
        rid.rid_set_residual(h, rid.RID_RESIDUAL_AUTO)
    acc = {"RID_RESIDUAL_DOT2": "dot2", "RID_RESIDUAL_FP64": "fp64",
           "RID_RESIDUAL_FP32": "fp32"}[kind]
    s = float(host(sigma)[0])
    check_sigma_call_for_call(A128, r["J"], r["P"], s, 3, q, acc=acc, hist=host(hist))
    print("%s %s %dx%d rho=%g: |dsigma|/sigma = %.2e" % (kind, np.dtype(dt).name, m, n, rho,
                                                          abs(s - r["sigma"]) / r["sigma"]))


def test_residual_follows_the_form_by_default(h):
    # RID_RESIDUAL_AUTO: compensated for RID_FP64, plain double for the
    # reduced-precision forms -- the same values as the explicit kinds
    m, n, k, l, q = 1000, 500, 20, 30, 6
    A = lowrank64(m, n, k, 1e-3, seed=9)
    r = oracle.decompose(A.astype(np.complex128), k, l, seed=3, q=q)
    J, P = torch.from_numpy(r["J"]).cuda(), dev(r["P"])
    out = {}
    for prec in ("RID_FP64", "RID_FP32", "RID_BF16X2"):
        out[prec] = rid.rid_residual(h, dev(A), J, P, q, 3, prec=getattr(rid, prec))[0]
    for kind in ("RID_RESIDUAL_DOT2", "RID_RESIDUAL_FP64"):
        rid.rid_set_residual(h, getattr(rid, kind))
        out[kind] = rid.rid_residual(h, dev(A), J, P, q, 3)[0]
    rid.rid_set_residual(h, rid.RID_RESIDUAL_AUTO)
    assert torch.equal(out["RID_FP64"], out["RID_RESIDUAL_DOT2"])
    assert torch.equal(out["RID_FP32"], out["RID_RESIDUAL_FP64"])
    assert torch.equal(out["RID_BF16X2"], out["RID_RESIDUAL_FP64"])
    with pytest.raises(rid.RidError) as ei:
        rid.rid_set_residual(h, 9)
    assert ei.value.status == rid.RID_ERR_INVALID_ARG


@pytest.mark.parametrize("kind", ["RID_RESIDUAL_DOT2", "RID_RESIDUAL_FP64", "RID_RESIDUAL_FP32"])
@pytest.mark.parametrize("m,n,pad,offset", [(1600, 300, 2, 0), (1600, 300, 1, 0),
                                            (1600, 300, 3, 0), (1601, 300, 0, 1),
                                            (1600, 300, 2, 1), (1024, 300, 1, 0)])
def test_residual_complex64_padded_leading_dimension(h, kind, m, n, pad, offset):
    # three whole 512-row slabs and a ragged one (or two whole slabs, which
    # with an odd lda take the general loop); lda = m + pad, even or odd
    # (odd: every other column starts 8 bytes past a 16-byte boundary); with
    # offset 1 the matrix starts one entry into its buffer, so its base is
    # not 16-byte aligned and no pair loads are taken
    k, l, q = 12, 20, 6
    A = lowrank64(m, n, k, 1e-3, seed=m + pad)
    A128 = A.astype(np.complex128)
    r = oracle.decompose(A128, k, l, seed=3, q=q)
    ld = m + pad
    flat = torch.zeros(offset + ld * n, dtype=torch.complex64, device="cuda")
    buf = flat[offset:].view(n, ld)
    buf[:, :m] = torch.from_numpy(np.ascontiguousarray(A.T)).to("cuda")
    Ad = buf[:, :m].t()                       # m x n, column stride m + pad
    assert Ad.stride() == (1, ld)
    assert (Ad.data_ptr() % 16 == 0) == (offset == 0)
    rid.rid_set_residual(h, getattr(rid, kind))
    try:
        sigma, hist = rid.rid_residual(h, Ad, torch.from_numpy(r["J"]).cuda(), dev(r["P"]), q, 3)
    finally:
        rid.rid_set_residual(h, rid.RID_RESIDUAL_AUTO)
    acc = {"RID_RESIDUAL_DOT2": "dot2", "RID_RESIDUAL_FP64": "fp64",
           "RID_RESIDUAL_FP32": "fp32"}[kind]
    check_sigma_call_for_call(A128, r["J"], r["P"], float(host(sigma)[0]), 3, q, acc=acc,
                              hist=host(hist))


# per form: (pivot-gap tolerance tau_J, P bar relative to max(1, max|P|),
# rank tolerance above the form's rounding floor)
FORM_BARS = {"RID_FP32": (1e-4, 1e-3, 1e-5), "RID_BF16X3": (1e-4, 1e-3, 1e-5),
             "RID_BF16X2": (1e-3, 1e-2, 1e-4)}


@pytest.mark.parametrize("rho", [1e-3, 1e-6])
@pytest.mark.parametrize("prec", ["RID_FP32", "RID_BF16X3", "RID_BF16X2"])
@pytest.mark.parametrize("m,n,k,l", [(1000, 500, 20, 30), (2048, 700, 64, 72)])
def test_decompose_complex64_reduced_precision(h, prec, m, n, k, l, rho):
    # sigma_{k+1} ~ rho ||A||_2 for both levels of the precision workload;
    # J and P are checked at every step and entry on the GPU's own pivots
    tau, ptol, rank_tol = FORM_BARS[prec]
    A = lowrank64(m, n, k, rho, seed=m + k)
    A128 = A.astype(np.complex128)
    ref = oracle.decompose(A128, k, l, seed=0, q=8)
    J, P, sigma, used = rid.rid_decompose(h, dev(A), k, l, seed=0, q=8,
                                          prec=getattr(rid, prec), rank_tol=rank_tol)
    J, P, s = host(J), host(P), float(host(sigma)[0])
    assert used == ref["seed_used"]
    r = check_decompose(A128, ref["Y"], J, P, s, 0, 8, tau=tau, ptol=ptol, ref=ref,
                        sigma_factor=2.0)
    print("%s rho=%g %dx%d: near-ties %d, max|dP| %.2e, sigma/ref %.4f" % (
        prec, rho, m, n, r["near_ties"], np.abs(P - r["P"]).max(), s / r["sigma_ref"]))


def test_decompose_complex64_fp64_matches_double_oracle(h):
    m, n, k, l = 1000, 500, 20, 30
    A = lowrank64(m, n, k, 1e-3, seed=5)
    ref = oracle.decompose(A.astype(np.complex128), k, l, seed=0, q=8)
    J, P, sigma, used = rid.rid_decompose(h, dev(A), k, l, seed=0, q=8, prec=rid.RID_FP64)
    J, P, s = host(J), host(P), float(host(sigma)[0])
    check_decompose(A.astype(np.complex128), ref["Y"], J, P, s, 0, 8, ref=ref)


# uneven jobs over several row-tile buckets (l = 14 .. 200: 1 .. 13 row tiles
# of Y), ragged 128-column blocks and ragged K splits (m not a multiple of
# the 1024-row split or of 16)
BF16_BATCH = [(1500, 300, 20, 28), (700, 130, 6, 14), (2100, 257, 40, 48), (300, 129, 60, 72),
              (1030, 520, 100, 108), (900, 300, 190, 200)]


@pytest.mark.parametrize("dt", [np.complex64, np.complex128])
@pytest.mark.parametrize("prec", ["RID_BF16X2", "RID_BF16X3"])
def test_bf16_batches_match_the_oracle(h, prec, dt):
    # each job's J at every step, P entry by entry on the GPU's pivots and
    # sigma, to the form's bars; and each job bitwise as when batched alone
    # (a job's plan depends on the job only)
    tau, ptol, rank_tol = FORM_BARS[prec]
    p = getattr(rid, prec)
    As = [lowrank64(m, n, k, 1e-3, seed=11 + i).astype(dt) for i, (m, n, k, l) in
          enumerate(BF16_BATCH)]
    Ad = [dev(A) for A in As]
    ks, ls = [s[2] for s in BF16_BATCH], [s[3] for s in BF16_BATCH]
    seeds = [3 + i for i in range(len(BF16_BATCH))]
    Js, Ps, sig, status, used = rid.rid_decompose_batched(h, Ad, ks, ls, seeds, q=6, prec=p,
                                                          rank_tol=rank_tol)
    assert status == [0] * len(BF16_BATCH)
    for i, (m, n, k, l) in enumerate(BF16_BATCH):
        A128 = As[i].astype(np.complex128)
        ref = oracle.decompose(A128, k, l, seed=seeds[i], q=6)
        assert used[i] == ref["seed_used"]
        Jb, Pb, sb = host(Js[i]), host(Ps[i]), float(host(sig[i])[0])
        check_decompose(A128, ref["Y"], Jb, Pb, sb, used[i], 6, tau=tau, ptol=ptol, ref=ref,
                        sigma_factor=2.0)
    for i in (1, 5):
        J1, P1, s1, _, _ = rid.rid_decompose_batched(h, [Ad[i]], [ks[i]], [ls[i]], [seeds[i]],
                                                     q=6, prec=p, rank_tol=rank_tol)
        assert torch.equal(J1[0], Js[i]) and torch.equal(P1[0], Ps[i])
        assert torch.equal(s1[0], sig[i])


def test_precision_codes_follow_the_abi():
    assert (rid.RID_FP64, rid.RID_FP32, rid.RID_BF16X2, rid.RID_BF16X3) == (0, 1, 2, 3)
