"""rid_pivqr_static, the entry point that allocates nothing (its scratch is
the library's static device array), against rid_pivqr on the same inputs:
two calls in a row, the second smaller; J, the gaps and R bit for bit, and
the oracle's bars (J exact beyond the pivot-gap tolerance, P within 1e-10
on the GPU's pivots).  Problems beyond the array are refused before any
launch."""
import ctypes

import numpy as np
import pytest

import synth
from parity import check_P, check_pivots

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
rid = pytest.importorskip("paper_1205_3830_amd")


def dev(A):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A).T)).to("cuda").t()


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hd = rid.rid_create(0)
    yield hd
    rid.rid_destroy(hd)


@pytest.mark.parametrize("kind", ["householder", "cgs2"])
def test_pivqr_static_equals_pivqr_on_two_calls(h, kind):
    rid.rid_set_qr(h, rid.RID_QR_CGS2 if kind == "cgs2" else rid.RID_QR_HOUSEHOLDER)
    try:
        # the second call is smaller: what the first left in the array must
        # not leak into it
        for l, n, k, seed in [(208, 9000, 200, 1), (30, 500, 20, 2)]:
            Y = synth.lowrank(l, n, k, 1e-9, seed=seed)
            Y1, Y2 = dev(Y), dev(Y)
            p1, g1 = rid.rid_pivqr(h, Y1, k)
            p2, g2 = rid.rid_pivqr_static(h, Y2, k)
            torch.cuda.synchronize()
            assert rid.rid_query_status(h) == rid.RID_OK
            assert torch.equal(p1, p2) and torch.equal(g1, g2)
            assert torch.equal(Y1[:k], Y2[:k])
            J = p2[:k].cpu().numpy()
            r = check_pivots(Y, J, 1e-10)
            P = rid.rid_interp(h, Y2[:k], p2[:k].clone()).cpu().numpy()
            assert np.array_equal(P[:, J], np.eye(k))
            check_P(P, r["P"], 1e-10)
    finally:
        rid.rid_set_qr(h, rid.RID_QR_HOUSEHOLDER)


def test_pivqr_static_rank_failure_sets_status(h):
    A = synth.lowrank(200, 80, 5, 0.0, seed=11)
    G = np.random.default_rng(0).standard_normal((10, 200))
    Y = G @ A                                       # rank 5
    rid.rid_pivqr_static(h, dev(Y), 6)
    assert rid.rid_query_status(h) == rid.RID_ERR_RANK
    rid.rid_pivqr_static(h, dev(Y), 5)
    assert rid.rid_query_status(h) == rid.RID_OK


def test_pivqr_static_refuses_problems_beyond_its_array(h):
    # the size check comes before any launch, so a small buffer stands in
    # for the 2000 x 40000 Y it is told about
    lib = rid.load()
    buf = torch.zeros(64, dtype=torch.complex128, device="cuda")
    perm = torch.zeros(64, dtype=torch.int64, device="cuda")
    P = ctypes.c_void_p
    st = lib.rid_pivqr_static(h, None, 2000, 40000, 100, P(buf.data_ptr()), 2000,
                              P(perm.data_ptr()), None, 1e-12)
    assert st == rid.RID_ERR_NOMEM
    st = lib.rid_pivqr_static(h, None, 10, 20, 11, P(buf.data_ptr()), 10, P(perm.data_ptr()),
                              None, 1e-12)
    assert st == rid.RID_ERR_INVALID_ARG               # k > l
