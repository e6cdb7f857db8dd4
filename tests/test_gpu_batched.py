"""GPU tests of the batched form: many IDs of uneven sizes in one call.

Each job of a batch must give the result of the single-job path with the
same inputs (and of the oracle): J exact beyond the pivot-gap tolerance,
P within 1e-10 (FP64 products; the batch sums the sketch over different
K splits, so Y differs in the last bits), sigma within the end-to-end bound.
A rank-deficient job fails alone; the graph-captured and directly launched
batches give bitwise the same results; repeated calls are bitwise equal.
"""
import os

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
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A).T)).to("cuda").t()


def host(t):
    return t.detach().cpu().numpy()


def make_jobs(count, seed, dtype=np.complex128, noise=1e-9, mmax=1500, nmax=700):
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(count):
        m = int(np.exp(rng.uniform(np.log(100), np.log(mmax))))
        n = int(np.exp(rng.uniform(np.log(40), np.log(nmax))))
        k = int(rng.integers(4, min(40, n, m - 8) + 1))
        l = k + 8
        A = synth.lowrank(m, n, k, noise, seed=1000 + i).astype(dtype)
        jobs.append((A, k, l, 17 + i))
    return jobs


def test_batch_matches_single_and_oracle_fp64(h):
    jobs = make_jobs(12, 1)
    As = [dev(A) for A, _, _, _ in jobs]
    Js, Ps, sig, status, used = rid.rid_decompose_batched(
        h, As, [j[1] for j in jobs], [j[2] for j in jobs], [j[3] for j in jobs], q=6)
    assert status == [0] * len(jobs)
    for i, (A, k, l, s) in enumerate(jobs):
        J1, P1, s1, u1 = rid.rid_decompose(h, As[i], k, l, seed=s, q=6)
        assert used[i] == u1
        Jb, Pb, sb = host(Js[i]), host(Ps[i]), float(host(sig[i])[0])
        r = oracle.decompose(A, k, l, seed=s, q=6)
        check_decompose(A, r["Y"], Jb, Pb, sb, s, 6, ref=r)
        if np.array_equal(Jb, host(J1)):
            assert np.abs(Pb - host(P1)).max() <= 1e-10 * max(1.0, np.abs(host(P1)).max())
        else:       # a near-tie broken the other way: the single path is checked alone
            check_decompose(A, r["Y"], host(J1), host(P1), float(host(s1)[0]), s, 6, ref=r)


def test_batch_complex64_fp32(h):
    jobs = make_jobs(10, 2, dtype=np.complex64, noise=1e-2)
    As = [dev(A) for A, _, _, _ in jobs]
    Js, Ps, sig, status, _ = rid.rid_decompose_batched(
        h, As, [j[1] for j in jobs], [j[2] for j in jobs], [j[3] for j in jobs], q=6,
        prec=rid.RID_FP32, rank_tol=1e-5)
    assert status == [0] * len(jobs)
    for i, (A, k, l, s) in enumerate(jobs):
        A128 = A.astype(np.complex128)
        r = oracle.decompose(A128, k, l, seed=s, q=6)
        Jb, Pb, sb = host(Js[i]), host(Ps[i]), float(host(sig[i])[0])
        # J at every step, P entry by entry (on the batch's pivots), sigma
        # within a factor 2: the reduced-precision bars
        check_decompose(A128, r["Y"], Jb, Pb, sb, s, 6, tau=1e-4, ptol=1e-3, ref=r,
                        sigma_factor=2.0)


def test_batch_rank_failure_is_per_job(h):
    jobs = make_jobs(5, 3)
    bad = synth.lowrank(300, 120, 3, 0.0, seed=9)       # rank 3 < k = 6
    jobs.insert(2, (bad, 6, 10, 5))
    As = [dev(A) for A, _, _, _ in jobs]
    Js, Ps, sig, status, used = rid.rid_decompose_batched(
        h, As, [j[1] for j in jobs], [j[2] for j in jobs], [j[3] for j in jobs], q=3,
        max_retries=1, raise_on_rank=False)
    assert status[2] == rid.RID_ERR_RANK and used[2] == 6
    assert all(st == 0 for i, st in enumerate(status) if i != 2)
    with pytest.raises(rid.RidError) as ei:
        rid.rid_decompose_batched(h, As, [j[1] for j in jobs], [j[2] for j in jobs],
                                  [j[3] for j in jobs], q=3, max_retries=0)
    assert ei.value.status == rid.RID_ERR_RANK


def test_batch_graph_and_direct_launch_agree_bitwise(h, monkeypatch):
    jobs = make_jobs(7, 4)
    As = [dev(A) for A, _, _, _ in jobs]
    args = ([j[1] for j in jobs], [j[2] for j in jobs], [j[3] for j in jobs])
    a = rid.rid_decompose_batched(h, As, *args, q=4)
    b = rid.rid_decompose_batched(h, As, *args, q=4)
    monkeypatch.setenv("RID_BATCH_GRAPH", "0")
    c = rid.rid_decompose_batched(h, As, *args, q=4)
    for i in range(len(jobs)):
        for res in (b, c):
            assert torch.equal(a[0][i], res[0][i])
            assert torch.equal(a[1][i], res[1][i])
            assert torch.equal(a[2][i], res[2][i])


def test_batch_qr_one_launch_equals_per_step_launches(h, monkeypatch):
    # the QR of a batch as one launch per pivot step over all jobs (default)
    # and as one launch with a workgroup per job (RID_BATCH_QR=jobs): the
    # same arithmetic, so J, P and sigma agree bit for bit; jobs of 1 to 4
    # rows per lane, n from below one column block to several, and a
    # rank-deficient job
    jobs = make_jobs(9, 8, mmax=2500, nmax=1500)
    bad = synth.lowrank(300, 130, 3, 0.0, seed=19)       # rank 3 < k = 6
    jobs.insert(4, (bad, 6, 10, 5))
    jobs.append((synth.lowrank(600, 40, 30, 1e-9, seed=21), 30, 200, 3))   # l = 200: 4 rows/lane
    As = [dev(A) for A, _, _, _ in jobs]
    args = ([j[1] for j in jobs], [j[2] for j in jobs], [j[3] for j in jobs])
    a = rid.rid_decompose_batched(h, As, *args, q=4, max_retries=0, raise_on_rank=False)
    monkeypatch.setenv("RID_BATCH_QR", "jobs")
    b = rid.rid_decompose_batched(h, As, *args, q=4, max_retries=0, raise_on_rank=False)
    assert a[3] == b[3] and a[3][4] == rid.RID_ERR_RANK
    assert sum(st == 0 for st in a[3]) == len(jobs) - 1
    for i in range(len(jobs)):
        if a[3][i] != 0:
            continue
        assert torch.equal(a[0][i], b[0][i]), i
        assert torch.equal(a[1][i], b[1][i]), i
        assert torch.equal(a[2][i], b[2][i]), i
    # and against the oracle on the batch's pivots
    for i in (0, len(jobs) - 1):
        A, k, l, s = jobs[i]
        r = oracle.decompose(A, k, l, seed=s, q=4)
        check_decompose(A, r["Y"], host(a[0][i]), host(a[1][i]), float(host(a[2][i])[0]), s, 4,
                        ref=r)


def test_batch_invalid_job_rejected(h):
    A = dev(synth.lowrank(50, 20, 3, 0.0, seed=1))
    with pytest.raises(rid.RidError) as ei:
        rid.rid_decompose_batched(h, [A], [5], [4], [0])       # l < k
    assert ei.value.status == rid.RID_ERR_INVALID_ARG
    with pytest.raises(rid.RidError) as ei:
        rid.rid_decompose_batched(h, [A], [3], [300], [0])     # l > m, and > 224
    assert ei.value.status == rid.RID_ERR_INVALID_ARG


def test_autotuner_picks_candidates_and_keeps_parity(h):
    jobs = make_jobs(10, 6)
    As = [dev(A) for A, _, _, _ in jobs]
    ks, ls, seeds = [j[1] for j in jobs], [j[2] for j in jobs], [j[3] for j in jobs]
    keep = rid.rid_get_batch_plan(h)
    try:
        rows, blk, cols = rid.rid_tune_batched(h, As, ks, ls, seeds, q=4)
        assert rows in (128, 256, 512, 1024, 2048, 4096)
        assert blk in tuple(x << 10 for x in (32, 64, 128, 256, 512, 1024))
        assert cols in (4, 8)
        assert rid.rid_get_batch_plan(h) == (rows, blk, cols)
        # every plan gives results within the FP64 tolerances of the oracle
        for plan in ((rows, blk, cols), (128, 32 << 10, 4), (4096, 1 << 20, 8)):
            rid.rid_set_batch_plan(h, *plan)
            Js, Ps, sig, status, _ = rid.rid_decompose_batched(h, As, ks, ls, seeds, q=4)
            assert status == [0] * len(jobs)
            for i, (A, k, l, s) in enumerate(jobs):
                r = oracle.decompose(A, k, l, seed=s, q=4)
                check_decompose(A, r["Y"], host(Js[i]), host(Ps[i]), float(host(sig[i])[0]),
                                s, 4, ref=r)
        with pytest.raises(rid.RidError):
            rid.rid_set_batch_plan(h, 100, 1 << 20)        # not a multiple of 16
        with pytest.raises(rid.RidError):
            rid.rid_set_batch_plan(h, 1024, 100)           # below 4 KiB
        with pytest.raises(rid.RidError):
            rid.rid_set_batch_plan(h, 1024, 1 << 18, 6)    # 4 or 8 columns per wave
    finally:
        rid.rid_set_batch_plan(h, *keep)


# The batched workload itself: 512 jobs drawn as the benchmark draws them
# (m log-uniform in [256, 4096], n in [128, 2048], k in [8, 64], l = k + 8,
# A = X W + 1e-7 N stored complex64), run as one batch; a seeded sample of
# 16 jobs is checked against the oracle on the same stored values.  With
# FP32 sketch products J and P keep their reduced-precision bars, but at this
# noise level (ID error about 1e-6 of ||A||) the FP32-level change of P moves
# ||A - A(:,J) P|| by more than the error itself, so sigma is held to the
# end-to-end bound in ||dP|| and, call for call, to the oracle's iteration
# on the batch's own J and P (plain double sums over A with FP32 products:
# within u sqrt(m + n) ||A||_F (1 + ||P||) times 10).
@pytest.mark.parametrize("prec", ["RID_FP64", "RID_FP32", "RID_BF16X2"])
def test_batch_of_the_512_job_workload_sampled_against_oracle(h, prec):
    import bench
    shapes = bench.batch_shapes(512)
    As = [synth.lowrank_device(m, n, k, 1e-7, seed=i, dtype=torch.complex64).t()
          for i, (m, n, k, l) in enumerate(shapes)]
    ks, ls = [s[2] for s in shapes], [s[3] for s in shapes]
    seeds = list(range(len(shapes)))
    q = 4
    p = getattr(rid, prec)
    tol = {rid.RID_FP64: 1e-12, rid.RID_FP32: 1e-5, rid.RID_BF16X2: 1e-4}[p]
    Js, Ps, sig, status, used = rid.rid_decompose_batched(h, As, ks, ls, seeds, q=q, prec=p,
                                                          rank_tol=tol)
    assert status == [0] * len(shapes)
    rng = np.random.default_rng(2024)
    sample = sorted(rng.choice(len(shapes), 16, replace=False).tolist())
    sample[-1] = int(np.argmax([m * n for m, n, _, _ in shapes]))   # and the largest job
    for i in sample:
        m, n, k, l = shapes[i]
        A = As[i].t().contiguous().cpu().numpy().T.astype(np.complex128)
        r = oracle.decompose(A, k, l, seed=used[i], q=q, max_retries=0)
        assert r["status"] == oracle.OK
        Jb, Pb, sb = host(Js[i]), host(Ps[i]), float(host(sig[i])[0])
        if p == rid.RID_FP64:
            check_decompose(A, r["Y"], Jb, Pb, sb, used[i], q, ref=r)
            # compensated sums over A (odd and even m: both complex64 loops)
            check_sigma_call_for_call(A, Jb, Pb, sb, used[i], q, acc="dot2")
        else:
            # the reduced-precision bars (BF16x2: its 2^-16 split error)
            tau, ptol = (1e-4, 1e-3) if p == rid.RID_FP32 else (1e-3, 1e-2)
            c = check_decompose(A, r["Y"], Jb, Pb, sb, used[i], q, tau=tau, ptol=ptol, ref=r)
            # reduced-precision products: the residual's sums over A are plain double
            check_sigma_call_for_call(A, Jb, Pb, sb, used[i], q, acc="fp64")
            print("job %d %dx%d k=%d: sigma %s / FP64 oracle = %.2f" % (
                i, m, n, k, prec, sb / c["sigma_ref"]))
