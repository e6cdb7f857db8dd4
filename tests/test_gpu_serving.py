"""GPU tests of the served form (rid_server_*): continuous batching with
admission by device footprint.

* Each result in the mix equals, bitwise, the result of the entry point
  that ran it called alone on the same inputs (rid_decompose, or
  rid_decompose_batched with that one job: a batched job's results do not
  depend on the rest of its batch), and both entry points meet the FP64 bars
  against the oracle (J exact beyond the pivot-gap tolerance and valid at
  near-ties, P within 1e-10, sigma within the end-to-end bound).
* Two big jobs whose footprints do not fit the budget together run one
  after the other; the peak admitted footprint stays within the budget.
* Small jobs submitted after a big job are admitted and finish while the
  big job is still running (their work overlaps on the device).
* A failing fill callback fails only its own job; a request larger than the
  budget is refused at submission.
* The lanes' workspaces stay counted while held: a request that fits the
  budget only if an idle lane gives its workspace up waits for that, and
  then runs.
"""
import threading

import numpy as np
import pytest

import oracle
import synth
from parity import check_decompose

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


def host(t):
    return t.detach().cpu().numpy()


class Inputs:
    """Deterministic device inputs by (shape, seed); kept for the alone runs."""

    def __init__(self):
        self.lock = threading.Lock()
        self.A = {}

    def fill(self, ticket, req):
        dt = torch.complex128 if req["dtype"] == rid.RID_C128 else torch.complex64
        A = synth.lowrank_device(req["m"], req["n"], req["rank"], req["noise"],
                                 seed=req["gen_seed"], dtype=dt).t()
        with self.lock:
            self.A[ticket] = A
        return A


def shapes(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        m = int(np.exp(rng.uniform(np.log(256), np.log(1500))))
        n = int(np.exp(rng.uniform(np.log(128), np.log(700))))
        k = int(rng.integers(8, min(40, n, m - 8) + 1))
        out.append((m, n, k, k + 8))
    return out


def test_results_alone_equal_results_in_the_mix(h):
    inp = Inputs()
    srv = rid.RidServer(inp.fill, big_bytes=8 << 20, big_lanes=2, batch_lanes=2, max_batch=8)
    jobs = [(m, n, k, l, rid.RID_C64) for m, n, k, l in shapes(14, 5)]
    jobs += [(2048, 1100, 24, 32, rid.RID_C64), (1800, 700, 16, 24, rid.RID_C128)]
    tickets = []
    try:
        for i, (m, n, k, l, dt) in enumerate(jobs):
            tickets.append(srv.submit(m, n, k, l, dtype=dt, prec=rid.RID_FP64, seed=40 + i, q=6,
                                      rank=k, noise=1e-7, gen_seed=100 + i))
        srv.drain()
        st = srv.stats()
        assert st["completed"] == len(jobs)
        for i, t in enumerate(tickets):
            res = srv.result(t)
            m, n, k, l, dt = jobs[i]
            assert res["status"] == 0, (i, res)
            A = inp.A[t]
            J1, P1, s1, u1 = rid.rid_decompose(h, A, k, l, seed=40 + i, q=6)
            Jb, Pb, sb, stb, ub = rid.rid_decompose_batched(h, [A], [k], [l], [40 + i], q=6)
            assert stb == [0] and ub[0] == u1 == res["seed_used"]
            same_single = (torch.equal(res["J"], J1) and torch.equal(res["P"], P1)
                           and torch.equal(res["sigma"], s1))
            same_batch = (torch.equal(res["J"], Jb[0]) and torch.equal(res["P"], Pb[0])
                          and torch.equal(res["sigma"], sb[0]))
            assert same_single or same_batch, i
            # both entry points meet the FP64 bars against the oracle (each on
            # its own pivots, so a near-tie broken either way is checked too)
            Ah = A.t().contiguous().cpu().numpy().T.astype(np.complex128)
            r = oracle.decompose(Ah, k, l, seed=u1, q=6, max_retries=0)
            assert r["status"] == oracle.OK
            check_decompose(Ah, r["Y"], host(J1), host(P1), float(host(s1)[0]), u1, 6, ref=r)
            check_decompose(Ah, r["Y"], host(Jb[0]), host(Pb[0]), float(host(sb[0])[0]), u1, 6,
                            ref=r)
    finally:
        srv.close()


def test_admission_keeps_big_jobs_within_the_budget(h):
    inp = Inputs()
    m, n, k, l = 32768, 4096, 16, 24
    abytes = m * n * 16
    fill = 2 * abytes
    budget = int(1.6 * (abytes + fill))          # one big job fits, two do not
    srv = rid.RidServer(inp.fill, hbm_budget=budget, big_bytes=1 << 20, big_lanes=2,
                        batch_lanes=1, max_batch=16)
    try:
        t1 = srv.submit(m, n, k, l, dtype=rid.RID_C128, seed=1, q=3, fill_bytes=fill, rank=k,
                        noise=1e-10, gen_seed=7)
        t2 = srv.submit(m, n, k, l, dtype=rid.RID_C128, seed=2, q=3, fill_bytes=fill, rank=k,
                        noise=1e-10, gen_seed=8)
        small = [srv.submit(300, 200, 8, 16, dtype=rid.RID_C128, seed=10 + i, q=3, rank=8,
                            noise=1e-10, gen_seed=20 + i) for i in range(6)]
        srv.drain()
        r1, r2 = srv.result(t1), srv.result(t2)
        assert r1["status"] == 0 and r2["status"] == 0
        first, second = sorted([r1, r2], key=lambda r: r["times"][1])
        assert second["times"][1] >= first["times"][3]     # admitted after the first is done
        for t in small:
            assert srv.result(t)["status"] == 0
        assert 0 < srv.stats()["peak_bytes"] <= budget
    finally:
        srv.close()


def test_small_jobs_overlap_a_running_big_job(h):
    inp = Inputs()
    srv = rid.RidServer(inp.fill, big_bytes=64 << 20, big_lanes=1, batch_lanes=1, max_batch=64)
    try:
        tb = srv.submit(65536, 4096, 32, 40, dtype=rid.RID_C128, seed=3, q=10, rank=32,
                        noise=1e-10, gen_seed=11)
        ts = [srv.submit(400, 200, 8, 16, dtype=rid.RID_C64, seed=50 + i, q=4, rank=8,
                         noise=1e-7, gen_seed=60 + i) for i in range(24)]
        srv.drain()
        big = srv.result(tb)
        assert big["status"] == 0
        done_before = [t for t in ts if srv.result(t)["times"][3] < big["times"][3]]
        admitted_after = [t for t in done_before
                          if srv.result(t)["times"][1] >= big["times"][1]]
        assert admitted_after, "no small job ran while the big job was on the device"
        assert all(srv.result(t)["status"] == 0 for t in ts)
    finally:
        srv.close()


def test_failures_are_per_request(h):
    def fill(ticket, req):
        if req.get("boom"):
            raise RuntimeError("fill failed on purpose")
        return synth.lowrank_device(req["m"], req["n"], 4, 1e-9, seed=ticket).t()

    srv = rid.RidServer(fill, hbm_budget=1 << 30, big_lanes=0, batch_lanes=1, max_batch=8)
    try:
        ok = [srv.submit(200, 100, 4, 8, seed=i, q=3) for i in range(3)]
        bad = srv.submit(200, 100, 4, 8, seed=9, q=3, boom=True)
        with pytest.raises(rid.RidError) as ei:
            srv.submit(1 << 17, 1 << 14, 10, 20, seed=0, q=3)      # 32 GiB > budget
        assert ei.value.status == rid.RID_ERR_NOMEM
        with pytest.raises(rid.RidError) as ei:
            srv.submit(200, 100, 9, 8, seed=0, q=3)                # k > l
        assert ei.value.status == rid.RID_ERR_INVALID_ARG
        srv.drain()
        assert srv.result(bad)["status"] == rid.RID_ERR_INVALID_ARG
        assert "on purpose" in srv.result(bad)["error"]
        assert all(srv.result(t)["status"] == 0 for t in ok)
    finally:
        srv.close()


def _footprint(m, n, k, l, dtype, q):
    """The smallest budget that accepts the request at submission (its data
    and its workspace alone), by bisection on the submit-time refusal."""
    def refuse(ticket, req):
        raise RuntimeError("probe only")

    def accepted(budget):
        srv = rid.RidServer(refuse, hbm_budget=budget, big_lanes=0, batch_lanes=1, max_batch=1)
        try:
            srv.submit(m, n, k, l, dtype=dtype, seed=0, q=q)
            return True
        except rid.RidError as e:
            assert e.status == rid.RID_ERR_NOMEM
            return False
        finally:
            srv.close()

    es = 16 if dtype == rid.RID_C128 else 8
    lo, hi = m * n * es + k * n * 16, m * n * es + (1 << 34)   # refused, accepted
    assert not accepted(lo) and accepted(hi)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if accepted(mid):
            hi = mid
        else:
            lo = mid
    return hi


def test_admission_counts_held_workspaces(h):
    # Job 2 fits the budget only with every lane's workspace let go: after
    # job 1, its lane holds job 1's workspace (more than 1 MiB), so job 2
    # waits until that idle lane frees it, then runs.
    inp = Inputs()
    j1 = (16384, 4096, 16, 24)
    j2 = (32768, 4096, 16, 24)
    f2 = _footprint(*j2, rid.RID_C128, 3)
    budget = f2 + (1 << 20)
    srv = rid.RidServer(inp.fill, hbm_budget=budget, big_bytes=1 << 20, big_lanes=2,
                        batch_lanes=1, max_batch=8)
    try:
        t1 = srv.submit(*j1, dtype=rid.RID_C128, seed=1, q=3, rank=16, noise=1e-10, gen_seed=31)
        t2 = srv.submit(*j2, dtype=rid.RID_C128, seed=2, q=3, rank=16, noise=1e-10, gen_seed=32)
        srv.drain()
        r1, r2 = srv.result(t1), srv.result(t2)
        assert r1["status"] == 0 and r2["status"] == 0
        assert r2["times"][1] >= r1["times"][3]            # admitted after job 1 was done
        assert 0 < srv.stats()["peak_bytes"] <= budget
    finally:
        srv.close()
