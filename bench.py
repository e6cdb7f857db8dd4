#!/usr/bin/env python3
"""Benchmark of the randomized interpolative decomposition on one MI355X.

A step is one whole ID through the C ABI (rid_decompose): Gaussian sketch
Y = G A, pivoted QR of Y, P = [I T], and the power-iteration estimate of
||A - A(:,J) P||_2 with q = 10 steps -- 1 + (2q - 1) = 2q passes over A.
Workload: A = X W + 1e-12 N, complex128, m = 131072, n = 16384, k = 100,
l = 108 (34.4 GB), X, W, N i.i.d. complex Gaussian, generated on the GPU
before the timed region (synthetic stand-in for the Gaussian low-rank test
matrices of arXiv 1205.3830, Sec. 3.3).

Prints one JSON line: value = GB/s of A streamed (2q passes of A's bytes per
ID), plus IDs/s, the roofline of the dominant kernel (event-timed inside the
timed region), and the CPU oracle timed on a bounded column sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP64_PEAK_TFS = 78.6         # MI355X FP64 matrix (dense)
FP32_PEAK_TFS = 157.3        # MI355X FP32 matrix (dense)
BF16_PEAK_TFS = 2500.0       # MI355X BF16 matrix (dense)

# sketch product arithmetic by command-line name
PRECS = {"fp64": lambda rid: rid.RID_FP64, "fp32": lambda rid: rid.RID_FP32,
         "bf16x2": lambda rid: rid.RID_BF16X2, "bf16x3": lambda rid: rid.RID_BF16X3}
# rank tolerance of the QR per sketch arithmetic: above each form's rounding
# floor (|R_kk| / |R_11| of the workloads is about 1e-2)
RANK_TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x2": 1e-4, "bf16x3": 1e-5}
DTYPE_TEXT = {"fp64": "f64", "fp32": "f32 sketch products, f64 QR/solve/residual",
              "bf16x2": "bf16x2-split sketch products (f32 accumulate), f64 QR/solve/residual",
              "bf16x3": "bf16x3-split sketch products (f32 accumulate), f64 QR/solve/residual"}


def _traffic(kernel_name: str, src_file: str, measured_config: bool = True):
    """HBM bytes per launch from a committed counter summary, if it was
    taken on the current kernel source (matching sha256) and on this
    configuration; else None."""
    if not measured_config:
        return None
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % kernel_name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    with open(os.path.join(ROOT, "paper_1205_3830_amd", "csrc", src_file), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if rec.get("source_sha256") != sha:
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(A_dev, k, l, q, cols):
    """The oracle, untuned, on columns [0, cols) of the same A."""
    import numpy as np

    import oracle
    m = A_dev.shape[0]
    Ah = A_dev[:, :cols].t().contiguous().cpu().numpy().T   # (m, cols), Fortran order
    Ah = np.asfortranarray(Ah)
    t0 = time.perf_counter()
    r = oracle.decompose(Ah, k, l, seed=0, q=q)
    dt = time.perf_counter() - t0
    gbs = 2 * q * 16.0 * m * cols / dt / 1e9
    return {"value": gbs, "unit": "GB/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "oracle.decompose on columns 0..%d of the same A (%d x %d complex128, "
                      "%.0f MB), k=%d, l=%d, q=%d; %.1f s; status %d"
                      % (cols - 1, m, cols, 16.0 * m * cols / 1e6, k, l, q, dt, r["status"]),
            "seconds": dt}


def batch_shapes(count: int, seed: int = 0):
    """m, n log-uniform in [256, 4096] and [128, 2048], k uniform in [8, 64],
    l = k + 8 (the batched workload)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        m = int(round(np.exp(rng.uniform(np.log(256), np.log(4096)))))
        n = int(round(np.exp(rng.uniform(np.log(128), np.log(2048)))))
        k = int(rng.integers(8, 65))
        k = min(k, n, m - 8)
        out.append((m, n, k, k + 8))
    return out


def bench_batched(args, torch, rid, synth) -> int:
    print(json.dumps(batched_result(args, torch, rid, synth)))
    return 0


def batched_result(args, torch, rid, synth) -> dict:
    q = args.q
    shapes = batch_shapes(args.jobs)
    dt = torch.complex64 if args.dtype == "c64" else torch.complex128
    esize = 8 if args.dtype == "c64" else 16
    prec = PRECS[args.prec](rid)
    tol = RANK_TOL[args.prec]
    print("generating %d matrices" % len(shapes), file=sys.stderr, flush=True)
    As = [synth.lowrank_device(m, n, k, 1e-7, seed=i, dtype=dt).t()
          for i, (m, n, k, l) in enumerate(shapes)]
    torch.cuda.synchronize()
    ks = [s[2] for s in shapes]
    ls = [s[3] for s in shapes]
    seeds = list(range(len(shapes)))
    bytes_a = float(sum(esize * m * n for m, n, _, _ in shapes))
    h = rid.rid_create(0)

    def batch(p):
        return rid.rid_decompose_batched(h, As, ks, ls, seeds, q=q, prec=p, rank_tol=tol)

    def timed():
        batch(prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            Js, Ps, sig, status, _ = batch(prec)
        torch.cuda.synchronize()
        assert all(s == 0 for s in status)
        return (time.perf_counter() - t0) / args.steps

    plan_default = rid.rid_get_batch_plan(h)
    t_default = timed()
    plan = plan_default
    t_batch = t_default
    if not args.no_tune:
        print("autotuning the batch plan", file=sys.stderr, flush=True)
        plan = rid.rid_tune_batched(h, As, ks, ls, seeds, q=q, prec=prec)
        t_batch = timed()
    # one more batch with the library's event timing (launched directly): the
    # grouped passes over A of all jobs, for their roofline
    rid.rid_profile(h, True)
    batch(prec)
    torch.cuda.synchronize()
    rid.rid_profile(h, False)
    kern = {}
    for kid, name in rid.KERNEL_NAMES.items():
        tot, cnt = rid.rid_profile_read(h, kid)
        if cnt:
            kern[name] = {"total_ms": tot, "launches": cnt, "avg_ms": tot / cnt}
    rooflines = {}
    for name in ("residual_ax", "residual_ahz"):
        if name in kern:
            ach = bytes_a / (kern[name]["avg_ms"] * 1e-3) / 1e9
            rooflines[name] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                               "algorithmic_bytes_per_launch": bytes_a,
                               "avg_launch_ms": kern[name]["avg_ms"]}
    if args.no_single:
        As = []
    # the plain FP64 single-ID path, one ID at a time, same matrices
    for i in range(min(4, len(As))):
        rid.rid_decompose(h, As[i], ks[i], ls[i], seed=seeds[i], q=q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat = []
    for i in range(len(As)):
        a = time.perf_counter()
        rid.rid_decompose(h, As[i], ks[i], ls[i], seed=seeds[i], q=q)
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    rid.rid_destroy(h)
    import numpy as np
    single = None
    if lat:
        single = {"ids_per_s": len(lat) / t_single,
                  "p50_ms": float(np.percentile(lat, 50) * 1e3),
                  "p99_ms": float(np.percentile(lat, 99) * 1e3)}
    out = {
        "metric": "A GB/s streamed & IDs/sec at <=1e-10 rel err; p50/p99 latency vs plain FP64",
        "value": 2 * q * bytes_a / t_batch / 1e9,
        "unit": "GB/s",
        "ids_per_s": len(shapes) / t_batch,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": t_batch * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE_TEXT[args.prec],
        "data": "synthetic",
        "config": {"workload": "batched randomized IDs: %d jobs, m log-uniform [256, 4096], "
                               "n log-uniform [128, 2048], k uniform [8, 64], l = k + 8, "
                               "A = X W + 1e-7 N %s, q=%d" % (len(shapes), args.dtype, q),
                   "jobs": len(shapes), "bytes_A": bytes_a, "storage": args.dtype,
                   "sketch_products": args.prec},
        "plan": {"sketch_split_rows": plan[0], "ax_block_bytes": plan[1],
                 "ahz_cols_per_wave": plan[2], "tuned": not args.no_tune,
                 "default_plan": {"sketch_split_rows": plan_default[0],
                                  "ax_block_bytes": plan_default[1],
                                  "ahz_cols_per_wave": plan_default[2],
                                  "ms_per_step": t_default * 1e3}},
        "single_fp64_one_at_a_time": single,
        "speedup_vs_single": t_single / t_batch if lat else None,
        "kernels": kern,
        "rooflines": rooflines,
    }
    del As
    torch.cuda.empty_cache()
    return out


def serving_trace(args, seed: int = 0):
    """Arrival times (Poisson, args.rate per second over args.duration s)
    and per-request shapes: with probability p_big a big complex128 job,
    otherwise a job of the batched workload's distribution (complex64)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    small = iter(batch_shapes(1 << 16, seed + 1))
    while True:
        t += rng.exponential(1.0 / args.rate)
        if t >= args.duration:
            break
        if rng.uniform() < args.p_big:
            k = args.big_k
            out.append((t, True, args.big_m, args.big_n, k, k + 8))
        else:
            m, n, k, l = next(small)
            out.append((t, False, m, n, k, l))
    return out


def run_trace(rid, synth, torch, trace, q, big_lanes, batch_lanes, max_batch, prec):
    """Submit `trace` at its arrival times; returns per-request records."""
    import numpy as np
    chunk = 1024

    def fill(ticket, req):
        dt = torch.complex128 if req["dtype"] == rid.RID_C128 else torch.complex64
        noise = 1e-12 if req["big"] else 1e-7
        return synth.lowrank_device(req["m"], req["n"], req["k"], noise, seed=req["gen_seed"],
                                    dtype=dt, col_chunk=chunk).t()

    srv = rid.RidServer(fill, big_bytes=1 << 30, big_lanes=big_lanes, batch_lanes=batch_lanes,
                        max_batch=max_batch)
    try:
        def submit(i, big, m, n, k, l):
            dt = rid.RID_C128 if big else rid.RID_C64
            fb = 4 * m * chunk * 16 if big else 4 * m * n * 8
            return srv.submit(m, n, k, l, dtype=dt, prec=prec, seed=i, q=q, rank_tol=1e-12,
                              fill_bytes=fb, big=big, gen_seed=i)

        # warm-up: small jobs, and one big job per big lane, grow the lanes'
        # workspaces before the clock starts
        big0 = next((r for r in trace if r[1]), None)
        for i in range(8):
            submit(10 ** 6 + i, False, 1024, 512, 16, 24)
        if big0 is not None:
            for i in range(max(1, big_lanes)):
                submit(10 ** 6 + 99 + i, *big0[1:])
        srv.drain()
        t_base = time.perf_counter()
        tick = []
        for i, (ta, big, m, n, k, l) in enumerate(trace):
            d = t_base + ta - time.perf_counter()
            if d > 0:
                time.sleep(d)
            tick.append(submit(i, big, m, n, k, l))
            if i % 200 == 0:
                print("submitted %d/%d" % (i, len(trace)), file=sys.stderr, flush=True)
        srv.drain()
        recs = []
        for i, t in enumerate(tick):
            r = srv.result(t)
            ta, big, m, n, k, l = trace[i]
            recs.append(dict(big=big, status=r["status"], times=r["times"],
                             bytes=m * n * (16 if big else 8)))
        stats = srv.stats()
    finally:
        srv.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    T = np.array([r["times"] for r in recs])
    lat = T[:, 3] - T[:, 0]
    wall = T[:, 3].max() - T[:, 0].min()
    big = np.array([r["big"] for r in recs])

    def pct(x):
        if len(x) == 0:
            return None
        return {"p50_ms": float(np.percentile(x, 50) * 1e3),
                "p99_ms": float(np.percentile(x, 99) * 1e3), "count": int(len(x))}

    return {
        "ids_per_s": len(recs) / wall,
        "gb_per_s": sum(2 * q * r["bytes"] for r in recs) / wall / 1e9,
        "wall_s": float(wall),
        "all": pct(lat), "small": pct(lat[~big]), "big": pct(lat[big]),
        "fill_ms_p50": float(np.percentile(T[:, 2] - T[:, 1], 50) * 1e3),
        "queue_ms_p99": float(np.percentile(T[:, 1] - T[:, 0], 99) * 1e3),
        "small_service_ms_p99": (float(np.percentile((T[:, 3] - T[:, 2])[~big], 99) * 1e3)
                                 if (~big).any() else None),
        "big_fill_ms": [float(x) * 1e3 for x in (T[:, 2] - T[:, 1])[big]],
        "big_service_ms": [float(x) * 1e3 for x in (T[:, 3] - T[:, 2])[big]],
        "failed": int(sum(r["status"] != 0 for r in recs)),
        "peak_admitted_GB": stats["peak_bytes"] / 1e9,
        "runs": stats["batches"],
    }


def bench_serving(args, torch, rid, synth) -> int:
    print(json.dumps(serving_result(args, torch, rid, synth)))
    return 0


def serving_result(args, torch, rid, synth) -> dict:
    trace = serving_trace(args)
    prec = PRECS[args.prec](rid)
    n_big = sum(1 for r in trace if r[1])
    print("serving trace: %d requests (%d big)" % (len(trace), n_big), file=sys.stderr, flush=True)
    served = run_trace(rid, synth, torch, trace, args.q, big_lanes=args.big_lanes,
                       batch_lanes=args.batch_lanes, max_batch=512, prec=prec)
    print("served: %.1f IDs/s" % served["ids_per_s"], file=sys.stderr, flush=True)
    base = None
    if not args.no_baseline:
        base = run_trace(rid, synth, torch, trace, args.q, big_lanes=0, batch_lanes=1,
                         max_batch=1, prec=rid.RID_FP64)
    out = {
        "metric": "A GB/s streamed & IDs/sec at <=1e-10 rel err; p50/p99 latency vs plain FP64",
        "value": served["ids_per_s"],
        "unit": "IDs/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE_TEXT[args.prec],
        "data": "synthetic",
        "config": {"workload": "served ID requests: Poisson %.0f/s for %.1f s; small jobs m "
                               "log-uniform [256, 4096], n log-uniform [128, 2048], k uniform "
                               "[8, 64], l = k + 8, c64, 1e-7 noise; with probability %.3f a "
                               "c128 %dx%d k=%d l=%d job, 1e-12 noise; q=%d" % (
                                   args.rate, args.duration, args.p_big, args.big_m, args.big_n,
                                   args.big_k, args.big_k + 8, args.q),
                   "requests": len(trace), "big_requests": n_big,
                   "server": "%d batch lanes (up to 512 jobs per batch) + %d big lanes, "
                             "admission by device footprint" % (args.batch_lanes,
                                                                args.big_lanes)},
        "served": served,
        "plain_fp64_one_at_a_time": base,
        # A streamed over the trace's wall time against the HBM peak
        "roofline": {"bound": "hbm", "achieved": served["gb_per_s"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": served["gb_per_s"] / HBM_PEAK_GBS},
    }
    return out


# The shapes of Table 1 (k, m, n) with, as context from another machine, the
# best overall runtime the paper reports for each over 4..128 XMT processors
# (Table 1, seconds) and its error ||A - BP||_2 (Table 5).
TABLE1 = [
    (100, 1 << 14, 1 << 14, 7.16, 5e-11),
    (100, 1 << 16, 1 << 14, 20.46, 1e-10),
    (400, 1 << 16, 1 << 14, 44.2, 2e-10),
    (400, 1 << 18, 1 << 14, 76.83, 4e-10),
    (100, 1 << 16, 1 << 16, 67.87, 2e-10),
    (1000, 1 << 16, 1 << 16, 444.01, 6e-10),
    (400, 1 << 14, 1 << 18, 310.0, 3e-10),
    (1000, 1 << 14, 1 << 18, 1099.0, 6e-10),
]


def bench_sweep(args, torch, rid, synth) -> int:
    """One FP64 ID per Table 1 shape: A = B P (complex Gaussian factors, no
    noise), l = 2k, q power steps; phase times from the library's event
    timing, the whole ID by wall clock."""
    idx = range(len(TABLE1)) if args.shapes == "all" else [int(x) for x in args.shapes.split(",")]
    q = args.q
    h = rid.rid_create(0)
    if args.sketch == "srft":
        rid.rid_set_sketch(h, rid.RID_SKETCH_SRFT)
    rows = []
    for i in idx:
        k, m, n, paper_s, paper_err = TABLE1[i]
        l = 2 * k
        print("shape %d: k=%d m=%d n=%d" % (i, k, m, n), file=sys.stderr, flush=True)
        A = synth.lowrank_device(m, n, k, 0.0, seed=i, col_chunk=1024).t()
        torch.cuda.synchronize()
        rid.rid_decompose(h, A, k, l, seed=0, q=2)          # warm-up (workspace, code)
        torch.cuda.synchronize()
        rid.rid_profile(h, True)
        t0 = time.perf_counter()
        J, P, sigma, used = rid.rid_decompose(h, A, k, l, seed=0, q=q)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        rid.rid_profile(h, False)
        phase = {}
        for kid, name in rid.KERNEL_NAMES.items():
            tot, cnt = rid.rid_profile_read(h, kid)
            if cnt:
                phase[name] = tot
        # norm of A by a few power steps is not needed: sigma_hat / ||A||_F as scale
        a_fro = float(torch.linalg.vector_norm(A).item())
        rows.append({
            "shape": {"k": k, "m": m, "n": n, "l": l, "bytes_A": 16 * m * n},
            "ms": {"id": wall * 1e3,
                   "sketch": phase.get("sketch"), "gram_schmidt_qr": phase.get("pivqr"),
                   "factor_R": phase.get("interp"),
                   "residual": (phase.get("residual_ax", 0.0) + phase.get("residual_ahz", 0.0))},
            "A_GB_per_s": 2 * q * 16.0 * m * n / wall / 1e9,
            "sigma_hat": float(sigma.cpu()[0]), "A_fro": a_fro, "seed_used": used,
            "identity_on_J": bool((P[:, J.cpu()].cpu() ==
                                   torch.eye(k, dtype=torch.complex128)).all()),
            "paper_context": {"best_xmt_runtime_s": paper_s, "error": paper_err},
        })
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
        del A, J, P, sigma
        torch.cuda.empty_cache()
    rid.rid_destroy(h)
    out = {
        "metric": "A GB/s streamed & IDs/sec at <=1e-10 rel err; p50/p99 latency vs plain FP64",
        "value": None, "unit": "GB/s", "n_gpus": 1, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "the paper's Table 1 shapes, A = B P with complex Gaussian "
                               "B (m x k) and P (k x n), no noise, l = 2k, q=%d, %s operator"
                               % (q, "S F D" if args.sketch == "srft" else "Gaussian")},
        "rows": rows,
    }
    print(json.dumps(out))
    return 0


QR_SHAPES = [(108, 16384, 100), (200, 16384, 100), (800, 16384, 400), (2000, 65536, 1000),
             (800, 1 << 18, 400), (2000, 1 << 18, 1000)]


def bench_qr(args, torch, rid, synth) -> int:
    """The two pivoted-QR methods on the same sketches (l x n, first k
    pivots): Householder against CGS2, Sec. 3.2's comparison.  The last two
    shapes are the Y of the sweep's k = 400 and k = 1000 rows at n = 2^18
    (the panel form)."""
    idx = range(len(QR_SHAPES)) if args.shapes == "all" else [int(x) for x in args.shapes.split(",")]
    kinds = [("householder", rid.RID_QR_HOUSEHOLDER), ("cgs2", rid.RID_QR_CGS2)]
    if args.qr_kinds != "both":
        kinds = [kd for kd in kinds if kd[0] == args.qr_kinds]
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    h = rid.rid_create(0)
    rows = []
    for i in idx:
        l, n, k = QR_SHAPES[i]
        Y0 = synth.lowrank_device(l, n, k, 1e-10, seed=l).t()   # l x n, column-major
        res = {}
        for name, kind in kinds:
            rid.rid_set_qr(h, kind)
            Y = Y0.clone()
            rid.rid_pivqr(h, Y, k)                                 # warm-up
            torch.cuda.synchronize()
            best = None
            for _ in range(3):
                Y = Y0.clone()
                torch.cuda.synchronize()
                rid.rid_profile(h, True)
                perm, _ = rid.rid_pivqr(h, Y, k)
                torch.cuda.synchronize()
                rid.rid_profile(h, False)
                ms, _ = rid.rid_profile_read(h, rid.RID_KERNEL_PIVQR)
                best = ms if best is None else min(best, ms)
            res[name] = {"ms": best, "J": perm[:k].cpu()}
        row = {"l": l, "n": n, "k": k}
        for name in res:
            row[name + "_ms"] = res[name]["ms"]
        if len(res) == 2:
            row["cgs2_over_householder"] = res["cgs2"]["ms"] / res["householder"]["ms"]
            row["same_J"] = bool(torch.equal(res["householder"]["J"], res["cgs2"]["J"]))
        rows.append(row)
        del Y0, Y
        torch.cuda.empty_cache()
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    rid.rid_set_qr(h, rid.RID_QR_HOUSEHOLDER)
    rid.rid_destroy(h)
    print(json.dumps({"metric": "pivoted QR time, Householder vs CGS2", "rows": rows}))
    return 0


def bench_svd(args, torch, rid, synth) -> int:
    """The SVD built on the ID (rid_svd) after one ID of the benchmark matrix:
    time per SVD, Jacobi sweeps, and the orthogonality of U and V."""
    m, n, k, l, q = args.m, args.n, args.k, args.l, args.q
    torch.cuda.set_device(0)
    print("generating A %d x %d c128 on the GPU" % (m, n), file=sys.stderr, flush=True)
    A = synth.lowrank_device(m, n, k, args.noise, seed=0).t()
    h = rid.rid_create(0)
    rid.rid_reserve(h, m, n, l, k)
    t0 = time.perf_counter()
    J, P, sigma, _ = rid.rid_decompose(h, A, k, l, seed=0, q=q)
    torch.cuda.synchronize()
    id_ms = (time.perf_counter() - t0) * 1e3
    U = torch.empty((k, m), dtype=torch.complex128, device="cuda").t()
    V = torch.empty((k, n), dtype=torch.complex128, device="cuda").t()
    S = torch.zeros(k, dtype=torch.float64, device="cuda")
    sweeps = 0
    for i in range(args.warmup):
        _, _, _, sweeps = rid.rid_svd(h, A, J, P, U=U, S=S, V=V)
        print("warmup %d done (%d sweeps)" % (i, sweeps), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, _, sweeps = rid.rid_svd(h, A, J, P, U=U, S=S, V=V)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    eye = torch.eye(k, dtype=torch.complex128, device="cuda")
    orth_u = float((U.conj().t() @ U - eye).abs().max())
    orth_v = float((V.conj().t() @ V - eye).abs().max())
    Sh = S.cpu().numpy()
    rid.rid_destroy(h)
    print(json.dumps({"metric": "SVD of A(:,J) P after the ID", "m": m, "n": n, "k": k,
                      "ms_per_svd": ms, "id_ms_first_call": id_ms, "sweeps": sweeps,
                      "orth_U": orth_u, "orth_V": orth_v, "S0": float(Sh[0]),
                      "S_k_over_S0": float(Sh[-1] / Sh[0]),
                      "sigma_id": float(sigma.cpu()[0])}))
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--m", type=int, default=131072)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--k", type=int, default=100)
    ap.add_argument("--l", type=int, default=108)
    ap.add_argument("--q", type=int, default=10)
    ap.add_argument("--noise", type=float, default=1e-12)
    ap.add_argument("--rho", type=float, default=None,
                    help="set the noise so that sigma_{k+1} ~ rho ||A||_2 (overrides --noise)")
    ap.add_argument("--dtype", choices=["c128", "c64"], default="c128",
                    help="storage of A")
    ap.add_argument("--prec", choices=["fp64", "fp32", "bf16x2", "bf16x3"], default="fp64",
                    help="arithmetic of the sketch products (QR, solve, residual stay double)")
    ap.add_argument("--sketch", choices=["gaussian", "srft"], default="gaussian",
                    help="random operator: Gaussian G, or the paper's S F D (four-step DFT "
                         "form when m is a multiple of 8)")
    ap.add_argument("--compare-fp64", action="store_true",
                    help="with --prec fp32/bf16x2/bf16x3: also run the FP64-products ID on the same A "
                         "(same seed) and report J agreement and the P and sigma differences")
    ap.add_argument("--cpu-cols", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--form", choices=["single", "batched", "serving", "sweep", "qr", "svd"],
                    default="single",
                    help="single: one large ID per step (default); batched: many uneven IDs "
                         "per call, compared with the single-ID FP64 path run one at a time; "
                         "serving: a Poisson request stream through the continuous-batching "
                         "server, compared with the plain FP64 path one request at a time; "
                         "sweep: the paper's Table 1 shapes (l = 2k, A = B P) with per-phase "
                         "times; qr: Householder against CGS2 pivoted QR; svd: the SVD built "
                         "on the ID")
    ap.add_argument("--qr-kinds", choices=["both", "householder", "cgs2"], default="both",
                    help="qr: the QR methods to time")
    ap.add_argument("--shapes", default="all",
                    help="sweep (qr): comma-separated indices into the Table 1 shapes "
                         "(QR_SHAPES), or all")
    ap.add_argument("--rate", type=float, default=200.0, help="serving: requests per second")
    ap.add_argument("--duration", type=float, default=4.0,
                    help="serving: seconds of arrivals")
    ap.add_argument("--p-big", type=float, default=0.01,
                    help="serving: probability that a request is a big complex128 job")
    ap.add_argument("--big-m", type=int, default=262144)
    ap.add_argument("--big-n", type=int, default=16384)
    ap.add_argument("--big-k", type=int, default=64)
    ap.add_argument("--batch-lanes", type=int, default=2, help="serving: batch lanes")
    ap.add_argument("--big-lanes", type=int, default=2, help="serving: big-job lanes")
    ap.add_argument("--no-baseline", action="store_true",
                    help="serving: skip the one-at-a-time replay")
    ap.add_argument("--jobs", type=int, default=512, help="IDs per batch (--form batched)")
    ap.add_argument("--no-tune", action="store_true",
                    help="--form batched: time the default batch plan only (no autotuning)")
    ap.add_argument("--no-single", action="store_true",
                    help="--form batched: skip the one-at-a-time comparison")
    ap.add_argument("--no-forms", action="store_true",
                    help="default line only: skip the precision, batched and served forms "
                         "that follow it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run three plain 1 GiB device copies (torch copy_), the "
                         "reference kernel for scaling HBM counter readings")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d, WORLD_SIZE %d requested)" % (args.gpus, world), file=sys.stderr)
        return 2

    import torch

    import paper_1205_3830_amd as rid
    import synth

    if args.form == "batched":
        return bench_batched(args, torch, rid, synth)
    if args.form == "serving":
        return bench_serving(args, torch, rid, synth)
    if args.form == "sweep":
        return bench_sweep(args, torch, rid, synth)
    if args.form == "qr":
        return bench_qr(args, torch, rid, synth)
    if args.form == "svd":
        return bench_svd(args, torch, rid, synth)

    out = single_result(args, torch, rid, synth)
    default_cfg = (args.dtype == "c128" and args.prec == "fp64" and args.sketch == "gaussian"
                   and (args.m, args.n, args.k, args.l, args.q) == (131072, 16384, 100, 108, 10))
    if default_cfg and not args.no_forms:
        out["forms"] = forms_result(args, torch, rid, synth, out)
    print(json.dumps(out))
    return 0


def single_result(args, torch, rid, synth, A=None) -> dict:
    """One large ID per step (the single form); A is generated here unless
    given.  Returns the result record."""
    m, n, k, l, q = args.m, args.n, args.k, args.l, args.q
    torch.cuda.set_device(0)
    tdt = torch.complex128 if args.dtype == "c128" else torch.complex64
    esize = 16 if args.dtype == "c128" else 8
    prec = PRECS[args.prec](rid)
    noise = args.noise
    if args.rho is not None:
        # ||X W||_2 ~ (sqrt(m) + sqrt(k)) (sqrt(n) + sqrt(k)) for Gaussian factors
        noise = args.rho * (m ** 0.5 + k ** 0.5) * (n ** 0.5 + k ** 0.5) / (m ** 0.5 + n ** 0.5)
    own_A = A is None
    if own_A:
        print("generating A %d x %d %s on the GPU" % (m, n, args.dtype), file=sys.stderr,
              flush=True)
        A = synth.lowrank_device(m, n, k, noise, seed=0, dtype=tdt).t()  # (m, n), stride (1, m)
        torch.cuda.synchronize()
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    h = rid.rid_create(0)
    if args.sketch == "srft":
        rid.rid_set_sketch(h, rid.RID_SKETCH_SRFT)
    rid.rid_reserve(h, m, n, l, k)
    J = torch.empty(k, dtype=torch.int64, device="cuda")
    P = torch.empty((n, k), dtype=torch.complex128, device="cuda").t()
    sigma = torch.zeros(1, dtype=torch.float64, device="cuda")

    def step():
        return rid.rid_decompose(h, A, k, l, seed=0, q=q, J=J, P=P, sigma=sigma, prec=prec,
                                 rank_tol=RANK_TOL[args.prec])

    for i in range(args.warmup):
        step()
        print("warmup %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    rid.rid_profile(h, True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rid.rid_profile(h, False)
    ms = (t1 - t0) * 1e3 / args.steps
    bytes_a = float(esize) * m * n
    passes = 2 * q
    gbs = passes * bytes_a / (ms * 1e-3) / 1e9

    kern = {}
    for kid, name in rid.KERNEL_NAMES.items():
        tot, cnt = rid.rid_profile_read(h, kid)
        if cnt:
            kern[name] = {"total_ms": tot, "launches": cnt, "avg_ms": tot / cnt}
    default_cfg = (args.dtype == "c128" and args.prec == "fp64" and args.sketch == "gaussian"
                   and (m, n, k, l, q) == (131072, 16384, 100, 108, 10))
    rooflines = {}
    for name, src in (("residual_ax", "residual.hip"), ("residual_ahz", "residual.hip")):
        if name in kern:
            avg = kern[name]["avg_ms"] * 1e-3
            ach = bytes_a / avg / 1e9
            rooflines[name] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                               "traffic": _traffic(name, src, default_cfg),
                               "algorithmic_bytes_per_launch": bytes_a,
                               "avg_launch_ms": kern[name]["avg_ms"]}
    if "sketch" in kern and args.sketch == "gaussian":
        avg = kern["sketch"]["avg_ms"] * 1e-3
        # the bf16 split forms do six (three) bf16 products per real product
        flops = 8.0 * l * m * n * {"bf16x3": 6, "bf16x2": 3}.get(args.prec, 1)
        ach = flops / avg / 1e12
        peak = {"fp64": FP64_PEAK_TFS, "fp32": FP32_PEAK_TFS, "bf16x2": BF16_PEAK_TFS,
                "bf16x3": BF16_PEAK_TFS}[args.prec]
        rooflines["sketch"] = {"bound": "mfma", "achieved": ach, "peak": peak,
                               "unit": "TFLOP/s", "frac": ach / peak,
                               "traffic": _traffic("sketch", "sketch_f64.hip", default_cfg),
                               "algorithmic_flops_per_launch": flops,
                               "avg_launch_ms": kern["sketch"]["avg_ms"]}
    dominant = max(kern, key=lambda x: kern[x]["total_ms"]) if kern else None
    roof = dict(rooflines.get(dominant, {}))
    if roof:
        roof["kernel"] = dominant

    J_h = J.cpu()
    ok = bool((P[:, J_h].cpu() == torch.eye(k, dtype=torch.complex128)).all())
    vs64 = None
    if args.compare_fp64 and args.prec != "fp64":
        # the FP64-products path on the same A and seed; it is held to 1e-10
        # of the FP64 oracle, which cannot itself run at this size
        J64, P64, s64, _ = rid.rid_decompose(h, A, k, l, seed=0, q=q, prec=rid.RID_FP64)
        torch.cuda.synchronize()
        j_lo, j_hi = J_h.tolist(), J64.cpu().tolist()
        lead = next((t for t in range(k) if j_lo[t] != j_hi[t]), k)
        pmax = float(P64.abs().max())
        s_lo, s_hi = float(sigma.cpu()[0]), float(s64.cpu()[0])
        vs64 = {"J_leading_match": lead, "J_same_set": sorted(j_lo) == sorted(j_hi),
                "P_max_abs_diff_rel": float((P - P64).abs().max()) / max(1.0, pmax),
                "sigma": s_lo, "sigma_fp64": s_hi, "sigma_rel_diff": abs(s_lo - s_hi) / s_hi}

    out = {
        "metric": "A GB/s streamed & IDs/sec at <=1e-10 rel err; p50/p99 latency vs plain FP64",
        "value": gbs,
        "unit": "GB/s",
        "ids_per_s": 1e3 / ms,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE_TEXT[args.prec],
        "data": "synthetic",
        "config": {"workload": "%s randomized ID, A = X W + %g N %s, "
                               "%d x %d, k=%d, l=%d, q=%d power steps (%d passes over A)"
                               % ("plain FP64" if args.prec == "fp64" and args.dtype == "c128"
                                  else "%s storage, %s sketch" % (args.dtype, args.prec),
                                  noise, args.dtype, m, n, k, l, q, passes)
                               + ("" if args.sketch == "gaussian" else
                                  ", S F D operator (four-step DFT)"),
                   "m": m, "n": n, "k": k, "l": l, "q": q, "bytes_A": bytes_a,
                   "storage": args.dtype, "sketch_products": args.prec,
                   "operator": args.sketch},
        "roofline": roof,
        "kernels": kern,
        "rooflines": rooflines,
        "sigma": float(sigma.cpu()[0]),
        "identity_on_J": ok,
    }
    if vs64 is not None:
        out["vs_fp64_path"] = vs64
    if (not args.no_cpu_baseline and args.cpu_cols > 0 and args.dtype == "c128"
            and args.sketch == "gaussian"):
        print("timing the CPU oracle on a column sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(A, k, l, q, min(args.cpu_cols, n))
    rid.rid_destroy(h)
    if own_A:
        del A
        torch.cuda.empty_cache()
    return out




def forms_result(args, torch, rid, synth, fp64_line) -> dict:
    """The precision, batched and served forms, each in short, next to the
    plain FP64 line: complex64 storage of the same shape at rho = 1e-6 with
    FP64, FP32, BF16x2 and BF16x3 sketch products; the 512-job batch with
    FP64 and FP32 products; a 2-second served trace against the plain FP64
    path one request at a time."""
    import copy
    ms64 = fp64_line["ms_per_step"]

    def frac(rec, name):
        r = rec.get("rooflines", {}).get(name)
        return round(r["frac"], 4) if r else None

    forms = {}
    pa = copy.copy(args)
    pa.dtype, pa.rho, pa.steps, pa.warmup = "c64", 1e-6, 3, 1
    pa.no_cpu_baseline, pa.compare_fp64 = True, True
    m, n, k = pa.m, pa.n, pa.k
    noise = pa.rho * (m ** 0.5 + k ** 0.5) * (n ** 0.5 + k ** 0.5) / (m ** 0.5 + n ** 0.5)
    print("forms: precision (c64, rho 1e-6)", file=sys.stderr, flush=True)
    A = synth.lowrank_device(m, n, k, noise, seed=0, dtype=torch.complex64).t()
    torch.cuda.synchronize()
    prec_rows = {}
    for p in ("fp64", "fp32", "bf16x2", "bf16x3"):
        pa.prec = p
        pa.compare_fp64 = p != "fp64"
        rec = single_result(pa, torch, rid, synth, A=A)
        print("forms: precision %s: %.2f ms per ID" % (p, rec["ms_per_step"]), file=sys.stderr,
              flush=True)
        row = {"ms": round(rec["ms_per_step"], 3), "ids_per_s": round(rec["ids_per_s"], 3),
               "A_GB_per_s": round(rec["value"], 1),
               "speedup_vs_plain_fp64": round(ms64 / rec["ms_per_step"], 3),
               "sketch_frac": frac(rec, "sketch"), "ax_hbm_frac": frac(rec, "residual_ax"),
               "ahz_hbm_frac": frac(rec, "residual_ahz")}
        v = rec.get("vs_fp64_path")
        if v:
            row.update({"J_leading_match": v["J_leading_match"],
                        "P_diff_rel": float("%.3g" % v["P_max_abs_diff_rel"]),
                        "sigma_rel_diff": float("%.3g" % v["sigma_rel_diff"])})
        prec_rows[p] = row
    del A
    torch.cuda.empty_cache()
    forms["precision_c64_rho1e-6"] = prec_rows

    ba = copy.copy(args)
    ba.jobs, ba.dtype, ba.steps, ba.no_tune, ba.no_single = 512, "c64", 5, False, False
    batch_rows = {}
    single_ids = 0.0
    for p in ("fp64", "fp32", "bf16x2", "bf16x3"):
        ba.prec = p
        # the one-at-a-time FP64 comparison is the same for every row
        ba.no_single = p not in ("fp64", "fp32")
        print("forms: batched %s" % p, file=sys.stderr, flush=True)
        rec = batched_result(ba, torch, rid, synth)
        print("forms: batched %s: %.2f ms per batch" % (p, rec["ms_per_step"]), file=sys.stderr,
              flush=True)
        single = rec["single_fp64_one_at_a_time"] or {}
        if single:
            single_ids = single["ids_per_s"]
        batch_rows[p] = {"ms": round(rec["ms_per_step"], 3), "ids_per_s": round(rec["ids_per_s"], 1),
                         "A_GB_per_s": round(rec["value"], 1),
                         "ax_hbm_frac": frac(rec, "residual_ax"),
                         "ahz_hbm_frac": frac(rec, "residual_ahz"),
                         "single_fp64_ids_per_s": round(single_ids, 1),
                         "speedup_vs_single": round(rec["ids_per_s"] / single_ids, 2)
                         if single_ids else None}
    forms["batched_512_c64"] = batch_rows

    sa = copy.copy(args)
    sa.duration, sa.rate, sa.prec, sa.no_baseline = 2.0, 200.0, "fp64", False
    print("forms: serving", file=sys.stderr, flush=True)
    rec = serving_result(sa, torch, rid, synth)
    print("forms: serving: %.1f IDs/s" % rec["value"], file=sys.stderr, flush=True)
    sv, base = rec["served"], rec["plain_fp64_one_at_a_time"] or {}

    def lat(x, key):
        return round(x[key], 2) if x else None

    forms["serving_2s"] = {
        "requests": rec["config"]["requests"], "big": rec["config"]["big_requests"],
        "ids_per_s": round(sv["ids_per_s"], 1), "A_GB_per_s": round(sv["gb_per_s"], 1),
        "hbm_frac": round(rec["roofline"]["frac"], 4),
        "small_p50_ms": lat(sv["small"], "p50_ms"), "small_p99_ms": lat(sv["small"], "p99_ms"),
        "big_p50_ms": lat(sv["big"], "p50_ms"),
        "plain_fp64": {"ids_per_s": round(base.get("ids_per_s", 0.0), 1),
                       "small_p50_ms": lat(base.get("small"), "p50_ms"),
                       "small_p99_ms": lat(base.get("small"), "p99_ms"),
                       "big_p50_ms": lat(base.get("big"), "p50_ms")},
        "failed": sv["failed"]}
    return forms


if __name__ == "__main__":
    sys.exit(main())
