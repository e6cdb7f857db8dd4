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
    q = args.q
    shapes = batch_shapes(args.jobs)
    dt = torch.complex64 if args.dtype == "c64" else torch.complex128
    esize = 8 if args.dtype == "c64" else 16
    prec = rid.RID_FP64 if args.prec == "fp64" else rid.RID_FP32
    tol = 1e-12 if prec == rid.RID_FP64 else 1e-5
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

    batch(prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        Js, Ps, sig, status, _ = batch(prec)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    assert all(s == 0 for s in status)
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
        "dtype": "f64" if args.prec == "fp64" else "f32 sketch products, f64 QR/solve/residual",
        "data": "synthetic",
        "config": {"workload": "batched randomized IDs: %d jobs, m log-uniform [256, 4096], "
                               "n log-uniform [128, 2048], k uniform [8, 64], l = k + 8, "
                               "A = X W + 1e-7 N %s, q=%d" % (len(shapes), args.dtype, q),
                   "jobs": len(shapes), "bytes_A": bytes_a, "storage": args.dtype,
                   "sketch_products": args.prec},
        "single_fp64_one_at_a_time": single,
        "speedup_vs_single": t_single / t_batch if lat else None,
    }
    print(json.dumps(out))
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
    ap.add_argument("--prec", choices=["fp64", "fp32"], default="fp64",
                    help="arithmetic of the sketch products (QR, solve, residual stay double)")
    ap.add_argument("--cpu-cols", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--form", choices=["single", "batched"], default="single",
                    help="single: one large ID per step (default); batched: many uneven IDs "
                         "per call, compared with the single-ID FP64 path run one at a time")
    ap.add_argument("--jobs", type=int, default=512, help="IDs per batch (--form batched)")
    ap.add_argument("--no-single", action="store_true",
                    help="--form batched: skip the one-at-a-time comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run three plain 1 GiB device copies (torch copy_), the "
                         "reference kernel for scaling HBM counter readings")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d, WORLD_SIZE %d requested)" % (args.gpus, world), file=sys.stderr)
        return 2

    import torch

    import paper_1205_3830_amd as rid
    import synth

    if args.form == "batched":
        return bench_batched(args, torch, rid, synth)

    m, n, k, l, q = args.m, args.n, args.k, args.l, args.q
    torch.cuda.set_device(0)
    tdt = torch.complex128 if args.dtype == "c128" else torch.complex64
    esize = 16 if args.dtype == "c128" else 8
    prec = rid.RID_FP64 if args.prec == "fp64" else rid.RID_FP32
    noise = args.noise
    if args.rho is not None:
        # ||X W||_2 ~ (sqrt(m) + sqrt(k)) (sqrt(n) + sqrt(k)) for Gaussian factors
        noise = args.rho * (m ** 0.5 + k ** 0.5) * (n ** 0.5 + k ** 0.5) / (m ** 0.5 + n ** 0.5)
    print("generating A %d x %d %s on the GPU" % (m, n, args.dtype), file=sys.stderr, flush=True)
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
    rid.rid_reserve(h, m, n, l, k)
    J = torch.empty(k, dtype=torch.int64, device="cuda")
    P = torch.empty((n, k), dtype=torch.complex128, device="cuda").t()
    sigma = torch.zeros(1, dtype=torch.float64, device="cuda")

    def step():
        return rid.rid_decompose(h, A, k, l, seed=0, q=q, J=J, P=P, sigma=sigma, prec=prec,
                                 rank_tol=1e-12 if prec == rid.RID_FP64 else 1e-5)

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
    default_cfg = (args.dtype == "c128" and args.prec == "fp64" and (m, n, k, l, q) ==
                   (131072, 16384, 100, 108, 10))
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
    if "sketch" in kern:
        avg = kern["sketch"]["avg_ms"] * 1e-3
        ach = 8.0 * l * m * n / avg / 1e12
        peak = FP64_PEAK_TFS if args.prec == "fp64" else FP32_PEAK_TFS
        rooflines["sketch"] = {"bound": "mfma", "achieved": ach, "peak": peak,
                               "unit": "TFLOP/s", "frac": ach / peak,
                               "traffic": _traffic("sketch", "sketch_f64.hip", default_cfg),
                               "algorithmic_flops_per_launch": 8.0 * l * m * n,
                               "avg_launch_ms": kern["sketch"]["avg_ms"]}
    dominant = max(kern, key=lambda x: kern[x]["total_ms"]) if kern else None
    roof = dict(rooflines.get(dominant, {}))
    if roof:
        roof["kernel"] = dominant

    J_h = J.cpu()
    ok = bool((P[:, J_h].cpu() == torch.eye(k, dtype=torch.complex128)).all())

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
        "dtype": "f64" if args.prec == "fp64" else "f32 sketch products, f64 QR/solve/residual",
        "data": "synthetic",
        "config": {"workload": "%s randomized ID, A = X W + %g N %s, "
                               "%d x %d, k=%d, l=%d, q=%d power steps (%d passes over A)"
                               % ("plain FP64" if args.prec == "fp64" and args.dtype == "c128"
                                  else "%s storage, %s sketch" % (args.dtype, args.prec),
                                  noise, args.dtype, m, n, k, l, q, passes),
                   "m": m, "n": n, "k": k, "l": l, "q": q, "bytes_A": bytes_a,
                   "storage": args.dtype, "sketch_products": args.prec},
        "roofline": roof,
        "kernels": kern,
        "rooflines": rooflines,
        "sigma": float(sigma.cpu()[0]),
        "identity_on_J": ok,
    }
    if not args.no_cpu_baseline and args.cpu_cols > 0 and args.dtype == "c128":
        print("timing the CPU oracle on a column sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(A, k, l, q, min(args.cpu_cols, n))
    rid.rid_destroy(h)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
