"""Benchmark: time-to-solution of the mixed-precision nested RAS-BiCGStab
solver on one MI355X, beside the plain FP64 BiCGStab on the same GPU, plus
the Wilson-clover D-apply against the HBM roofline.

Workload (one step = one complete solve to |eta - D phi|/|eta| <= 1e-10):
  16^3 x 32 lattice, random SU(3) links exp(i eps H) with eps = 0.5 (seed 1),
  kappa = 0.125, c_sw = 1.0, Gaussian source (seed 2); FP64 outer / FP32 inner
  BiCGStab preconditioned by RAS with 8^4 domains, overlap s (default 0),
  N_dominv = 4 minimal-residual steps, NRAS = 3 sweeps.
Inputs are resident in HBM before the timed region.

Prints one JSON line (see the design doc for every field).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-solution @1e-10 residual vs plain FP64 BiCGStab; D-apply GB/s; p99 ms"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per site of one D application (links 12 reals x 4 + clover
# 72 reals + spinor in + spinor out, each field touched once)
DAPPLY_BYTES = {0: 1344, 1: 672, 2: 348}
DAPPLY_FLOPS = 1872


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--overlap", type=int, default=0, help="RAS overlap s (depth d = 2s)")
    ap.add_argument("--block", default="8x8x8x8", help="RAS domain shape, e.g. 8x8x8x8 or 4x4x4x4")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16"], help="RAS storage precision")
    ap.add_argument("--n-dominv", type=int, default=4)
    ap.add_argument("--n-ras", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dapply", action="store_true")
    ap.add_argument("--mode", default="full", choices=["full", "dapply", "copyref"],
                    help="dapply: only the 32^4 FP32 D-apply loop; copyref: a 1 GiB device copy "
                         "(the reference kernel for scaling rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    return ap.parse_args()


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("wcl_dslash.hip", "wcl_device.h", "wcl_internal.h"):
        with open(os.path.join(ROOT, "paper_1011_3318_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(prec: int, V: int):
    """HBM bytes per launch from the rocprofv3 FETCH_SIZE/WRITE_SIZE runs,
    if they were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "dapply_counters.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = rec.get(str(prec))
    if not ent or rec.get("source_hash") != kernel_source_hash() or ent.get("V") != V:
        return None
    return ent.get("bytes_per_launch")


def time_dapply(W, torch, lat, prec, n_warm=10, n_timed=100):
    import numpy as np
    from paper_1011_3318_amd import inputs as I
    psi = I.gaussian_source(lat.dims, 2)
    xs = [lat.pack(psi, prec) for _ in range(3)]
    ys = [lat.empty(prec) for _ in range(3)]
    for k in range(n_warm):
        lat.apply_D(prec, 0.125, 1.0, xs[k % 3], ys[k % 3])
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for k in range(n_timed):
        lat.apply_D(prec, 0.125, 1.0, xs[k % 3], ys[(k + 1) % 3])
    e.record()
    torch.cuda.synchronize()
    us = s.elapsed_time(e) / n_timed * 1e3
    del xs, ys
    _ = np
    return us


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path in this build "
              "(every domain of the lattice lives on one device); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1011_3318_amd import inputs as I
    from paper_1011_3318_amd import wcl as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.mode == "copyref":
        n = 1 << 30
        a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(5):
            b.copy_(a)
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / 5
        print(json.dumps({"mode": "copyref", "bytes_read_per_copy": n, "bytes_written_per_copy": n, "copies": 6,
                          "ms_per_copy": ms, "GBps_read_plus_write": 2 * n / ms / 1e6}))
        return
    if args.mode == "dapply":
        ctx = W.Context(0)
        big = (32, 32, 32, 32)
        lb = W.Lattice(ctx, big)
        lb.upload_gauge(I.random_gauge(big, 1.0, 1))
        us = time_dapply(W, torch, lb, 1, n_warm=3, n_timed=10)
        print(json.dumps({"mode": "dapply", "V": lb.V, "us": us, "launches": 13}))
        lb.close()
        ctx.close()
        return
    dims = (16, 16, 16, 32)
    kappa, csw, tol = 0.125, 1.0, 1e-10
    block = tuple(int(v) for v in args.block.split("x"))
    s, nd, nras = args.overlap, args.n_dominv, args.n_ras
    storage = W.F16 if args.storage == "f16" else W.F32
    ctx = W.Context(0)
    lat = W.Lattice(ctx, dims)
    U = I.random_gauge(dims, 0.5, 1)
    lat.upload_gauge(U)
    eta = I.gaussian_source(dims, 2)
    e = lat.pack(eta, W.F64)
    phi = lat.zeros(W.F64)
    params = W.SolverParams.make(tol_outer=tol, tol_inner=1e-4, max_outer=200, max_inner=100,
                                 ras=W.RasParams.make(block=block, s=s, n_ras=nras, n_dominv=nd, storage=storage))

    # ---- nested RAS solve: warmup, then exactly K timed steps
    for _ in range(args.warmup):
        lat.solve_nested(params, kappa, csw, e, phi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(args.steps):
        rc, st = lat.solve_nested(params, kappa, csw, e, phi)
        stats.append(st)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    ms_per_step = T / args.steps * 1e3
    true_res = max(st["true_resid"] for st in stats)

    # ---- plain FP64 BiCGStab on the same GPU and input
    for _ in range(args.warmup):
        lat.solve_bicgstab_f64(tol, 100000, kappa, csw, e, phi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rc, pst = lat.solve_bicgstab_f64(tol, 100000, kappa, csw, e, phi)
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t0) / args.steps * 1e3
    lat.close()

    # ---- D-apply against the HBM roofline at 32^4 (does not fit the 256 MB
    # Infinity Cache), FP32 as the graded kernel, FP16/FP64 alongside
    roof = None
    dapply = {}
    if not args.no_dapply:
        big = (32, 32, 32, 32)
        lb = W.Lattice(ctx, big)
        lb.upload_gauge(I.random_gauge(big, 1.0, 1))
        for prec in (1, 2, 0):
            us = time_dapply(W, torch, lb, prec)
            gbs = DAPPLY_BYTES[prec] * lb.V / us / 1e3
            dapply[{0: "f64", 1: "f32", 2: "f16"}[prec]] = {
                "us": round(us, 2), "GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                "gflops": round(DAPPLY_FLOPS * lb.V / us / 1e3, 1)}
        V = lb.V
        f32 = dapply["f32"]
        tb = measured_traffic(1, V)
        roof = {"bound": "hbm", "achieved": f32["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": f32["frac"], "traffic": tb,
                "kernel": "k_dslash<F32> (D-apply, 32^4, 672 B/site algorithmic)"}
        lb.close()

    # ---- CPU baseline: the FP64 oracle's nested RAS solve on the same input
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import Oracle
        o = Oracle(dims, U)
        t0 = time.perf_counter()
        _, info = o.nested(eta, kappa, csw, tol=tol, tol_inner=1e-4, max_inner=100, ras=True, block=block, s=s,
                           n_ras=nras, n_dominv=nd)
        tc = time.perf_counter() - t0
        cpu = {"value": round(1.0 / tc, 5), "unit": "solves/s", "cores": Oracle.num_threads(), "kind": "oracle",
               "sample": f"one complete FP64 nested RAS-BiCGStab solve of the same 16^3x32 system "
                         f"({info['outer_iters']} outer / {info['inner_iters']} inner iterations, {tc:.1f} s)"}

    st0 = stats[-1]
    out = {
        "metric": METRIC,
        "value": round(args.steps / T, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64/f32 (outer FP64, inner and RAS FP32)",
        "data": "synthetic (seeded random SU(3) gauge field and Gaussian source)",
        "config": {"workload": "16^3x32 nested RAS-BiCGStab solve to 1e-10",
                   "lattice": list(dims), "eps": 0.5, "kappa": kappa, "csw": csw, "rhs": 1,
                   "ras": {"block": list(block), "s": s, "n_dominv": nd, "n_ras": nras, "storage": args.storage},
                   "parallelism": "single GPU"},
        "time_to_solution_ms": round(ms_per_step, 3),
        "true_residual": true_res,
        "solve_stats": {k: st0[k] for k in ("outer_iters", "inner_iters", "dslash_full", "dslash_block",
                                             "ras_sweeps")},
        "plain_f64_bicgstab_ms": round(plain_ms, 3),
        "plain_f64_iters": pst["outer_iters"],
        "speedup_vs_plain_f64": round(plain_ms / ms_per_step, 3),
        "dapply_32x4": dapply,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
