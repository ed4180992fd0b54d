"""Benchmark: time-to-solution of the mixed-precision nested RAS-BiCGStab
solver on one MI355X, beside the plain FP64 BiCGStab on the same GPU, plus
the Wilson-clover D-apply against the HBM roofline, the 12-source batched
solve, the 32^4 FP16-storage solve and the serving loop.

One step = one complete solve of D phi = eta to |eta - D phi|/|eta| <= 1e-10 on
  16^3 x 32, random SU(3) links exp(i eps H), eps = 0.5 (seed 1),
  kappa = 0.125, c_sw = 1.0, Gaussian source (seed 2);
  FP64 outer / FP32 inner BiCGStab right-preconditioned by RAS
  (N_dominv = 4 minimal-residual steps per sweep).  The domain shape, overlap,
  storage, sweeps and inner tolerance are picked by the library's autotuner
  before the timed region; the literal 8^4 (s = 0 and s = 1) domain solves are
  timed beside it.
Inputs are resident in HBM before every timed region.

Prints one JSON line; --mode selects a single section (dapply, copyref, serve).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-solution @1e-10 residual vs plain FP64 BiCGStab; D-apply GB/s; p99 ms"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per site of one D application: links (4 x 12 reals),
# clover (72 reals), spinor in and out (24 reals each), every field once;
# the FP16 fields carry one FP32 scale per site (spinor in/out, clover)
DAPPLY_BYTES = {0: 1344, 1: 672, 2: 348}
DAPPLY_12RHS_BYTES_F32 = 12 * 192 + 480
DAPPLY_FLOPS = 1872
SERVE_SIZES = [(8, 8, 8, 8), (16, 16, 16, 32), (24, 24, 24, 48), (32, 32, 32, 32)]
SERVE_WEIGHTS = [4, 3, 2, 1]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", default="full", choices=["full", "dapply", "copyref", "serve", "solve", "sweep", "paper"],
                    help="dapply: only the 32^4 FP32 D-apply loop; copyref: a 1 GiB device copy "
                         "(the reference kernel for scaling rocprofv3 FETCH_SIZE/WRITE_SIZE); serve: only the "
                         "serving run; solve: K timed 16^3x32 solves with the RAS parameters given below "
                         "(no autotuning), for kernel traces; sweep: 55 launches of one RAS sweep (NRAS = 1) of the "
                         "on-chip domain solver with those parameters, for counters; paper: the paper's 32^4 "
                         "x-split table with the NRAS x N_dominv scan")
    ap.add_argument("--block", default="4x4x4x4", help="solve mode: domain shape")
    ap.add_argument("--overlap", type=int, default=0, help="solve mode: overlap s")
    ap.add_argument("--storage", default="f16", choices=["f32", "f16"], help="solve mode: RAS storage")
    ap.add_argument("--dapply-prec", default="f32", choices=["f64", "f32", "f16"], help="dapply mode: precision")
    ap.add_argument("--n-ras", type=int, default=3)
    ap.add_argument("--n-dominv", type=int, default=4)
    ap.add_argument("--tol-inner", type=float, default=1e-4)
    ap.add_argument("--point-sources", action="store_true", help="solve mode: the 12 point sources in one batch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dapply", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the 12-source, 32^4 and serving sections")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper's 32^4 x-split table")
    ap.add_argument("--paper-eps", type=float, default=0.3, help="paper mode: gauge-field eps")
    ap.add_argument("--paper-scan", action="store_true", help="paper mode: add the NRAS x N_dominv scan")
    ap.add_argument("--requests", type=int, default=512, help="serving: number of requests")
    ap.add_argument("--slots", type=int, default=4, help="serving: concurrent solve slots")
    return ap.parse_args()


DAPPLY_SOURCES = ("wcl_dslash.hip", "wcl_device.h", "wcl_internal.h")
DOMAIN_SOURCES = ("wcl_block.hip", "wcl_device.h", "wcl_internal.h")
# FP32 VALU peak without packed-FP32 instructions (the library is built
# without them): 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz
VALU_F32_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# flops of the Wilson-clover operator per site: site term (two 6x6 Hermitian
# mat-vecs + the combination) and one hop (projection, two SU(3) mat-vecs,
# accumulation); 552 + 8 x 165 = 1872
SITE_TERM_FLOPS, HOP_FLOPS = 552, 165
# one minimal-residual step besides q = D rho: <q, rho>, <q, q>, x += a rho, rho -= a q
MR_FLOPS = 96 + 48 + 96 + 96


def source_hash(files) -> str:
    """Hash of the kernel sources with comments and blank lines removed, so
    that a comment edit does not invalidate the stored counter runs."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1011_3318_amd", "csrc", f)) as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for ln in text.splitlines():
            ln = re.sub(r"//.*", "", ln).strip()
            if ln:
                h.update(ln.encode() + b"\n")
    return h.hexdigest()[:16]


def kernel_source_hash() -> str:
    return source_hash(DAPPLY_SOURCES)


def measured_traffic(name: str, files, key: str, V: int):
    """HBM bytes per launch from the rocprofv3 FETCH_SIZE/WRITE_SIZE runs
    stored in profiles/<name>, scaled by the copy-kernel factor, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = rec.get(key)
    if not ent or rec.get("source_hash") != source_hash(files) or ent.get("V") != V:
        return None
    return ent.get("bytes_per_launch")


def domain_sweep_flops(dims, ras, nblocks, ev):
    """Algorithmic flops of one sweep of the domain solver: N_dominv MR steps
    on every extended site, each the Dirichlet domain operator (only the hops
    that stay inside the extended domain) plus the MR vector work."""
    hops = 0.0
    for mu in range(4):
        e = ras.block[mu] + (2 * ras.s if ras.block[mu] < dims[mu] else 0)
        hops += 2.0 * ((e - 1) / e if e < dims[mu] else 1.0)
    per_site = SITE_TERM_FLOPS + HOP_FLOPS * hops + MR_FLOPS
    return per_site * nblocks * ev * ras.n_dominv


def event_time_us(torch, fn, n):
    """Average duration of fn() over n launches on the current stream (HIP events)."""
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for k in range(n):
        fn(k)
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / n * 1e3


def time_dapply(torch, I, lat, prec, nrhs=1, n_warm=10, n_timed=100):
    """D-apply timing: three input and three output copies rotated so that no
    launch starts with its operands in cache."""
    import numpy as np
    psi = I.gaussian_source(lat.dims, 2, nrhs) if nrhs > 1 else I.gaussian_source(lat.dims, 2)
    xs = [lat.pack(psi, prec, nrhs) for _ in range(3)]
    ys = [lat.empty(prec, nrhs) for _ in range(3)]
    for k in range(n_warm):
        lat.apply_D(prec, 0.125, 1.0, xs[k % 3], ys[k % 3], nrhs)
    torch.cuda.synchronize()
    us = event_time_us(torch, lambda k: lat.apply_D(prec, 0.125, 1.0, xs[k % 3], ys[(k + 1) % 3], nrhs), n_timed)
    del xs, ys
    _ = np
    return us


def timed_solves(torch, lat, params, kappa, csw, e, phi, steps, warmup, nrhs=1):
    for _ in range(warmup):
        lat.solve_nested(params, kappa, csw, e, phi, nrhs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(steps):
        _, st = lat.solve_nested(params, kappa, csw, e, phi, nrhs)
        stats.append(st)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3, stats


def time_domain_sweep(torch, W, lat, dims, ras, eta, kappa, csw, n=50):
    """Average duration (HIP events) of one launch of the on-chip domain
    solver: ras_precondition with NRAS = 1 is exactly one k_blk_fused launch
    (projection of the FP32 residual, N_dominv MR steps, restriction)."""
    nb, ev = lat.block_info(ras)
    one = W.RasParams.make(block=tuple(ras.block), s=ras.s, n_ras=1, n_dominv=ras.n_dominv, storage=ras.storage,
                           kernel=W.BLOCK_FUSED)
    r32 = lat.pack(eta, W.F32)
    v32 = lat.empty(W.F32)
    for _ in range(5):
        lat.ras_precondition(one, kappa, csw, r32, v32)
    torch.cuda.synchronize()
    us = event_time_us(torch, lambda k: lat.ras_precondition(one, kappa, csw, r32, v32), n)
    return us, domain_sweep_flops(dims, ras, nb, ev)


def paper_table(torch, W, ctx, dims, U, eta, kappa=0.126, csw=1.0, tol=1e-14, n_ras=3, n_dominv=5, scan=False):
    """The paper's benchmark (Sec. 5, Table 1) on one GPU: 32^4 lattice,
    kappa 0.126, c_SW 1.0, |eta - D phi|/|eta| < 1e-14, the nested solver
    without preconditioner and with RAS on the x-only split into 8 domains
    (L_x/8 x L_y x L_z x L_t) with overlap depth d = 2s = 0, 2, 4, NRAS = 3,
    N_dominv = 5.  Reports time, the full-lattice D count and the domain work;
    with scan=True also the NRAS x N_dominv scan of d = 0."""
    lat = W.Lattice(ctx, dims)
    lat.upload_gauge(U)
    e = lat.pack(eta, W.F64)
    phi = lat.zeros(W.F64)
    xb = (dims[0] // 8, dims[1], dims[2], dims[3])
    out = {"lattice": list(dims), "kappa": kappa, "csw": csw, "tol": tol, "domains": list(xb),
           "n_ras": n_ras, "n_dominv": n_dominv}

    def run(p):
        lat.solve_nested(p, kappa, csw, e, phi, raise_on_notconv=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = lat.solve_nested(p, kappa, csw, e, phi, raise_on_notconv=False)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3, st

    base = dict(tol_outer=tol, tol_inner=1e-4, max_outer=200, max_inner=1000)
    ms, st = run(W.SolverParams.make(precond=W.PRECOND_NONE, **base))
    out["no_prec"] = {"ms": round(ms, 3), "dv_count": st["dslash_full"], "outer_iters": st["outer_iters"],
                      "inner_iters": st["inner_iters"], "true_resid": st["true_resid"],
                      "converged": bool(st["converged"])}
    for s in (0, 1, 2):
        ras = W.RasParams.make(block=xb, s=s, n_ras=n_ras, n_dominv=n_dominv, storage=W.F32)
        ms, st = run(W.SolverParams.make(ras=ras, **base))
        # the domain solver alone: one sweep timed with HIP events, times the sweeps of the solve
        one = W.RasParams.make(block=xb, s=s, n_ras=1, n_dominv=n_dominv, storage=W.F32)
        r32 = lat.pack(eta, W.F32)
        v32 = lat.empty(W.F32)
        lat.ras_precondition(one, kappa, csw, r32, v32)
        torch.cuda.synchronize()
        us_sweep = event_time_us(torch, lambda k: lat.ras_precondition(one, kappa, csw, r32, v32), 5)
        out[f"ras_d{2 * s}"] = {"ms": round(ms, 3), "dv_count": st["dslash_full"], "outer_iters": st["outer_iters"],
                                "inner_iters": st["inner_iters"], "ras_sweeps": st["ras_sweeps"],
                                "domain_mr_steps": st["dslash_block"], "true_resid": st["true_resid"],
                                "converged": bool(st["converged"]),
                                "dominv_ms_est": round(us_sweep * st["ras_sweeps"] / 1e3, 3)}
        del r32, v32
    if scan:
        grid = {}
        for nr in range(1, 11):
            for nd in (1, 2, 3, 4, 5, 6, 8, 10, 12, 15, 20):
                ras = W.RasParams.make(block=xb, s=0, n_ras=nr, n_dominv=nd, storage=W.F32)
                ms, st = run(W.SolverParams.make(ras=ras, **base))
                grid[f"{nr}x{nd}"] = {"ms": round(ms, 3), "dv_count": st["dslash_full"],
                                      "converged": bool(st["converged"])}
            log(f"scan NRAS={nr}: " + ", ".join(f"{k}: {v['ms']:.0f} ms" for k, v in grid.items()
                                                 if k.startswith(f"{nr}x")))
        best = min((k for k in grid if grid[k]["converged"]), key=lambda k: grid[k]["ms"])
        out["scan_d0"] = {"best": best, "grid": grid}
    lat.close()
    return out


def ras_desc(p):
    r = p.ras
    return {"block": list(r.block), "s": r.s, "n_ras": r.n_ras, "n_dominv": r.n_dominv,
            "storage": {0: "f64", 1: "f32", 2: "f16"}[r.storage], "tol_inner": p.tol_inner}


def stats_desc(st):
    return {k: st[k] for k in ("outer_iters", "inner_iters", "restarts", "dslash_full", "dslash_block",
                               "ras_sweeps", "true_resid")}


def pct(a, q):
    import numpy as np
    return float(np.percentile(np.asarray(a), q)) if len(a) else None


def serve_bench(W, I, np, ctx, n_req, slots):
    """Serving mix: lattices 8^4, 16^3x32, 24^3x48, 32^4 with weights 4:3:2:1,
    kappa ~ U[0.115, 0.125], c_sw in {1.0, 1.5}, eps = 0.5 gauge fields (seed 1,
    resident), Gaussian sources with seed 1000 + request id, tolerance 1e-10.
    The request stream (sizes, couplings, Poisson gaps) is drawn from seed 5.
    First a closed loop with 2 x slots requests in flight gives the saturated
    throughput X; then an open loop of Poisson arrivals at rate 0.8 X runs with
    an HBM budget of 24 GB, so admission by free memory binds."""
    from concurrent.futures import ThreadPoolExecutor
    rng = np.random.default_rng(5)
    w = np.asarray(SERVE_WEIGHTS, dtype=float)
    kind = rng.choice(len(SERVE_SIZES), size=n_req, p=w / w.sum())
    kappa = rng.uniform(0.115, 0.125, size=n_req)
    csw = rng.choice(np.array([1.0, 1.5]), size=n_req)
    gaps = rng.exponential(1.0, size=n_req)
    gauges = {}
    for k, d in enumerate(SERVE_SIZES):
        gauges[k] = I.random_gauge(d, 0.5, 1)
    log("serving: gauge fields generated")
    # every source is drawn before the timed runs (12 host threads), so the
    # request loop only submits and polls
    with ThreadPoolExecutor(12) as pool:
        sources = list(pool.map(lambda i: I.gaussian_source(SERVE_SIZES[kind[i]], 1000 + int(i)), range(n_req)))
    log("serving: sources generated")

    def run(budget, arrivals):
        srv = W.Server(ctx, max_slots=slots, hbm_budget=budget)
        for k, d in enumerate(SERVE_SIZES):
            srv.register_gauge(k, d, gauges[k])
        free = {k: [] for k in range(len(SERVE_SIZES))}   # solution buffers returned by finished requests
        inflight, done = {}, []
        nxt, late = 0, 0
        t0 = time.monotonic()
        window = 2 * slots
        while len(done) < n_req:
            while nxt < n_req:
                if arrivals is None and len(inflight) >= window:
                    break
                if arrivals is not None and time.monotonic() < t0 + arrivals[nxt]:
                    break
                if arrivals is not None and time.monotonic() > t0 + arrivals[nxt] + 0.005:
                    late += 1
                k = int(kind[nxt])
                phi = free[k].pop() if free[k] else np.empty_like(sources[nxt])
                t = srv.submit(k, float(kappa[nxt]), float(csw[nxt]), sources[nxt], phi=phi)
                inflight[t] = nxt
                nxt += 1
            for t in list(inflight):
                r = srv.poll(t)
                if r is not None:
                    i = inflight.pop(t)
                    free[int(kind[i])].append(r[0])
                    done.append((i, r[1]))
            time.sleep(0.0005)
        T = time.monotonic() - t0
        srv.close()
        bad = [i for i, r in done if r["status"] != 0 or not r["converged"] or r["true_resid"] > 1e-10]
        lat_ms = []
        for i, r in done:
            # open loop: latency from the scheduled arrival; closed loop: from submit
            start = r["t_submit"] if arrivals is None else t0 + arrivals[i]
            lat_ms.append((r["t_done"] - start) * 1e3)
        svc_ms = [(r["t_done"] - r["t_admit"]) * 1e3 for _, r in done]
        wait_ms = [(r["t_admit"] - r["t_submit"]) * 1e3 for _, r in done]
        per_size = {}
        for k, d in enumerate(SERVE_SIZES):
            ls = [lat_ms[j] for j, (i, _) in enumerate(done) if kind[i] == k]
            per_size["x".join(map(str, d))] = {"n": len(ls), "p50_ms": round(pct(ls, 50), 3) if ls else None,
                                               "p99_ms": round(pct(ls, 99), 3) if ls else None}
        return {"requests": n_req, "seconds": round(T, 3), "solves_per_s": round(n_req / T, 3),
                "p50_ms": round(pct(lat_ms, 50), 3), "p99_ms": round(pct(lat_ms, 99), 3),
                "service_p50_ms": round(pct(svc_ms, 50), 3), "admission_wait_p99_ms": round(pct(wait_ms, 99), 3),
                "failed": len(bad), "late_submits": late, "per_size": per_size}

    closed = run(0, None)
    log(f"serving: closed loop {closed['solves_per_s']} solves/s")
    lam = 0.8 * closed["solves_per_s"]
    arrivals = np.cumsum(gaps) / lam
    opened = run(24 << 30, arrivals)
    opened["rate_per_s"] = round(lam, 3)
    opened["hbm_budget_bytes"] = 24 << 30
    log(f"serving: Poisson p50 {opened['p50_ms']} ms p99 {opened['p99_ms']} ms")
    return {"closed_loop": closed, "poisson": opened, "slots": slots,
            "mix": {"x".join(map(str, d)): wt for d, wt in zip(SERVE_SIZES, SERVE_WEIGHTS)}}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: every domain of the lattice lives on one device and the library has "
              "no multi-GPU path; run it with --gpus 1", file=sys.stderr)
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
        ms = event_time_us(torch, lambda k: b.copy_(a), 5) / 1e3
        print(json.dumps({"mode": "copyref", "bytes_read_per_copy": n, "bytes_written_per_copy": n, "copies": 6,
                          "ms_per_copy": ms, "GBps_read_plus_write": 2 * n / ms / 1e6}))
        return
    ctx = W.Context(0)
    if args.mode == "dapply":
        big = (32, 32, 32, 32)
        lb = W.Lattice(ctx, big)
        lb.upload_gauge(I.random_gauge(big, 1.0, 1))
        prec = {"f64": 0, "f32": 1, "f16": 2}[args.dapply_prec]
        us = time_dapply(torch, I, lb, prec, n_warm=3, n_timed=10)
        print(json.dumps({"mode": "dapply", "prec": args.dapply_prec, "V": lb.V, "us": us,
                          "GBps": DAPPLY_BYTES[prec] * lb.V / us / 1e3, "launches": 13}))
        lb.close()
        ctx.close()
        return
    if args.mode == "paper":
        big = (32, 32, 32, 32)
        tab = paper_table(torch, W, ctx, big, I.random_gauge(big, args.paper_eps, 1), I.gaussian_source(big, 2),
                          scan=args.paper_scan)
        tab["eps"] = args.paper_eps
        print(json.dumps({"mode": "paper", "paper_table1": tab}))
        ctx.close()
        return
    if args.mode == "serve":
        print(json.dumps({"mode": "serve", "serving": serve_bench(W, I, np, ctx, args.requests, args.slots)}))
        ctx.close()
        return

    dims = (16, 16, 16, 32)
    kappa, csw, tol = 0.125, 1.0, 1e-10
    if args.mode == "sweep":
        lat = W.Lattice(ctx, dims)
        lat.upload_gauge(I.random_gauge(dims, 0.5, 1))
        eta = I.gaussian_source(dims, 2)
        ras = W.RasParams.make(block=tuple(int(v) for v in args.block.split("x")), s=args.overlap,
                               n_dominv=args.n_dominv, storage=W.F16 if args.storage == "f16" else W.F32)
        us, fl = time_domain_sweep(torch, W, lat, dims, ras, eta, kappa, csw)
        ras.n_ras = 1
        print(json.dumps({"mode": "sweep", "us": us, "flops": fl, "ras": ras_desc(W.SolverParams.make(ras=ras))}))
        lat.close()
        ctx.close()
        return
    if args.mode == "solve":
        lat = W.Lattice(ctx, dims)
        lat.upload_gauge(I.random_gauge(dims, 0.5, 1))
        nrhs = 12 if args.point_sources else 1
        src = I.point_sources(dims, 3)[1] if args.point_sources else I.gaussian_source(dims, 2)
        e = lat.pack(src, W.F64, nrhs)
        phi = lat.zeros(W.F64, nrhs)
        p = W.SolverParams.make(tol_outer=tol, tol_inner=args.tol_inner, max_outer=200, max_inner=100,
                                ras=W.RasParams.make(block=tuple(int(v) for v in args.block.split("x")),
                                                     s=args.overlap, n_ras=args.n_ras, n_dominv=args.n_dominv,
                                                     storage=W.F16 if args.storage == "f16" else W.F32))
        ms, sts = timed_solves(torch, lat, p, kappa, csw, e, phi, args.steps, args.warmup, nrhs)
        print(json.dumps({"mode": "solve", "ms": ms, "nrhs": nrhs, "ras": ras_desc(p), "stats": stats_desc(sts[-1])}))
        lat.close()
        ctx.close()
        return
    lat = W.Lattice(ctx, dims)
    U = I.random_gauge(dims, 0.5, 1)
    lat.upload_gauge(U)
    eta = I.gaussian_source(dims, 2)
    e = lat.pack(eta, W.F64)
    phi = lat.zeros(W.F64)
    log("16^3x32 fields resident")

    # ---- autotuner (not timed): domain shape, overlap, storage, sweeps, N_dominv, inner tolerance
    base = W.SolverParams.make(tol_outer=tol, tol_inner=1e-4, max_outer=200, max_inner=100)
    t0 = time.perf_counter()
    tuned, tuned_ms = W.autotune(lat, base, kappa, csw, e, 1)
    tune_s = time.perf_counter() - t0
    log(f"autotuned in {tune_s:.1f} s: {ras_desc(tuned)}")

    # ---- the timed steps: K complete solves with the tuned parameters
    ms_per_step, stats = timed_solves(torch, lat, tuned, kappa, csw, e, phi, args.steps, args.warmup)
    true_res = max(st["true_resid"] for st in stats)
    sol = lat.unpack(phi, W.F64)
    log(f"headline solve {ms_per_step:.3f} ms")

    # ---- the dominant kernel of the step: the on-chip domain solver, one
    # sweep (NRAS = 1) of the tuned domains, timed with HIP events
    roof_dom = None
    nb, ev = lat.block_info(tuned.ras)
    if ev <= 256:   # the fused (on-chip) domain solver
        us_dom, fl = time_domain_sweep(torch, W, lat, dims, tuned.ras, eta, kappa, csw)
        tf = fl / us_dom / 1e6
        key = "fused_" + "x".join(map(str, tuned.ras.block)) + f"_s{tuned.ras.s}_nd{tuned.ras.n_dominv}_" + \
              {1: "f32", 2: "f16"}[tuned.ras.storage]
        roof_dom = {"bound": "alu", "achieved": round(tf, 2), "peak": round(VALU_F32_PEAK_TFLOPS, 1),
                    "unit": "TFLOP/s", "frac": round(tf / VALU_F32_PEAK_TFLOPS, 4),
                    "traffic": measured_traffic("domain_counters.json", DOMAIN_SOURCES, key, lat.V),
                    "kernel": f"k_blk_fused (one RAS sweep: {nb} domains x {ev} sites x {tuned.ras.n_dominv} MR steps "
                              f"on chip, {fl / 1e9:.3f} GFLOP per launch)", "us_per_launch": round(us_dom, 2)}
        log(f"domain sweep {us_dom:.1f} us, {tf:.1f} TFLOP/s")

    # ---- the literal 8^4-domain configurations, s = 0 and s = 1
    literal = {}
    for s in (0, 1):
        p = W.SolverParams.make(tol_outer=tol, tol_inner=1e-4, max_outer=200, max_inner=100,
                                ras=W.RasParams.make(block=(8, 8, 8, 8), s=s, n_ras=3, n_dominv=4, storage=W.F32))
        ms, sts = timed_solves(torch, lat, p, kappa, csw, e, phi, max(2, args.steps // 2), 1)
        literal[f"8x8x8x8_s{s}"] = {"ms": round(ms, 3), "stats": stats_desc(sts[-1])}
        log(f"8^4 s={s}: {ms:.3f} ms")

    # ---- plain FP64 BiCGStab on the same GPU and input
    for _ in range(args.warmup):
        lat.solve_bicgstab_f64(tol, 100000, kappa, csw, e, phi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, pst = lat.solve_bicgstab_f64(tol, 100000, kappa, csw, e, phi)
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t0) / args.steps * 1e3
    log(f"plain FP64 {plain_ms:.3f} ms")

    # ---- the 4^4 plain-method anchor (eps 0.5, kappa 0.12): launch-bound FP64 BiCGStab
    small = None
    if not args.no_extra:
        d4 = (4, 4, 4, 4)
        l4 = W.Lattice(ctx, d4)
        U4 = I.random_gauge(d4, 0.5, 1)
        l4.upload_gauge(U4)
        eta4 = I.gaussian_source(d4, 2)
        e4, p4 = l4.pack(eta4, W.F64), l4.zeros(W.F64)
        l4.solve_bicgstab_f64(1e-10, 1000, 0.12, 1.0, e4, p4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            _, st4 = l4.solve_bicgstab_f64(1e-10, 1000, 0.12, 1.0, e4, p4)
        torch.cuda.synchronize()
        ms4 = (time.perf_counter() - t0) / 20 * 1e3
        small = {"lattice": list(d4), "kappa": 0.12, "ms": round(ms4, 3), "iters": st4["outer_iters"],
                 "true_resid": st4["true_resid"], "us_per_iter": round(ms4 * 1e3 / st4["outer_iters"], 1)}
        l4.close()
        log(f"4^4 plain FP64: {small}")

    # ---- 12 spin-colour point sources batched in one solve (same lattice)
    multi = None
    if not args.no_extra:
        x0, eta12 = I.point_sources(dims, 3)
        e12 = lat.pack(eta12, W.F64, 12)
        phi12 = lat.zeros(W.F64, 12)
        # the batch and the single point source are each autotuned for themselves (not timed)
        tuned12, _ = W.autotune(lat, base, kappa, csw, e12, 12)
        ms12, st12 = timed_solves(torch, lat, tuned12, kappa, csw, e12, phi12, max(2, args.steps // 2), 1, nrhs=12)
        p1 = lat.pack(eta12[0], W.F64)
        f1 = lat.zeros(W.F64)
        tuned1, _ = W.autotune(lat, base, kappa, csw, p1, 1)
        ms1, _ = timed_solves(torch, lat, tuned1, kappa, csw, p1, f1, max(2, args.steps // 2), 1)
        multi = {"rhs": 12, "source_site": x0, "ms_per_batch": round(ms12, 3),
                 "solves_per_s": round(12e3 / ms12, 2), "ms_single_point_source": round(ms1, 3),
                 "per_rhs_cost_vs_single": round(ms12 / 12 / ms1, 3),
                 "max_true_resid": st12[-1]["true_resid"], "ras_batch": ras_desc(tuned12),
                 "ras_single": ras_desc(tuned1), "stats": stats_desc(st12[-1])}
        del e12, phi12, p1, f1
        log(f"12 rhs: {ms12:.3f} ms per batch")
    lat.close()

    # ---- D-apply against the HBM roofline at 32^4 (1.4 GB FP64 / 705 MB FP32,
    # larger than the 256 MB Infinity Cache)
    roof, dapply, big32 = None, {}, None
    big = (32, 32, 32, 32)
    if not args.no_dapply or not args.no_extra:
        big32 = {1.0: I.random_gauge(big, 1.0, 1)}
    if not args.no_dapply:
        lb = W.Lattice(ctx, big)
        lb.upload_gauge(big32[1.0])
        for prec in (1, 2, 0):
            us = time_dapply(torch, I, lb, prec)
            gbs = DAPPLY_BYTES[prec] * lb.V / us / 1e3
            dapply[{0: "f64", 1: "f32", 2: "f16"}[prec]] = {
                "us": round(us, 2), "GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                "gflops": round(DAPPLY_FLOPS * lb.V / us / 1e3, 1), "bytes_per_site": DAPPLY_BYTES[prec]}
        us12 = time_dapply(torch, I, lb, 1, nrhs=12, n_warm=3, n_timed=20)
        gbs12 = DAPPLY_12RHS_BYTES_F32 * lb.V / us12 / 1e3
        dapply["f32_12rhs"] = {"us": round(us12, 2), "GBps": round(gbs12, 1), "frac": round(gbs12 / HBM_PEAK_GBS, 4),
                               "gflops": round(12 * DAPPLY_FLOPS * lb.V / us12 / 1e3, 1),
                               "bytes_per_site": DAPPLY_12RHS_BYTES_F32}
        V = lb.V
        f32 = dapply["f32"]
        tb = measured_traffic("dapply_counters.json", DAPPLY_SOURCES, "1", V)
        roof = {"bound": "hbm", "achieved": f32["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": f32["frac"], "traffic": tb,
                "kernel": "k_dslash_xy<F32> full-lattice D-apply, 32^4, 672 algorithmic B/site x 1048576 sites "
                          "per launch", "us_per_launch": f32["us"]}
        lb.close()
        log(f"D-apply 32^4: {dapply}")

    # ---- 32^4, eps in {0.3, 1.0}: FP16-storage RAS, autotuned domain shape
    c3 = None
    if not args.no_extra:
        c3 = {}
        big32[0.3] = I.random_gauge(big, 0.3, 1)
        eta32 = I.gaussian_source(big, 2)
        for eps in (0.3, 1.0):
            lb = W.Lattice(ctx, big)
            lb.upload_gauge(big32[eps])
            e32 = lb.pack(eta32, W.F64)
            f32v = lb.zeros(W.F64)
            b16 = W.SolverParams.make(tol_outer=tol, tol_inner=1e-4, max_outer=200, max_inner=100,
                                      ras=W.RasParams.make(block=(4, 4, 4, 4), storage=W.F16))
            t16, _ = W.autotune(lb, b16, kappa, csw, e32, 1)
            t16.ras.storage = W.F16
            ms32, st32 = timed_solves(torch, lb, t16, kappa, csw, e32, f32v, 2, 1)
            lb.solve_bicgstab_f64(tol, 100000, kappa, csw, e32, f32v)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, pst32 = lb.solve_bicgstab_f64(tol, 100000, kappa, csw, e32, f32v)
            torch.cuda.synchronize()
            pl32 = (time.perf_counter() - t0) * 1e3
            c3[f"eps{eps}"] = {"ms": round(ms32, 3), "ras": ras_desc(t16), "stats": stats_desc(st32[-1]),
                               "plain_f64_ms": round(pl32, 3), "plain_f64_iters": pst32["outer_iters"],
                               "speedup_vs_plain_f64": round(pl32 / ms32, 3)}
            lb.close()
            log(f"32^4 eps={eps}: {ms32:.3f} ms (plain {pl32:.3f} ms)")

    paper = None
    if not args.no_extra and not args.no_paper:
        paper = paper_table(torch, W, ctx, big, big32[0.3], eta32)
        paper["eps"] = 0.3
        log(f"paper table: {paper}")
    del big32

    serving = None
    if not args.no_extra and not args.no_serve:
        serving = serve_bench(W, I, np, ctx, args.requests, args.slots)

    # ---- CPU baseline: the FP64 oracle's nested RAS solve on the same input and parameters
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import Oracle
        o = Oracle(dims, U)
        r = tuned.ras
        t0 = time.perf_counter()
        osol, info = o.nested(eta, kappa, csw, tol=tol, tol_inner=tuned.tol_inner, max_inner=100, ras=True,
                              block=tuple(r.block), s=r.s, n_ras=r.n_ras, n_dominv=r.n_dominv)
        tc = time.perf_counter() - t0
        # the GPU solution, checked by the oracle's own operator
        gres = float(np.linalg.norm(eta - o.apply_D(sol, kappa, csw)) / np.linalg.norm(eta))
        cpu = {"value": round(1.0 / tc, 5), "unit": "solves/s", "cores": Oracle.num_threads(), "kind": "oracle",
               "sample": f"one complete FP64 nested RAS-BiCGStab solve of the same 16^3x32 system with the same "
                         f"RAS parameters ({info['outer_iters']} outer / {info['inner_iters']} inner iterations, "
                         f"{tc:.1f} s)",
               "gpu_solution_true_resid_by_oracle": gres}
        log(f"oracle solve {tc:.1f} s")
        # the 4^4 plain-method anchor on the host, beside the GPU's plain_4x4_f64
        d4 = (4, 4, 4, 4)
        o4 = Oracle(d4, I.random_gauge(d4, 0.5, 1))
        t0 = time.perf_counter()
        _, inf4 = o4.bicgstab(I.gaussian_source(d4, 2), 0.12, 1.0, tol=1e-10)
        cpu["plain_4x4_f64"] = {"ms": round((time.perf_counter() - t0) * 1e3, 3), "iters": inf4["iters"]}

    st0 = stats[-1]
    out = {
        "metric": METRIC,
        "value": round(1e3 / ms_per_step, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64/f32 (outer FP64; inner BiCGStab and RAS arithmetic FP32)",
        "data": "synthetic (seeded random SU(3) gauge field eps=0.5 and Gaussian source)",
        "config": {"workload": "16^3x32 nested RAS-BiCGStab solve to 1e-10 (kappa 0.125, c_sw 1.0)",
                   "lattice": list(dims), "eps": 0.5, "kappa": kappa, "csw": csw, "rhs": 1,
                   "ras": ras_desc(tuned), "parallelism": "single GPU"},
        "time_to_solution_ms": round(ms_per_step, 3),
        "true_residual": true_res,
        "solve_stats": stats_desc(st0),
        "autotune_s": round(tune_s, 2),
        "plain_f64_bicgstab_ms": round(plain_ms, 3),
        "plain_f64_iters": pst["outer_iters"],
        "speedup_vs_plain_f64": round(plain_ms / ms_per_step, 3),
        "literal_8x8x8x8": literal,
        "plain_4x4_f64": small,
        "multi_rhs_12": multi,
        "solve_32x4_f16": c3,
        "paper_table1_32x4": paper,
        "dapply_32x4": dapply,
        "serving": serving,
        "roofline": roof_dom,
        "roofline_dapply": roof,
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
