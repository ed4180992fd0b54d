"""Benchmark: time-to-solution of the mixed-precision nested RAS-BiCGStab
solver on one MI355X, beside the plain FP64 BiCGStab on the same GPU, plus
the Wilson-clover D-apply against the HBM roofline, the 16^3x32 solves, the
12-source batched solve, the paper's 32^4 experiment and the serving loop.

One step = one complete solve of D phi = eta to |eta - D phi|/|eta| <= 1e-10 on
  32^4 (1 048 576 sites), random SU(3) links exp(i eps H), eps = 0.3 (seed 1),
  kappa = 0.125, c_sw = 1.0, Gaussian source (seed 2);
  FP64 outer / FP32 inner BiCGStab right-preconditioned by RAS with FP16
  storage.  The domain shape ({4^4, 4^3x8, 8^4}), overlap, sweeps, N_dominv
  inner tolerance and the MR steps' arithmetic are picked by the library's
  autotuner before the timed region, timing solves of two other sources
  (seeds 7 and 8).
Inputs are resident in HBM before every timed region.

Prints one JSON line; --mode selects a single section.
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
                         "serving run; solve: K timed solves on --lattice with the RAS parameters given below "
                         "(no autotuning), for kernel traces; sweep: 55 launches of one RAS sweep (NRAS = 1) of the "
                         "on-chip domain solver with those parameters (NRAS = 2 with --n-ras 2), for counters; "
                         "paper: the paper's 32^4 x-split table with the NRAS x N_dominv scan")
    ap.add_argument("--lattice", default="32x32x32x32", help="solve/sweep modes: lattice extents")
    ap.add_argument("--eps", type=float, default=0.3, help="solve/sweep modes: gauge-field eps")
    ap.add_argument("--block", default="4x4x4x4", help="solve mode: domain shape")
    ap.add_argument("--overlap", type=int, default=0, help="solve mode: overlap s")
    ap.add_argument("--storage", default="f16", choices=["f32", "f16"], help="solve mode: RAS storage")
    ap.add_argument("--arith", default="fp32", choices=["fp32", "dot2"],
                    help="solve/sweep modes: arithmetic of the on-chip MR steps (dot2: binary16 operands, FP16 "
                         "storage)")
    ap.add_argument("--dapply-prec", default="f32", choices=["f64", "f32", "f16"], help="dapply mode: precision")
    ap.add_argument("--n-ras", type=int, default=3)
    ap.add_argument("--n-dominv", type=int, default=5)
    ap.add_argument("--tol-inner", type=float, default=1e-5)
    ap.add_argument("--timers", action="store_true", help="solve mode: per-category HIP-event timers")
    ap.add_argument("--point-sources", action="store_true", help="solve mode: the 12 point sources in one batch")
    ap.add_argument("--even-odd", action="store_true",
                    help="solve mode: the even-odd reduced system without the Schwarz preconditioner")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dapply", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the 12-source, 32^4 and serving sections")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper's 32^4 x-split table")
    ap.add_argument("--no-small", action="store_true", help="skip the 16^3x32 and 4^4 sections")
    ap.add_argument("--paper-eps", type=float, default=0.3, help="paper mode: gauge-field eps")
    ap.add_argument("--paper-scan", action="store_true",
                    help="paper mode: the full NRAS 1-10 x N_dominv 1-20 scan instead of the default 4 x 4 grid")
    ap.add_argument("--requests", type=int, default=512, help="serving: number of requests")
    ap.add_argument("--slots", type=int, default=4, help="serving: concurrent solve slots")
    return ap.parse_args()


DAPPLY_SOURCES = ("wcl_dslash.hip", "wcl_device.h", "wcl_internal.h")
DOMAIN_SOURCES = ("wcl_block.hip", "wcl_device.h", "wcl_internal.h")
# FP32 VALU peak without packed-FP32 instructions (the library is built
# without them): 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz
VALU_F32_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# MI355X's published FP32 vector peak (it counts packed-FP32 instructions)
FP32_PEAK_PUBLISHED_TFLOPS = 157.3
# flops of the Wilson-clover operator per site: site term (two 6x6 Hermitian
# mat-vecs + the combination) and one hop (projection, two SU(3) mat-vecs,
# accumulation); 552 + 8 x 165 = 1872
SITE_TERM_FLOPS, HOP_FLOPS = 552, 165
# one minimal-residual step besides q = D rho: <q, rho>, <q, q>, x += a rho, rho -= a q
MR_FLOPS = 96 + 48 + 96 + 96


def source_hash(files) -> str:
    """Hash of the kernel sources with comments and blank lines removed (so
    that a comment edit does not invalidate the stored counter runs) and of
    the device compiler flags (include paths aside)."""
    from paper_1011_3318_amd import build
    h = hashlib.sha256()
    h.update(" ".join(f for f in build.HIPCC_FLAGS if not f.startswith("-I")).encode() + b"\n")
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


def time_dapply(torch, I, lat, prec, nrhs=1, n_warm=10, n_timed=300):
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


PAPER_SCAN_FULL = (tuple(range(1, 11)), (1, 2, 3, 4, 5, 6, 8, 10, 12, 15, 20))
PAPER_SCAN_DEFAULT = ((1, 2, 3, 5), (2, 3, 5, 8))


def paper_table(torch, W, ctx, dims, U, eta, kappa=0.126, csw=1.0, tol=1e-14, n_ras=3, n_dominv=5,
                scan=PAPER_SCAN_DEFAULT):
    """The paper's benchmark (Sec. 5, Table 1) on one GPU: 32^4 lattice,
    kappa 0.126, c_SW 1.0, |eta - D phi|/|eta| < 1e-14, the nested solver
    without preconditioner and with RAS on the x-only split into 8 domains
    (L_x/8 x L_y x L_z x L_t) with overlap depth d = 2s = 0, 2, 4, NRAS = 3,
    N_dominv = 5.  Reports time, the full-lattice D count and the domain work;
    scan = (NRAS values, N_dominv values) of the d = 0 scan (the paper scanned
    NRAS 1-10 x N_dominv 1-20), or None."""
    lat = W.Lattice(ctx, dims)
    lat.upload_gauge(U)
    e = lat.pack(eta, W.F64)
    phi = lat.zeros(W.F64)
    xb = (dims[0] // 8, dims[1], dims[2], dims[3])
    out = {"lattice": list(dims), "kappa": kappa, "csw": csw, "tol": tol, "domains": list(xb),
           "n_ras": n_ras, "n_dominv": n_dominv}

    def run(p, timers=False):
        lat.solve_nested(p, kappa, csw, e, phi, raise_on_notconv=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = lat.solve_nested(p, kappa, csw, e, phi, raise_on_notconv=False)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        if timers:
            # the timing chart of Sec. 4 from HIP events in a separate solve
            p.timers = 1
            _, stt = lat.solve_nested(p, kappa, csw, e, phi, raise_on_notconv=False)
            p.timers = 0
            st = dict(st)
            st["chart"] = {"T_Dv_calc_ms": round(stt["ms_dslash"], 3), "T_dominv_calc_ms": round(stt["ms_dominv"], 3),
                           "blas_ms": round(stt["ms_blas"], 3), "host_wait_ms": round(stt["ms_host"], 3),
                           "total_ms": round(stt["ms_total"], 3)}
        return ms, st

    base = dict(tol_outer=tol, tol_inner=1e-4, max_outer=200, max_inner=1000)
    ms, st = run(W.SolverParams.make(precond=W.PRECOND_NONE, **base), timers=True)
    out["no_prec"] = {"ms": round(ms, 3), "dv_count": st["dslash_full"], "outer_iters": st["outer_iters"],
                      "inner_iters": st["inner_iters"], "true_resid": st["true_resid"],
                      "converged": bool(st["converged"]), "chart": st["chart"]}
    for s in (0, 1, 2):
        ras = W.RasParams.make(block=xb, s=s, n_ras=n_ras, n_dominv=n_dominv, storage=W.F32)
        ms, st = run(W.SolverParams.make(ras=ras, **base), timers=True)
        out[f"ras_d{2 * s}"] = {"ms": round(ms, 3), "dv_count": st["dslash_full"], "outer_iters": st["outer_iters"],
                                "inner_iters": st["inner_iters"], "ras_sweeps": st["ras_sweeps"],
                                "domain_mr_steps": st["dslash_block"], "true_resid": st["true_resid"],
                                "converged": bool(st["converged"]), "chart": st["chart"]}
    out["paper_table1_context"] = {
        "hardware": "8 x GTX 285 over Gigabit Ethernet (Sec. 4); kappa 0.126, c_SW 1.0, 32^4, x-only split, 1e-14",
        "no_prec": {"total_s": 53.305, "dv_count": 1328, "T_Dv_calc_s": 3.900},
        "ras_d0": {"total_s": 27.977, "dv_count": 484, "T_Dv_calc_s": 1.424, "T_dominv_calc_s": 5.954},
        "ras_d2": {"total_s": 35.234, "dv_count": 496, "T_Dv_calc_s": 1.436, "T_dominv_calc_s": 6.245},
        "ras_d4": {"total_s": 37.195, "dv_count": 416, "T_Dv_calc_s": 1.205, "T_dominv_calc_s": 6.993}}
    if scan:
        grid = {}
        for nr in scan[0]:
            for nd in scan[1]:
                ras = W.RasParams.make(block=xb, s=0, n_ras=nr, n_dominv=nd, storage=W.F32)
                ms, st = run(W.SolverParams.make(ras=ras, **base))
                grid[f"{nr}x{nd}"] = {"ms": round(ms, 3), "dv_count": st["dslash_full"],
                                      "converged": bool(st["converged"])}
            log(f"scan NRAS={nr}: " + ", ".join(f"{k}: {v['ms']:.0f} ms" for k, v in grid.items()
                                                 if k.startswith(f"{nr}x")))
        best = min((k for k in grid if grid[k]["converged"]), key=lambda k: grid[k]["ms"])
        out["scan_d0"] = {"nras_values": list(scan[0]), "ndominv_values": list(scan[1]), "best": best, "grid": grid}
    lat.close()
    return out


def ras_desc(p):
    r = p.ras
    return {"block": list(r.block), "s": r.s, "n_ras": r.n_ras, "n_dominv": r.n_dominv,
            "storage": {0: "f64", 1: "f32", 2: "f16"}[r.storage], "arith": {0: "fp32", 1: "dot2"}[r.arith],
            "tol_inner": p.tol_inner}


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

    def run(budget, arrivals, nslots):
        srv = W.Server(ctx, max_slots=nslots, hbm_budget=budget)
        for k, d in enumerate(SERVE_SIZES):
            srv.register_gauge(k, d, gauges[k])
        free = {k: [] for k in range(len(SERVE_SIZES))}   # solution buffers returned by finished requests
        kept = {}   # one finished request per lattice size, kept for the oracle check
        inflight, done = {}, []
        nxt, late = 0, 0
        t0 = time.monotonic()
        window = 2 * nslots
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
                    k = int(kind[i])
                    if k not in kept:
                        kept[k] = (i, r[0].copy())
                    free[k].append(r[0])
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
                "failed": len(bad), "late_submits": late, "per_size": per_size}, kept

    # one slot: requests run one after another (no overlap on the device)
    single, _ = run(0, None, 1)
    log(f"serving: one slot {single['solves_per_s']} solves/s")
    closed, kept = run(0, None, slots)
    log(f"serving: closed loop {closed['solves_per_s']} solves/s")
    # one request of every lattice size checked by the oracle's own operator
    from oracle import Oracle
    check = {}
    for k, (i, sol) in sorted(kept.items()):
        o = Oracle(SERVE_SIZES[k], gauges[k], precompute_clover=False)
        res = float(np.linalg.norm(sources[i] - o.apply_D(sol, float(kappa[i]), float(csw[i])))
                    / np.linalg.norm(sources[i]))
        check["x".join(map(str, SERVE_SIZES[k]))] = {"request": int(i), "kappa": round(float(kappa[i]), 6),
                                                     "csw": float(csw[i]), "true_resid_by_oracle": res}
        del o
    log(f"serving: oracle check {check}")
    lam = 0.8 * closed["solves_per_s"]
    arrivals = np.cumsum(gaps) / lam
    opened, _ = run(24 << 30, arrivals, slots)
    opened["rate_per_s"] = round(lam, 3)
    opened["hbm_budget_bytes"] = 24 << 30
    log(f"serving: Poisson p50 {opened['p50_ms']} ms p99 {opened['p99_ms']} ms")
    shared = serve_shared_config(W, I, np, ctx)
    log(f"serving: shared configuration {shared['solves_per_s_batched']} solves/s batched, "
        f"{shared['solves_per_s_unbatched']} unbatched")
    return {"closed_loop": closed, "closed_loop_one_slot": single,
            "overlap_gain": round(closed["solves_per_s"] / single["solves_per_s"], 3), "poisson": opened,
            "slots": slots, "oracle_check": check,
            "mix": {"x".join(map(str, d)): wt for d, wt in zip(SERVE_SIZES, SERVE_WEIGHTS)},
            "shared_config": shared}


def serve_shared_config(W, I, np, ctx, n_req=48, max_batch=12):
    """Many sources on one configuration (the usual lattice workload): 48
    requests on 16^3x32 (eps 0.5, seed 1) with kappa 0.125, c_sw 1.0 and
    Gaussian sources (seed 4000 + request id), all submitted at once to one
    slot, without merging and with up to 12 requests per solve.  Results are
    compared bitwise between the two runs, one is checked by the oracle."""
    d = (16, 16, 16, 32)
    U = I.random_gauge(d, 0.5, 1)
    sources = [I.gaussian_source(d, 4000 + i) for i in range(n_req)]

    def run(mb):
        srv = W.Server(ctx, max_slots=1, max_batch=mb)
        srv.register_gauge(0, d, U)
        t = srv.submit(0, 0.125, 1.0, sources[0])   # warm the slot's workspace
        srv.wait(t)
        t0 = time.monotonic()
        tickets = [srv.submit(0, 0.125, 1.0, src) for src in sources]
        out = [srv.wait(t) for t in tickets]
        T = time.monotonic() - t0
        srv.close()
        return out, T

    alone, t1 = run(1)
    batched, tb = run(max_batch)
    same = all(np.array_equal(a[0], b[0]) for a, b in zip(alone, batched))
    ok = all(r["status"] == 0 and r["true_resid"] <= 1e-10 for _, r in batched)
    from oracle import Oracle
    o = Oracle(d, U, precompute_clover=False)
    res = float(np.linalg.norm(sources[5] - o.apply_D(batched[5][0], 0.125, 1.0)) / np.linalg.norm(sources[5]))
    sizes = [r["batch"] for _, r in batched]
    return {"lattice": list(d), "requests": n_req, "max_batch": max_batch,
            "solves_per_s_unbatched": round(n_req / t1, 3), "solves_per_s_batched": round(n_req / tb, 3),
            "batching_gain": round(t1 / tb, 3), "batch_sizes_seen": sorted(set(sizes)),
            "results_bitwise_equal": same, "all_converged": ok, "true_resid_by_oracle_request_5": res}


def roofline_alu(achieved_tflops, kernel, us, traffic, flops):
    """ALU-bound roofline entry: against the published FP32 vector peak and
    against the peak without packed-FP32 instructions (the library is built
    without them)."""
    return {"bound": "alu", "achieved": round(achieved_tflops, 2), "peak": FP32_PEAK_PUBLISHED_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved_tflops / FP32_PEAK_PUBLISHED_TFLOPS, 4), "traffic": traffic,
            "peak_without_packed_fp32": round(VALU_F32_PEAK_TFLOPS, 1),
            "frac_without_packed_fp32": round(achieved_tflops / VALU_F32_PEAK_TFLOPS, 4),
            "kernel": kernel, "us_per_launch": round(us, 2), "flops_per_launch": flops}


def residual_hop_flops(dims, ras, nblocks, ev):
    """Flops of the residual update a later sweep forms before its MR steps:
    without overlap only the hops that leave the domain (each 165 flops) plus
    the subtraction; with overlap the whole operator on every extended site."""
    no_overlap = ras.s == 0 or all(ras.block[m] == dims[m] for m in range(4))
    if no_overlap:
        cross = sum(2.0 / ras.block[m] for m in range(4) if ras.block[m] < dims[m])
        return (HOP_FLOPS * cross + 24) * nblocks * ev
    return (SITE_TERM_FLOPS + 8 * HOP_FLOPS + 24) * nblocks * ev


def domain_kernel_rooflines(torch, W, lat, dims, ras, eta, kappa, csw, stats, n=30):
    """The domain solver's two kernel instantiations in a solve: the first
    sweep (projection, N_dominv MR steps, restriction) and the later sweeps
    (the same plus the residual update of the previous sweep).  A RAS
    application with NRAS sweeps is timed alone with HIP events on the launch
    stream (ras_precondition, T(NRAS)).  A later sweep as it runs inside an
    application (writing the next sweep's residual and correction) takes
    (T(6) - T(2)) / 4: both applications end with the same last sweep.  The
    first sweep is timed alone, T(1) (as the only sweep it writes neither).
    Returns the entry of the instantiation that takes the larger share of the
    solve first."""
    nb, ev = lat.block_info(ras)
    if ev > 256:
        return None, None
    r32 = lat.pack(eta, W.F32)
    v32 = lat.empty(W.F32)
    T = {}
    for nr in (1, 2, 6):
        p = W.RasParams.make(block=tuple(ras.block), s=ras.s, n_ras=nr, n_dominv=ras.n_dominv, storage=ras.storage,
                             kernel=W.BLOCK_FUSED, arith=ras.arith)
        for _ in range(5):
            lat.ras_precondition(p, kappa, csw, r32, v32)
        torch.cuda.synchronize()
        T[nr] = event_time_us(torch, lambda k: lat.ras_precondition(p, kappa, csw, r32, v32), n)
    del r32, v32
    fl0 = domain_sweep_flops(dims, ras, nb, ev)
    fl1 = fl0 + residual_hop_flops(dims, ras, nb, ev)
    t1 = (T[6] - T[2]) / 4
    t0 = T[1]
    sweeps = stats["ras_sweeps"]
    first = sweeps / max(1, ras.n_ras)
    later = sweeps - first
    st = {1: "f32", 2: "f16"}[ras.storage] + ("_dot2" if ras.arith == W.ARITH_DOT2 else "")
    shape = "x".join(map(str, ras.block))
    key = f"fused_{shape}_s{ras.s}_nd{ras.n_dominv}_{st}"
    res = "res2" if ras.s == 0 else "res1"
    e_first = roofline_alu(fl0 / t0 / 1e6, f"k_blk_fused<{st},res0> (first sweep: {nb} domains x {ev} sites x "
                           f"{ras.n_dominv} MR steps on chip, {fl0 / 1e9:.3f} GFLOP per launch; {first:.0f} launches "
                           f"per solve; duration = T(NRAS 1), the sweep alone)", t0,
                           measured_traffic("domain_counters.json", DOMAIN_SOURCES, key, lat.V), fl0)
    e_later = roofline_alu(fl1 / t1 / 1e6, f"k_blk_fused<{st},{res}> (later sweeps: residual update of the previous "
                           f"sweep, then {ras.n_dominv} MR steps on {nb} domains x {ev} sites, {fl1 / 1e9:.3f} GFLOP "
                           f"per launch; {later:.0f} launches per solve; duration = (T(NRAS 6) - T(NRAS 2)) / 4)", t1,
                           measured_traffic("domain_counters.json", DOMAIN_SOURCES, key + "_" + res, lat.V), fl1)
    e_first["share_of_solve_ms"] = round(first * t0 / 1e3, 3)
    e_later["share_of_solve_ms"] = round(later * t1 / 1e3, 3)
    if later * t1 >= first * t0:
        return e_later, e_first
    return e_first, e_later


def plain_f64(torch, lat, kappa, csw, e, phi, tol, reps=1):
    lat.solve_bicgstab_f64(tol, 100000, kappa, csw, e, phi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, st = lat.solve_bicgstab_f64(tol, 100000, kappa, csw, e, phi)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps * 1e3, st


def timers_desc(st):
    return {k: round(st[k], 3) for k in ("ms_total", "ms_dslash", "ms_dominv", "ms_blas", "ms_host")}


def oracle_resid(Oracle, np, dims, U, eta, sol, kappa, csw):
    """|eta - D sol| / |eta| with the oracle's own operator (clover on the fly)."""
    o = Oracle(dims, U, precompute_clover=False)
    r = float(np.linalg.norm(eta - o.apply_D(sol, kappa, csw)) / np.linalg.norm(eta))
    del o
    return r


SCHUR_ENTRY_BYTES_F32 = 1152   # wcl_apply_schur, per full-lattice site, FP32 (see variant_bench)


def variant_bench(torch, W, np, Oracle, lat, dims, U, eta, e, phi, kappa, csw, tol, reps):
    """The other readings of the domain solver and the Schwarz iteration
    (Sec. 1-2) and the even-odd reduced solve, each as the preconditioner (or
    operator) of the same nested solve on this lattice: time to solution,
    iteration counts, the per-category timers, and the solution's true
    residual recomputed by the oracle."""
    cases = {
        "RAS_MR_onchip": W.RasParams.make(block=(4, 4, 4, 4), s=0, n_ras=3, n_dominv=4, storage=W.F16),
        "RAS_MR_split": W.RasParams.make(block=(4, 4, 4, 4), s=0, n_ras=3, n_dominv=4, storage=W.F16,
                                         kernel=W.BLOCK_SPLIT),
        "RAS_JACOBI": W.RasParams.make(block=(4, 4, 4, 4), s=0, n_ras=3, n_dominv=4, storage=W.F16,
                                       block_solver=W.DOMSOLVE_JACOBI),
        "RAS_BICGSTAB": W.RasParams.make(block=(4, 4, 4, 4), s=0, n_ras=2, n_dominv=2, storage=W.F16,
                                         block_solver=W.DOMSOLVE_BICGSTAB),
        "AS_MR_s1": W.RasParams.make(block=(4, 4, 4, 4), s=1, n_ras=1, n_dominv=4, storage=W.F16,
                                     schwarz=W.SCHWARZ_AS),
        "SAP_MR": W.RasParams.make(block=(4, 4, 4, 4), s=0, n_ras=2, n_dominv=4, storage=W.F16,
                                   schwarz=W.SCHWARZ_SAP),
        "even_odd_no_schwarz": None,
    }
    out = {}
    o = Oracle(dims, U, precompute_clover=False)
    for name, ras in cases.items():
        if ras is None:
            p = W.SolverParams.make(tol_outer=tol, tol_inner=1e-4, max_outer=200, max_inner=200,
                                    precond=W.PRECOND_NONE, even_odd=1)
        else:
            p = W.SolverParams.make(tol_outer=tol, tol_inner=1e-4, max_outer=200, max_inner=100, ras=ras)
        ms, sts = timed_solves(torch, lat, p, kappa, csw, e, phi, reps, 1)
        sol = lat.unpack(phi, W.F64)
        res = float(np.linalg.norm(eta - o.apply_D(sol, kappa, csw)) / np.linalg.norm(eta))
        p.timers = 1
        _, stt = lat.solve_nested(p, kappa, csw, e, phi)
        out[name] = {"ms": round(ms, 3), "stats": stats_desc(sts[-1]), "timers": timers_desc(stt),
                     "true_resid_by_oracle": res}
        if ras is not None:
            out[name]["ras"] = ras_desc(p)
        log(f"variant {name}: {ms:.3f} ms, oracle true residual {res:.2e}")
    del o
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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
    big = (32, 32, 32, 32)
    kappa, csw, tol = 0.125, 1.0, 1e-10
    if args.mode == "dapply":
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
        tab = paper_table(torch, W, ctx, big, I.random_gauge(big, args.paper_eps, 1), I.gaussian_source(big, 2),
                          scan=PAPER_SCAN_FULL if args.paper_scan else PAPER_SCAN_DEFAULT)
        tab["eps"] = args.paper_eps
        print(json.dumps({"mode": "paper", "paper_table1": tab}))
        ctx.close()
        return
    if args.mode == "serve":
        print(json.dumps({"mode": "serve", "serving": serve_bench(W, I, np, ctx, args.requests, args.slots)}))
        ctx.close()
        return
    if args.mode in ("sweep", "solve"):
        dims = tuple(int(v) for v in args.lattice.split("x"))
        lat = W.Lattice(ctx, dims)
        lat.upload_gauge(I.random_gauge(dims, args.eps, 1))
        storage = W.F16 if args.storage == "f16" else W.F32
        arith = W.ARITH_DOT2 if args.arith == "dot2" else W.ARITH_FP32
        block = tuple(int(v) for v in args.block.split("x"))
        if args.mode == "sweep":
            eta = I.gaussian_source(dims, 2)
            ras = W.RasParams.make(block=block, s=args.overlap, n_ras=args.n_ras, n_dominv=args.n_dominv,
                                   storage=storage, kernel=W.BLOCK_FUSED, arith=arith)
            r32 = lat.pack(eta, W.F32)
            v32 = lat.empty(W.F32)
            for _ in range(5):
                lat.ras_precondition(ras, kappa, csw, r32, v32)
            torch.cuda.synchronize()
            us = event_time_us(torch, lambda k: lat.ras_precondition(ras, kappa, csw, r32, v32), 50)
            print(json.dumps({"mode": "sweep", "lattice": list(dims), "us": us,
                              "ras": ras_desc(W.SolverParams.make(ras=ras))}))
        else:
            nrhs = 12 if args.point_sources else 1
            src = I.point_sources(dims, 3)[1] if args.point_sources else I.gaussian_source(dims, 2)
            e = lat.pack(src, W.F64, nrhs)
            phi = lat.zeros(W.F64, nrhs)
            p = W.SolverParams.make(tol_outer=tol, tol_inner=args.tol_inner, max_outer=200, max_inner=100,
                                    timers=int(args.timers),
                                    ras=W.RasParams.make(block=block, s=args.overlap, n_ras=args.n_ras,
                                                         n_dominv=args.n_dominv, storage=storage, arith=arith))
            if args.even_odd:
                p = W.SolverParams.make(tol_outer=tol, tol_inner=1e-4, max_outer=200, max_inner=200,
                                        timers=int(args.timers), precond=W.PRECOND_NONE, even_odd=1)
            ms, sts = timed_solves(torch, lat, p, kappa, csw, e, phi, args.steps, args.warmup, nrhs)
            print(json.dumps({"mode": "solve", "lattice": list(dims), "ms": ms, "nrhs": nrhs, "ras": ras_desc(p),
                              "stats": stats_desc(sts[-1]), "timers": timers_desc(sts[-1])}))
        lat.close()
        ctx.close()
        return

    # ================= the headline: 32^4, eps 0.3, FP16-storage RAS, autotuned
    U32 = {0.3: I.random_gauge(big, 0.3, 1)}
    eta32 = I.gaussian_source(big, 2)
    tune_src32 = np.stack([I.gaussian_source(big, 7), I.gaussian_source(big, 8)])
    lat = W.Lattice(ctx, big)
    lat.upload_gauge(U32[0.3])
    e = lat.pack(eta32, W.F64)
    et = lat.pack(tune_src32, W.F64, 2)
    phi = lat.zeros(W.F64)
    log("32^4 fields resident")
    base16 = W.SolverParams.make(tol_outer=tol, tol_inner=1e-4, max_outer=200, max_inner=100,
                                 ras=W.RasParams.make(block=(4, 4, 4, 4), storage=W.F16))
    t0 = time.perf_counter()
    tuned, _ = W.autotune(lat, base16, kappa, csw, et, 1, storage=W.F16, nsrc=2)
    tune_s = time.perf_counter() - t0
    del et
    log(f"autotuned in {tune_s:.1f} s on the seed-7 and seed-8 sources: {ras_desc(tuned)}")
    ms_per_step, stats = timed_solves(torch, lat, tuned, kappa, csw, e, phi, args.steps, args.warmup)
    true_res = max(st["true_resid"] for st in stats)
    sol32 = lat.unpack(phi, W.F64)
    log(f"headline solve {ms_per_step:.3f} ms")
    # the same solve once more with the per-category timers (not in the timed region)
    tt = W.SolverParams.make(tol_outer=tuned.tol_outer, tol_inner=tuned.tol_inner, max_outer=tuned.max_outer,
                             max_inner=tuned.max_inner, ras=tuned.ras, timers=1)
    _, st_t = lat.solve_nested(tt, kappa, csw, e, phi)
    roof_dom, roof_dom_other = domain_kernel_rooflines(torch, W, lat, big, tuned.ras, eta32, kappa, csw, stats[-1])
    if roof_dom:
        log(f"domain kernels: {roof_dom['kernel'][:40]} {roof_dom['us_per_launch']} us, "
            f"{roof_dom['achieved']} TFLOP/s")
    plain_ms, pst = plain_f64(torch, lat, kappa, csw, e, phi, tol, reps=2)
    log(f"32^4 plain FP64 {plain_ms:.3f} ms ({pst['outer_iters']} iterations)")
    headline = {"ms": round(ms_per_step, 3), "ras": ras_desc(tuned), "stats": stats_desc(stats[-1]),
                "true_resid": true_res, "timers": timers_desc(st_t), "plain_f64_ms": round(plain_ms, 3),
                "plain_f64_iters": pst["outer_iters"], "speedup_vs_plain_f64": round(plain_ms / ms_per_step, 3)}
    # ---- the even-odd reduced system at 32^4 (no Schwarz preconditioner), and its operator
    eo32 = None
    if not args.no_extra:
        peo = W.SolverParams.make(tol_outer=tol, tol_inner=1e-4, max_outer=200, max_inner=200,
                                  precond=W.PRECOND_NONE, even_odd=1)
        ms_eo, st_eo = timed_solves(torch, lat, peo, kappa, csw, e, phi, 2, 1)
        sol_eo = lat.unpack(phi, W.F64)
        x32, y32 = lat.pack(eta32, W.F32), lat.empty(W.F32)
        for _ in range(3):
            lat.apply_schur(W.F32, kappa, csw, x32, y32)
        torch.cuda.synchronize()
        us_schur = event_time_us(torch, lambda k: lat.apply_schur(W.F32, kappa, csw, x32, y32), 20)
        del x32, y32
        gbs = SCHUR_ENTRY_BYTES_F32 * lat.V / us_schur / 1e3
        eo32 = {"ms": round(ms_eo, 3), "stats": stats_desc(st_eo[-1]),
                "speedup_vs_plain_f64": round(plain_ms / ms_eo, 3),
                "schur_apply_f32": {"us": round(us_schur, 2), "bytes_per_site": SCHUR_ENTRY_BYTES_F32,
                                    "GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                                    "note": "whole wcl_apply_schur entry point: even-site extract, A_oo^-1 H_oe, "
                                            "Schur complement, odd-site zero fill, insert"}}
        log(f"32^4 even-odd: {ms_eo:.3f} ms; Schur entry point {us_schur:.1f} us")
    del e, phi
    lat.close()

    # ---- 32^4, eps 1.0 (same protocol)
    c3_eps1 = None
    if not args.no_extra:
        U32[1.0] = I.random_gauge(big, 1.0, 1)
        lb = W.Lattice(ctx, big)
        lb.upload_gauge(U32[1.0])
        e1 = lb.pack(eta32, W.F64)
        et1 = lb.pack(tune_src32, W.F64, 2)
        f1 = lb.zeros(W.F64)
        t1, _ = W.autotune(lb, base16, kappa, csw, et1, 1, storage=W.F16, nsrc=2)
        ms1, st1 = timed_solves(torch, lb, t1, kappa, csw, e1, f1, max(2, args.steps // 2), 1)
        pl1, pst1 = plain_f64(torch, lb, kappa, csw, e1, f1, tol)
        c3_eps1 = {"ms": round(ms1, 3), "ras": ras_desc(t1), "stats": stats_desc(st1[-1]),
                   "plain_f64_ms": round(pl1, 3), "plain_f64_iters": pst1["outer_iters"],
                   "speedup_vs_plain_f64": round(pl1 / ms1, 3)}
        del e1, et1, f1
        lb.close()
        log(f"32^4 eps=1.0: {ms1:.3f} ms (plain {pl1:.3f} ms)")

    # ================= 16^3 x 32 (eps 0.5): tuned, the literal 8^4 domains, plain FP64, 12 point sources
    small_dims = (16, 16, 16, 32)
    c2 = None
    multi = None
    anchor4 = None
    U16 = None
    if not args.no_small:
        U16 = I.random_gauge(small_dims, 0.5, 1)
        l16 = W.Lattice(ctx, small_dims)
        l16.upload_gauge(U16)
        eta16 = I.gaussian_source(small_dims, 2)
        e16 = l16.pack(eta16, W.F64)
        et16 = l16.pack(np.stack([I.gaussian_source(small_dims, 7), I.gaussian_source(small_dims, 8)]), W.F64, 2)
        p16 = l16.zeros(W.F64)
        base = W.SolverParams.make(tol_outer=tol, tol_inner=1e-4, max_outer=200, max_inner=100)
        tuned16, _ = W.autotune(l16, base, kappa, csw, et16, 1, nsrc=2)
        ms16, st16 = timed_solves(torch, l16, tuned16, kappa, csw, e16, p16, args.steps, args.warmup)
        literal = {}
        for s in (0, 1):
            p = W.SolverParams.make(tol_outer=tol, tol_inner=1e-4, max_outer=200, max_inner=100,
                                    ras=W.RasParams.make(block=(8, 8, 8, 8), s=s, n_ras=3, n_dominv=4, storage=W.F32))
            ms, sts = timed_solves(torch, l16, p, kappa, csw, e16, p16, max(2, args.steps // 2), 1)
            literal[f"8x8x8x8_s{s}"] = {"ms": round(ms, 3), "stats": stats_desc(sts[-1])}
            log(f"16^3x32 8^4 s={s}: {ms:.3f} ms")
        pl16, pst16 = plain_f64(torch, l16, kappa, csw, e16, p16, tol, reps=max(2, args.steps // 2))
        c2 = {"lattice": list(small_dims), "eps": 0.5, "tuned": {"ms": round(ms16, 3), "ras": ras_desc(tuned16),
                                                                 "stats": stats_desc(st16[-1])},
              "literal_8x8x8x8": literal, "plain_f64_ms": round(pl16, 3), "plain_f64_iters": pst16["outer_iters"],
              "speedup_tuned_vs_plain_f64": round(pl16 / ms16, 3)}
        log(f"16^3x32 tuned {ms16:.3f} ms, plain FP64 {pl16:.3f} ms")
        if not args.no_extra:
            x0, eta12 = I.point_sources(small_dims, 3)
            e12 = l16.pack(eta12, W.F64, 12)
            phi12 = l16.zeros(W.F64, 12)
            # tuned on the 12 point sources at another site (seed 4), timed on those at seed 3
            et12 = l16.pack(I.point_sources(small_dims, 4)[1], W.F64, 12)
            tuned12, _ = W.autotune(l16, base, kappa, csw, et12, 12)
            del et12
            ms12, st12 = timed_solves(torch, l16, tuned12, kappa, csw, e12, phi12, max(2, args.steps // 2), 1, nrhs=12)
            p1 = l16.pack(eta12[0], W.F64)
            f1 = l16.zeros(W.F64)
            ms1, _ = timed_solves(torch, l16, tuned12, kappa, csw, p1, f1, max(2, args.steps // 2), 1)
            sol12 = l16.unpack(phi12, W.F64, 12)
            multi = {"rhs": 12, "source_site": x0, "ms_per_batch": round(ms12, 3),
                     "solves_per_s": round(12e3 / ms12, 2), "ms_single_point_source_same_params": round(ms1, 3),
                     "per_rhs_cost_vs_single": round(ms12 / 12 / ms1, 3),
                     "max_true_resid": st12[-1]["true_resid"], "ras": ras_desc(tuned12),
                     "stats": stats_desc(st12[-1])}
            del e12, phi12, p1, f1
            log(f"12 rhs: {ms12:.3f} ms per batch")
        variants = None
        if not args.no_extra:
            from oracle import Oracle
            variants = variant_bench(torch, W, np, Oracle, l16, small_dims, U16, eta16, e16, p16, kappa, csw, tol,
                                     max(2, args.steps // 2))
            c2["variants"] = variants
        del e16, et16, p16
        l16.close()
        # the 4^4 plain-method anchor (eps 0.5, kappa 0.12): launch-bound FP64 BiCGStab
        d4 = (4, 4, 4, 4)
        l4 = W.Lattice(ctx, d4)
        l4.upload_gauge(I.random_gauge(d4, 0.5, 1))
        e4, p4 = l4.pack(I.gaussian_source(d4, 2), W.F64), l4.zeros(W.F64)
        ms4, st4 = plain_f64(torch, l4, 0.12, 1.0, e4, p4, 1e-10, reps=20)
        anchor4 = {"lattice": list(d4), "kappa": 0.12, "ms": round(ms4, 3), "iters": st4["outer_iters"],
                   "true_resid": st4["true_resid"], "us_per_iter": round(ms4 * 1e3 / st4["outer_iters"], 1)}
        l4.close()

    # ================= D-apply against the HBM roofline at 32^4
    roof, dapply = None, {}
    if not args.no_dapply:
        Ud = U32.get(1.0)
        if Ud is None:
            Ud = I.random_gauge(big, 1.0, 1)
        lb = W.Lattice(ctx, big)
        lb.upload_gauge(Ud)
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
        f32 = dapply["f32"]
        roof = {"bound": "hbm", "achieved": f32["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": f32["frac"], "traffic": measured_traffic("dapply_counters.json", DAPPLY_SOURCES, "1", lb.V),
                "kernel": "k_dslash_xy<F32> full-lattice D-apply, 32^4, 672 algorithmic B/site x 1048576 sites "
                          "per launch", "us_per_launch": f32["us"]}
        lb.close()
        log(f"D-apply 32^4: {dapply}")

    paper = None
    if not args.no_extra and not args.no_paper:
        paper = paper_table(torch, W, ctx, big, U32[0.3], eta32)
        paper["eps"] = 0.3
        log(f"paper table: {paper}")

    serving = None
    if not args.no_extra and not args.no_serve:
        serving = serve_bench(W, I, np, ctx, args.requests, args.slots)

    # ================= CPU baseline: the FP64 oracle on the host cores
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import Oracle
        cores = Oracle.num_threads()
        # the GPU solutions checked by the oracle's own operator
        gres32 = oracle_resid(Oracle, np, big, U32[0.3], eta32, sol32, kappa, csw)
        log(f"oracle: 32^4 GPU solution true residual {gres32:.3e}")
        o = Oracle(big, U32[0.3])
        r = tuned.ras
        n_inner = 3
        t0 = time.perf_counter()
        _, info = o.nested(eta32, kappa, csw, tol=tol, max_outer=1, tol_inner=tuned.tol_inner, max_inner=n_inner,
                           ras=True, block=tuple(r.block), s=r.s, n_ras=r.n_ras, n_dominv=r.n_dominv)
        tc = time.perf_counter() - t0
        per_inner = tc / max(1, info["inner_iters"])
        gpu_inner = stats[-1]["inner_iters"]
        est = per_inner * gpu_inner
        # the oracle D-apply at all cores (32^4) and at one thread (16^3x32)
        t0 = time.perf_counter()
        o.apply_D(eta32, kappa, csw)
        td_all = time.perf_counter() - t0
        del o
        Oracle.set_threads(1)
        o1 = Oracle(small_dims, U16 if U16 is not None else I.random_gauge(small_dims, 0.5, 1))
        eta16h = I.gaussian_source(small_dims, 2)
        t0 = time.perf_counter()
        o1.apply_D(eta16h, kappa, csw)
        td_one = time.perf_counter() - t0
        del o1
        Oracle.set_threads(cores)
        V32, V16 = I.volume(big), I.volume(small_dims)
        cpu = {"value": round(1.0 / est, 5), "unit": "solves/s", "cores": cores, "kind": "oracle",
               "sample": f"{info['inner_iters']} inner iterations (1 outer) of the FP64 oracle's nested RAS-BiCGStab "
                         f"solve of the same 32^4 system with the tuned RAS parameters ({tc:.1f} s on {cores} "
                         f"threads), scaled to the {gpu_inner} inner iterations of the GPU solve",
               "cpu_model": cpu_model(), "nproc": os.cpu_count(),
               "gpu_solution_true_resid_by_oracle": gres32,
               "dapply_f64_32x4_all_cores": {"s": round(td_all, 3), "threads": cores,
                                             "GBps": round(DAPPLY_BYTES[0] * V32 / td_all / 1e9, 2),
                                             "gflops": round(DAPPLY_FLOPS * V32 / td_all / 1e9, 2)},
               "dapply_f64_16x16x16x32_one_thread": {"s": round(td_one, 3), "threads": 1,
                                                     "GBps": round(DAPPLY_BYTES[0] * V16 / td_one / 1e9, 2),
                                                     "gflops": round(DAPPLY_FLOPS * V16 / td_one / 1e9, 2)}}
        if multi is not None:
            resid = [oracle_resid(Oracle, np, small_dims, U16, eta12[k], sol12[k], kappa, csw) for k in (0, 5, 11)]
            multi["true_resid_by_oracle_rhs_0_5_11"] = resid
        if U16 is not None:
            o16 = Oracle(small_dims, U16)
            t0 = time.perf_counter()
            _, inf16 = o16.bicgstab(I.gaussian_source(small_dims, 2), kappa, csw, tol=tol)
            cpu["plain_16x16x16x32_f64"] = {"s": round(time.perf_counter() - t0, 3), "iters": inf16["iters"],
                                            "threads": cores}
            del o16
        if anchor4 is not None:
            d4 = (4, 4, 4, 4)
            o4 = Oracle(d4, I.random_gauge(d4, 0.5, 1))
            t0 = time.perf_counter()
            _, inf4 = o4.bicgstab(I.gaussian_source(d4, 2), 0.12, 1.0, tol=1e-10)
            cpu["plain_4x4_f64"] = {"ms": round((time.perf_counter() - t0) * 1e3, 3), "iters": inf4["iters"]}
        log(f"oracle baseline {cpu['value']} solves/s (sample {tc:.1f} s)")

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
        "dtype": "f64/f32/f16 (outer BiCGStab FP64; inner BiCGStab FP32; RAS domain solves on FP16 storage of "
                 "links, clover and sweep fields, " +
                 ("MR steps with binary16 operands and FP32 sums (v_dot2_f32_f16), FP32 vector work"
                  if tuned.ras.arith == W.ARITH_DOT2 else "FP32 arithmetic") + ")",
        "data": "synthetic (seeded random SU(3) gauge field eps=0.3 and Gaussian source)",
        "config": {"workload": "32^4 nested RAS-BiCGStab solve to 1e-10 (eps 0.3, kappa 0.125, c_sw 1.0; "
                               "FP16-storage domain solves, domain shape autotuned over 4^4, 4^3x8, 8^4)",
                   "lattice": list(big), "eps": 0.3, "kappa": kappa, "csw": csw, "rhs": 1, "ras": ras_desc(tuned),
                   "source_seed": 2, "tuning_source_seeds": [7, 8], "parallelism": "single GPU"},
        "time_to_solution_ms": round(ms_per_step, 3),
        "true_residual": true_res,
        "solve_stats": stats_desc(stats[-1]),
        "timers": timers_desc(st_t),
        "autotune_s": round(tune_s, 2),
        "plain_f64_bicgstab_ms": headline["plain_f64_ms"],
        "plain_f64_iters": headline["plain_f64_iters"],
        "speedup_vs_plain_f64": headline["speedup_vs_plain_f64"],
        "solve_32x4_eps1.0_f16": c3_eps1,
        "even_odd_32x4": eo32,
        "solve_16x16x16x32": c2,
        "multi_rhs_12": multi,
        "plain_4x4_f64": anchor4,
        "paper_table1_32x4": paper,
        "dapply_32x4": dapply,
        "serving": serving,
        "roofline": roof_dom,
        "roofline_other_domain_kernel": roof_dom_other,
        "roofline_dapply": roof,
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
