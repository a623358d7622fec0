"""Benchmark: FP32-accurate GEMM at one TPU core's block shape on one MI355X.

Workload (one "step"): C = A B with A 16384 x 32768 and B 32768 x 16384, FP32
entries i.i.d. N(0, 1) (seeds 201, 202), through la_gemm with the 3xBF16 split
(the paper's local block GEMM, eq. Matmul of section III.A, at the
(16384, 32768) per-core block of section I).  The same inputs are also run with
the plain FP32-MFMA and the 6xBF16 paths and reported beside the headline.

Prints ONE JSON line.  `value` is TFLOP/s = 2 M N K / (time per step), with
inputs resident in HBM and the time from HIP events on the launch stream.
`roofline` compares the GEMM kernel's rate with the BF16 MFMA peak divided by
the three products one FP32-accurate multiply-add costs.  `cpu_baseline` times
the FP64 CPU oracle on sampled 64 x 64 output tiles (full K) and checks those
tiles against the GPU result.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

M, N, K = 16384, 16384, 32768
PEAK_BF16 = 2516.6      # TFLOP/s, dense BF16 MFMA, MI355X
PEAK_FP32 = 157.3       # TFLOP/s, FP32 MFMA, MI355X
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_packed_bf16x3_16384x16384x32768_traffic.json")
MFMA_FILE = os.path.join(ROOT, "profiles", "gemm_packed_bf16x3_16384x16384x32768_mfma.json")
KERNEL_SOURCES = ["paper_2112_09017_amd/csrc/gemm_tile.h", "paper_2112_09017_amd/csrc/gemm_x3.hip"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if the kernel source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def load_mfma():
    """Matrix-core busy fraction and clock of the packed kernel from the
    committed rocprofv3 counter summary, or None if the kernel source changed
    since the counters were taken."""
    try:
        with open(MFMA_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return {k: t[k] for k in ("mfma_busy", "clock_ghz", "bf16_mfma_tflops", "source") if k in t}


def time_launches(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def cpu_baseline(A, B, C_gpu, budget_s: float, seed: int = 203):
    """FP64 oracle on sampled 64 x 64 output tiles (full K): its rate, and the
    normwise error of the GPU result estimated from those tiles."""
    import oracle

    g = np.random.default_rng(seed)
    T = 64
    corners = [(0, 0), (0, N - T), (M - T, 0), (M - T, N - T)]
    flops = 0.0
    err2 = 0.0
    tiles = 0
    t0 = time.perf_counter()
    while True:
        if tiles < len(corners):
            r, c = corners[tiles]
        else:
            r = int(g.integers(0, M // T)) * T
            c = int(g.integers(0, N // T)) * T
        ref = oracle.gemm(A[r:r + T], np.ascontiguousarray(B[:, c:c + T].T), trans_b=True)
        err2 += float(np.sum((C_gpu[r:r + T, c:c + T].astype(np.float64) - ref) ** 2))
        flops += 2.0 * T * T * K
        tiles += 1
        if time.perf_counter() - t0 >= budget_s and tiles >= len(corners):
            break
    dt = time.perf_counter() - t0
    nA = float(np.linalg.norm(A.astype(np.float64)))
    nB = float(np.linalg.norm(B.astype(np.float64)))
    est = np.sqrt(err2 * (M * N) / (tiles * T * T)) / (nA * nB)
    return {
        "value": flops / dt / 1e12,
        "unit": "TFLOP/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{tiles} output tiles of 64x64 (4 corners + random, seed {seed}), full K={K}, "
                  f"FP64, {flops:.3g} flop in {dt:.1f} s",
    }, float(est), tiles


def polar_errors(torch, Ad, U, H, V, sd):
    """Exact FP64 ||U^T U - I||_F / sqrt(n), ||A - U H||_F / ||A||_F and
    ||H - V diag(s) V^T||_F / ||A||_F, by torch products on the GPU (checks
    only, outside the timed region)."""
    n = U.shape[1]
    U64 = U.double()
    G = U64.t().contiguous() @ U64
    G.diagonal().sub_(1.0)
    orth = torch.linalg.norm(G).item() / n ** 0.5
    del G
    A64 = Ad.double()
    nA = torch.linalg.norm(A64).item()
    resid = torch.linalg.norm(A64 - U64 @ H.double()).item() / nA
    del A64, U64
    dh = torch.linalg.norm(H.double() - (V * sd[None, :]) @ V.t().contiguous()).item() / nA
    torch.cuda.empty_cache()
    return {"orth": float(f"{orth:.3g}"), "resid": float(f"{resid:.3g}"),
            "h_err": float(f"{dh:.3g}")}


def polar_section(la, torch, m=16384, n=16384, lo=1e-6, seeds=(301, 302, 303),
                  counter_run=False):
    """Polar factorisation of an m x n A = Q diag(s) V^T (cond 1/lo), AUTO policy
    (6xBF16 preconditioning and H, 3xBF16 Newton-Schulz) and all-FP32-MFMA.
    counter_run: build the inputs on the host and skip the FP64 error checks,
    so that only this library's kernels run on the GPU (counter collection)."""
    import la_inputs

    t0 = time.perf_counter()
    A, Q, s, V = la_inputs.polar_case_torch(
        m, n, lo, seeds, device="cpu" if counter_run else "cuda",
        progress=lambda w: print(f"[bench] polar input {w} ready after "
                                 f"{time.perf_counter() - t0:.1f} s", file=sys.stderr,
                                 flush=True))
    del Q
    V = V.to("cuda:0")
    torch.cuda.empty_cache()
    sd = torch.from_numpy(s).to("cuda:0")
    Ad = torch.from_numpy(A).to("cuda:0")
    U = torch.empty_like(Ad)
    H = torch.empty((n, n), dtype=torch.float32, device="cuda:0")
    print(f"[bench] polar inputs {m}x{n} in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)
    out = {"workload": f"polar {m}x{n} FP32, A = Q diag(s) V^T, Haar Q, V, s log-uniform "
                       f"in [{lo:g}, 1], seeds {seeds[0]}/{seeds[1]}/{seeds[2]}"}
    mn2 = float(m) * float(n) * float(n)
    policies = {"auto": {}, "fp32": dict(prec_precond=1, prec_ns=1, prec_h=1)}
    for name, opts in policies.items():
        la.polar(Ad, U=U, H=H, **opts)          # warm-up (same work)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, _, info = la.polar(Ad, U=U, H=H, **opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        k = info["iters_precond"] + info["iters_ns"]
        alg = (3.0 * k + 2.0) * mn2          # Gram mn^2 + update 2mn^2 per step, H 2mn^2
        paper_eq = 2.0 * (2 * k + 1) * mn2   # "about 50 matmuls" convention
        out[name] = {"seconds": round(dt, 3), "iters_precond": info["iters_precond"],
                     "iters_ns": info["iters_ns"], "tflops_algorithmic": round(alg / dt / 1e12, 1),
                     "tflops_paper_equivalent": round(paper_eq / dt / 1e12, 1)}
        if not counter_run:
            out[name].update(polar_errors(torch, Ad, U, H, V, sd))
        print(f"[bench] polar {m}x{n} {name}: {dt:.2f} s, {out[name]}", file=sys.stderr,
              flush=True)
    out["speedup_auto_vs_fp32"] = round(out["fp32"]["seconds"] / out["auto"]["seconds"], 2)
    return out


def oracle_polar_timing(sizes=(256, 512, 1024), lo=1e-6, seeds=(103, 104, 105)):
    """The FP64 oracle polar (same s0 and eps as the FP32 paths, so the same
    iteration counts) timed on the host at small n; its per-step rate
    extrapolated by n^3 to the large workloads (labelled extrapolated)."""
    import la_inputs
    import oracle

    eps = 2.0 ** -23
    res = {}
    for n in sizes:
        A = la_inputs.polar_case(n, n, lo, seeds).A32.astype(np.float64)
        t0 = time.perf_counter()
        _, _, info = oracle.polar(A, s_minus=0.1, s0=eps, eps=eps, max_iter=100)
        dt = time.perf_counter() - t0
        k = info.iters_precond + info.iters_ns
        res[n] = {"seconds": round(dt, 3), "iters": k,
                  "gflops": round((3.0 * k + 2.0) * n ** 3 / dt / 1e9, 2)}
        print(f"[bench] oracle polar {n}: {dt:.2f} s, {res[n]}", file=sys.stderr, flush=True)
    big = max(sizes)
    rate = res[big]["gflops"] * 1e9
    return {"kind": "oracle", "cores": oracle.num_threads(), "measured": res,
            "extrapolated_seconds": {
                "16384x16384 (28 steps)": round((3.0 * 28 + 2.0) * 16384.0 ** 3 / rate, 0),
                "131072x4096 (24 steps)": round((3.0 * 24 + 2.0) * 131072.0 * 4096.0 ** 2 / rate, 0)},
            "note": f"rate of the FP64 oracle at n={big}, scaled by flops; extrapolated, not run"}


def inverse_section(la, torch, n=16384, lo=1e-2, seeds=(601, 602, 603)):
    """Newton-Schulz inversion of an n x n A = Q diag(s) V^T (cond 1/lo), AUTO
    (3xBF16 steps + one 6xBF16 step) and all-FP32-MFMA."""
    import la_inputs

    t0 = time.perf_counter()
    A, Q, s, V = la_inputs.polar_case_torch(n, n, lo, seeds)
    del Q, V
    torch.cuda.empty_cache()
    Ad = torch.from_numpy(A).to("cuda:0")
    X = torch.empty_like(Ad)
    print(f"[bench] inverse inputs {n}x{n} in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)
    out = {"workload": f"Newton-Schulz inverse {n}x{n} FP32, A = Q diag(s) V^T, Haar Q, V, "
                       f"s log-uniform in [{lo:g}, 1], seeds {seeds[0]}/{seeds[1]}/{seeds[2]}"}
    for name, opts in (("auto", {}), ("fp32", dict(prec=1))):
        la.inverse(Ad, X=X, **opts)          # warm-up (same work)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, info = la.inverse(Ad, X=X, **opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        k = info["iters"]
        alg = (4.0 * k + 1.0) * float(n) ** 3     # two 2n^3 products per step, Gram n^3
        g = torch.randn((n, 16), dtype=torch.float64, device="cuda:0",
                        generator=torch.Generator(device="cuda:0").manual_seed(604))
        y = Ad.double() @ (X.double() @ g) - g          # residual probes (check only)
        res = float(torch.sqrt((y * y).sum() / 16)) / n ** 0.5
        out[name] = {"seconds": round(dt, 3), "iters": k,
                     "tflops_algorithmic": round(alg / dt / 1e12, 1),
                     "residual_probe": float(f"{res:.3g}")}
        print(f"[bench] inverse {name}: {dt:.2f} s, {out[name]}", file=sys.stderr, flush=True)
        del y, g
    out["speedup_auto_vs_fp32"] = round(out["fp32"]["seconds"] / out["auto"]["seconds"], 2)
    return out


def matfunc_section(la, torch, n=8192, degree=16, seed=701):
    """Chebyshev series of degree 16 (Clenshaw, 15 products) and a 5-term odd
    singular-value series (Gram + 3 Horner products + final product) of an
    n x n A, AUTO (6xBF16) and all-FP32-MFMA."""
    import la_inputs

    g = torch.Generator(device="cuda:0").manual_seed(seed)
    A = torch.randn((n, n), device="cuda:0", generator=g) / (2.0 * n ** 0.5)
    A = 0.5 * (A + A.T)                                   # symmetric, spectrum in ~[-1, 1]
    F = torch.empty_like(A)
    c = la_inputs.rng(seed).standard_normal(degree + 1)
    c5 = [0.9, -0.6, 0.35, -0.2, 0.05]
    ws = torch.empty(la.lib().la_matfunc_workspace_size(n, n) + 256, dtype=torch.uint8,
                     device="cuda:0")
    out = {"workload": f"Chebyshev series degree {degree} on [-1, 1] and 5-term odd series of a "
                       f"{n}x{n} symmetric Gaussian A (seed {seed})"}
    for name, prec in (("auto", la.Precision.AUTO), ("fp32", la.Precision.FP32)):
        res = {}
        for kind, fn, flops in (
                ("cheb", lambda: la.matfunc_cheb(A, -1.0, 1.0, c, F=F, prec=prec, workspace=ws),
                 2.0 * (degree - 1) * float(n) ** 3),
                ("odd", lambda: la.matfunc_odd(A, c5, F=F, prec=prec, workspace=ws),
                 (1.0 + 2.0 * (len(c5) - 2) + 2.0) * float(n) ** 3)):
            fn()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            res[kind] = {"seconds": round(dt, 4), "tflops_algorithmic": round(flops / dt / 1e12, 1)}
        out[name] = res
        print(f"[bench] matfunc {name}: {res}", file=sys.stderr, flush=True)
    return out


def qr_section(la, torch, n=16384, panel=64, tall=(131072, 64), seed=801):
    """Algorithm caqr on an n x n Gaussian A (R alone, then R and Q) at AUTO
    (6xBF16 updates) and all-FP32 MFMA, and Algorithm tsqr of a tall panel.
    Rates use the Householder operation counts: 4/3 n^3 for R, as much again
    for Q; 2 m k^2 - 2/3 k^3 for R and as much for Q of an m x k panel."""
    g = torch.Generator(device="cuda:0").manual_seed(seed)
    A = torch.randn((n, n), device="cuda:0", generator=g)
    X = torch.empty_like(A)
    out = {"workload": f"CAQR of a {n}x{n} Gaussian A (seed {seed}), panel {panel}; TSQR of a "
                       f"{tall[0]}x{tall[1]} Gaussian panel"}
    for name, prec in (("auto", la.Precision.AUTO), ("fp32", la.Precision.FP32)):
        res = {}
        for want_q in (False, True):
            ws = torch.empty(la.caqr_workspace_size(n, n, panel, want_q) + 256,
                             dtype=torch.uint8, device="cuda:0")
            got = {}

            def run():
                X.copy_(A)
                got["Q"], _ = la.caqr(X, panel=panel, want_q=want_q, inplace=True, prec=prec,
                                      workspace=ws)
            run()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            run()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            flops = 4.0 / 3.0 * float(n) ** 3 * (2.0 if want_q else 1.0)
            entry = {"seconds": round(dt, 4), "tflops_algorithmic": round(flops / dt / 1e12, 2)}
            if want_q:
                # FP64 probes (check only): ||A - QR||_F / ||A||_F and
                # ||Q^T Q - I||_F / sqrt(n), from E||M g||^2 = ||M||_F^2, g ~ N(0, I)
                pg = torch.randn((n, 16), dtype=torch.float64, device="cuda:0",
                                 generator=torch.Generator(device="cuda:0").manual_seed(802))
                Qd = got["Q"].double()
                r1 = A.double() @ pg - Qd @ (torch.triu(X[:n]).double() @ pg)
                entry["backward_probe"] = float(f"{float(torch.sqrt((r1 * r1).sum() / 16)) / float(torch.linalg.norm(A.double())):.3g}")
                r2 = Qd.T @ (Qd @ pg) - pg
                entry["orthogonality_probe"] = float(f"{float(torch.sqrt((r2 * r2).sum() / 16)) / n ** 0.5:.3g}")
                del Qd, r1, r2, pg
            res["r_and_q" if want_q else "r_only"] = entry
            del ws, got
            torch.cuda.empty_cache()
        out[name] = res
        print(f"[bench] caqr {name}: {res}", file=sys.stderr, flush=True)
    m, k = tall
    T = torch.randn((m, k), device="cuda:0", generator=g)
    la.tsqr(T)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    la.tsqr(T)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    flops = 2.0 * (2.0 * m * k * k - 2.0 / 3.0 * k ** 3)
    out["tsqr"] = {"seconds": round(dt, 5), "tflops_algorithmic": round(flops / dt / 1e12, 2)}
    print(f"[bench] tsqr {m}x{k}: {out['tsqr']}", file=sys.stderr, flush=True)
    return out


def serving_pool(torch, pool_size=48, seed=401):
    """Pool of square polar inputs (n log-uniform in [128, 4096], cond 10^U(1,6))."""
    import la_inputs

    t0 = time.perf_counter()
    g = la_inputs.rng(seed + 1)
    sizes = la_inputs.serve_sizes(pool_size, seed + 2)
    conds = 10.0 ** g.uniform(1.0, 6.0, size=pool_size)
    pool = [la_inputs.polar_case_torch(int(n), int(n), 1.0 / c,
                                       (seed * 1000 + 3 * i, seed * 1000 + 3 * i + 1,
                                        seed * 1000 + 3 * i + 2))[0]
            for i, (n, c) in enumerate(zip(sizes, conds))]
    torch.cuda.empty_cache()
    print(f"[bench] serving pool of {pool_size} in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    return pool


def served_errors(torch, A, U, H):
    """FP64 orthogonality and residual of one served result (check only)."""
    n = U.shape[1]
    Ad = torch.from_numpy(A).to("cuda:0").double()
    Ud = torch.from_numpy(U).to("cuda:0").double()
    G = Ud.t().contiguous() @ Ud
    G.diagonal().sub_(1.0)
    orth = torch.linalg.norm(G).item() / n ** 0.5
    resid = (torch.linalg.norm(Ad - Ud @ torch.from_numpy(H).to("cuda:0").double()).item() /
             torch.linalg.norm(Ad).item())
    return orth, resid


def serving_section(la, pool, rate=100.0, duration=30.0, seed=401, exclude_s=1.0,
                    check_every=25):
    """Poisson stream of requests from the pool against the continuous-batching
    server; p50/p99 latency from submit to completed poll, over the requests
    submitted after the first exclude_s seconds (warm-up of the queue).  Only
    requests that end with status OK count; every check_every-th result is
    checked afterwards (FP64 orthogonality and residual <= 1e-5)."""
    import torch

    import la_inputs

    stream = la_inputs.serve_stream(rate, duration, seed, len(pool))
    lat = []
    flops = 0.0
    bad = 0
    done = 0
    samples = []
    with la.Server(16 << 30, max_slots=64) as srv:
        w = srv.submit(pool[0])            # touch the code paths once
        while srv.poll(w) is None:
            time.sleep(0.001)
        pending = {}
        start = time.perf_counter()
        i = 0
        while i < len(stream) or pending:
            now = time.perf_counter() - start
            while i < len(stream) and stream[i][0] <= now:
                A = pool[stream[i][1]]
                t_sub = time.perf_counter()
                rid = srv.submit(A)
                pending[rid] = (t_sub, stream[i][1], stream[i][0] >= exclude_s)
                i += 1
            for rid in list(pending):
                sample = (done + 1) % check_every == 0
                r = srv.poll(rid, want_h=sample)
                if r is not None:
                    t_sub, pi, counted = pending.pop(rid)
                    done += 1
                    if r[0] != la.Status.OK:
                        bad += 1
                        continue
                    if counted:
                        lat.append(time.perf_counter() - t_sub)
                    k = r[3]["iters_precond"] + r[3]["iters_ns"]
                    flops += (3.0 * k + 2.0) * float(pool[pi].shape[0]) ** 3
                    if sample:
                        samples.append((pi, r[1], r[2]))
            time.sleep(0.0002)
        wall = time.perf_counter() - start
        st = srv.stats()
    checks = [served_errors(torch, pool[pi], U, H) for pi, U, H in samples]
    worst = max((max(o, r) for o, r in checks), default=float("nan"))
    lat_ms = np.array(lat) * 1e3
    out = {"workload": f"Poisson arrivals at {rate:g} req/s for {duration:g} s, square n "
                       f"log-uniform in [128, 4096] (x64), cond 10^U(1,6), pool of {len(pool)} "
                       f"(seed {seed}), AUTO policy; latency over arrivals after {exclude_s:g} s",
           "requests": int(len(stream)), "latency_samples": int(len(lat)),
           "failed_requests": int(bad),
           "p50_ms": round(float(np.percentile(lat_ms, 50)), 2),
           "p99_ms": round(float(np.percentile(lat_ms, 99)), 2),
           "mean_ms": round(float(lat_ms.mean()), 2),
           "throughput_req_s": round(len(stream) / wall, 1),
           "tflops_algorithmic": round(flops / wall / 1e12, 2),
           "ticks": int(st["ticks"]), "gpu_busy_frac": round(st["busy_seconds"] / wall, 3),
           "arena_high_water_gib": round(st["arena_high_water"] / 2 ** 30, 2),
           "checked_results": len(checks), "checked_worst_orth_or_resid": float(f"{worst:.3g}"),
           "checked_all_within_1e-5": bool(checks) and worst <= 1e-5}
    print(f"[bench] serving {rate:g} req/s: {out}", file=sys.stderr, flush=True)
    return out


def serving_saturation(la, pool, depth=96, seconds=8.0, warm_s=1.0, seed=402):
    """Sustained capacity: `depth` requests kept outstanding (a new one is
    submitted as each completes, drawn from the pool), completions counted
    over `seconds` after `warm_s`.  The pinned staging of every pool size is
    warmed first, so the figure is the server's and not the first submits'
    allocations."""
    g = np.random.default_rng(seed)
    with la.Server(16 << 30, max_slots=64) as srv:
        for w in [srv.submit(p) for p in pool]:
            while srv.poll(w, want_h=False) is None:
                time.sleep(0.001)
        pending = {}

        def add():
            j = int(g.integers(0, len(pool)))
            pending[srv.submit(pool[j])] = (time.perf_counter(), pool[j].shape[0])

        for _ in range(depth):
            add()
        t0 = time.perf_counter()
        win = None
        done = bad = 0
        flops = 0.0
        lat = []
        while True:
            now = time.perf_counter()
            if win is None and now - t0 >= warm_s:
                win = now
            if win is not None and now - win >= seconds:
                break
            for rid in list(pending):
                r = srv.poll(rid, want_h=False)
                if r is None:
                    continue
                ts, n = pending.pop(rid)
                if win is not None:
                    if r[0] != la.Status.OK:
                        bad += 1
                    else:
                        done += 1
                        k = r[3]["iters_precond"] + r[3]["iters_ns"]
                        flops += (3.0 * k + 2.0) * float(n) ** 3
                        lat.append(time.perf_counter() - ts)
                add()
            time.sleep(0.0003)
        wall = time.perf_counter() - win
        st = srv.stats()
        while pending:
            for rid in list(pending):
                if srv.poll(rid, want_h=False) is not None:
                    pending.pop(rid)
            time.sleep(0.001)
    out = {"kind": f"closed loop: {depth} requests outstanding, 64 slots, {seconds:g} s after "
                   f"{warm_s:g} s", "completed": done, "failed_requests": bad,
           "throughput_req_s": round(done / wall, 1),
           "tflops_algorithmic": round(flops / wall / 1e12, 1),
           "p50_ms": round(float(np.median(lat)) * 1e3, 1) if lat else None,
           "ticks": int(st["ticks"])}
    print(f"[bench] serving saturation: {out}", file=sys.stderr, flush=True)
    return out


def serving_burst(la, pool, count=480, seed=402):
    """All `count` requests submitted at once: completion throughput, with
    the cost of the submits (each copies its input to pinned memory) and of
    the first pinned allocations inside it."""
    g = np.random.default_rng(seed)
    idx = g.integers(0, len(pool), size=count)
    flops = 0.0
    with la.Server(16 << 30, max_slots=64) as srv:
        start = time.perf_counter()
        pending = {srv.submit(pool[int(j)]): pool[int(j)].shape[0] for j in idx}
        bad = 0
        while pending:
            for rid in list(pending):
                r = srv.poll(rid, want_h=False)
                if r is not None:
                    n = pending.pop(rid)
                    if r[0] != la.Status.OK:
                        bad += 1
                        continue
                    k = r[3]["iters_precond"] + r[3]["iters_ns"]
                    flops += (3.0 * k + 2.0) * float(n) ** 3
            time.sleep(0.0005)
        wall = time.perf_counter() - start
    out = {"requests": count, "failed_requests": bad, "seconds": round(wall, 2),
           "throughput_req_s": round((count - bad) / wall, 1),
           "tflops_algorithmic": round(flops / wall / 1e12, 1)}
    print(f"[bench] serving burst: {out}", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-polar", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving stream (for profiling the grouped kernels)")
    ap.add_argument("--serving-sweep", action="store_true",
                    help="also run the serving stream at 25/50/150/200 req/s and a saturation "
                         "burst (about 1.5 minutes more)")
    ap.add_argument("--serving-seconds", type=float, default=30.0,
                    help="length of the Poisson stream")
    ap.add_argument("--no-tall", action="store_true", help="skip the 131072 x 4096 polar")
    ap.add_argument("--no-oracle-polar", action="store_true")
    ap.add_argument("--no-inverse", action="store_true")
    ap.add_argument("--no-matfunc", action="store_true")
    ap.add_argument("--no-qr", action="store_true")
    ap.add_argument("--qr-only", action="store_true",
                    help="run only the QR section (for profiling its kernels)")
    ap.add_argument("--polar-only", action="store_true",
                    help="run only the polar sections (16384^2 and, unless --no-tall, "
                         "131072 x 4096), for profiling their kernels")
    ap.add_argument("--counter-run", action="store_true",
                    help="with --polar-only: build the polar inputs on the host and skip "
                         "the FP64 error checks, so that only this library's kernels run "
                         "on the GPU (rocprofv3 --pmc runs)")
    ap.add_argument("--only", choices=["BF16X3", "FP32", "BF16X6"], default=None,
                    help="time one precision only (for profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (3 launches), to scale the "
                         "FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30,
                          "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU SUMMA path is not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    import la_inputs
    import paper_2112_09017_amd as la

    if args.qr_only:
        print(json.dumps({"qr": qr_section(la, torch)}), flush=True)
        return
    if args.polar_only:
        res = {"polar": polar_section(la, torch, counter_run=args.counter_run)}
        torch.cuda.empty_cache()
        if not args.no_tall:
            res["polar_tall"] = polar_section(la, torch, 131072, 4096, 1e-4, (501, 502, 503),
                                              counter_run=args.counter_run)
        print(json.dumps(res), flush=True)
        return
    if args.serving_only:
        pool = serving_pool(torch)
        res = serving_section(la, pool, duration=args.serving_seconds)
        res["saturation"] = serving_saturation(la, pool)
        res["burst"] = serving_burst(la, pool)
        print(json.dumps({"serving": res}), flush=True)
        return

    dev = torch.device("cuda:0")
    t_gen = time.perf_counter()
    A = la_inputs.gaussian((M, K), 201)
    B = la_inputs.gaussian((K, N), 202)
    Ad = torch.from_numpy(A).to(dev)
    Bd = torch.from_numpy(B).to(dev)
    Cd = torch.empty((M, N), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    print(f"[bench] inputs ready in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr,
          flush=True)
    flops = 2.0 * M * N * K

    rates = {}
    precs = [args.only] if args.only else ["BF16X3", "FP32", "BF16X6"]
    kernel_ms = None
    for p in precs:
        prec = getattr(la.Precision, p)
        steps = args.steps if p == precs[0] else max(2, args.steps // 3)
        warm = args.warmup if p == precs[0] else 1
        if p == "BF16X3":
            # the step: la_gemm_ws = pack op(A), pack op(B) (one HBM pass each) +
            # the packed-operand GEMM kernel
            ws = torch.empty(la.gemm_workspace_size(M, N, K) + 256, dtype=torch.uint8,
                             device=dev)
            ms = time_launches(lambda: la.gemm_ws(Ad, Bd, Cd, prec=prec, workspace=ws), steps,
                               warm, torch)
            # the GEMM kernel alone, on operands packed once
            Ap = la.pack_bf16x3(Ad)
            Bp = la.pack_bf16x3(Bd.T)
            kernel_ms = time_launches(lambda: la.gemm_packed(Ap, Bp, M, N, K, Cd), steps, 1,
                                      torch)
            del Ap, Bp, ws
            torch.cuda.empty_cache()
            # the unpacked kernel (la_gemm), for comparison
            ums = time_launches(lambda: la.gemm(Ad, Bd, Cd, prec=prec), max(2, steps // 3), 1,
                                torch)
            rates["BF16X3_unpacked"] = (ums, flops / ums / 1e9)
            print(f"[bench] BF16X3 la_gemm (unpacked): {ums:.2f} ms, {flops / ums / 1e9:.1f} "
                  f"TFLOP/s; packed kernel alone {kernel_ms:.2f} ms", file=sys.stderr, flush=True)
        else:
            ms = time_launches(lambda: la.gemm(Ad, Bd, Cd, prec=prec), steps, warm, torch)
        rates[p] = (ms, flops / ms / 1e9)
        print(f"[bench] {p}: {ms:.2f} ms/step, {rates[p][1]:.1f} TFLOP/s", file=sys.stderr,
              flush=True)
    head = precs[0]
    ms, tflops = rates[head]
    kernel_tflops = flops / kernel_ms / 1e9 if kernel_ms else tflops

    # the product once more, untimed, for the oracle's sampled-tile check
    if head == "BF16X3":
        la.gemm_ws(Ad, Bd, Cd, prec=la.Precision.BF16X3)
    else:
        la.gemm(Ad, Bd, Cd, prec=getattr(la.Precision, head))
    torch.cuda.synchronize()

    ceiling = PEAK_BF16 / 3.0 if head == "BF16X3" else (
        PEAK_BF16 / 6.0 if head == "BF16X6" else PEAK_FP32)
    traffic = load_traffic() if head == "BF16X3" else None
    out = {
        "metric": "FP32-accurate GEMM/polar TFLOP/s (3xBF16 vs fp32 MFMA); serve p50/p99 ms",
        "value": round(tflops, 2),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3" if head == "BF16X3" else head.lower(),
        "data": "synthetic",
        "config": {"workload": "block GEMM C=A*B, A 16384x32768, B 32768x16384, FP32 "
                               "entries N(0,1) seeds 201/202",
                   "m": M, "n": N, "k": K, "precision": head,
                   "step": ("la_gemm_ws: pack op(A) and op(B) into bf16 hi/lo tiles, then "
                            "the packed-operand GEMM") if head == "BF16X3" else "la_gemm"},
        "roofline": {
            "bound": "mfma",
            "kernel": ("la::dev::gemm_packed_kernel<34> (3xBF16 on packed operands, "
                       "256x256 tiles)") if head == "BF16X3" else f"la::dev::gemm_kernel ({head})",
            "achieved": round(kernel_tflops, 2),
            "peak": round(ceiling, 1),
            "unit": "TFLOP/s",
            "frac": round(kernel_tflops / ceiling, 4),
            "kernel_ms": round(kernel_ms, 3) if kernel_ms else round(ms, 3),
            "traffic": traffic,
            "mfma_util": load_mfma() if head == "BF16X3" else None,
            "peak_basis": ("BF16 dense MFMA 2516.6 TFLOP/s / 3 BF16 products per FP32-accurate "
                           "multiply-add" if head == "BF16X3" else
                           "BF16 dense MFMA / 6" if head == "BF16X6" else "FP32 MFMA 157.3"),
        },
        "other_precisions": {p: {"ms_per_step": round(v[0], 3), "tflops": round(v[1], 2)}
                             for p, v in rates.items() if p != head},
        "bf16_mfma_util": round(3 * tflops / PEAK_BF16, 4) if head == "BF16X3" else None,
        "paper_context": "TPU v3 pod: ~21 PFLOPS fp32 on 2048 cores (~10.3 TFLOPS/core); "
                         "N=2^20 product in ~2 min (context only, other hardware)",
    }
    if not args.no_cpu_baseline:
        C = Cd.cpu().numpy()
        cb, err, tiles = cpu_baseline(A, B, C, args.cpu_seconds)
        out["cpu_baseline"] = cb
        out["sampled_normwise_error"] = err
        out["sampled_tiles"] = tiles
    del Ad, Bd, Cd, A, B
    torch.cuda.empty_cache()
    if not args.no_polar and args.only is None:
        out["polar"] = polar_section(la, torch)
        torch.cuda.empty_cache()
        if not args.no_tall:
            out["polar_tall"] = polar_section(la, torch, 131072, 4096, 1e-4, (501, 502, 503))
            torch.cuda.empty_cache()
        if not args.no_oracle_polar:
            out["polar"]["cpu_oracle"] = oracle_polar_timing()
    if not args.no_inverse and args.only is None:
        out["inverse"] = inverse_section(la, torch)
        torch.cuda.empty_cache()
    if not args.no_matfunc and args.only is None:
        out["matfunc"] = matfunc_section(la, torch)
    if not args.no_qr and args.only is None:
        out["qr"] = qr_section(la, torch)
        torch.cuda.empty_cache()
    if not args.no_serving and args.only is None:
        pool = serving_pool(torch)
        out["serving"] = serving_section(la, pool, duration=args.serving_seconds)
        out["serving"]["saturation"] = serving_saturation(la, pool)
        out["serving"]["burst"] = serving_burst(la, pool)
        if args.serving_sweep:
            out["serving_sweep"] = {f"{r:g}": serving_section(la, pool, rate=r,
                                                              duration=args.serving_seconds)
                                    for r in (25.0, 50.0, 150.0, 200.0)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
