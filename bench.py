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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_bf16x3_16384x16384x32768_traffic.json")
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    for p in precs:
        prec = getattr(la.Precision, p)
        ms = time_launches(lambda: la.gemm(Ad, Bd, Cd, prec=prec),
                           args.steps if p == precs[0] else max(2, args.steps // 3),
                           args.warmup if p == precs[0] else 1, torch)
        rates[p] = (ms, flops / ms / 1e9)
        print(f"[bench] {p}: {ms:.2f} ms/step, {rates[p][1]:.1f} TFLOP/s", file=sys.stderr,
              flush=True)
    head = precs[0]
    ms, tflops = rates[head]

    # headline result for the baseline check (recompute, untimed)
    la.gemm(Ad, Bd, Cd, prec=getattr(la.Precision, head))
    torch.cuda.synchronize()

    ceiling = PEAK_BF16 / 3.0 if head == "BF16X3" else (
        PEAK_BF16 / 6.0 if head == "BF16X6" else PEAK_FP32)
    traffic = load_traffic() if head == "BF16X3" else None
    out = {
        "metric": "FP32-accurate GEMM TFLOP/s (3xBF16 split on BF16 MFMA, FP32 accumulate)",
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
                   "m": M, "n": N, "k": K, "precision": head},
        "roofline": {
            "bound": "mfma",
            "achieved": round(tflops, 2),
            "peak": round(ceiling, 1),
            "unit": "TFLOP/s",
            "frac": round(tflops / ceiling, 4),
            "traffic": traffic,
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
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
