#!/usr/bin/env python3
"""Throughput of the PSD-cone projection on one MI355X.

Default workload: the n = 625 (d = 5) warm-start sequence -- 50 SCS-like
iterates X_{k+1} = X_k + 1e-3 (H_k + H_k^H)/2 of a Hermitian (G + G^H)/2 --
each projected by the FP64 eigen path (unpack, blocked Householder
tridiagonalisation, divide and conquer, back-transform, fused clamp +
reconstruction + svec pack).  One step = the 50 projections.  Inputs are
resident in HBM before the timed region.

Prints one JSON line: projections/s, algorithmic TFLOP/s, the roofline of the
dominant kernel (per-column HEMV of the tridiagonalisation, timed live with
HIP events on its launch stream) and the CPU oracle timed on a bounded
sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload c2|c1|c5]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0        # MI355X HBM3E
PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 (vector = MFMA)

WORKLOADS = {
    # name: (n, iterates, seed, description)
    "c2": (625, 50, 1002, "d=5 warm-start sequence: 50 iterates of a 625x625 Hermitian block, FP64 eig path"),
    "c1": (16, 50, 1001, "d=2 process matrix 16x16, 50 seeded blocks, FP64 eig path"),
    "c5": (4096, 2, 1005, "d=8 process matrix 4096x4096, FP64 eig path"),
}


def flops_eig(n: int, k: int) -> float:
    """Algorithmic real flops of one FP64-path projection: tridiagonalisation
    16/3 n^3, back-transform 8 n^2 k and reconstruction 4 n^2 k (k columns of
    the smaller sign side; 8 flops per complex multiply-add)."""
    return 16.0 / 3.0 * n ** 3 + 8.0 * n * n * k + 4.0 * n * n * k


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2, help="iterates projected by the CPU oracle")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; --gpus must be 1 "
                                   "(the projection of one block does not shard across GPUs here)"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2606_20519_amd as P
    from paper_2606_20519_amd import _lib
    from paper_2606_20519_amd import workloads as W

    n, count, seed, desc = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    if args.workload == "c2":
        xs_np = W.warm_sequence(n, seed, count)
    else:
        xs_np = [W.gue(n, seed + i) for i in range(count)]
    X = torch.from_numpy(np.stack(xs_np)).to(dev)          # resident in HBM
    Y = torch.empty_like(X)
    stream = torch.cuda.current_stream(dev)

    def step():
        for i in range(count):
            P.project(X[i], n, out=Y[i])

    # side counts (k = min(k+, k-)) for the algorithmic flops, outside timing
    ks = []
    for i in range(count):
        _, inf = P.project(X[i], n, out=Y[i], info=True)
        ks.append(min(inf["n_pos"], inf["n_neg"]))
    flops_step = sum(flops_eig(n, k) for k in ks)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region; the dominant kernel is timed with HIP events on its own
    # launch stream: the library brackets the HEMV launches of the first
    # projection of the timed region (n-1 launches, one per column)
    hemv_sample = max(1, n - 1) if n > 64 else 0
    if hemv_sample:
        _lib.timing_start(_lib.KF_HEMV, hemv_sample)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hemv = _lib.timing_stop() if hemv_sample else (0.0, 0, 0.0)

    wall = t1 - t0
    ms_per_step = 1e3 * wall / args.steps
    proj_s = count * args.steps / wall
    tflops = flops_step * args.steps / wall / 1e12

    roofline = None
    if hemv[1] > 0:
        avg_ms = hemv[0] / hemv[1]
        bytes_per_launch = hemv[2] / hemv[1]
        achieved = hemv[2] / (hemv[0] * 1e-3) / 1e9
        roofline = {
            "kernel": "hemv_kernel (per-column Hermitian matrix-vector tiles, tridiagonalisation)",
            "bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
            "launches_timed": hemv[1], "avg_launch_us": round(1e3 * avg_ms, 3),
            "algorithmic_bytes_per_launch": round(bytes_per_launch, 1),
            "sample": "all HEMV launches of the first projection in the timed region",
            "share_of_projection": round(hemv[0] / (ms_per_step / count), 4),
        }

    # parity of the timed output on a sample, and the CPU oracle baseline
    cpu = None
    err = None
    if not args.no_cpu_baseline:
        import oracle
        m = max(1, min(args.cpu_sample, count))
        t = time.perf_counter()
        refs = [oracle.project(xs_np[i], n) for i in range(m)]
        dt = time.perf_counter() - t
        ycpu = Y[:m].cpu().numpy()
        err = max(float(np.linalg.norm(ycpu[i] - refs[i]) / np.linalg.norm(refs[i])) for i in range(m))
        cpu = {"value": round(m / dt, 5), "unit": "projections/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"first {m} of the {count} iterates (n={n}), cyclic Jacobi round-robin FP64, "
                         f"{dt:.1f} s"}

    out = {
        "metric": "PSD projections/sec (FP64 eig path)",
        "value": round(proj_s, 3),
        "unit": "projections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "blocks_per_step": count, "mode": "fp64",
                   "algorithmic_tflops": round(tflops, 3),
                   "fp64_peak_frac": round(tflops / PEAK_FP64_TFLOPS, 4),
                   "gpu_ms_per_step": round(ev0.elapsed_time(ev1) / args.steps, 3),
                   "rel_err_vs_oracle": err},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
