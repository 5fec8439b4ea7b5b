#!/usr/bin/env python3
"""Throughput of the PSD-cone projection on one MI355X.

Default workload (c5): one d = 8 process-matrix block, n = d^4 = 4096, X =
(G + G^H)/2 with G iid circular CN(0,1) (seed 1005), projected by the FP64
eigen path (unpack, blocked Householder tridiagonalisation, divide and
conquer, back-transform, fused clamp + reconstruction + svec pack) -- the
paper's c128 arithmetic at its largest size (Table III, d = 8).  One step =
one projection; inputs are resident in HBM before the timed region.  Context
fields of the same line: the derivative (VJP) rate from the saved eigen-pair;
the FP32- and BF16-mixed rates at the same order; the error of every form
against the closed form on a constructed spectrum of the same order (Haar U,
|lambda| log-uniform in [1e-6, 1], half negative); the FP64 GEMMs' MFMA rate;
the composite bound T* = F_MFMA / P_FP64 + B_HEMV / BW; and a NumPy eigh-based
projection on the host (the paper's CPU column, Table III "NumPy c128").

Other workloads (one JSON line each, selected with --workload):
  c1  50 blocks of order 16 (d = 2), one batched launch per step
  c2  the n = 625 (d = 5) warm-start sequence: 50 SCS-like iterates
      X_{k+1} = X_k + 1e-3 (H_k + H_k^H)/2 projected one after another
      (--warm: iterates 1.. by psd_project_warm, each from the eigen-pair
      the previous one left; the roofline is then the FP64 GEMMs')
  c3  orders 1296 and 2401 (d = 6, 7), spectra in [-1,-1e-6] u [1e-6,1],
      --mode mixed_bf16 | mixed_bf16x3 | mixed_fp32 | fp64 (--n picks the order)
  c4  one cone of 32 instances x [W (d^4) + 8 Choi (d^2)] by one graph
      launch per step (--d picks d, --mode the precision; the plan is
      autotuned first unless --no-tune)
  c5  (default) order 4096, --mode fp64 | mixed_*

The JSON line carries the roofline of the dominant kernel, timed live with
HIP events recorded by the library on the kernel's own launch stream (FP64:
the tridiagonalisation's HEMV; mixed: the Newton-Schulz products or the FP64
products, whichever takes more of a projection in an untimed probe, with the
other as context), and the CPU oracle timed on a bounded sample of the same
workload.  Its "traffic" is the HBM bytes per launch that rocprofv3 counters
measured for that kernel (profiles/traffic_*.txt, scaled by the counters of a
plain copy of known size, --copy-calibration); it is null when the kernel's
source files no longer have the hash recorded with the counters.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload c5]
"""
import hashlib
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_FP64_TFLOPS = 78.6        # MI355X dense FP64 (vector = MFMA)
PEAK_FP32_TFLOPS = 157.3       # MI355X dense FP32 MFMA
PEAK_BF16_TFLOPS = 2500.0      # MI355X dense BF16 MFMA


def flops_eig(n: int, k: int) -> float:
    """Algorithmic real flops of one FP64-path projection: tridiagonalisation
    16/3 n^3, back-transform 8 n^2 k and reconstruction 4 n^2 k (k columns of
    the smaller sign side; 8 flops per complex multiply-add)."""
    return 16.0 / 3.0 * n ** 3 + 8.0 * n * n * k + 4.0 * n * n * k


def flops_ns(n: int, iters: int, corr: int) -> float:
    """Algorithmic real flops of one mixed projection: per Newton-Schulz step
    two Hermitian products (lower half: 4 n^3 each), per FP64 correction two
    Hermitian products (lower half: 4 n^3 each), and the final full product
    X S (8 n^3; its Hermitian and anti-Hermitian parts are both used)."""
    return iters * 2 * 4.0 * n ** 3 + corr * 2 * 4.0 * n ** 3 + 8.0 * n ** 3


def flops_mfma_eig(n: int, k: int) -> float:
    """GEMM-shaped part of the FP64 path: the rank-2k trailing updates of the
    tridiagonalisation (half of its 16/3 n^3), back-transform and
    reconstruction."""
    return 8.0 / 3.0 * n ** 3 + 12.0 * n * n * k


def bytes_hemv(n: int) -> float:
    """Bytes the tridiagonalisation's HEMVs must stream: the lower triangle of
    each trailing matrix once per column, 16 bytes per complex entry."""
    return 8.0 / 3.0 * n ** 3


def log(msg):
    """Progress of the benchmark's phases (stderr; stdout carries the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_cpu():
    """CPU model and socket count of the host (from /proc/cpuinfo)."""
    model, sockets = None, set()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name") and model is None:
                    model = line.split(":", 1)[1].strip()
                elif line.startswith("physical id"):
                    sockets.add(line.split(":", 1)[1].strip())
    except OSError:
        pass
    return model, (len(sockets) or None)


def measured_traffic(kernel, n, sources):
    """HBM bytes per launch of `kernel` at order n from the committed counter
    summary, or None if there is none or the kernel's sources have changed
    (sha256 over the files in `sources`, concatenated in that order)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_n{n}.txt")
    srcs = [os.path.join(ROOT, "paper_2606_20519_amd", "csrc", f) for f in sources]
    if not (os.path.exists(path) and all(os.path.exists(f) for f in srcs)):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in srcs:
        with open(f, "rb") as fh:
            h.update(fh.read())
    digest = h.hexdigest()
    if fields.get("source_sha256") != digest:
        return None
    try:
        return round(float(fields["hbm_bytes_per_launch"]), 1)
    except (KeyError, ValueError):
        return None


def mfma_roofline(fp64_gemm, mode, n, timed, warm=False):
    """Roofline entry of an MFMA kernel family from (ms, launches, flops):
    the FP64 GEMM or the Newton-Schulz products."""
    achieved = timed[2] / (timed[0] * 1e-3) / 1e12
    if fp64_gemm:
        use = ("the split-K products of the warm refinement (A X, X^H A X, X^H X, X E) and the "
               "reconstruction, with the cold first iterate's trailing updates and back-transform" if warm else
               "the FP64 corrections and the final product X S of the mixed form")
        return {"kernel": f"gemm_kernel<cd,...> (FP64 complex GEMM, 64x64 tiles: {use})",
                "bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": None,
                "algorithmic_flops_per_launch": round(timed[2] / timed[1], 1)}
    peak = PEAK_FP32_TFLOPS if mode == "mixed_fp32" else PEAK_BF16_TFLOPS
    npad = (n + 63) // 64 * 64
    kname = ("ns_gemm128_kernel (128x128 tiles, direct global-to-LDS loads; split tail summed by "
             "ns128_tail_kernel)" if mode == "mixed_bf16" and npad >= 2048 else
             "ns_gemm128_kernel<split> (128x128 tiles, eight planes direct to LDS, hi*hi + hi*lo + lo*hi)"
             if mode == "mixed_bf16x3" and npad >= 2048 else
             "ns_gemm_kernel<bf16, split> (64x64 tiles, hi*hi + hi*lo + lo*hi)" if mode == "mixed_bf16x3" else
             f"ns_gemm_kernel<{'bf16' if mode == 'mixed_bf16' else 'f32'}> (64x64 tiles)")
    out = {"kernel": kname + ", Hermitian-half complex GEMM of the Newton-Schulz steps",
           "bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
           "frac": round(achieved / peak, 4), "traffic": None,
           "algorithmic_flops_per_launch": round(timed[2] / timed[1], 1)}
    if mode == "mixed_bf16x3":
        # three BF16 products per real product: the MFMA work executed
        out["executed_bf16_tflops"] = round(3 * achieved, 3)
        out["executed_frac"] = round(3 * achieved / peak, 4)
    return out


def oracle_single_thread(n: int) -> dict:
    """The oracle on one thread (a child process with OMP_NUM_THREADS=1, no
    GPU use): one projection of the first iterate of the n-order sequence."""
    import subprocess
    code = ("import sys, time; sys.path.insert(0, sys.argv[1]); import oracle; "
            "from paper_2606_20519_amd import workloads as W; x = W.warm_sequence(int(sys.argv[2]), 1002, 1)[0]; "
            "oracle.project(x[:16], 4); t = time.perf_counter(); oracle.project(x, int(sys.argv[2])); "
            "print(time.perf_counter() - t)")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code, ROOT, str(n)], env=env, capture_output=True, text=True,
                       timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr.strip()[-200:]}
    dt = float(r.stdout.strip().splitlines()[-1])
    return {"value": round(1.0 / dt, 6), "unit": "projections/s", "cores": 1, "seconds": round(dt, 2),
            "sample": f"one oracle projection of the first iterate (n={n}), one thread"}


def c5_closed_form_errors(P, oracle, W, n, g_np, dev, extra):
    """Errors of the FP64, FP32-, BF16- and BF16x3-mixed projections and of the
    derivative against the closed forms on a constructed spectrum of order n
    (seed 1009, |lambda| log-uniform in [1e-6, 1], half negative).  Returns
    the FP64 error; the others go to `extra`."""
    import numpy as np
    import torch
    log("closed-form errors on a constructed spectrum")
    s, u, lam = W.constructed(n, 1009, gap=1e-6)
    exact = oracle.constructed_projection(u, lam)
    xc = torch.from_numpy(s).to(dev)
    nrm = np.linalg.norm(exact)
    out = None
    for mm in ("fp64", "mixed_fp32", "mixed_bf16", "mixed_bf16x3"):
        y, inf = P.project(xc, n, mm, info=True)
        e = float(np.linalg.norm(y.cpu().numpy() - exact) / nrm)
        if mm == "fp64":
            out = e
        else:
            extra[f"{mm}_rel_err_vs_closed_form"] = e
            extra[f"{mm}_est_rel_err"] = inf["est_rel_err"]
    gx = P.vjp(torch.from_numpy(g_np).to(dev), n, x=xc).cpu().numpy()
    ref = oracle.constructed_vjp(u, lam, g_np)
    extra["vjp_rel_err_vs_closed_form"] = float(np.linalg.norm(gx - ref) / np.linalg.norm(ref))
    extra["closed_form_input"] = "Haar U, |lambda| log-uniform in [1e-6, 1], half negative (seed 1009)"
    return out


def numpy_eigh_baseline(np, oracle, x_svec, n):
    """The paper's CPU column (Table III, NumPy c128): numpy.linalg.eigh of
    the block, negative eigenvalues set to zero, reconstruction by a BLAS
    product; timed on the host cores."""
    try:
        from threadpoolctl import threadpool_info
        pools = [{"api": p.get("internal_api"), "threads": p.get("num_threads"), "version": p.get("version")}
                 for p in threadpool_info()]
    except Exception:
        pools = None
    log("NumPy eigh projection on the host")
    a = oracle.unpack(x_svec, n)
    t = time.perf_counter()
    w, v = np.linalg.eigh(a)
    p = (v * np.maximum(w, 0.0)) @ v.conj().T
    dt = time.perf_counter() - t
    del p
    model, sockets = host_cpu()
    return {"seconds": round(dt, 3), "proj_per_s": round(1.0 / dt, 5), "blas": pools, "cpu_model": model,
            "sockets": sockets}


def scs_context(P, W, torch, dev) -> dict:
    import numpy as np
    """The whole SCS iteration (App. D) on GPU-resident data: a GYNI process
    SDP from a seeded pair of random feasible instruments solved to
    eps = 1e-5 at d = 5 (plain, with Anderson memory 5, and with warm cone
    steps: psd_project_warm from the previous step's eigen-pair), and the
    per-iteration time at d = 8 over a fixed iteration count (FP64 cone
    steps, then mixed-precision ones).  The
    paper's wall-clock table for comparison (T4 GPU / one CPU, other
    hardware): d = 5, 275 iterations, 21 s; d = 8, 300 iterations, 44 min
    (SCS on the CPU: 4.4 h)."""
    out = {}
    for d, eps, iters in ((5, 1e-5, 5000), (8, 0.0, 8)):
        g = torch.from_numpy(W.upper_pack(W.gyni_objective(d, 7))).to(dev)
        P.scs_solve(g, d, eps=0.0, max_iters=2, post=False)     # warm-up (code objects, workspace)
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = P.scs_solve(g, d, eps=eps, max_iters=iters, post=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        rec = {"eps": eps, "status": r["status"], "iterations": r["iters"], "seconds": round(dt, 3),
               "ms_per_iteration": round(1e3 * dt / r["iters"], 3), "value": r["pobj"], "dual_bound": r["dobj"],
               "residuals": [r["res_pri"], r["res_dual"], r["gap"]]}
        if d == 5:
            t = time.perf_counter()
            ra = P.scs_solve(g, d, eps=eps, max_iters=iters, post=False, anderson=5)
            torch.cuda.synchronize()
            rec["anderson5"] = {"iterations": ra["iters"], "seconds": round(time.perf_counter() - t, 3),
                                "value": ra["pobj"], "accepted": ra["aa_accepted"], "rejected": ra["aa_rejected"]}
            # FP64 cone steps refined from the previous step's eigen-pair
            t = time.perf_counter()
            rw = P.scs_solve(g, d, eps=eps, max_iters=iters, post=False, warm_proj=True)
            torch.cuda.synchronize()
            rec["warm_cone_steps"] = {"iterations": rw["iters"], "seconds": round(time.perf_counter() - t, 3),
                                      "value": rw["pobj"], "refined": rw["warm_refined"],
                                      "fallbacks": rw["warm_fallbacks"]}
        if d == 8:
            rec["projected_300_iterations_s"] = round(0.3 * dt / r["iters"] * 1e3, 1)
            for mm in ("mixed_fp32", "mixed_bf16", "mixed_bf16x3"):
                t = time.perf_counter()
                rm = P.scs_solve(g, d, eps=0.0, max_iters=iters, mixed_iters=iters, mixed_mode=mm, post=False)
                torch.cuda.synchronize()
                rec[f"ms_per_iteration_{mm}"] = round(1e3 * (time.perf_counter() - t) / rm["iters"], 3)
        out[f"d{d}"] = rec
        log(f"SCS d={d}: {rec}")
    # many independent d = 5 solves in lockstep (the paper's exploration
    # stage runs the see-saw from many random starts): per-iteration rate of
    # a batch of 32 against one instance
    d, B, its = 5, 32, 10
    G = torch.from_numpy(np.stack([W.upper_pack(W.gyni_objective(d, 100 + b)) for b in range(B)])).to(dev)
    P.scs_solve_batched(G[:2], d, eps=0.0, max_iters=2, post=False)
    torch.cuda.synchronize()
    t = time.perf_counter()
    P.scs_solve_batched(G, d, eps=0.0, max_iters=its, post=False)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t) / its
    out["batched_d5"] = {"instances": B, "ms_per_iteration": round(1e3 * tb, 3),
                         "ms_per_instance_iteration": round(1e3 * tb / B, 4),
                         "throughput_vs_single": round(out["d5"]["ms_per_iteration"] * 1e-3 * B / tb, 2)}
    log(f"SCS batched d=5: {out['batched_d5']}")
    out["paper_t4_gpu"] = {"d5": {"iterations": 275, "seconds": 21}, "d8": {"iterations": 300, "seconds": 2640}}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--mode", default=None, help="fp64 | mixed_bf16 | mixed_bf16x3 | mixed_fp32")
    ap.add_argument("--n", type=int, default=1296, help="order for c3")
    ap.add_argument("--d", type=int, default=5, help="local dimension for c4")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=10, help="blocks projected by the CPU oracle (bounded sample)")
    ap.add_argument("--no-context", action="store_true",
                    help="skip the context measurements after the timed region (counter runs)")
    ap.add_argument("--no-tune", action="store_true",
                    help="c4: run the plan at its default concurrency and group size (no autotuning)")
    ap.add_argument("--warm", action="store_true",
                    help="c2: iterates 1.. by psd_project_warm from the pair the previous one left")
    ap.add_argument("--blocks", type=int, default=50, help="blocks per step for c1 / c2 (counter runs use fewer)")
    ap.add_argument("--counter-run", action="store_true",
                    help="only project the workload's inputs once (one step, no probes, no JSON line): the "
                         "program profiled by the rocprofv3 counter runs")
    ap.add_argument("--scs-run", type=int, default=0, metavar="D",
                    help="only run the SCS solver on the GYNI objective at local dimension D for --scs-iters "
                         "iterations (no JSON line): the program profiled for the solver's kernel trace")
    ap.add_argument("--scs-iters", type=int, default=5)
    ap.add_argument("--scs-anderson", type=int, default=0)
    ap.add_argument("--scs-batch", type=int, default=1,
                    help="with --scs-run: solve this many instances (seeds 7, 8, ...) in one batched call")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB device to device 3 times (counter calibration) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU only; --gpus must be 1 "
                                   "(each cone block is projected on one GPU here)"}))
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        nbytes = 256 << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read_per_launch": nbytes,
                          "bytes_written_per_launch": nbytes, "launches": 3}), flush=True)
        return

    import paper_2606_20519_amd as P
    from paper_2606_20519_amd import _lib
    from paper_2606_20519_amd import workloads as W

    if args.scs_run:
        d = args.scs_run
        nb = max(1, args.scs_batch)
        log(f"SCS run: d={d}, {nb} instance(s), {args.scs_iters} iterations, Anderson memory {args.scs_anderson}")
        g = torch.from_numpy(np.stack([W.upper_pack(W.gyni_objective(d, 7 + b)) for b in range(nb)])).to("cuda:0")
        t = time.perf_counter()
        if nb == 1:
            rs = [P.scs_solve(g[0], d, eps=0.0, max_iters=args.scs_iters, anderson=args.scs_anderson, post=False)]
        else:
            rs = P.scs_solve_batched(g, d, eps=0.0, max_iters=args.scs_iters, anderson=args.scs_anderson, post=False)
        torch.cuda.synchronize()
        log(f"SCS run done: {rs[0]['iters']} iterations of {nb} instance(s) in {time.perf_counter() - t:.3f} s, "
            f"tau {rs[0]['tau']:.6e}")
        return

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    wl = args.workload
    mode = args.mode or ("mixed_bf16" if wl == "c3" else "fp64")
    extra = {}
    corr = -1
    P.set_ns_iterations(0, corr)  # automatic step count (scaled schedule) and corrections
    iters = 0
    if mode != "fp64":
        _, inf = P.project(torch.from_numpy(W.gue(100, 1)).to(dev), 100, mode, info=True)
        iters = inf["iters"]
        extra["ns_steps"] = iters
        extra["fp64_corrections"] = 1 if mode == "mixed_bf16" else 0

    # ---- inputs (host, seeded) -> HBM
    log(f"workload {wl} mode {mode}: building inputs")
    plan = None
    if wl == "c2":
        n, count = 625, args.blocks
        xs_np = W.warm_sequence(n, 1002, count)
        desc = (f"d=5 warm-start sequence: {count} iterates of a 625x625 Hermitian block, "
                "projected one after another")
        if args.warm:
            assert mode == "fp64", "--warm is an FP64 path"
            desc += (" (iterate 0 by the cold path, saving its eigen-pair; iterates 1.. by psd_project_warm from "
                     "the pair the previous one left)")
        sizes = [n] * count
    elif wl == "c1":
        n, count = 16, args.blocks
        xs_np = [W.gue(n, 1001 + i) for i in range(count)]
        desc = f"d=2 process matrices: {count} blocks of order 16, one batched launch"
        sizes = [n] * count
    elif wl == "c3":
        n, count = args.n, 2
        cons = [W.constructed(n, 1003 + i, gap=1e-6) for i in range(count)]
        xs_np = [c[0] for c in cons]
        desc = f"order {n}, spectra in [-1,-1e-6] u [1e-6,1] (constructed, Haar U)"
        sizes = [n] * count
    elif wl == "c4":
        d = args.d
        x_cone, sizes = W.cone(d, 32)
        n, count = d ** 4, 1
        xs_np = [x_cone]
        desc = f"one cone, d={d}: 32 instances x [W {d**4}x{d**4} + 8 Choi {d*d}x{d*d}], one graph launch"
    else:  # c5
        n, count = 4096, 1
        xs_np = [W.gue(n, 1005)]
        g_np = W.gue(n, 1006)
        desc = ("d=8 process matrix: one 4096x4096 complex Hermitian block (G+G^H)/2, projected one "
                "after another")
        sizes = [n]
    if wl in ("c2", "c3", "c5"):
        X = torch.from_numpy(np.stack(xs_np)).to(dev)
        Y = torch.empty_like(X)
    else:
        X = torch.from_numpy(np.concatenate(xs_np)).to(dev)
        Y = torch.empty_like(X)

    if wl == "c4":
        plan = P.Plan(sizes, mode)

        def step():
            plan.execute(X, out=Y)
    elif wl == "c1":
        def step():
            P.project_batched(X, sizes, mode, out=Y)
    elif wl == "c2" and args.warm:
        SAVED = torch.empty(P.saved_numel(n), dtype=torch.float64, device=dev)

        def step():
            P.project(X[0], n, mode, out=Y[0], saved=SAVED)
            for i in range(1, count):
                P.project_warm(X[i], n, SAVED, out=Y[i])
    else:
        def step():
            for i in range(count):
                P.project(X[i], n, mode, out=Y[i])

    if args.counter_run:
        log("counter run: one step")
        step()
        torch.cuda.synchronize()
        log("counter run done")
        return

    # side counts for the algorithmic flops (outside timing)
    ks = []
    if wl in ("c2", "c5") or (wl == "c3" and mode == "fp64"):
        for i in range(count):
            _, inf = P.project(X[i], n, "fp64", out=Y[i], info=True)
            ks.append(min(inf["n_pos"], inf["n_neg"]))
    if mode == "fp64":
        if wl == "c4":
            flops_step = sum(flops_eig(m, m // 2) for m in sizes if m > 64)
        elif wl == "c1":
            flops_step = 0.0
        else:
            flops_step = sum(flops_eig(n, k) for k in ks)
    else:
        flops_step = sum(flops_ns(m, iters, extra["fp64_corrections"]) for m in sizes if m > 64)

    if wl == "c4":
        # the autotuner picks the group size and the concurrency (outside
        # timing; its cache goes to a temporary file unless PSD_TUNE_CACHE is set)
        if not os.environ.get("PSD_TUNE_CACHE"):
            import tempfile
            os.environ["PSD_TUNE_CACHE"] = os.path.join(tempfile.gettempdir(), "psdproj_bench_tune.jsonl")
        if not args.no_tune:
            plan.tune(X, Y, reps=3 if args.d <= 6 else 2, max_concurrency=8)
        plan.execute(X, out=Y)   # capture outside timing
    log("warm-up")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # dominant kernel: HEMV of the tridiagonalisation (FP64) or the
    # Newton-Schulz GEMMs (mixed); the library brackets its launches with HIP
    # events on their launch stream -- the first projection's launches
    fam = None
    other = None
    if wl == "c2" and args.warm:
        # the FP64 GEMMs of the first timed step (mostly the refinements'
        # products); per-iterate refinement steps and fallbacks from an
        # untimed pass of the sequence
        _lib.timing_start(_lib.KF_GEMM, 4096)
        step()
        torch.cuda.synchronize()
        fam, sample = _lib.KF_GEMM, _lib.timing_stop()[1]   # the GEMM launches of one step
        steps, falls = [], 0
        P.project(X[0], n, mode, out=Y[0], saved=SAVED)
        for i in range(1, count):
            _, inf = P.project_warm(X[i], n, SAVED, out=Y[i], info=True)
            steps.append(inf["iters"])
            falls += inf["fallback"]
        extra["warm"] = {"refinement_steps": {str(k): steps.count(k) for k in sorted(set(steps))},
                         "fallbacks": falls, "iterates": count - 1}
        flops_step = flops_eig(n, ks[0]) + sum(8.0 * n ** 3 * (3.0 * k + 0.5) for k in steps)
    elif mode == "fp64" and n > 64 and wl != "c4":
        # one projection's HEMV launches (the columns before the LDS tail),
        # counted by an untimed probe
        _lib.timing_start(_lib.KF_HEMV, n)
        P.project(X[0], n, mode, out=Y[0])
        torch.cuda.synchronize()
        fam, sample = _lib.KF_HEMV, _lib.timing_stop()[1]
        # the per-column w / next-column step between the HEMV launches
        # (latency bound: no roofline, its launches kept as context)
        _lib.timing_start(_lib.KF_WSTEP, n)
        P.project(X[0], n, mode, out=Y[0])
        torch.cuda.synchronize()
        other = (_lib.KF_WSTEP, _lib.timing_stop())
    elif mode != "fp64" and wl != "c4":
        # the Newton-Schulz products or the FP64 products (corrections and
        # the final X S) -- whichever family takes more of one projection,
        # from an untimed probe of each (the other is kept as context)
        probe = {}
        for f in (_lib.KF_NS, _lib.KF_GEMM):
            _lib.timing_start(f, 4096)
            P.project(X[0], n, mode, out=Y[0])
            torch.cuda.synchronize()
            probe[f] = _lib.timing_stop()
        fam = max(probe, key=lambda f: probe[f][0])
        sample = probe[fam][1]
        o = _lib.KF_GEMM if fam == _lib.KF_NS else _lib.KF_NS
        if probe[o][1] > 0:
            other = (o, probe[o])
    log(f"timing {args.steps} steps")
    if fam:
        _lib.timing_start(fam, sample)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timed = _lib.timing_stop() if fam else (0.0, 0, 0.0)

    wall = t1 - t0
    ms_per_step = 1e3 * wall / args.steps
    blocks_per_step = len(sizes) if wl in ("c1", "c4") else count
    value = (1 if wl == "c4" else blocks_per_step) * args.steps / wall
    tflops = flops_step * args.steps / wall / 1e12

    roofline = None
    if timed[1] > 0:
        avg_ms = timed[0] / timed[1]
        if fam == _lib.KF_HEMV:
            achieved = timed[2] / (timed[0] * 1e-3) / 1e9
            roofline = {"kernel": "hemv_kernel (per-column Hermitian matrix-vector tiles, tridiagonalisation)",
                        "bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": round(achieved / PEAK_HBM_GBS, 4),
                        "traffic": measured_traffic("hemv_kernel", n, ("tridiag.hip", "common.h")),
                        "algorithmic_bytes_per_launch": round(timed[2] / timed[1], 1)}
            if other and other[1][1] > 0:
                pr = other[1]
                roofline["other_kernel"] = {
                    "kernel": "w_kernel (per-column w / next-column step, tridiagonalisation)", "bound": "latency",
                    "avg_launch_us": round(1e3 * pr[0] / pr[1], 3), "launches": pr[1],
                    "share_of_projection_ms": round(pr[0], 3), "sample": "untimed probe projection (HIP events)"}
        else:
            roofline = mfma_roofline(fam == _lib.KF_GEMM, mode, n, timed, warm=args.warm)
            if other:
                o, pr = other
                ctx = mfma_roofline(o == _lib.KF_GEMM, mode, n, pr)
                ctx.update({"avg_launch_us": round(1e3 * pr[0] / pr[1], 3), "launches": pr[1],
                            "share_of_projection_ms": round(pr[0], 3),
                            "sample": "untimed probe projection (HIP events)"})
                roofline["other_mfma_kernel"] = ctx
        # the timed launches belong to the first projection of the step (with
        # --warm: to the whole first step)
        per_proj_ms = ms_per_step / (1 if wl == "c4" else blocks_per_step)
        roofline.update({"launches_timed": timed[1], "avg_launch_us": round(1e3 * avg_ms, 3),
                         "sample": ("GEMM launches of the first step in the timed region" if args.warm else
                                    "launches of the first projection in the timed region")})
        if args.warm:
            roofline["share_of_step"] = round(timed[0] / ms_per_step, 4)
        else:
            roofline["share_of_projection"] = round(timed[0] / per_proj_ms, 4)

    if wl == "c2" and mode == "fp64" and not args.no_context:
        # context only: the same iterates as independent blocks of one batched
        # call (lockstep groups), which SCS cannot do with its own iterates
        flat = X.reshape(-1)
        yb = P.project_batched(flat, sizes, mode)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(2):
            P.project_batched(flat, sizes, mode, out=yb)
        torch.cuda.synchronize()
        extra["independent_batch_proj_per_s"] = round(2 * count / (time.perf_counter() - t), 2)
        extra["independent_batch_max_abs_diff"] = float((yb.reshape(Y.shape) - Y).abs().max())

    if wl == "c1":
        # context: one block of order 16 as a one-block plan, 10^4 graph replays
        p1 = P.Plan([n], mode)
        x1 = X[:n * n].clone()
        y1 = p1.execute(x1)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(10000):
            p1.execute(x1, out=y1)
        torch.cuda.synchronize()
        extra["single_block_latency_us_graph"] = round((time.perf_counter() - t) / 10000 * 1e6, 2)
        p1.close()
        t = time.perf_counter()
        for _ in range(10000):
            P.project(x1, n, mode, out=y1)
        torch.cuda.synchronize()
        extra["single_block_latency_us_eager"] = round((time.perf_counter() - t) / 10000 * 1e6, 2)
    if wl == "c4":
        extra["block_projections_per_s"] = round(value * len(sizes), 1)

    if wl == "c5" and mode == "fp64" and not args.no_context:
        log("context: derivative, FP64 GEMMs, mixed forms")
        per_proj_ms = ms_per_step
        k = ks[0]
        # derivative after the forward (eigen-pair saved by the forward)
        sv = torch.empty(P.saved_numel(n), dtype=torch.float64, device=dev)
        G = torch.from_numpy(g_np).to(dev)
        P.project(X[0], n, "fp64", out=Y[0], saved=sv)
        gx = P.vjp(G, n, saved=sv)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            P.vjp(G, n, saved=sv, out=gx)
        torch.cuda.synchronize()
        extra["vjp_per_s"] = round(args.steps / (time.perf_counter() - t), 4)
        extra["vjp_algorithmic_tflops"] = round(32.0 * n ** 3 * extra["vjp_per_s"] / 1e12, 3)
        # the FP64 GEMMs of one projection (HER2K updates, back-transform,
        # reconstruction): algorithmic MFMA flops over their summed launch time
        _lib.timing_start(_lib.KF_GEMM, 4096)
        P.project(X[0], n, mode, out=Y[0])
        torch.cuda.synchronize()
        gms, glaunch, _ = _lib.timing_stop()
        fm = flops_mfma_eig(n, k)
        gt = fm / (gms * 1e-3) / 1e12
        extra["fp64_gemm_mfma"] = {"kernel": "gemm_kernel<cd,...> (FP64 complex GEMMs: rank-2k updates, "
                                             "back-transform, reconstruction)",
                                   "achieved": round(gt, 2), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                   "frac": round(gt / PEAK_FP64_TFLOPS, 4), "launches": glaunch,
                                   "ms_per_projection": round(gms, 3),
                                   "algorithmic_flops": fm}
        # composite bound: MFMA work at the FP64 peak plus the HEMV stream at HBM peak
        tstar = (fm / (PEAK_FP64_TFLOPS * 1e12) + bytes_hemv(n) / (PEAK_HBM_GBS * 1e9)) * 1e3
        extra["composite_bound_ms"] = round(tstar, 3)
        extra["frac_of_composite_bound"] = round(tstar / per_proj_ms, 4)
        # the mixed forms at the same order (their error against the closed
        # form is measured in the baseline leg below)
        for mm, reps in (("mixed_fp32", 3), ("mixed_bf16", 5), ("mixed_bf16x3", 3)):
            _, inf = P.project(X[0], n, mm, out=Y[0], info=True)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                P.project(X[0], n, mm, out=Y[0])
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) / reps
            extra[f"{mm}_proj_per_s"] = round(1.0 / dt, 3)
            extra[f"{mm}_est_rel_err_gue"] = inf["est_rel_err"]
        P.project(X[0], n, mode, out=Y[0])   # Y holds the FP64 result again
        torch.cuda.synchronize()
        # the affine step on either side of the projection (App. D.2), same order
        dloc = round(n ** 0.25)
        if dloc ** 4 == n:
            nx, _ = P.affine_dims(dloc)
            ax = torch.randn(nx, dtype=torch.float64, device=dev)
            zx, zy = P.affine_step(ax, X[0], dloc)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(args.steps):
                P.affine_step(ax, X[0], dloc, zx=zx, zy=zy)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) / args.steps
            minbytes = 16.0 * (nx + n * n)   # read a_x, a_y; write z_x, z_y
            extra["affine_step"] = {"ms": round(1e3 * dt, 3), "share_of_projection": round(1e3 * dt / per_proj_ms, 4),
                                    "nx": nx, "min_hbm_gbs": round(minbytes / dt / 1e9, 1),
                                    "passes": "per direction: modes 2+3 with the svec unpack/pack, mode 1, mode 0 with the "
                                              "gather/scatter (each input read once through LDS)"}
        if wl == "c5" and not args.no_context:
            log("SCS solves (GYNI, d = 5 to 1e-5; d = 8 per-iteration time)")
            extra["scs"] = scs_context(P, W, torch, dev)

    # parity on a sample of the timed outputs; CPU oracle baseline
    cpu, err = None, None
    if not args.no_cpu_baseline:
        log("CPU baselines and errors against the oracle / closed forms")
        import oracle
        y_np = Y.cpu().numpy()
        if wl in ("c1", "c4"):
            flat_x, flat_y = xs_np[0] if wl == "c4" else np.concatenate(xs_np), y_np.reshape(-1)
            offs, o = [], 0
            for m in sizes:
                offs.append(o)
                o += m * m
            # bounded sample: the first W block when the oracle finishes it in
            # seconds (order <= 1300), then Choi blocks
            pick = ([0] if sizes[0] <= 1300 else []) + [i for i, m in enumerate(sizes) if m <= 64]
            pick = pick[:max(1, args.cpu_sample)]
            t = time.perf_counter()
            refs = [oracle.project(flat_x[offs[i]:offs[i] + sizes[i] ** 2], sizes[i]) for i in pick]
            dt = time.perf_counter() - t
            err = max(float(np.linalg.norm(flat_y[offs[i]:offs[i] + sizes[i] ** 2] - r) / np.linalg.norm(r))
                      for i, r in zip(pick, refs))
            sample = f"blocks {pick} of the cone (orders {[sizes[i] for i in pick]})"
            value_cpu = len(pick) / dt
            unit = "block projections/s"
        elif wl == "c5":
            # bounded sample: the oracle's Jacobi at n = 4096 takes several
            # minutes per sweep; one full oracle projection of a 1024 x 1024
            # block of the same construction is timed and scaled by
            # (1024/4096)^3 (its sweep count grows slowly with n: 11 at 512,
            # 12 at 1024)
            ns = 1024
            xs_s = W.gue(ns, 1005)
            t = time.perf_counter()
            oracle.project(xs_s, ns)
            dt = time.perf_counter() - t
            value_cpu = (ns / n) ** 3 / dt
            unit = "projections/s"
            sample = (f"one oracle projection (cyclic Jacobi, round-robin, FP64) of a {ns}x{ns} block of the same "
                      f"construction, {dt:.1f} s, scaled to n={n} by ({ns}/{n})^3")
            if not args.no_context:
                err = c5_closed_form_errors(P, oracle, W, n, g_np, dev, extra)
                extra["numpy_eigh_projection"] = numpy_eigh_baseline(np, oracle, xs_np[0], n)
        else:
            m = max(1, min(args.cpu_sample, count))
            if n > 1300:
                # bounded sample: the oracle's Jacobi at this order takes minutes
                sample = f"skipped at n={n} (oracle Jacobi at this order exceeds the time bound)"
                value_cpu, dt, unit = None, 0.0, "projections/s"
                if wl == "c3":
                    exact = oracle.constructed_projection(cons[0][1], cons[0][2])
                    err = float(np.linalg.norm(y_np[0] - exact) / np.linalg.norm(exact))
            else:
                t = time.perf_counter()
                refs = [oracle.project(xs_np[i], n) for i in range(m)]
                dt = time.perf_counter() - t
                err = max(float(np.linalg.norm(y_np[i] - refs[i]) / np.linalg.norm(refs[i])) for i in range(m))
                sample = f"first {m} of the {count} blocks (n={n}), cyclic Jacobi round-robin FP64, {dt:.1f} s"
                value_cpu = m / dt
                unit = "projections/s"
            if wl == "c3" and mode != "fp64":
                # truncation alone: the same scaled schedule in exact arithmetic
                # per eigenvalue (the rest of the error is low-precision rounding)
                _, inf0 = P.project(X[0], n, mode, info=True)
                sched = oracle.ns_schedule(iters=inf0["iters"])
                exact = oracle.constructed_projection(cons[0][1], cons[0][2])
                trunc = oracle.ns_constructed_projection(cons[0][1], cons[0][2], inf0["scale"], inf0["iters"], sched)
                extra["ns_truncation_rel_err"] = float(np.linalg.norm(trunc - exact) / np.linalg.norm(exact))
        model, sockets = host_cpu()
        cpu = {"value": round(value_cpu, 6) if value_cpu else None, "unit": unit, "cores": oracle.num_threads(),
               "kind": "oracle", "sample": sample, "cpu_model": model, "sockets": sockets}
        if wl == "c2":
            cpu["single_thread"] = oracle_single_thread(n)

    metric = {"c4": "PSD cone projections/sec (one graph launch per cone)"}.get(wl, "PSD projections/sec")
    out = {
        "metric": metric + f" ({mode})",
        "value": round(value, 4),
        "unit": "cones/s" if wl == "c4" else "projections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "mixed_bf16": "bf16+f64", "mixed_fp32": "f32+f64", "mixed_bf16x3": "bf16x3+f64"}[mode],
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "blocks_per_step": blocks_per_step, "mode": mode,
                   "algorithmic_tflops": round(tflops, 3),
                   "peak_frac": round(tflops / (PEAK_FP64_TFLOPS if mode == "fp64" else
                                                (PEAK_FP32_TFLOPS if mode == "mixed_fp32" else PEAK_BF16_TFLOPS)), 5),
                   "gpu_ms_per_step": round(ev0.elapsed_time(ev1) / args.steps, 3),
                   "rel_err_vs_oracle": err, **extra},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if plan is not None:
        out["config"]["concurrency"] = plan.concurrency
        out["config"]["group_size"] = plan.group_size
        out["config"]["ns_tile_threshold"] = plan.ns_tile_threshold
        plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
