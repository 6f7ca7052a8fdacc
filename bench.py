"""Throughput of the Vecchia log-likelihood + gradient + Fisher-information
path on one MI355X.

Workload: the satellite-shaped space-time problem, n = 1,048,576 observations
(64 time slices x 64 passes x 256 points), m = 30 nearest previously ordered
neighbours, space-time exponential covariance (sigma2, rho_space, rho_time,
tau2), intercept only, FP64 throughout.

One step = one Fisher-scoring iteration on the device: the fused
per-neighbourhood kernel over all n neighbourhoods, the fixed-order
reduction, the combine step and the Eq. (4) update, replayed from a captured
HIP graph.  Inputs are resident in device memory before timing starts.

Prints one JSON line.  `value` is neighbourhoods per second (n x steps /
elapsed).  `roofline` reports the fused kernel (timed alone with HIP events
on its stream) against the FP64 vector peak; `cpu_baseline` times the CPU
oracle on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "neighbourhoods/s (loglik+grad+Fisher), n=1M m=30; plain FP64 vs chosen form"
PEAK_FP64_VECTOR_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_flops(k: int, d: int, p: int, R: int) -> int:
    """FP64 flops one neighbourhood of k = m + 1 observations needs
    (transcendentals excluded): covariance k(k-1)/2 (3d + 2), Cholesky k^3/3,
    forward solves (1 + p) k^2, back solve for u k^2, per range parameter the
    derivative entries 3k(k+1)/2, the symmetric product 2k^2 and a forward
    solve k^2, the nugget solve k^2, the residual derivatives
    (R + 2) 2k(1 + p) and the information (R + 2)(R + 3) k."""
    return int(k * (k - 1) // 2 * (3 * d + 2) + k ** 3 / 3 + (1 + p) * k * k + k * k
               + R * (3 * k * (k + 1) // 2 + 3 * k * k) + k * k + (R + 2) * 2 * k * (1 + p)
               + (R + 2) * (R + 3) * k)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--cpu-sample", type=int, default=262_144)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 512 MiB device-to-device copy (a kernel of known traffic "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; run with --gpus 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2407_02740_amd import synthetic as S
    from paper_2407_02740_amd import vecchia as V

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    log("generating the satellite space-time workload (n = 1,048,576, m = 30)")
    w = S.satellite_spacetime()
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s")
    n, m, d, p = w["n"], w["m"], w["d"], w["p"]
    start_theta = w["covparms"] * np.array([0.7, 1.3, 0.8, 1.5])  # a fit starts off the truth

    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ev = V.Vecchia(w["locs"], w["NN"], w["y"], w["X"], w["family"], w["nu"], w["nspace"])
        cp = ev.covparms(start_theta)
        ev.workspace()
    torch.cuda.synchronize()

    # warm-up steps (also loads the code objects)
    with torch.cuda.stream(stream):
        ev.fisher_fit(cp, args.warmup, use_graph=True, check=False)
    torch.cuda.synchronize()
    ev.check_status("warmup")
    log(f"warm-up done ({args.warmup} steps)")

    # timed steps
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    with torch.cuda.stream(stream):
        ev.fisher_fit(cp, args.steps, use_graph=True, check=False)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ev.check_status("timed steps")
    elapsed = t2 - t1
    ms_per_step = 1e3 * elapsed / args.steps
    value = n * args.steps / elapsed
    res = V.unpack_out(ev.out, p, ev.P)
    log(f"{args.steps} steps in {elapsed * 1e3:.2f} ms -> {value:.4e} nbhd/s; "
        f"loglik {res['loglik']:.6f} theta {cp.cpu().numpy()}")

    # the fused kernel alone, HIP events on its stream
    with torch.cuda.stream(stream):
        ev.block_sums(cp)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.kernel_reps):
            ev.block_sums(cp)
        e1.record(stream)
    torch.cuda.synchronize()
    ev.check_status("kernel timing")
    kernel_ms = e0.elapsed_time(e1) / args.kernel_reps
    R = ev.P - 2
    F = algorithmic_flops(m + 1, d, p, R)
    achieved = F * n / (kernel_ms * 1e-3) / 1e12
    log(f"fused kernel {kernel_ms:.4f} ms, {F} flop/nbhd -> {achieved:.2f} TFLOP/s")

    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 2 x 536870912-byte device copies")

    cpu = None
    if not args.no_cpu:
        import oracle

        oracle.build()
        threads = min(16, os.cpu_count() or 1)
        S_ = min(args.cpu_sample, n)
        log(f"CPU oracle on observations [{n - S_}, {n}) with {threads} threads")
        tc = time.perf_counter()
        oracle.raw_sums(w["locs"], w["NN"], w["y"], w["X"], w["covparms"], w["family"], w["nu"],
                        w["nspace"], i0=n - S_, i1=n, threads=threads)
        dtc = time.perf_counter() - tc
        cpu = {"value": S_ / dtc, "unit": "neighbourhoods/s", "cores": threads, "kind": "oracle",
               "sample": f"last {S_} of {n} neighbourhoods (m=30) of the same workload, "
                         f"{dtc:.2f} s wall"}
        log(f"CPU oracle {cpu['value']:.4e} nbhd/s")

    line = {
        "metric": METRIC, "value": value, "unit": "neighbourhoods/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "satellite_spacetime", "n": n, "m": m, "d": d, "p": p,
                   "covariance": "space-time exponential (sigma2, rho_s, rho_t, tau2)",
                   "step": "Fisher-scoring iteration: fused sums + reduce + combine + update, "
                           "HIP graph replay"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR_TFLOPS,
                     "traffic": None},
        "cpu_baseline": cpu,
        "detail": {"kernel": "sums_kernel<31,1,2>", "kernel_ms": kernel_ms,
                   "flop_per_neighbourhood": F, "loglik": res["loglik"]},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
