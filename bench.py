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
on its stream) against the FP64 vector peak; `traffic` is the HBM traffic per
launch read from the committed rocprofv3 counter summary when that summary
was taken on the current kernel source, else null.  `cpu_baseline` times the
CPU oracle on a bounded sample of the same workload.

`--workload batched_uneven` measures the batched persistent path instead:
512 independent 2-D datasets (n uniform in [1000, 50000], m from
{10, 20, 30, 40}, Matern covariance parameters and smoothness drawn per
dataset), schedule picked by the autotuner, one step = one Fisher-scoring
iteration of every dataset replayed from a captured HIP graph.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "neighbourhoods/s (loglik+grad+Fisher), n=1M m=30; plain FP64 vs chosen form"
METRIC_BATCHED = "neighbourhoods/s (loglik+grad+Fisher), 512 uneven datasets, m in {10,20,30,40}"
METRIC_SURROGATE = "neighbourhoods/s (loglik), surrogate with exact hand-back, n=4M m=30, |dloglik|/n<=1e-6"
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_FP64_VECTOR_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
PROFILE = os.path.join(ROOT, "profiles", "sums_kernel_satellite_spacetime_n1M_m30.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2407_02740_amd", "csrc", f)
                  for f in ("vecchia_kernels.hpp", "exp_table.inc", "dpp_fmac.inc")] + \
                 [os.path.join(ROOT, "paper_2407_02740_amd", "build.py")]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_flops(k: int, d: int, p: int, R: int) -> int:
    """FP64 flops one neighbourhood of k = m + 1 observations needs
    (transcendentals excluded): covariance k(k-1)/2 (3d + 2), Cholesky k^3/3,
    forward solves (1 + p) k^2, back solve for u k^2, per range parameter the
    derivative entries 3k(k+1)/2, the symmetric product 2k^2 and a forward
    solve k^2, the nugget solve k^2, the residual derivatives
    (R + 2) 2k(1 + p) and the information (R + 2)(R + 3) k."""
    return algorithmic_flops_block(k, 1, d, p, R)


def algorithmic_flops_block(k: int, b: int, d: int, p: int, R: int) -> int:
    """The same count for a block of b observations conditioned jointly
    (grouped Vecchia; k = conditioning set + b): the terms that act on the
    self vector u (its back solve, the per-range products and solves, the
    nugget solve, the residual derivatives and the information) are needed
    once per block member."""
    return int(k * (k - 1) // 2 * (3 * d + 2) + k ** 3 / 3 + (1 + p) * k * k + b * k * k
               + R * (3 * k * (k + 1) // 2 + 3 * b * k * k) + b * k * k
               + b * (R + 2) * 2 * k * (1 + p) + b * (R + 2) * (R + 3) * k)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic():
    """HBM bytes per launch of the fused kernel from the committed counter
    summary, if it was taken on the current kernel source."""
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    fields = dict(re.findall(r"^([a-z_0-9]+):\s*(\S+)\s*$", text, flags=re.M))
    if fields.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_cpu():
    """(CPU model, logical CPUs the OS reports, threads this job may use).
    The oracle's all-core leg uses the CPUs this process may run on, at most
    16 (the host share of one GPU)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, os.cpu_count() or 1, max(1, min(16, avail))


def oracle_baseline(w, sample_all: int, sample_one: int, what: str) -> dict:
    """The CPU oracle timed on the last `sample_all` neighbourhoods with every
    thread this job may use and on the last `sample_one` with one thread
    (the paper's 1-core / multi-core framing of its CPU baseline)."""
    import oracle

    oracle.build()
    model, nproc, threads = host_cpu()
    n = w["n"]
    rates = {}
    for nt, S_ in ((threads, min(sample_all, n)), (1, min(sample_one, n))):
        log(f"CPU oracle on observations [{n - S_}, {n}) with {nt} thread(s)")
        tc = time.perf_counter()
        oracle.raw_sums(w["locs"], w["NN"], w["y"], w["X"], w["covparms"], w["family"], w["nu"],
                        w["nspace"], i0=n - S_, i1=n, threads=nt)
        rates[nt] = (S_ / (time.perf_counter() - tc), S_, time.perf_counter() - tc)
        log(f"CPU oracle, {nt} thread(s): {rates[nt][0]:.4e} nbhd/s")
    v, S_all, t_all = rates[threads]
    v1, S_one, t_one = rates[1]
    return {"value": v, "unit": "neighbourhoods/s", "cores": threads, "kind": "oracle",
            "sample": f"last {S_all} of {n} neighbourhoods ({what}) on {threads} threads, "
                      f"{t_all:.2f} s wall; last {S_one} on 1 thread, {t_one:.2f} s wall",
            "value_1core": v1, "nproc": nproc, "cpu_model": model}


def calibration_kernel():
    """A kernel of known HBM traffic for scaling the FETCH_SIZE / WRITE_SIZE
    counters: an in-place multiply of 512 MiB reads and writes 512 MiB."""
    import torch

    x = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
    for _ in range(2):
        x.mul_(0.5)
    torch.cuda.synchronize()
    log("calibration: 2 x in-place multiply of 536870912 bytes")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--cpu-sample", type=int, default=524_288)
    ap.add_argument("--cpu-sample-1core", type=int, default=65_536)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibration", action="store_true",
                    help="also run a kernel of known traffic (512 MiB read + 512 MiB write) "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--workload", default="satellite_spacetime",
                    choices=["satellite_spacetime", "batched_uneven", "surrogate_plane",
                             "sweep", "predict", "neighbours", "attributes_18d",
                             "grouped_plane", "pipeline"])
    ap.add_argument("--sweep-sizes", default="32768,131072,524288,2097152,4194304",
                    help="sweep workload: comma-separated n values")
    ap.add_argument("--sweep-ms", default="10,30,40,60", help="sweep workload: comma-separated m")
    ap.add_argument("--train-neighbourhoods", type=int, default=10_000_000)
    ap.add_argument("--epochs", type=int, default=2)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; run with --gpus 1"}))
        sys.exit(2)
    if args.workload == "batched_uneven":
        return bench_batched(args)
    if args.workload == "surrogate_plane":
        return bench_surrogate(args)
    if args.workload == "sweep":
        return bench_sweep(args)
    if args.workload == "predict":
        return bench_predict(args)
    if args.workload == "neighbours":
        return bench_neighbours(args)
    if args.workload == "attributes_18d":
        return bench_attributes(args)
    if args.workload == "grouped_plane":
        return bench_grouped(args)
    if args.workload == "pipeline":
        return bench_pipeline(args)

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

    # the other passes of the fused kernel on the same workload: the
    # reverse-mode gradient (adjoint, at the GLS estimate) and the loglik-only
    # forward that the autograd function pairs it with
    beta = torch.as_tensor(res["betahat"], dtype=torch.float64, device="cuda")
    passes = {}
    for name, fn in (("adjoint", lambda: ev.loglik_adjoint(cp, beta, check=False)),
                     ("loglik_only", lambda: ev.loglik(cp, check=False))):
        with torch.cuda.stream(stream):
            fn()
            a0 = torch.cuda.Event(enable_timing=True)
            a1 = torch.cuda.Event(enable_timing=True)
            a0.record(stream)
            for _ in range(args.kernel_reps):
                fn()
            a1.record(stream)
        torch.cuda.synchronize()
        passes[name] = a0.elapsed_time(a1) / args.kernel_reps
        log(f"{name} pass {passes[name]:.4f} ms ({n / (passes[name] * 1e-3):.4e} nbhd/s)")
    ev.check_status("adjoint and loglik-only passes")

    if args.calibration:
        calibration_kernel()

    cpu = None
    if not args.no_cpu:
        cpu = oracle_baseline(w, args.cpu_sample, args.cpu_sample_1core,
                              "m=30, same workload")

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
                     "traffic": profiled_traffic()},
        "cpu_baseline": cpu,
        "detail": {"kernel": "sums_kernel<31,1,2,0,false>", "kernel_ms": kernel_ms,
                   "flop_per_neighbourhood": F, "loglik": res["loglik"],
                   "adjoint_pass_ms": passes["adjoint"], "loglik_only_pass_ms": passes["loglik_only"],
                   "kernel_source_sha256_16": kernel_source_hash()},
    }
    print(json.dumps(line), flush=True)


def bench_batched(args):
    import numpy as np
    import torch

    import paper_2407_02740_amd.autotune as AT
    from paper_2407_02740_amd import synthetic as S
    from paper_2407_02740_amd import vecchia as V

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    log("generating 512 uneven datasets")
    w = S.batched_uneven()
    ntot = int(w["n"].sum())
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s: {ntot} observations")
    start = w["covparms"] * np.array([0.8, 1.3, 1.5])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        vb = V.VecchiaBatch(w["locs"], w["NN"], w["y"], w["X"], w["obs_offset"], w["nn_offset"],
                            w["n"], w["m"], w["nu"], w["family"], w["nspace"])
        cp = vb.covparms(start)
        sched, table = AT.tune_batch(vb, cp, log=log)
    torch.cuda.synchronize()
    log(f"schedule: tile {list(sched.tile)}, blocks/CU {list(sched.blocks_per_cu)}")
    with torch.cuda.stream(stream):
        vb.fisher_fit(cp, args.warmup, use_graph=True, check=False)
    torch.cuda.synchronize()
    vb.check_status("warmup")
    t1 = time.perf_counter()
    with torch.cuda.stream(stream):
        vb.fisher_fit(cp, args.steps, use_graph=True, check=False)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    vb.check_status("timed steps")
    elapsed = t2 - t1
    value = ntot * args.steps / elapsed
    log(f"{args.steps} steps in {elapsed * 1e3:.2f} ms -> {value:.4e} nbhd/s")
    # per class: algorithmic flops over the best measured time of its launch
    classes = {}
    for c, rows in table.items():
        sel = [b for b in range(w["nsets"]) if min(k for k, K in enumerate(V.CLASS_K)
                                                   if w["m"][b] + 1 <= K) == c]
        flops = sum(int(w["n"][b]) * algorithmic_flops(int(w["m"][b]) + 1, 2, 1, 1) for b in sel)
        ms = min(r[2] for r in rows)
        classes[V.CLASS_K[c]] = dict(datasets=len(sel), ms=ms, tflops=flops / (ms * 1e-3) / 1e12)
    dom = max(classes, key=lambda k: classes[k]["ms"])
    achieved = classes[dom]["tflops"]
    cpu = None
    if not args.no_cpu:
        import oracle

        oracle.build()
        threads = min(16, os.cpu_count() or 1)
        picks = [int(np.flatnonzero(w["m"] == m)[0]) for m in (10, 20, 30, 40)]
        tc = time.perf_counter()
        nn = 0
        for b in picks:
            d = S.batch_member(w, b)
            oracle.raw_sums(d["locs"], d["NN"], d["y"], d["X"], d["covparms"], d["family"],
                            d["nu"], d["nspace"], threads=threads)
            nn += d["n"]
        dtc = time.perf_counter() - tc
        cpu = {"value": nn / dtc, "unit": "neighbourhoods/s", "cores": threads, "kind": "oracle",
               "sample": f"one dataset of each m in 10/20/30/40 ({nn} neighbourhoods), "
                         f"{dtc:.2f} s wall"}
        log(f"CPU oracle {cpu['value']:.4e} nbhd/s")
    line = {
        "metric": METRIC_BATCHED, "value": value, "unit": "neighbourhoods/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "batched_uneven", "datasets": int(w["nsets"]),
                   "neighbourhoods": ntot, "m": [10, 20, 30, 40], "d": 2, "p": 1,
                   "covariance": "Matern nu in {0.5, 1.5, 2.5} (sigma2, rho, tau2) per dataset",
                   "step": "Fisher-scoring iteration of every dataset: persistent class "
                           "launches + per-dataset reduce + combine + update, HIP graph replay"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR_TFLOPS,
                     "traffic": None},
        "cpu_baseline": cpu,
        "detail": {"dominant_kernel": f"sums_kernel<{dom},1,1,0,true>", "classes": classes,
                   "schedule": {"tile": list(sched.tile),
                                "blocks_per_cu": list(sched.blocks_per_cu)}},
    }
    print(json.dumps(line), flush=True)


def bench_surrogate(args):
    import numpy as np
    import torch

    from paper_2407_02740_amd import surrogate as SG
    from paper_2407_02740_amd import synthetic as S
    from paper_2407_02740_amd import vecchia as V

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    log(f"training set: {args.train_neighbourhoods} neighbourhoods from the exact kernel")
    x, raw, dist = SG.training_set(args.train_neighbourhoods, seed=6, log=log)
    lv = raw[:, SG.M]
    shift, scale = float(lv.mean()), float(lv.std())
    t = SG.targets_of(raw, shift, scale)
    del raw
    log(f"training set ready in {time.perf_counter() - t0:.1f} s: {x.shape[0]} rows, "
        f"offset lengths [{dist[0]:.4g}, {dist[1]:.4g}]")
    mlp = SG.MLP(seed=0, lv_shift=shift, lv_scale=scale)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hist = SG.train(mlp, x, t, epochs=args.epochs, batch=4096, lr=2e-3, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    del x, t
    log(f"trained {args.epochs} epochs in {train_s:.1f} s, loss {hist[-1]:.4e}")
    # gate calibrated on a held-out problem of the same shape, then applied
    cal_w = S.surrogate_plane(seed=55, n=262_144)
    cal_ev = V.Vecchia(cal_w["locs"], cal_w["NN"], cal_w["y"], cal_w["X"], V.FAMILY_ISO, 1.5, 0)
    cp = np.array(cal_w["covparms"])
    cal = SG.calibrate_floor(cal_ev, mlp, dist, cp, bound=1e-6)
    for row in cal["sweep"]:
        log(f"calibration floor {row['floor']:.3g}: |dloglik|/n {row['err']:.3e}, served "
            f"{row['served']} of {cal_ev.n}")
    floor = cal["chosen"]["floor"]
    del cal_ev
    log("generating the evaluation problem (n = 4,194,304, m = 30)")
    w = S.surrogate_plane(log=log)
    n = w["n"]
    ev = V.Vecchia(w["locs"], w["NN"], w["y"], w["X"], V.FAMILY_ISO, 1.5, 0)
    gated = SG.SurrogateLoglik(ev, mlp, dist, lv_floor=floor)
    served_all = SG.SurrogateLoglik(ev, mlp, dist, lv_slack=50.0)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - a) / reps

    ex, t_exact = timed(lambda: SG.exact_loglik(ev, cp), args.steps)
    rg, t_gate = timed(lambda: gated.evaluate(cp), args.steps)
    ra, t_all = timed(lambda: served_all.evaluate(cp), args.steps)
    err_g = abs(rg["loglik"] - ex["loglik"]) / n
    err_a = abs(ra["loglik"] - ex["loglik"]) / n
    log(f"exact {n / t_exact:.4e} nbhd/s; gated {n / t_gate:.4e} nbhd/s, served "
        f"{rg['served']}, |dloglik|/n {err_g:.3e}; served-all {n / t_all:.4e} nbhd/s, "
        f"|dloglik|/n {err_a:.3e}")
    # the network pass alone over one chunk (HIP events on the current stream)
    rows = served_all.chunk
    feat, _ = SG.features(ev, cp, 0, rows, 0.0, 1e30)
    mlp.forward(feat)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        mlp.forward(feat)
    e1.record()
    torch.cuda.synchronize()
    mlp_ms = e0.elapsed_time(e1) / 5
    macs = 64 * 256 + 2 * 256 * 256 + 256 * 32
    achieved = 2.0 * macs * rows / (mlp_ms * 1e-3) / 1e12
    cpu = None
    if not args.no_cpu:
        import oracle

        oracle.build()
        threads = min(16, os.cpu_count() or 1)
        S_ = min(args.cpu_sample, n)
        tc = time.perf_counter()
        oracle.raw_sums(w["locs"], w["NN"], w["y"], w["X"], w["covparms"], w["family"], w["nu"],
                        w["nspace"], i0=n - S_, i1=n, threads=threads)
        dtc = time.perf_counter() - tc
        cpu = {"value": S_ / dtc, "unit": "neighbourhoods/s", "cores": threads, "kind": "oracle",
               "sample": f"last {S_} of {n} neighbourhoods (loglik, gradient and Fisher sums), "
                         f"{dtc:.2f} s wall"}
    line = {
        "metric": METRIC_SURROGATE, "value": n / t_gate, "unit": "neighbourhoods/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": 1e3 * t_gate,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16/f32 network + f64 loglik", "data": "synthetic",
        "config": {"workload": "surrogate_plane", "n": n, "m": 30, "d": 2, "p": 1,
                   "covariance": "Matern 3/2 (1.0, 0.05, 0.05)",
                   "step": "features + network + FP64 sums + exact hand-back + combine",
                   "training": {"neighbourhoods": int(args.train_neighbourhoods),
                                "epochs": args.epochs, "seconds": train_s,
                                "final_loss": hist[-1]}},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_MFMA_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_BF16_MFMA_TFLOPS,
                     "traffic": None},
        "cpu_baseline": cpu,
        "detail": {"gate_floor_log_v": floor, "served": rg["served"], "dloglik_per_n": err_g,
                   "exact_loglik_only_nbhd_per_s": n / t_exact,
                   "served_all_nbhd_per_s": n / t_all, "served_all_dloglik_per_n": err_a,
                   "network_kernel_ms_per_chunk": mlp_ms, "chunk_rows": rows,
                   "calibration": cal["sweep"]},
    }
    print(json.dumps(line), flush=True)


def bench_sweep(args):
    """Throughput over problem sizes and neighbour counts, the grid of the
    paper's size study (n = 2^15 .. 2^22, m = 10, 30, 60; plus m = 40): 2-D
    Matern 3/2 (1.0, 0.05, 0.05), loglik + gradient + Fisher; kernel-only
    time (HIP events, median of the repetitions) and end-to-end time from host
    arrays (host-to-device copies, evaluation, result back on the host).
    Points uniform on the unit square in the coarse-to-fine order, the
    neighbour arrays from the library's own search (m = 60, columns cut for
    smaller m), y a random-Fourier-feature draw plus nugget."""
    import statistics

    import numpy as np
    import torch

    from paper_2407_02740_amd import synthetic as S
    from paper_2407_02740_amd import vecchia as V

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    rows = []
    cp = np.array((1.0, 0.05, 0.05))
    sizes = [int(v) for v in args.sweep_sizes.split(",")]
    ms = [int(v) for v in args.sweep_ms.split(",")]
    assert max(ms) <= 60, "the sweep's neighbour arrays hold 60 neighbours"
    for n in sizes:
        rng = np.random.default_rng(7)
        locs = rng.random((n, 2))
        locs = np.ascontiguousarray(locs[S.maxmin_approx(locs, 7)])
        NN60 = V.ordered_nn(torch.as_tensor(locs, device="cuda"), 60).cpu().numpy()
        y = S.rff_field(locs / cp[1], 1.5, 128, rng) + np.sqrt(cp[2]) * rng.standard_normal(n)
        X = np.ones((n, 1))
        for m in ms:
            NN = np.ascontiguousarray(NN60[:, :m + 1])
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                ev = V.Vecchia(locs, NN, y, X, V.FAMILY_ISO, 1.5, 0)
                cpd = ev.covparms(cp)
                ev.loglik_grad_info(cpd, check=False)
                times = []
                for _ in range(max(5, args.steps)):
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    ev.loglik_grad_info(cpd, check=False)
                    e1.record(stream)
                    e1.synchronize()
                    times.append(e0.elapsed_time(e1))
            ev.check_status("sweep")
            kern = statistics.median(times)
            del ev
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            with torch.cuda.stream(stream):
                ev2 = V.Vecchia(locs, NN, y, X, V.FAMILY_ISO, 1.5, 0)
                out = ev2.loglik_grad_info(ev2.covparms(cp), check=False).cpu()
            e2e = (time.perf_counter() - t0) * 1e3
            del ev2
            F = algorithmic_flops(m + 1, 2, 1, 1)
            row = dict(n=n, m=m, kernel_ms=kern, nbhd_per_s=n / (kern * 1e-3), end_to_end_ms=e2e,
                       end_to_end_nbhd_per_s=n / (e2e * 1e-3), loglik=float(out[0]),
                       kernel="fused" if m + 1 <= 61 else "wave", flop_per_neighbourhood=F,
                       fp64_frac=F * n / (kern * 1e-3) / 78.6e12)
            rows.append(row)
            log(f"n={n} m={m}: {kern:.3f} ms ({row['nbhd_per_s']:.3e} nbhd/s, "
                f"{100 * row['fp64_frac']:.1f} % of FP64 peak), end to end {e2e:.1f} ms")
    line = {"metric": "neighbourhoods/s (loglik+grad+Fisher) over n and m, 2-D Matern 3/2",
            "value": None, "unit": "neighbourhoods/s", "n_gpus": 1, "steps": args.steps,
            "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "sweep"}, "roofline": None, "cpu_baseline": None,
            "detail": {"rows": rows}}
    print(json.dumps(line), flush=True)


def bench_predict(args):
    """Kriging prediction with 60 observed neighbours (the paper's Table 3
    setting) on the Matern plane (262,144 points, Matern 3/2, p = 3).

    Hold-out check: a random 10 % of the points is held out, the model is
    fitted to the other 90 % (re-ordered coarse to fine, m = 30, 20
    Fisher-scoring iterations on the device from a start off the truth) and
    the held-out responses are predicted from their 60 nearest training
    points; the line reports the RMSE against the held-out values beside that
    of the training mean.  Throughput: 262,144 new points predicted from
    their 60 nearest of all 262,144 observations (weights pass + mean kernel,
    HIP events, median of the repetitions)."""
    import statistics

    import numpy as np
    import torch

    from paper_2407_02740_amd import synthetic as S
    from paper_2407_02740_amd import vecchia as V

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    mp = 60
    w = S.matern_plane()
    n = w["n"]
    rng = np.random.default_rng(12)

    # ---- 90/10 hold-out split
    test = np.zeros(n, dtype=bool)
    test[rng.choice(n, n // 10, replace=False)] = True
    tr = np.flatnonzero(~test)
    te = np.flatnonzero(test)
    ltr = w["locs"][tr]
    otr = S.maxmin_approx(ltr, 12)
    ltr, ytr, Xtr = ltr[otr], w["y"][tr][otr], w["X"][tr][otr]
    NNtr = S.find_ordered_nn(ltr, 30)
    start = np.asarray(w["covparms"]) * np.array([0.7, 1.4, 2.0])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        evtr = V.Vecchia(ltr, NNtr, ytr, Xtr, w["family"], w["nu"], 0)
        cpt = evtr.covparms(start)
        evtr.fisher_fit(cpt, 20, use_graph=True)
        beta_t = evtr.loglik(cpt)[1:4].clone()
        NNte = S.nn_among(ltr, w["locs"][te], mp)
        mean_te, _ = V.Predictor(evtr, w["locs"][te], w["X"][te], NNte).predict(cpt, beta_t)
    torch.cuda.synchronize()
    evtr.check_status("hold-out fit")
    err = mean_te.cpu().numpy() - w["y"][te]
    rmse = float(np.sqrt(np.mean(err ** 2)))
    rmse_mean = float(np.sqrt(np.mean((w["y"][te] - ytr.mean()) ** 2)))
    theta_hat = cpt.cpu().numpy()
    log(f"hold-out: {len(te)} points, RMSE {rmse:.5f} (training mean {rmse_mean:.5f}), "
        f"theta {theta_hat}")
    del evtr

    # ---- throughput at 60 neighbours
    npred = 262_144
    lp = rng.random((npred, 2))
    Xp = np.column_stack([np.ones(npred), lp[:, 0], lp[:, 1]])
    NNp = S.nn_among(w["locs"], lp, mp)
    with torch.cuda.stream(stream):
        ev = V.Vecchia(w["locs"], w["NN"], w["y"], w["X"], w["family"], w["nu"], 0)
        cp = ev.covparms(w["covparms"])
        beta = ev.loglik(cp)[1:4].clone()
        pr = V.Predictor(ev, lp, Xp, NNp)
        pr.predict(cp, beta)
        times = []
        for _ in range(max(5, args.steps)):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            mean, var = pr.predict(cp, beta, check=False)
            e1.record(stream)
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
    ev.check_status("predict")
    ms = statistics.median(times)
    log(f"{npred} predictions from {mp} neighbours in {ms:.3f} ms")
    line = {"metric": f"kriging predictions/s (m={mp} observed neighbours), Matern plane",
            "value": npred / (ms * 1e-3), "unit": "predictions/s", "n_gpus": 1,
            "steps": len(times), "warmup": 1, "ms_per_step": ms, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "predict", "n_obs": n, "n_pred": npred, "m": mp},
            "roofline": None, "cpu_baseline": None,
            "detail": {"holdout_points": int(len(te)), "holdout_rmse": rmse,
                       "holdout_rmse_training_mean": rmse_mean,
                       "fitted_theta": theta_hat.tolist(), "true_theta": list(w["covparms"]),
                       "mean_of_means": float(mean.mean()), "mean_var": float(var.mean())}}
    print(json.dumps(line), flush=True)


def bench_neighbours(args):
    """Preparation of the hot path's inputs on the device: coarse-to-fine
    ordering of n = 1,048,576 uniform 2-D points and the search of their m =
    30 nearest previously ordered neighbours (the NNarray), against the same
    two steps on the host (input module: numpy ordering, k-d tree search)."""
    import statistics

    import numpy as np
    import torch

    from paper_2407_02740_amd import synthetic as S
    from paper_2407_02740_amd import vecchia as V

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    n, m = 1 << 20, 30
    rng = np.random.default_rng(13)
    locs = rng.random((n, 2))
    tie = rng.random(n)
    x = torch.as_tensor(locs, device="cuda")
    t = torch.as_tensor(tie, device="cuda")
    V.ordered_nn(V.maxmin_order(x, t)[1], m)
    torch.cuda.synchronize()
    t_ord, t_nn, t_all = [], [], []
    for _ in range(max(3, args.steps)):
        t0 = time.perf_counter()
        order, xo = V.maxmin_order(x, t)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        NN = V.ordered_nn(xo, m)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        t_ord.append(t1 - t0)
        t_nn.append(t2 - t1)
        t_all.append(t2 - t0)
    t_gpu = statistics.median(t_all)
    log(f"device ordering {statistics.median(t_ord) * 1e3:.2f} ms, "
        f"search {statistics.median(t_nn) * 1e3:.2f} ms")
    cpu, detail = None, {"ordering_ms": 1e3 * statistics.median(t_ord),
                         "search_ms": 1e3 * statistics.median(t_nn)}
    if not args.no_cpu:
        threads = min(16, os.cpu_count() or 1)
        tc = time.perf_counter()
        ref_order = S.maxmin_approx(locs, tie=tie)
        tm = time.perf_counter()
        ref = S.find_ordered_nn(locs[ref_order], m, workers=threads)
        t_cpu = time.perf_counter() - tc
        assert np.array_equal(ref_order, order.cpu().numpy()), "device and host orderings differ"
        assert np.array_equal(ref, NN.cpu().numpy()), "device and host searches differ"
        cpu = {"value": n / t_cpu, "unit": "points/s", "cores": threads,
               "kind": "host ordering (numpy) and k-d tree search (scipy cKDTree)",
               "sample": f"all {n} points, {t_cpu:.2f} s wall"}
        detail.update(host_ordering_s=tm - tc, host_search_s=t_cpu - (tm - tc))
        log(f"host ordering {tm - tc:.2f} s, search {t_cpu - (tm - tc):.2f} s")
    line = {"metric": "points/s, ordering + ordered nearest-neighbour search (n=1M, m=30, 2-D)",
            "value": n / t_gpu, "unit": "points/s", "n_gpus": 1, "steps": len(t_all),
            "warmup": 1, "ms_per_step": 1e3 * t_gpu, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "neighbours", "n": n, "m": m, "d": 2}, "roofline": None,
            "cpu_baseline": cpu, "detail": detail}
    print(json.dumps(line), flush=True)


def bench_attributes(args):
    """Fisher scoring with one range per coordinate on the 18-attribute
    regression workload (n = 14,939, m = 30, P = 20): the wave-per-
    neighbourhood kernel + reduce + combine + update, HIP graph replay."""
    import numpy as np
    import torch

    from paper_2407_02740_amd import synthetic as S
    from paper_2407_02740_amd import vecchia as V

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    w = S.attributes_18d()
    n, m, d, p = w["n"], w["m"], w["d"], w["p"]
    start = w["covparms"] * np.r_[0.7, np.full(d, 1.3), 1.5]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ev = V.Vecchia(w["locs"], w["NN"], w["y"], w["X"], w["family"], w["nu"])
        cp = ev.covparms(start)
        ev.workspace()
        ev.fisher_fit(cp, args.warmup, use_graph=True, check=False)
    torch.cuda.synchronize()
    ev.check_status("warmup")
    t1 = time.perf_counter()
    with torch.cuda.stream(stream):
        ev.fisher_fit(cp, args.steps, use_graph=True, check=False)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    ev.check_status("timed steps")
    value = n * args.steps / elapsed
    # a whole fit of 40 iterations from the same start, inputs resident
    with torch.cuda.stream(stream):
        cp40 = ev.covparms(start)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    with torch.cuda.stream(stream):
        ev.fisher_fit(cp40, 40, use_graph=True, check=False)
    torch.cuda.synchronize()
    fit40 = time.perf_counter() - t3
    ev.check_status("40-iteration fit")
    with torch.cuda.stream(stream):
        ev.block_sums(cp)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.kernel_reps):
            ev.block_sums(cp)
        e1.record(stream)
    torch.cuda.synchronize()
    kernel_ms = e0.elapsed_time(e1) / args.kernel_reps
    F = algorithmic_flops(m + 1, d, p, d)
    achieved = F * n / (kernel_ms * 1e-3) / 1e12
    log(f"{args.steps} steps {elapsed * 1e3:.2f} ms; kernel {kernel_ms:.4f} ms, {F} flop/nbhd "
        f"-> {achieved:.2f} TFLOP/s; 40-iteration fit {fit40 * 1e3:.1f} ms")
    cpu = None
    if not args.no_cpu:
        import oracle

        oracle.build()
        threads = min(16, os.cpu_count() or 1)
        tc = time.perf_counter()
        oracle.raw_sums(w["locs"], w["NN"], w["y"], w["X"], w["covparms"], w["family"], w["nu"],
                        threads=threads)
        dtc = time.perf_counter() - tc
        cpu = {"value": n / dtc, "unit": "neighbourhoods/s", "cores": threads, "kind": "oracle",
               "sample": f"all {n} neighbourhoods of the workload, {dtc:.2f} s wall"}
    res = V.unpack_out(ev.out, p, ev.P)
    # the neighbour arrays of this workload on the device (exhaustive search
    # in 18 range-scaled coordinates) against the host k-d tree search
    scaled = torch.as_tensor(w["locs"] / w["covparms"][1:-1], device="cuda")
    V.ordered_nn(scaled, m)
    torch.cuda.synchronize()
    tn = time.perf_counter()
    NNd = V.ordered_nn(scaled, m)
    torch.cuda.synchronize()
    nn_ms = 1e3 * (time.perf_counter() - tn)
    th = time.perf_counter()
    NNh = S.find_ordered_nn(w["locs"] / w["covparms"][1:-1], m, workers=min(16, os.cpu_count() or 1))
    nn_host_ms = 1e3 * (time.perf_counter() - th)
    assert np.array_equal(NNd.cpu().numpy(), NNh), "device and host neighbour arrays differ"
    log(f"neighbours: device {nn_ms:.2f} ms, host {nn_host_ms:.1f} ms")
    line = {
        "metric": "neighbourhoods/s (loglik+grad+Fisher), 18 attributes with one range each, "
                  "n=14939 m=30",
        "value": value, "unit": "neighbourhoods/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "attributes_18d", "n": n, "m": m, "d": d, "p": p,
                   "covariance": "exponential, one range per attribute (sigma2, rho_1..rho_18, "
                                 "tau2), P = 20",
                   "step": "Fisher-scoring iteration: sums + reduce + combine + update, HIP "
                           "graph replay"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR_TFLOPS,
                     "traffic": None},
        "cpu_baseline": cpu,
        "detail": {"kernel": f"wave_kernel<{32 if m + 1 <= 32 else 64}, 20, 1>", "kernel_ms": kernel_ms,
                   "flop_per_neighbourhood": F, "fit_40_iterations_ms": 1e3 * fit40,
                   "loglik": res["loglik"], "neighbours_device_ms": nn_ms,
                   "neighbours_host_ms": nn_host_ms},
    }
    print(json.dumps(line), flush=True)


def bench_grouped(args):
    """Grouped Vecchia on a Terra-sized plane: n = 262,144 uniform 2-D points,
    Matern 3/2 (1.0, 0.05, 0.05), blocks of <= 4 nearby points conditioning
    on the m = 30 earlier points nearest to any member; one Fisher-scoring
    step of the grouped likelihood (wave kernel + reduce + combine + update,
    HIP graph), beside the ungrouped step on the same points (maxmin order,
    m = 30)."""
    import numpy as np
    import torch

    from paper_2407_02740_amd import synthetic as S
    from paper_2407_02740_amd import vecchia as V

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    n, m, g = 262_144, 30, 4
    rng = np.random.default_rng(21)
    locs = rng.random((n, 2))
    cp0 = np.array((1.0, 0.05, 0.05))
    tg = time.perf_counter()
    order, bs, cs, cond = S.group_cells(locs, g, m, seed=21)
    log(f"grouping {time.perf_counter() - tg:.1f} s: {len(bs) - 1} blocks")
    pts = locs[order]
    f = S.rff_field(pts / cp0[1], 1.5, 512, rng)
    y = f + np.sqrt(cp0[2]) * rng.standard_normal(n)
    X = np.ones((n, 1))
    start = cp0 * np.array([0.7, 1.3, 1.5])
    stream = torch.cuda.Stream()

    def timed(ev):
        with torch.cuda.stream(stream):
            cp = ev.covparms(start)
            ev.workspace()
            ev.fisher_fit(cp, args.warmup, use_graph=True, check=False)
        torch.cuda.synchronize()
        ev.check_status("warmup")
        t1 = time.perf_counter()
        with torch.cuda.stream(stream):
            ev.fisher_fit(cp, args.steps, use_graph=True, check=False)
        torch.cuda.synchronize()
        ev.check_status("timed")
        return (time.perf_counter() - t1) / args.steps, V.unpack_out(ev.out, 1, 3)

    with torch.cuda.stream(stream):
        evg = V.GroupedVecchia(pts, y, X, bs, cs, cond, V.FAMILY_ISO, 1.5)
    tgs, resg = timed(evg)
    o2 = S.maxmin_approx(locs, 21)
    p2 = locs[o2]
    NN = S.find_ordered_nn(p2, m)
    f2 = S.rff_field(p2 / cp0[1], 1.5, 512, np.random.default_rng(22))
    y2 = f2 + np.sqrt(cp0[2]) * np.random.default_rng(23).standard_normal(n)
    with torch.cuda.stream(stream):
        evs = V.Vecchia(p2, NN, y2, X, V.FAMILY_ISO, 1.5)
    tss, _ = timed(evs)
    log(f"grouped step {tgs * 1e3:.3f} ms, ungrouped step {tss * 1e3:.3f} ms")
    # the grouped sums alone (wave kernel and its device reduction), HIP
    # events on their stream; algorithmic flops summed over the blocks
    with torch.cuda.stream(stream):
        cpg = evg.covparms(cp0)
        evg.raw_sums(cpg, check=False)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.kernel_reps):
            evg.raw_sums(cpg, check=False)
        e1.record(stream)
    torch.cuda.synchronize()
    evg.check_status("kernel timing")
    kernel_ms = e0.elapsed_time(e1) / args.kernel_reps
    bsz = np.diff(np.asarray(bs, dtype=np.int64))
    ksz = np.diff(np.asarray(cs, dtype=np.int64)) + bsz
    F = sum(algorithmic_flops_block(int(k), int(b), 2, 1, 1) for k, b in zip(ksz, bsz))
    achieved = F / (kernel_ms * 1e-3) / 1e12
    log(f"grouped sums {kernel_ms:.4f} ms, {F:.4e} flop -> {achieved:.2f} TFLOP/s")
    line = {
        "metric": "observations/s (grouped loglik+grad+Fisher), n=262144, blocks <= 4, m=30",
        "value": n / tgs, "unit": "observations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * tgs, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "grouped_plane", "n": n, "m": m, "max_block": g,
                   "blocks": int(len(bs) - 1), "covariance": "Matern 3/2 (1.0, 0.05, 0.05)",
                   "step": "Fisher-scoring iteration of the grouped likelihood, HIP graph"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR_TFLOPS,
                     "traffic": None},
        "cpu_baseline": None,
        "detail": {"ungrouped_step_ms": 1e3 * tss, "ungrouped_obs_per_s": n / tss,
                   "grouped_loglik": resg["loglik"], "grouped_sums_ms": kernel_ms,
                   "flop_per_step": F},
    }
    print(json.dumps(line), flush=True)


def bench_pipeline(args):
    """From raw points to a fitted model on the device: the satellite
    space-time points (n = 1,048,576) in acquisition order are ordered
    coarse to fine in range-scaled coordinates, their m = 30 ordered
    neighbours found, and 20 Fisher-scoring iterations run (HIP graph).
    The host preparation (numpy ordering, k-d tree search) is timed beside
    it; inputs start resident in device memory."""
    import numpy as np
    import torch

    from paper_2407_02740_amd import synthetic as S
    from paper_2407_02740_amd import vecchia as V

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    m, iters = 30, 20
    rng = np.random.default_rng(3)
    lon, lat, t = S.satellite_tracks(64, 64, 256, rng)
    la, lo = np.radians(lat), np.radians(lon)
    xyz = np.column_stack([np.cos(la) * np.cos(lo), np.cos(la) * np.sin(lo), np.sin(la)])
    locs = np.ascontiguousarray(np.column_stack([xyz, t]))
    n = len(locs)
    cp = np.array((1.0, S.RHO_SPACE_5DEG, 3.0, 0.1))
    scaled = np.ascontiguousarray(np.column_stack([xyz / cp[1], t / cp[2]]))
    y = 0.5 + S.rff_field(scaled, 0.5, 512, rng) + np.sqrt(cp[3]) * rng.standard_normal(n)
    tie = rng.random(n)
    start = cp * np.array([0.7, 1.3, 0.8, 1.5])
    dev = "cuda"
    d_locs, d_scaled = torch.as_tensor(locs, device=dev), torch.as_tensor(scaled, device=dev)
    d_y, d_tie = torch.as_tensor(y, device=dev), torch.as_tensor(tie, device=dev)
    X = torch.ones(n, 1, dtype=torch.float64, device=dev)

    def run():
        t0 = time.perf_counter()
        order, sc = V.maxmin_order(d_scaled, d_tie)
        NN = V.ordered_nn(sc, m)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ev = V.Vecchia(d_locs.index_select(0, order), NN, d_y.index_select(0, order), X,
                       V.FAMILY_SPACETIME, 0.5, 3)
        th = ev.covparms(start)
        ev.fisher_fit(th, iters, use_graph=True, check=False)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ev.check_status("pipeline")
        return t1 - t0, t2 - t1, th.cpu().numpy(), ev

    run()
    prep, fit, theta, ev = run()
    res = V.unpack_out(ev.out, 1, 4)
    log(f"device: preparation {prep * 1e3:.1f} ms, 20 iterations {fit * 1e3:.1f} ms; theta {theta}")
    cpu = None
    if not args.no_cpu:
        th0 = time.perf_counter()
        o = S.maxmin_approx(scaled, tie=tie)
        S.find_ordered_nn(scaled[o], m, workers=min(16, os.cpu_count() or 1))
        host = time.perf_counter() - th0
        cpu = {"value": host, "unit": "s", "cores": min(16, os.cpu_count() or 1),
               "kind": "host preparation only (numpy ordering, scipy k-d tree search)",
               "sample": f"all {n} points"}
        log(f"host preparation {host:.2f} s")
    total = prep + fit
    line = {"metric": "seconds from raw points to 20 Fisher-scoring iterations (ordering, "
                      "neighbours, fit), space-time n=1M m=30",
            "value": total, "unit": "s", "n_gpus": 1, "steps": iters, "warmup": 1,
            "ms_per_step": 1e3 * fit / iters, "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "pipeline", "n": n, "m": m, "d": 4,
                       "covariance": "space-time exponential (sigma2, rho_s, rho_t, tau2)"},
            "roofline": None, "cpu_baseline": cpu,
            "detail": {"preparation_ms": 1e3 * prep, "fit_ms": 1e3 * fit, "loglik": res["loglik"],
                       "theta": [float(v) for v in theta]}}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
