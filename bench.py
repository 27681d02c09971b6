#!/usr/bin/env python3
"""Throughput of the stochastic relativistic MP2 hot path on one MI355X.

One step = one Metropolis move of all m walker pairs + inverse-CDF tau
samples + one evaluation of the redundant-walker estimator (spinor values,
G-/G+ for every walker pair, direct/exchange contraction, compensated sums),
all on the GPU through libmcmp2.  Inputs are synthetic and seeded (see synth/).

Prints one JSON line: MC steps/s, variance x time of the per-step estimates
(blocking with N_b = 100), the roofline position of the dominant kernel
(Green's-function GEMM + contraction, timed with HIP events on the stream it
runs on) and the FP64 CPU oracle timed on a bounded sample of the same
workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MC steps/s and var×time for E2(+grad), FP32/BF16 vs FP64, 1 MI355X"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0}
WORKLOADS = {
    "C1": "plain FP64: 3 nuclei (triangle, 4.894 bohr), 200 L / 460 S Cartesian primitives, "
          "40 occupied / 300 virtual spinors, m=128 walker pairs, 2 tau per step",
    "C0": "tiny FP64: 2 nuclei 1.5 bohr apart, 12 L / 32 S primitives, 4 occupied / 16 virtual "
          "spinors, m=16 walker pairs, 1 tau per step",
}


def green_flops(m: int, n_sp: int, n_tau: int) -> float:
    """Algorithmic flops of G- and G+ over all walker pairs p < q for one
    launch: 8x8 complex blocks, n_sp complex multiply-adds (8 flops) each."""
    return 512.0 * (m * (m - 1) / 2.0) * n_sp * n_tau


def cpu_baseline(inp, wk0, key, delta, seconds: float):
    import numpy as np
    import torch

    from oracle.integrand import step_estimate
    from oracle.sampling import metropolis_step, sample_tau
    from oracle.weights import n_g, pair_weight, tau_lambda

    Ng = n_g(inp.nuc_xyz, inp.wfn)
    lam = tau_lambda(inp.eps, inp.n_occ)
    wk = wk0.copy()
    w = pair_weight(wk[:, 0], wk[:, 1], inp.nuc_xyz, inp.wfn, Ng)
    keyu = np.array(key, dtype=np.uint64)
    n = 0
    t0 = time.perf_counter()
    while True:
        wk, w, _ = metropolis_step(wk, w, keyu, n, delta, inp.nuc_xyz, inp.wfn, Ng)
        taus = sample_tau(keyu, n, inp.n_tau, lam)
        step_estimate(inp, wk, taus, lam, Ng)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds and n >= 2:
            break
    return {"value": n / el, "unit": "MC steps/s", "cores": int(torch.get_num_threads()), "kind": "oracle",
            "sample": f"{n} consecutive steps (Metropolis move, tau samples, estimator) of the same workload, "
                      f"{el:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--burnin", type=int, default=300, help="untimed Metropolis steps adapting delta")
    ap.add_argument("--config", default="C1", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle sample length (0: skip)")
    ap.add_argument("--no-kernel-timing", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build runs a single chain on one MI355X); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from oracle.blocking import blocking
    from paper_2203_05632_amd import Context
    from synth import initial_walkers, make_inputs

    torch.cuda.set_device(0)
    inp = make_inputs(args.config)
    ctx = Context.from_inputs(inp, precision=args.precision)
    key = (0, 0)
    wk0 = initial_walkers(inp)
    wk = torch.as_tensor(wk0, device="cuda")
    w = torch.zeros(inp.m, dtype=torch.float64, device="cuda")
    n_acc = torch.zeros(1, dtype=torch.int32, device="cuda")
    tau = torch.zeros(inp.n_tau, dtype=torch.float64, device="cuda")
    ctx.pair_weights(wk, w)

    delta = 0.5
    step = 0
    for b in range(args.burnin // 10):
        n_acc.zero_()
        for _ in range(10):
            ctx.metropolis(wk, w, key, step, delta, n_acc)
            step += 1
        rate = n_acc.item() / (10.0 * inp.m)
        delta *= 1.1 if rate > 0.5 else 0.9

    K, W = args.steps, args.warmup
    hist = torch.zeros((max(K, W), inp.n_tau, 3), dtype=torch.float64, device="cuda")

    def one(s, out):
        ctx.advance(wk, w, key, s, delta, tau, n_acc)   # Metropolis move + tau samples (one launch)
        ctx.step(wk, tau, out)                          # estimator of Eq. redundant

    for i in range(W):
        one(step, hist[i])
        step += 1
    torch.cuda.synchronize()
    if not args.no_kernel_timing:
        ctx.profile_begin(["green_contract"], K)
    t0 = time.perf_counter()
    for i in range(K):
        one(step, hist[i])
        step += 1
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = {} if args.no_kernel_timing else ctx.profile_end()

    vals = hist[:K].mean(dim=1).cpu().numpy()          # per-step estimate (mean over tau)
    ms_per_step = 1e3 * elapsed / K
    steps_per_s = K / elapsed
    var_time = None
    e2_mean = float(vals[:, 2].mean())
    if K >= 200:
        I, sbar = blocking(vals[:, 2], 100)
        var_time = sbar ** 2 * elapsed

    n_sp = inp.n_occ + inp.n_vir
    roofline = None
    if "green_contract" in prof:
        tot_ms, n_l = prof["green_contract"]
        avg_s = tot_ms / n_l / 1e3
        flops = green_flops(inp.m, n_sp, inp.n_tau)
        ach = flops / avg_s / 1e12
        peak = PEAK_TFLOPS[args.precision]
        roofline = {"bound": "mfma", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
                    "frac": round(ach / peak, 4), "traffic": None, "kernel": "green_contract",
                    "avg_us": round(avg_s * 1e6, 2), "flops_per_launch": flops}

    cpu = None
    if args.cpu_seconds > 0:
        cpu = cpu_baseline(inp, wk0, key, delta, args.cpu_seconds)
        cpu["value"] = round(cpu["value"], 4)

    out = {
        "metric": METRIC, "value": round(steps_per_s, 2), "unit": "MC steps/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.config} {WORKLOADS[args.config]}", "m": inp.m, "n_tau": inp.n_tau,
                   "n_L": inp.n_L, "n_S": inp.n_S, "n_occ": inp.n_occ, "n_vir": inp.n_vir,
                   "precision": args.precision, "grad": False},
        "var_x_time": None if var_time is None else float(f"{var_time:.6g}"),
        "var_x_time_unit": "Eh^2 s",
        "e2_mean": float(f"{e2_mean:.6g}"),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
