#!/usr/bin/env python3
"""Throughput of the stochastic relativistic MP2 hot path on one MI355X.

One step = one Metropolis move of all m walker pairs + inverse-CDF tau
samples + one evaluation of the redundant-walker estimator (spinor values,
G-/G+ for every walker pair, direct/exchange contraction, compensated sums),
all on the GPU through libmcmp2; with gradients, also the adjoint (eps and
coefficient gradients) and their compensated accumulation over steps.
Inputs are synthetic and seeded (synth/).

Prints one JSON line.  The headline `value` is MC steps/s of the FP64 path
on the chosen workload (default: the 340-spinor, 128-walker-pair FP64
baseline workload).  Every variant (FP32 / BF16 / FP16 operands, with and
without gradients) replays the same burned-in walker trajectory, so its
per-step values pair with the FP64 ones: `systematic_over_sigma` is
|mean(low - FP64)| / sigma_bar(FP64) (blocking, N_b = 100).  `roofline`
places the dominant kernel (Green's-function GEMMs + pair contraction) on the
FP64 MFMA roofline from HIP-event timings taken on the library's stream;
`cpu_baseline` is the FP64 CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PROFILED = ["spinor_gemm", "green_contract", "grad", "coef_grad"]
METRIC = "MC steps/s and var×time for E2(+grad), FP32/BF16 vs FP64, 1 MI355X"
# published dense peaks of one MI355X (TFLOP/s) for the GEMM operand type
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0}
WORKLOADS = {
    "C0": "tiny: 2 nuclei 1.5 bohr apart, 12 L / 32 S Cartesian primitives, 4 occupied / 16 virtual "
          "spinors, m=16 walker pairs, 1 tau per step",
    "C1": "FP64 baseline: 3 nuclei (triangle, edge 4.894 bohr), 200 L / 460 S Cartesian primitives, "
          "40 occupied / 300 virtual spinors, m=128 walker pairs, 2 tau per step",
    "C3": "precision workload: 4 nuclei (tetrahedron), 600 L / 1380 S primitives, 80 occupied / 900 virtual "
          "spinors, m=256 walker pairs, 1 tau per step",
    "C4": "largest: 6 nuclei (octahedron), 1000 L / 2300 S primitives, 120 occupied / 1500 virtual spinors, "
          "m=512 walker pairs, 4 tau per step",
}


def green_flops(m: int, n_sp: int, n_tau: int) -> float:
    """Algorithmic flops of G- and G+ over all walker pairs p < q for one
    step: 8x8 complex blocks, n_sp complex multiply-adds (8 flops) each, per tau."""
    return 512.0 * (m * (m - 1) / 2.0) * n_sp * n_tau


def kernel_flops(inp) -> dict:
    """Algorithmic flops per step of each GEMM-shaped kernel (complex MAC = 8,
    real-by-complex MAC = 4; zero walker blocks and padding not counted)."""
    m, nsp, nb, nt = inp.m, inp.n_sp, inp.n_b, inp.n_tau
    return {
        "spinor_gemm": 16.0 * m * nsp * nb,          # 2m points x 4 components x nsp, real x complex over n_L or n_S
        "green_contract": green_flops(m, nsp, nt),
        "grad": 512.0 * m * (m - 1) * nsp * nt,      # Psibar = sum_t H_t Psi S_t, off-diagonal walker blocks
        "coef_grad": 16.0 * m * nsp * nb,            # Cbar = X^T Psibar: same shape as the spinor GEMM
    }


def operand_type(prec: str, kernel: str) -> str:
    """MFMA operand type of a kernel in a precision mode.  BF16 / FP16 modes:
    spinor GEMM on split BF16 operands (hi + lo, three BF16 products: its
    algorithmic flops are priced at the BF16 peak), adjoint GEMM and
    coefficient gradient on BF16, Green's GEMMs on the mode's type.  FP32 mode:
    FP32 spinor and Green's GEMMs, FP64 adjoint and coefficient gradient."""
    if prec == "fp64":
        return "fp64"
    if prec == "fp32":
        return "fp64" if kernel in ("grad", "coef_grad") else "fp32"
    return prec if kernel == "green_contract" else "bf16"


def kernel_table(prof: dict, kflops: dict, K: int, prec: str) -> dict:
    out = {}
    for k, (tot_ms, _) in prof.items():
        avg_s = tot_ms / K / 1e3
        tf = kflops[k] / avg_s / 1e12
        op = operand_type(prec, k)
        out[k] = {"us_per_step": round(avg_s * 1e6, 2), "tflops": round(tf, 2), "operands": op,
                  "peak_frac": round(tf / PEAK_TFLOPS[op], 4)}
    return out


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
    return {"value": round(n / el, 4), "unit": "MC steps/s", "cores": int(torch.get_num_threads()),
            "kind": "oracle",
            "sample": f"{n} consecutive steps (Metropolis move, tau samples, estimator) of the same workload, "
                      f"{el:.1f} s on the host"}


def run_variant(inp, precision, grad, state, K, W, profile):
    """Replay the burned-in trajectory for W + K steps; time the last K."""
    import torch

    from paper_2203_05632_amd import Context
    ctx = Context.from_inputs(inp, precision=precision, want_grad=grad)
    wk, w = state["wk"].clone(), state["w"].clone()
    key, delta, step = state["key"], state["delta"], state["step"]
    tau = torch.zeros(inp.n_tau, dtype=torch.float64, device="cuda")
    hist = torch.zeros((K, inp.n_tau, 3), dtype=torch.float64, device="cuda")
    scratch = torch.zeros((inp.n_tau, 3), dtype=torch.float64, device="cuda")
    g = {}
    if grad:
        g["eps"] = torch.zeros(inp.n_sp, dtype=torch.float64, device="cuda")
        g["c"] = torch.zeros((2, inp.n_b, inp.n_sp), dtype=torch.complex128, device="cuda")
        g["eps_s"], g["eps_c"] = torch.zeros_like(g["eps"]), torch.zeros_like(g["eps"])
        g["c_s"], g["c_c"] = torch.zeros_like(g["c"]), torch.zeros_like(g["c"])

    def one(s, out):
        ctx.advance(wk, w, key, s, delta, tau)          # Metropolis move + tau samples (one launch)
        if grad:
            ctx.step(wk, tau, out, grad_eps=g["eps"], grad_coeffs=g["c"])
            ctx.accumulate(g["eps"], g["eps_s"], g["eps_c"])   # compensated sums over steps
            ctx.accumulate(g["c"], g["c_s"], g["c_c"])
        else:
            ctx.step(wk, tau, out)                      # estimator of Eq. redundant

    for i in range(W):
        one(step + i, scratch)
    torch.cuda.synchronize()
    if profile:
        ctx.profile_begin(PROFILED, K * len(PROFILED))
    t0 = time.perf_counter()
    for i in range(K):
        one(step + W + i, hist[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = ctx.profile_end() if profile else {}
    ctx.close()
    return elapsed, hist.mean(dim=1)[:, 2].cpu().numpy(), prof


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--burnin", type=int, default=300, help="untimed Metropolis steps adapting delta")
    ap.add_argument("--config", default="C1", choices=sorted(WORKLOADS))
    ap.add_argument("--variant-steps", type=int, default=None, help="timed steps per variant (default: --steps)")
    ap.add_argument("--no-variants", action="store_true", help="FP64 headline only")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle sample length (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (one MC chain on one MI355X); --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from oracle.blocking import blocking
    from paper_2203_05632_amd import Context
    from synth import initial_walkers, make_inputs

    torch.cuda.set_device(0)
    inp = make_inputs(args.config)
    key = (0, 0)
    wk0 = initial_walkers(inp)
    # burn-in on an FP64 context (walker moves do not depend on the operand precision)
    drv = Context.from_inputs(inp)
    wk = torch.as_tensor(wk0, device="cuda")
    w = torch.zeros(inp.m, dtype=torch.float64, device="cuda")
    n_acc = torch.zeros(1, dtype=torch.int32, device="cuda")
    drv.pair_weights(wk, w)
    delta, step = 0.5, 0
    for _ in range(args.burnin // 10):
        n_acc.zero_()
        for _ in range(10):
            drv.metropolis(wk, w, key, step, delta, n_acc)
            step += 1
        delta *= 1.1 if n_acc.item() / (10.0 * inp.m) > 0.5 else 0.9
    torch.cuda.synchronize()
    drv.close()
    state = {"wk": wk, "w": w, "key": key, "delta": delta, "step": step}

    K, W = args.steps, args.warmup
    elapsed, ref_vals, prof = run_variant(inp, "fp64", False, state, K, W, profile=True)
    steps_per_s = K / elapsed
    sbar = blocking(ref_vals, 100)[1] if K >= 200 else None
    flops = green_flops(inp.m, inp.n_sp, inp.n_tau)
    kflops = kernel_flops(inp)
    roofline = None
    if "green_contract" in prof:
        tot_ms, n_l = prof["green_contract"]
        avg_s = tot_ms / K / 1e3                      # per step (one launch per group of <= 4 tau)
        ach = flops / avg_s / 1e12
        roofline = {"bound": "mfma", "achieved": round(ach, 3), "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                    "frac": round(ach / PEAK_TFLOPS["fp64"], 4), "traffic": None, "kernel": "green_contract",
                    "avg_us": round(tot_ms / n_l * 1e3, 2), "launches_per_step": n_l // K,
                    "flops_per_launch": flops / (n_l // K)}

    variants = {}
    if not args.no_variants:
        Kv = args.variant_steps or K
        for prec, grad in (("fp32", False), ("bf16", False), ("fp16", False), ("fp64", True), ("bf16", True),
                           ("fp16", True)):
            el, vals, vprof = run_variant(inp, prec, grad, state, Kv, W, profile=True)
            name = prec + ("+grad" if grad else "")
            v = {"steps_per_s": round(Kv / el, 2), "ms_per_step": round(1e3 * el / Kv, 5),
                 "speedup_vs_fp64": round((Kv / el) / steps_per_s, 3)}
            if grad and "fp64+grad" in variants:
                v["speedup_vs_fp64_grad"] = round((Kv / el) / variants["fp64+grad"]["steps_per_s"], 3)
            kern = kernel_table(vprof, kflops, Kv, prec)
            v["kernels"] = kern
            if Kv == K and Kv >= 200:
                d = vals - ref_vals
                v["systematic_over_sigma"] = float(f"{abs(d.mean()) / sbar:.3e}")
                v["var_x_time"] = float(f"{blocking(vals, 100)[1] ** 2 * el:.6g}")
            variants[name] = v

    cpu = cpu_baseline(inp, wk0, key, delta, args.cpu_seconds) if args.cpu_seconds > 0 else None
    out = {
        "metric": METRIC, "value": round(steps_per_s, 2), "unit": "MC steps/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": round(1e3 * elapsed / K, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.config} {WORKLOADS[args.config]}", "m": inp.m, "n_tau": inp.n_tau,
                   "n_L": inp.n_L, "n_S": inp.n_S, "n_occ": inp.n_occ, "n_vir": inp.n_vir,
                   "precision": "fp64", "grad": False},
        "var_x_time": None if sbar is None else float(f"{sbar ** 2 * elapsed:.6g}"),
        "var_x_time_unit": "Eh^2 s",
        "e2_mean": float(f"{ref_vals.mean():.6g}"),
        "sigma_bar": None if sbar is None else float(f"{sbar:.6g}"),
        "roofline": roofline,
        "kernels": kernel_table(prof, kflops, K, "fp64"),
        "variants": variants,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
