#!/usr/bin/env python3
"""Throughput of the stochastic relativistic MP2 hot path on one MI355X.

One step = one Metropolis move of all m walker pairs + inverse-CDF tau
samples + one evaluation of the redundant-walker estimator (spinor values,
G-/G+ for every walker pair, direct/exchange contraction, compensated sums),
all on the GPU through libmcmp2; with gradients, also the adjoint (eps and
coefficient gradients) and their compensated accumulation over steps.
Inputs are synthetic and seeded (synth/).

Prints one JSON line (progress goes to stderr).  The headline `value` is MC
steps/s of the FP64 path on the chosen workload (default: the 340-spinor,
128-walker-pair FP64 baseline workload).  `largest` repeats the FP64, FP64 +
gradient and BF16 / FP16 (+ gradient) runs on the largest workload (1620
spinors, 512 walker pairs, 4 tau per step), where the mixed-precision path
with gradients is compared with the FP64 path with gradients.  Every variant (FP32 / BF16 / FP16 operands, with and
without gradients) replays the same burned-in walker trajectory, so its
per-step values pair with the FP64 ones: `systematic_over_sigma` is
|mean(low - FP64)| / sigma_bar(FP64) (blocking, N_b = 100).  `roofline`
places the dominant kernel (Green's-function GEMMs + pair contraction) on the
FP64 MFMA roofline from HIP-event timings taken on the library's stream
around every launch of a 300-step pass that follows each throughput run (the
events cost ~10% of a small step, so throughput is timed without them);
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
HBM_PEAK_GBS = 8000.0   # published HBM3E bandwidth of one MI355X
PROFILE_STEPS = 300   # steps of the HIP-event-timed pass after each throughput run
# (operand precision, gradients[, interaction]); the interaction variants run the
# Gaunt / Breit terms of the electron-electron operator (FP64, no gradients)
HEADLINE_VARIANTS = [("fp32", False), ("bf16", False), ("fp16", False), ("fp64", True), ("bf16", True),
                     ("fp16", True), ("fp64", False, "gaunt"), ("fp64", False, "breit")]
LARGEST_VARIANTS = [("fp64", True), ("fp32", True), ("bf16", False), ("bf16", True), ("fp16", True)]
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


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "green_contract_C1_fp64_traffic.md")


def sources_sha256(files) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(config: str):
    """HBM bytes per launch of the Green's-function kernel from the committed
    rocprofv3 counter record (FETCH_SIZE + WRITE_SIZE, scaled by the same
    counters on a copy of known size), or None when no record matches this
    workload or the kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            text = fh.read()
        rec = json.loads(text.split("```json")[1].split("```")[0])
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("workload") != config or rec.get("sources_sha256") != sources_sha256(rec.get("sources", [])):
        return None
    return rec["hbm_bytes_per_launch"]


def progress(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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
        # Cbar = X^T Psibar: same shape as the spinor GEMM (its epilogue also adds the result
        # to the compensated running sums over steps: 4 doubles moved per element)
        "coef_grad": 16.0 * m * nsp * nb,
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


def run_variant(inp, precision, grad, state, K, W, Kp, interaction="coulomb"):
    """Replay the burned-in trajectory: W warmup steps, K timed steps, then Kp
    more steps with HIP-event timing of the GEMM kernels (recording events
    around every launch costs ~10% of a small step, so it stays out of the
    throughput region).  Returns (elapsed of the K steps, per-step values of
    the K steps, per-kernel event totals over the Kp steps)."""
    import torch

    from paper_2203_05632_amd import Context
    ctx = Context.from_inputs(inp, precision=precision, want_grad=grad)
    ctx.set_interaction(interaction)
    wk, w = state["wk"].clone(), state["w"].clone()
    key, delta, step = state["key"], state["delta"], state["step"]
    tau = torch.zeros(inp.n_tau, dtype=torch.float64, device="cuda")
    hist = torch.zeros((K, inp.n_tau, 3), dtype=torch.float64, device="cuda")
    scratch = torch.zeros((inp.n_tau, 3), dtype=torch.float64, device="cuda")
    g = {}
    if grad:  # compensated running sums of both gradients over the steps
        for k in ("eps_s", "eps_c"):
            g[k] = torch.zeros(inp.n_sp, dtype=torch.float64, device="cuda")
        for k in ("c_s", "c_c"):
            g[k] = torch.zeros((2, inp.n_b, inp.n_sp), dtype=torch.complex128, device="cuda")

    def one(s, out):
        ctx.advance(wk, w, key, s, delta, tau)          # Metropolis move + tau samples (one launch)
        if grad:
            # estimator and both gradients, added to the running sums in the gradient kernels
            ctx.step_accumulate(wk, tau, out, g["eps_s"], g["eps_c"], g["c_s"], g["c_c"])
        else:
            ctx.step(wk, tau, out)                      # estimator of Eq. redundant

    for i in range(W):
        one(step + i, scratch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        one(step + W + i, hist[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = {}
    if Kp > 0:
        ctx.profile_begin(PROFILED, Kp * (len(PROFILED) + 1))
        for i in range(Kp):
            one(step + W + K + i, scratch)
        prof = ctx.profile_end()
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
    ap.add_argument("--no-largest", action="store_true", help="skip the largest-workload (C4) section")
    ap.add_argument("--study", choices=["convergence", "scaling", "chains"], default=None,
                    help="instead of the benchmark: redundant-walker convergence vs m, cost vs basis size, or "
                         "independent chains on concurrent streams")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first copy this many MiB device to device (a known-size kernel for counter calibration)")
    ap.add_argument("--largest-steps", type=int, default=1000, help="timed C4 steps per variant")
    ap.add_argument("--largest-grad-steps", type=int, default=200,
                    help="timed C4 steps of the gradient runs with an FP64 adjoint (FP64, FP32 modes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (one MC chain on one MI355X); --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    if args.study:
        out = {"convergence": study_convergence, "scaling": study_scaling, "chains": study_chains}[args.study](args)
        print(json.dumps(out), flush=True)
        return
    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    head = measure_workload(args.config, args.steps, args.warmup, args.burnin,
                            [] if args.no_variants else HEADLINE_VARIANTS, args.variant_steps)
    K, inp, elapsed, sbar = args.steps, head["inp"], head["elapsed"], head["sbar"]
    largest = None
    if not args.no_largest and args.config != "C4":
        lw = measure_workload("C4", args.largest_steps, 5, 50, LARGEST_VARIANTS, None,
                              grad_steps=args.largest_grad_steps)
        largest = {"workload": f"C4 {WORKLOADS['C4']}", "fp64": lw["fp64"], "variants": lw["variants"]}
        g64 = lw["variants"].get("fp64+grad", {}).get("steps_per_s")
        b16 = lw["variants"].get("bf16+grad", {})
        if g64 and b16:
            largest["bf16_grad_over_fp64_grad"] = round(b16["steps_per_s"] / g64, 3)
            largest["bf16_grad_over_fp64"] = round(b16["steps_per_s"] / lw["fp64"]["steps_per_s"], 3)
            largest["bf16_grad_green_mfma_frac"] = b16["kernels"]["green_contract"]["peak_frac"]
            largest["bf16_grad_systematic_over_sigma"] = b16.get("systematic_over_sigma")
        f32 = lw["variants"].get("fp32+grad", {})
        if f32:
            largest["fp32_grad_green_mfma_frac"] = f32["kernels"]["green_contract"]["peak_frac"]

    cpu = cpu_baseline(inp, head["wk0"], head["key"], head["delta"], args.cpu_seconds) if args.cpu_seconds > 0 \
        else None
    out = {
        "metric": METRIC, "value": round(K / elapsed, 2), "unit": "MC steps/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / K, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.config} {WORKLOADS[args.config]}", "m": inp.m, "n_tau": inp.n_tau,
                   "n_L": inp.n_L, "n_S": inp.n_S, "n_occ": inp.n_occ, "n_vir": inp.n_vir,
                   "precision": "fp64", "grad": False},
        "var_x_time": None if sbar is None else float(f"{sbar ** 2 * elapsed:.6g}"),
        "var_x_time_unit": "Eh^2 s",
        "e2_mean": float(f"{head['ref_vals'].mean():.6g}"),
        "sigma_bar": None if sbar is None else float(f"{sbar:.6g}"),
        "roofline": head["roofline"],
        "kernels": head["fp64"]["kernels"],
        "variants": head["variants"],
        "largest": largest,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def study_convergence(args):
    """Redundant-walker estimator vs the number of walker pairs m (Sec. III:
    all m(m-1)/2 pairs of m independent walkers enter every step, at a cost
    per step growing like m^2): for each m, FP64 steps/s, sigma_bar of the
    step mean (blocking, N_b = 100), the per-step variance sigma_bar^2 N and
    var x time.  The 340-spinor shapes with basis exponents in [0.3, 1.2]:
    with the full exponent range and synthetic orbitals the estimator is
    heavy-tailed and sigma_bar does not settle within a few thousand steps."""
    from oracle.blocking import blocking
    from synth import initial_walkers, make_inputs
    K = max(args.steps, 5000)
    rows = []
    for m in (8, 16, 32, 64, 128, 256, 512):
        inp = make_inputs("C1", m=m, exp_range=(0.3, 1.2))
        state = burn_in(inp, initial_walkers(inp), (0, m), args.burnin)
        el, vals, _ = run_variant(inp, "fp64", False, state, K, args.warmup, 0)
        sb = blocking(vals, 100)[1]
        rows.append({"m": m, "pairs": m * (m - 1) // 2, "steps": K, "steps_per_s": round(K / el, 2),
                     "e2_mean": float(f"{vals.mean():.6g}"), "sigma_bar": float(f"{sb:.4g}"),
                     "var_per_step": float(f"{sb * sb * K:.4g}"), "var_x_time": float(f"{sb * sb * el:.4g}")})
        progress(f"convergence m={m}: {rows[-1]}")
    return {"study": "redundant-walker convergence vs m",
            "workload": "C1 shapes (3 nuclei, 200 L / 460 S primitives, 40 occupied / 300 virtual spinors, "
                        "2 tau per step) with basis exponents in [0.3, 1.2]",
            "precision": "fp64", "rows": rows}


def study_scaling(args):
    """Cost per step vs basis size at fixed m = 128 and 1 tau per step, on the
    synthetic size ladder of the workloads (n_L = 12 ... 1000 primitives,
    n_sp = 20 ... 1620 spinors): FP64 and BF16 steps/s, with and without
    gradients, and the log-log slope of time per step against n_b."""
    import numpy as np

    from synth import initial_walkers, make_inputs
    K = 200
    rows = []
    for name in ("C0", "C1", "C3", "C4"):
        inp = make_inputs(name, m=128, n_tau=1)
        state = burn_in(inp, initial_walkers(inp), (0, 0), 50)
        row = {"workload": name, "n_b": inp.n_b, "n_occ": inp.n_occ, "n_sp": inp.n_sp}
        for prec, grad in (("fp64", False), ("fp64", True), ("bf16", False), ("bf16", True)):
            el, _, _ = run_variant(inp, prec, grad, state, K, 10, 0)
            row[prec + ("+grad" if grad else "")] = round(K / el, 2)
        rows.append(row)
        progress(f"scaling {name}: {row}")
    out = {"study": "cost per step vs basis size (m = 128, 1 tau)", "rows": rows}
    nb = np.log([r["n_b"] for r in rows[1:]])
    for key in ("fp64", "fp64+grad", "bf16", "bf16+grad"):
        t = np.log([1.0 / r[key] for r in rows[1:]])
        out[f"slope_{key}"] = round(float(np.polyfit(nb, t, 1)[0]), 3)   # d log(time) / d log(n_b), C1..C4
    return out


def study_chains(args):
    """Independent chains (the paper's parallel model, Sec. III) on separate
    HIP streams of one GPU: aggregate MC steps/s of k = 1, 2, 4, 8 chains of
    the 340-spinor FP64 workload, launched block by block in turn, and the
    merged estimate."""
    import torch

    from paper_2203_05632_amd import Chain, Context, merge
    from synth import initial_walkers, make_inputs
    inp = make_inputs("C1")
    K = max(args.steps, 1000)
    rows = []
    for k in (1, 2, 4, 8):
        streams = [torch.cuda.Stream() for _ in range(k)]
        chains = [Chain(Context.from_inputs(inp, stream=streams[c]), initial_walkers(inp, chain=c), key=(7, c))
                  for c in range(k)]
        for ch in chains:
            ch.burn_in(args.burnin)
            ch.run(50, block=50)            # warmup
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K // 100):
            for ch in chains:
                ch.run(100, block=100)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res = merge([ch.result() for ch in chains])
        rows.append({"chains": k, "steps_total": k * (K // 100) * 100, "steps_per_s": round(k * (K // 100) * 100 / el, 1),
                     "e2_merged": float(f"{res.mean[2]:.6g}"), "sigma_merged": float(f"{res.sigma[2]:.4g}")})
        progress(f"chains k={k}: {rows[-1]}")
        for ch in chains:
            ch.ctx.close()
    return {"study": "independent chains on concurrent streams", "workload": f"C1 {WORKLOADS['C1']}",
            "precision": "fp64", "rows": rows}


def burn_in(inp, wk0, key, n_burn):
    """Metropolis burn-in on an FP64 context (walker moves do not depend on
    the operand precision), adapting delta toward acceptance 0.5."""
    import torch

    from paper_2203_05632_amd import Context
    drv = Context.from_inputs(inp)
    wk = torch.as_tensor(wk0, device="cuda")
    w = torch.zeros(inp.m, dtype=torch.float64, device="cuda")
    n_acc = torch.zeros(1, dtype=torch.int32, device="cuda")
    drv.pair_weights(wk, w)
    delta, step = 0.5, 0
    for _ in range(n_burn // 10):
        n_acc.zero_()
        for _ in range(10):
            drv.metropolis(wk, w, key, step, delta, n_acc)
            step += 1
        delta *= 1.1 if n_acc.item() / (10.0 * inp.m) > 0.5 else 0.9
    torch.cuda.synchronize()
    drv.close()
    return {"wk": wk, "w": w, "key": key, "delta": delta, "step": step}


def measure_workload(name, K, W, n_burn, variants, Kv=None, grad_steps=None):
    """FP64 reference run plus the listed (precision, grad) variants, all
    replaying one burned-in trajectory."""
    from oracle.blocking import blocking
    from synth import initial_walkers, make_inputs

    inp = make_inputs(name)
    key = (0, 0)
    wk0 = initial_walkers(inp)
    state = burn_in(inp, wk0, key, n_burn)
    progress(f"{name}: inputs ready, burn-in done")
    Kp = min(K, PROFILE_STEPS)
    elapsed, ref_vals, prof = run_variant(inp, "fp64", False, state, K, W, Kp)
    steps_per_s = K / elapsed
    progress(f"{name} fp64: {steps_per_s:.2f} steps/s")
    sbar = blocking(ref_vals, 100)[1] if K >= 200 else None
    flops = green_flops(inp.m, inp.n_sp, inp.n_tau)
    kflops = kernel_flops(inp)
    roofline = None
    if "green_contract" in prof:
        tot_ms, n_l = prof["green_contract"]
        avg_s = tot_ms / Kp / 1e3                     # per step (one launch per step)
        ach = flops / avg_s / 1e12
        roofline = {"bound": "mfma", "achieved": round(ach, 3), "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                    "frac": round(ach / PEAK_TFLOPS["fp64"], 4), "traffic": recorded_traffic(name),
                    "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE)",
                    "kernel": "green_contract",
                    "avg_us": round(tot_ms / n_l * 1e3, 2), "launches_per_step": n_l // Kp,
                    "flops_per_launch": flops / (n_l // Kp), "event_steps": Kp}
    out_vars = {}
    for var in variants:
        prec, grad = var[0], var[1]
        inter = var[2] if len(var) > 2 else "coulomb"
        # runs with an FP64 adjoint GEMM (FP64 and FP32 modes) are ~10x slower: fewer steps
        Kn = (grad_steps if (grad and prec in ("fp64", "fp32") and grad_steps) else (Kv or K))
        Kpn = min(Kn, PROFILE_STEPS)
        el, vals, vprof = run_variant(inp, prec, grad, state, Kn, W, Kpn, inter)
        vname = prec + ("+grad" if grad else "") + ("" if inter == "coulomb" else "+" + inter)
        v = {"steps": Kn, "steps_per_s": round(Kn / el, 2), "ms_per_step": round(1e3 * el / Kn, 5),
             "speedup_vs_fp64": round((Kn / el) / steps_per_s, 3)}
        if grad and "fp64+grad" in out_vars:
            v["speedup_vs_fp64_grad"] = round((Kn / el) / out_vars["fp64+grad"]["steps_per_s"], 3)
        v["kernels"] = kernel_table(vprof, kflops, Kpn, prec)
        if Kn == K and Kn >= 200:
            d = vals - ref_vals
            if inter == "coulomb":  # same estimator at lower precision: the difference is its error
                v["systematic_over_sigma"] = float(f"{abs(d.mean()) / sbar:.3e}")
            else:  # another estimator: the mean shift from the Coulomb one, in its standard errors
                v["mean_shift_over_sigma"] = float(f"{d.mean() / sbar:.3e}")
            v["var_x_time"] = float(f"{blocking(vals, 100)[1] ** 2 * el:.6g}")
        out_vars[vname] = v
        progress(f"{name} {vname}: {v['steps_per_s']} steps/s")
    return {"inp": inp, "wk0": wk0, "key": key, "delta": state["delta"], "elapsed": elapsed, "ref_vals": ref_vals,
            "sbar": sbar, "roofline": roofline,
            "fp64": {"steps": K, "steps_per_s": round(steps_per_s, 2), "ms_per_step": round(1e3 * elapsed / K, 5),
                     "kernels": kernel_table(prof, kflops, Kp, "fp64")},
            "variants": out_vars}


if __name__ == "__main__":
    main()
