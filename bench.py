#!/usr/bin/env python3
"""Throughput of the stochastic relativistic MP2 hot path on one MI355X.

One step = one Metropolis move of all m walker pairs + inverse-CDF tau
samples + one evaluation of the redundant-walker estimator (spinor values,
G-/G+ for every walker pair, direct/exchange contraction, compensated sums),
all on the GPU through libmcmp2; with gradients, also the adjoint (eps and
coefficient gradients) added to compensated running sums over the steps.
Inputs are synthetic and seeded (synth/).

Prints one JSON line (progress goes to stderr).  Default workload: the largest
one (6 nuclei, 1000 L / 2300 S primitives, 120 occupied / 1500 virtual
spinors, 512 walker pairs, 4 tau per step).  The headline `value` is MC
steps/s of the FP64 path with both gradients; `variants` repeats the step
with FP32 / BF16 / FP16 operands (with and without gradients) and FP64
without gradients on the same burned-in walker trajectory, each with
`speedup_vs_fp64_grad`.

Every timed region records HIP events on the library's stream around each
dispatch of the Green's-function GEMM kernel and of the adjoint GEMM kernel
(a few event pairs per step of >= 0.7 ms); `roofline` places the headline's
dominant kernel on the MFMA roofline of its operand type from those events.

Statistics come from separate replays of `--stat-steps` steps (default 1000,
whatever --steps is) of the same trajectory with per-step outputs: sigma_bar
of the step value by blocking (N_b = 100, Sec. III), var x time =
sigma_bar_N^2 T_N with T_N = N x the variant's time per step, and, for every
reduced-precision mode, the systematic error of the step value, of every eps
gradient component and of 16 fixed random projections Re<D_j, Cbar> of the
coefficient gradient: |mean(low - FP64)| / sigma_bar(FP64) with the paired
standard error of the difference.  `cpu_baseline` times the FP64 CPU oracle
on the same workload (forward + gradients).
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

STAGES = ["spinor_gemm", "green_contract", "grad", "coef_grad"]
DISPATCH = ["green_gemm", "adj_gemm"]   # single dispatches of the two dominant GEMM kernels
HBM_PEAK_GBS = 8000.0   # published HBM3E bandwidth of one MI355X
# published dense peaks of one MI355X (TFLOP/s) for the GEMM operand type
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0}
METRIC = "MC steps/s and var×time for E2(+grad), FP32/BF16 vs FP64, 1 MI355X"
# (operand precision, gradients[, interaction]) replayed after the headline (FP64 + gradients)
VARIANTS = {
    "C4": [("fp64", False), ("fp32", True), ("bf16", False), ("bf16", True), ("fp16", True)],
    "C3": [("fp64", False), ("fp32", True), ("bf16", False), ("bf16", True), ("fp16", True)],
    "C1": [("fp64", False), ("fp32", False), ("bf16", False), ("fp16", False), ("bf16", True), ("fp16", True),
           ("fp64", False, "gaunt"), ("fp64", False, "breit"), ("bf16", False, "breit"),
           ("fp64", True, "breit"), ("bf16", True, "breit")],
    "C0": [("fp64", False), ("bf16", True)],
}
STAT_PRECISIONS = ["fp32", "bf16", "fp16"]   # replayed with gradients against the FP64 replay
N_PROJ = 16                                  # random projections of the coefficient gradient
WORKLOADS = {
    "C0": "tiny: 2 nuclei 1.5 bohr apart, 12 L / 32 S Cartesian primitives, 4 occupied / 16 virtual "
          "spinors, m=16 walker pairs, 1 tau per step",
    "C1": "FP64 baseline: 3 nuclei (triangle, edge 4.894 bohr), 200 L / 460 S Cartesian primitives, "
          "40 occupied / 300 virtual spinors, m=128 walker pairs, 2 tau per step",
    "C3": "precision workload: 4 nuclei (tetrahedron), 600 L / 1380 S primitives, 80 occupied / 900 virtual "
          "spinors, m=256 walker pairs, 1 tau per step",
    "C4": "largest: 6 nuclei (octahedron, edge 4.894 bohr), 1000 L / 2300 S Cartesian primitives, "
          "120 occupied / 1500 virtual spinors, m=512 walker pairs, 4 tau per step",
}
TRAFFIC_RECORDS = os.path.join(ROOT, "profiles")


def progress(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sources_sha256(files) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel: str, workload: str, precision: str):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter
    record under profiles/ (FETCH_SIZE + WRITE_SIZE per dispatch, scaled by
    the same counters on a copy of known size), or None when no record covers
    this kernel, workload and precision for the current kernel sources."""
    import glob
    for path in sorted(glob.glob(os.path.join(TRAFFIC_RECORDS, "*traffic*.md"))):
        try:
            with open(path) as fh:
                text = fh.read()
            rec = json.loads(text.split("```json")[1].split("```")[0])
        except (OSError, IndexError, ValueError):
            continue
        if (rec.get("kernel_id") == kernel and rec.get("workload") == workload and rec.get("precision") == precision
                and rec.get("sources_sha256") == sources_sha256(rec.get("sources", []))):
            return rec["hbm_bytes_per_launch"]
    return None


def kernel_flops(inp) -> dict:
    """Algorithmic flops per step of each GEMM-shaped stage (complex MAC = 8,
    real-by-complex MAC = 4; zero walker blocks and padding not counted)."""
    m, nsp, nb, nt = inp.m, inp.n_sp, inp.n_b, inp.n_tau
    return {
        "spinor_gemm": 16.0 * m * nsp * nb,               # 2m points x 4 components x nsp, real x complex over n_L or n_S
        "green_contract": 512.0 * (m * (m - 1) / 2.0) * nsp * nt,   # 8x8 complex blocks p < q, per tau
        "grad": 512.0 * m * (m - 1) * nsp * nt,           # Psibar = sum_t H_t Psi S_t, off-diagonal walker blocks
        "coef_grad": 16.0 * m * nsp * nb,                 # Cbar = X^T Psibar, the spinor GEMM's shape
    }


def operand_type(prec: str, kernel: str) -> str:
    """MFMA operand type of a kernel in a precision mode.  BF16 / FP16 modes:
    spinor GEMM on split BF16 operands (three BF16 products; its algorithmic
    flops are priced at the BF16 peak), adjoint GEMM and coefficient gradient
    on BF16, Green's GEMMs on the mode's type.  FP32 mode: FP32 spinor and
    Green's GEMMs, FP64 adjoint and coefficient gradient."""
    if prec == "fp64":
        return "fp64"
    if prec == "fp32":
        return "fp64" if kernel in ("grad", "coef_grad", "adj_gemm") else "fp32"
    return prec if kernel in ("green_contract", "green_gemm") else "bf16"


def stage_table(prof: dict, kflops: dict, K: int, prec: str) -> dict:
    out = {}
    for k, (tot_ms, _) in prof.items():
        if k not in kflops:
            continue
        avg_s = tot_ms / K / 1e3
        tf = kflops[k] / avg_s / 1e12
        op = operand_type(prec, k)
        out[k] = {"us_per_step": round(avg_s * 1e6, 2), "tflops": round(tf, 2), "operands": op,
                  "peak_frac": round(tf / PEAK_TFLOPS[op], 4)}
    return out


def dispatch_table(prof: dict, kflops: dict, K: int, prec: str) -> dict:
    """Per-dispatch duration of the Green's and adjoint GEMM kernels (HIP
    events in the timed region) with their algorithmic flops per dispatch."""
    out = {}
    for k, stage in (("green_gemm", "green_contract"), ("adj_gemm", "grad")):
        if k not in prof:
            continue
        tot_ms, n = prof[k]
        per_step = n / K
        flops = kflops[stage] / per_step
        avg_s = tot_ms / n / 1e3
        op = operand_type(prec, k)
        ach = flops / avg_s / 1e12
        out[k] = {"avg_us": round(avg_s * 1e6, 2), "launches_per_step": round(per_step, 3),
                  "flops_per_launch": flops, "tflops": round(ach, 2), "operands": op,
                  "peak_frac": round(ach / PEAK_TFLOPS[op], 4)}
    return out


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
    for _ in range(max(1, n_burn // 10)):
        n_acc.zero_()
        for _ in range(10):
            drv.metropolis(wk, w, key, step, delta, n_acc)
            step += 1
        delta *= 1.1 if n_acc.item() / (10.0 * inp.m) > 0.5 else 0.9
    torch.cuda.synchronize()
    drv.close()
    return {"wk": wk, "w": w, "key": key, "delta": delta, "step": step}


def run_timed(inp, precision, grad, state, K, W, interaction="coulomb", stage_steps=20):
    """Replay the burned-in trajectory: W warmup steps, then K timed steps with
    HIP events around every Green's / adjoint GEMM dispatch, then stage_steps
    more with events around every stage.  Gradients go to compensated running
    sums (mcmp2_step_accumulate).  Returns (elapsed s, dispatch events,
    stage events)."""
    import torch

    from paper_2203_05632_amd import Context
    ctx = Context.from_inputs(inp, precision=precision, want_grad=grad)
    ctx.set_interaction(interaction)
    wk, w = state["wk"].clone(), state["w"].clone()
    key, delta, step = state["key"], state["delta"], state["step"]
    tau = torch.zeros(inp.n_tau, dtype=torch.float64, device="cuda")
    e2 = torch.zeros((inp.n_tau, 3), dtype=torch.float64, device="cuda")
    g = {}
    if grad:
        for k in ("eps_s", "eps_c"):
            g[k] = torch.zeros(inp.n_sp, dtype=torch.float64, device="cuda")
        for k in ("c_s", "c_c"):
            g[k] = torch.zeros((2, inp.n_b, inp.n_sp), dtype=torch.complex128, device="cuda")

    def one(s):
        ctx.advance(wk, w, key, s, delta, tau)          # Metropolis move + tau samples (one launch)
        if grad:
            ctx.step_accumulate(wk, tau, e2, g["eps_s"], g["eps_c"], g["c_s"], g["c_c"])
        else:
            ctx.step(wk, tau, e2)                       # estimator of Eq. redundant

    for i in range(W):
        one(step + i)
    torch.cuda.synchronize()
    ctx.profile_begin(DISPATCH, 8 * K)
    t0 = time.perf_counter()
    for i in range(K):
        one(step + W + i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    disp = ctx.profile_end()
    stages = {}
    if stage_steps > 0:
        ctx.profile_begin(STAGES, stage_steps * (len(STAGES) + 1))
        for i in range(stage_steps):
            one(step + W + K + i)
        stages = ctx.profile_end()
    ctx.close()
    return elapsed, disp, stages


def stat_replay(inp, precision, state, N, D):
    """N steps of the trajectory with per-step outputs: the step value, the
    eps gradient and the projections D @ (Re, Im of the coefficient
    gradient).  Returns numpy arrays (value [N], geps [N, n_sp], gproj [N, n_proj])."""
    import torch

    from paper_2203_05632_amd import Context
    ctx = Context.from_inputs(inp, precision=precision, want_grad=True)
    wk, w = state["wk"].clone(), state["w"].clone()
    key, delta, step = state["key"], state["delta"], state["step"]
    tau = torch.zeros(inp.n_tau, dtype=torch.float64, device="cuda")
    e2 = torch.zeros((inp.n_tau, 3), dtype=torch.float64, device="cuda")
    val = torch.zeros((N, 1), dtype=torch.float64, device="cuda")
    geps = torch.zeros((N, inp.n_sp), dtype=torch.float64, device="cuda")
    gc = torch.zeros((2, inp.n_b, inp.n_sp), dtype=torch.complex128, device="cuda")
    gproj = torch.zeros((N, D.shape[0]), dtype=torch.float64, device="cuda")
    gflat = torch.view_as_real(gc).reshape(-1)
    for i in range(N):
        ctx.advance(wk, w, key, step + i, delta, tau)
        ctx.step(wk, tau, e2, grad_eps=geps[i], grad_coeffs=gc, value=val[i])
        torch.mv(D, gflat, out=gproj[i])
    torch.cuda.synchronize()
    ctx.close()
    return val[:, 0].cpu().numpy(), geps.cpu().numpy(), gproj.cpu().numpy()


def statistics(inp, state, N, precisions, progress_label):
    """FP64 replay plus one replay per reduced precision; sigma_bar and the
    systematic errors of value, eps gradient and coefficient-gradient
    projections."""
    import numpy as np
    import torch

    from paper_2203_05632_amd import blocking_sigma
    gen = torch.Generator(device="cuda")
    gen.manual_seed(20220311)
    D = torch.randn((N_PROJ, 4 * inp.n_b * inp.n_sp), generator=gen, dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    ref = stat_replay(inp, "fp64", state, N, D)
    progress(f"{progress_label} fp64 replay of {N} steps: {time.perf_counter() - t0:.1f} s")
    sb = [blocking_sigma(x, 100) for x in ref]           # sigma_bar per observable (FP64)
    out = {"fp64": {"steps": N, "e2_mean": float(f"{ref[0].mean():.6g}"), "sigma_bar": float(f"{sb[0]:.6g}"),
                    "series": ref[0]}}
    for prec in precisions:
        t0 = time.perf_counter()
        low = stat_replay(inp, prec, state, N, D)
        progress(f"{progress_label} {prec} replay of {N} steps: {time.perf_counter() - t0:.1f} s")
        rec = {"steps": N, "e2_mean": float(f"{low[0].mean():.6g}"),
               "sigma_bar": float(f"{blocking_sigma(low[0], 100):.6g}"), "series": low[0]}
        for name, x, y, s in (("value", ref[0], low[0], sb[0]), ("grad_eps", ref[1], low[1], sb[1]),
                              ("grad_coeffs_proj", ref[2], low[2], sb[2])):
            d = y - x
            ratio = np.abs(d.mean(axis=0)) / s
            se = blocking_sigma(d, 100) / s
            if np.ndim(ratio) == 0:
                rec[f"{name}_systematic_over_sigma"] = float(f"{ratio:.3e}")
                rec[f"{name}_systematic_se_over_sigma"] = float(f"{se:.3e}")
            else:
                j = int(np.argmax(ratio))
                rec[f"{name}_systematic_over_sigma_max"] = float(f"{ratio[j]:.3e}")
                rec[f"{name}_systematic_se_over_sigma_at_max"] = float(f"{se[j]:.3e}")
                rec[f"{name}_systematic_over_sigma_median"] = float(f"{np.median(ratio):.3e}")
                rec[f"{name}_components"] = int(ratio.size)
        out[prec] = rec
    del D
    return out


def cpu_baseline(inp, wk0, key, delta, seconds: float):
    """The FP64 CPU oracle on the same workload: consecutive MC steps
    (Metropolis move, tau samples, estimator and both gradients by reverse-mode
    differentiation of the oracle's forward) for at least `seconds` and at
    least two steps, then two forward-only steps."""
    import numpy as np
    import torch

    from oracle.gradient import step_value_and_grad
    from oracle.integrand import step_estimate
    from oracle.sampling import metropolis_step, sample_tau
    from oracle.weights import n_g, pair_weight, tau_lambda

    Ng = n_g(inp.nuc_xyz, inp.wfn)
    lam = tau_lambda(inp.eps, inp.n_occ)
    wk = wk0.copy()
    w = pair_weight(wk[:, 0], wk[:, 1], inp.nuc_xyz, inp.wfn, Ng)
    keyu = np.array(key, dtype=np.uint64)

    def run(grad, min_steps, min_s, n0):
        nonlocal wk, w
        n, t0 = 0, time.perf_counter()
        while True:
            wk, w, _ = metropolis_step(wk, w, keyu, n0 + n, delta, inp.nuc_xyz, inp.wfn, Ng)
            taus = sample_tau(keyu, n0 + n, inp.n_tau, lam)
            if grad:
                step_value_and_grad(inp, wk, taus, lam, Ng)
            else:
                step_estimate(inp, wk, taus, lam, Ng)
            n += 1
            el = time.perf_counter() - t0
            if n >= min_steps and el >= min_s:
                return n, el

    n_g_steps, el_g = run(True, 2, seconds, 0)
    n_f_steps, el_f = run(False, 2, 0.0, n_g_steps)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return {"value": round(n_g_steps / el_g, 5), "unit": "MC steps/s", "cores": int(torch.get_num_threads()),
            "kind": "oracle",
            "sample": f"{n_g_steps} consecutive MC steps of the same workload with both gradients (Metropolis move, "
                      f"tau samples, estimator, reverse-mode gradients of the FP64 oracle), {el_g:.1f} s",
            "forward_only": {"value": round(n_f_steps / el_f, 5), "steps": n_f_steps, "seconds": round(el_f, 2)},
            "nproc": nproc, "cpu_model": model or platform.processor(), "torch_threads": int(torch.get_num_threads())}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed steps of the headline (FP64 + gradients)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--burnin", type=int, default=100, help="untimed Metropolis steps adapting delta")
    ap.add_argument("--config", default="C4", choices=sorted(WORKLOADS))
    ap.add_argument("--variant-steps", type=int, default=None,
                    help="timed steps of each variant (default: max(--steps, 200), 1000 for >= 5 x faster ones)")
    ap.add_argument("--stat-steps", type=int, default=1000, help="steps of each statistics replay (0: skip)")
    ap.add_argument("--no-variants", action="store_true", help="headline only")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle sample length (0: skip)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first copy this many MiB device to device (a known-size kernel for counter calibration)")
    ap.add_argument("--study", choices=["convergence", "scaling", "chains"], default=None,
                    help="instead of the benchmark: sigma_bar vs steps for several m, time to sigma_bar/|E2| = 0.1 "
                         "vs basis size and occupied count, or independent chains on concurrent streams")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (one MC chain on one MI355X); --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
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

    from synth import initial_walkers, make_inputs
    name = args.config
    inp = make_inputs(name)
    key = (0, 0)
    wk0 = initial_walkers(inp)
    state = burn_in(inp, wk0, key, args.burnin)
    progress(f"{name}: inputs ready, burn-in done (delta {state['delta']:.3f})")
    kflops = kernel_flops(inp)

    K, W = args.steps, args.warmup
    el, disp, stages = run_timed(inp, "fp64", True, state, K, W)
    sps = K / el
    head = {"steps": K, "steps_per_s": round(sps, 3), "ms_per_step": round(1e3 * el / K, 4),
            "kernels": stage_table(stages, kflops, 20, "fp64"), "dispatch": dispatch_table(disp, kflops, K, "fp64")}
    progress(f"{name} fp64+grad: {sps:.2f} steps/s")

    variants = {}
    if not args.no_variants:
        for var in VARIANTS[name]:
            prec, grad = var[0], var[1]
            inter = var[2] if len(var) > 2 else "coulomb"
            vname = prec + ("+grad" if grad else "") + ("" if inter == "coulomb" else "+" + inter)
            fast = not (grad and prec in ("fp64", "fp32"))
            Kv = args.variant_steps or (max(K, 1000) if fast else max(K, 200))
            elv, dv, sv = run_timed(inp, prec, grad, state, Kv, W, inter)
            v = {"steps": Kv, "steps_per_s": round(Kv / elv, 3), "ms_per_step": round(1e3 * elv / Kv, 4),
                 "speedup_vs_fp64_grad": round((Kv / elv) / sps, 3),
                 "kernels": stage_table(sv, kflops, 20, prec), "dispatch": dispatch_table(dv, kflops, Kv, prec)}
            variants[vname] = v
            progress(f"{name} {vname}: {v['steps_per_s']} steps/s ({v['speedup_vs_fp64_grad']}x FP64 + grad)")

    stats = None
    if args.stat_steps >= 200:
        stats = statistics(inp, state, args.stat_steps, STAT_PRECISIONS if not args.no_variants else [], name)
        n_blocks = args.stat_steps // 100
        rel_se = float(np.sqrt(2.0 / max(n_blocks - 1, 1)))   # relative SE of a variance from n_blocks block means

        def vxt(sigma, ms):
            return float(f"{sigma ** 2 * args.stat_steps * ms / 1e3:.6g}")
        s64 = stats["fp64"]["sigma_bar"]
        head["var_x_time"] = vxt(s64, head["ms_per_step"])
        for vname, v in variants.items():
            prec = vname.split("+")[0]
            src = stats.get(prec) if prec != "fp64" else stats["fp64"]
            if src is None or "+gaunt" in vname or "+breit" in vname:
                continue
            v["var_x_time"] = vxt(src["sigma_bar"], v["ms_per_step"])
            if prec != "fp64":
                v["systematic"] = {k: x for k, x in src.items() if k not in ("series", "steps")}
        stat_summary = {"steps": args.stat_steps, "n_b": 100, "e2_mean": stats["fp64"]["e2_mean"],
                        "sigma_bar": s64, "var_x_time_rel_se": round(rel_se, 3),
                        "projections": N_PROJ}
    else:
        stat_summary = None

    dom_key = max(head["dispatch"], key=lambda k: head["dispatch"][k]["avg_us"] * head["dispatch"][k]["launches_per_step"])
    dom = head["dispatch"][dom_key]
    kernel_names = {"green_gemm": "green_contract_kernel<double, NT, true, false> (FP64 Green's GEMMs + contraction "
                                  "+ adjoint contraction)",
                    "adj_gemm": "grad_gemm_kernel<NT, double2> (FP64 adjoint GEMM, NT = 2 tau per dispatch)"}
    roofline = {"bound": "mfma", "achieved": dom["tflops"], "peak": PEAK_TFLOPS[dom["operands"]], "unit": "TFLOP/s",
                "frac": dom["peak_frac"], "traffic": recorded_traffic(dom_key, name, "fp64"),
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "kernel": kernel_names.get(dom_key, dom_key), "avg_us": dom["avg_us"],
                "launches_per_step": dom["launches_per_step"], "flops_per_launch": dom["flops_per_launch"],
                "timed_launches": int(round(dom["launches_per_step"] * K))}
    cpu = cpu_baseline(inp, wk0, key, state["delta"], args.cpu_seconds) if args.cpu_seconds > 0 else None
    def target(vname):
        v = variants.get(vname)
        if v is None:
            return None
        return {"steps_per_s": v["steps_per_s"], "speedup_vs_fp64_grad": v["speedup_vs_fp64_grad"],
                "green_gemm_mfma_frac": v["dispatch"].get("green_gemm", {}).get("peak_frac"),
                "adj_gemm_mfma_frac": v["dispatch"].get("adj_gemm", {}).get("peak_frac"),
                "systematic": v.get("systematic")}
    out = {
        "metric": METRIC, "value": round(sps, 3), "unit": "MC steps/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{name} {WORKLOADS[name]}", "m": inp.m, "n_tau": inp.n_tau,
                   "n_L": inp.n_L, "n_S": inp.n_S, "n_occ": inp.n_occ, "n_vir": inp.n_vir,
                   "precision": "fp64", "grad": True},
        "var_x_time": head.get("var_x_time"), "var_x_time_unit": "Eh^2 s",
        "e2_mean": None if stats is None else stats["fp64"]["e2_mean"],
        "sigma_bar": None if stats is None else stats["fp64"]["sigma_bar"],
        "statistics": stat_summary,
        "roofline": roofline,
        "kernels": head["kernels"], "dispatch": head["dispatch"],
        "variants": variants,
        # the mixed-precision paths with gradients (16-bit Green's-function and adjoint GEMMs)
        "target_path": {k: target(k) for k in ("bf16+grad", "fp16+grad") if k in variants},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def replay_values(inp, precision, state, K, W=10):
    """K steps (no gradients) of the burned-in trajectory; returns (elapsed s
    of the K steps, per-step direct / exchange / total averaged over tau [K, 3])."""
    import torch

    from paper_2203_05632_amd import Context
    ctx = Context.from_inputs(inp, precision=precision)
    wk, w = state["wk"].clone(), state["w"].clone()
    key, delta, step = state["key"], state["delta"], state["step"]
    tau = torch.zeros(inp.n_tau, dtype=torch.float64, device="cuda")
    hist = torch.zeros((K + W, inp.n_tau, 3), dtype=torch.float64, device="cuda")
    for i in range(W):
        ctx.advance(wk, w, key, step + i, delta, tau)
        ctx.step(wk, tau, hist[i])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(W, W + K):
        ctx.advance(wk, w, key, step + i, delta, tau)
        ctx.step(wk, tau, hist[i])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.close()
    return el, hist[W:].mean(dim=1).cpu().numpy()


FINITE_VARIANCE_EXPONENTS = (0.3, 1.2)


def study_convergence(args):
    """Redundant walkers (Sec. III, Eq. redundant): every step uses all
    m(m-1)/2 pairs of m walkers, so sigma_bar at fixed N falls roughly like
    1/m while the cost of a step grows like m^2 (Figs. 1-2 of the paper show
    sigma_bar and the error against the number of steps for several m).  For
    m = 8 ... 512 on the tiny two-nucleus system (whose deterministic E2 is
    stored in tests/golden/c0_narrow_e2.json) and on the 340-spinor
    three-nucleus shapes, both with basis exponents in [0.3, 1.2] (finite
    variance with the Table 1 weight function; with the full exponent range
    and synthetic orbitals the estimator is heavy-tailed), one FP64 chain of
    `max(--steps, 5000)` steps after 300 steps of burn-in: I_N and sigma_bar_N
    (blocking, N_b = 100) of the direct, exchange and total parts at
    N = 500 ... K, the error of the total against the deterministic value
    where it exists, steps/s and var x time."""
    import numpy as np

    from paper_2203_05632_amd import blocking_sigma
    from synth import initial_walkers, make_inputs
    with open(os.path.join(ROOT, "tests", "golden", "c0_narrow_e2.json")) as fh:
        ref = json.load(fh)
    K = max(args.steps, 5000)
    marks = [n for n in (500, 1000, 2000, 3000, 4000, 5000, 10000, 20000) if n <= K]
    out = {"study": "redundant-walker convergence: I_N and sigma_bar_N vs N for several m (FP64)",
           "n_b": 100, "steps": K, "burn_in": 300, "exponent_range": FINITE_VARIANCE_EXPONENTS, "workloads": []}
    for wl, label, e_ref in (("C0", "tiny: 2 nuclei, 12 L / 32 S primitives, 4 occupied / 16 virtual spinors, 1 tau",
                              ref["total"]),
                             ("C1", "3 nuclei, 200 L / 460 S primitives, 40 occupied / 300 virtual spinors, 2 tau",
                              None)):
        rows = []
        base = make_inputs(wl, exp_range=FINITE_VARIANCE_EXPONENTS)
        for m in (8, 16, 32, 64, 128, 256, 512):
            inp = base.with_(m=m)
            state = burn_in(inp, initial_walkers(inp), (1, m), 300)
            el, vals = replay_values(inp, "fp64", state, K)
            curve = []
            for n in marks:
                sb = blocking_sigma(vals[:n], 100)
                pt = {"N": n, "I_N": [float(f"{v:.6g}") for v in vals[:n].mean(axis=0)],
                      "sigma_bar_N": [float(f"{v:.4g}") for v in sb]}
                if e_ref is not None:
                    pt["error_total"] = float(f"{vals[:n, 2].mean() - e_ref:.4g}")
                curve.append(pt)
            sb = float(blocking_sigma(vals[:, 2], 100))
            rows.append({"m": m, "pairs": m * (m - 1) // 2, "steps_per_s": round(K / el, 1),
                         "var_per_step": float(f"{sb * sb * K:.4g}"), "var_x_time": float(f"{sb * sb * el:.4g}"),
                         "curve": curve})
            progress(f"convergence {wl} m={m}: {K / el:.0f} steps/s, I={vals[:, 2].mean():.5g} +- {sb:.3g}")
        out["workloads"].append({"workload": wl, "shapes": label, "e2_deterministic": e_ref, "rows": rows})
    return out


def study_scaling(args):
    """Cost of the method against system size (Sec. IV, Figs. 3-4 of the
    paper: wall time to reach sigma_bar/|E2| = 0.1 against the number of
    basis functions and of electrons).  Two synthetic ladders on the
    three-nucleus shapes with basis exponents in [0.3, 1.2], one tau per step:
      n_bas: (s, p, d) shells x 4 ... 60 (40 ... 600 L primitives), 20
             occupied spinors, n_L - 20 virtual (as many spinors as L
             primitives: the narrow exponent range leaves the basis too close
             to linear dependence for 2 n_L);
      n_occ: the 200-primitive L set, n_occ = 4 ... 120 occupied of 400 spinors.
    For m = 8 and 12 (the paper's) and 128, 512, FP64 (and BF16 at 512):
    time per step t, the per-step variance v = sigma_bar_N^2 N (blocking,
    N_b = 100) and the time to sigma_bar/|E2| = 0.1, v t / (0.1 E2)^2, with E2
    from the m = 512 FP64 run of the same point; then log-log slopes against
    n_b and n_occ."""
    import numpy as np

    from paper_2203_05632_amd import blocking_sigma
    from synth import initial_walkers, make_inputs
    runs = [(8, "fp64", 2000), (12, "fp64", 2000), (128, "fp64", 1000), (512, "fp64", 1000), (512, "bf16", 1000)]
    ladders = {
        "n_bas": [dict(shell_reps=r, n_occ=20, n_vir=10 * r - 20) for r in (4, 8, 12, 20, 40, 60)],
        "n_occ": [dict(n_occ=o, n_vir=400 - o) for o in (4, 10, 20, 40, 80, 120)],
    }
    out = {"study": "time to sigma_bar/|E2| = 0.1 vs basis size and occupied count", "n_b": 100,
           "exponent_range": FINITE_VARIANCE_EXPONENTS, "n_tau": 1, "ladders": {}}
    for lad, points in ladders.items():
        rows = []
        for kw in points:
            base = make_inputs("C1", exp_range=FINITE_VARIANCE_EXPONENTS, n_tau=1, **kw)
            row = {"n_L": base.n_L, "n_S": base.n_S, "n_b": base.n_b, "n_occ": base.n_occ, "n_vir": base.n_vir,
                   "runs": {}}
            for m, prec, K in runs:
                inp = base.with_(m=m)
                state = burn_in(inp, initial_walkers(inp), (2, m), 300)
                el, vals = replay_values(inp, prec, state, K)
                sb = float(blocking_sigma(vals[:, 2], 100))
                row["runs"][f"m{m}_{prec}"] = {"steps": K, "ms_per_step": round(1e3 * el / K, 4),
                                               "e2_mean": float(f"{vals[:, 2].mean():.6g}"),
                                               "sigma_bar": float(f"{sb:.4g}"),
                                               "var_per_step": float(f"{sb * sb * K:.4g}")}
            e2 = row["runs"]["m512_fp64"]["e2_mean"]
            row["e2_reference"] = e2
            for r in row["runs"].values():
                r["time_to_0.1_s"] = float(f"{r['var_per_step'] * r['ms_per_step'] / 1e3 / (0.1 * e2) ** 2:.4g}")
            rows.append(row)
            progress(f"scaling {lad} n_L={base.n_L} n_occ={base.n_occ}: "
                     + ", ".join(f"{k} {v['ms_per_step']} ms, t(0.1) {v['time_to_0.1_s']} s"
                                 for k, v in row["runs"].items()))
        xs = np.log([r["n_b"] if lad == "n_bas" else r["n_occ"] for r in rows])
        slopes = {}
        for key in rows[0]["runs"]:
            for q in ("ms_per_step", "time_to_0.1_s"):
                ys = np.log([r["runs"][key][q] for r in rows])
                slopes[f"{key}_{q}"] = round(float(np.polyfit(xs, ys, 1)[0]), 3)
        out["ladders"][lad] = {"rows": rows, "loglog_slopes_vs_" + ("n_b" if lad == "n_bas" else "n_occ"): slopes}
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
        rows.append({"chains": k, "steps_total": k * (K // 100) * 100,
                     "steps_per_s": round(k * (K // 100) * 100 / el, 1),
                     "e2_merged": float(f"{res.mean[2]:.6g}"), "sigma_merged": float(f"{res.sigma[2]:.4g}")})
        progress(f"chains k={k}: {rows[-1]}")
        for ch in chains:
            ch.ctx.close()
    return {"study": "independent chains on concurrent streams", "workload": f"C1 {WORKLOADS['C1']}",
            "precision": "fp64", "rows": rows}


if __name__ == "__main__":
    main()
