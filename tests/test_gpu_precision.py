"""Low-precision operand modes (FP32, BF16, FP16 MFMA operands, FP32
accumulation; scalings, weights and sums in FP64, the pair contraction in
FP64 (FP32 mode) or FP32 (BF16 / FP16 modes)).

* Per step at fixed walkers and tau: deviation from the FP64 oracle, measured
  on the scale of the pair terms (mean |pair term|), within a bound set by the
  operand precision.  In the BF16 / FP16 modes every Green's-function operand
  (spinor value times sqrt(exp(+-eps tau))) is rounded once to the operand
  type (the spinor GEMM -- split BF16 when it has a 128x128 tile per CU, FP32
  below that -- adds at most about 2^-16), and a pair term has
  degree 8 in the spinor values: bound 8 u for unit roundoff u = 2^-8 (BF16),
  2^-11 (FP16).  FP32 mode: bound 1e-6 (about 17 u).
* Over a chain (1000 steps of the 340-spinor workload and of the 980-spinor
  precision workload): the systematic error -- mean over steps of the paired
  difference low - FP64 on the same walker trajectory (valid because the
  walker weights do not depend on the operand precision) -- must stay below
  1% of the FP64 estimator's blocking standard error.
* Gradients with low-precision G tiles against the FP64 gradients.
"""
import numpy as np
import pytest
import torch

from gpu_util import dev, requires_gpu
from oracle import integrand as oi
from oracle.blocking import blocking
from oracle.weights import n_g, tau_lambda
from synth import initial_walkers, make_inputs

pytestmark = [pytest.mark.gpu, requires_gpu]
BOUND = {"fp32": 1e-6, "bf16": 8 * 2.0 ** -8, "fp16": 8 * 2.0 ** -11}


def _ctx(inp, **kw):
    from paper_2203_05632_amd import Context
    return Context.from_inputs(inp, **kw)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("name,over,taus", [("C0", dict(n_tau=2), [0.3, 1.4]),
                                             ("C0", dict(m=13, n_occ=6, n_vir=10, n_tau=3), [0.1, 0.6, 3.0]),
                                             ("C1", dict(), [0.2, 0.9]),
                                             # 273 (tau, 16-walker tile pair) items: the BF16 / FP16 modes take
                                             # the 128x128-tile kernel; m = 200 leaves a half-filled last tile
                                             ("C1", dict(m=200, n_tau=3), [0.15, 0.6, 2.0]),
                                             # one tau per step: 276 tile pairs of 16 walkers (m = 360, a
                                             # half-filled last tile) still take the 128x128-tile kernel
                                             ("C0", dict(m=360, n_occ=6, n_vir=10, n_tau=1), [0.4]),
                                             # 1440 points: the split-BF16 spinor GEMM has 2 x 11 x 12 = 264
                                             # 128x128 tiles (>= one per two CUs) and runs; at the sizes
                                             # above the BF16 / FP16 modes take the FP32 spinor kernel
                                             ("C1", dict(m=720, n_tau=1), [0.5])])
def test_low_precision_step_near_oracle(prec, name, over, taus):
    inp = make_inputs(name, **over)
    wk = initial_walkers(inp)
    ctx = _ctx(inp, precision=prec)
    e2 = torch.zeros((len(taus), 3), dtype=torch.float64, device="cuda")
    ctx.step(dev(wk), dev(taus), e2)
    got = e2.cpu().numpy()
    res, pairs = oi.step_estimate(inp, wk, np.array(taus), tau_lambda(inp.eps, inp.n_occ),
                                  n_g(inp.nuc_xyz, inp.wfn), return_pairs=True)
    ref = res.numpy()
    for t in range(len(taus)):
        scale = float(pairs[t].real.abs().mean())
        err = np.max(np.abs(got[t] - ref[t])) / scale
        print(f"{prec} {name} {over} tau={taus[t]}: error / pair scale = {err:.3e}", flush=True)
        assert err < BOUND[prec]


def _chain(name, n_burn, n, delta, key):
    """One trajectory evaluated in every mode on the same walkers and tau
    (the walker weights do not depend on the operand precision)."""
    from paper_2203_05632_amd import Context
    inp = make_inputs(name)
    ctxs = {p: Context.from_inputs(inp, precision=p) for p in ("fp64", "fp32", "bf16", "fp16")}
    drv = ctxs["fp64"]
    wk = dev(initial_walkers(inp))
    w = torch.zeros(inp.m, dtype=torch.float64, device="cuda")
    drv.pair_weights(wk, w)
    tau = torch.zeros(inp.n_tau, dtype=torch.float64, device="cuda")
    for s in range(n_burn):
        drv.metropolis(wk, w, key, s, delta)
    hist = {p: torch.zeros((n, inp.n_tau, 3), dtype=torch.float64, device="cuda") for p in ctxs}
    for i in range(n):
        drv.advance(wk, w, key, n_burn + i, delta, tau)
        for p, c in ctxs.items():
            c.step(wk, tau, hist[p][i])
    torch.cuda.synchronize()
    return {p: h.mean(dim=1).cpu().numpy()[:, 2] for p, h in hist.items()}


@pytest.fixture(scope="module")
def chain_runs():
    """The 340-spinor workload (m = 128, 2 tau per step): 1000 steps."""
    return _chain("C1", 200, 1000, 0.45, (1, 0))


@pytest.fixture(scope="module")
def chain_runs_c3():
    """The precision workload (980 spinors, m = 256, 1 tau per step): 1000 steps."""
    return _chain("C3", 100, 1000, 0.3, (2, 0))


def _check_systematic(runs, prec, label):
    ref = runs["fp64"]
    d = runs[prec] - ref
    _, sbar = blocking(ref, 100)
    mean_d = float(d.mean())
    _, se_d = blocking(d, 100)
    print(f"{label} {prec}: systematic {mean_d:.3e} +- {se_d:.3e}, sigma_bar(FP64) {sbar:.3e}, "
          f"ratio {abs(mean_d) / sbar:.2e}", flush=True)
    assert abs(mean_d) < 0.01 * sbar


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_systematic_error_below_one_percent_of_sigma(chain_runs, prec):
    _check_systematic(chain_runs, prec, "C1")


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_systematic_error_below_one_percent_of_sigma_precision_workload(chain_runs_c3, prec):
    _check_systematic(chain_runs_c3, prec, "C3")


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("name,over,taus", [("C1", dict(), [0.3, 1.0]),
                                             ("C0", dict(m=13, n_occ=6, n_vir=10, n_tau=3), [0.2, 0.7, 2.5]),
                                             ("C1", dict(m=200, n_tau=3), [0.15, 0.6, 2.0]),
                                             ("C0", dict(m=360, n_occ=6, n_vir=10, n_tau=1), [0.4]),
                                             ("C1", dict(m=720, n_tau=1), [0.5])])
def test_low_precision_gradients_near_fp64(prec, name, over, taus):
    """FP32 mode keeps an FP64 adjoint GEMM; BF16 and FP16 modes run the
    adjoint GEMM on BF16 operands (adjoint blocks and psi S_t)."""
    inp = make_inputs(name, **over)
    wk = dev(initial_walkers(inp))
    taus = dev(taus)
    out = {}
    for p in ("fp64", prec):
        ctx = _ctx(inp, precision=p, want_grad=True)
        e2 = torch.zeros((inp.n_tau, 3), dtype=torch.float64, device="cuda")
        ge = torch.zeros(inp.n_sp, dtype=torch.float64, device="cuda")
        gc = torch.zeros((2, inp.n_b, inp.n_sp), dtype=torch.complex128, device="cuda")
        ctx.step(wk, taus, e2, grad_eps=ge, grad_coeffs=gc)
        torch.cuda.synchronize()
        out[p] = (ge.cpu().numpy(), gc.cpu().numpy())
    for a, b in zip(out[prec], out["fp64"]):
        err = np.max(np.abs(a - b)) / np.max(np.abs(b))
        print(f"{prec} {name} {over}: gradient max-norm relative deviation {err:.3e}", flush=True)
        assert err < (1e-5 if prec == "fp32" else 0.01)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_set_coefficients_refreshes_low_precision_operands(prec):
    """After mcmp2_set_coefficients the step equals, bit for bit, the step of
    a context built with the new coefficients (the split BF16 coefficient
    copy of the BF16 / FP16 modes is rebuilt on the context's stream)."""
    inp = make_inputs("C1", n_tau=2)
    wk = dev(initial_walkers(inp))
    taus = dev([0.3, 1.1])
    rng = np.random.default_rng(11)
    C2 = inp.coeffs * (1.0 + 0.05 * rng.standard_normal(inp.coeffs.shape))
    eps2 = inp.eps.copy()
    eps2[0] -= 0.01   # the lowest occupied energy: lambda (HOMO-LUMO gap) unchanged
    a = _ctx(inp, precision=prec)
    a.set_coefficients(torch.tensor(C2, device="cuda"), torch.tensor(eps2, device="cuda"))
    ea = torch.zeros((2, 3), dtype=torch.float64, device="cuda")
    a.step(wk, taus, ea)
    from paper_2203_05632_amd import Context
    b = Context(inp.nuc_xyz, inp.wfn, inp.n_L, inp.n_S, inp.prim_xyz, inp.prim_exp, inp.prim_lxyz, inp.prim_norm,
                C2, eps2, inp.n_occ, inp.n_vir, inp.m, 2, precision=prec)
    assert b.lam == a.lam   # lambda is frozen at init; this change of energies leaves it unchanged
    eb = torch.zeros((2, 3), dtype=torch.float64, device="cuda")
    b.step(wk, taus, eb)
    torch.cuda.synchronize()
    assert np.array_equal(ea.cpu().numpy(), eb.cpu().numpy())
