"""Parity at the largest workload's full size and launch configuration (6
nuclei, 1000 L / 2300 S primitives, 120 occupied / 1500 virtual spinors,
m = 512 walker pairs, 4 tau per step -- the shapes bench.py times): the FP64
kernels with two tau per block and the LDS-tiled spinor GEMM, the BF16 / FP16
128x128-tile Green's kernel and split-BF16 spinor GEMM, the FP32 path, and the
Breit contraction, each against the FP64 oracle on the same walkers and tau.

Gradients at this size are checked through properties that hold at any size:
the FP64 gradients (Coulomb and Breit interaction) against central finite
differences of the (oracle-pinned) FP64 forward step along random directions,
with walkers and tau fixed and lambda frozen; the BF16 gradients against the
FP64 ones.
"""
import numpy as np
import pytest
import torch

from gpu_util import dev, rel_err, requires_gpu
from oracle import integrand as oi
from oracle.weights import n_g, tau_lambda
from synth import initial_walkers, make_inputs

pytestmark = [pytest.mark.gpu, requires_gpu]
TAUS = [0.12, 0.5, 1.3, 3.1]
# FP64: the parity bar.  FP32 / BF16 / FP16: the regression guards of the
# reduced-precision step tests (three times the largest deviation measured
# there); measured here: FP32 6e-7, BF16 7e-4, FP16 9e-5 of the pair scale.
BOUND = {"fp64": 1e-10, "fp32": 1e-6, "bf16": 1e-2, "fp16": 5e-4}


@pytest.fixture(scope="module")
def c4():
    inp = make_inputs("C4")
    wk = initial_walkers(inp)
    lam, Ng = tau_lambda(inp.eps, inp.n_occ), n_g(inp.nuc_xyz, inp.wfn)
    res, pairs = oi.step_estimate(inp, wk, np.array(TAUS), lam, Ng, return_pairs=True)
    scale = np.array([float(p.real.abs().mean()) for p in pairs])
    return inp, wk, res.numpy(), scale


def _ctx(inp, **kw):
    from paper_2203_05632_amd import Context
    return Context.from_inputs(inp, **kw)


def _step(ctx, wk, taus, **g):
    e2 = torch.zeros((len(taus), 3), dtype=torch.float64, device="cuda")
    ctx.step(dev(wk), dev(taus), e2, **g)
    torch.cuda.synchronize()
    return e2.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "fp16"])
def test_full_size_step_matches_oracle(c4, prec):
    inp, wk, ref, scale = c4
    got = _step(_ctx(inp, precision=prec), wk, TAUS)
    for t in range(len(TAUS)):
        err = rel_err(got[t], ref[t], norm=scale[t])
        print(f"{prec} C4 tau={TAUS[t]}: error / scale = {err:.3e}", flush=True)
        assert err < BOUND[prec]


@pytest.fixture(scope="module")
def c4_breit(c4):
    inp, wk, _, _ = c4
    taus = [0.4]
    res, pairs = oi.step_estimate(inp, wk, np.array(taus), tau_lambda(inp.eps, inp.n_occ),
                                  n_g(inp.nuc_xyz, inp.wfn), return_pairs=True, interaction="breit")
    return taus, res.numpy(), float(pairs[0].real.abs().mean())


@pytest.mark.parametrize("prec", ["fp64", "bf16", "fp16"])
def test_full_size_breit_matches_oracle(c4, c4_breit, prec):
    inp, wk, _, _ = c4
    taus, ref, scale = c4_breit
    ctx = _ctx(inp, precision=prec, n_tau_max=1)
    ctx.set_interaction("breit")
    got = _step(ctx, wk, taus)
    err = rel_err(got[0], ref[0], norm=scale)
    print(f"breit {prec} C4: error / scale = {err:.3e}", flush=True)
    assert err < BOUND[prec]


def _value(ctx, wk, taus):
    return float(_step(ctx, wk, taus)[:, 2].mean())


@pytest.mark.parametrize("kind", ["coulomb", "breit"])
def test_full_size_fp64_gradients_match_finite_differences(c4, kind):
    inp, wk, _, _ = c4
    ctx = _ctx(inp, want_grad=True)
    ctx.set_interaction(kind)
    ge = torch.zeros(inp.n_sp, dtype=torch.float64, device="cuda")
    gc = torch.zeros((2, inp.n_b, inp.n_sp), dtype=torch.complex128, device="cuda")
    _step(ctx, wk, TAUS, grad_eps=ge, grad_coeffs=gc)
    ge, gc = ge.cpu().numpy(), gc.cpu().numpy()
    rng = np.random.default_rng(5)
    eps0 = np.asarray(inp.eps, dtype=np.float64)
    C0 = np.asarray(inp.coeffs, dtype=np.complex128)
    h = 1e-6
    # direction in eps
    d = rng.standard_normal(inp.n_sp)
    vals = []
    for sgn in (1.0, -1.0):
        e = dev(eps0 + sgn * h * d)  # referenced until the step that reads it has finished
        ctx.set_coefficients(eps=e)
        vals.append(_value(ctx, wk, TAUS))
    e = dev(eps0)
    ctx.set_coefficients(eps=e)
    fd = (vals[0] - vals[1]) / (2 * h)
    an = float(ge @ d)
    print(f"{kind} eps direction: analytic {an:.12e} fd {fd:.12e}", flush=True)
    assert abs(an - fd) <= 1e-6 * float(np.abs(ge) @ np.abs(d))
    # direction in the coefficients
    D = rng.standard_normal(C0.shape) + 1j * rng.standard_normal(C0.shape)
    vals = []
    for sgn in (1.0, -1.0):
        c = dev(C0 + sgn * h * D, dtype=torch.complex128)
        ctx.set_coefficients(coeffs=c)
        vals.append(_value(ctx, wk, TAUS))
    fd = (vals[0] - vals[1]) / (2 * h)
    an = float(np.real(np.vdot(gc, D)))  # Re(conj(g) . D) with g = dV/dRe C + i dV/dIm C
    print(f"{kind} coefficient direction: analytic {an:.12e} fd {fd:.12e}", flush=True)
    assert abs(an - fd) <= 1e-6 * float(np.abs(gc).ravel() @ np.abs(D).ravel())


def test_full_size_bf16_gradients_near_fp64(c4):
    inp, wk, _, _ = c4
    out = {}
    for p in ("fp64", "bf16"):
        ctx = _ctx(inp, precision=p, want_grad=True)
        ge = torch.zeros(inp.n_sp, dtype=torch.float64, device="cuda")
        gc = torch.zeros((2, inp.n_b, inp.n_sp), dtype=torch.complex128, device="cuda")
        _step(ctx, wk, TAUS, grad_eps=ge, grad_coeffs=gc)
        out[p] = (ge.cpu().numpy(), gc.cpu().numpy())
        ctx.close()
    for a, b in zip(out["bf16"], out["fp64"]):
        err = np.max(np.abs(a - b)) / np.max(np.abs(b))
        print(f"bf16 C4 gradient max-norm relative deviation {err:.3e}", flush=True)
        assert err < 0.01
