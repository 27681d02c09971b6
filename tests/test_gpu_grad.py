"""GPU parity of the hand-written adjoint: dV/d eps and dV/dC from the HIP
library against reverse-mode differentiation of the FP64 oracle on identical
walkers and tau samples (V = mean over tau of the step's total), plus the
torch.autograd.Function wrapper and finite differences through the library.

Tolerance: 1e-9 relative in the max norm of each gradient array.
"""
import numpy as np
import pytest
import torch

from gpu_util import dev, requires_gpu
from oracle.gradient import step_value_and_grad
from oracle.weights import n_g, tau_lambda
from synth import initial_walkers, make_inputs

pytestmark = [pytest.mark.gpu, requires_gpu]
TOL = 1e-9


def _ctx(inp, **kw):
    from paper_2203_05632_amd import Context
    return Context.from_inputs(inp, want_grad=True, **kw)


def _gpu_grad(ctx, inp, wk, taus):
    e2 = torch.zeros((len(taus), 3), dtype=torch.float64, device="cuda")
    ge = torch.zeros(inp.n_sp, dtype=torch.float64, device="cuda")
    gc = torch.zeros((2, inp.n_b, inp.n_sp), dtype=torch.complex128, device="cuda")
    ctx.step(dev(wk), dev(taus), e2, grad_eps=ge, grad_coeffs=gc)
    torch.cuda.synchronize()
    return e2.cpu().numpy(), ge.cpu().numpy(), gc.cpu().numpy()


def _normrel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


CASES = [
    ("C0", dict(n_tau=2), [0.3, 1.1]),
    ("C0", dict(m=13, n_occ=6, n_vir=10, n_tau=3), [0.2, 0.7, 2.5]),   # ragged tiles, odd tau count
    ("C1", dict(), [0.17, 0.83]),
    # 980 spinors, 600 + 1380 primitives: 512 tiles of 64 x 64, the tiled coefficient-gradient kernel
    ("C3", dict(m=16, n_tau=1), [0.4]),
]


@pytest.mark.parametrize("name,over,taus", CASES)
def test_gradients_match_oracle_autograd(name, over, taus):
    inp = make_inputs(name, **over)
    wk = initial_walkers(inp)
    ctx = _ctx(inp, n_tau_max=len(taus))
    e2, ge, gc = _gpu_grad(ctx, inp, wk, np.array(taus))
    parts, val, oge, ogc = step_value_and_grad(inp, wk, np.array(taus), tau_lambda(inp.eps, inp.n_occ),
                                               n_g(inp.nuc_xyz, inp.wfn))
    print(f"case {name} {over}: value gpu {e2[:, 2].mean():.12e} oracle {val:.12e}; "
          f"eps err {_normrel(ge, oge):.2e} coef err {_normrel(gc, ogc):.2e}", flush=True)
    assert abs(e2[:, 2].mean() - val) <= 1e-10 * max(abs(val), np.abs(parts).max())
    assert _normrel(ge, oge) < TOL
    assert _normrel(gc, ogc) < TOL


def test_gradient_invariants_on_gpu():
    inp = make_inputs("C1")
    wk = initial_walkers(inp)
    ctx = _ctx(inp)
    e2, ge, gc = _gpu_grad(ctx, inp, wk, np.array([0.4, 1.3]))
    V = e2[:, 2].mean()
    assert abs(ge.sum()) <= 1e-10 * np.abs(ge).sum()
    no = inp.n_occ
    occ = np.sum((inp.coeffs.conj() * gc)[:, :, :no]).real
    vir = np.sum((inp.coeffs.conj() * gc)[:, :, no:]).real
    scale = np.abs(inp.coeffs.conj() * gc).sum()
    assert abs(occ - 4 * V) <= 1e-10 * scale
    assert abs(vir - 4 * V) <= 1e-10 * scale


def test_coefficient_gradient_phase_invariance_on_gpu():
    """V is invariant under psi_k -> e^{i theta} psi_k (every spinor enters G
    as psi psi^dagger), so Im sum_{s,mu} conj(C[s][mu][k]) Cbar[s][mu][k] = 0
    for each k; checked in every precision mode."""
    inp = make_inputs("C1")
    wk = initial_walkers(inp)
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-6), ("bf16", 1e-2), ("fp16", 1e-2)):
        ctx = _ctx(inp, precision=prec)
        _, _, gc = _gpu_grad(ctx, inp, wk, np.array([0.4, 1.3]))
        per_k = np.sum(inp.coeffs.conj() * gc, axis=(0, 1))
        scale = np.abs(inp.coeffs.conj() * gc).sum(axis=(0, 1)).max()
        print(f"{prec}: max |Im sum conj(C) Cbar| / scale = {np.abs(per_k.imag).max() / scale:.2e}", flush=True)
        assert np.abs(per_k.imag).max() <= tol * scale


def test_forward_identical_with_and_without_gradient():
    inp = make_inputs("C1")
    wk = initial_walkers(inp)
    ctx = _ctx(inp)
    taus = np.array([0.5, 0.9])
    e2a = torch.zeros((2, 3), dtype=torch.float64, device="cuda")
    ctx.step(dev(wk), dev(taus), e2a)
    e2b, _, _ = _gpu_grad(ctx, inp, wk, taus)
    assert np.array_equal(e2a.cpu().numpy(), e2b)


def test_autograd_function_and_finite_differences():
    from paper_2203_05632_amd import mcmp2_value
    inp = make_inputs("C0", n_tau=2)
    wk = dev(initial_walkers(inp))
    taus = dev([0.35, 1.2])
    ctx = _ctx(inp)
    C = torch.tensor(inp.coeffs, dtype=torch.complex128, device="cuda", requires_grad=True)
    e = torch.tensor(inp.eps, dtype=torch.float64, device="cuda", requires_grad=True)
    V = mcmp2_value(C, e, wk, taus, ctx)
    (2.0 * V).backward()
    gC, ge = C.grad.clone(), e.grad.clone()
    h = 1e-5
    rng = np.random.default_rng(7)
    with torch.no_grad():
        for _ in range(4):
            k = int(rng.integers(inp.n_sp))
            ep, em = e.detach().clone(), e.detach().clone()
            ep[k] += h
            em[k] -= h
            fd = (mcmp2_value(C.detach(), ep, wk, taus, ctx) - mcmp2_value(C.detach(), em, wk, taus, ctx)) / (2 * h)
            assert abs(2.0 * fd.item() - ge[k].item()) <= 1e-6 * ge.abs().max().item()
            s, mu = int(rng.integers(2)), int(rng.integers(inp.n_b))
            for unit, part in ((1.0, "re"), (1j, "im")):
                Cp, Cm = C.detach().clone(), C.detach().clone()
                Cp[s, mu, k] += unit * h
                Cm[s, mu, k] -= unit * h
                fd = (mcmp2_value(Cp, e.detach(), wk, taus, ctx) - mcmp2_value(Cm, e.detach(), wk, taus, ctx)) / (2 * h)
                an = gC[s, mu, k].real if part == "re" else gC[s, mu, k].imag
                assert abs(2.0 * fd.item() - an.item()) <= 1e-6 * gC.abs().max().item()


def test_autograd_function_on_a_side_stream_context():
    """A context on its own stream gives the value and gradients of a
    default-stream context bit for bit, with inputs produced on the current
    stream just before the call (the function orders the two streams)."""
    from paper_2203_05632_amd import mcmp2_value
    inp = make_inputs("C1")
    wk = dev(initial_walkers(inp))
    taus = dev([0.35, 1.2])
    side = torch.cuda.Stream()
    out = []
    for ctx in (_ctx(inp), _ctx(inp, stream=side)):
        # inputs written by a kernel on the current stream right before the call
        C = torch.tensor(inp.coeffs, dtype=torch.complex128, device="cuda") * 1.0
        e = torch.tensor(inp.eps, dtype=torch.float64, device="cuda") * 1.0
        C.requires_grad_(True)
        e.requires_grad_(True)
        V = mcmp2_value(C, e, wk, taus, ctx)
        V.backward()
        out.append((V.detach().clone(), C.grad.clone(), e.grad.clone()))
    torch.cuda.synchronize()
    e2 = torch.zeros((2, 3), dtype=torch.float64, device="cuda")
    _ctx(inp).step(wk, taus, e2)
    torch.cuda.synchronize()
    assert abs(out[0][0].item() - e2[:, 2].mean().item()) <= 1e-15 * abs(e2[:, 2].mean().item())
    for a, b in zip(out[0], out[1]):
        assert torch.equal(a, b)


def test_gradient_needs_want_grad():
    from paper_2203_05632_amd import Context, MCMP2Error
    inp = make_inputs("C0")
    ctx = Context.from_inputs(inp)
    e2 = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    ge = torch.zeros(inp.n_sp, dtype=torch.float64, device="cuda")
    with pytest.raises(MCMP2Error) as ei:
        ctx.step(dev(initial_walkers(inp)), dev([0.3]), e2, grad_eps=ge)
    assert ei.value.code == -4


@pytest.mark.parametrize("name,prec", [("C0", "fp64"), ("C1", "fp64"), ("C1", "fp32"),
                                       # 66 coefficient-gradient tiles: gradients staged, then added
                                       ("C1", "bf16"),
                                       # 1326 tiles: added to the sums in the kernel's epilogue
                                       ("C4", "bf16")])
def test_step_accumulate_equals_step_then_accumulate(name, prec):
    """The fused entry point leaves e2 and both compensated gradient sums bit
    for bit as step() followed by accumulate() of each gradient, over
    several steps with different walkers and tau."""
    inp = make_inputs(name)
    ctx = _ctx(inp, precision=prec)
    rng = np.random.default_rng(9)
    wk0 = initial_walkers(inp)
    n_tau = inp.n_tau

    def zeros(shape, dt=torch.float64):
        return torch.zeros(shape, dtype=dt, device="cuda")

    a = [zeros(inp.n_sp), zeros(inp.n_sp), zeros((2, inp.n_b, inp.n_sp), torch.complex128),
         zeros((2, inp.n_b, inp.n_sp), torch.complex128)]
    b = [x.clone() for x in a]
    ge, gc = zeros(inp.n_sp), zeros((2, inp.n_b, inp.n_sp), torch.complex128)
    for s in range(3):
        wk = dev(wk0 + 0.05 * s * rng.standard_normal(wk0.shape))
        taus = dev(rng.uniform(0.05, 2.0, n_tau))
        e2a, e2b = zeros((n_tau, 3)), zeros((n_tau, 3))
        ctx.step_accumulate(wk, taus, e2a, *a)
        ctx.step(wk, taus, e2b, grad_eps=ge, grad_coeffs=gc)
        ctx.accumulate(ge, b[0], b[1])
        ctx.accumulate(gc, b[2], b[3])
        torch.cuda.synchronize()
        assert torch.equal(e2a, e2b)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    assert float(a[0].abs().max()) > 0 and float(a[2].abs().max()) > 0


def test_step_accumulate_errors():
    from paper_2203_05632_amd import Context, MCMP2Error
    inp = make_inputs("C0")
    wk, taus = dev(initial_walkers(inp)), dev([0.4])
    e2 = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    acc = [torch.zeros(inp.n_sp, dtype=torch.float64, device="cuda") for _ in range(2)] + \
          [torch.zeros((2, inp.n_b, inp.n_sp), dtype=torch.complex128, device="cuda") for _ in range(2)]
    with pytest.raises(MCMP2Error) as ei:
        Context.from_inputs(inp).step_accumulate(wk, taus, e2, *acc)      # no want_grad
    assert ei.value.code == -4
    ctx = _ctx(inp, precision="bf16")
    ctx.set_interaction("breit")  # gradients with the Breit interaction in every mode
    ctx.step_accumulate(wk, taus, e2, *acc)
    torch.cuda.synchronize()
    assert float(acc[2].abs().max()) > 0
