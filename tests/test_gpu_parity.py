"""GPU parity: the HIP hot path through the C ABI against the FP64 oracle on
identical seeded walkers and tau samples.

Tolerance (FP64 path): 1e-10 relative per tau and per part (direct,
exchange, total).  The two sides sum the same terms in different orders
(MFMA K-loop, tiled pair sums, compensated reductions vs BLAS and a plain
mean), so differences are a few ulps of the largest partial sums; the bound
is taken relative to max(|value|, mean |pair term|) so that a per-step value
that cancels to near zero is compared on the scale of the terms that built it.
"""
import numpy as np
import pytest
import torch

from gpu_util import dev, rel_err, requires_gpu
from oracle import integrand as oi
from oracle import sampling as osamp
from oracle.weights import n_g, pair_weight, tau_lambda
from synth import initial_walkers, make_inputs

pytestmark = [pytest.mark.gpu, requires_gpu]
TOL = 1e-10


def _ctx(inp, **kw):
    from paper_2203_05632_amd import Context
    return Context.from_inputs(inp, **kw)


def _oracle_step(inp, wk, taus):
    Ng = n_g(inp.nuc_xyz, inp.wfn)
    lam = tau_lambda(inp.eps, inp.n_occ)
    res, pairs = oi.step_estimate(inp, wk, taus, lam, Ng, return_pairs=True)
    scale = np.array([float(p.real.abs().mean()) for p in pairs])
    return res.numpy(), scale


def _gpu_step(ctx, wk, taus):
    e2 = torch.zeros((len(taus), 3), dtype=torch.float64, device="cuda")
    ctx.step(dev(wk), dev(taus), e2)
    torch.cuda.synchronize()
    return e2.cpu().numpy()


CASES = [
    # name, overrides, taus
    ("C0", {}, [0.31]),
    ("C0", dict(n_tau=3), [0.0, 0.9, 4.5]),
    ("C0", dict(m=13, n_occ=6, n_vir=10), [0.2, 1.3]),          # ragged m, ragged K tails
    ("C0", dict(m=2, n_occ=2, n_vir=2), [0.5]),                 # one pair, minimal sizes
    ("C0", dict(m=37, n_occ=10, n_vir=22, n_tau=2), [0.05, 2.0]),
    ("C1", {}, [0.17, 0.83]),                                    # full C1 workload shape
]


@pytest.mark.parametrize("name,over,taus", CASES)
def test_step_matches_oracle(name, over, taus):
    over = dict(over)
    n_tau = max(len(taus), over.pop("n_tau", 1))
    inp = make_inputs(name, n_tau=n_tau, **over)
    wk = initial_walkers(inp)
    ctx = _ctx(inp, n_tau_max=n_tau)
    got = _gpu_step(ctx, wk, np.array(taus))
    ref, scale = _oracle_step(inp, wk, taus)
    print(f"case {name} {over} taus={taus}\n gpu={got}\n ref={ref}", flush=True)
    for t in range(len(taus)):
        assert rel_err(got[t], ref[t], norm=scale[t]) < TOL


def test_constants_match_oracle():
    inp = make_inputs("C1")
    ctx = _ctx(inp)
    assert abs(ctx.lam - tau_lambda(inp.eps, inp.n_occ)) == 0.0
    assert abs(ctx.Ng - n_g(inp.nuc_xyz, inp.wfn)) < 1e-13 * abs(ctx.Ng)


def test_step_is_bitwise_deterministic():
    inp = make_inputs("C1")
    wk = initial_walkers(inp)
    ctx = _ctx(inp)
    a = _gpu_step(ctx, wk, np.array([0.4, 1.1]))
    b = _gpu_step(ctx, wk, np.array([0.4, 1.1]))
    assert np.array_equal(a, b)


def test_pair_weights_and_tau_sampler():
    inp = make_inputs("C1")
    ctx = _ctx(inp)
    wk = initial_walkers(inp)
    w = torch.zeros(inp.m, dtype=torch.float64, device="cuda")
    ctx.pair_weights(dev(wk), w)
    ref = pair_weight(wk[:, 0], wk[:, 1], inp.nuc_xyz, inp.wfn, ctx.Ng)
    assert rel_err(w.cpu().numpy(), ref) < 1e-13
    tau = torch.zeros(7, dtype=torch.float64, device="cuda")
    for step in (0, 1, 12345, 2**40 + 3):
        ctx.sample_tau((3, 4), step, tau)
        ref = osamp.sample_tau(np.array([3, 4], dtype=np.uint64), step, 7, ctx.lam)
        assert rel_err(tau.cpu().numpy(), ref) < 1e-14


def test_metropolis_trajectory_identical_to_oracle():
    """Walker positions are bit-identical to the oracle's for 1000 steps (the
    position update is exact IEEE arithmetic on identical Philox draws; the
    acceptance test compares weight ratios that agree to a few ulps)."""
    inp = make_inputs("C1")
    ctx = _ctx(inp)
    wk0 = initial_walkers(inp)
    key = (11, 3)
    wk = dev(wk0)
    w = torch.zeros(inp.m, dtype=torch.float64, device="cuda")
    ctx.pair_weights(wk, w)
    n_acc = torch.zeros(1, dtype=torch.int32, device="cuda")
    o_wk = wk0.copy()
    o_w = pair_weight(o_wk[:, 0], o_wk[:, 1], inp.nuc_xyz, inp.wfn, ctx.Ng)
    o_acc = 0
    keyu = np.array(key, dtype=np.uint64)
    for s in range(1000):
        ctx.metropolis(wk, w, key, s, 0.7, n_acc)
        o_wk, o_w, acc = osamp.metropolis_step(o_wk, o_w, keyu, s, 0.7, inp.nuc_xyz, inp.wfn, ctx.Ng)
        o_acc += int(acc.sum())
    torch.cuda.synchronize()
    assert np.array_equal(wk.cpu().numpy(), o_wk)
    assert int(n_acc.item()) == o_acc
    assert rel_err(w.cpu().numpy(), o_w) < 1e-12


def test_invalid_arguments_raise():
    from paper_2203_05632_amd import MCMP2Error
    inp = make_inputs("C0")
    ctx = _ctx(inp)
    e2 = torch.zeros((2, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(MCMP2Error) as ei:
        ctx.step(dev(initial_walkers(inp)), dev([0.1, 0.2]), e2)       # n_tau > n_tau_max
    assert ei.value.code == -1
    with pytest.raises(MCMP2Error):
        ctx.metropolis(dev(initial_walkers(inp)), torch.ones(inp.m, dtype=torch.float64, device="cuda"),
                       (0, 0), 0, -1.0)
    with pytest.raises(MCMP2Error):
        _ctx(inp.with_(m=1))
    with pytest.raises(KeyError):
        _ctx(inp, precision="fp8")


def test_advance_equals_metropolis_then_sample_tau():
    inp = make_inputs("C1")
    ctx = _ctx(inp)
    wk0 = dev(initial_walkers(inp))
    w0 = torch.zeros(inp.m, dtype=torch.float64, device="cuda")
    ctx.pair_weights(wk0, w0)
    a_wk, a_w, b_wk, b_w = wk0.clone(), w0.clone(), wk0.clone(), w0.clone()
    a_tau = torch.zeros(3, dtype=torch.float64, device="cuda")
    b_tau = torch.zeros(3, dtype=torch.float64, device="cuda")
    na = torch.zeros(1, dtype=torch.int32, device="cuda")
    nb = torch.zeros(1, dtype=torch.int32, device="cuda")
    for s in range(50):
        ctx.advance(a_wk, a_w, (5, 6), s, 0.6, a_tau, na)
        ctx.metropolis(b_wk, b_w, (5, 6), s, 0.6, nb)
        ctx.sample_tau((5, 6), s, b_tau)
    torch.cuda.synchronize()
    assert torch.equal(a_wk, b_wk) and torch.equal(a_w, b_w) and torch.equal(a_tau, b_tau)
    assert int(na.item()) == int(nb.item()) > 0


def test_accumulate_is_compensated():
    """Neumaier accumulation of many values of mixed magnitude matches
    math.fsum (exactly rounded) to a few ulps of the total."""
    import math
    inp = make_inputs("C0")
    ctx = _ctx(inp)
    rng = np.random.default_rng(3)
    steps = [rng.standard_normal(5) * 10.0 ** rng.integers(-8, 9, size=5) for _ in range(400)]
    s = torch.zeros(5, dtype=torch.float64, device="cuda")
    c = torch.zeros(5, dtype=torch.float64, device="cuda")
    for v in steps:
        ctx.accumulate(dev(v), s, c)
    got = (s + c).cpu().numpy()
    for i in range(5):
        ref = math.fsum(v[i] for v in steps)
        assert abs(got[i] - ref) <= 4 * np.spacing(abs(ref)) + 1e-300
    # both kernel paths: 16-byte aligned arrays with an odd length (pairs plus
    # a last element) and arrays offset by one double (element-wise path)
    n = 1001
    vals = [rng.standard_normal(n + 1) * 10.0 ** rng.integers(-8, 9, size=n + 1) for _ in range(60)]
    for off in (0, 1):
        sb = torch.zeros(n + 1, dtype=torch.float64, device="cuda")
        cb = torch.zeros(n + 1, dtype=torch.float64, device="cuda")
        for v in vals:
            src = dev(v)  # referenced until the accumulation that reads it has finished
            ctx.accumulate(src[off:off + n], sb[off:off + n], cb[off:off + n])
            torch.cuda.synchronize()
        got = (sb + cb).cpu().numpy()[off:off + n]
        ref = np.array([math.fsum(v[off + i] for v in vals) for i in range(n)])
        assert np.all(np.abs(got - ref) <= 4 * np.spacing(np.abs(ref)) + 1e-300)
        untouched = 0 if off == 1 else n  # the element outside the view stays zero
        assert float(sb[untouched].item()) == 0.0 and float(cb[untouched].item()) == 0.0
    # complex tensors are accumulated as interleaved doubles
    z = torch.zeros(3, dtype=torch.complex128, device="cuda")
    zc = torch.zeros(3, dtype=torch.complex128, device="cuda")
    ctx.accumulate(dev(np.array([1 + 2j, 3 - 1j, 0.5j]), torch.complex128), z, zc)
    ctx.accumulate(dev(np.array([1 + 2j, 3 - 1j, 0.5j]), torch.complex128), z, zc)
    assert np.allclose((z + zc).cpu().numpy(), [2 + 4j, 6 - 2j, 1j], rtol=0, atol=0)
