"""The chain driver on the GPU: parity of a whole run with the oracle chain,
bit-identical resume from a checkpoint, and independence of chains run
concurrently on separate streams."""
import numpy as np
import pytest
import torch

from gpu_util import requires_gpu
from synth import initial_walkers, make_inputs

pytestmark = [pytest.mark.gpu, requires_gpu]


def _chain(inp, key=(3, 1), want_grad=False, stream=None, **kw):
    from paper_2203_05632_amd import Chain, Context
    ctx = Context.from_inputs(inp, want_grad=want_grad, stream=stream, **kw)
    return Chain(ctx, initial_walkers(inp, chain=key[1]), key=key, delta=0.4, want_grad=want_grad)


def test_gpu_chain_matches_oracle_chain():
    """Whole run (fixed-delta moves, then 200 steps of move + tau + estimator):
    walker positions bit-identical, per-step values within 1e-10 of the
    oracle's chain on the same key."""
    from oracle.chain import Chain as OracleChain
    inp = make_inputs("C0", n_tau=2)
    key = (3, 1)
    ch = _chain(inp, key)
    ch.burn_in(50, adapt=False)
    ch.run(200, block=64)
    ref = OracleChain(inp, initial_walkers(inp, chain=1), key=key, delta=0.4)
    ref.burn_in(50, adapt=False)
    ref_vals = ref.run(200, n_tau=2)
    got = ch.series()
    scale = np.abs(ref_vals).max()
    print(f"max per-step deviation / max |value| = {np.abs(got - ref_vals).max() / scale:.2e}", flush=True)
    assert np.abs(got - ref_vals).max() <= 1e-10 * scale
    assert np.array_equal(ch.walkers.cpu().numpy(), ref.walkers)


@pytest.mark.parametrize("grad", [False, True])
def test_resume_from_checkpoint_is_bit_identical(tmp_path, grad):
    inp = make_inputs("C0", n_tau=2)
    a = _chain(inp, want_grad=grad)
    a.burn_in(100)
    a.run(240, block=100)
    b = _chain(inp, want_grad=grad)
    b.burn_in(100)
    b.run(120, block=100)
    path = str(tmp_path / "chain.npz")
    b.save(path)
    from paper_2203_05632_amd import Chain, Context
    c = Chain.load(Context.from_inputs(inp, want_grad=grad), path, want_grad=grad)
    c.run(120, block=100)
    assert np.array_equal(a.series(), c.series())
    assert np.array_equal(a.walkers.cpu().numpy(), c.walkers.cpu().numpy())
    ra, rc = a.result(), c.result()
    assert np.array_equal(ra.mean, rc.mean)
    if grad:
        assert np.array_equal(ra.grad_eps, rc.grad_eps) and np.array_equal(ra.grad_coeffs, rc.grad_coeffs)


def test_chains_on_concurrent_streams_match_sequential_runs():
    from paper_2203_05632_amd import merge
    inp = make_inputs("C0", n_tau=2)
    seq = []
    for c in range(3):
        ch = _chain(inp, key=(5, c))
        ch.burn_in(50)
        ch.run(150, block=50)
        seq.append(ch)
    streams = [torch.cuda.Stream() for _ in range(3)]
    par = [_chain(inp, key=(5, c), stream=streams[c]) for c in range(3)]
    for ch in par:
        ch.burn_in(50)
    for _ in range(3):          # interleave the chains' launches block by block
        for ch in par:
            ch.run(50, block=50)
    torch.cuda.synchronize()
    for s, p in zip(seq, par):
        assert np.array_equal(s.series(), p.series())
    m = merge([ch.result() for ch in par])
    assert m.steps == 450
    assert np.allclose(m.mean, np.mean([ch.result().mean for ch in par], axis=0))


@pytest.mark.parametrize("grad", [False, True])
def test_run_directory_resume_after_a_stop(tmp_path, grad):
    """A chain writing records and checkpoints into a run directory is
    stopped after its second block (a clean stop) and its context released;
    a fresh context resumes from the directory -- past a torn temporary file
    and a damaged newer checkpoint -- and ends bit for bit where an
    uninterrupted run ends: per-step series, walkers, gradient sums and the
    block records (except their wall-clock rates).  Whether the chain
    accumulates gradients comes from the checkpoint."""
    from paper_2203_05632_amd import Chain, Context
    from paper_2203_05632_amd.chain import checkpoint_path, read_records
    inp = make_inputs("C0", n_tau=2)
    da, db = str(tmp_path / "a"), str(tmp_path / "b")

    def fresh(run_dir):
        ctx = Context.from_inputs(inp, want_grad=grad)
        return Chain(ctx, initial_walkers(inp, chain=1), key=(3, 1), delta=0.4, want_grad=grad, run_dir=run_dir)

    a = fresh(da)
    a.burn_in(60)
    a.run(400, block=100)
    b = fresh(db)
    b.burn_in(60)
    b.run(200, block=100)
    stop_step = b.step
    b.ctx.close()
    del b
    good = open(checkpoint_path(db, stop_step), "rb").read()
    with open(checkpoint_path(db, stop_step + 100), "wb") as fh:      # damaged newer checkpoint
        fh.write(good[: len(good) // 3])
    with open(checkpoint_path(db, stop_step + 200) + ".123.tmp", "wb") as fh:
        fh.write(good[:64])
    c = Chain.resume(Context.from_inputs(inp, want_grad=grad), db)
    assert c.want_grad == grad and c.step == stop_step
    c.run(200, block=100)
    assert np.array_equal(a.series(), c.series())
    assert np.array_equal(a.walkers.cpu().numpy(), c.walkers.cpu().numpy())
    ra, rc = a.result(), c.result()
    assert np.array_equal(ra.mean, rc.mean) and np.array_equal(ra.sigma, rc.sigma)
    if grad:
        assert np.array_equal(ra.grad_eps, rc.grad_eps) and np.array_equal(ra.grad_coeffs, rc.grad_coeffs)
    recs_a, recs_c = read_records(da), read_records(db)
    assert [r["N"] for r in recs_a] == [100, 200, 300, 400]
    for x, y in zip(recs_a, recs_c):
        x.pop("steps_per_s"), y.pop("steps_per_s")
    assert recs_a == recs_c
    assert recs_a[-1]["I_N"] == [float(v) for v in ra.mean]
    assert 0.0 < recs_a[-1]["acceptance"] < 1.0


def test_gpu_chain_mean_within_three_sigma_of_deterministic_mp2():
    """The whole estimator on the GPU (Metropolis walk, tau sampling, every
    kernel of the step) against Eq. FinalMP2: on the tiny two-nucleus system
    with basis exponents in [0.3, 1.2] (finite variance), 64 walker pairs,
    6000 steps after 300 of burn-in, the direct and exchange parts and the
    total lie within 3 blocking standard errors of the deterministic values
    stored in tests/golden/c0_narrow_e2.json (written from the oracle's
    McMurchie-Davidson integrals and four-index transformation)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "c0_narrow_e2.json")) as fh:
        ref = json.load(fh)
    inp = make_inputs("C0", exp_range=(0.3, 1.2), m=64)
    ch = _chain(inp, key=(11, 0))
    ch.burn_in(300)
    ch.run(6000, block=100)
    res = ch.result()
    for col, name in enumerate(("direct", "exchange", "total")):
        z = (res.mean[col] - ref[name]) / res.sigma[col]
        print(f"{name}: {res.mean[col]:.6f} +- {res.sigma[col]:.6f} (deterministic {ref[name]:.6f}, z = {z:+.2f})",
              flush=True)
        assert abs(z) < 3.0
        assert res.sigma[col] < 0.2 * abs(ref[name])   # the check has power
