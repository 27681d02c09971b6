"""One Markov chain of the stochastic MP2 method on the GPU, with burn-in,
blocking statistics, checkpoint / resume and the merge of independent chains
(Sec. III of the paper: each processor runs its own chain and the results are
combined as weighted averages at the end).

Every random number of a chain comes from the counter-based generator of the
library (key = (seed, chain), counter = step), and every kernel sums in a
fixed order, so a chain resumed from a checkpoint continues bit for bit as if
it had never stopped.  Chains on separate HIP streams of one GPU run
concurrently and independently.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Sequence

import numpy as np
import torch

from .context import Context


def blocking_sigma(x: np.ndarray, n_b: int = 100) -> float:
    """Standard error of the mean of a correlated series (Sec. III): blocks of
    n_b consecutive values, population variance of the block means, divided
    by the number of complete blocks; an incomplete last block is dropped."""
    n_blocks = len(x) // n_b
    if n_blocks < 2:
        return float("nan")
    means = np.asarray(x[: n_blocks * n_b], dtype=np.float64).reshape(n_blocks, n_b).mean(axis=1)
    return float(math.sqrt(means.var() / n_blocks))


@dataclass
class ChainResult:
    steps: int             # post-burn-in steps
    mean: np.ndarray       # [3] direct, exchange, total (mean over steps of the per-step value)
    sigma: np.ndarray      # [3] blocking standard errors
    grad_eps: np.ndarray = None     # mean over steps of dV/d eps (with gradients)
    grad_coeffs: np.ndarray = None  # mean over steps of dV/dC


def merge(results: Sequence[ChainResult]) -> ChainResult:
    """Combine independent chains: means weighted by post-burn-in step counts
    (unbiased for any chain lengths), standard errors combined as independent
    estimates with the same weights."""
    n = np.array([r.steps for r in results], dtype=np.float64)
    w = n / n.sum()
    mean = sum(wi * r.mean for wi, r in zip(w, results))
    sigma = np.sqrt(sum((wi * r.sigma) ** 2 for wi, r in zip(w, results)))
    ge = gc = None
    if all(r.grad_eps is not None for r in results):
        ge = sum(wi * r.grad_eps for wi, r in zip(w, results))
        gc = sum(wi * r.grad_coeffs for wi, r in zip(w, results))
    return ChainResult(int(n.sum()), mean, sigma, ge, gc)


class Chain:
    """A chain over one Context.  walkers0: initial positions [m][2][3]
    (bohr, host or device); key = (seed, chain) of the generator."""

    def __init__(self, ctx: Context, walkers0, key=(0, 0), delta: float = 0.5, n_tau: int = None,
                 want_grad: bool = False):
        self.ctx = ctx
        self.key = (int(key[0]), int(key[1]))
        self.delta = float(delta)
        self.n_tau = ctx.n_tau_max if n_tau is None else int(n_tau)
        self.want_grad = bool(want_grad)
        self.step = 0          # counter of the next Metropolis move
        self.n_burn = 0        # moves spent in burn-in
        self.values = []       # host blocks of per-step [direct, exchange, total] (tau-averaged)
        dev = torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.stream(ctx.stream):
            self.walkers = torch.as_tensor(np.asarray(walkers0, dtype=np.float64), device=dev).contiguous().clone()
            self.w = torch.zeros(ctx.m, dtype=torch.float64, device=dev)
            self.tau = torch.zeros(self.n_tau, dtype=torch.float64, device=dev)
            self.n_acc = torch.zeros(1, dtype=torch.int32, device=dev)
            if self.want_grad:  # compensated running sums of both gradients
                self.acc = {k: torch.zeros(ctx.n_sp, dtype=torch.float64, device=dev) for k in ("eps_s", "eps_c")}
                self.acc.update({k: torch.zeros((2, ctx.n_b, ctx.n_sp), dtype=torch.complex128, device=dev)
                                 for k in ("c_s", "c_c")})
        ctx.pair_weights(self.walkers, self.w)

    # -- sampling ---------------------------------------------------------------
    def burn_in(self, n_steps: int, target: float = 0.5, window: int = 10, adapt: bool = True):
        """Metropolis moves only (excluded from the averages); with adapt,
        delta is scaled by 1.1 or 0.9 after every window of moves toward the
        acceptance ratio `target`, and frozen afterwards."""
        if not adapt:
            for _ in range(n_steps):
                self.ctx.metropolis(self.walkers, self.w, self.key, self.step, self.delta)
                self.step += 1
            self.n_burn = self.step
            return
        for _ in range(n_steps // window):
            with torch.cuda.stream(self.ctx.stream):
                self.n_acc.zero_()
            for _ in range(window):
                self.ctx.metropolis(self.walkers, self.w, self.key, self.step, self.delta, self.n_acc)
                self.step += 1
            with torch.cuda.stream(self.ctx.stream):  # the count is read after the moves on the chain's stream
                acc = self.n_acc.item() / float(window * self.ctx.m)
            self.delta *= 1.1 if acc > target else 0.9
        self.n_burn = self.step

    def run(self, n_steps: int, block: int = 1000):
        """n_steps MC steps (move, tau samples, estimator and, with gradients,
        the adjoint and its compensated accumulation); per-step values are
        copied to the host every `block` steps."""
        ctx = self.ctx
        done = 0
        while done < n_steps:
            nb = min(block, n_steps - done)
            with torch.cuda.stream(ctx.stream):
                hist = torch.empty((nb, self.n_tau, 3), dtype=torch.float64, device=self.w.device)
            for i in range(nb):
                ctx.advance(self.walkers, self.w, self.key, self.step, self.delta, self.tau)
                if self.want_grad:
                    ctx.step_accumulate(self.walkers, self.tau, hist[i], self.acc["eps_s"], self.acc["eps_c"],
                                        self.acc["c_s"], self.acc["c_c"])
                else:
                    ctx.step(self.walkers, self.tau, hist[i])
                self.step += 1
            with torch.cuda.stream(ctx.stream):
                self.values.append(hist.mean(dim=1).cpu().numpy())
            done += nb

    # -- results ----------------------------------------------------------------
    def series(self) -> np.ndarray:
        """[steps][3] per-step direct, exchange, total."""
        return np.concatenate(self.values) if self.values else np.zeros((0, 3))

    def result(self, n_b: int = 100) -> ChainResult:
        x = self.series()
        mean = x.mean(axis=0) if len(x) else np.full(3, np.nan)
        sigma = np.array([blocking_sigma(x[:, j], n_b) for j in range(3)])
        ge = gc = None
        if self.want_grad and len(x):
            torch.cuda.current_stream().wait_stream(self.ctx.stream)
            ge = ((self.acc["eps_s"] + self.acc["eps_c"]) / len(x)).cpu().numpy()
            gc = ((self.acc["c_s"] + self.acc["c_c"]) / len(x)).cpu().numpy()
        return ChainResult(len(x), mean, sigma, ge, gc)

    # -- checkpoint / resume ------------------------------------------------------
    def state_dict(self) -> dict:
        torch.cuda.current_stream().wait_stream(self.ctx.stream)
        st = {"walkers": self.walkers.cpu().numpy(), "w": self.w.cpu().numpy(), "key": np.array(self.key),
              "step": np.int64(self.step), "n_burn": np.int64(self.n_burn), "delta": np.float64(self.delta),
              "n_tau": np.int64(self.n_tau), "values": self.series()}
        if self.want_grad:
            for k, v in self.acc.items():
                st["acc_" + k] = v.cpu().numpy()
        return st

    def save(self, path: str):
        """Write the chain state (walkers, weights, counters, delta, the
        per-step series and gradient accumulators) as an .npz file."""
        np.savez(path, **self.state_dict())

    @classmethod
    def load(cls, ctx: Context, path: str, want_grad: bool = False) -> "Chain":
        """Resume a saved chain on a context built from the same inputs."""
        st = np.load(path, allow_pickle=False)
        ch = cls(ctx, st["walkers"], key=tuple(int(k) for k in st["key"]), delta=float(st["delta"]),
                 n_tau=int(st["n_tau"]), want_grad=want_grad)
        with torch.cuda.stream(ctx.stream):
            ch.w.copy_(torch.as_tensor(st["w"], device=ch.w.device))
            if want_grad:
                for k in ch.acc:
                    ch.acc[k].copy_(torch.as_tensor(st["acc_" + k], device=ch.w.device))
        ch.step, ch.n_burn = int(st["step"]), int(st["n_burn"])
        vals = st["values"]
        ch.values = [vals] if len(vals) else []
        return ch
