"""One Markov chain of the stochastic MP2 method on the GPU, with burn-in,
blocking statistics, periodic records, checkpoint / resume and the merge of
independent chains (Sec. III of the paper: each processor runs its own chain,
periodically records how many steps it has done with the running mean and
its statistical uncertainty, so that a job killed at any time loses nothing,
and the results are combined as weighted averages at the end).

Every random number of a chain comes from the counter-based generator of the
library (key = (seed, chain), counter = step), and every kernel sums in a
fixed order, so a chain resumed from a checkpoint continues bit for bit as if
it had never stopped.  Chains on separate HIP streams of one GPU run
concurrently and independently.

Run directory (``Chain(..., run_dir=...)``):
  records.jsonl           one JSON record per block of steps: N (post-burn-in
                          steps so far), step (counter of the next move),
                          I_N and sigma_bar_N of the direct / exchange / total
                          parts, the block's acceptance ratio and steps/s;
  chain-<step>.npz        checkpoints, written to a temporary file, flushed to
                          disk and renamed into place, so a checkpoint file is
                          either complete or absent; the newest two are kept.
``Chain.resume(ctx, run_dir)`` continues from the newest checkpoint that
loads completely (a torn temporary file or a damaged newer file is skipped)
and drops the records written after it.
"""
from __future__ import annotations

import glob
import json
import os
import time
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from .context import Context


def blocking_sigma(x: np.ndarray, n_b: int = 100):
    """Standard error of the mean of a correlated series (Sec. III): blocks of
    n_b consecutive values, population variance of the block means, divided
    by the number of complete blocks; an incomplete last block is dropped.
    A 1-d series gives a float; an [N, ...] array gives one standard error per
    trailing index (steps along axis 0)."""
    x = np.asarray(x, dtype=np.float64)
    n_blocks = x.shape[0] // n_b
    if n_blocks < 2:
        return float("nan") if x.ndim == 1 else np.full(x.shape[1:], np.nan)
    means = x[: n_blocks * n_b].reshape((n_blocks, n_b) + x.shape[1:]).mean(axis=1)
    sig = np.sqrt(means.var(axis=0) / n_blocks)
    return float(sig) if x.ndim == 1 else sig


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


CHECKPOINT_FORMAT = 2
_CKPT_KEYS = ("format", "walkers", "w", "key", "step", "n_burn", "delta", "n_tau", "values", "want_grad",
              "accepted", "proposed")


def atomic_savez(path: str, **arrays) -> None:
    """np.savez to `path` so that `path` is either the complete new file or
    untouched: write a temporary file in the same directory, flush it to
    disk, rename it over `path`, then flush the directory entry."""
    d = os.path.dirname(os.path.abspath(path))
    tmp = os.path.join(d, f".{os.path.basename(path)}.{os.getpid()}.tmp")
    with open(tmp, "wb") as fh:
        np.savez(fh, **arrays)
        fh.flush()
        os.fsync(fh.fileno())
    os.replace(tmp, path)
    fd = os.open(d, os.O_RDONLY)
    try:
        os.fsync(fd)
    finally:
        os.close(fd)


def read_checkpoint(path: str) -> Optional[dict]:
    """The arrays of a chain checkpoint, or None if the file is missing,
    truncated, of another format or lacks a field."""
    try:
        with np.load(path, allow_pickle=False) as z:
            st = {k: z[k] for k in z.files}
    except Exception:
        return None
    if any(k not in st for k in _CKPT_KEYS) or int(st["format"]) != CHECKPOINT_FORMAT:
        return None
    if bool(st["want_grad"]) and any("acc_" + k not in st for k in ("eps_s", "eps_c", "c_s", "c_c")):
        return None
    return st


def checkpoint_path(run_dir: str, step: int) -> str:
    return os.path.join(run_dir, f"chain-{step:012d}.npz")


def latest_checkpoint(run_dir: str) -> Optional[str]:
    """Newest checkpoint of a run directory that loads completely."""
    for path in sorted(glob.glob(os.path.join(run_dir, "chain-*.npz")), reverse=True):
        if read_checkpoint(path) is not None:
            return path
    return None


def read_records(run_dir: str) -> list:
    """The block records of a run directory (a torn last line is ignored)."""
    out = []
    try:
        with open(os.path.join(run_dir, "records.jsonl")) as fh:
            for line in fh:
                try:
                    out.append(json.loads(line))
                except ValueError:
                    break
    except FileNotFoundError:
        pass
    return out


def truncate_records(run_dir: str, n_steps: int) -> None:
    """Keep the records up to N = n_steps (those a checkpoint covers),
    rewriting the file atomically."""
    keep = [r for r in read_records(run_dir) if r["N"] <= n_steps]
    path = os.path.join(run_dir, "records.jsonl")
    tmp = os.path.join(run_dir, f".records.jsonl.{os.getpid()}.tmp")
    with open(tmp, "w") as fh:
        for r in keep:
            fh.write(json.dumps(r) + "\n")
        fh.flush()
        os.fsync(fh.fileno())
    os.replace(tmp, path)


class Chain:
    """A chain over one Context.  walkers0: initial positions [m][2][3]
    (bohr, host or device); key = (seed, chain) of the generator.  With
    run_dir, run() appends one record per block to run_dir/records.jsonl and
    writes a checkpoint every `checkpoint_every` blocks (0: never)."""

    def __init__(self, ctx: Context, walkers0, key=(0, 0), delta: float = 0.5, n_tau: int = None,
                 want_grad: bool = False, run_dir: str = None, checkpoint_every: int = 1):
        self.ctx = ctx
        self.key = (int(key[0]), int(key[1]))
        self.delta = float(delta)
        self.n_tau = ctx.n_tau_max if n_tau is None else int(n_tau)
        self.want_grad = bool(want_grad)
        self.step = 0          # counter of the next Metropolis move
        self.n_burn = 0        # moves spent in burn-in
        self.values = []       # host blocks of per-step [direct, exchange, total] (tau-averaged)
        self.accepted = 0      # accepted / proposed moves after burn-in
        self.proposed = 0
        self.run_dir = run_dir
        self.checkpoint_every = int(checkpoint_every)
        self._blocks = 0
        if run_dir is not None:
            os.makedirs(run_dir, exist_ok=True)
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

    def run(self, n_steps: int, block: int = 100):
        """n_steps MC steps (move, tau samples, estimator and, with gradients,
        the adjoint and its compensated accumulation); per-step values are
        copied to the host every `block` steps (N_b = 100 by default), when
        the block's record and, on schedule, a checkpoint are written."""
        ctx = self.ctx
        done = 0
        while done < n_steps:
            nb = min(block, n_steps - done)
            t0 = time.perf_counter()
            with torch.cuda.stream(ctx.stream):
                hist = torch.empty((nb, self.n_tau, 3), dtype=torch.float64, device=self.w.device)
                self.n_acc.zero_()
            for i in range(nb):
                ctx.advance(self.walkers, self.w, self.key, self.step, self.delta, self.tau, self.n_acc)
                if self.want_grad:
                    ctx.step_accumulate(self.walkers, self.tau, hist[i], self.acc["eps_s"], self.acc["eps_c"],
                                        self.acc["c_s"], self.acc["c_c"])
                else:
                    ctx.step(self.walkers, self.tau, hist[i])
                self.step += 1
            with torch.cuda.stream(ctx.stream):
                self.values.append(hist.mean(dim=1).cpu().numpy())
                acc = int(self.n_acc.item())
            self.accepted += acc
            self.proposed += nb * ctx.m
            done += nb
            self._blocks += 1
            if self.run_dir is not None:
                self._record(nb, acc, time.perf_counter() - t0)
                if self.checkpoint_every > 0 and self._blocks % self.checkpoint_every == 0:
                    self.checkpoint()

    def _record(self, nb: int, acc: int, seconds: float) -> None:
        x = self.series()
        rec = {"N": int(len(x)), "step": int(self.step), "key": list(self.key),
               "I_N": [float(v) for v in x.mean(axis=0)],
               "sigma_bar_N": [float(blocking_sigma(x[:, j])) for j in range(3)],
               "acceptance": acc / float(nb * self.ctx.m), "steps_per_s": nb / seconds}
        with open(os.path.join(self.run_dir, "records.jsonl"), "a") as fh:
            fh.write(json.dumps(rec) + "\n")
            fh.flush()
            os.fsync(fh.fileno())

    def checkpoint(self) -> str:
        """Write a checkpoint into the run directory and keep the newest two."""
        path = checkpoint_path(self.run_dir, self.step)
        self.save(path)
        for old in sorted(glob.glob(os.path.join(self.run_dir, "chain-*.npz")))[:-2]:
            os.remove(old)
        return path

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
        st = {"format": np.int64(CHECKPOINT_FORMAT), "walkers": self.walkers.cpu().numpy(),
              "w": self.w.cpu().numpy(), "key": np.array(self.key),
              "step": np.int64(self.step), "n_burn": np.int64(self.n_burn), "delta": np.float64(self.delta),
              "n_tau": np.int64(self.n_tau), "values": self.series(), "want_grad": np.bool_(self.want_grad),
              "accepted": np.int64(self.accepted), "proposed": np.int64(self.proposed)}
        if self.want_grad:
            for k, v in self.acc.items():
                st["acc_" + k] = v.cpu().numpy()
        return st

    def save(self, path: str):
        """Write the chain state (walkers, weights, counters, delta, the
        per-step series and gradient accumulators) as an .npz file, atomically
        (the file at `path` is the old one or the complete new one)."""
        atomic_savez(path, **self.state_dict())

    @classmethod
    def load(cls, ctx: Context, path: str, want_grad: bool = None, run_dir: str = None,
             checkpoint_every: int = 1) -> "Chain":
        """Resume a saved chain on a context built from the same inputs.
        Whether the chain accumulates gradients comes from the checkpoint;
        a want_grad that contradicts it raises ValueError."""
        st = read_checkpoint(path)
        if st is None:
            raise ValueError(f"{path} is not a complete chain checkpoint")
        saved_grad = bool(st["want_grad"])
        if want_grad is not None and bool(want_grad) != saved_grad:
            raise ValueError(f"checkpoint has want_grad={saved_grad}, caller asked for {bool(want_grad)}")
        ch = cls(ctx, st["walkers"], key=tuple(int(k) for k in st["key"]), delta=float(st["delta"]),
                 n_tau=int(st["n_tau"]), want_grad=saved_grad, run_dir=run_dir, checkpoint_every=checkpoint_every)
        with torch.cuda.stream(ctx.stream):
            ch.w.copy_(torch.as_tensor(st["w"], device=ch.w.device))
            if saved_grad:
                for k in ch.acc:
                    ch.acc[k].copy_(torch.as_tensor(st["acc_" + k], device=ch.w.device))
        ch.step, ch.n_burn = int(st["step"]), int(st["n_burn"])
        ch.accepted, ch.proposed = int(st["accepted"]), int(st["proposed"])
        vals = st["values"]
        ch.values = [vals] if len(vals) else []
        return ch

    @classmethod
    def resume(cls, ctx: Context, run_dir: str, checkpoint_every: int = 1) -> "Chain":
        """Continue the run in `run_dir` from its newest complete checkpoint;
        records written after that checkpoint are dropped (the resumed chain
        writes them again, identically)."""
        path = latest_checkpoint(run_dir)
        if path is None:
            raise FileNotFoundError(f"no complete checkpoint in {run_dir}")
        ch = cls.load(ctx, path, run_dir=run_dir, checkpoint_every=checkpoint_every)
        truncate_records(run_dir, len(ch.series()))
        return ch
