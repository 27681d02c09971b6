"""Python binding of the C ABI: argument marshalling only.

Device buffers are torch tensors on a HIP device (float64, contiguous); the
library enqueues its kernels on the stream given at construction (by default
torch's current stream on the tensors' device).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import INTERACTIONS, KERNELS, PRECISIONS, Basis, check, load


def _host(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _dev(t: torch.Tensor, shape=None, dtype=torch.float64, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _basis(nuc_xyz, wfn, n_L: int, n_S: int, prim_xyz, prim_exp, prim_lxyz, prim_norm):
    """mcmp2_basis over contiguous host copies (returned with the copies, which must outlive the call)."""
    n_b = int(n_L) + int(n_S)
    keep = dict(nuc=_host(nuc_xyz, np.float64), wfn=_host(wfn, np.float64), pxyz=_host(prim_xyz, np.float64),
                pexp=_host(prim_exp, np.float64), plxyz=_host(prim_lxyz, np.int32),
                pnorm=_host(prim_norm, np.float64))
    n_nuc = keep["nuc"].shape[0]
    if keep["nuc"].shape != (n_nuc, 3) or keep["wfn"].shape != (n_nuc, 4):
        raise ValueError("nuc_xyz must be [n_nuc, 3] and wfn [n_nuc, 4]")
    for k, shp in (("pxyz", (n_b, 3)), ("plxyz", (n_b, 3)), ("pexp", (n_b,)), ("pnorm", (n_b,))):
        if keep[k].shape != shp:
            raise ValueError(f"basis array {k} has shape {keep[k].shape}, expected {shp}")
    basis = Basis(n_nuc, keep["nuc"].ctypes.data, keep["wfn"].ctypes.data, int(n_L), int(n_S),
                  keep["pxyz"].ctypes.data, keep["pexp"].ctypes.data, keep["plxyz"].ctypes.data,
                  keep["pnorm"].ctypes.data)
    return basis, keep


def step_noalloc(inp, coeffs: torch.Tensor, walkers: torch.Tensor, tau: torch.Tensor, e2_out: torch.Tensor,
                 value: torch.Tensor = None, stream: torch.cuda.Stream = None) -> torch.Tensor:
    """mcmp2_step_noalloc: the FP64 estimator without a context or any device
    allocation.  `inp` carries the mcmp2_basis fields, eps, n_occ, n_vir and m;
    coeffs is a complex128 device tensor [2, n_b, n_sp]; walkers, tau, e2_out
    and value as for Context.step.  Synchronises the stream before returning."""
    lib = load()
    basis, keep = _basis(inp.nuc_xyz, inp.wfn, inp.n_L, inp.n_S, inp.prim_xyz, inp.prim_exp, inp.prim_lxyz,
                         inp.prim_norm)
    n_sp = int(inp.n_occ) + int(inp.n_vir)
    eps = _host(inp.eps, np.float64)
    if eps.shape != (n_sp,):
        raise ValueError("eps must have n_occ + n_vir entries")
    n_tau = int(tau.shape[0])
    m = int(walkers.shape[0])
    st = torch.cuda.current_stream() if stream is None else stream
    check(lib.mcmp2_step_noalloc(
        ctypes.byref(basis), _dev(coeffs, (2, int(inp.n_L) + int(inp.n_S), n_sp), torch.complex128, name="coeffs"),
        ctypes.c_void_p(eps.ctypes.data), int(inp.n_occ), int(inp.n_vir), m,
        _dev(walkers, (m, 2, 3), name="walkers"), _dev(tau, (n_tau,), name="tau"), n_tau,
        _dev(e2_out, (n_tau, 3), name="e2_out"), None if value is None else _dev(value, (1,), name="value"),
        ctypes.c_void_p(st.cuda_stream)))
    del keep
    return e2_out


class Context:
    """Owns one mcmp2_ctx (device copies of basis, coefficients, energies and
    every per-step work buffer)."""

    def __init__(self, nuc_xyz, wfn, n_L: int, n_S: int, prim_xyz, prim_exp, prim_lxyz, prim_norm,
                 coeffs, eps, n_occ: int, n_vir: int, m: int, n_tau_max: int = 1,
                 precision: str = "fp64", want_grad: bool = False, stream: torch.cuda.Stream = None):
        lib = load()
        self._lib = lib
        self._h = ctypes.c_void_p()
        self.m, self.n_occ, self.n_vir, self.n_tau_max = int(m), int(n_occ), int(n_vir), int(n_tau_max)
        self.n_sp = self.n_occ + self.n_vir
        self.n_b = int(n_L) + int(n_S)
        self.stream = torch.cuda.current_stream() if stream is None else stream
        basis, keep = _basis(nuc_xyz, wfn, n_L, n_S, prim_xyz, prim_exp, prim_lxyz, prim_norm)
        keep["eps"] = _host(eps, np.float64)
        C = np.ascontiguousarray(np.asarray(coeffs, dtype=np.complex128))
        if C.shape != (2, self.n_b, self.n_sp):
            raise ValueError(f"coeffs has shape {C.shape}, expected {(2, self.n_b, self.n_sp)}")
        if keep["eps"].shape != (self.n_sp,):
            raise ValueError("eps must have n_occ + n_vir entries")
        check(lib.mcmp2_init(ctypes.byref(basis), ctypes.c_void_p(C.ctypes.data),
                             ctypes.c_void_p(keep["eps"].ctypes.data), self.n_occ, self.n_vir, self.m,
                             self.n_tau_max, PRECISIONS[precision], int(bool(want_grad)),
                             ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._h)))
        lam, ng = ctypes.c_double(), ctypes.c_double()
        check(lib.mcmp2_constants(self._h, ctypes.byref(lam), ctypes.byref(ng)))
        self.lam, self.Ng = lam.value, ng.value

    @classmethod
    def from_inputs(cls, inp, m: int = None, n_tau_max: int = None, **kw) -> "Context":
        """Build from an object carrying the mcmp2_basis fields, coeffs and eps."""
        return cls(inp.nuc_xyz, inp.wfn, inp.n_L, inp.n_S, inp.prim_xyz, inp.prim_exp, inp.prim_lxyz,
                   inp.prim_norm, inp.coeffs, inp.eps, inp.n_occ, inp.n_vir,
                   inp.m if m is None else m, inp.n_tau if n_tau_max is None else n_tau_max, **kw)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.mcmp2_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- entry points -------------------------------------------------------------------------
    def step(self, walkers: torch.Tensor, tau: torch.Tensor, e2_out: torch.Tensor,
             grad_eps: torch.Tensor = None, grad_coeffs: torch.Tensor = None,
             value: torch.Tensor = None) -> torch.Tensor:
        """One step; value (float64 [1], optional) receives the tau average of e2_out[:, 2]."""
        n_tau = int(tau.shape[0])
        check(self._lib.mcmp2_step(
            self._h, _dev(walkers, (self.m, 2, 3), name="walkers"), _dev(tau, (n_tau,), name="tau"), n_tau,
            _dev(e2_out, (n_tau, 3), name="e2_out"),
            None if value is None else _dev(value, (1,), name="value"),
            None if grad_eps is None else _dev(grad_eps, (self.n_sp,), name="grad_eps"),
            None if grad_coeffs is None else _dev(grad_coeffs, (2, self.n_b, self.n_sp), torch.complex128,
                                                  name="grad_coeffs")))
        return e2_out

    def step_accumulate(self, walkers: torch.Tensor, tau: torch.Tensor, e2_out: torch.Tensor,
                        eps_sum: torch.Tensor, eps_comp: torch.Tensor, coeffs_sum: torch.Tensor,
                        coeffs_comp: torch.Tensor) -> torch.Tensor:
        """step() with both gradients added to compensated running sums
        ((eps_sum, eps_comp): float64 [n_sp]; (coeffs_sum, coeffs_comp):
        complex128 [2, n_b, n_sp]) instead of written out; bitwise the same as
        step() followed by accumulate() of each gradient."""
        n_tau = int(tau.shape[0])
        check(self._lib.mcmp2_step_accumulate(
            self._h, _dev(walkers, (self.m, 2, 3), name="walkers"), _dev(tau, (n_tau,), name="tau"), n_tau,
            _dev(e2_out, (n_tau, 3), name="e2_out"), _dev(eps_sum, (self.n_sp,), name="eps_sum"),
            _dev(eps_comp, (self.n_sp,), name="eps_comp"),
            _dev(coeffs_sum, (2, self.n_b, self.n_sp), torch.complex128, name="coeffs_sum"),
            _dev(coeffs_comp, (2, self.n_b, self.n_sp), torch.complex128, name="coeffs_comp")))
        return e2_out

    def set_coefficients(self, coeffs: torch.Tensor = None, eps: torch.Tensor = None) -> None:
        """Replace the spinor coefficients / energies with device tensors (init layout)."""
        check(self._lib.mcmp2_set_coefficients(
            self._h,
            None if coeffs is None else _dev(coeffs, (2, self.n_b, self.n_sp), torch.complex128, name="coeffs"),
            None if eps is None else _dev(eps, (self.n_sp,), name="eps")))

    def set_interaction(self, kind: str) -> None:
        """Electron-electron interaction of the following steps: "coulomb"
        (default), "gaunt" or "breit" (any precision, with or without gradients)."""
        check(self._lib.mcmp2_set_interaction(self._h, INTERACTIONS[kind]))

    def pair_weights(self, walkers: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
        check(self._lib.mcmp2_pair_weights(self._h, _dev(walkers, (self.m, 2, 3), name="walkers"),
                                           _dev(w, (self.m,), name="w")))
        return w

    def metropolis(self, walkers: torch.Tensor, w: torch.Tensor, key, step: int, delta: float,
                   n_accepted: torch.Tensor = None) -> None:
        check(self._lib.mcmp2_metropolis(
            self._h, _dev(walkers, (self.m, 2, 3), name="walkers"), _dev(w, (self.m,), name="w"),
            int(key[0]), int(key[1]), int(step), float(delta),
            None if n_accepted is None else _dev(n_accepted, (1,), torch.int32, name="n_accepted")))

    def advance(self, walkers: torch.Tensor, w: torch.Tensor, key, step: int, delta: float, tau: torch.Tensor,
                n_accepted: torch.Tensor = None) -> torch.Tensor:
        """Metropolis move and tau samples of MC step `step` in one launch."""
        n = int(tau.shape[0])
        check(self._lib.mcmp2_advance(
            self._h, _dev(walkers, (self.m, 2, 3), name="walkers"), _dev(w, (self.m,), name="w"),
            int(key[0]), int(key[1]), int(step), float(delta),
            None if n_accepted is None else _dev(n_accepted, (1,), torch.int32, name="n_accepted"),
            n, _dev(tau, (n,), name="tau")))
        return tau

    def sample_tau(self, key, step: int, tau: torch.Tensor) -> torch.Tensor:
        n = int(tau.shape[0])
        check(self._lib.mcmp2_sample_tau(self._h, int(key[0]), int(key[1]), int(step), n,
                                         _dev(tau, (n,), name="tau")))
        return tau

    def accumulate(self, src: torch.Tensor, acc_sum: torch.Tensor, acc_comp: torch.Tensor) -> None:
        """Compensated accumulation (acc_sum, acc_comp) += src (float64 or complex128 device tensors)."""
        if not (src.shape == acc_sum.shape == acc_comp.shape and src.dtype == acc_sum.dtype == acc_comp.dtype):
            raise ValueError("src, acc_sum and acc_comp must share shape and dtype")
        if src.dtype not in (torch.float64, torch.complex128):
            raise TypeError("accumulate takes float64 or complex128 tensors")
        n = src.numel() * (2 if src.is_complex() else 1)
        check(self._lib.mcmp2_accumulate(self._h, _dev(src, dtype=src.dtype, name="src"),
                                         _dev(acc_sum, dtype=src.dtype, name="acc_sum"),
                                         _dev(acc_comp, dtype=src.dtype, name="acc_comp"), n))

    def profile_begin(self, kernels, max_launches: int) -> None:
        """Time every launch of the named kernels with HIP events on the context's stream."""
        mask = 0
        for k in kernels:
            mask |= 1 << KERNELS.index(k)
        check(self._lib.mcmp2_profile_begin(self._h, mask, int(max_launches)))

    def profile_end(self) -> dict:
        """{kernel: (total_ms, launches)} for the kernels timed since profile_begin."""
        ms = np.zeros(len(KERNELS), dtype=np.float64)
        n = np.zeros(len(KERNELS), dtype=np.int64)
        check(self._lib.mcmp2_profile_end(self._h, ctypes.c_void_p(ms.ctypes.data), ctypes.c_void_p(n.ctypes.data)))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNELS) if n[i] > 0}
