"""Python side of the McMurchie-Davidson integrals (oracle/eri_md.c).

Test infrastructure: part of the FP64 oracle.  The C file is compiled with
gcc into oracle/_eri_md.so on first use (or by the package build step).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eri_md.c")
_LIB = os.path.join(_HERE, "_eri_md.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C part of the oracle (gcc -O2 -shared)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        _lib.oracle_boys.argtypes = [ctypes.c_int, ctypes.c_double, dp]
        _lib.oracle_boys.restype = None
        _lib.oracle_eri_pairs.argtypes = [ctypes.c_int, dp, dp, ip, dp, ctypes.c_int, ip, ip, dp]
        _lib.oracle_eri_pairs.restype = ctypes.c_int
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def boys(nmax: int, T: float) -> np.ndarray:
    """[F_0(T), ..., F_nmax(T)]."""
    F = np.zeros(nmax + 1)
    _load().oracle_boys(int(nmax), float(T), _dp(F))
    return F


def eri_pairs(xyz, alpha, lxyz, norm, pi, pj) -> np.ndarray:
    """Matrix (pi[P] pj[P] | pi[Q] pj[Q]) over a list of charge distributions."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    lxyz = np.ascontiguousarray(lxyz, dtype=np.int32)
    norm = np.ascontiguousarray(norm, dtype=np.float64)
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    pj = np.ascontiguousarray(pj, dtype=np.int32)
    out = np.zeros((pi.shape[0], pi.shape[0]))
    rc = _load().oracle_eri_pairs(int(alpha.shape[0]), _dp(xyz), _dp(alpha), _ip(lxyz), _dp(norm),
                                  int(pi.shape[0]), _ip(pi), _ip(pj), _dp(out))
    if rc != 0:
        raise ValueError("angular momentum above the supported maximum")
    return out


def eri_full(xyz, alpha, lxyz, norm, blocks=None) -> np.ndarray:
    """Dense (mu nu | kappa lambda) [n, n, n, n].

    blocks: optional list of index ranges; only charge distributions mu nu
    with both indices in the same range are computed (the others are left
    zero).  For the four-component problem the ranges are the L and S sets,
    because rho = phi^dagger phi never pairs an L with an S component.
    """
    n = alpha.shape[0]
    if blocks is None:
        blocks = [range(n)]
    pi, pj = [], []
    for blk in blocks:
        idx = list(blk)
        for a in range(len(idx)):
            for b in range(a + 1):
                pi.append(idx[a])
                pj.append(idx[b])
    M = eri_pairs(xyz, alpha, lxyz, norm, pi, pj)
    out = np.zeros((n, n, n, n))
    pi = np.array(pi)
    pj = np.array(pj)
    for (a, b) in ((pi, pj), (pj, pi)):
        for (c, d) in ((pi, pj), (pj, pi)):
            out[a[:, None], b[:, None], c[None, :], d[None, :]] = M
    return out
