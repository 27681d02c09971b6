"""ctypes loader of libmcmp2.so (the HIP implementation).

Fails loudly: if the library has not been built, importing the binding
raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcmp2.so")

MCMP2_OK, MCMP2_EINVAL, MCMP2_ENOMEM, MCMP2_EDEVICE, MCMP2_ESTATE = 0, -1, -2, -3, -4
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3}
INTERACTIONS = {"coulomb": 0, "gaunt": 1, "breit": 2}

# Every symbol declared in include/mcmp2.h.
EXPORTS = ["mcmp2_init", "mcmp2_step", "mcmp2_step_accumulate", "mcmp2_set_coefficients", "mcmp2_set_interaction", "mcmp2_pair_weights", "mcmp2_metropolis", "mcmp2_sample_tau",
           "mcmp2_advance", "mcmp2_accumulate", "mcmp2_constants", "mcmp2_profile_begin", "mcmp2_profile_end", "mcmp2_step_noalloc",
           "mcmp2_destroy", "mcmp2_last_error"]
KERNELS = ["walker_weights", "step_prep", "spinor_gemm", "green_contract", "reduce", "metropolis", "sample_tau",
           "advance", "grad", "accumulate", "coef_grad", "green_gemm", "adj_gemm"]


class Basis(ctypes.Structure):
    _fields_ = [
        ("n_nuc", ctypes.c_int32),
        ("nuc_xyz", ctypes.c_void_p),
        ("wfn", ctypes.c_void_p),
        ("n_L", ctypes.c_int32),
        ("n_S", ctypes.c_int32),
        ("prim_xyz", ctypes.c_void_p),
        ("prim_exp", ctypes.c_void_p),
        ("prim_lxyz", ctypes.c_void_p),
        ("prim_norm", ctypes.c_void_p),
    ]


class MCMP2Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mcmp2 error {code}: {msg}")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
    lib.mcmp2_init.argtypes = [ctypes.POINTER(Basis), vp, vp, i32, i32, i32, i32, i32, i32, vp,
                               ctypes.POINTER(vp)]
    lib.mcmp2_init.restype = ctypes.c_int
    lib.mcmp2_step.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp]
    lib.mcmp2_step.restype = ctypes.c_int
    lib.mcmp2_step_accumulate.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, vp]
    lib.mcmp2_step_accumulate.restype = ctypes.c_int
    lib.mcmp2_set_coefficients.argtypes = [vp, vp, vp]
    lib.mcmp2_set_coefficients.restype = ctypes.c_int
    lib.mcmp2_set_interaction.argtypes = [vp, i32]
    lib.mcmp2_set_interaction.restype = ctypes.c_int
    lib.mcmp2_pair_weights.argtypes = [vp, vp, vp]
    lib.mcmp2_pair_weights.restype = ctypes.c_int
    lib.mcmp2_metropolis.argtypes = [vp, vp, vp, u64, u64, u64, dbl, vp]
    lib.mcmp2_metropolis.restype = ctypes.c_int
    lib.mcmp2_sample_tau.argtypes = [vp, u64, u64, u64, i32, vp]
    lib.mcmp2_sample_tau.restype = ctypes.c_int
    lib.mcmp2_advance.argtypes = [vp, vp, vp, u64, u64, u64, dbl, vp, i32, vp]
    lib.mcmp2_advance.restype = ctypes.c_int
    lib.mcmp2_accumulate.argtypes = [vp, vp, vp, vp, ctypes.c_int64]
    lib.mcmp2_accumulate.restype = ctypes.c_int
    lib.mcmp2_constants.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    lib.mcmp2_constants.restype = ctypes.c_int
    lib.mcmp2_profile_begin.argtypes = [vp, ctypes.c_uint32, i32]
    lib.mcmp2_profile_begin.restype = ctypes.c_int
    lib.mcmp2_profile_end.argtypes = [vp, vp, vp]
    lib.mcmp2_profile_end.restype = ctypes.c_int
    lib.mcmp2_step_noalloc.argtypes = [ctypes.POINTER(Basis), vp, vp, i32, i32, i32, vp, vp, i32, vp, vp, vp]
    lib.mcmp2_step_noalloc.restype = ctypes.c_int
    lib.mcmp2_destroy.argtypes = [vp]
    lib.mcmp2_destroy.restype = None
    lib.mcmp2_last_error.argtypes = []
    lib.mcmp2_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != MCMP2_OK:
        raise MCMP2Error(rc, load().mcmp2_last_error().decode())
