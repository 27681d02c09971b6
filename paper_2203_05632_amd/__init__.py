"""MI355X implementation of the per-step hot path of stochastic
four-component relativistic MP2 (Cruz, Garza, Yanai, Hirata, arXiv 2203.05632).

The work happens in libmcmp2.so (HIP kernels for gfx950 behind the C ABI of
include/mcmp2.h).  This package is a thin ctypes binding: it marshals
arguments (PyTorch tensors serve only as device memory and stream handles)
and never computes any step of the method itself.
"""
from .autograd import MCMP2Step, mcmp2_value  # noqa: F401
from .chain import Chain, ChainResult, blocking_sigma, merge  # noqa: F401
from .context import Context, step_noalloc  # noqa: F401
from ._lib import EXPORTS, MCMP2Error, PRECISIONS, load  # noqa: F401
