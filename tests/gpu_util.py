"""Helpers for the GPU parity tests (HIP library vs the FP64 oracle)."""
import numpy as np
import pytest
import torch

requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no HIP device")


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def rel_err(got, ref, norm=None):
    """max |got - ref| / max(|ref|, norm) elementwise-normalised."""
    got = np.asarray(got, dtype=float)
    ref = np.asarray(ref, dtype=float)
    den = np.abs(ref) if norm is None else np.maximum(np.abs(ref), norm)
    return float(np.max(np.abs(got - ref) / np.where(den == 0, 1.0, den)))
