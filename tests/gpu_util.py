"""Helpers shared by the GPU parity tests (no simulation arithmetic here)."""
import numpy as np
import pytest

TOL = {"c128": 1e-12, "c64": 2e-5}


def torch_dtype(name):
    import torch
    return torch.complex128 if name == "c128" else torch.complex64


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def to_host(state) -> np.ndarray:
    return state.amps.detach().cpu().numpy().astype(np.complex128)


def max_err(a, b) -> float:
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) if np.size(a) else 0.0
