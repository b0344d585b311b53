"""Helpers shared by the GPU parity tests (no simulation arithmetic here).

Tolerances (the parity contract, no multipliers):
  * complex128 amplitudes: max |delta| <= 1e-12 against the complex128 oracle;
  * complex64 amplitudes: max |delta| <= 2e-5, and the whole error vector
    within the normwise rounding bound ||delta||_2 <= (10 G + 1) 2^-24 for a
    unit-norm state after G gates (each float gate adds at most about
    10 * 2^-24 * ||psi||: 2 * 4 * 2^-24 from the two 4-term complex dot
    products of a pair, sqrt(2) * 2^-24 from the matrix rounded to float; the
    initial rounding of the state adds 2^-24; a unitary keeps earlier errors'
    norm);
  * complex128 read-outs: |delta| <= 1e-12 * max(1, |value|);
  * complex64 read-outs of an observable O: |delta| <= 2 ||O|| ||delta psi||_2
    (+ second order), so max(2e-5, 2 (10 G + 1) 2^-24) * max(1, ||O||).
Every check records the observed error and its bound; the session prints them.
"""
import os

import numpy as np
import pytest

TOL = {"c128": 1e-12, "c64": 2e-5}
EPS32 = 2.0 ** -24
RECORDS = []  # (test, what, observed, bound)


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


def record(what: str, observed: float, bound: float) -> None:
    test = os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0]
    RECORDS.append((test, what, float(observed), float(bound)))
    print(f"[parity] {test} {what}: observed {observed:.3e} bound {bound:.3e}", flush=True)
    assert observed <= bound, f"{what}: observed {observed:.3e} > bound {bound:.3e}"


def c64_norm_bound(gates: int) -> float:
    return (10 * gates + 1) * EPS32


def _chunked_stats(got, want, chunk=1 << 24):
    """(max |delta|, ||delta||_2, max |want|) without whole-register temporaries."""
    mx = nrm = amax = 0.0
    for i in range(0, len(want), chunk):
        g = np.asarray(got[i:i + chunk]).astype(np.complex128, copy=False)
        w = np.asarray(want[i:i + chunk])
        d = np.abs(g - w)
        if d.size:
            mx = max(mx, float(d.max()))
            nrm += float(np.dot(d, d))
            amax = max(amax, float(np.abs(w).max()))
    return mx, nrm ** 0.5, amax


def check_amps(got, want, dt: str, what: str = "amplitudes", gates: int = 1, amplify: float = 1.0) -> float:
    """Amplitude parity: max |delta| <= TOL[dt]; for complex64 also the
    normwise bound for `gates` float gates (times `amplify` where a
    renormalisation scales the error).  Returns max |delta|."""
    mx, nrm, amax = _chunked_stats(got, want)
    record(f"{what} max|d|", mx, TOL[dt])
    if dt == "c64":
        record(f"{what} ||d||_2 (max|d|/max|a| = {mx / max(amax, 1e-300):.2e})", nrm, c64_norm_bound(gates) * amplify)
    return mx


def readout_tol(dt: str, value: float = 0.0, opnorm: float = 1.0, gates: int = 1) -> float:
    if dt == "c128":
        return TOL["c128"] * max(1.0, abs(value))
    return max(TOL["c64"], 2 * c64_norm_bound(gates)) * max(1.0, opnorm)


def check_val(got, want, dt: str, what: str, opnorm: float = 1.0, gates: int = 1) -> float:
    """Read-out parity (scalars or arrays compared element by element)."""
    got, want = np.asarray(got, dtype=np.float64), np.asarray(want, dtype=np.float64)
    err = float(np.max(np.abs(got - want))) if got.size else 0.0
    value = float(np.max(np.abs(want))) if want.size else 0.0
    record(what, err, readout_tol(dt, value, opnorm, gates))
    return err
