"""CPU oracle for the state-vector simulator — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (the HIP library and its
Python binding) never imports it, and it never imports the product: the two
share only the seeded inputs of ``paper_2001_10554_amd.workloads``.

The arithmetic lives in ``qsim_ref.c`` (plain complex128 C, one gate at a time,
long-double sequential reductions).  This module is ctypes marshalling plus a
few numpy-level compositions that are plain definitions (trajectory averages).

Every function here is pinned by a ``-m "not gpu"`` test against something
other than itself (Kronecker-product unitaries, closed forms, the paper's
worked example, published Philox known-answer vectors, a density-matrix
computation).  No function is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qsim_ref.c")
_LIB_PATH = os.path.join(_HERE, "libqsim_ref.so")

_c_cplx_p = np.ctypeslib.ndpointer(dtype=np.complex128, flags="C_CONTIGUOUS")
_c_f64_p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_c_i32_p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_c_u32_p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_c_u64_p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP on element-wise loops only)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-fvisibility=hidden",
               _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        c_int, c_double, c_u64, c_i64, c_u32 = ctypes.c_int, ctypes.c_double, ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32
        vp = ctypes.c_void_p
        sig = {
            "ref_philox4x32_10": (None, [_c_u32_p, _c_u32_p, _c_u32_p]),
            "ref_apply_1q": (None, [_c_cplx_p, c_int, c_int, _c_f64_p]),
            "ref_apply_c1q": (None, [_c_cplx_p, c_int, c_int, c_int, _c_f64_p]),
            "ref_apply_diag2": (None, [_c_cplx_p, c_int, c_int, c_int, _c_f64_p]),
            "ref_apply_swap": (None, [_c_cplx_p, c_int, c_int, c_int]),
            "ref_apply_gates": (c_int, [_c_cplx_p, c_int, vp, c_int]),
            "ref_init_basis": (None, [_c_cplx_p, c_int, c_u64]),
            "ref_init_uniform": (None, [_c_cplx_p, c_int]),
            "ref_init_random": (None, [_c_cplx_p, c_int, c_u64]),
            "ref_cut_value": (c_double, [c_u64, c_int, _c_i32_p, vp]),
            "ref_apply_cut_phase": (None, [_c_cplx_p, c_int, c_int, _c_i32_p, vp, c_double]),
            "ref_norm2": (c_double, [_c_cplx_p, c_int]),
            "ref_prob_one": (c_double, [_c_cplx_p, c_int, c_int]),
            "ref_expect_z_all": (None, [_c_cplx_p, c_int, _c_f64_p]),
            "ref_expect_cut": (c_double, [_c_cplx_p, c_int, c_int, _c_i32_p, vp]),
            "ref_expect_diag": (c_double, [_c_cplx_p, c_int, _c_f64_p]),
            "ref_expect_pauli": (c_int, [_c_cplx_p, c_int, c_u64, c_u64, _c_f64_p]),
            "ref_inner": (None, [_c_cplx_p, _c_cplx_p, c_int, _c_f64_p]),
            "ref_sample": (c_int, [_c_cplx_p, c_int, c_i64, c_u64, _c_u64_p, _c_f64_p]),
            "ref_qaoa_state": (c_double, [_c_cplx_p, c_int, c_int, _c_i32_p, vp, c_int, _c_f64_p]),
            "ref_qaoa_energy": (c_double, [c_int, c_int, _c_i32_p, vp, c_int, _c_f64_p]),
            "ref_qaoa_grad": (c_double, [c_int, c_int, _c_i32_p, vp, c_int, _c_f64_p, _c_f64_p]),
            "ref_qaoa_grad_fd": (None, [c_int, c_int, _c_i32_p, vp, c_int, _c_f64_p, c_double, _c_f64_p]),
            "ref_depol_threshold": (c_u32, [c_double]),
            "ref_traj_run_one": (c_int, [_c_cplx_p, c_int, vp, c_int, c_double, c_u64, c_u32, vp, c_int]),
            "ref_threads": (c_int, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _u8(m) -> np.ndarray:
    m = np.asarray(m)
    if m.shape == (8,) and m.dtype == np.float64:
        return np.ascontiguousarray(m)
    m = np.asarray(m, dtype=np.complex128).reshape(-1)
    out = np.empty(2 * m.size, dtype=np.float64)
    out[0::2], out[1::2] = m.real, m.imag
    return out


def _edges(edges) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))


def _w(w):
    if w is None:
        return None, None
    arr = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    return arr, arr.ctypes.data_as(ctypes.c_void_p)


def _nq(psi: np.ndarray) -> int:
    n = int(psi.size).bit_length() - 1
    assert psi.size == 1 << n and psi.dtype == np.complex128 and psi.flags.c_contiguous
    return n


def threads() -> int:
    """OpenMP threads the oracle's element-wise loops use."""
    return int(lib().ref_threads())


# ---------------------------------------------------------------- RNG
def philox4x32_10(ctr, key) -> np.ndarray:
    out = np.zeros(4, dtype=np.uint32)
    lib().ref_philox4x32_10(np.asarray(ctr, dtype=np.uint32), np.asarray(key, dtype=np.uint32), out)
    return out


def depol_threshold(p: float) -> int:
    return int(lib().ref_depol_threshold(p))


# ---------------------------------------------------------------- state init
def init_basis(n: int, index: int) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().ref_init_basis(psi, n, index)
    return psi


def init_uniform(n: int) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().ref_init_uniform(psi, n)
    return psi


def init_random(n: int, seed: int) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().ref_init_random(psi, n, seed)
    return psi


# ---------------------------------------------------------------- gates (in place)
def apply_1q(psi, q, m):
    lib().ref_apply_1q(psi, _nq(psi), q, _u8(m))


def apply_c1q(psi, c, t, m):
    lib().ref_apply_c1q(psi, _nq(psi), c, t, _u8(m))


def apply_diag2(psi, q0, q1, d):
    lib().ref_apply_diag2(psi, _nq(psi), q0, q1, _u8(d))


def apply_swap(psi, a, b):
    lib().ref_apply_swap(psi, _nq(psi), a, b)


def apply_gates(psi, gates: np.ndarray):
    g = np.ascontiguousarray(gates)
    rc = lib().ref_apply_gates(psi, _nq(psi), g.ctypes.data_as(ctypes.c_void_p), len(g))
    if rc != 0:
        raise ValueError("bad gate kind")


def apply_cut_phase(psi, edges, gamma, w=None):
    e = _edges(edges)
    warr, wp = _w(w)
    lib().ref_apply_cut_phase(psi, _nq(psi), len(e), e, wp, gamma)


# ---------------------------------------------------------------- read-outs
def norm2(psi) -> float:
    return lib().ref_norm2(psi, _nq(psi))


def prob_one(psi, q) -> float:
    return lib().ref_prob_one(psi, _nq(psi), q)


def expect_z_all(psi) -> np.ndarray:
    n = _nq(psi)
    out = np.zeros(n, dtype=np.float64)
    lib().ref_expect_z_all(psi, n, out)
    return out


def cut_value(k: int, edges, w=None) -> float:
    e = _edges(edges)
    warr, wp = _w(w)
    return lib().ref_cut_value(k, len(e), e, wp)


def expect_cut(psi, edges, w=None) -> float:
    e = _edges(edges)
    warr, wp = _w(w)
    return lib().ref_expect_cut(psi, _nq(psi), len(e), e, wp)


def expect_diag(psi, d) -> float:
    return lib().ref_expect_diag(psi, _nq(psi), np.ascontiguousarray(d, dtype=np.float64))


def expect_pauli(psi, xmask: int, zmask: int) -> complex:
    out = np.zeros(2, dtype=np.float64)
    if lib().ref_expect_pauli(psi, _nq(psi), xmask, zmask, out) != 0:
        raise MemoryError
    return complex(out[0], out[1])


def inner(a, b) -> complex:
    out = np.zeros(2, dtype=np.float64)
    lib().ref_inner(a, b, _nq(a), out)
    return complex(out[0], out[1])


def sample(psi, shots: int, seed: int):
    out = np.zeros(shots, dtype=np.uint64)
    margin = np.zeros(shots, dtype=np.float64)
    if lib().ref_sample(psi, _nq(psi), shots, seed, out, margin) != 0:
        raise MemoryError
    return out, margin


# ---------------------------------------------------------------- QAOA
def qaoa_state(n, edges, p, theta, w=None):
    e = _edges(edges)
    warr, wp = _w(w)
    psi = np.empty(1 << n, dtype=np.complex128)
    energy = lib().ref_qaoa_state(psi, n, len(e), e, wp, p, np.ascontiguousarray(theta, dtype=np.float64))
    return psi, energy


def qaoa_energy(n, edges, p, theta, w=None) -> float:
    e = _edges(edges)
    warr, wp = _w(w)
    return lib().ref_qaoa_energy(n, len(e), e, wp, p, np.ascontiguousarray(theta, dtype=np.float64))


def qaoa_grad(n, edges, p, theta, w=None):
    e = _edges(edges)
    warr, wp = _w(w)
    grad = np.zeros(2 * p, dtype=np.float64)
    energy = lib().ref_qaoa_grad(n, len(e), e, wp, p, np.ascontiguousarray(theta, dtype=np.float64), grad)
    return energy, grad


def qaoa_grad_fd(n, edges, p, theta, h=1e-6, w=None):
    e = _edges(edges)
    warr, wp = _w(w)
    grad = np.zeros(2 * p, dtype=np.float64)
    lib().ref_qaoa_grad_fd(n, len(e), e, wp, p, np.ascontiguousarray(theta, dtype=np.float64), h, grad)
    return grad


# ---------------------------------------------------------------- trajectories
def traj_run_one(psi, gates, p, seed, t, log_cap=64):
    g = np.ascontiguousarray(gates)
    log = np.zeros(max(log_cap, 1), dtype=np.uint32)
    nins = lib().ref_traj_run_one(psi, _nq(psi), g.ctypes.data_as(ctypes.c_void_p), len(g), p, seed, t,
                                  log.ctypes.data_as(ctypes.c_void_p), log_cap)
    return nins, log[:min(nins, log_cap)].copy()


def expect_x_all(psi) -> np.ndarray:
    n = _nq(psi)
    return np.array([expect_pauli(psi, 1 << q, 0).real for q in range(n)])


def traj_ensemble(n, gates, basis_index, n_traj, p, seed, log_cap=64, ideal=None):
    """Per-trajectory read-outs of the noisy circuit on |basis_index>:
    <Z_i>, <X_i>, fidelity |<ideal|psi_t>|^2, insertion counts and logs, and
    the trajectory-mean computational-basis probabilities."""
    if ideal is None:
        ideal = init_basis(n, basis_index)
        apply_gates(ideal, gates)
    z = np.zeros((n_traj, n))
    x = np.zeros((n_traj, n))
    fid = np.zeros(n_traj)
    counts = np.zeros(n_traj, dtype=np.int64)
    logs = []
    prob_sum = np.zeros(1 << n)
    for t in range(n_traj):
        psi = init_basis(n, basis_index)
        nins, log = traj_run_one(psi, gates, p, seed, t, log_cap)
        counts[t] = nins
        logs.append(log)
        z[t] = expect_z_all(psi)
        x[t] = expect_x_all(psi)
        fid[t] = abs(inner(ideal, psi)) ** 2
        prob_sum += np.abs(psi) ** 2
    return dict(z=z, x=x, fid=fid, counts=counts, logs=logs, prob_mean=prob_sum / n_traj)
