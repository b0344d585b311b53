"""CPU oracle for the state-vector simulator — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (the HIP library and its
Python binding) never imports it, and it never imports the product: the two
share only the seeded inputs of ``paper_2001_10554_amd.workloads``.

The arithmetic lives in ``qsim_ref.c`` (plain complex128 C, one gate at a time,
long-double sequential reductions, chunked for whole-register expectations).
This module is ctypes marshalling plus a
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
    """Compile the oracle with gcc (OpenMP on element-wise loops and on the
    fixed chunks of its long sums)."""
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
            "ref_random_raw": (None, [c_u64, c_u64, c_u64, _c_cplx_p]),
            "ref_cut_value": (c_double, [c_u64, c_int, _c_i32_p, vp]),
            "ref_cut_max": (c_double, [c_int, c_int, _c_i32_p, vp, _c_u64_p]),
            "ref_apply_kq": (c_int, [_c_cplx_p, c_int, _c_i32_p, c_int, _c_f64_p]),
            "ref_collapse": (c_double, [_c_cplx_p, c_int, c_int, c_int]),
            "ref_measure": (c_int, [_c_cplx_p, c_int, c_int, c_u64, _c_f64_p]),
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
            "ref_traj_run_one": (c_int, [vp, c_int, vp, c_int, c_double, c_u64, c_u32, vp, c_int, c_double, c_double]),
            "ref_threads": (c_int, []),
            "ref_set_threads": (None, [c_int]),
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


def set_threads(t: int) -> None:
    """Threads for the oracle's element-wise loops (results do not depend on it)."""
    lib().ref_set_threads(int(t))


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


def random_raw(seed: int, first: int, count: int) -> np.ndarray:
    """Amplitudes first .. first+count-1 of init_random's definition before
    the division by the norm (indices may exceed any register held here)."""
    out = np.empty(count, dtype=np.complex128)
    lib().ref_random_raw(seed, first, count, out)
    return out


# ---------------------------------------------------------------- gates (in place)
def apply_1q(psi, q, m):
    lib().ref_apply_1q(psi, _nq(psi), q, _u8(m))


def apply_c1q(psi, c, t, m):
    lib().ref_apply_c1q(psi, _nq(psi), c, t, _u8(m))


def apply_diag2(psi, q0, q1, d):
    lib().ref_apply_diag2(psi, _nq(psi), q0, q1, _u8(d))


def apply_swap(psi, a, b):
    lib().ref_apply_swap(psi, _nq(psi), a, b)


def apply_kq(psi, qubits, m):
    """k-qubit matrix m (2^k x 2^k, row = output); bit j of its index is qubits[j]."""
    qs = np.ascontiguousarray(qubits, dtype=np.int32)
    m = np.asarray(m, dtype=np.complex128)
    u = np.empty(2 * m.size)
    u[0::2], u[1::2] = m.real.reshape(-1), m.imag.reshape(-1)
    if lib().ref_apply_kq(psi, _nq(psi), qs, len(qs), u) != 0:
        raise ValueError("k must be in [1, 5]")


def collapse(psi, q, outcome) -> float:
    return lib().ref_collapse(psi, _nq(psi), q, int(outcome))


def measure(psi, q, seed):
    prob = np.zeros(1)
    out = lib().ref_measure(psi, _nq(psi), q, seed, prob)
    return int(out), float(prob[0])


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


def cut_max(n: int, edges, w=None):
    """(E_exact, smallest maximiser): the Max-Cut optimum by enumeration."""
    e = _edges(edges)
    warr, wp = _w(w)
    arg = np.zeros(1, dtype=np.uint64)
    best = lib().ref_cut_max(n, len(e), e, wp, arg)
    return best, int(arg[0])


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
def _inv(T):
    return 0.0 if T is None or not np.isfinite(T) else 1.0 / T


def traj_run_one(psi, gates, p, seed, t, log_cap=64, T1=None, T2=None):
    """Trajectory t in place on psi; psi = None makes the draws only."""
    g = np.ascontiguousarray(gates)
    log = np.zeros(max(log_cap, 1), dtype=np.uint32)
    n = 0 if psi is None else _nq(psi)
    nins = lib().ref_traj_run_one(None if psi is None else psi.ctypes.data_as(ctypes.c_void_p), n,
                                  g.ctypes.data_as(ctypes.c_void_p), len(g), p, seed, t,
                                  log.ctypes.data_as(ctypes.c_void_p), log_cap, _inv(T1), _inv(T2))
    return nins, log[:min(nins, log_cap)].copy()


def traj_draws(gates, p, seed, t, log_cap=64):
    """Insertion count and log of trajectory t (the draws of traj_run_one
    without the state)."""
    return traj_run_one(None, gates, p, seed, t, log_cap)


def expect_x_all(psi) -> np.ndarray:
    n = _nq(psi)
    return np.array([expect_pauli(psi, 1 << q, 0).real for q in range(n)])


def traj_ensemble(n, gates, basis_index, n_traj, p, seed, log_cap=64, ideal=None, T1=None, T2=None, diag=None):
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
    dval = np.zeros(n_traj)
    for t in range(n_traj):
        psi = init_basis(n, basis_index)
        nins, log = traj_run_one(psi, gates, p, seed, t, log_cap, T1, T2)
        if diag is not None:
            dval[t] = expect_diag(psi, diag)
        counts[t] = nins
        logs.append(log)
        z[t] = expect_z_all(psi)
        x[t] = expect_x_all(psi)
        fid[t] = abs(inner(ideal, psi)) ** 2
        prob_sum += np.abs(psi) ** 2
    return dict(z=z, x=x, fid=fid, counts=counts, logs=logs, prob_mean=prob_sum / n_traj, diag=dval)


# ---------------------------------------------------------------- particle swarm
# Sec. "Particle Swarm / QAOA Simulation": each particle is one virtual
# device evaluating L(theta) = <C> at its position theta (2p angles); every
# graph has its own swarm of R particles.  Positions and velocities start
# uniform in [0, 2 pi); after each round of evaluations the personal and
# global bests are updated and the velocity follows eq. (4), then the
# particle moves by its velocity.
#
# Readings where the paper is silent or at odds with itself:
# * eq. (4) as printed pulls along (theta_k - best); the standard form of its
#   cited source pulls toward the best, (best - theta_k).  `attract = +1`
#   (default) takes the standard form, `attract = -1` the printed one.
# * r_p and r_g are scalars per particle and round (as written), not
#   per-coordinate draws.
# * bests maximise <C> (the largest eigenvalue of the cut observable is
#   sought); a personal or global best moves only on strict improvement,
#   the global best to the lowest-index particle among equal maxima.
# * positions are not wrapped into [0, 2 pi).
# Draws: Philox4x32-10 with key = seed and counter (c, d, 5, 0) for the
# initial position / velocity of coordinate d of particle c = g R + k
# (position 2 pi u53(x0, x1), velocity 2 pi u53(x2, x3)); counter
# (c, round, 4, 0) for r_p = u53(x0, x1) and r_g = u53(x2, x3).
TAG_PSO, TAG_PSO_INIT = 4, 5
TWO_PI = 2.0 * np.pi
PSO_PAPER = dict(omega=0.66, phi_p=1.6, phi_g=0.62)


def _u53(lo, hi) -> float:
    return float(((int(hi) << 32) | int(lo)) >> 11) * 2.0 ** -53


def _draw(seed: int, w0: int, w1: int, tag: int) -> np.ndarray:
    return philox4x32_10([w0, w1, tag, 0], [seed & 0xFFFFFFFF, seed >> 32])


def pso_init(G: int, R: int, D: int, seed: int):
    """Swarm state dict: pos, vel, pbest [G, R, D]; pbest_val [G, R];
    gbest [G, D]; gbest_val [G] (values -inf before the first round)."""
    pos = np.empty((G, R, D))
    vel = np.empty((G, R, D))
    for g in range(G):
        for k in range(R):
            for d in range(D):
                x = _draw(seed, g * R + k, d, TAG_PSO_INIT)
                pos[g, k, d] = TWO_PI * _u53(x[0], x[1])
                vel[g, k, d] = TWO_PI * _u53(x[2], x[3])
    return dict(pos=pos, vel=vel, pbest=pos.copy(), pbest_val=np.full((G, R), -np.inf),
                gbest=np.zeros((G, D)), gbest_val=np.full(G, -np.inf))


def pso_update_bests(sw, E):
    """Fold one round of evaluations E [G, R] into the personal and global bests."""
    G, R = E.shape
    for g in range(G):
        for k in range(R):
            if E[g, k] > sw["pbest_val"][g, k]:
                sw["pbest_val"][g, k] = E[g, k]
                sw["pbest"][g, k] = sw["pos"][g, k]
        for k in range(R):
            if sw["pbest_val"][g, k] > sw["gbest_val"][g]:
                sw["gbest_val"][g] = sw["pbest_val"][g, k]
                sw["gbest"][g] = sw["pbest"][g, k]


def pso_move(sw, rnd: int, seed: int, omega=0.66, phi_p=1.6, phi_g=0.62, attract=1):
    """Eq. (4) for every particle, then theta <- theta + v."""
    G, R, D = sw["pos"].shape
    for g in range(G):
        for k in range(R):
            x = _draw(seed, g * R + k, rnd, TAG_PSO)
            rp, rg = _u53(x[0], x[1]), _u53(x[2], x[3])
            th = sw["pos"][g, k]
            to_p = (sw["pbest"][g, k] - th) * attract
            to_g = (sw["gbest"][g] - th) * attract
            sw["vel"][g, k] = omega * sw["vel"][g, k] + phi_p * rp * to_p + phi_g * rg * to_g
            sw["pos"][g, k] = th + sw["vel"][g, k]


def pso_run(objective, G: int, R: int, D: int, rounds: int, seed: int, attract=1, **params):
    """`rounds` rounds of evaluation (the first at the initial positions);
    the swarm moves between rounds.  objective(pos [G, R, D]) -> E [G, R].
    Returns (swarm, history [rounds, G] of the global best after each round,
    evaluations [rounds, G, R])."""
    prm = dict(PSO_PAPER, **params)
    sw = pso_init(G, R, D, seed)
    hist = np.zeros((rounds, G))
    evals = np.zeros((rounds, G, R))
    for r in range(rounds):
        E = np.asarray(objective(sw["pos"]), dtype=np.float64).reshape(G, R)
        evals[r] = E
        pso_update_bests(sw, E)
        hist[r] = sw["gbest_val"]
        if r + 1 < rounds:
            pso_move(sw, r, seed, attract=attract, **prm)
    return sw, hist, evals


def qaoa_objective(graphs, n_qubits, p: int):
    """<C> of the QAOA circuit of graph g at each particle's angles."""
    def f(pos):
        G, R, _ = pos.shape
        return np.array([[qaoa_energy(int(n_qubits[g]), graphs[g], p, pos[g, k]) for k in range(R)] for g in range(G)])
    return f
