"""Pins for the oracle's stochastic noise gates (one-qubit rotations with
random angles whose ensemble average is the T1/T2 decoherence channel).

The trajectory averages are checked against a density-matrix computation in
which each noise gate is the Pauli channel that scales the qubit's Bloch
vector by (e^{-d/T2}, e^{-d/T2}, e^{-d/T1}) (solved here from those three
factors, not from the rotation angles), and the angle distribution itself
through the first two moments of cos(a) for a normal angle a.
"""
import math

import numpy as np

import oracle
from paper_2001_10554_amd import workloads as W

P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)
PAULIS = [W.PAULI_X, W.PAULI_Y, W.PAULI_Z]


def op(n, factors):
    m = np.array([[1.0 + 0j]])
    for q in range(n - 1, -1, -1):
        m = np.kron(m, factors.get(q, np.eye(2)))
    return m


def pauli_probs(d, T1, T2):
    """(p_X, p_Y, p_Z) of the Pauli channel with Bloch factors
    lx = ly = e^{-d/T2}, lz = e^{-d/T1}: lx = 1 - 2(p_Y + p_Z), etc."""
    lx = ly = math.exp(-d / T2)
    lz = math.exp(-d / T1)
    A = np.array([[0, 1, 1], [1, 0, 1], [1, 1, 0]], dtype=float)
    return np.linalg.solve(A, [(1 - lx) / 2, (1 - ly) / 2, (1 - lz) / 2])


def density_matrix(n, gates, x, p, T1, T2):
    N = 1 << n
    rho = np.zeros((N, N), dtype=np.complex128)
    rho[x, x] = 1
    for gr in gates:
        k, a, b, u = int(gr["kind"]), int(gr["q0"]), int(gr["q1"]), gr["u"]
        if k == W.G_NOISE:
            probs = pauli_probs(u[0], T1, T2)
            rho = (1 - probs.sum()) * rho + sum(pp * op(n, {a: s}) @ rho @ op(n, {a: s}) for pp, s in zip(probs, PAULIS))
            continue
        if k == W.G_1Q:
            G = op(n, {a: W.u8_to_mat(u)})
        elif k == W.G_C1Q:
            G = op(n, {a: P0}) + op(n, {a: P1, b: W.u8_to_mat(u)})
        elif k == W.G_DIAG2:
            d = u[0::2] + 1j * u[1::2]
            G = sum(d[2 * b1 + b0] * op(n, {a: [P0, P1][b0], b: [P0, P1][b1]}) for b0 in (0, 1) for b1 in (0, 1))
        elif k == W.G_SWAP:
            G = 0.5 * (np.eye(N) + sum(op(n, {a: s, b: s}) for s in PAULIS))
        rho = G @ rho @ G.conj().T
        for q in ([a] if k == W.G_1Q else [a, b]):
            rho = (1 - p) * rho + (p / 3) * sum(op(n, {q: s}) @ rho @ op(n, {q: s}) for s in PAULIS)
    return rho


def test_noise_angle_moments():
    """|+>, one noise gate with T1 = inf: only R_Z(a) acts, <X> = cos(a) with
    a ~ N(0, 2d/T2), so E[cos a] = e^{-d/T2} and E[cos^2 a] = (1 + e^{-4d/T2}) / 2."""
    d, T2, T = 1.0, 3.0, 6000
    gates = W.with_noise_gates(W.gates_array([W.gate(W.G_1Q, 0, -1, W.HADAMARD)]), d)
    ens = oracle.traj_ensemble(1, gates, 0, T, 0.0, seed=9, T1=math.inf, T2=T2)
    c = ens["x"][:, 0]
    m1, m2 = math.exp(-d / T2), (1 + math.exp(-4 * d / T2)) / 2
    assert abs(c.mean() - m1) < 4 * c.std() / math.sqrt(T)
    assert abs((c ** 2).mean() - m2) < 4 * (c ** 2).std() / math.sqrt(T)
    assert np.all(np.abs(ens["z"]) < 1e-12)  # a Z rotation keeps |+> on the equator


def test_noise_gates_match_decoherence_channel():
    n, p, T, T1, T2 = 3, 0.02, 3000, 5.0, 4.0
    base = W.random_block(n, 14, seed=3)
    gates = W.with_noise_gates(base, 0.7)
    x = 5
    rho = density_matrix(n, gates, x, p, T1, T2)
    ideal = oracle.init_basis(n, x)
    oracle.apply_gates(ideal, gates)  # noise gates are the identity in the noiseless circuit
    ref_ideal = oracle.init_basis(n, x)
    oracle.apply_gates(ref_ideal, base)
    assert np.max(np.abs(ideal - ref_ideal)) == 0
    ens = oracle.traj_ensemble(n, gates, x, T, p, seed=21, ideal=ideal, T1=T1, T2=T2)
    f_exact = np.vdot(ideal, rho @ ideal).real
    assert abs(ens["fid"].mean() - f_exact) < 4 * ens["fid"].std() / math.sqrt(T) + 1e-12
    for q in range(n):
        for key, P in (("x", W.PAULI_X), ("z", W.PAULI_Z)):
            e = np.trace(op(n, {q: P}) @ rho).real
            v = ens[key][:, q]
            assert abs(v.mean() - e) < 4 * v.std() / math.sqrt(T) + 1e-12, (q, key)
    # noise gates draw no insertion slots
    slots = T * sum(1 if int(g["kind"]) == W.G_1Q else 2 for g in base)
    assert abs(ens["counts"].sum() / slots - p) < 4 * math.sqrt(p * (1 - p) / slots)


def test_noise_gates_without_decay_are_identity():
    n = 4
    gates = W.with_noise_gates(W.qft_circuit(n), 2.0)
    ideal = oracle.init_basis(n, 6)
    oracle.apply_gates(ideal, gates)
    psi = oracle.init_basis(n, 6)
    nins, _ = oracle.traj_run_one(psi, gates, 0.0, 1, 0, T1=math.inf, T2=math.inf)
    assert nins == 0 and np.max(np.abs(psi - ideal)) < 1e-15
