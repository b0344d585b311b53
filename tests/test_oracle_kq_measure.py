"""Pins for the oracle's dense k-qubit gate, collapse and Born measurement,
and for the named-gate table of the product's Python layer.

The k-qubit gate is checked against numpy tensor contraction over the
register viewed as an n-axis tensor (a different algorithm), against the
one- and two-qubit oracle gates it must reduce to, and against Kronecker
products of one-qubit gates.  Collapse is checked against explicit
projectors, measurement against the Born frequencies over many seeds.  The
named gates are checked against matrix exponentials of Pauli generators and
projector forms.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

import oracle
from paper_2001_10554_amd import gates as G
from paper_2001_10554_amd import workloads as W


def rand_state(n, seed):
    g = np.random.default_rng(seed)
    v = g.standard_normal(1 << n) + 1j * g.standard_normal(1 << n)
    return v / np.linalg.norm(v)


def rand_unitary(k, seed):
    g = np.random.default_rng(seed)
    a = g.standard_normal((1 << k, 1 << k)) + 1j * g.standard_normal((1 << k, 1 << k))
    q, r = np.linalg.qr(a)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def tensordot_apply(psi, n, qubits, U):
    """Register as a tensor with axis a = qubit n-1-a; U reshaped to
    (2,)*2k with matrix bit m <-> qubit qubits[m]."""
    k = len(qubits)
    t = psi.reshape((2,) * n)
    u = U.reshape((2,) * (2 * k))
    # matrix row/col index bits are big-endian in the reshape: axis i <-> bit k-1-i
    in_axes = [n - 1 - qubits[k - 1 - i] for i in range(k)]
    out = np.tensordot(u, t, axes=(list(range(k, 2 * k)), in_axes))
    # out axes: k output axes (bits k-1..0) followed by the untouched axes in order
    rest = [a for a in range(n) if a not in in_axes]
    order = [None] * n
    for i in range(k):
        order[in_axes[i]] = i
    for j, a in enumerate(rest):
        order[a] = k + j
    return np.transpose(out, order).reshape(-1)


@pytest.mark.parametrize("qubits", [[0], [3], [2, 5], [5, 2], [0, 6, 3], [1, 4, 0, 6], [6, 0, 3, 2, 5]])
def test_kq_vs_tensor_contraction(qubits):
    n = 7
    U = rand_unitary(len(qubits), sum(qubits) + 10 * len(qubits))
    psi = rand_state(n, 1)
    ref = tensordot_apply(psi, n, qubits, U)
    oracle.apply_kq(psi, qubits, U)
    assert np.max(np.abs(psi - ref)) < 1e-13


def test_kq_reduces_to_one_and_two_qubit_gates():
    n = 6
    U = W.haar_2x2(np.random.default_rng(3))
    a = rand_state(n, 2)
    b = a.copy()
    oracle.apply_kq(a, [4], U)
    oracle.apply_1q(b, 4, U)
    assert np.max(np.abs(a - b)) < 1e-15
    # CNOT(c=1, t=3): qubit list [c, t], flip matrix bit 1 when bit 0 is set
    cx = np.eye(4, dtype=np.complex128)[[0, 3, 2, 1]]
    a = rand_state(n, 3)
    b = a.copy()
    oracle.apply_kq(a, [1, 3], cx)
    oracle.apply_c1q(b, 1, 3, G.X)
    assert np.max(np.abs(a - b)) < 1e-15
    d = np.exp(1j * np.array([0.1, 0.2, 0.3, 0.4]))
    a = rand_state(n, 4)
    b = a.copy()
    oracle.apply_kq(a, [5, 0], np.diag(d))
    oracle.apply_diag2(b, 5, 0, d)
    assert np.max(np.abs(a - b)) < 1e-15
    # Kronecker product: bit 0 of the matrix index is the first listed qubit
    U0, U1 = W.haar_2x2(np.random.default_rng(5)), W.haar_2x2(np.random.default_rng(6))
    a = rand_state(n, 5)
    b = a.copy()
    oracle.apply_kq(a, [2, 4], np.kron(U1, U0))
    oracle.apply_1q(b, 2, U0)
    oracle.apply_1q(b, 4, U1)
    assert np.max(np.abs(a - b)) < 1e-14
    with pytest.raises(ValueError):
        oracle.apply_kq(rand_state(7, 1), [0, 1, 2, 3, 4, 5], np.eye(64))


def _proj(n, q, v):
    idx = np.arange(1 << n)
    return ((idx >> q) & 1) == v


@pytest.mark.parametrize("q,outcome", [(0, 0), (0, 1), (3, 1), (5, 0)])
def test_collapse_vs_projector(q, outcome):
    n = 6
    psi = rand_state(n, 7)
    keep = _proj(n, q, outcome)
    P = np.sum(np.abs(psi[keep]) ** 2)
    ref = np.where(keep, psi, 0) / math.sqrt(P)
    p = oracle.collapse(psi, q, outcome)
    assert abs(p - P) < 1e-15
    assert np.max(np.abs(psi - ref)) < 1e-15
    assert abs(oracle.norm2(psi) - 1) < 1e-14
    # a second collapse onto the same outcome is certain and changes nothing
    before = psi.copy()
    assert abs(oracle.collapse(psi, q, outcome) - 1) < 1e-14
    assert np.max(np.abs(psi - before)) < 1e-15
    # the other outcome now has probability 0: the state becomes 0
    assert oracle.collapse(psi, q, 1 - outcome) == 0 and not np.any(psi)


def test_measure_born_frequencies_and_post_state():
    n, q = 5, 2
    base = oracle.init_basis(n, 0)
    oracle.apply_1q(base, q, G.ry(2 * math.acos(math.sqrt(0.3))))  # P(0) = 0.3
    oracle.apply_1q(base, 4, G.H)
    ones = 0
    trials = 4000
    for seed in range(trials):
        psi = base.copy()
        out, p = oracle.measure(psi, q, seed)
        assert abs(p - (0.7 if out else 0.3)) < 1e-14
        assert abs(oracle.expect_z_all(psi)[q] - (-1 if out else 1)) < 1e-14
        assert abs(oracle.norm2(psi) - 1) < 1e-14
        ones += out
    # binomial(4000, 0.7): 4 standard deviations
    assert abs(ones - 0.7 * trials) < 4 * math.sqrt(trials * 0.21)
    assert scipy.stats.binomtest(ones, trials, 0.7).pvalue > 1e-4
    # certain outcomes
    psi = oracle.init_basis(n, 1 << q)
    assert oracle.measure(psi, q, 123)[0] == 1
    psi = oracle.init_basis(n, 0)
    assert oracle.measure(psi, q, 123)[0] == 0


def _expm_rot(P, theta):
    return scipy.linalg.expm(-0.5j * theta * P)


def test_named_gate_table():
    for th in (0.3, -1.7, 2.9):
        assert np.allclose(G.rx(th), _expm_rot(G.X, th), atol=1e-15)
        assert np.allclose(G.ry(th), _expm_rot(G.Y, th), atol=1e-15)
        assert np.allclose(G.rz(th), _expm_rot(G.Z, th), atol=1e-15)
        ph = np.exp(0.5j * th)  # phase(th) = e^{i th / 2} Rz(th)
        assert np.allclose(G.phase(th), ph * G.rz(th), atol=1e-15)
    t, p, l = 0.7, 1.1, -0.4
    ref = G.rz(p) @ G.ry(t) @ G.rz(l)
    m = G.u3(t, p, l)
    c = m[0, 0] / ref[0, 0]
    assert abs(abs(c) - 1) < 1e-14 and np.allclose(m, c * ref, atol=1e-14)
    assert np.allclose(G.H @ G.H, np.eye(2)) and np.allclose(G.H @ G.X @ G.H, G.Z)
    assert np.allclose(G.S @ G.S, G.Z) and np.allclose(G.T @ G.T, G.S) and np.allclose(G.SX @ G.SX, G.X)
    assert np.allclose(G.S @ G.SDG, np.eye(2)) and np.allclose(G.T @ G.TDG, np.eye(2))
    assert np.allclose(np.diag(G.CZ_DIAG), scipy.linalg.expm(1j * math.pi * np.diag([0, 0, 0, 1.0])))
    # iSWAP = exp(i pi/4 (XX + YY))
    assert np.allclose(G.ISWAP, scipy.linalg.expm(0.25j * math.pi * (np.kron(G.X, G.X) + np.kron(G.Y, G.Y))), atol=1e-14)
    # Toffoli on list [c0, c1, t]: matrix bit m <-> list entry m, so kron(t, c1, c0)
    P0, P1, I = np.diag([1, 0]).astype(complex), np.diag([0, 1]).astype(complex), np.eye(2)
    tof = np.kron(I, np.eye(4)) - np.kron(I, np.kron(P1, P1)) + np.kron(G.X, np.kron(P1, P1))
    assert np.array_equal(G.TOFFOLI, tof)
    # Fredkin on [c, a, b]: controlled swap of a and b
    sw = np.eye(4)[[0, 2, 1, 3]]  # swap of the two bits of a 2-bit index
    fred = np.kron(np.eye(4), P0) + np.kron(sw, P1)
    assert np.array_equal(G.FREDKIN, fred)
