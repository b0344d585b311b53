"""Pins for the CPU oracle against things other than itself.

Each check compares the oracle (plain C) with an independent construction:
explicit Kronecker-product operators built with numpy, scipy's matrix
exponential, closed forms, the paper's worked example, published Philox
known-answer vectors, or a density-matrix computation.  A plausible mistake in
the oracle (dropped term, wrong sign or index, transposed operand, swapped
qubit order) fails at least one of these.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_2001_10554_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

I2 = np.eye(2, dtype=np.complex128)
P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)


def op(n, factors):
    """Full 2^n operator: kron over qubits n-1 (leftmost) .. 0 (rightmost)."""
    m = np.array([[1.0 + 0j]])
    for q in range(n - 1, -1, -1):
        m = np.kron(m, factors.get(q, I2))
    return m


def rand_state(n, seed):
    g = np.random.default_rng(seed)
    v = g.standard_normal(1 << n) + 1j * g.standard_normal(1 << n)
    return v / np.linalg.norm(v)


# ------------------------------------------------------------------ Philox
def test_philox_known_answer_vectors():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = oracle.philox4x32_10(v[0:4], v[4:6])
        assert list(out) == v[6:10]


# ------------------------------------------------------------------ gates vs Kronecker
@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_apply_1q_matches_kronecker(n):
    for q in range(n):
        psi = rand_state(n, 10 * n + q)
        U = W.haar_list(100 + q, 1)[0]
        want = op(n, {q: U}) @ psi
        got = psi.copy()
        oracle.apply_1q(got, q, U)
        assert np.max(np.abs(got - want)) < 1e-14


def test_apply_1q_nonunitary_orientation():
    # A non-symmetric, non-unitary matrix distinguishes U from U^T and rows from columns.
    M = np.array([[1 + 2j, 3 - 1j], [-0.5j, 4.0]])
    n = 3
    for q in range(n):
        psi = rand_state(n, q)
        got = psi.copy()
        oracle.apply_1q(got, q, M)
        assert np.allclose(got, op(n, {q: M}) @ psi, atol=1e-13)


@pytest.mark.parametrize("n", [2, 3, 6])
def test_apply_c1q_matches_projector_form(n):
    g = np.random.default_rng(n)
    for _ in range(6):
        c, t = (int(x) for x in g.choice(n, 2, replace=False))
        U = W.haar_2x2(g)
        full = op(n, {c: P0}) + op(n, {c: P1, t: U})
        psi = rand_state(n, c * 7 + t)
        got = psi.copy()
        oracle.apply_c1q(got, c, t, U)
        assert np.max(np.abs(got - full @ psi)) < 1e-14


def test_apply_diag2_and_swap():
    n = 5
    g = np.random.default_rng(3)
    X = W.PAULI_X
    Y = W.PAULI_Y
    Z = W.PAULI_Z
    for _ in range(6):
        a, b = (int(x) for x in g.choice(n, 2, replace=False))
        d = np.exp(1j * g.uniform(0, 6.3, 4))
        full = sum(d[2 * b1 + b0] * op(n, {a: [P0, P1][b0], b: [P0, P1][b1]}) for b0 in (0, 1) for b1 in (0, 1))
        psi = rand_state(n, a + 11 * b)
        got = psi.copy()
        oracle.apply_diag2(got, a, b, d)
        assert np.max(np.abs(got - full @ psi)) < 1e-14
        # SWAP = (I + XX + YY + ZZ) / 2
        sw = 0.5 * (np.eye(1 << n) + op(n, {a: X, b: X}) + op(n, {a: Y, b: Y}) + op(n, {a: Z, b: Z}))
        got = psi.copy()
        oracle.apply_swap(got, a, b)
        assert np.max(np.abs(got - sw @ psi)) < 1e-14


def test_gate_list_is_product_of_kronecker_unitaries():
    n = 6
    gates = W.random_block(n, 40, seed=5)
    Ufull = np.eye(1 << n, dtype=np.complex128)
    for gr in gates:
        k, a, b, u = int(gr["kind"]), int(gr["q0"]), int(gr["q1"]), gr["u"]
        m = W.u8_to_mat(u)
        if k == W.G_1Q:
            G = op(n, {a: m})
        elif k == W.G_C1Q:
            G = op(n, {a: P0}) + op(n, {a: P1, b: m})
        elif k == W.G_DIAG2:
            d = u[0::2] + 1j * u[1::2]
            G = sum(d[2 * b1 + b0] * op(n, {a: [P0, P1][b0], b: [P0, P1][b1]}) for b0 in (0, 1) for b1 in (0, 1))
        else:
            G = 0.5 * (np.eye(1 << n) + op(n, {a: W.PAULI_X, b: W.PAULI_X}) + op(n, {a: W.PAULI_Y, b: W.PAULI_Y})
                       + op(n, {a: W.PAULI_Z, b: W.PAULI_Z}))
        Ufull = G @ Ufull
    psi = rand_state(n, 1)
    got = psi.copy()
    oracle.apply_gates(got, gates)
    assert np.max(np.abs(got - Ufull @ psi)) < 1e-13
    assert abs(oracle.norm2(got) - 1.0) < 1e-13


# ------------------------------------------------------------------ initialisation
def test_init_basis_uniform():
    for n in (1, 4, 9):
        psi = oracle.init_uniform(n)
        assert np.max(np.abs(psi - 2 ** (-n / 2))) < 1e-15
        b = oracle.init_basis(n, (1 << n) - 1)
        assert b[-1] == 1 and np.count_nonzero(b) == 1


def test_init_random_normalised_and_seeded():
    a = oracle.init_random(12, 2)
    b = oracle.init_random(12, 2)
    c = oracle.init_random(12, 3)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert abs(np.linalg.norm(a) - 1.0) < 1e-14
    # Components are scaled uniforms on [-1, 1): zero mean, variance 1/3 before normalisation.
    s = a * np.sqrt(oracle.norm2(a)) / np.sqrt(np.mean(np.abs(a) ** 2)) / np.sqrt(2 / 3)
    assert abs(np.mean(s.real)) < 0.05 and abs(np.mean(s.imag)) < 0.05
    # First amplitude from the Philox words directly: (2u-1) + i(2v-1) up to the norm.
    x = oracle.philox4x32_10([0, 0, 1, 0], [2, 0]).astype(np.uint64)
    u = float(((x[1] << np.uint64(32)) | x[0]) >> np.uint64(11)) / 2 ** 53
    v = float(((x[3] << np.uint64(32)) | x[2]) >> np.uint64(11)) / 2 ** 53
    raw = complex(2 * u - 1, 2 * v - 1)
    scale = raw / a[0]
    assert abs(scale.imag) < 1e-12 and scale.real > 0


def _philox_np(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 (Salmon et al., SC'11) on numpy uint64 arrays of 32-bit
    words, written here independently of the oracle's C; pinned by the
    published known-answer vectors below."""
    m32 = np.uint64(0xFFFFFFFF)
    c = [np.asarray(x, dtype=np.uint64) & m32 for x in (c0, c1, c2, c3)]
    k = [np.uint64(k0), np.uint64(k1)]
    for r in range(10):
        if r:
            k = [(k[0] + np.uint64(0x9E3779B9)) & m32, (k[1] + np.uint64(0xBB67AE85)) & m32]
        p0 = np.uint64(0xD2511F53) * c[0]
        p1 = np.uint64(0xCD9E8D57) * c[2]
        c = [((p1 >> np.uint64(32)) ^ c[1] ^ k[0]) & m32, p1 & m32, ((p0 >> np.uint64(32)) ^ c[3] ^ k[1]) & m32, p0 & m32]
    return c


def test_numpy_philox_matches_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if l.strip() and not l.startswith("#")]
    for r in rows:
        v = [int(x, 16) for x in r]
        out = _philox_np(*[np.array([x]) for x in v[0:4]], v[4], v[5])
        assert [int(o[0]) for o in out] == v[6:10]


@pytest.mark.parametrize("first", [0, (1 << 32) - 8, 1 << 32, (1 << 33) + 12345, (1 << 34) - 16, (1 << 35) + 7])
def test_init_random_counter_layout_at_any_index(first):
    """init_random's definition at indices up to 2^35 (registers the CPU
    cannot hold): amplitude i before normalisation is (2u - 1) + i(2v - 1)
    with u, v the 53-bit uniforms of Philox(key = seed, counter = (i mod
    2^32, i div 2^32, 1, 0)), words (0, 1) and (2, 3)."""
    seed = 0x1234_5678_9ABC
    idx = np.arange(first, first + 16, dtype=np.uint64)
    x = _philox_np(idx & np.uint64(0xFFFFFFFF), idx >> np.uint64(32), np.full(16, 1), np.zeros(16),
                   seed & 0xFFFFFFFF, seed >> 32)
    u = ((x[1] << np.uint64(32)) | x[0]) >> np.uint64(11)
    v = ((x[3] << np.uint64(32)) | x[2]) >> np.uint64(11)
    want = (2 * (u.astype(np.float64) * 2.0 ** -53) - 1) + 1j * (2 * (v.astype(np.float64) * 2.0 ** -53) - 1)
    got = oracle.random_raw(seed, first, 16)
    assert np.array_equal(got, want)
    # the high counter word matters: index i and i + 2^32 differ
    if first >= 1 << 32:
        assert not np.array_equal(got, oracle.random_raw(seed, first - (1 << 32), 16))


def test_init_random_is_raw_over_norm():
    n, seed = 10, 77
    raw = oracle.random_raw(seed, 0, 1 << n)
    psi = oracle.init_random(n, seed)
    assert np.max(np.abs(psi - raw / np.linalg.norm(raw))) < 1e-16


# ------------------------------------------------------------------ paper's worked examples
def test_paper_basic_use_listing():
    rows = {}
    amps = []
    for l in open(os.path.join(GOLDEN, "paper_basic_use.txt")):
        if l.startswith("#") or not l.strip():
            continue
        f = l.split()
        if f[0] == "amp":
            amps.append((int(f[1]), complex(float(f[2]), float(f[3]))))
        else:
            rows[f[0]] = f[1:]
    n = int(rows["n"][0])
    psi = oracle.init_basis(n, int(rows["init_basis"][0]))
    oracle.apply_1q(psi, 1, W.PAULI_X)
    oracle.apply_1q(psi, 0, W.HADAMARD)
    oracle.apply_c1q(psi, 1, 0, W.PAULI_X)
    p = oracle.prob_one(psi, 1)
    assert abs(p - float(rows["prob_one"][1])) < 1e-15
    z = -1 * p + 1 * (1 - p)
    assert abs(z - float(rows["expect_z"][1])) < 1e-15
    assert abs(oracle.expect_z_all(psi)[1] - z) < 1e-15
    want = np.zeros(1 << n, dtype=np.complex128)
    for i, a in amps:
        want[i] = a
    assert np.max(np.abs(psi - want)) < 1e-15


def test_appendix_rotation_circuit_noiseless():
    """Appendix (pool of states): RX by random angles on each of 10 qubits from
    |0..0>; without noise P(q0 = 1) = sin^2(theta_0 / 2) for RX = exp(-i theta X/2)."""
    n = 10
    theta = np.random.default_rng(777777).uniform(0, math.pi, n)
    psi = oracle.init_basis(n, 0)
    for q in range(n):
        oracle.apply_1q(psi, q, W.rot_x(theta[q]))
    for q in range(n):
        assert abs(oracle.prob_one(psi, q) - math.sin(theta[q] / 2) ** 2) < 1e-14


# ------------------------------------------------------------------ read-outs
def test_probabilities_and_z_vs_marginals():
    n = 7
    psi = rand_state(n, 9)
    p = np.abs(psi) ** 2
    z = oracle.expect_z_all(psi)
    for q in range(n):
        marg = p.reshape(1 << (n - q - 1), 2, 1 << q).sum(axis=(0, 2))
        assert abs(oracle.prob_one(psi, q) - marg[1]) < 1e-15
        assert abs(z[q] - (marg[0] - marg[1])) < 1e-15
        Zq = op(n, {q: W.PAULI_Z})
        assert abs(z[q] - np.vdot(psi, Zq @ psi).real) < 1e-14


@pytest.mark.parametrize("xmask,zmask", [(0, 0), (1, 0), (0, 4), (5, 5), (0b1011, 0b0110), (0b1111111, 0b1010101)])
def test_expect_pauli_vs_kronecker(xmask, zmask):
    n = 7
    psi = rand_state(n, xmask * 31 + zmask)
    f = {}
    for q in range(n):
        x, z = (xmask >> q) & 1, (zmask >> q) & 1
        if x and z:
            f[q] = W.PAULI_Y
        elif x:
            f[q] = W.PAULI_X
        elif z:
            f[q] = W.PAULI_Z
    want = np.vdot(psi, op(n, f) @ psi)
    got = oracle.expect_pauli(psi, xmask, zmask)
    assert abs(got - want) < 1e-14
    assert abs(got.imag) < 1e-14


def test_inner_and_norm():
    a, b = rand_state(6, 1), rand_state(6, 2)
    assert abs(oracle.inner(a, b) - np.vdot(a, b)) < 1e-15
    assert abs(oracle.norm2(3 * a) - 9.0) < 1e-13


def test_cut_value_and_expectation_closed_forms():
    # Max over k of C(k): the maximum cut.  K4 (3-regular): 4.  Ring of even n: n.
    k4 = np.array([(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)], dtype=np.int32)
    assert max(oracle.cut_value(k, k4) for k in range(16)) == 4
    ring = W.ring_graph(8)
    assert max(oracle.cut_value(k, ring) for k in range(256)) == 8
    # C as sum_e (I - Z_u Z_v)/2 built from Kronecker products.
    g = W.random_regular_graph(8, 3, seed=1)
    n = 8
    C = sum(0.5 * (np.eye(1 << n) - op(n, {int(u): W.PAULI_Z, int(v): W.PAULI_Z})) for u, v in g)
    diag = np.real(np.diag(C))
    assert all(oracle.cut_value(k, g) == diag[k] for k in range(1 << n))
    psi = rand_state(n, 4)
    assert abs(oracle.expect_cut(psi, g) - np.vdot(psi, C @ psi).real) < 1e-13
    assert abs(oracle.expect_diag(psi, diag) - np.vdot(psi, C @ psi).real) < 1e-13
    # Uniform superposition cuts each edge with probability 1/2.
    assert abs(oracle.expect_cut(oracle.init_uniform(n), g) - len(g) / 2) < 1e-13
    # Weighted edges: weights scale each edge term.
    w = np.linspace(0.5, 2.0, len(g))
    Cw = sum(wi * 0.5 * (np.eye(1 << n) - op(n, {int(u): W.PAULI_Z, int(v): W.PAULI_Z})) for wi, (u, v) in zip(w, g))
    assert abs(oracle.expect_cut(psi, g, w) - np.vdot(psi, Cw @ psi).real) < 1e-13
    # Cost phase equals expm(-i gamma C).
    ph = psi.copy()
    oracle.apply_cut_phase(ph, g, 0.37)
    assert np.max(np.abs(ph - scipy.linalg.expm(-1j * 0.37 * C) @ psi)) < 1e-13


def test_sample_distribution_and_rule():
    n = 6
    psi = rand_state(n, 12)
    shots = 200000
    s, margin = oracle.sample(psi, shots, seed=99)
    p = np.abs(psi) ** 2
    cnt = np.bincount(s.astype(np.int64), minlength=1 << n)
    chi2 = np.sum((cnt - shots * p) ** 2 / (shots * p))
    # 63 degrees of freedom: mean 63, sd ~ 11.2; 5 sigma bound.
    assert chi2 < 63 + 5 * math.sqrt(2 * 63)
    # Rule: smallest i with CDF(i) > u, CDF from numpy's cumulative sum.
    x = [oracle.philox4x32_10([k, 0, 2, 0], [99, 0]).astype(np.uint64) for k in range(50)]
    u = np.array([float(((w[1] << np.uint64(32)) | w[0]) >> np.uint64(11)) / 2 ** 53 for w in x])
    assert np.array_equal(s[:50], np.searchsorted(np.cumsum(p), u, side="right"))
    # Degenerate: a basis state always yields its index.
    b = oracle.init_basis(5, 19)
    sb, _ = oracle.sample(b, 1000, seed=3)
    assert np.all(sb == 19)


# ------------------------------------------------------------------ QFT (trajectory circuit)
@pytest.mark.parametrize("n", [3, 5, 8])
def test_qft_gate_list_matches_textbook(n):
    gates = W.qft_circuit(n)
    assert len(gates) == n + n * (n - 1) // 2 + n // 2
    N = 1 << n
    for x in (0, 1, N // 3, N - 1):
        psi = oracle.init_basis(n, x)
        oracle.apply_gates(psi, gates)
        y = np.arange(N)
        want = np.exp(2j * math.pi * x * y / N) / math.sqrt(N)
        assert np.max(np.abs(psi - want)) < 1e-13


# ------------------------------------------------------------------ QAOA
def _qaoa_brute(n, edges, p, theta):
    C = sum(0.5 * (np.eye(1 << n) - op(n, {int(u): W.PAULI_Z, int(v): W.PAULI_Z})) for u, v in edges)
    B = sum(op(n, {j: W.PAULI_X}) for j in range(n))
    psi = np.ones(1 << n, dtype=np.complex128) / math.sqrt(1 << n)
    for l in range(p):
        psi = scipy.linalg.expm(-1j * theta[l] * C) @ psi
        psi = scipy.linalg.expm(-1j * theta[p + l] * B) @ psi
    return np.vdot(psi, C @ psi).real


@pytest.mark.parametrize("n", [4, 6, 8, 10])
def test_qaoa_p1_ring_closed_form(n):
    """p = 1 on a ring: E = n (1/2 + 1/4 sin(4 beta) sin(2 gamma)) for n >= 4."""
    ring = W.ring_graph(n)
    for gamma, beta in [(0.3, 0.7), (1.1, -0.4), (2.5, 2.9)]:
        th = np.array([gamma, beta])
        e, g = oracle.qaoa_grad(n, ring, 1, th)
        assert abs(e - n * (0.5 + 0.25 * math.sin(4 * beta) * math.sin(2 * gamma))) < 1e-13
        assert abs(g[0] - 0.5 * n * math.sin(4 * beta) * math.cos(2 * gamma)) < 1e-12
        assert abs(g[1] - n * math.cos(4 * beta) * math.sin(2 * gamma)) < 1e-12
        assert abs(oracle.qaoa_energy(n, ring, 1, th) - e) < 1e-14


def test_qaoa_energy_vs_matrix_exponential():
    n, p = 6, 3
    g = W.random_regular_graph(n, 3, seed=7)
    th = W.qaoa_angles(p, seed=8)
    assert abs(oracle.qaoa_energy(n, g, p, th) - _qaoa_brute(n, g, p, th)) < 1e-12
    # Zero angles: the uniform state, <C> = |E|/2.
    assert abs(oracle.qaoa_energy(n, g, p, np.zeros(2 * p)) - len(g) / 2) < 1e-13


def test_qaoa_adjoint_gradient_vs_richardson_fd_of_expm_energy():
    n, p = 6, 2
    g = W.random_regular_graph(n, 3, seed=11)
    th = W.qaoa_angles(p, seed=12)
    _, grad = oracle.qaoa_grad(n, g, p, th)
    h = 1e-2
    fd = np.zeros(2 * p)
    for k in range(2 * p):
        def f(dh):
            t = th.copy()
            t[k] += dh
            return _qaoa_brute(n, g, p, t)
        d1 = (f(h) - f(-h)) / (2 * h)
        d2 = (f(h / 2) - f(-h / 2)) / h
        d3 = (f(h / 4) - f(-h / 4)) / (h / 2)
        r1 = (4 * d2 - d1) / 3
        r2 = (4 * d3 - d2) / 3
        fd[k] = (16 * r2 - r1) / 15
    assert np.max(np.abs(grad - fd)) < 1e-9


def test_qaoa_fd_mode_consistent_with_adjoint():
    n, p = 8, 3
    g = W.random_regular_graph(n, 3, seed=21)
    th = W.qaoa_angles(p, seed=22)
    _, grad = oracle.qaoa_grad(n, g, p, th)
    fd = oracle.qaoa_grad_fd(n, g, p, th, h=1e-5)
    assert np.max(np.abs(grad - fd)) < 1e-8


# ------------------------------------------------------------------ trajectories
def test_depol_threshold():
    assert oracle.depol_threshold(0.0) == 0
    assert oracle.depol_threshold(1e-3) == math.floor(1e-3 * 2 ** 32)
    assert oracle.depol_threshold(1.0) == 2 ** 32 - 1


def test_trajectory_noiseless_equals_ideal_and_invariants():
    n = 6
    gates = W.qft_circuit(n)
    x = 37
    ens = oracle.traj_ensemble(n, gates, x, 4, p=0.0, seed=1)
    assert np.all(ens["counts"] == 0)
    assert np.allclose(ens["fid"], 1.0, atol=1e-13)
    # Heavily noisy QFT on a basis state: still a product of equal-magnitude
    # qubit states, so <Z_i> = 0 and p(k) = 2^-n in every trajectory.
    ens = oracle.traj_ensemble(n, gates, x, 8, p=0.3, seed=2)
    assert ens["counts"].sum() > 0
    assert np.max(np.abs(ens["z"])) < 1e-13
    assert np.max(np.abs(ens["prob_mean"] - 2.0 ** -n)) < 1e-14


def _density_matrix_reference(n, gates, x, p):
    N = 1 << n
    rho = np.zeros((N, N), dtype=np.complex128)
    rho[x, x] = 1
    paulis = [W.PAULI_X, W.PAULI_Y, W.PAULI_Z]
    for gr in gates:
        k, a, b, u = int(gr["kind"]), int(gr["q0"]), int(gr["q1"]), gr["u"]
        if k == W.G_1Q:
            G = op(n, {a: W.u8_to_mat(u)})
        elif k == W.G_DIAG2:
            d = u[0::2] + 1j * u[1::2]
            G = sum(d[2 * b1 + b0] * op(n, {a: [P0, P1][b0], b: [P0, P1][b1]}) for b0 in (0, 1) for b1 in (0, 1))
        elif k == W.G_SWAP:
            G = 0.5 * (np.eye(N) + sum(op(n, {a: s, b: s}) for s in paulis))
        else:
            raise AssertionError
        rho = G @ rho @ G.conj().T
        for q in ([a] if k == W.G_1Q else [a, b]):
            rho = (1 - p) * rho + (p / 3) * sum(op(n, {q: s}) @ rho @ op(n, {q: s}) for s in paulis)
    return rho


def test_trajectory_means_converge_to_density_matrix():
    """Unravelling check: trajectory averages of fidelity and <X_i> agree with the
    depolarizing channel's density matrix within 4 standard errors."""
    n, p, T = 4, 0.05, 3000
    gates = W.qft_circuit(n)
    x = 11
    ideal = oracle.init_basis(n, x)
    oracle.apply_gates(ideal, gates)
    rho = _density_matrix_reference(n, gates, x, p)
    ens = oracle.traj_ensemble(n, gates, x, T, p, seed=5, ideal=ideal)
    f_exact = np.vdot(ideal, rho @ ideal).real
    se = ens["fid"].std() / math.sqrt(T)
    assert abs(ens["fid"].mean() - f_exact) < 4 * se + 1e-12
    for q in range(n):
        xe = np.trace(op(n, {q: W.PAULI_X}) @ rho).real
        se = ens["x"][:, q].std() / math.sqrt(T)
        assert abs(ens["x"][:, q].mean() - xe) < 4 * se + 1e-12
    # Insertion statistics: rate p per slot, Paulis uniform over X, Y, Z.
    slots = T * sum(1 if int(gr["kind"]) == W.G_1Q else 2 for gr in gates)
    rate = ens["counts"].sum() / slots
    assert abs(rate - p) < 4 * math.sqrt(p * (1 - p) / slots)
    kinds = np.concatenate([l & 3 for l in ens["logs"] if len(l)])
    frac = np.bincount(kinds, minlength=4)[1:] / len(kinds)
    assert np.all(np.abs(frac - 1 / 3) < 0.03)


def test_trajectory_draws_only_mode_and_decision_rule():
    """The draws-only mode gives the full run's insertion counts and logs, and
    both follow the decision rule computed here from an independent Philox:
    slot s of trajectory t inserts iff x0 < floor(p 2^32), Pauli 1 + floor(3 x1 / 2^32)."""
    n, p, seed = 5, 0.02, 0xABCDEF0123
    gates = W.qft_circuit(n)
    slots = sum(1 if int(gr["kind"]) == W.G_1Q else 2 for gr in gates)
    thr = np.uint64(math.floor(p * 2 ** 32))
    assert oracle.depol_threshold(p) == int(thr)
    s = np.arange(slots, dtype=np.uint64)
    total = 0
    for t in range(300):
        psi = oracle.init_basis(n, 3)
        full = oracle.traj_run_one(psi, gates, p, seed, t, log_cap=32)
        only = oracle.traj_draws(gates, p, seed, t, log_cap=32)
        assert full[0] == only[0] and np.array_equal(full[1], only[1])
        x = _philox_np(np.full(slots, t), s, np.full(slots, 3), np.zeros(slots), seed & 0xFFFFFFFF, seed >> 32)
        hit = x[0] < thr
        want = (s[hit] << np.uint64(2)) | (np.uint64(1) + ((x[1][hit] * np.uint64(3)) >> np.uint64(32)))
        assert only[0] == int(hit.sum()) and np.array_equal(only[1], want.astype(np.uint32))
        total += only[0]
    assert total > 50
