"""Seeded synthetic inputs for the state-vector simulator and its checks.

This module only *draws inputs*: gate matrices, circuits as gate lists, graphs,
angle sets and seeds.  It performs none of the simulation arithmetic, so the
same inputs can be handed unchanged to the HIP path and to the CPU oracle.

Every generator takes an explicit integer seed and uses numpy's PCG64, so the
two sides see bit-identical inputs.

Workload shapes follow the paper:
  * random one-qubit gates applied to every qubit (Scaling Experiments, strong
    scaling: a random 2x2 matrix applied to all qubits of a 32-qubit state);
  * QAOA Max-Cut on random 3-regular graphs (Particle Swarm / QAOA section,
    18-qubit p=4 instances; 16-qubit p=4 for the noise study);
  * a pool of circuits that differ only in their parameters (Software
    description, "Pool of multiple states").
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Gate kinds of a gate record (kind, q0, q1, u[8]).  The numeric values are the
# ones the C-ABI uses; they are part of the interface, not of the arithmetic.
G_1Q = 1      # 2x2 matrix u on qubit q0
G_C1Q = 2     # 2x2 matrix u on target q1 iff control q0 is |1>
G_DIAG2 = 3   # diagonal diag(d00, d01, d10, d11) on (q0, q1); entry index = 2*b(q1) + b(q0)
G_SWAP = 4    # exchange qubits q0 and q1
G_NOISE = 5   # stochastic noise gate on qubit q0 for the duration u[0] (trajectories only)

GATE_DTYPE = np.dtype([("kind", np.int32), ("q0", np.int32), ("q1", np.int32),
                       ("pad", np.int32), ("u", np.float64, (8,))], align=True)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def mat_to_u8(m: np.ndarray) -> np.ndarray:
    """2x2 complex matrix -> row-major interleaved [re00, im00, re01, im01, re10, im10, re11, im11]."""
    m = np.asarray(m, dtype=np.complex128).reshape(2, 2)
    out = np.empty(8, dtype=np.float64)
    out[0::2] = m.reshape(-1).real
    out[1::2] = m.reshape(-1).imag
    return out


def u8_to_mat(u: np.ndarray) -> np.ndarray:
    u = np.asarray(u, dtype=np.float64).reshape(8)
    return (u[0::2] + 1j * u[1::2]).reshape(2, 2)


def haar_2x2(g: np.random.Generator) -> np.ndarray:
    """Haar-random U(2) element: QR of a complex Ginibre matrix with the
    diagonal-phase correction of Mezzadri (2007)."""
    z = (g.standard_normal((2, 2)) + 1j * g.standard_normal((2, 2))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return q * (d / np.abs(d))[np.newaxis, :]


def haar_list(seed: int, count: int) -> list[np.ndarray]:
    g = rng(seed)
    return [haar_2x2(g) for _ in range(count)]


# Named constant gates (matrices only).
PAULI_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PAULI_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PAULI_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
HADAMARD = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)


def rot_x(theta: float) -> np.ndarray:
    """RX(theta) = exp(-i theta X / 2)."""
    c, s = math.cos(theta / 2.0), math.sin(theta / 2.0)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def cphase_diag(phi: float) -> np.ndarray:
    """Controlled phase diag(1, 1, 1, e^{i phi}) as four complex entries."""
    return np.array([1, 1, 1, np.exp(1j * phi)], dtype=np.complex128)


def gate(kind: int, q0: int, q1: int = -1, m=None) -> np.void:
    rec = np.zeros((), dtype=GATE_DTYPE)
    rec["kind"], rec["q0"], rec["q1"] = kind, q0, q1
    if m is not None:
        m = np.asarray(m, dtype=np.complex128).reshape(-1)
        rec["u"][0::2] = m.real
        rec["u"][1::2] = m.imag
    return rec


def gates_array(recs) -> np.ndarray:
    arr = np.zeros(len(recs), dtype=GATE_DTYPE)
    for i, r in enumerate(recs):
        arr[i] = r
    return arr


# ----------------------------------------------------------------------------
# Circuits
# ----------------------------------------------------------------------------

def brick_circuit(n: int, layers: int, seed: int) -> np.ndarray:
    """Layers of a Haar 1q gate on every qubit followed by CZ on brick pairs.

    Even layers pair (0,1),(2,3),...; odd layers (1,2),(3,4),...; no wrap.
    Draw order is layer-major, qubit-minor.  CZ is encoded as DIAG2.
    """
    g = rng(seed)
    recs = []
    cz = np.array([1, 1, 1, -1], dtype=np.complex128)
    for layer in range(layers):
        for q in range(n):
            recs.append(gate(G_1Q, q, -1, haar_2x2(g)))
        start = layer % 2
        for a in range(start, n - 1, 2):
            recs.append(gate(G_DIAG2, a, a + 1, cz))
    return gates_array(recs)


def sweep_circuit(n: int, seed: int) -> tuple[list[np.ndarray], list[tuple[int, int]]]:
    """Haar 1q gates on qubits 0..n-1 in order, then CNOT(q, q+1) for q = 0..n-2."""
    mats = haar_list(seed, n)
    cnots = [(q, q + 1) for q in range(n - 1)]
    return mats, cnots


def qft_circuit(n: int) -> np.ndarray:
    """Textbook QFT as a gate list, most significant qubit first.

    For j = n-1 .. 0: H on j, then controlled phases 2*pi/2^(j-m+1) from each
    lower qubit m = j-1 .. 0; finally floor(n/2) SWAPs reverse the qubit order.
    """
    recs = []
    for j in range(n - 1, -1, -1):
        recs.append(gate(G_1Q, j, -1, HADAMARD))
        for m in range(j - 1, -1, -1):
            recs.append(gate(G_DIAG2, m, j, cphase_diag(2.0 * math.pi / 2 ** (j - m + 1))))
    for q in range(n // 2):
        recs.append(gate(G_SWAP, q, n - 1 - q))
    return gates_array(recs)


def random_block(n: int, count: int, seed: int, kinds=(G_1Q, G_C1Q, G_DIAG2, G_SWAP)) -> np.ndarray:
    """Random mixed gate list for fused-block parity checks."""
    g = rng(seed)
    recs = []
    for _ in range(count):
        kind = int(g.choice(kinds))
        if kind == G_1Q or n < 2:
            recs.append(gate(G_1Q, int(g.integers(n)), -1, haar_2x2(g)))
        else:
            a, b = (int(x) for x in g.choice(n, size=2, replace=False))
            if kind == G_C1Q:
                recs.append(gate(G_C1Q, a, b, haar_2x2(g)))
            elif kind == G_DIAG2:
                ph = g.uniform(0, 2 * math.pi, size=4)
                recs.append(gate(G_DIAG2, a, b, np.exp(1j * ph)))
            else:
                recs.append(gate(G_SWAP, a, b))
    return gates_array(recs)


# ----------------------------------------------------------------------------
# Graphs and QAOA parameters
# ----------------------------------------------------------------------------

def random_regular_graph(n: int, d: int, seed: int) -> np.ndarray:
    """Uniform random d-regular simple graph by the pairing (configuration)
    model with rejection of self-loops and multi-edges.  Returns int32 [E, 2]
    with u < v, edges sorted."""
    if (n * d) % 2 or d >= n:
        raise ValueError(f"no {d}-regular graph on {n} vertices")
    g = rng(seed)
    stubs = np.repeat(np.arange(n), d)
    for _ in range(100000):
        perm = g.permutation(stubs)
        pairs = perm.reshape(-1, 2)
        if np.any(pairs[:, 0] == pairs[:, 1]):
            continue
        e = np.sort(pairs, axis=1)
        keys = e[:, 0] * n + e[:, 1]
        if len(np.unique(keys)) != len(keys):
            continue
        order = np.argsort(keys)
        return e[order].astype(np.int32)
    raise RuntimeError("pairing model did not produce a simple graph")


def ring_graph(n: int) -> np.ndarray:
    return np.array([(min(i, (i + 1) % n), max(i, (i + 1) % n)) for i in range(n)], dtype=np.int32)


def qaoa_angles(p: int, seed: int, lo: float = 0.0, hi: float = math.pi, count: int | None = None) -> np.ndarray:
    """Angle vectors [gamma_1..gamma_p, beta_1..beta_p], uniform in [lo, hi)."""
    g = rng(seed)
    shape = (2 * p,) if count is None else (count, 2 * p)
    return g.uniform(lo, hi, size=shape)


@dataclass
class PoolWorkload:
    """Many QAOA Max-Cut instances, each with several angle sets."""
    graphs: list = field(default_factory=list)      # int32 [E, 2] per graph
    n_qubits: list = field(default_factory=list)    # qubit count per graph
    angles: list = field(default_factory=list)      # float64 [sets, 2p] per graph
    p: int = 4


def pool_workload(num_graphs: int, sets_per_graph: int, p: int, seed: int,
                  n_choices=(14, 16, 18, 20, 22)) -> PoolWorkload:
    """Qubit counts uniform over n_choices (even, so a 3-regular graph exists);
    angles uniform in [0, 2*pi) as in a particle swarm's initial positions."""
    g = rng(seed)
    w = PoolWorkload(p=p)
    for i in range(num_graphs):
        n = int(g.choice(n_choices))
        gseed = int(g.integers(2 ** 62))
        w.n_qubits.append(n)
        w.graphs.append(random_regular_graph(n, 3, gseed))
        w.angles.append(g.uniform(0.0, 2 * math.pi, size=(sets_per_graph, 2 * p)))
    return w


def random_basis_index(n: int, seed: int) -> int:
    return int(rng(seed).integers(2 ** n))


def with_noise_gates(gates: np.ndarray, duration: float = 1.0) -> np.ndarray:
    """Schedule for stochastic noise gates: after every gate, one noise gate of
    `duration` on each qubit the gate touches (q0, then q1)."""
    recs = []
    for g in np.asarray(gates, dtype=GATE_DTYPE):
        recs.append(g)
        touched = [int(g["q0"])] if g["kind"] == G_1Q else [int(g["q0"]), int(g["q1"])]
        for q in touched:
            r = np.zeros((), dtype=GATE_DTYPE)
            r["kind"], r["q0"], r["q1"] = G_NOISE, q, -1
            r["u"][0] = duration
            recs.append(r)
    return gates_array(recs)


def dressed_qaoa_circuit(n: int, edges, p: int, seed: int) -> np.ndarray:
    """The QAOA circuit (seeded angles) with a seeded Haar one-qubit gate on
    both qubits after every two-qubit diagonal: the shape of a noisy QAOA
    schedule with fixed gates in place of the noise, whose passes shrink
    when gates that commute are moved ahead of those that do not fit."""
    g = rng(seed)
    recs = []
    for x in qaoa_circuit(n, edges, p, qaoa_angles(p, seed=seed)):
        recs.append(x)
        if int(x["kind"]) == G_DIAG2:
            for q in (int(x["q0"]), int(x["q1"])):
                recs.append(gate(G_1Q, q, -1, haar_2x2(g)))
    return gates_array(recs)


def qaoa_circuit(n: int, edges, p: int, theta) -> np.ndarray:
    """QAOA Max-Cut circuit as a gate list: H on every qubit, then per layer l
    a two-qubit diagonal diag(1, e^{-i g}, e^{-i g}, 1) per edge (g = gamma_l)
    and RX(2 beta_l) = exp(-i beta_l X) on every qubit."""
    theta = np.asarray(theta, dtype=np.float64)
    recs = [gate(G_1Q, q, -1, HADAMARD) for q in range(n)]
    for l in range(p):
        g, b = theta[l], theta[p + l]
        d = np.array([1.0, np.exp(-1j * g), np.exp(-1j * g), 1.0])
        for u, v in np.asarray(edges).reshape(-1, 2):
            recs.append(gate(G_DIAG2, int(u), int(v), d))
        rx = np.array([[math.cos(b), -1j * math.sin(b)], [-1j * math.sin(b), math.cos(b)]])
        for q in range(n):
            recs.append(gate(G_1Q, q, -1, rx))
    return gates_array(recs)
