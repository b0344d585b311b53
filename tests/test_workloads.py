"""Seeded input generators: shapes, determinism and basic validity."""
import numpy as np
import pytest

from paper_2001_10554_amd import workloads as W


def test_haar_unitary_and_seeded():
    a = W.haar_list(1, 50)
    b = W.haar_list(1, 50)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
        assert np.max(np.abs(u.conj().T @ u - np.eye(2))) < 1e-15


def test_u8_roundtrip():
    u = W.haar_list(3, 1)[0]
    assert np.array_equal(W.u8_to_mat(W.mat_to_u8(u)), u)


@pytest.mark.parametrize("n", [4, 8, 14, 16, 18, 20, 22, 24])
def test_random_regular_graph(n):
    e = W.random_regular_graph(n, 3, seed=n)
    assert e.shape == (3 * n // 2, 2)
    assert np.all(e[:, 0] < e[:, 1])
    assert np.all(np.bincount(e.reshape(-1), minlength=n) == 3)
    assert len({(int(u), int(v)) for u, v in e}) == len(e)
    with pytest.raises(ValueError):
        W.random_regular_graph(n + 1, 3, seed=0)


def test_brick_circuit_counts():
    g = W.brick_circuit(12, 20, seed=1)
    assert len(g) == 350
    assert np.sum(g["kind"] == W.G_1Q) == 240 and np.sum(g["kind"] == W.G_DIAG2) == 110


def test_qft_counts():
    g = W.qft_circuit(16)
    assert len(g) == 144
    assert np.sum(g["kind"] == W.G_SWAP) == 8


def test_pool_workload():
    w = W.pool_workload(16, 4, 4, seed=4)
    assert len(w.graphs) == 16
    assert set(w.n_qubits) <= {14, 16, 18, 20, 22}
    for a in w.angles:
        assert a.shape == (4, 8) and np.all((a >= 0) & (a < 2 * np.pi))
