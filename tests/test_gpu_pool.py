"""GPU parity for the pool of uneven QAOA circuits (one captured graph per pool).

Every checked circuit is compared with the oracle's energy (<= 1e-10) and
adjoint gradient (<= 1e-9).  The second run of a pool replays the captured
hipGraph with new angles written in place, so it checks that the replay reads
them.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2001_10554_amd import workloads as W
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _check(pool, graphs, ns, angles, circuits, check_grad=True):
    E = pool.E.cpu().numpy()
    G = pool.G.cpu().numpy() if pool.G is not None else None
    for c in circuits:
        g = c // pool.sets
        e_ref, g_ref = oracle.qaoa_grad(ns[g], graphs[g], pool.p, angles[c])
        assert abs(E[c] - e_ref) < 1e-10, (c, ns[g])
        if check_grad:
            assert np.max(np.abs(G[c] - g_ref)) < 1e-9, (c, ns[g])


def _mixed(seed, sizes):
    graphs = [W.random_regular_graph(n, 3, seed=seed + i) for i, n in enumerate(sizes)]
    return graphs, list(sizes)


def test_pool_mixed_sizes_and_replay():
    import torch
    from paper_2001_10554_amd.qsim import Pool
    graphs, ns = _mixed(40, [4, 6, 8, 10, 12, 14, 6, 12, 16])
    sets, p = 3, 2
    pool = Pool(graphs, ns, sets, p)
    a1 = W.qaoa_angles(p, seed=41, hi=2 * math.pi, count=pool.count)
    pool.run(torch.tensor(a1, device="cuda"))
    _check(pool, graphs, ns, a1, range(pool.count))
    a2 = W.qaoa_angles(p, seed=42, hi=2 * math.pi, count=pool.count)
    pool.run(torch.tensor(a2, device="cuda"))  # graph replay
    _check(pool, graphs, ns, a2, range(pool.count))


def test_pool_small_workspace_forces_batches():
    import torch
    from paper_2001_10554_amd.qsim import Pool
    graphs, ns = _mixed(50, [12, 14, 12, 14])
    sets, p = 5, 2
    full = Pool(graphs, ns, sets, p)
    per_circuit = full.ws.numel() // sets
    pool = Pool(graphs, ns, sets, p, ws_bytes=2 * per_circuit)
    a = W.qaoa_angles(p, seed=51, hi=2 * math.pi, count=pool.count)
    pool.run(torch.tensor(a, device="cuda"))
    _check(pool, graphs, ns, a, range(pool.count))


def test_pool_energy_only():
    import torch
    from paper_2001_10554_amd.qsim import Pool
    graphs, ns = _mixed(60, [8, 10, 12])
    pool = Pool(graphs, ns, 4, 3, grad=False)
    a = W.qaoa_angles(3, seed=61, hi=2 * math.pi, count=pool.count)
    pool.run(torch.tensor(a, device="cuda"))
    _check(pool, graphs, ns, a, range(pool.count), check_grad=False)


def test_pool_config4_subset():
    """Pool in the shape of the 256-graph workload (qubit counts uniform over
    {14, ..., 22}, p = 4, swarm-style angles in [0, 2 pi)), 32 graphs x 64 angle
    sets; a seeded sample of circuits from every size is checked against the
    oracle."""
    import torch
    from paper_2001_10554_amd.qsim import Pool
    w = W.pool_workload(32, 64, 4, seed=4)
    pool = Pool(w.graphs, w.n_qubits, 64, 4)
    a = np.concatenate(w.angles)
    pool.run(torch.tensor(a, device="cuda"))
    rng = np.random.default_rng(4)
    sample = []
    for n in sorted(set(w.n_qubits)):
        gs = [g for g in range(32) if w.n_qubits[g] == n]
        g = gs[int(rng.integers(len(gs)))]
        sample += [g * 64 + int(rng.integers(64)) for _ in range(2 if n < 22 else 1)]
    _check(pool, w.graphs, w.n_qubits, a, sample)
    assert np.all(np.isfinite(pool.E.cpu().numpy()))
