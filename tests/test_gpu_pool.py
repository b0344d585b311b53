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
from gpu_util import record, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _check(pool, graphs, ns, angles, circuits, check_grad=True, workers=1):
    """Energies within 1e-10 and adjoint gradients within 1e-9 of the oracle's
    (the oracle runs `workers` circuits at a time; it is ctypes code that
    releases the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    E = pool.E.cpu().numpy()
    G = pool.G.cpu().numpy() if pool.G is not None else None

    def ref(c):
        g = c // pool.sets
        return oracle.qaoa_grad(ns[g], graphs[g], pool.p, angles[c])

    circuits = list(circuits)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        refs = list(ex.map(ref, circuits))
    e_err = max(abs(E[c] - r[0]) for c, r in zip(circuits, refs))
    record(f"pool energies ({len(circuits)} circuits)", e_err, 1e-10)
    if check_grad:
        g_err = max(float(np.max(np.abs(G[c] - r[1]))) for c, r in zip(circuits, refs))
        record(f"pool adjoint gradients ({len(circuits)} circuits)", g_err, 1e-9)


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


def test_pool_config4_seeded_64_circuits():
    """The whole 256-graph pool workload (qubit counts uniform over
    {14, ..., 22}, random 3-regular graphs, p = 4, 64 swarm-style angle sets
    per graph in [0, 2 pi): 16384 circuits, energies and adjoint gradients in
    one replayed graph); a seeded subset of 64 circuits is checked against
    the oracle, and every energy lies in [0, |E|]."""
    import torch
    from paper_2001_10554_amd.qsim import Pool
    w = W.pool_workload(256, 64, 4, seed=4)
    pool = Pool(w.graphs, w.n_qubits, 64, 4)
    a = np.concatenate(w.angles)
    pool.run(torch.tensor(a, device="cuda"))
    torch.cuda.synchronize()
    sample = np.sort(np.random.default_rng(4).choice(pool.count, 64, replace=False))
    sizes = np.bincount([w.n_qubits[c // 64] for c in sample])
    print("subset sizes:", {n: int(k) for n, k in enumerate(sizes) if k})
    _check(pool, w.graphs, w.n_qubits, a, sample, workers=4)
    E = pool.E.cpu().numpy().reshape(256, 64)
    num_edges = np.array([len(g) for g in w.graphs], dtype=np.float64)
    assert np.all(np.isfinite(E)) and np.all(E >= -1e-12) and np.all(E <= num_edges[:, None] + 1e-12)
    del pool
    torch.cuda.empty_cache()
