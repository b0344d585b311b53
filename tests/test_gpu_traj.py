"""GPU parity for noise trajectories (stochastic Pauli insertion).

Insertion counts and logs must be bit-identical to the oracle's (integer
decisions from the same Philox draws).  Per-trajectory <Z_q>, <X_q>, fidelity
and the trajectory-mean probabilities must match the oracle, which applies
every inserted Pauli to the amplitudes, while the GPU tracks them as a Pauli
frame: agreement checks the frame rules for every gate kind.
"""
import numpy as np
import pytest

import oracle
from paper_2001_10554_amd import workloads as W
from gpu_util import TOL, require_gpu, torch_dtype

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _compare(n, gates, x0, T, p, seed, dt, log_cap=32, tol_scale=8):
    from paper_2001_10554_amd.qsim import traj_run
    res = traj_run(n, gates, x0, T, p, seed, dtype=torch_dtype(dt), log_cap=log_cap)
    ens = oracle.traj_ensemble(n, gates, x0, T, p, seed, log_cap=log_cap)
    counts = res["counts"].cpu().numpy()
    assert np.array_equal(counts, ens["counts"])
    logs = res["log"].cpu().numpy().astype(np.uint32)
    for t in range(T):
        k = min(counts[t], log_cap)
        assert np.array_equal(logs[t, :k], ens["logs"][t][:k])
    tol = TOL[dt] * tol_scale
    assert np.max(np.abs(res["z"].cpu().numpy() - ens["z"])) < tol
    assert np.max(np.abs(res["x"].cpu().numpy() - ens["x"])) < tol
    assert np.max(np.abs(res["fid"].cpu().numpy() - ens["fid"])) < tol
    assert np.max(np.abs(res["prob_mean"].cpu().numpy() - ens["prob_mean"])) < tol
    return res, ens


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_qft_trajectories_small(dt):
    n = 8
    res, ens = _compare(n, W.qft_circuit(n), 173, 40, 0.05, seed=11, dt=dt)
    assert ens["counts"].sum() > 20  # the noise actually fired


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_mixed_gate_kinds_frames(dt):
    """Random 1Q / C1Q / DIAG2 / SWAP circuit with heavy noise: exercises every
    frame-conjugation rule (controls flipped by X, diagonals permuted, swaps
    relabelling the frame)."""
    n = 7
    gates = W.random_block(n, 60, seed=3)
    _compare(n, gates, 5, 48, 0.2, seed=4, dt=dt)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_reordered_passes_frames(dt):
    """A circuit whose passes move commuting gates ahead (14 qubits, tiles of
    12: a one-qubit gate after every two-qubit diagonal on both of its
    qubits).  Each gate keeps the frame of its list position, and a
    trajectory leaves the noiseless run at the first executed gate that sees
    a non-identity frame."""
    n = 14
    gates = W.dressed_qaoa_circuit(n, W.random_regular_graph(n, 3, seed=3), 2, seed=5)
    res, ens = _compare(n, gates, 77, 32, 0.01, seed=6, dt=dt)
    assert 0 < ens["counts"].sum() and (ens["counts"] == 0).sum() > 0


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_reordered_passes_all_gate_kinds(dt):
    """14 qubits, random 1Q / C1Q / DIAG2 / SWAP circuit whose plan moves
    commuting gates ahead (5 passes instead of 8): controls flipped by the
    frame, permuted diagonals and frame-relabelling swaps under reordering."""
    n = 14
    _compare(n, W.random_block(n, 120, seed=12), 321, 24, 0.008, seed=7, dt=dt)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_insertions_after_the_last_simulated_gate(dt):
    """Trajectories whose insertions all follow the last simulated gate are not
    simulated: they read the noiseless state through their own Pauli frame.
    One gate (every insertion comes after it), and a circuit ending in SWAPs
    (the trailing SWAPs are folded into the read-outs): fidelity, <Z>, <X>,
    the probability mean and a diagonal observable against the oracle."""
    import torch
    from paper_2001_10554_amd.qsim import traj_run
    g = np.random.default_rng(4)
    n = 4
    one = W.gates_array([W.gate(W.G_1Q, 1, -1, W.haar_2x2(g))])
    tail = np.concatenate([W.random_block(n, 12, seed=9),
                           W.gates_array([W.gate(W.G_SWAP, 0, 3), W.gate(W.G_SWAP, 1, 2), W.gate(W.G_SWAP, 0, 1)])])
    d = g.standard_normal(1 << n)
    tol = TOL[dt] * 8
    for gates, p in ((one, 0.5), (tail, 0.1)):
        res = traj_run(n, gates, 6, 48, p, seed=3, dtype=torch_dtype(dt), log_cap=16,
                       diag=torch.tensor(d, device="cuda"))
        ens = oracle.traj_ensemble(n, gates, 6, 48, p, 3, log_cap=16, diag=d)
        assert np.array_equal(res["counts"].cpu().numpy(), ens["counts"])
        for key in ("z", "x", "fid", "prob_mean", "diag"):
            err = np.max(np.abs(res[key].cpu().numpy() - ens[key]))
            assert err < tol * (4 if key == "diag" else 1), (key, err)
        assert np.min(ens["fid"]) < 0.9  # some frames move the state away from the noiseless one


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_qft20_largest_register(dt):
    """20 qubits, the largest trajectory register: several tile passes, 256
    read-out chunks per state and the QFT's ten final SWAPs folded into the
    read-outs."""
    n = 20
    _compare(n, W.qft_circuit(n), W.random_basis_index(n, 21), 6, 0.004, seed=13, dt=dt, log_cap=16)


def test_noiseless_and_certain_insertion():
    n = 6
    gates = W.random_block(n, 30, seed=8)
    _compare(n, gates, 9, 8, 0.0, seed=1, dt="c128")
    _compare(n, gates, 9, 8, 1.0, seed=2, dt="c128", log_cap=64)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_config5_qft16_1024_trajectories(dt):
    """16-qubit QFT on a seeded basis state, p = 1e-3 per touched qubit, 1024
    trajectories in one call.  Every trajectory's counts/logs are checked
    against the oracle's draws; a sample of trajectories (all noisy ones up to
    16, plus noiseless ones) is re-simulated by the oracle; the structural
    invariants <Z_q> = 0 and p(k) = 2^-16 hold in every trajectory."""
    import torch
    from paper_2001_10554_amd.qsim import traj_run
    n, T, p, seed = 16, 1024, 1e-3, 5
    gates = W.qft_circuit(n)
    x0 = W.random_basis_index(n, 5)
    res = traj_run(n, gates, x0, T, p, seed, dtype=torch_dtype(dt), log_cap=8)
    counts = res["counts"].cpu().numpy()
    noisy = np.nonzero(counts)[0]
    assert 0.1 < len(noisy) / T < 0.45  # E[insertions] = 0.272 per trajectory
    ideal = oracle.init_basis(n, x0)
    oracle.apply_gates(ideal, gates)
    sample = list(noisy[:16]) + list(np.nonzero(counts == 0)[0][:4])
    tol = TOL[dt] * 8
    for t in sample:
        psi = oracle.init_basis(n, x0)
        nins, log = oracle.traj_run_one(psi, gates, p, seed, int(t), log_cap=8)
        assert nins == counts[t]
        assert np.array_equal(res["log"][t, :min(nins, 8)].cpu().numpy().astype(np.uint32), log)
        assert np.max(np.abs(res["x"][t].cpu().numpy() - oracle.expect_x_all(psi))) < tol
        assert abs(res["fid"][t].item() - abs(oracle.inner(ideal, psi)) ** 2) < tol
    assert torch.max(torch.abs(res["z"])).item() < tol
    assert torch.max(torch.abs(res["prob_mean"] - 2.0 ** -n)).item() < TOL[dt] * 1e-4
    # Draw counts of every trajectory against the oracle's decision rule.
    thr = oracle.depol_threshold(p)
    slots = sum(1 if int(g["kind"]) == W.G_1Q else 2 for g in gates)
    for t in range(0, T, 97):
        c = sum(int(oracle.philox4x32_10([t, s, 3, 0], [seed, 0])[0] < thr) for s in range(slots))
        assert c == counts[t]
