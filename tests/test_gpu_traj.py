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
from gpu_util import TOL, check_val, record, require_gpu, torch_dtype

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _slots(gates):
    return sum(1 if int(g["kind"]) == W.G_1Q else 2 for g in gates)


# Read-outs and their operator norms (the fidelity involves two computed
# states, hence 2); a trajectory applies at most len(gates) + slots float gates.
OPNORM = {"z": 1.0, "x": 1.0, "fid": 2.0, "prob_mean": 1.0}


def _compare(n, gates, x0, T, p, seed, dt, log_cap=32):
    from paper_2001_10554_amd.qsim import traj_run
    res = traj_run(n, gates, x0, T, p, seed, dtype=torch_dtype(dt), log_cap=log_cap)
    ens = oracle.traj_ensemble(n, gates, x0, T, p, seed, log_cap=log_cap)
    counts = res["counts"].cpu().numpy()
    assert np.array_equal(counts, ens["counts"])
    logs = res["log"].cpu().numpy().astype(np.uint32)
    for t in range(T):
        k = min(counts[t], log_cap)
        assert np.array_equal(logs[t, :k], ens["logs"][t][:k])
    G = len(gates) + _slots(gates) + 1
    for key in ("z", "x", "fid", "prob_mean"):
        check_val(res[key].cpu().numpy(), ens[key], dt, key, opnorm=OPNORM[key], gates=G)
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
    opnorm = dict(OPNORM, diag=float(np.max(np.abs(d))))
    for gates, p in ((one, 0.5), (tail, 0.1)):
        res = traj_run(n, gates, 6, 48, p, seed=3, dtype=torch_dtype(dt), log_cap=16,
                       diag=torch.tensor(d, device="cuda"))
        ens = oracle.traj_ensemble(n, gates, 6, 48, p, 3, log_cap=16, diag=d)
        assert np.array_equal(res["counts"].cpu().numpy(), ens["counts"])
        G = len(gates) + _slots(gates) + 1
        for key in ("z", "x", "fid", "prob_mean", "diag"):
            check_val(res[key].cpu().numpy(), ens[key], dt, f"{len(gates)} gates: {key}", opnorm=opnorm[key], gates=G)
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
    trajectories in one call.  Every trajectory's insertion count and log are
    compared bit for bit with the oracle's draws; every noisy trajectory and
    a sample of noiseless ones are re-simulated by the oracle (<X_q> and
    fidelity); the structural invariants <Z_q> = 0 and p(k) = 2^-16 hold in
    every trajectory."""
    import torch
    from paper_2001_10554_amd.qsim import traj_run
    n, T, p, seed, cap = 16, 1024, 1e-3, 5, 8
    gates = W.qft_circuit(n)
    x0 = W.random_basis_index(n, 5)
    res = traj_run(n, gates, x0, T, p, seed, dtype=torch_dtype(dt), log_cap=cap)
    counts = res["counts"].cpu().numpy()
    logs = res["log"].cpu().numpy().astype(np.uint32)
    bad = 0
    for t in range(T):
        nins, log = oracle.traj_draws(gates, p, seed, t, log_cap=cap)
        bad += int(nins != counts[t] or not np.array_equal(logs[t, :min(nins, cap)], log))
    record(f"trajectories (of {T}) whose insertion count or log differs", bad, 0)
    assert counts.max() <= cap  # every log was compared in full
    noisy = np.nonzero(counts)[0]
    assert 0.1 < len(noisy) / T < 0.45  # E[insertions] = 0.272 per trajectory
    ideal = oracle.init_basis(n, x0)
    oracle.apply_gates(ideal, gates)
    sample = list(noisy) + list(np.nonzero(counts == 0)[0][:8])
    G = len(gates) + _slots(gates) + 1
    xs, fs, xw, fw = [], [], [], []
    for t in sample:
        psi = oracle.init_basis(n, x0)
        oracle.traj_run_one(psi, gates, p, seed, int(t), log_cap=cap)
        xs.append(res["x"][t].cpu().numpy())
        xw.append(oracle.expect_x_all(psi))
        fs.append(res["fid"][t].item())
        fw.append(abs(oracle.inner(ideal, psi)) ** 2)
    check_val(np.array(xs), np.array(xw), dt, f"<X_q> of {len(sample)} re-simulated trajectories", gates=G)
    check_val(np.array(fs), np.array(fw), dt, "fidelity of the same", opnorm=2.0, gates=G)
    check_val(res["z"].cpu().numpy(), np.zeros((T, n)), dt, "<Z_q> = 0 in every trajectory", gates=G)
    # |a_k| = 2^-8 in every trajectory, so amplitude errors within TOL move
    # p(k) by at most 2 * 2^-8 * TOL.
    pm_err = float(np.max(np.abs(res["prob_mean"].cpu().numpy() - 2.0 ** -n)))
    record("p(k) = 2^-16", pm_err, 2 * 2.0 ** (-n / 2) * TOL[dt])
