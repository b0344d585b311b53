"""GPU parity for trajectories with stochastic noise gates (T1/T2 rotations
with Box-Muller angles) on top of Pauli insertion, per trajectory against the
oracle, which draws the same angles from its own Philox and applies the
three rotations one after the other."""
import math

import numpy as np
import pytest

import oracle
from paper_2001_10554_amd import workloads as W
from gpu_util import check_val, require_gpu, torch_dtype

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _cut_diag(n, edges):
    k = np.arange(1 << n)
    return sum(((k >> u) ^ (k >> v)) & 1 for u, v in edges).astype(np.float64)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_noise_gates_per_trajectory(dt):
    import torch
    from paper_2001_10554_amd.qsim import traj_run
    n, T, p, seed, T1, T2 = 7, 40, 0.03, 17, 6.0, 5.0
    gates = W.with_noise_gates(W.random_block(n, 24, seed=4), 0.8)
    x0 = 77
    edges = W.random_regular_graph(6, 3, seed=1)
    d = _cut_diag(n, edges)
    r = traj_run(n, gates, x0, T, p, seed, dtype=torch_dtype(dt), log_cap=16, T1=T1, T2=T2,
                 diag=torch.tensor(d, device="cuda"))
    ref = oracle.traj_ensemble(n, gates, x0, T, p, seed, log_cap=16, T1=T1, T2=T2, diag=d)
    assert np.array_equal(r["counts"].cpu().numpy(), ref["counts"])
    log = r["log"].cpu().numpy().astype(np.uint32)
    for t in range(T):
        assert np.array_equal(log[t, :len(ref["logs"][t])], ref["logs"][t])
    # A noise gate is three rotations and an insertion one more gate: at most
    # 3 * len(gates) + slots float gate applications per trajectory.
    G = 3 * len(gates) + 2 * len(gates) + 1
    opnorm = {"z": 1.0, "x": 1.0, "fid": 2.0, "prob_mean": 1.0, "diag": float(np.max(np.abs(d)))}
    for key in ("z", "x", "fid", "prob_mean", "diag"):
        check_val(r[key].cpu().numpy(), ref[key], dt, key, opnorm=opnorm[key], gates=G)
    # noise gates act on every trajectory: none equals the noiseless state
    assert np.all(r["fid"].cpu().numpy() < 1 - 1e-6)


def test_noise_qaoa16_p4_against_oracle():
    """The paper's noisy-QAOA shape: 16 qubits, 3-regular graph, p = 4, a noise
    gate of one gate time on every touched qubit after every gate,
    T1 = 500, T2 = 250 gate times."""
    import torch
    from paper_2001_10554_amd.qsim import traj_run
    n, p, T = 16, 4, 12
    edges = W.random_regular_graph(n, 3, seed=8)
    theta = W.qaoa_angles(p, seed=8)
    gates = W.with_noise_gates(W.qaoa_circuit(n, edges, p, theta), 1.0)
    d = _cut_diag(n, edges)
    r = traj_run(n, gates, 0, T, 0.0, 31, T1=500.0, T2=250.0, diag=torch.tensor(d, device="cuda"), prob_mean=False)
    ref = oracle.traj_ensemble(n, gates, 0, T, 0.0, 31, T1=500.0, T2=250.0, diag=d)
    check_val(r["diag"].cpu().numpy(), ref["diag"], "c128", "per-trajectory <C>")
    check_val(r["fid"].cpu().numpy(), ref["fid"], "c128", "fidelity")
    check_val(r["x"].cpu().numpy(), ref["x"], "c128", "<X_q>")
    # Only the diagonal read-out asked for: the same per-trajectory values,
    # bit for bit, and no <X_q> / <Z_q> / fidelity outputs.
    r2 = traj_run(n, gates, 0, T, 0.0, 31, T1=500.0, T2=250.0, diag=torch.tensor(d, device="cuda"), prob_mean=False, readouts=())
    assert not {"x", "z", "fid"} & set(r2)
    assert np.array_equal(r2["diag"].cpu().numpy(), r["diag"].cpu().numpy())
    assert np.array_equal(r2["counts"].cpu().numpy(), r["counts"].cpu().numpy())
    # the noiseless energy of the same circuit
    e0 = oracle.qaoa_energy(n, edges, p, theta)
    ideal = oracle.init_basis(n, 0)
    oracle.apply_gates(ideal, gates)
    check_val(oracle.expect_diag(ideal, d), e0, "c128", "oracle: noiseless <C> of the gate list vs the QAOA energy")


def test_noise_without_decay_and_validation():
    import torch
    from paper_2001_10554_amd.qsim import QsimError, State, traj_run
    n = 5
    gates = W.with_noise_gates(W.qft_circuit(n), 1.0)
    r = traj_run(n, gates, 3, 8, 0.0, 2, T1=math.inf, T2=math.inf)
    check_val(r["fid"].cpu().numpy(), np.ones(8), "c128", "fidelity without decay")
    with pytest.raises(QsimError):
        traj_run(n, gates, 3, 8, 0.0, 2, T1=1.0, T2=2.5)  # T2 > 2 T1
    with pytest.raises(QsimError):
        State(n).apply_block(gates)  # noise gates belong to trajectories only
    bad = gates.copy()
    bad[1]["u"][0] = -1.0
    with pytest.raises(QsimError):
        traj_run(n, bad, 3, 8, 0.0, 2, T1=1.0, T2=1.0)
