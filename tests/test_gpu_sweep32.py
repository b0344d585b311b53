"""Full-size parity for the 32-qubit complex128 sweep (64 GiB register), in
the launch configuration bench.py times.

The oracle cannot hold a 64 GiB state in a test, but a one-qubit gate only
couples the two amplitudes of each pair (eq. 3).  So for every gate of the
sweep, 2^16 random pairs are read back before and after the kernel, packed
into a 17-qubit register (pair partner on qubit 16) and pushed through the
oracle's gate; the GPU result must match to 1e-12.  The initial random state
is checked through its definition (a common positive scale times the raw
Philox draws) and its norm.
"""
import numpy as np
import pytest

import oracle
from paper_2001_10554_amd import workloads as W
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu

N = 32
K = 1 << 16


def _pairs(rng, q, n, ctrl=None):
    k = rng.integers(0, 1 << (n - 1), size=K, dtype=np.int64)
    i0 = ((k >> q) << (q + 1)) | (k & ((1 << q) - 1))
    if ctrl is not None:
        i0 |= 1 << ctrl
    return i0, i0 | (1 << q)


def _oracle_pairs(a, b, m):
    buf = np.concatenate([a, b]).astype(np.complex128)  # qubit 16 selects the partner
    oracle.apply_1q(buf, 16, m)
    return buf[:K], buf[K:]


def test_sweep_32q_pair_spot_checks():
    require_gpu()
    import torch

    from paper_2001_10554_amd.qsim import State

    free, total = torch.cuda.mem_get_info()
    if free < (16 << N) + (4 << 30):
        pytest.skip("needs > 68 GiB of free device memory")
    rng = np.random.default_rng(32)
    mats, cnots = W.sweep_circuit(N, seed=2)
    s = State(N, torch.complex128).init_random(2)
    amps = s.amps

    # Initial state: a_i = scale * raw_i with one positive scale, norm 1.
    idx = np.sort(rng.integers(0, 1 << N, size=4096))
    got = amps[torch.from_numpy(idx).cuda()].cpu().numpy()
    raw = np.array([oracle.philox4x32_10([int(i) & 0xFFFFFFFF, int(i) >> 32, 1, 0], [2, 0]) for i in idx[:256]], dtype=np.uint64)
    u = ((raw[:, 1] << np.uint64(32)) | raw[:, 0]) >> np.uint64(11)
    v = ((raw[:, 3] << np.uint64(32)) | raw[:, 2]) >> np.uint64(11)
    rawc = (2 * u.astype(np.float64) / 2 ** 53 - 1) + 1j * (2 * v.astype(np.float64) / 2 ** 53 - 1)
    scale = got[:256] / rawc
    assert np.max(np.abs(scale.imag)) < 1e-15 and np.ptp(scale.real) < 1e-12 * scale.real.mean()
    assert abs(s.norm2().item() - 1.0) < 1e-12

    for q in range(N):
        i0, i1 = _pairs(rng, q, N)
        ti0, ti1 = torch.from_numpy(i0).cuda(), torch.from_numpy(i1).cuda()
        a, b = amps[ti0].cpu().numpy(), amps[ti1].cpu().numpy()
        s.apply_1q(q, mats[q])
        ga, gb = amps[ti0].cpu().numpy(), amps[ti1].cpu().numpy()
        wa, wb = _oracle_pairs(a, b, mats[q])
        err = max(np.max(np.abs(ga - wa)), np.max(np.abs(gb - wb)))
        assert err < 1e-12, f"1q q={q} err={err}"
    for c, t in cnots:
        i0, i1 = _pairs(rng, t, N)
        on = (i0 >> c) & 1 == 1
        ti0, ti1 = torch.from_numpy(i0).cuda(), torch.from_numpy(i1).cuda()
        a, b = amps[ti0].cpu().numpy(), amps[ti1].cpu().numpy()
        s.apply_c1q(c, t, W.PAULI_X)
        ga, gb = amps[ti0].cpu().numpy(), amps[ti1].cpu().numpy()
        wa, wb = _oracle_pairs(a, b, W.PAULI_X)
        wa = np.where(on, wa, a)
        wb = np.where(on, wb, b)
        err = max(np.max(np.abs(ga - wa)), np.max(np.abs(gb - wb)))
        assert err < 1e-12, f"cnot ({c},{t}) err={err}"
    assert abs(s.norm2().item() - 1.0) < 1e-11
    del s, amps
    torch.cuda.empty_cache()


def test_sweep_32q_fused_block_matches_gate_by_gate():
    """The sweep as one fused block (the passes the bench times at 32 qubits)
    against the same gates applied one by one, whose kernels the pair spot
    checks above tie to the oracle: 2^16 sampled amplitudes agree to 1e-12,
    and the norm stays 1."""
    require_gpu()
    import torch

    from paper_2001_10554_amd.qsim import State, block_passes
    from gpu_util import record

    free, total = torch.cuda.mem_get_info()
    if free < (16 << N) + (4 << 30):
        pytest.skip("needs > 68 GiB of free device memory")
    mats, cnots = W.sweep_circuit(N, seed=2)
    gates = W.gates_array([W.gate(W.G_1Q, q, -1, m) for q, m in enumerate(mats)]
                          + [W.gate(W.G_C1Q, c, t, W.PAULI_X) for c, t in cnots])
    assert block_passes(N, gates) >= 3
    idx = torch.from_numpy(np.sort(np.random.default_rng(33).integers(0, 1 << N, size=K))).cuda()
    s = State(N, torch.complex128).init_random(2)
    for q in range(N):
        s.apply_1q(q, mats[q])
    for c, t in cnots:
        s.apply_c1q(c, t, W.PAULI_X)
    want = s.amps[idx].cpu().numpy()
    s.init_random(2)
    s.apply_block(gates)
    got = s.amps[idx].cpu().numpy()
    record("fused 32q sweep vs gate by gate: max |amplitude error|", float(np.max(np.abs(got - want))), 1e-12)
    record("fused 32q sweep: |norm^2 - 1|", abs(s.norm2().item() - 1.0), 1e-11)
    del s
    torch.cuda.empty_cache()
