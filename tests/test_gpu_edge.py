"""GPU edge cases: a large register checked element by element, argument
validation at the boundary, and degenerate inputs."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2001_10554_amd import workloads as W
from gpu_util import check_amps, check_val, max_err, require_gpu, to_host, torch_dtype

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_sweep_26q_full_state(dt):
    """The bench's sweep (Haar 1q on every qubit, then the CNOT chain) on a
    26-qubit register, compared amplitude by amplitude with the oracle."""
    from paper_2001_10554_amd.qsim import State
    n = 26
    mats, cnots = W.sweep_circuit(n, seed=2)
    s = State(n, torch_dtype(dt)).init_random(2)
    ref = oracle.init_random(n, 2)
    for q in range(n):
        s.apply_1q(q, mats[q])
        oracle.apply_1q(ref, q, mats[q])
    for c, t in cnots:
        s.apply_c1q(c, t, W.PAULI_X)
        oracle.apply_c1q(ref, c, t, W.PAULI_X)
    G = n + len(cnots) + 1
    check_amps(to_host(s), ref, dt, "26q sweep", gates=G)
    check_val(s.expect_z_all().cpu().numpy(), oracle.expect_z_all(ref), dt, "<Z_q> all", gates=G)


def test_state_validation():
    import torch
    from paper_2001_10554_amd.qsim import QS_ERR_ARG, QS_ERR_DTYPE, QS_ERR_SIZE, check, lib
    h = ctypes.c_void_p()
    buf = torch.empty(16, dtype=torch.complex128, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    assert lib().qs_state_create(4, 2, p, 256, None, ctypes.byref(h)) == 0
    assert lib().qs_state_destroy(h) == 0
    assert lib().qs_state_create(5, 2, p, 256, None, ctypes.byref(h)) == QS_ERR_SIZE  # buffer too small
    assert lib().qs_state_create(35, 2, p, 1 << 62, None, ctypes.byref(h)) == QS_ERR_SIZE  # above the c128 limit
    assert lib().qs_state_create(4, 3, p, 256, None, ctypes.byref(h)) == QS_ERR_DTYPE
    assert lib().qs_state_create(0, 2, p, 256, None, ctypes.byref(h)) == QS_ERR_ARG
    assert lib().qs_state_create(4, 2, None, 256, None, ctypes.byref(h)) == QS_ERR_ARG
    assert b"" != lib().qs_last_error()
    assert lib().qs_apply_1q(None, 0, None) == QS_ERR_ARG


def test_misc_validation():
    import torch
    from paper_2001_10554_amd.qsim import QS_ERR_ARG, Qaoa, QsimError, State, traj_run
    s = State(6)
    s.init_basis(3)
    s.apply_block(W.random_block(6, 0, 1))  # empty block: no-op
    assert abs(s.amps[3].item() - 1) == 0
    with pytest.raises(QsimError):
        s.apply_diag2(2, 2, np.ones(4))
    with pytest.raises(QsimError):
        s.apply_swap(0, 6)
    with pytest.raises(QsimError):
        s.apply_cut_phase(np.array([[0, 6]]), 0.1)
    with pytest.raises(QsimError):
        s.sample(1 << 33, 1)
    with pytest.raises(QsimError):
        Qaoa(4, np.array([[0, 0]]), 1).run(torch.zeros(2, dtype=torch.float64, device="cuda"))
    with pytest.raises(QsimError):
        traj_run(4, W.qft_circuit(4), 0, 4, 1.5, 1)
    with pytest.raises(QsimError):
        traj_run(4, W.qft_circuit(4), 16, 4, 0.1, 1)


def test_single_qubit_register():
    from paper_2001_10554_amd.qsim import State
    s = State(1).init_basis(0)
    s.apply_1q(0, W.HADAMARD)
    assert max_err(to_host(s), [2 ** -0.5, 2 ** -0.5]) < 1e-15
    assert abs(s.expect_pauli(1, 0)[0].item() - 1.0) < 1e-15
    assert abs(s.prob_one(0).item() - 0.5) < 1e-15
    sm = s.sample(4000, 3).cpu().numpy()
    assert set(np.unique(sm)) <= {0, 1} and 1700 < sm.sum() < 2300


def test_30q_full_state_selected_targets():
    """A 30-qubit complex128 register (16 GiB) checked amplitude by amplitude
    after one-qubit gates on low, middle and top targets and a CNOT on the top
    qubits."""
    from paper_2001_10554_amd.qsim import State
    n = 30
    mats = W.haar_list(31, 6)
    s = State(n).init_random(30)
    ref = oracle.init_random(n, 30)
    for i, q in enumerate((0, 5, 11, 17, 29)):
        s.apply_1q(q, mats[i])
        oracle.apply_1q(ref, q, mats[i])
    s.apply_c1q(28, 29, W.PAULI_X)
    oracle.apply_c1q(ref, 28, 29, W.PAULI_X)
    check_amps(s.amps.cpu().numpy(), ref, "c128", "30q after 6 gates")


@pytest.mark.parametrize("n", [26, 30])
def test_cut_layer_and_expectation_large(n):
    """The chunked cut kernels (per-thread constants, loop-bit coefficients
    and a per-block table) at sizes where the loop spans 7 and 11 bits: the
    expectation and the phase layer, element by element."""
    import torch
    from paper_2001_10554_amd.qsim import State
    edges = W.random_regular_graph(n, 3, seed=n)
    w = np.random.default_rng(n).uniform(0.2, 1.5, len(edges))
    s = State(n).init_random(n)
    ref = oracle.init_random(n, n)
    check_val(s.expect_cut(edges).item(), oracle.expect_cut(ref, edges), "c128", "<C>")
    check_val(s.expect_cut(edges, w).item(), oracle.expect_cut(ref, edges, w), "c128", "<C_w>")
    s.apply_cut_phase(edges, 0.37)
    oracle.apply_cut_phase(ref, edges, 0.37)
    check_amps(s.amps.cpu().numpy(), ref, "c128", "unit-weight phase layer")
    s.apply_cut_phase(edges, -0.81, w)
    oracle.apply_cut_phase(ref, edges, -0.81, w)
    check_amps(s.amps.cpu().numpy(), ref, "c128", "weighted phase layer")
    check_val(s.expect_cut(edges).item(), oracle.expect_cut(ref, edges), "c128", "<C> after the layers")
    del s, ref
    torch.cuda.empty_cache()
