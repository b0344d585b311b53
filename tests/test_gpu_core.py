"""GPU parity: state initialisation, single gates, fused blocks, read-outs and
sampling through the C-ABI, element by element against the CPU oracle.

Sizes span one tile (n <= 12), several tiles with a ragged structure (odd n,
n = 13..20) and the small degenerate registers (n = 1, 2).  Tolerances:
complex128 amplitudes 1e-12 abs, complex64 2e-5 abs (against the complex128
oracle), FP64 read-outs 1e-12 * max(1, |value|); complex64 states also meet
the normwise rounding bound of their gate count (the helpers in gpu_util state
and print every bound).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2001_10554_amd import workloads as W
from gpu_util import check_amps, check_val, max_err, record, require_gpu, to_host, torch_dtype

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _state(n, dt="c128"):
    from paper_2001_10554_amd.qsim import State
    return State(n, torch_dtype(dt))


DTS = ["c128", "c64"]


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("n", [1, 2, 5, 12, 13, 17])
def test_init_parity(n, dt):
    s = _state(n, dt)
    s.init_basis((1 << n) - 1)
    assert max_err(to_host(s), oracle.init_basis(n, (1 << n) - 1)) == 0
    s.init_uniform()
    check_amps(to_host(s), oracle.init_uniform(n), dt, "uniform", gates=1)
    s.init_random(1234)
    check_amps(to_host(s), oracle.init_random(n, 1234), dt, "random", gates=1)


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 16, 19, 20])
def test_1q_every_target(n, dt):
    mats = W.haar_list(n, n)
    s = _state(n, dt).init_random(7)
    ref = oracle.init_random(n, 7)
    for q in range(n):
        s.apply_1q(q, mats[q])
        oracle.apply_1q(ref, q, mats[q])
        check_amps(to_host(s), ref, dt, f"after q={q}", gates=q + 2)


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("n", [2, 5, 14])
def test_c1q_pairs(n, dt):
    g = np.random.default_rng(n)
    s = _state(n, dt).init_random(3)
    ref = oracle.init_random(n, 3)
    pairs = [(c, t) for c in range(n) for t in range(n) if c != t]
    if len(pairs) > 40:
        pairs = [pairs[i] for i in g.choice(len(pairs), 40, replace=False)]
    for c, t in pairs:
        U = W.haar_2x2(g)
        s.apply_c1q(c, t, U)
        oracle.apply_c1q(ref, c, t, U)
    check_amps(to_host(s), ref, dt, f"{len(pairs)} controlled gates", gates=len(pairs) + 1)


@pytest.mark.parametrize("dt", DTS)
def test_diag2_swap(dt):
    n = 11
    g = np.random.default_rng(5)
    s = _state(n, dt).init_random(4)
    ref = oracle.init_random(n, 4)
    for _ in range(20):
        a, b = (int(x) for x in g.choice(n, 2, replace=False))
        d = np.exp(1j * g.uniform(0, 6.3, 4))
        d[0] = 1.0  # exercise the touch mask
        s.apply_diag2(a, b, d)
        oracle.apply_diag2(ref, a, b, d)
        s.apply_swap(a, b)
        oracle.apply_swap(ref, a, b)
    check_amps(to_host(s), ref, dt, "20 diagonal + 20 swap gates", gates=41)


@pytest.mark.parametrize("dt", DTS)
# n = 22: complex128 plans mix 12- and 13-bit compiled passes from 22 qubits on.
@pytest.mark.parametrize("n,count,seed", [(1, 10, 1), (3, 30, 2), (9, 80, 3), (12, 120, 4), (14, 150, 5), (17, 200, 6), (22, 200, 7)])
def test_block_matches_sequential(n, count, seed, dt):
    gates = W.random_block(n, count, seed) if n > 1 else W.random_block(n, count, seed, kinds=(W.G_1Q,))
    s = _state(n, dt).init_random(seed)
    ref = oracle.init_random(n, seed)
    s.apply_block(gates)
    oracle.apply_gates(ref, gates)
    check_amps(to_host(s), ref, dt, "first call", gates=count + 1)
    # Second call hits the cached plan.
    s.apply_block(gates)
    oracle.apply_gates(ref, gates)
    check_amps(to_host(s), ref, dt, "cached plan", gates=2 * count + 1)


@pytest.mark.parametrize("dt", DTS)
def test_block_reordered_passes(dt):
    """16 qubits, a circuit whose passes move commuting gates ahead of those
    that do not fit the tile (diagonals past one-qubit gates on other qubits)."""
    n = 16
    gates = W.dressed_qaoa_circuit(n, W.random_regular_graph(n, 3, seed=3), 2, seed=5)
    s = _state(n, dt).init_random(9)
    ref = oracle.init_random(n, 9)
    s.apply_block(gates)
    oracle.apply_gates(ref, gates)
    check_amps(to_host(s), ref, dt, "reordered block", gates=len(gates) + 1)


@pytest.mark.parametrize("dt", DTS)
def test_fused_sweep_26q(dt):
    """The sweep's gate list (Haar 1q on every qubit, then the CNOT chain) as
    one fused block on 26 qubits: 3 passes whose tiles cover different qubit
    sets, full-state parity with the gates applied one by one by the oracle."""
    from paper_2001_10554_amd.qsim import block_passes
    n = 26
    mats, cnots = W.sweep_circuit(n, seed=2)
    gates = W.gates_array([W.gate(W.G_1Q, q, -1, m) for q, m in enumerate(mats)]
                          + [W.gate(W.G_C1Q, c, t, W.PAULI_X) for c, t in cnots])
    assert block_passes(n, gates, torch_dtype(dt)) == 3
    s = _state(n, dt).init_random(4)
    ref = oracle.init_random(n, 4)
    s.apply_block(gates)
    oracle.apply_gates(ref, gates)
    check_amps(to_host(s), ref, dt, "fused 26q sweep", gates=len(gates) + 1)


def test_brick_circuit_12q():
    """12-qubit complex128 brick circuit from |0>: 20 layers of Haar 1q gates and
    CZ bricks; all amplitudes and <Z_i>."""
    n = 12
    gates = W.brick_circuit(n, 20, seed=1)
    s = _state(n).init_basis(0)
    s.apply_block(gates)
    ref = oracle.init_basis(n, 0)
    oracle.apply_gates(ref, gates)
    check_amps(to_host(s), ref, "c128", "brick amplitudes")
    check_val(s.expect_z_all().cpu().numpy(), oracle.expect_z_all(ref), "c128", "<Z_i>")


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("n", [3, 11, 12, 15, 20])
def test_readouts(n, dt):
    import torch
    U = W.haar_list(1, 1)[0]
    s = _state(n, dt).init_random(11)
    s.apply_1q(0, U)
    ref = oracle.init_random(n, 11)
    oracle.apply_1q(ref, 0, U)
    z = s.expect_z_all().cpu().numpy()
    check_val(z, oracle.expect_z_all(ref), dt, "<Z_q> all", gates=2)
    check_val(s.norm2().item(), oracle.norm2(ref), dt, "norm2", gates=2)
    for q in {0, n // 2, n - 1}:
        check_val(s.prob_one(q).item(), oracle.prob_one(ref, q), dt, f"P(q{q}=1)", gates=2)
    g = np.random.default_rng(n)
    for _ in range(4):
        x, z_ = int(g.integers(1 << n)), int(g.integers(1 << n))
        got = s.expect_pauli(x, z_).cpu().numpy()
        want = oracle.expect_pauli(ref, x, z_)
        check_val(got, [want.real, want.imag], dt, f"Pauli x={x:#x} z={z_:#x}", gates=2)
    d = torch.tensor(g.standard_normal(1 << n), device="cuda")
    dh = d.cpu().numpy()
    check_val(s.expect_diag(d).item(), oracle.expect_diag(ref, dh), dt, "sum d|a|^2", opnorm=float(np.max(np.abs(dh))), gates=2)
    if n >= 4:
        e = W.random_regular_graph(n if n % 2 == 0 else n - 1, 3, seed=n)
        check_val(s.expect_cut(e).item(), oracle.expect_cut(ref, e), dt, "<C>", opnorm=len(e), gates=2)
        w = g.uniform(0.5, 2, len(e))
        check_val(s.expect_cut(e, w).item(), oracle.expect_cut(ref, e, w), dt, "<C_w>", opnorm=float(w.sum()), gates=2)
    t = _state(n, dt).init_random(12)
    got = s.inner(t).cpu().numpy()
    want = oracle.inner(ref, oracle.init_random(n, 12))
    check_val(got, [want.real, want.imag], dt, "<a|b>", gates=2)


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("n", [4, 12, 16])
def test_cut_phase(n, dt):
    e = W.random_regular_graph(n, 3, seed=n + 1)
    s = _state(n, dt).init_random(2)
    ref = oracle.init_random(n, 2)
    s.apply_cut_phase(e, 0.731)
    oracle.apply_cut_phase(ref, e, 0.731)
    check_amps(to_host(s), ref, dt, "unit weights", gates=2)
    w = np.linspace(0.3, 1.7, len(e))
    s.apply_cut_phase(e, -1.2, w)
    oracle.apply_cut_phase(ref, e, -1.2, w)
    check_amps(to_host(s), ref, dt, "weighted", gates=3)


def _sample_check(s, psi_host, shots, seed):
    """Draws of qs_sample against the oracle's sampling of the same amplitudes.
    The oracle's CDF is the exact prefix sum rounded to FP64 (long-double
    accumulation); the kernel's FP64 CDF (chunk sums, a two-level prefix over
    at most 2^18 chunks, a wavefront scan inside the chunk) carries at most
    about 1.5e3 roundings of 2^-53 on the way to any index, i.e. < 2e-13.  So
    draws must agree exactly, except that one within 1e-12 of an exact bin edge
    may land on the neighbouring index; their number is reported."""
    got = s.sample(shots, seed=seed).cpu().numpy().astype(np.uint64)
    want, margin = oracle.sample(psi_host, shots, seed=seed)
    close = margin < 1e-12
    far_mismatch = int(np.count_nonzero(got[~close] != want[~close]))
    record(f"sample n={s.n} shots={shots}: mismatches away from bin edges ({int(close.sum())} draws near an edge)", far_mismatch, 0)
    step = np.abs(got[close].astype(np.int64) - want[close].astype(np.int64))
    record("sample: index distance of near-edge draws", int(step.max()) if step.size else 0, 1)


@pytest.mark.parametrize("n", [1, 6, 12, 14, 19])
def test_sample_parity(n):
    U = W.haar_list(9, 1)[0]
    s = _state(n).init_random(5)
    s.apply_1q(n - 1, U)
    ref = oracle.init_random(n, 5)
    oracle.apply_1q(ref, n - 1, U)
    _sample_check(s, ref, 5000, 77)


@pytest.mark.parametrize("n,dt", [(21, "c128"), (21, "c64"), (24, "c128"), (24, "c64"), (30, "c128"), (30, "c64"), (31, "c64")])
def test_sample_parity_large(n, dt):
    """Registers whose chunk scan gives each thread several chunks (n >= 21)
    and whose chunks widen beyond 2^12 amplitudes (n >= 31).  The oracle
    samples the same amplitudes the kernel sampled (complex64 values are exact
    in complex128), with a gate on the top qubit so the distribution is not
    the initial one."""
    import torch
    nbytes = (1 << n) * (16 if dt == "c128" else 8)
    if n >= 30:
        free, _ = torch.cuda.mem_get_info()
        if free < nbytes + (4 << 30):
            pytest.skip(f"needs {nbytes >> 30} GiB of free device memory")
    U = W.haar_list(n, 1)[0]
    s = _state(n, dt).init_random(n)
    s.apply_1q(n - 1, U)
    host = s.amps.cpu().numpy()
    if dt == "c64":
        host = host.astype(np.complex128)
    _sample_check(s, host, 1 << 16, 1000 + n)
    del s, host
    torch.cuda.empty_cache()


def test_sample_degenerate():
    s = _state(9).init_basis(300)
    assert np.all(s.sample(1000, seed=1).cpu().numpy() == 300)
    assert s.sample(0, seed=1).numel() == 0


def test_errors_are_reported():
    from paper_2001_10554_amd.qsim import QsimError, QS_ERR_ARG
    s = _state(4)
    with pytest.raises(QsimError) as e:
        s.apply_1q(4, np.eye(2))
    assert e.value.code == QS_ERR_ARG
    with pytest.raises(QsimError):
        s.apply_c1q(1, 1, np.eye(2))
    with pytest.raises(QsimError):
        s.init_basis(16)
    with pytest.raises(QsimError):
        s.expect_pauli(16, 0)
    bad = W.random_block(4, 3, 1)
    bad[1]["kind"] = 9
    with pytest.raises(QsimError):
        s.apply_block(bad)
