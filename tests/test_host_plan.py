"""Pass planning of the fused block (host logic, no GPU): qs_block_passes
returns how many read+write passes of the state qs_apply_block takes.

Tiles hold 12 qubits for complex128 and 13 for complex64, always including
the lowest 3 (c128) or 4 (c64) qubits, so a pass can add 9 new target qubits.
The expected counts below follow from that by hand.
"""
import numpy as np
import pytest
import torch

from paper_2001_10554_amd import workloads as W
from paper_2001_10554_amd.qsim import QsimError, block_passes

X = W.PAULI_X


def one_q(qubits):
    return W.gates_array([W.gate(W.G_1Q, q, -1, X) for q in qubits])


def test_empty_and_single_tile():
    assert block_passes(20, W.gates_array([])) == 0
    # 12 qubits fit one c128 tile whatever the gates
    assert block_passes(12, W.brick_circuit(12, 20, seed=1)) == 1


@pytest.mark.parametrize("n", [16, 24, 30])
@pytest.mark.parametrize("dt,tb,low", [(torch.complex128, 12, 3), (torch.complex64, 13, 4)])
def test_one_gate_per_qubit(n, dt, tb, low):
    # the first pass covers qubits 0..tb-1, every further one tb - low new qubits
    want = 1 + -(-(n - tb) // (tb - low))
    assert block_passes(n, one_q(range(n)), dt) == want


def test_diagonal_gates_ride_along():
    d = np.exp(1j * np.arange(4))
    g = W.gates_array([W.gate(W.G_DIAG2, a, b, d) for a in range(20) for b in range(a + 1, 20)])
    assert block_passes(20, g) == 1
    # one 1q gate joins any tile; 1q gates on all 20 qubits need 1 + ceil(8 / 9) = 2
    # passes with or without the diagonals around them
    assert block_passes(20, np.concatenate([g, one_q([19]), g])) == 1
    assert block_passes(20, np.concatenate([g, one_q(range(20)), g])) == 2


def test_commuting_gates_move_ahead():
    """14 qubits, c128.  List order: [q3..q11] fills the tile, q12 starts a
    second pass that also takes q3..q10, q11 a third: 3 passes.  The gates on
    q3..q11 commute with the q12 gate left behind, so the first pass takes
    both rounds and the two q12 gates share the second: 2 passes."""
    mid = list(range(3, 12))
    assert block_passes(14, one_q(mid + [12] + mid + [12])) == 2
    # a gate on q12 between the rounds that does not commute with a later
    # gate on q3 keeps that gate behind, but the others still move: 2 passes
    d = np.exp(1j * np.arange(4))
    g = np.concatenate([one_q(mid + [12]), W.gates_array([W.gate(W.G_DIAG2, 12, 3, d)]), one_q(mid + [12])])
    assert block_passes(14, g) == 2


def test_list_order_kept_without_gain():
    """The second round of controlled gates shares qubit 12 with the 1q gate
    on it, so nothing moves: list order, i.e. [C(12, 3..11)] (tile full),
    [X(12), C(12, 3..10)], [C(12, 11)]: 3 passes."""
    g = W.gates_array([W.gate(W.G_C1Q, 12, t, X) for t in range(3, 12)] + [W.gate(W.G_1Q, 12, -1, X)]
                      + [W.gate(W.G_C1Q, 12, t, X) for t in range(3, 12)])
    assert block_passes(14, g) == 3


def test_errors():
    with pytest.raises(QsimError):
        block_passes(0, one_q([0]))
    with pytest.raises(QsimError):
        block_passes(4, one_q([4]))  # qubit out of range
    with pytest.raises(QsimError):
        block_passes(40, one_q([0]))  # above the register limit
