"""Named gates as matrices for the C-ABI's gate calls (host-side tables only).

Conventions: a one-qubit matrix is 2x2 with row = output index (eq. (3));
rotations are R_P(theta) = exp(-i theta P / 2) for P in {X, Y, Z}; two- and
three-qubit matrices index their rows and columns with bit m = qubit m of the
call's qubit list (so for TOFFOLI(c0, c1, t) the list is [c0, c1, t]).
"""
from __future__ import annotations

import math

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)
S = np.array([[1, 0], [0, 1j]], dtype=np.complex128)
SDG = S.conj().T
T = np.array([[1, 0], [0, np.exp(0.25j * math.pi)]], dtype=np.complex128)
TDG = T.conj().T
SX = 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=np.complex128)  # square root of X


def rx(theta: float) -> np.ndarray:
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def ry(theta: float) -> np.ndarray:
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def rz(theta: float) -> np.ndarray:
    return np.array([[np.exp(-0.5j * theta), 0], [0, np.exp(0.5j * theta)]], dtype=np.complex128)


def phase(phi: float) -> np.ndarray:
    return np.array([[1, 0], [0, np.exp(1j * phi)]], dtype=np.complex128)


def u3(theta: float, phi: float, lam: float) -> np.ndarray:
    """General one-qubit unitary Rz(phi) Ry(theta) Rz(lam) up to a global phase."""
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array([[c, -np.exp(1j * lam) * s], [np.exp(1j * phi) * s, np.exp(1j * (phi + lam)) * c]], dtype=np.complex128)


def cphase_diag(phi: float) -> np.ndarray:
    """Diagonal of the controlled phase on (q0, q1): entries d[2 b1 + b0]."""
    return np.array([1, 1, 1, np.exp(1j * phi)], dtype=np.complex128)


CZ_DIAG = cphase_diag(math.pi)


def _perm(n_bits: int, f) -> np.ndarray:
    D = 1 << n_bits
    m = np.zeros((D, D), dtype=np.complex128)
    for j in range(D):
        m[f(j), j] = 1.0
    return m


# qubit list [c0, c1, t]: flip bit 2 when bits 0 and 1 are set
TOFFOLI = _perm(3, lambda j: j ^ 4 if (j & 3) == 3 else j)
# qubit list [c, a, b]: exchange bits 1 and 2 when bit 0 is set
FREDKIN = _perm(3, lambda j: (j & 1) | ((j >> 1) & 2) | ((j << 1) & 4) if j & 1 else j)
# qubit list [a, b]: |01> -> i|10>, |10> -> i|01>
ISWAP = np.array([[1, 0, 0, 0], [0, 0, 1j, 0], [0, 1j, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)
