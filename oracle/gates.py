"""The oracle's own gate table, written from the gates' definitions.

Convention: a one-qubit matrix is indexed U[out, in].  The paper names the
gates (H, CZ, sqrt X, sqrt Y, T) in its circuit prescription but prints no
matrices; the readings used here are the standard ones:

* H = (1/sqrt2) [[1, 1], [1, -1]]
* sqrt X, sqrt Y: the principal square roots of the Pauli X and Y
  (eigenvalue +1 kept, eigenvalue -1 mapped to +i):
  sqrt X = 1/2 [[1+i, 1-i], [1-i, 1+i]],  sqrt Y = 1/2 [[1+i, -1-i], [1+i, 1+i]]
* T = diag(1, e^{i pi/4})
* CZ = diag(1, 1, 1, -1) on the two-qubit basis |q0 q1>.
"""

import numpy as np

GATE_H, GATE_SQRT_X, GATE_SQRT_Y, GATE_T, GATE_CZ = 0, 1, 2, 3, 4

_s2 = 1.0 / np.sqrt(2.0)

ORACLE_GATES = {
    GATE_H: np.array([[_s2, _s2], [_s2, -_s2]], dtype=np.complex128),
    GATE_SQRT_X: 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=np.complex128),
    GATE_SQRT_Y: 0.5 * np.array([[1 + 1j, -1 - 1j], [1 + 1j, 1 + 1j]], dtype=np.complex128),
    GATE_T: np.array([[1, 0], [0, np.exp(1j * np.pi / 4)]], dtype=np.complex128),
    GATE_CZ: np.diag(np.array([1, 1, 1, -1], dtype=np.complex128)),
}

DIAGONAL = {GATE_T, GATE_CZ}


def gate_matrix(kind: int) -> np.ndarray:
    return ORACLE_GATES[int(kind)].copy()
