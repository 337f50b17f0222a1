"""O1: the amplitude by its definition, psi = U_L ... U_1 e_0 in complex128.

Qubit q is bit (n-1-q) of the basis index, i.e. qubit 0 is the most
significant bit, and idx(x) = sum_q x[q] 2^(n-1-q).  Gates are applied one
at a time in the order given; a one-qubit gate U acts as
psi'[..., a, ...] = sum_b U[a, b] psi[..., b, ...] on its qubit's axis.
"""

import numpy as np

from .gates import GATE_CZ, GATE_T, gate_matrix


def index_of(bits) -> int:
    bits = np.asarray(bits, dtype=np.int64)
    n = bits.shape[-1]
    return int(np.sum(bits * (1 << np.arange(n - 1, -1, -1, dtype=np.int64))))


def statevector(n_qubits: int, circuit, impl: str = "auto") -> np.ndarray:
    """``impl``: "numpy" (this function's loop), "c" (the same definition in
    plain C with OpenMP, ``sv.c``), or "auto" (C from 18 qubits up)."""
    if impl == "c" or (impl == "auto" and int(n_qubits) >= 18):
        from .csv import statevector_c
        return statevector_c(n_qubits, circuit)
    circuit = np.asarray(circuit)
    n = int(n_qubits)
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    for kind, q0, q1, _moment in circuit:
        kind, q0, q1 = int(kind), int(q0), int(q1)
        if kind == GATE_CZ:
            a, b = min(q0, q1), max(q0, q1)
            v = psi.reshape(1 << a, 2, 1 << (b - a - 1), 2, 1 << (n - b - 1))
            v[:, 1, :, 1, :] *= -1.0
        elif kind == GATE_T:
            v = psi.reshape(1 << q0, 2, 1 << (n - q0 - 1))
            v[:, 1, :] *= gate_matrix(GATE_T)[1, 1]
        else:
            u = gate_matrix(kind)
            v = psi.reshape(1 << q0, 2, 1 << (n - q0 - 1))
            lo = v[:, 0, :].copy()
            hi = v[:, 1, :].copy()
            v[:, 0, :] = u[0, 0] * lo + u[0, 1] * hi
            v[:, 1, :] = u[1, 0] * lo + u[1, 1] * hi
    return psi


def amplitudes_sv(n_qubits: int, circuit, bitstrings) -> np.ndarray:
    """amp(x) for each row x of ``bitstrings`` (uint8 [n_bs, n])."""
    psi = statevector(n_qubits, circuit)
    bs = np.atleast_2d(np.asarray(bitstrings))
    return np.array([psi[index_of(x)] for x in bs], dtype=np.complex128)
