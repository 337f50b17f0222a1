"""The amplitude as an explicit path sum over wire segments (brute force).

Each qubit's wire is cut at every non-diagonal gate (H, sqrt X, sqrt Y); a
piece of wire between two cuts is a segment carrying one bit.  The input
segment of every qubit is 0 and its output segment is x[q].  For one
assignment of all other segments the path weight is the product over gates,
in order, of U[new segment, old segment] for a non-diagonal U, T[s, s] for a
T, and the CZ diagonal entry for a CZ; the amplitude is the sum of the path
weights over all assignments.  Vectorised over assignments with numpy, so it
is only for circuits with at most ~22 free segments.
"""

import numpy as np

from .gates import GATE_CZ, GATE_T, gate_matrix


def pathsum_amplitude(n_qubits: int, circuit, bitstring, max_free: int = 24) -> complex:
    circuit = np.asarray(circuit)
    x = np.asarray(bitstring, dtype=np.int64)
    n = int(n_qubits)
    # Count non-diagonal gates per qubit to know which segment is the output.
    n_cut = np.zeros(n, dtype=np.int64)
    for kind, q0, _q1, _m in circuit:
        if int(kind) not in (GATE_T, GATE_CZ):
            n_cut[int(q0)] += 1
    # Free segments: every segment that is neither an input nor an output.
    free = {}
    for q in range(n):
        for o in range(1, int(n_cut[q])):
            free[(q, o)] = len(free)
    F = len(free)
    if F > max_free:
        raise ValueError(f"{F} free segments: too many for the brute-force path sum")
    assign = (np.arange(1 << F, dtype=np.int64)[:, None] >> np.arange(F, dtype=np.int64)[None, :]) & 1

    def seg_value(q, o):
        if o == 0:
            return np.zeros(1 << F, dtype=np.int64)
        if o == n_cut[q]:
            return np.full(1 << F, x[q], dtype=np.int64)
        return assign[:, free[(q, o)]]

    ordinal = np.zeros(n, dtype=np.int64)
    weight = np.ones(1 << F, dtype=np.complex128)
    for kind, q0, q1, _m in circuit:
        kind, q0, q1 = int(kind), int(q0), int(q1)
        if kind == GATE_CZ:
            a = seg_value(q0, ordinal[q0])
            b = seg_value(q1, ordinal[q1])
            weight = weight * np.where((a & b) == 1, -1.0, 1.0)
        elif kind == GATE_T:
            s = seg_value(q0, ordinal[q0])
            weight = weight * gate_matrix(GATE_T)[s, s]
        else:
            old = seg_value(q0, ordinal[q0])
            ordinal[q0] += 1
            new = seg_value(q0, ordinal[q0])
            weight = weight * gate_matrix(kind)[new, old]
    # A qubit with no non-diagonal gate has one segment that is both the
    # input (0) and the output (x[q]): the amplitude vanishes unless x[q] = 0.
    for q in range(n):
        if n_cut[q] == 0 and x[q] != 0:
            return 0j
    return complex(weight.sum())
