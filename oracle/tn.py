"""O2/O3: a plain tensor network, one tensor per gate, contracted pairwise.

Every gate is its own tensor with explicit input and output wire indices
(a one-qubit gate is U[out, in]; a CZ is the 2x2x2x2 tensor
CZ[a', b', a, b] = delta(a', a) delta(b', b) (-1)^(a b)).  Each qubit starts
with the vector <0| ... i.e. e_0 on its first wire index and ends with
e_{x[q]} on its last.  Every index joins exactly two tensors, so there are no
hyper-edges here: this is deliberately a different formulation from the
library's hypergraph network (the paper's Section "Benchmarking and the
Experimental Setup" describes the library's form, a node per tensor and a
hyper-edge per running index).

Slicing (the paper's subtasks whose results add up to the amplitude): a
segment (q, o) is the piece of qubit q's wire after its o-th non-diagonal
gate (o = 0: from the input) up to the next non-diagonal gate.  All plain
wire indices on that piece pass only through diagonal gates, so in every
non-zero term they carry the same bit.  ``sliced_value`` fixes every one of
them to bit j of the slice id s, for the j-th listed segment; the sum of the
sliced values over all s is the amplitude.

The contraction order is the oracle's own: either a greedy pairwise order
(``order="greedy"``: merge the pair of neighbouring tensors whose result
minimises size(C) - size(A) - size(B)) or a sweep that folds the tensors in
creation order into one accumulator (``order="sweep"``, tiny circuits only).
"""

import itertools
import string

import numpy as np

from .gates import GATE_CZ, GATE_T, gate_matrix

_LETTERS = string.ascii_letters


def _cz4() -> np.ndarray:
    t = np.zeros((2, 2, 2, 2), dtype=np.complex128)
    for a, b in itertools.product((0, 1), repeat=2):
        t[a, b, a, b] = -1.0 if (a and b) else 1.0
    return t


def segment_counts(n_qubits: int, circuit) -> np.ndarray:
    """Number of non-diagonal gates per qubit (= ordinal of its output segment)."""
    cnt = np.zeros(int(n_qubits), dtype=np.int64)
    for kind, q0, _q1, _m in np.asarray(circuit):
        if int(kind) not in (GATE_T, GATE_CZ):
            cnt[int(q0)] += 1
    return cnt


def build_plain_network(n_qubits: int, circuit, bitstring):
    """Returns (tensors, segment_of): tensors is a list of (array, [index ids]),
    segment_of maps each wire index id to its segment (q, ordinal)."""
    circuit = np.asarray(circuit)
    x = np.asarray(bitstring, dtype=np.int64)
    n = int(n_qubits)
    tensors = []
    segment_of = {}
    next_id = itertools.count()
    wire = [0] * n
    ordinal = [0] * n
    for q in range(n):
        w = next(next_id)
        segment_of[w] = (q, 0)
        wire[q] = w
        tensors.append((np.array([1.0, 0.0], dtype=np.complex128), [w]))
    for kind, q0, q1, _m in circuit:
        kind, q0, q1 = int(kind), int(q0), int(q1)
        if kind == GATE_CZ:
            a, b = next(next_id), next(next_id)
            segment_of[a] = (q0, ordinal[q0])
            segment_of[b] = (q1, ordinal[q1])
            tensors.append((_cz4(), [a, b, wire[q0], wire[q1]]))
            wire[q0], wire[q1] = a, b
        else:
            if kind != GATE_T:
                ordinal[q0] += 1
            w = next(next_id)
            segment_of[w] = (q0, ordinal[q0])
            tensors.append((gate_matrix(kind), [w, wire[q0]]))
            wire[q0] = w
    for q in range(n):
        e = np.zeros(2, dtype=np.complex128)
        e[x[q]] = 1.0
        tensors.append((e, [wire[q]]))
    return tensors, segment_of


def _fix_indices(tensors, fixed: dict):
    """Select the sub-block index = value in every tensor, for each fixed index."""
    out = []
    for arr, idx in tensors:
        sel = tuple(fixed[i] if i in fixed else slice(None) for i in idx)
        out.append((np.array(arr[sel], dtype=np.complex128), [i for i in idx if i not in fixed]))
    return out


def _pair(a, b):
    """Contract two tensors over their shared indices (each index in <= 2 tensors)."""
    arr_a, ia = a
    arr_b, ib = b
    shared = set(ia) & set(ib)
    out_idx = [i for i in ia if i not in shared] + [i for i in ib if i not in shared]
    letters = {}
    for i in list(ia) + list(ib):
        if i not in letters:
            letters[i] = _LETTERS[len(letters)]
    spec = "".join(letters[i] for i in ia) + "," + "".join(letters[i] for i in ib) \
        + "->" + "".join(letters[i] for i in out_idx)
    return np.einsum(spec, arr_a, arr_b), out_idx


def _greedy(tensors):
    live = {k: t for k, t in enumerate(tensors)}
    holders = {}
    for k, (_a, idx) in live.items():
        for i in idx:
            holders.setdefault(i, set()).add(k)
    next_key = len(tensors)
    while len(live) > 1:
        best = None
        for i, hs in holders.items():
            if len(hs) != 2:
                continue
            ka, kb = sorted(hs)
            ia, ib = live[ka][1], live[kb][1]
            shared = set(ia) & set(ib)
            rc = len(ia) + len(ib) - 2 * len(shared)
            key = ((1 << rc) - (1 << len(ia)) - (1 << len(ib)), rc, ka, kb)
            if best is None or key < best:
                best = key
        if best is None:
            # No shared index left: fold the two smallest tensors (outer product).
            ka, kb = sorted(sorted(live, key=lambda k: (live[k][0].size, k))[:2])
        else:
            ka, kb = best[2], best[3]
        ta, tb = live.pop(ka), live.pop(kb)
        for i in ta[1] + tb[1]:
            holders[i].discard(ka)
            holders[i].discard(kb)
        c = _pair(ta, tb)
        live[next_key] = c
        for i in c[1]:
            holders[i].add(next_key)
        for i in [i for i, hs in holders.items() if not hs]:
            del holders[i]
        next_key += 1
    (arr, idx), = live.values()
    assert not idx, "open indices left after contraction"
    return complex(arr.reshape(()))


def _sweep(tensors):
    acc = tensors[0]
    for t in tensors[1:]:
        acc = _pair(acc, t)
    arr, idx = acc
    assert not idx
    return complex(arr.reshape(()))


def contract_network(tensors, order: str = "greedy") -> complex:
    if order == "greedy":
        return _greedy(tensors)
    if order == "sweep":
        return _sweep(tensors)
    raise ValueError(order)


def tn_amplitude(n_qubits: int, circuit, bitstring, order: str = "greedy") -> complex:
    tensors, _ = build_plain_network(n_qubits, circuit, bitstring)
    return contract_network(tensors, order)


def sliced_value(n_qubits: int, circuit, bitstring, segments, s: int,
                 order: str = "greedy") -> complex:
    """Value of slice ``s``: segment segments[j] = (q, ordinal) is fixed to
    bit j of s (bit 0 = least significant) on every wire index it covers."""
    tensors, segment_of = build_plain_network(n_qubits, circuit, bitstring)
    seg_bit = {tuple(int(v) for v in seg): (int(s) >> j) & 1 for j, seg in enumerate(segments)}
    if len(seg_bit) != len(segments):
        raise ValueError("repeated segment in the slice list")
    fixed = {w: seg_bit[seg] for w, seg in segment_of.items() if seg in seg_bit}
    return contract_network(_fix_indices(tensors, fixed), order)
