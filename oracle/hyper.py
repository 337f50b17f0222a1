"""O4: the circuit's hypergraph network, contracted along a given pairwise tree.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``, never by the library.

The network is the paper's refactored form (Section "Benchmarking and the
Experimental Setup", refactoring paragraph: nodes hold tensors, hyper-edges
are running indices).  Every qubit's wire is cut at each non-diagonal gate
(H, sqrt X, sqrt Y); each piece (q, o) -- o counting the non-diagonal gates
applied to q before it -- is one binary index, held by every tensor that acts
on that piece.  The tensors, numbered as a plan's exported tree numbers them:

* t = q < n: qubit q's input state, the vector e_0 on (q, 0);
* t = n + g: gate g of the circuit --
  H, sqrt X, sqrt Y: U[new, old] on ((q, o + 1), (q, o));
  T: its diagonal (1, e^{i pi/4}) on (q, o);
  CZ: its diagonal as the 2x2 tensor D[a, b] = (-1)^(a b) on the two
  qubits' current pieces.

The value of a network is the sum, over all values of its indices, of the
product of its tensors' entries.  The output piece of qubit q is fixed to
x[q], and a sliced piece to its bit of the slice id, by taking that
sub-block of every tensor holding it; with all other indices summed, the
values of all slices add up to <x|C|0^n> (the paper's preprocessing
paragraph: subtask results add up to the amplitude).

Contraction: two tensors are multiplied entry by entry over their common
indices, and an index is summed as soon as no other remaining tensor holds
it; the result does not depend on the order of the pairwise products (up to
rounding).  The order is an input here -- a partition of the tensors into
leaves and a list of pairwise merges, as a plan exports it -- and is treated
as data only: it is validated, then followed.  Each product is computed in
complex128 with plain PyTorch CPU operations (multi-threaded): both operands
permuted to [batch, free, summed] and one batched matrix product; nothing is
blocked or fused.
Without a given tree, ``contract_greedy`` picks its own order (the pair
whose product is smallest, ties by id).

Pins (``tests/test_oracle_o4.py``): own order vs the state vector (O1) and
vs the plain network (O2); per-slice values along library trees vs the plain
network's sliced values (O3); slice sums vs O1; the same slice under two
different trees; rejection of invalid trees.
"""

import numpy as np
import torch

from .gates import GATE_CZ, GATE_T, gate_matrix


def hyper_network(n_qubits: int, circuit):
    """Returns (tensors, out_ordinal): tensors[t] = (array, [(q, o), ...]) in
    the numbering above, out_ordinal[q] = the ordinal of q's output piece."""
    n = int(n_qubits)
    ordinal = [0] * n
    tensors = [(np.array([1.0, 0.0], dtype=np.complex128), [(q, 0)]) for q in range(n)]
    cz = np.diag(gate_matrix(GATE_CZ)).reshape(2, 2)
    t_diag = np.diag(gate_matrix(GATE_T)).copy()
    for kind, q0, q1, _m in np.asarray(circuit):
        kind, q0, q1 = int(kind), int(q0), int(q1)
        if kind == GATE_CZ:
            tensors.append((cz.copy(), [(q0, ordinal[q0]), (q1, ordinal[q1])]))
        elif kind == GATE_T:
            tensors.append((t_diag.copy(), [(q0, ordinal[q0])]))
        else:
            old = (q0, ordinal[q0])
            ordinal[q0] += 1
            tensors.append((gate_matrix(kind), [(q0, ordinal[q0]), old]))
    return tensors, ordinal


def fix_pieces(tensors, fixed: dict):
    """Sub-block of every tensor with each index in ``fixed`` set to its value
    (as complex128 torch CPU tensors)."""
    out = []
    for arr, idx in tensors:
        sel = tuple(int(fixed[e]) if e in fixed else slice(None) for e in idx)
        sub = np.array(np.asarray(arr)[sel], dtype=np.complex128)
        out.append((torch.from_numpy(sub), [e for e in idx if e not in fixed]))
    return out


def _product(operands, ia, ib, keep):
    """A * B over their common indices, (A, B) = operands (the list is emptied
    so that the operands can be freed once permuted); an index in neither
    ``keep`` (held by another remaining tensor) is summed.  Result indices:
    batch, A-free, B-free."""
    A, B = operands
    operands.clear()
    sa, sb = set(ia), set(ib)
    only_a = [e for e in ia if e not in sb and e not in keep]
    only_b = [e for e in ib if e not in sa and e not in keep]
    if only_a:
        A = A.sum(dim=tuple(ia.index(e) for e in only_a))
        ia = [e for e in ia if e not in only_a]
    if only_b:
        B = B.sum(dim=tuple(ib.index(e) for e in only_b))
        ib = [e for e in ib if e not in only_b]
    sb = set(ib)
    batch = [e for e in ia if e in sb and e in keep]
    summed = [e for e in ia if e in sb and e not in keep]
    free_a = [e for e in ia if e not in sb]
    free_b = [e for e in ib if e not in set(ia)]
    nb, na, nk, nf = (1 << len(batch)), (1 << len(free_a)), (1 << len(summed)), (1 << len(free_b))
    At = A.permute([ia.index(e) for e in batch + free_a + summed]).reshape(nb, na, nk)
    Bt = B.permute([ib.index(e) for e in batch + summed + free_b]).reshape(nb, nk, nf)
    del A, B
    C = torch.bmm(At, Bt)
    out_idx = batch + free_a + free_b
    return C.reshape([2] * len(out_idx)), out_idx


class _Live:
    """Remaining tensors and, per index, how many of them hold it."""

    def __init__(self, tensors):
        self.t = {k: (arr, list(idx)) for k, (arr, idx) in enumerate(tensors)}
        self.count = {}
        for _arr, idx in tensors:
            for e in idx:
                self.count[e] = self.count.get(e, 0) + 1

    def merge(self, ka, kb, knew):
        ia, ib = self.t[ka][1], self.t[kb][1]
        for e in ia + ib:
            self.count[e] -= 1
        keep = {e for e in set(ia) | set(ib) if self.count[e] > 0}
        operands = [self.t.pop(ka)[0], self.t.pop(kb)[0]]
        C, ic = _product(operands, ia, ib, keep)
        for e in ic:
            self.count[e] += 1
        self.t[knew] = (C, ic)
        return C.numel()


def _greedy_pairs(live, keys, next_key):
    """Contracts the tensors ``keys`` of ``live`` into one by the smallest
    product first (ties by key); returns its key and the next free key."""
    keys = list(keys)
    while len(keys) > 1:
        best = None
        for i, ka in enumerate(keys):
            sa = set(live.t[ka][1])
            for kb in keys[i + 1:]:
                ib = live.t[kb][1]
                shared = sa & set(ib)
                if not shared and best is not None and best[0] == 0:
                    continue
                # Result rank if every shared index still held elsewhere stays.
                rank = len(sa | set(ib)) - sum(1 for e in shared if live.count[e] == 2)
                key = (0 if shared else 1, rank, ka, kb)
                if best is None or key < best:
                    best = key
        _c, _r, ka, kb = best
        live.merge(ka, kb, next_key)
        keys = [k for k in keys if k not in (ka, kb)] + [next_key]
        next_key += 1
    return keys[0], next_key


def _scalar(arr, idx):
    if idx:
        raise AssertionError(f"indices left open after the contraction: {idx}")
    return complex(arr.reshape(()).item())


def validate_tree(n_tensors: int, groups, merges):
    """Raises ValueError unless groups partition range(n_tensors) and merges
    form one binary tree over the groups (each node used once, operands of
    merge i among the leaves and merges before i)."""
    seen = np.zeros(int(n_tensors), dtype=np.int64)
    for g in groups:
        for t in g:
            if not 0 <= int(t) < n_tensors:
                raise ValueError(f"tensor id {t} out of range")
            seen[int(t)] += 1
    if len(groups) == 0 or (seen != 1).any():
        raise ValueError("the leaves do not partition the circuit's tensors")
    L = len(groups)
    merges = np.asarray(merges, dtype=np.int64).reshape(-1, 2)
    if len(merges) != L - 1:
        raise ValueError(f"{len(merges)} merges for {L} leaves")
    used = np.zeros(2 * L - 1, dtype=bool)
    for i, (a, b) in enumerate(merges):
        for v in (a, b):
            if not 0 <= v < L + i or used[v]:
                raise ValueError(f"merge {i}: node {v} invalid or used twice")
            used[v] = True
        if a == b:
            raise ValueError(f"merge {i} joins a node with itself")
    return merges


def contract_tree(tensors, groups, merges) -> complex:
    """Value of the network ``tensors`` (all open indices already fixed)
    along the tree (groups, merges)."""
    merges = validate_tree(len(tensors), groups, merges)
    live = _Live(tensors)
    next_key = len(tensors)
    node = []
    for g in groups:
        k, next_key = _greedy_pairs(live, sorted(int(t) for t in g), next_key)
        node.append(k)
    for a, b in merges:
        live.merge(node[a], node[b], next_key)
        node.append(next_key)
        next_key += 1
    (arr, idx), = live.t.values()
    return _scalar(arr, idx)


def contract_greedy(tensors) -> complex:
    """Value of the network with this module's own order."""
    live = _Live(tensors)
    k, _ = _greedy_pairs(live, range(len(tensors)), len(tensors))
    arr, idx = live.t[k]
    return _scalar(arr, idx)


def hyper_value(n_qubits: int, circuit, bitstring, segments=(), s: int = 0, tree=None) -> complex:
    """Value of slice ``s`` of <x|C|0^n>: segments[j] = (q, o) fixed to bit j
    of s (bit 0 least significant), output pieces to x[q]; contracted along
    ``tree`` = (groups, merges) if given, else in this module's own order."""
    tensors, out_ord = hyper_network(n_qubits, circuit)
    x = np.asarray(bitstring, dtype=np.int64)
    fixed = {(q, out_ord[q]): int(x[q]) for q in range(int(n_qubits))}
    for j, seg in enumerate(segments):
        key = (int(seg[0]), int(seg[1]))
        if key in fixed:
            raise ValueError(f"segment {key} is repeated or an output piece")
        if key[1] == 0:
            raise ValueError(f"segment {key} is an input piece")
        fixed[key] = (int(s) >> j) & 1
    t = fix_pieces(tensors, fixed)
    if tree is None:
        return contract_greedy(t)
    return contract_tree(t, tree[0], tree[1])
