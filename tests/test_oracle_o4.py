"""Pins for O4 (oracle/hyper.py): the hypergraph network contracted along a
tree given as data.

O4 is checked against formulations that share none of its code: the state
vector (O1), the path sum, the plain one-tensor-per-gate network (O2) and
its sliced values (O3), and closed forms.  The trees come from library plans
(read through ``qc_plan_export_tree``, data only) or from O4's own greedy.
Any valid tree must give the same value (the order of pairwise products
does not change a network's value); a tree that is not valid is rejected.
"""

import itertools

import numpy as np
import pytest

import oracle
import synth
from paper_1907_11217_amd import qcsim
from synth import GATE_CZ, GATE_T

W = np.exp(1j * np.pi / 4)


def _all_x(n):
    return np.array(list(itertools.product((0, 1), repeat=n)), dtype=np.uint8)


@pytest.mark.parametrize("shape,depth,seed", [((2, 2), 4, 1), ((2, 3), 5, 2), ((3, 3), 8, 3)])
def test_o4_own_order_equals_statevector_all_x(shape, depth, seed):
    lat = synth.grid(*shape)
    circ = synth.random_circuit(lat, depth, seed)
    psi = oracle.statevector(lat.n, circ, impl="numpy")
    xs = _all_x(lat.n)
    if len(xs) > 64:
        xs = xs[np.random.default_rng(seed).choice(len(xs), 64, replace=False)]
    for x in xs:
        assert abs(oracle.hyper_value(lat.n, circ, x) - psi[oracle.index_of(x)]) < 1e-14


def test_o4_equals_path_sum_and_plain_network():
    lat = synth.grid(2, 3)
    circ = synth.random_circuit(lat, 4, 17)
    for x in synth.random_bitstrings(lat.n, 4, 18):
        v = oracle.hyper_value(lat.n, circ, x)
        assert abs(v - oracle.pathsum_amplitude(lat.n, circ, x)) < 1e-14
        assert abs(v - oracle.tn_amplitude(lat.n, circ, x)) < 1e-14


def test_o4_walsh_sum_closed_form():
    # H - (CZ, T layers) - H on 3x3: amp(x) = 2^-n sum_z w^{T.z} (-1)^{E(z) + x.z}.
    lat = synth.grid(3, 3)
    n = lat.n
    circ = synth.random_circuit(lat, 6, 29, gate_set=(GATE_T, GATE_T, GATE_T))
    zs = _all_x(n).astype(np.int64)
    expo, sign = np.zeros(len(zs), np.int64), np.zeros(len(zs), np.int64)
    for k, a, b, _ in circ:
        if k == GATE_T:
            expo += zs[:, a]
        elif k == GATE_CZ:
            sign += zs[:, a] * zs[:, b]
    g = W ** expo * (-1.0) ** sign
    for x in synth.random_bitstrings(n, 8, 30):
        expect = (g * (-1.0) ** (zs @ x.astype(np.int64))).sum() / 2.0 ** n
        assert abs(oracle.hyper_value(n, circ, x) - expect) < 1e-14


def _plan(lat, circ, x, **kw):
    kw.setdefault("greedy_trials", 4)
    kw.setdefault("seed", 1)
    return qcsim.qc_plan_build(lat.n, circ, x, **kw)


def test_o4_c1_plan_tree_slices_equal_o3_and_sum_to_o1():
    lat, circ, _bs, _ = synth.config("c1")
    xs = synth.random_bitstrings(lat.n, 3, 77)
    plan = _plan(lat, circ, xs[0], log2_slices=4)
    tree = qcsim.qc_plan_export_tree(plan)
    segs = qcsim.qc_plan_sliced_segments(plan)
    assert len(segs) == 4
    psi = oracle.statevector(lat.n, circ)
    for x in xs:
        vals = [oracle.hyper_value(lat.n, circ, x, segs, s, tree) for s in range(16)]
        for s in (0, 5, 15):
            assert abs(vals[s] - oracle.sliced_value(lat.n, circ, x, segs, s)) < 1e-14
        assert abs(sum(vals) - psi[oracle.index_of(x)]) < 1e-14


def test_o4_c2_plan_tree_sums_to_statevector():
    lat, circ, bs, spec = synth.config("c2")
    plan = _plan(lat, circ, bs[0], log2_slices=spec["log2_slices"])
    tree = qcsim.qc_plan_export_tree(plan)
    segs = qcsim.qc_plan_sliced_segments(plan)
    psi = oracle.statevector(lat.n, circ)
    for x in bs[:2]:
        total = sum(oracle.hyper_value(lat.n, circ, x, segs, s, tree) for s in range(1 << len(segs)))
        ref = psi[oracle.index_of(x)]
        assert abs(total - ref) <= 1e-12 * abs(ref) + 1e-18


def test_o4_c2_slice_equals_o3():
    lat, circ, bs, spec = synth.config("c2")
    plan = _plan(lat, circ, bs[0], log2_slices=spec["log2_slices"])
    tree = qcsim.qc_plan_export_tree(plan)
    segs = qcsim.qc_plan_sliced_segments(plan)
    for s in synth.random_slices(len(segs), 2, 203):
        v4 = oracle.hyper_value(lat.n, circ, bs[1], segs, int(s), tree)
        v3 = oracle.sliced_value(lat.n, circ, bs[1], segs, int(s))
        assert abs(v4 - v3) <= 1e-12 * abs(v3) + 1e-18


def _rotated(tree, count, seed):
    """Another valid tree for the same leaves: ``count`` random rotations
    ((X Y) Z) -> (X (Y Z)) of merges whose third operand Z already exists
    when (X Y) is formed."""
    groups, merges = tree
    merges = np.array(merges, dtype=np.int64)
    L = len(groups)
    rng = np.random.default_rng(seed)
    done = 0
    for i in rng.permutation(len(merges)):
        if done == count:
            break
        for side in (0, 1):
            j = int(merges[i, side]) - L
            z = int(merges[i, 1 - side])
            if j >= 0 and z < L + j:
                x, y = merges[j]
                merges[j] = (y, z)
                merges[i] = (x, L + j)
                done += 1
                break
    assert done == count
    return groups, merges


def test_o4_same_slice_two_trees_70_qubits():
    # The 70-qubit diamond at depth 8: the plan's tree and a rotated version of
    # it must give the same slice values, and so must the plain network (O3,
    # its own order, no hyper-edges).
    lat = synth.diamond70()
    circ = synth.random_circuit(lat, 8, 411)
    x = synth.random_bitstrings(lat.n, 1, 412)[0]
    p1 = _plan(lat, circ, x, log2_slices=3, seed=1)
    segs = qcsim.qc_plan_sliced_segments(p1)
    t1 = qcsim.qc_plan_export_tree(p1)
    t2 = _rotated(t1, 12, 5)
    oracle.validate_tree(lat.n + len(circ), *t2)
    nonzero = 0
    for s in range(8):
        a = oracle.hyper_value(lat.n, circ, x, segs, s, t1)
        b = oracle.hyper_value(lat.n, circ, x, segs, s, t2)
        c = oracle.sliced_value(lat.n, circ, x, segs, s)
        scale = max(abs(c), 2.0 ** -lat.n)
        assert abs(a - b) <= 1e-12 * scale
        assert abs(a - c) <= 1e-12 * scale
        nonzero += abs(c) > 1e-15
    assert nonzero >= 2


def test_o4_rejects_invalid_trees():
    lat, circ, bs, _ = synth.config("c1")
    plan = _plan(lat, circ, bs[0], log2_slices=0)
    groups, merges = qcsim.qc_plan_export_tree(plan)
    tensors, _ = oracle.hyper_network(lat.n, circ)
    T = len(tensors)
    oracle.validate_tree(T, groups, merges)
    with pytest.raises(ValueError):          # a tensor left out
        oracle.validate_tree(T, [g[1:] if i == 0 else g for i, g in enumerate(groups)], merges)
    with pytest.raises(ValueError):          # a tensor in two leaves
        oracle.validate_tree(T, [g + groups[0][:1] if i == 1 else g for i, g in enumerate(groups)], merges)
    bad = merges.copy()
    bad[-1] = bad[0]
    with pytest.raises(ValueError):          # a node used twice
        oracle.validate_tree(T, groups, bad)
    with pytest.raises(ValueError):          # a merge missing
        oracle.validate_tree(T, groups, merges[:-1])
    bad = merges.copy()
    bad[0, 0] = len(groups) + 3              # a merge result used before it exists
    with pytest.raises(ValueError):
        oracle.validate_tree(T, groups, bad)


def test_o4_export_tree_is_a_partition_of_the_circuit():
    lat, circ, bs, spec = synth.config("c3")
    plan = _plan(lat, circ, bs[0], log2_slices=spec["log2_slices"], log2_max_entries=spec["log2_cap"], greedy_trials=2)
    groups, merges = qcsim.qc_plan_export_tree(plan)
    ids = np.sort(np.concatenate([np.asarray(g) for g in groups]))
    assert (ids == np.arange(lat.n + len(circ))).all()
    assert merges.shape == (len(groups) - 1, 2)
