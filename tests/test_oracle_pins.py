"""Pins for the FP64 oracle: closed forms, brute force and invariants.

Each test states what it fixes.  None of them re-calls the oracle's own
formula to produce its expected value: the expected values are closed forms
derived in the test from the gates' definitions, or come from a different
formulation (state vector vs. path sum vs. plain tensor network).
"""

import itertools

import numpy as np
import pytest

import oracle
import synth
from synth import GATE_CZ, GATE_H, GATE_SQRT_X, GATE_SQRT_Y, GATE_T

W = np.exp(1j * np.pi / 4)  # the T phase, e^{i pi/4}


def _all_x(n):
    return np.array(list(itertools.product((0, 1), repeat=n)), dtype=np.uint8)


def _circ(rows):
    return np.asarray(rows, dtype=np.int32).reshape(-1, 4)


# ---------------------------------------------------------------- gate table
def test_p1_gate_algebra():
    H, SX, SY, T, CZ = (oracle.gate_matrix(k) for k in (GATE_H, GATE_SQRT_X, GATE_SQRT_Y, GATE_T, GATE_CZ))
    X = np.array([[0, 1], [1, 0]])
    Y = np.array([[0, -1j], [1j, 0]])
    Z = np.diag([1, -1])
    I2 = np.eye(2)
    assert np.allclose(SX @ SX, X, atol=1e-15)
    assert np.allclose(SY @ SY, Y, atol=1e-15)
    assert np.allclose(T @ T, np.diag([1, 1j]), atol=1e-15)
    assert np.allclose(np.linalg.matrix_power(T, 8), I2, atol=1e-15)
    assert np.allclose(H @ H, I2, atol=1e-15)
    assert np.allclose(H, (X + Z) / np.sqrt(2), atol=1e-15)
    assert np.allclose(CZ @ CZ, np.eye(4), atol=1e-15)
    assert np.allclose(np.diag(CZ), [1, 1, 1, -1])
    for U in (H, SX, SY, T, CZ):
        assert np.allclose(U.conj().T @ U, np.eye(U.shape[0]), atol=1e-15)
    # Principal roots: eigenvalues {1, i} (not {1, -i}), trace 1 + i, det i.
    for R in (SX, SY):
        assert np.isclose(np.trace(R), 1 + 1j, atol=1e-15)
        assert np.isclose(np.linalg.det(R), 1j, atol=1e-15)


# ------------------------------------------------- single-gate closed forms
def _three_ways(n, circ, x):
    a = oracle.amplitudes_sv(n, circ, [x])[0]
    b = oracle.pathsum_amplitude(n, circ, x)
    c = oracle.tn_amplitude(n, circ, x)
    return a, b, c


@pytest.mark.parametrize("x,expect", [((0,), 0.5 * (1 + 1j)), ((1,), 0.5 * (1 + 1j))])
def test_sqrt_y_on_zero(x, expect):
    # sqrtY|0> = (1+i)/2 (|0> + |1>): first column of the principal root.
    for v in _three_ways(1, _circ([(GATE_SQRT_Y, 0, -1, 1)]), x):
        assert abs(v - expect) < 1e-15


@pytest.mark.parametrize("x,expect", [((0,), -0.5 * (1 + 1j)), ((1,), 0.5 * (1 + 1j))])
def test_sqrt_y_on_one(x, expect):
    # X|0> = |1>, then sqrtY|1> = (1+i)/2 (-|0> + |1>): second column, which
    # fixes the U[out, in] orientation (the transpose would flip the sign).
    circ = _circ([(GATE_SQRT_X, 0, -1, 1), (GATE_SQRT_X, 0, -1, 2), (GATE_SQRT_Y, 0, -1, 3)])
    for v in _three_ways(1, circ, x):
        assert abs(v - expect) < 1e-15


def test_p10_bit_order():
    # sqrtX sqrtX = X on qubit 0 of 3: the state is |100>, qubit 0 is the MSB.
    circ = _circ([(GATE_SQRT_X, 0, -1, 1), (GATE_SQRT_X, 0, -1, 2)])
    for v in _three_ways(3, circ, (1, 0, 0)):
        assert abs(v - 1) < 1e-15
    for v in _three_ways(3, circ, (0, 0, 1)):
        assert abs(v) < 1e-15
    psi = oracle.statevector(3, circ)
    assert abs(psi[4] - 1) < 1e-15


def test_hth_closed_form():
    # H T H |0>: amp(0) = (1 + w)/2, amp(1) = (1 - w)/2.
    circ = _circ([(GATE_H, 0, -1, 0), (GATE_T, 0, -1, 1), (GATE_H, 0, -1, 2)])
    for v in _three_ways(1, circ, (0,)):
        assert abs(v - (1 + W) / 2) < 1e-15
    for v in _three_ways(1, circ, (1,)):
        assert abs(v - (1 - W) / 2) < 1e-15


# ------------------------------------------------------- circuit closed forms
def test_p2_hadamard_layers_only():
    lat = synth.grid(3, 3)
    circ = synth.random_circuit(lat, 0, 1)
    psi = oracle.statevector(lat.n, circ)
    expect = np.zeros(1 << lat.n)
    expect[0] = 1
    assert np.abs(psi - expect).max() < 1e-14
    for x in _all_x(lat.n)[::37]:
        assert abs(oracle.tn_amplitude(lat.n, circ, x) - (1.0 if not x.any() else 0.0)) < 1e-14
        assert abs(oracle.pathsum_amplitude(lat.n, circ, x) - (1.0 if not x.any() else 0.0)) < 1e-14


def _diag_only_circuit(lat, depth, seed):
    """H layer, then CZ patterns with T drawn on idle qubits (no sqrt X/Y)."""
    return synth.random_circuit(lat, depth, seed, gate_set=(GATE_T, GATE_T, GATE_T), final_h=False)


def _phase_closed_form(n, circ, x):
    # After the H layer every basis state has amplitude 2^{-n/2}; each T on q
    # multiplies by w^{x_q}, each CZ(i, j) by (-1)^{x_i x_j}.
    ph = 1.0 + 0j
    for k, a, b, _ in circ:
        if k == GATE_T:
            ph *= W ** int(x[a])
        elif k == GATE_CZ:
            ph *= (-1) ** (int(x[a]) * int(x[b]))
    return ph * 2.0 ** (-n / 2)


def test_p3_no_final_h_diagonal_layers():
    lat = synth.grid(3, 4)
    circ = _diag_only_circuit(lat, 9, 17)
    assert (circ[:, 0] == GATE_T).any() and (circ[:, 0] == GATE_CZ).any()
    psi = oracle.statevector(lat.n, circ)
    xs = _all_x(lat.n)
    expect = np.array([_phase_closed_form(lat.n, circ, x) for x in xs])
    assert np.abs(psi - expect).max() < 1e-14
    for x in xs[::97]:
        assert abs(oracle.tn_amplitude(lat.n, circ, x) - _phase_closed_form(lat.n, circ, x)) < 1e-14
        assert abs(oracle.pathsum_amplitude(lat.n, circ, x) - _phase_closed_form(lat.n, circ, x)) < 1e-14


def test_p4_h_cz_t_h_walsh_sum():
    # H - (CZ, T layers) - H: amp(x) = 2^-n sum_z w^{#T.z} (-1)^{sum_E z_i z_j + x.z}.
    lat = synth.grid(4, 4)
    n = lat.n
    circ = synth.random_circuit(lat, 8, 23, gate_set=(GATE_T, GATE_T, GATE_T))
    zs = _all_x(n).astype(np.int64)
    expo_t = np.zeros(len(zs), dtype=np.int64)
    sign_cz = np.zeros(len(zs), dtype=np.int64)
    for k, a, b, _ in circ:
        if k == GATE_T:
            expo_t += zs[:, a]
        elif k == GATE_CZ:
            sign_cz += zs[:, a] * zs[:, b]
    g = W ** expo_t * (-1.0) ** sign_cz
    psi = oracle.statevector(n, circ)
    rng = np.random.default_rng(5)
    for i in rng.integers(0, 1 << n, size=48):
        x = np.array([(int(i) >> (n - 1 - q)) & 1 for q in range(n)], dtype=np.int64)
        expect = (g * (-1.0) ** (zs @ x)).sum() / 2.0 ** n
        assert abs(psi[int(i)] - expect) < 1e-14
    x = np.array([(int(rng.integers(0, 1 << n)) >> (n - 1 - q)) & 1 for q in range(n)], dtype=np.uint8)
    expect = (g * (-1.0) ** (zs @ x.astype(np.int64))).sum() / 2.0 ** n
    assert abs(oracle.tn_amplitude(n, circ, x) - expect) < 1e-14


def test_p5_clifford_probabilities_are_dyadic():
    lat = synth.grid(3, 4)
    circ = synth.random_circuit(lat, 10, 31, gate_set=(GATE_SQRT_X, GATE_SQRT_Y))
    p = np.abs(oracle.statevector(lat.n, circ)) ** 2
    nz = p[p > 1e-12]
    j = -np.log2(nz)
    assert np.abs(j - np.round(j)).max() < 1e-9
    assert (np.round(j) >= 0).all() and (np.round(j) <= lat.n).all()
    assert np.abs(p[p <= 1e-12]).max(initial=0) < 1e-25


# --------------------------------------------------------------- invariants
def test_p6_norm_c1():
    lat, circ, _bs, _ = synth.config("c1")
    psi = oracle.statevector(lat.n, circ)
    assert abs(np.sum(np.abs(psi) ** 2) - 1) < 1e-12


@pytest.mark.parametrize("shape,depth,seed", [((2, 2), 4, 1), ((2, 3), 3, 2), ((3, 3), 3, 3), ((3, 3), 2, 4)])
def test_p7_three_formulations_agree(shape, depth, seed):
    lat = synth.grid(*shape)
    circ = synth.random_circuit(lat, depth, seed)
    psi = oracle.statevector(lat.n, circ, impl="numpy")
    psi_c = oracle.statevector(lat.n, circ, impl="c")
    assert np.abs(psi - psi_c).max() < 1e-15
    xs = _all_x(lat.n)
    if len(xs) > 8:
        xs = xs[np.random.default_rng(seed).choice(len(xs), 8, replace=False)]
    for x in xs:
        ref = psi[oracle.index_of(x)]
        assert abs(oracle.pathsum_amplitude(lat.n, circ, x) - ref) < 1e-13
        assert abs(oracle.tn_amplitude(lat.n, circ, x) - ref) < 1e-13


def test_p8_slices_add_up():
    lat = synth.grid(3, 3)
    circ = synth.random_circuit(lat, 6, 8)
    x = synth.random_bitstrings(lat.n, 1, 9)[0]
    cnt = oracle.segment_counts(lat.n, circ)
    segs = [(q, o) for q in range(lat.n) for o in range(1, int(cnt[q]))][:: 3][:4]
    assert len(segs) == 4
    total = sum(oracle.sliced_value(lat.n, circ, x, segs, s) for s in range(16))
    ref = oracle.tn_amplitude(lat.n, circ, x)
    assert abs(total - ref) < 1e-13
    assert abs(ref - oracle.amplitudes_sv(lat.n, circ, [x])[0]) < 1e-13
    # A slice value is not the amplitude (the split is non-trivial).
    assert abs(oracle.sliced_value(lat.n, circ, x, segs, 0) - ref) > 1e-6


def test_p8_slices_add_up_c1():
    lat, circ, _bs, _ = synth.config("c1")
    x = synth.random_bitstrings(lat.n, 3, 77)[2]
    ref = oracle.amplitudes_sv(lat.n, circ, [x])[0]
    cnt = oracle.segment_counts(lat.n, circ)
    segs = [(5, 1), (6, 1), (9, 2), (10, 1)]
    assert all(1 <= o < cnt[q] for q, o in segs)
    total = sum(oracle.sliced_value(lat.n, circ, x, segs, s) for s in range(16))
    assert abs(total - ref) < 1e-13


def test_sliced_value_single_slice_brute_force():
    # A slice fixes segment bits: the path sum restricted to those bit values.
    lat = synth.grid(2, 3)
    circ = synth.random_circuit(lat, 4, 12)
    x = synth.random_bitstrings(lat.n, 1, 13)[0]
    cnt = oracle.segment_counts(lat.n, circ)
    segs = [(q, 1) for q in range(lat.n) if cnt[q] >= 2][:2]
    # Restrict by inserting projectors: fixing segment (q, o) to bit v equals
    # the amplitude of the circuit with |v><v| inserted on q right after its
    # o-th non-diagonal gate.  Do it on the state vector by hand.
    for s in range(4):
        psi = np.zeros(1 << lat.n, dtype=np.complex128)
        psi[0] = 1
        seen = [0] * lat.n
        fix = {seg: (s >> j) & 1 for j, seg in enumerate(segs)}
        n = lat.n
        for k, a, b, _ in circ:
            vec = psi.reshape([2] * n)
            if k == GATE_CZ:
                idx = [slice(None)] * n
                idx[a] = 1
                idx[b] = 1
                vec[tuple(idx)] *= -1
            else:
                U = oracle.gate_matrix(k)
                vec = np.moveaxis(np.tensordot(U, vec, axes=([1], [a])), 0, a)
                if k != GATE_T:
                    seen[a] += 1
                    if (a, seen[a]) in fix:
                        keep = fix[(a, seen[a])]
                        idx = [slice(None)] * n
                        idx[a] = 1 - keep
                        vec = vec.copy()
                        vec[tuple(idx)] = 0
            psi = np.ascontiguousarray(vec).reshape(-1)
        ref = psi[oracle.index_of(x)]
        assert abs(oracle.sliced_value(lat.n, circ, x, segs, s) - ref) < 1e-14


@pytest.mark.parametrize("seed", [3, 4])
def test_p9_two_orders_agree(seed):
    lat = synth.grid(2, 3)
    circ = synth.random_circuit(lat, 5, seed)
    x = synth.random_bitstrings(lat.n, 1, seed + 1)[0]
    tensors, _ = oracle.build_plain_network(lat.n, circ, x)
    a = oracle.contract_network(tensors, "greedy")
    b = oracle.contract_network(tensors, "sweep")
    assert abs(a - b) < 1e-13


# ----------------------------------------------------------- Porter-Thomas
def _pt_stats(p_scaled):
    m1 = p_scaled.mean()
    m2 = (p_scaled ** 2).mean()
    srt = np.sort(p_scaled)
    ecdf = np.arange(1, len(srt) + 1) / len(srt)
    ks = np.max(np.abs(ecdf - (1 - np.exp(-srt))))
    return m1, m2, ks


@pytest.mark.slow
def test_p13_porter_thomas_at_depth():
    # The paper's figure: N p is close to Exp(1) (Porter-Thomas) for random
    # circuits at depth.  On the 5x5 lattice the generator reaches it by
    # depth 24 (second moment 2N/(N+1) ~ 2).
    lat = synth.grid(5, 5)
    circ = synth.random_circuit(lat, 24, 201)
    psi = oracle.statevector(lat.n, circ)
    m1, m2, ks = _pt_stats(np.abs(psi) ** 2 * (1 << lat.n))
    assert abs(m1 - 1) < 1e-10
    assert 1.9 <= m2 <= 2.1, m2
    assert ks <= 0.01, ks


def test_p13_porter_thomas_20q_deep():
    lat = synth.grid(4, 5)
    circ = synth.random_circuit(lat, 40, 3)
    m1, m2, ks = _pt_stats(np.abs(oracle.statevector(lat.n, circ)) ** 2 * (1 << lat.n))
    assert abs(m1 - 1) < 1e-10
    assert 1.9 <= m2 <= 2.1, m2
    assert ks <= 0.01, ks


def test_p13_c2_depth16_not_yet_porter_thomas():
    # At depth 16 the 5x5 circuit is close to, but not at, Porter-Thomas: only
    # the identity mean(N p) = 1 is exact there.
    lat, circ, _bs, _ = synth.config("c2")
    m1, m2, _ks = _pt_stats(np.abs(oracle.statevector(lat.n, circ)) ** 2 * (1 << lat.n))
    assert abs(m1 - 1) < 1e-10
    assert 2.0 < m2 < 2.5


def test_p13_porter_thomas_c1_mean_only():
    lat, circ, _bs, _ = synth.config("c1")
    psi = oracle.statevector(lat.n, circ)
    m1, _m2, _ks = _pt_stats(np.abs(psi) ** 2 * (1 << lat.n))
    assert abs(m1 - 1) < 1e-10
