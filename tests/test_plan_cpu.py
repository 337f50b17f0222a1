"""Planner and lowering on the CPU: the library's exported program, run by the
test-only interpreter (tests/plan_interp.py), against the FP64 oracle; slice
enumeration; gate table; argument errors; exported symbols."""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth
from paper_1907_11217_amd import qcsim
from tests.plan_interp import check_liveness, run_program, sliced_amplitudes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _plan(key_or_lat, circ=None, **kw):
    if isinstance(key_or_lat, str):
        lat, circ, bs, spec = synth.config(key_or_lat)
        return lat, circ, bs, qcsim.qc_plan_build(lat.n, circ, bs[0], **kw)
    lat = key_or_lat
    return lat, circ, None, qcsim.qc_plan_build(lat.n, circ, None, **kw)


def test_library_exports_every_declared_symbol():
    declared = set()
    for h in ("qcsim.h", "qcsim_kernels.h"):  # every declared entry point
        hdr = open(os.path.join(ROOT, "include", h)).read()
        declared |= set(re.findall(r"\b(qc_[a-z_]+)\s*\(", hdr))
    lib = qcsim.load()
    missing = [s for s in sorted(declared) if not hasattr(lib, s)]
    assert not missing, missing
    assert declared == set(qcsim.EXPORTED)


def test_gemm_kparts_rule():
    # Large-tile shapes with fewer than 1024 tiles of 128x128 are split over
    # k into the smallest power of two reaching 1024 tiles, each part keeping
    # at least 256 of k, at most 64 parts.
    assert qcsim.qc_gemm_kparts(8, 128, 2048, 16384) == 8
    assert qcsim.qc_gemm_kparts(2, 128, 2048, 8192) == 32
    assert qcsim.qc_gemm_kparts(4, 256, 2048, 1024) == 4
    assert qcsim.qc_gemm_kparts(4, 1024, 4096, 1024) == 1
    assert qcsim.qc_gemm_kparts(1, 128, 128, 1 << 20) == 64
    assert qcsim.qc_gemm_kparts(1, 128, 128, 384) == 1
    assert qcsim.qc_gemm_kparts(1, 128, 128, 768) == 2
    # Small output tiles (m n <= 256) with k >= 1024 (the dot-tile form): the
    # smallest power of two p <= 1024 with nb p >= 1024, each part at least
    # 256 of k.
    assert qcsim.qc_gemm_kparts(1, 1, 1, 1 << 21) == 1024
    assert qcsim.qc_gemm_kparts(4, 8, 8, 16384) == 64
    assert qcsim.qc_gemm_kparts(1, 1, 1, 4096) == 16
    assert qcsim.qc_gemm_kparts(256, 16, 16, 16384) == 4
    assert qcsim.qc_gemm_kparts(2, 16, 16, 512) == 1
    # Other few-output shapes with a long k (the dot form): 1024 (output,
    # part) pairs, each part at least 4096 of k.
    assert qcsim.qc_gemm_kparts(1, 16, 32, 1 << 16) == 2
    assert qcsim.qc_gemm_kparts(2, 16, 64, 1 << 14) == 1
    # Shapes of the 32- and 64-wide MFMA forms: fewer than 4096 tiles of
    # 32x32, parts of at least 256 k, at most 64 parts; 32-aligned shapes
    # take this rule even with few outputs.
    assert qcsim.qc_gemm_kparts(1, 96, 128, 4096) == 16
    assert qcsim.qc_gemm_kparts(1, 64, 128, 1 << 20) == 64
    assert qcsim.qc_gemm_kparts(4, 32, 256, 16384) == 64
    assert qcsim.qc_gemm_kparts(4, 64, 32768, 32) == 1
    assert qcsim.qc_gemm_kparts(64, 64, 64, 1024) == 4
    assert qcsim.qc_gemm_kparts(64, 64, 64, 256) == 1
    assert qcsim.qc_gemm_kparts(16, 64, 64, 512) == 2
    assert qcsim.qc_gemm_kparts(1, 32, 32, 16384) == 64


def test_workspace_holds_split_over_k_scratch():
    # A 2-bit slicing of the 7x7 d24 circuit has a GEMM step split over k at
    # one slice in flight: the workspace grows by its scratch.
    lat, circ, bs, _ = synth.config("c3")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=2, greedy_trials=4, seed=1)
    steps = qcsim.qc_plan_export_steps(plan, 0, 0)
    need = [qcsim.qc_gemm_kparts(s["nb"], s["m"], s["n"], s["k"]) * s["nb"] * s["m"] * s["n"]
            for s in steps if s["kind"] == 1 and not s["micro"] and qcsim.qc_gemm_kparts(s["nb"], s["m"], s["n"], s["k"]) > 1]
    assert need
    desc = qcsim.qc_plan_describe(plan, 0, 0)
    ws = qcsim.qc_workspace_bytes(plan, 1, 1)
    assert ws >= (desc["tensor_elems"] + max(need)) * 8


def test_transposes_only_for_large_scattered_outputs():
    # Operands are produced in the layout their consumer reads: leaves are
    # instantiated in it, GEMM steps scatter their output into it -- except a
    # GEMM output of at least 2^20 entries whose consumer layout keeps fewer
    # than two of its natural lowest bits lowest, which is written in natural
    # order and moved by an explicit transpose.
    lat, circ, bs, _ = synth.config("c3")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=16, log2_max_entries=30, greedy_trials=8, seed=1)
    seen = 0
    for b, m in [(16, 0), (0, 0), (4, 2), (12, 0)]:
        desc = qcsim.qc_plan_describe(plan, b, m)
        T = desc["tensors"]
        produced_by = {op["c"]: op for op in desc["ops"] if op["op"] == "gemm"}
        for op in desc["ops"]:
            if op["op"] != "transpose":
                continue
            seen += 1
            nat, lay = T[op["src"]]["layout"], T[op["dst"]]["layout"]
            assert op["src"] in produced_by and sorted(nat) == sorted(lay) and len(nat) >= 20
            q = 0
            while q < len(nat) and lay[-1 - q] == nat[-1 - q]:
                q += 1
            assert q < 2
        assert any(op["op"] == "gemm" and op["c_nat"] != op["c"] for op in desc["ops"])
    assert seen > 0


def test_program_with_transposes_matches_statevector():
    # 5x5 at depth 1+28+1 with four bitstrings in flight: a program holding
    # explicit transposes, interpreted on the CPU, against the state vector.
    lat = synth.grid(5, 5)
    circ = synth.random_circuit(lat, 28, 201)
    xs = synth.random_bitstrings(lat.n, 4, 206)
    plan = qcsim.qc_plan_build(lat.n, circ, None, log2_slices=0, greedy_trials=8, seed=1)
    desc = qcsim.qc_plan_describe(plan, 0, 2)
    assert any(op["op"] == "transpose" for op in desc["ops"])
    got = run_program(desc, xs)[0]
    psi = oracle.statevector(lat.n, circ)
    ref = np.array([psi[oracle.index_of(x)] for x in xs])
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_gate_matrices_match_oracle_table():
    for kind in range(5):
        assert np.abs(qcsim.qc_gate_matrix(kind) - oracle.gate_matrix(kind)).max() < 1e-15


def test_c1_unsliced_program_matches_statevector():
    lat, circ, _bs, plan = _plan("c1")
    xs = synth.random_bitstrings(lat.n, 16, 1234)
    psi = oracle.statevector(lat.n, circ)
    desc = qcsim.qc_plan_describe(plan, 0, 4)
    got = run_program(desc, xs)[0]
    ref = np.array([psi[oracle.index_of(x)] for x in xs])
    assert np.abs(got - ref).max() < 1e-14


@pytest.mark.parametrize("b,m", [(0, 0), (2, 0), (4, 3), (3, 2)])
def test_c1_sliced_programs_match(b, m):
    lat, circ, _bs, plan = _plan("c1", log2_slices=4, greedy_trials=2, seed=3)
    info = qcsim.qc_plan_info(plan)
    assert info["log2_slices"] == 4
    xs = synth.random_bitstrings(lat.n, max(1, (1 << m) - 1), 99)
    psi = oracle.statevector(lat.n, circ)
    desc = qcsim.qc_plan_describe(plan, b, m)
    total, per_slice = sliced_amplitudes(desc, xs, 16)
    ref = np.array([psi[oracle.index_of(x)] for x in xs])
    assert np.abs(total - ref).max() < 1e-14
    # Per-slice values equal the oracle's own sliced contraction.
    segs = [tuple(s) for s in qcsim.qc_plan_sliced_segments(plan)]
    for s in (0, 5, 15):
        v = oracle.sliced_value(lat.n, circ, xs[0], segs, s)
        assert abs(per_slice[s, 0] - v) < 1e-14


def test_c2_program_matches_statevector_sample():
    lat, circ, bs, plan = _plan("c2", log2_slices=6, greedy_trials=4, seed=1)
    info = qcsim.qc_plan_info(plan)
    assert info["log2_slices"] == 6 and info["n_steps"] == info["n_leaves"] - 1
    xs = bs[:3]
    desc = qcsim.qc_plan_describe(plan, 6, 2)
    total, per_slice = sliced_amplitudes(desc, xs, 64)
    ref = np.array([oracle.tn_amplitude(lat.n, circ, x) for x in xs])
    assert np.abs(total - ref).max() < 1e-14 * max(1.0, np.abs(ref).max() * 1e6)
    segs = [tuple(s) for s in qcsim.qc_plan_sliced_segments(plan)]
    v = oracle.sliced_value(lat.n, circ, xs[1], segs, 37)
    assert abs(per_slice[37, 1] - v) < 1e-15


def test_explicit_slices_and_assignment():
    lat = synth.grid(3, 3)
    circ = synth.random_circuit(lat, 6, 8)
    cnt = oracle.segment_counts(lat.n, circ)
    want = [(q, 1) for q in range(lat.n) if cnt[q] >= 2][:3]
    plan = qcsim.qc_plan_build(lat.n, circ, None, log2_slices=5, explicit_segments=want)
    segs = [tuple(int(v) for v in s) for s in qcsim.qc_plan_sliced_segments(plan)]
    assert segs[:3] == want and len(segs) == 5
    k = 5
    for s in range(1 << k):
        assert list(qcsim.qc_plan_slice_assignment(plan, s)) == [(s >> j) & 1 for j in range(k)]
    with pytest.raises(qcsim.QcError) as e:
        qcsim.qc_plan_slice_assignment(plan, 1 << k)
    assert e.value.status == 2
    x = synth.random_bitstrings(lat.n, 1, 5)
    desc = qcsim.qc_plan_describe(plan, 2, 0)
    total, per_slice = sliced_amplitudes(desc, x, 1 << k)
    assert abs(total[0] - oracle.amplitudes_sv(lat.n, circ, x)[0]) < 1e-14
    for s in (0, 7, 31):
        assert abs(per_slice[s, 0] - oracle.sliced_value(lat.n, circ, x[0], segs, s)) < 1e-15


def test_slice_assignment_random_large_k():
    lat, circ, _bs, plan = _plan("c3", log2_slices=18, log2_max_entries=30)
    k = qcsim.qc_plan_info(plan)["log2_slices"]
    assert k >= 18
    rng = np.random.default_rng(0)
    for s in rng.integers(0, 1 << k, size=200):
        assert list(qcsim.qc_plan_slice_assignment(plan, int(s))) == [(int(s) >> j) & 1 for j in range(k)]


def test_cap_is_met_and_infeasible_is_reported():
    lat, circ, _bs, plan = _plan("c3", log2_slices=-1, log2_max_entries=20, greedy_trials=2)
    info = qcsim.qc_plan_info(plan)
    assert info["log2_max_entries"] <= 20 and info["log2_slices"] >= 1
    # Any cap can be met by slicing every summed index ...
    lat2 = synth.grid(2, 2)
    circ2 = synth.random_circuit(lat2, 4, 1)
    p2 = qcsim.qc_plan_build(lat2.n, circ2, None, log2_slices=-1, log2_max_entries=0.5)
    i2 = qcsim.qc_plan_info(p2)
    assert i2["log2_max_entries"] == 0 and i2["log2_slices"] == i2["n_indices"]
    # ... but not more slice bits than there are summed indices.
    with pytest.raises(qcsim.QcError) as e:
        qcsim.qc_plan_build(lat2.n, circ2, None, log2_slices=i2["n_indices"] + 1)
    assert e.value.status == 6


def test_invalid_arguments():
    lat = synth.grid(2, 2)
    bad = np.array([[9, 0, -1, 0]], dtype=np.int32)
    with pytest.raises(qcsim.QcError) as e:
        qcsim.qc_plan_build(lat.n, bad)
    assert e.value.status == 1
    bad = np.array([[4, 0, 0, 0]], dtype=np.int32)
    with pytest.raises(qcsim.QcError):
        qcsim.qc_plan_build(lat.n, bad)
    circ = synth.random_circuit(lat, 2, 1)
    with pytest.raises(qcsim.QcError):
        qcsim.qc_plan_build(lat.n, circ, np.array([0, 2, 0, 0], dtype=np.uint8))
    with pytest.raises(qcsim.QcError):
        qcsim.qc_plan_build(lat.n, circ, explicit_segments=[(0, 0)], log2_slices=1)
    plan = qcsim.qc_plan_build(lat.n, circ)
    lib = qcsim.load()
    assert lib.qc_workspace_bytes(plan.handle, 0, 1, 0) == 0
    assert lib.qc_workspace_bytes(plan.handle, 1, 0, 0) == 0
    assert lib.qc_workspace_bytes(plan.handle, 2, 1, 0) == 0  # more slices than the plan has
    assert lib.qc_workspace_bytes(plan.handle, 1, 4, 0) > 0
    # Host-side validation of qc_contract_slices happens before any device call.
    out = ctypes.c_void_p(1)
    bs = np.zeros(lat.n, dtype=np.uint8)
    st = lib.qc_contract_slices(plan.handle, 0, 2, bs.ctypes.data, 1, 0, out, 1 << 20, None, out, None)
    assert st == 2
    st = lib.qc_contract_slices(plan.handle, 0, 1, bs.ctypes.data, 1, 7, out, 1 << 20, None, out, None)
    assert st == 1
    bs[0] = 3
    st = lib.qc_contract_slices(plan.handle, 0, 1, bs.ctypes.data, 1, 0, out, 1 << 20, None, out, None)
    assert st == 1
    assert "0 or 1" in qcsim.qc_last_error()


@pytest.mark.parametrize("key,k", [("c1", 0), ("c2", 6), ("c3", 16)])
def test_fused_lds_arena_has_no_live_overlap(key, k):
    # The fused form runs all steps of a tree level together; two tensors
    # that coexist at some level (written at or before it, last read at or
    # after it) must not share LDS slots.
    lat, circ, bs, spec = synth.config(key)
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=k, log2_max_entries=spec.get("log2_cap", 0),
                               greedy_trials=4, seed=1)
    d = qcsim.qc_plan_describe(plan, 0, 0)
    tens = d["tensors"]
    level = {l["tensor"]: 0 for l in d["leaves"]}
    death = {}
    gemms = [op for op in d["ops"] if op["op"] == "gemm"]
    for op in gemms:
        level[op["c"]] = 1 + max(level[op["a_src"]], level[op["b_src"]])
        death[op["a_src"]] = level[op["c"]]
        death[op["b_src"]] = level[op["c"]]
    n_levels = max(level.values())
    used = sorted(level)
    for t in used:
        death.setdefault(t, n_levels + 1)  # the root is read after the last level
    spans = {t: (tens[t]["lds"], tens[t]["lds"] + (1 << len(tens[t]["layout"]))) for t in used}
    for t in used:
        assert 0 <= spans[t][0] and spans[t][1] <= d["lds_elems"]
    for i, t in enumerate(used):
        for u in used[i + 1:]:
            if max(level[t], level[u]) <= min(death[t], death[u]):
                assert spans[t][1] <= spans[u][0] or spans[u][1] <= spans[t][0], (t, u)


def test_idle_qubit_and_diagonal_only_wires():
    # A qubit with no gate at all: its amplitude factor is delta(x_q, 0).
    circ = np.array([[0, 0, -1, 0], [3, 0, -1, 1], [0, 0, -1, 2], [4, 0, 1, 3]], dtype=np.int32)
    plan = qcsim.qc_plan_build(3, circ)
    xs = np.array(list(np.ndindex(2, 2, 2)), dtype=np.uint8)
    desc = qcsim.qc_plan_describe(plan, 0, 3)
    got = run_program(desc, xs)[0]
    psi = oracle.statevector(3, circ)
    ref = np.array([psi[oracle.index_of(x)] for x in xs])
    assert np.abs(got - ref).max() < 1e-15


def test_export_steps_matches_description():
    lat, circ, bs, plan = _plan("c2", log2_slices=6, greedy_trials=2, seed=1)
    for b, m in [(0, 0), (6, 6), (3, 2)]:
        steps = qcsim.qc_plan_export_steps(plan, b, m)
        ops = qcsim.qc_plan_describe(plan, b, m)["ops"]
        assert len(steps) == len(ops)
        for st, op in zip(steps, ops):
            if op["op"] == "gemm":
                assert st["kind"] == 1 and (st["a"], st["b"], st["c"]) == (op["a"], op["b"], op["c"])
                assert (st["nb"], st["m"], st["n"], st["k"]) == (op["nb"], op["m"], op["n"], op["k"])
                assert (st["a_km"], st["b_nk"]) == (int(op["a_km"]), int(op["b_nk"]))
                assert st["flops"] == 8.0 * op["nb"] * op["m"] * op["n"] * op["k"]
            else:
                assert st["kind"] == 0 and (st["a"], st["c"]) == (op["src"], op["dst"]) and st["b"] == -1
    with pytest.raises(qcsim.QcError):
        qcsim.qc_plan_export_steps(plan, 7, 0)


def test_fused_shape_setter_validates_and_is_described():
    # The seven work-item shapes and (0, 0) are accepted and reported by
    # qc_plan_describe; anything else is rejected and leaves the setting.
    lat = synth.grid(2, 2)
    plan = qcsim.qc_plan_build(lat.n, synth.random_circuit(lat, 2, 1), None, log2_slices=0)
    for shape in [(1, 1), (2, 1), (4, 1), (1, 2), (1, 4), (1, 8), (1, 16), (0, 0), (1, 16)]:
        qcsim.qc_plan_set_fused_shape(plan, *shape)
        assert qcsim.qc_plan_describe(plan, 0, 0)["fused_shape_set"] == list(shape)
    for bad in [(3, 1), (2, 2), (1, 32), (0, 1), (1, 0), (-1, 1), (8, 1), (2, 16)]:
        with pytest.raises(qcsim.QcError):
            qcsim.qc_plan_set_fused_shape(plan, *bad)
    assert qcsim.qc_plan_describe(plan, 0, 0)["fused_shape_set"] == [1, 16]


# ------------------------------------------------ open output qubits
def _sv_block(psi, n, x, open_qubits):
    """State-vector amplitudes of the 2^m bitstrings equal to x outside the
    open qubits; entry o sets the i-th open qubit (ascending) to bit m-1-i."""
    oq = sorted(open_qubits)
    m = len(oq)
    out = np.zeros(1 << m, dtype=np.complex128)
    for o in range(1 << m):
        y = np.array(x, dtype=np.uint8).copy()
        for i, q in enumerate(oq):
            y[q] = (o >> (m - 1 - i)) & 1
        out[o] = psi[oracle.index_of(y)]
    return out


@pytest.mark.parametrize("b,m", [(0, 0), (2, 1), (4, 2)])
def test_open_outputs_c1_match_statevector(b, m):
    # 4x4 depth 1+10+1 with three open output qubits (given unsorted) and 16
    # slices: every one of the 8 amplitudes per bitstring against the state
    # vector, the program run in one NaN-poisoned buffer in device order.
    lat, circ, _bs, _ = synth.config("c1")
    oq = [12, 3, 7]
    plan = qcsim.qc_plan_build(lat.n, circ, None, log2_slices=4, greedy_trials=2, seed=3, open_qubits=oq)
    info = qcsim.qc_plan_info(plan)
    assert info["n_open"] == 3 and info["log2_slices"] == 4 and plan.n_amp == 8
    desc = qcsim.qc_plan_describe(plan, b, m)
    assert desc["open_qubits"] == sorted(oq)
    xs = synth.random_bitstrings(lat.n, max(1, (1 << m) - 1), 41)
    total, per_slice = sliced_amplitudes(desc, xs, 16, flat=True)
    psi = oracle.statevector(lat.n, circ)
    for i, x in enumerate(xs):
        assert np.abs(total[i] - _sv_block(psi, lat.n, x, oq)).max() < 1e-14
    # The bits of the open qubits in the bitstring are ignored.
    x2 = xs[:1].copy()
    x2[0, oq] ^= 1
    t2, _ = sliced_amplitudes(desc, x2, 16)
    assert np.abs(t2[0] - total[0]).max() < 1e-15


def test_all_outputs_open_give_the_state_vector():
    # Every output open: one contraction gives all 2^9 amplitudes of a 3x3
    # depth-8 circuit, which must be the state vector (and have norm 1).
    lat = synth.grid(3, 3)
    circ = synth.random_circuit(lat, 8, 17)
    plan = qcsim.qc_plan_build(lat.n, circ, None, log2_slices=2, greedy_trials=2, seed=1,
                               open_qubits=list(range(lat.n)))
    desc = qcsim.qc_plan_describe(plan, 1, 0)
    total, _ = sliced_amplitudes(desc, np.zeros((1, lat.n), np.uint8), 4, flat=True)
    psi = oracle.statevector(lat.n, circ)
    assert np.abs(total[0] - psi).max() < 1e-14
    assert abs(np.sum(np.abs(total[0]) ** 2) - 1.0) < 1e-12


def test_open_outputs_c2_program():
    # 5x5 depth 1+16+1, six open qubits, 2^6 slices: 64 amplitudes per
    # bitstring from one sliced contraction, against the state vector.
    lat, circ, bs, _ = synth.config("c2")
    oq = [0, 6, 12, 18, 20, 24]
    plan = qcsim.qc_plan_build(lat.n, circ, None, log2_slices=6, greedy_trials=4, seed=1, open_qubits=oq)
    desc = qcsim.qc_plan_describe(plan, 6, 1)
    total, _ = sliced_amplitudes(desc, bs[:2], 64, flat=True)
    psi = oracle.statevector(lat.n, circ)
    for i in range(2):
        ref = _sv_block(psi, lat.n, bs[i], oq)
        assert np.abs(total[i] - ref).max() < 1e-13 * np.abs(ref).max()
    check_liveness(desc)


def test_open_output_arguments_rejected():
    lat, circ, _bs, _ = synth.config("c1")
    for bad in ([3, 3], [16], [-1], list(range(16)) + [0]):
        with pytest.raises(qcsim.QcError) as e:
            qcsim.qc_plan_build(lat.n, circ, None, open_qubits=bad)
        assert e.value.status == 1, bad
    big = synth.grid(5, 5)
    c2 = synth.random_circuit(big, 4, 3)
    with pytest.raises(qcsim.QcError) as e:
        qcsim.qc_plan_build(big.n, c2, None, open_qubits=list(range(21)))
    assert e.value.status == 1


# ------------------------------------------------ buffer offsets (aliasing)
@pytest.mark.parametrize("key,b,m", [("c1", 0, 4), ("c2", 6, 2), ("c2", 3, 0)])
def test_flat_buffer_programs(key, b, m):
    # The programs run in one buffer at the offsets the device uses, in the
    # device's order, give the oracle's values (an aliasing mistake would
    # change them or leave NaN).
    lat, circ, bs, plan = _plan(key, log2_slices=4 if key == "c1" else 6, greedy_trials=4, seed=1)
    desc = qcsim.qc_plan_describe(plan, b, m)
    check_liveness(desc)
    xs = synth.random_bitstrings(lat.n, max(1, (1 << m) - 1), 7)
    n = 1 << qcsim.qc_plan_info(plan)["log2_slices"]
    total, _ = sliced_amplitudes(desc, xs, n, flat=True)
    psi = oracle.statevector(lat.n, circ)
    ref = np.array([psi[oracle.index_of(x)] for x in xs])
    assert np.abs(total - ref).max() < 1e-13 * np.abs(ref).max()


def test_flat_buffer_program_with_transposes():
    lat = synth.grid(5, 5)
    circ = synth.random_circuit(lat, 28, 201)
    xs = synth.random_bitstrings(lat.n, 4, 206)
    plan = qcsim.qc_plan_build(lat.n, circ, None, log2_slices=0, greedy_trials=8, seed=1)
    desc = qcsim.qc_plan_describe(plan, 0, 2)
    assert any(op["op"] == "transpose" for op in desc["ops"])
    check_liveness(desc)
    got = run_program(desc, xs, flat=True)[0]
    psi = oracle.statevector(lat.n, circ)
    ref = np.array([psi[oracle.index_of(x)] for x in xs])
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_diamond70_programs_liveness_and_sampled_slices():
    # The measured 70-qubit depth 1+32+1 plan (2^20 slices, cap 2^30): its
    # 64-slice program's buffer offsets checked statically in device order
    # (every step and kept transpose).  On the same lattice at depth 1+24+1
    # (per-slice tensors small enough for the CPU, 2^10 slices of at most 2^20
    # entries): eight slices of the 4-slice program run in one NaN-poisoned
    # buffer against O4, the oracle's own contraction of the circuit's network
    # along the plan's tree.  Some slices are exact zeros that both sides
    # reach only up to FP64 rounding of the leaf values, hence the rule
    # |v - v_ref| <= tol max(|v_ref|, rms) of the GPU slice tests.
    lat, circ, bs, spec = synth.config("c4")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=spec["log2_slices"],
                               log2_max_entries=spec["log2_cap"], greedy_trials=spec["trials"],
                               seed=spec["plan_seed"])
    desc = qcsim.qc_plan_describe(plan, 6, 0)
    assert check_liveness(desc) > 20
    assert any(op["op"] == "transpose" for op in desc["ops"])
    circ24 = synth.random_circuit(lat, 24, spec["seed"])
    small = qcsim.qc_plan_build(lat.n, circ24, bs[0], log2_slices=10, log2_max_entries=20, greedy_trials=8, seed=2)
    k = qcsim.qc_plan_info(small)["log2_slices"]
    d2 = qcsim.qc_plan_describe(small, 2, 0)
    check_liveness(d2)
    tree = qcsim.qc_plan_export_tree(small)
    segs = qcsim.qc_plan_sliced_segments(small)
    got, ref = [], []
    for s in (int(v) for v in synth.random_slices(k, 8, spec["seed"] + 2)):
        got.append(run_program(d2, bs[:1], s & ~3, check_einsum=False, flat=True)[s & 3, 0])
        ref.append(oracle.hyper_value(lat.n, circ24, bs[0], segs, s, tree))
    got, ref = np.array(got), np.array(ref)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    assert (np.abs(ref) > 1e-6 * rms).sum() >= 2
    assert (np.abs(got - ref) <= 1e-12 * np.maximum(np.abs(ref), rms)).all(), (got, ref)


def test_quick_search_plan_matches_statevector():
    # The quick search (greedy restarts and slicing, no reconfiguration)
    # gives another valid tree: same amplitudes.
    lat, circ, bs, _ = synth.config("c2")
    full = qcsim.qc_plan_build(lat.n, circ, None, log2_slices=6, greedy_trials=4, seed=1)
    quick = qcsim.qc_plan_build(lat.n, circ, None, log2_slices=6, greedy_trials=4, seed=1, quick=True)
    assert qcsim.qc_plan_info(quick)["log2_slices"] == 6
    assert qcsim.qc_plan_info(quick)["plan_seconds"] < qcsim.qc_plan_info(full)["plan_seconds"]
    desc = qcsim.qc_plan_describe(quick, 6, 1)
    check_liveness(desc)
    total, _ = sliced_amplitudes(desc, bs[:2], 64, flat=True)
    psi = oracle.statevector(lat.n, circ)
    ref = np.array([psi[oracle.index_of(x)] for x in bs[:2]])
    assert np.abs(total - ref).max() < 1e-13 * np.abs(ref).max()


def test_diamond72_degree_one_qubits_program():
    # The 72-qubit lattice with two degree-1 qubits (the 70-qubit lattice plus
    # two qubits whose only neighbour is on it): 125 couplers, qubits 0 and 71
    # with one coupler each.  At depth 1+24+1 (2^12 slices of at most 2^20
    # entries) eight slices of the 4-slice program, run in one NaN-poisoned
    # buffer, against O4 along the plan's tree.
    lat = synth.diamond72()
    pairs = {c for p in synth.cz_patterns(lat) for c in p}
    assert lat.n == 72 and len(pairs) == 125
    deg = np.zeros(lat.n, int)
    for a, b in pairs:
        deg[a] += 1
        deg[b] += 1
    assert sorted(np.flatnonzero(deg == 1).tolist()) == [0, 71] and deg.min() == 1
    circ = synth.random_circuit(lat, 24, 411)
    bs = synth.random_bitstrings(lat.n, 1, 412)
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=10, log2_max_entries=20, greedy_trials=8, seed=2)
    k = qcsim.qc_plan_info(plan)["log2_slices"]
    desc = qcsim.qc_plan_describe(plan, 2, 0)
    check_liveness(desc)
    tree = qcsim.qc_plan_export_tree(plan)
    segs = qcsim.qc_plan_sliced_segments(plan)
    got, ref = [], []
    for s in (int(v) for v in synth.random_slices(k, 8, 413)):
        got.append(run_program(desc, bs[:1], s & ~3, check_einsum=False, flat=True)[s & 3, 0])
        ref.append(oracle.hyper_value(lat.n, circ, bs[0], segs, s, tree))
    got, ref = np.array(got), np.array(ref)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    assert (np.abs(ref) > 1e-6 * rms).sum() >= 2
    assert (np.abs(got - ref) <= 1e-12 * np.maximum(np.abs(ref), rms)).all()
