"""End-to-end parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerance for complex FP32 (QC_C64): relative error <= 1e-5 on bitstrings
with N|a|^2 >= 1e-2, plus batch 2-norm and absolute-vs-RMS bounds (see
tests/gpu_util.check_amplitudes).  Slice enumeration is checked bit-exactly
through per-slice values against the oracle's own sliced contraction."""

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import check_amplitudes, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1907_11217_amd import qcsim  # noqa: E402

TOL_C64 = 1e-5


def _contract(plan, xs, s_begin, s_end, prec="c64", ws_bytes=None, chunk=None, per_slice=False):
    n_bs = len(xs)
    if ws_bytes is None:
        chunk = chunk or min(s_end - s_begin, 1 << 12)
        ws_bytes = qcsim.qc_workspace_bytes(plan, chunk, n_bs, prec)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    out = torch.zeros(n_bs, 2, dtype=torch.float64, device="cuda")
    ps = torch.zeros(s_end - s_begin, n_bs, 2, dtype=torch.float64, device="cuda") if per_slice else None
    qcsim.qc_contract_slices(plan, s_begin, s_end, xs, prec, ws, out, ps)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    amps = o[:, 0] + 1j * o[:, 1]
    if per_slice:
        p = ps.cpu().numpy()
        return amps, p[..., 0] + 1j * p[..., 1]
    return amps


def test_p2_hadamard_layers_gpu():
    lat = synth.grid(3, 3)
    circ = synth.random_circuit(lat, 0, 1)
    xs = np.array(list(np.ndindex(*([2] * lat.n))), dtype=np.uint8)
    plan = qcsim.qc_plan_build(lat.n, circ)
    say("P2 1+0+1 3x3 all bitstrings")
    got = _contract(plan, xs, 0, 1)
    ref = np.zeros(len(xs))
    ref[0] = 1
    assert np.abs(got - ref).max() <= 1e-7


MODES = ["fused", "stepwise"]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("shape,depth,seed", [((2, 2), 8, 1), ((2, 3), 8, 2), ((3, 3), 8, 3)])
def test_p6_unitarity_all_amplitudes(shape, depth, seed, mode):
    lat = synth.grid(*shape)
    circ = synth.random_circuit(lat, depth, seed)
    xs = np.array(list(np.ndindex(*([2] * lat.n))), dtype=np.uint8)
    # As many slice bits as the simplified network has, up to 2.
    n_idx = qcsim.qc_plan_info(qcsim.qc_plan_build(lat.n, circ))["n_indices"]
    k = min(2, n_idx)
    plan = qcsim.qc_plan_build(lat.n, circ, None, log2_slices=k, greedy_trials=2)
    qcsim.qc_plan_set_exec(plan, mode)
    say(f"P6 unitarity {shape} d{depth} {mode} k={k}")
    got = _contract(plan, xs, 0, 1 << k)
    assert abs(np.sum(np.abs(got) ** 2) - 1) <= 1e-5
    psi = oracle.statevector(lat.n, circ)
    check_amplitudes(got, psi, lat.n, TOL_C64)


@pytest.mark.parametrize("mode", MODES)
def test_c1_amplitudes(mode):
    lat, circ, bs, _ = synth.config("c1")
    xs = np.concatenate([bs, synth.random_bitstrings(lat.n, 255, 1001)])
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0])
    qcsim.qc_plan_set_exec(plan, mode)
    psi = oracle.statevector(lat.n, circ)
    ref = np.array([psi[oracle.index_of(x)] for x in xs])
    say(f"c1 4x4 d10, 256 bitstrings, unsliced, {mode}")
    got = _contract(plan, xs, 0, 1)
    info = check_amplitudes(got, ref, lat.n, TOL_C64)
    print("c1", info)


def test_c1_qc_amplitude():
    lat, circ, bs, _ = synth.config("c1")
    x = synth.random_bitstrings(lat.n, 3, 555)[2]
    plan = qcsim.qc_plan_build(lat.n, circ, x, log2_slices=3)
    ref = oracle.amplitudes_sv(lat.n, circ, [x])[0]
    say("c1 qc_amplitude k=3")
    got = qcsim.qc_amplitude(plan, x)
    assert abs(got - ref) <= TOL_C64 * max(abs(ref), 2.0 ** (-lat.n / 2))


@pytest.fixture(scope="module")
def c2_setup():
    # The benchmark's plan of this workload (quick search).
    lat, circ, bs, spec = synth.config("c2")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=spec["log2_slices"], greedy_trials=spec["trials"],
                               seed=spec["plan_seed"], quick=spec["quick"])
    psi = oracle.statevector(lat.n, circ)
    ref = np.array([psi[oracle.index_of(x)] for x in bs])
    return lat, circ, bs, plan, ref


@pytest.mark.parametrize("mode", MODES)
def test_c2_amplitudes_c64(c2_setup, mode):
    lat, circ, bs, plan, ref = c2_setup
    assert qcsim.qc_plan_info(plan)["log2_slices"] == 6
    qcsim.qc_plan_set_exec(plan, mode)
    say(f"c2 5x5 d16, 64 bitstrings x 64 slices, c64, {mode}")
    got = _contract(plan, bs, 0, 64)
    info = check_amplitudes(got, ref, lat.n, TOL_C64)
    print("c2", info)


@pytest.mark.parametrize("mode", MODES)
def test_c2_per_slice_values_match_oracle(c2_setup, mode):
    lat, circ, bs, plan, _ref = c2_setup
    qcsim.qc_plan_set_exec(plan, mode)
    segs = [tuple(int(v) for v in s) for s in qcsim.qc_plan_sliced_segments(plan)]
    say(f"c2 per-slice values, {mode}")
    amps, ps = _contract(plan, bs[:8], 0, 64, per_slice=True)
    assert np.abs(ps.sum(axis=0) - amps).max() <= 1e-15 + 1e-12 * np.abs(amps).max()
    vals = np.abs(ps).ravel()
    scale = np.sqrt(np.mean(vals ** 2))
    for s, j in [(0, 0), (37, 1), (63, 7), (12, 3)]:
        v = oracle.sliced_value(lat.n, circ, bs[j], segs, s)
        assert abs(ps[s, j] - v) <= TOL_C64 * max(abs(v), scale), (s, j, ps[s, j], v)


@pytest.mark.parametrize("fb", [0, 1, 2, 3, 4, 5, 6])
def test_c2_fused_slice_bits_match_oracle(fb):
    # The fused form with 2^fb slices per work item (the program lowered with
    # fb open slice bits): amplitudes against the state vector, per-slice
    # values against the oracle's sliced contraction, ranges that cut work
    # items against whole ones.
    lat, circ, bs, spec = synth.config("c2")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=6, greedy_trials=8, seed=1)
    qcsim.qc_plan_set_exec(plan, "fused")
    qcsim.qc_plan_set_fused_slice_bits(plan, fb)
    assert qcsim.qc_plan_describe(plan, 0, 0)["fused_slice_bits"] == fb
    psi = oracle.statevector(lat.n, circ)
    ref = np.array([psi[oracle.index_of(x)] for x in bs])
    say(f"c2 fused, {1 << fb} slices per work item, 64 bitstrings")
    amps, ps = _contract(plan, bs, 0, 64, per_slice=True)
    check_amplitudes(amps, ref, lat.n, TOL_C64)
    segs = [tuple(int(v) for v in s) for s in qcsim.qc_plan_sliced_segments(plan)]
    scale = np.sqrt(np.mean(np.abs(ps) ** 2))
    for s, j in [(0, 0), (37, 1), (63, 7), (12, 3), (5, 60)]:
        v = oracle.sliced_value(lat.n, circ, bs[j], segs, s)
        assert abs(ps[s, j] - v) <= TOL_C64 * max(abs(v), scale), (s, j, ps[s, j], v)
    # [3, 45) cuts work items at both ends; its slices equal the whole run's.
    part, pps = _contract(plan, bs[:5], 3, 45, per_slice=True)
    assert np.array_equal(pps, ps[3:45, :5])


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("shape,depth,seed,k", [((4, 4), 12, 31, 2), ((4, 5), 14, 33, 3), ((5, 5), 16, 32, 4)])
def test_paper_rule_circuits_match_state_vector(shape, depth, seed, k, mode):
    # Circuits drawn with the paper's own single-qubit rule (a sqrt X or sqrt Y
    # after a CZ, a T after a sqrt X, sqrt Y or H, nothing otherwise) through
    # the same plan and entry points, with k sliced segments.
    lat = synth.grid(*shape)
    circ = synth.random_circuit(lat, depth, seed, rule="paper")
    bs = synth.random_bitstrings(lat.n, 16, seed + 1)
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=k, greedy_trials=8, seed=1)
    assert qcsim.qc_plan_info(plan)["log2_slices"] == k
    qcsim.qc_plan_set_exec(plan, mode)
    say(f"paper-rule {shape[0]}x{shape[1]} d{depth} seed {seed}, 2^{k} slices x 16 bitstrings, {mode}")
    amps = _contract(plan, bs, 0, 1 << k)
    psi = oracle.statevector(lat.n, circ)
    ref = np.array([psi[oracle.index_of(x)] for x in bs])
    check_amplitudes(amps, ref, lat.n, TOL_C64)


FUSED_SHAPES = [(1, 1), (2, 1), (4, 1), (1, 2), (1, 4), (1, 8), (1, 16)]


@pytest.mark.parametrize("fb", [0, 6])
def test_c2_every_fused_shape_matches_oracle_with_the_same_bits(c2_setup, fb):
    # Each work-item shape (items per workgroup x wavefronts per item) runs the
    # same per-item arithmetic on another schedule (sixteen wavefronts rotate
    # three register sets of prefetched items, fewer load one pass ahead), so
    # every shape that fits in LDS gives the same bits, and they match the
    # state vector and the oracle's sliced values; a shape that does not fit
    # fails with an error before any launch.
    lat, circ, bs, _plan, ref = c2_setup
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=6, greedy_trials=8, seed=1)
    qcsim.qc_plan_set_exec(plan, "fused")
    qcsim.qc_plan_set_fused_slice_bits(plan, fb)
    pair_elems = (qcsim.qc_plan_describe(plan, fb, 0)["lds_elems"] + 2) & ~1
    segs = [tuple(int(v) for v in s) for s in qcsim.qc_plan_sliced_segments(plan)]
    first = None
    for shape in FUSED_SHAPES:
        qcsim.qc_plan_set_fused_shape(plan, *shape)
        assert qcsim.qc_plan_describe(plan, fb, 0)["fused_shape_set"] == list(shape)
        if shape[0] * pair_elems * 8 > 64 * 1024:
            say(f"c2 fused, {1 << fb} slices per work item, shape {shape}: does not fit, expect an error")
            with pytest.raises(qcsim.QcError):
                _contract(plan, bs[:4], 0, 64)
            continue
        say(f"c2 fused, {1 << fb} slices per work item, shape {shape}")
        amps, ps = _contract(plan, bs, 0, 64, per_slice=True)
        if first is None:
            first = (shape, amps, ps)
            check_amplitudes(amps, ref, lat.n, TOL_C64)
            scale = np.sqrt(np.mean(np.abs(ps) ** 2))
            for s, j in [(0, 0), (63, 7), (21, 40)]:
                v = oracle.sliced_value(lat.n, circ, bs[j], segs, s)
                assert abs(ps[s, j] - v) <= TOL_C64 * max(abs(v), scale), (s, j, ps[s, j], v)
        else:
            assert np.array_equal(ps, first[2]), (shape, first[0])
            assert np.array_equal(amps, first[1]), (shape, first[0])
    assert first is not None


def test_fused_slice_bits_rejects_bad_values(c2_setup):
    _lat, _circ, _bs, plan, _ref = c2_setup
    with pytest.raises(qcsim.QcError):
        qcsim.qc_plan_set_fused_slice_bits(plan, 7)
    lat = synth.grid(2, 2)
    small = qcsim.qc_plan_build(lat.n, synth.random_circuit(lat, 2, 1), None, log2_slices=0)
    with pytest.raises(qcsim.QcError):
        qcsim.qc_plan_set_fused_slice_bits(small, 1)


@pytest.mark.parametrize("mode", MODES)
def test_ranges_compose_and_repeat(c2_setup, mode):
    # Slices are summed in aligned blocks of 64; splits at multiples of 64
    # compose bitwise, other splits to rounding.
    lat, circ, bs, _plan, ref = c2_setup
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=8, greedy_trials=2, seed=5)
    qcsim.qc_plan_set_exec(plan, mode)
    xs = bs[:16]
    ws_bytes = qcsim.qc_workspace_bytes(plan, 64, len(xs))
    say("c2 circuit, 256 slices: [0,256) vs [0,128)+[128,256) vs [0,100)+[100,256)")
    whole = _contract(plan, xs, 0, 256, ws_bytes=ws_bytes)
    again = _contract(plan, xs, 0, 256, ws_bytes=ws_bytes)
    assert np.array_equal(whole, again)  # bitwise reproducible
    # A larger workspace lowers the plan for more slices in flight: the GEMM
    # steps change shape (and small ones move into the micro-step kernel), so
    # each FP32 slice value may round differently; the FP64 sums then agree to
    # FP32 rounding of the per-slice values only.
    big = _contract(plan, xs, 0, 256)
    assert np.abs(big - whole).max() <= 1e-5 * np.abs(whole).max()
    assert np.array_equal(big, _contract(plan, xs, 0, 256))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    out = torch.zeros(len(xs), 2, dtype=torch.float64, device="cuda")
    qcsim.qc_contract_slices(plan, 0, 128, xs, "c64", ws, out)
    qcsim.qc_contract_slices(plan, 128, 256, xs, "c64", ws, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert np.array_equal(o[:, 0] + 1j * o[:, 1], whole)
    out.zero_()
    qcsim.qc_contract_slices(plan, 0, 100, xs, "c64", ws, out)
    qcsim.qc_contract_slices(plan, 100, 256, xs, "c64", ws, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert np.abs((o[:, 0] + 1j * o[:, 1]) - whole).max() <= 1e-12 * np.abs(whole).max()
    check_amplitudes(whole, ref[:16], lat.n, TOL_C64)


@pytest.mark.parametrize("mode", MODES)
def test_workspace_too_small(c2_setup, mode):
    lat, circ, bs, plan, _ref = c2_setup
    qcsim.qc_plan_set_exec(plan, mode)
    need = qcsim.qc_workspace_bytes(plan, 1, len(bs))
    ws = torch.empty(max(need // 2, 1), dtype=torch.uint8, device="cuda")
    out = torch.zeros(len(bs), 2, dtype=torch.float64, device="cuda")
    with pytest.raises(qcsim.QcError) as e:
        qcsim.qc_contract_slices(plan, 0, 64, bs, "c64", ws, out)
    assert e.value.status == 3


def test_fused_mode_rejected_when_too_large():
    lat, circ, bs, _ = synth.config("c3")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=0)
    qcsim.qc_plan_set_exec(plan, "fused")
    with pytest.raises(qcsim.QcError) as e:
        qcsim.qc_workspace_bytes(plan, 1, 1)
    assert "does not fit" in str(e.value)


@pytest.mark.parametrize("mode", MODES)
def test_device_resident_bitstrings_match_host(c2_setup, mode):
    # 37 bitstrings: the padded rows of the batch reuse the last row.
    lat, circ, bs, plan, ref = c2_setup
    qcsim.qc_plan_set_exec(plan, mode)
    xs = bs[:37]
    ws = torch.empty(qcsim.qc_workspace_bytes(plan, 64, len(xs)), dtype=torch.uint8, device="cuda")
    out_h = torch.zeros(len(xs), 2, dtype=torch.float64, device="cuda")
    out_d = torch.zeros(len(xs), 2, dtype=torch.float64, device="cuda")
    say(f"c2 device-resident bitstrings, 37 rows, {mode}")
    qcsim.qc_contract_slices(plan, 0, 64, xs, "c64", ws, out_h)
    bits_dev = torch.from_numpy(np.ascontiguousarray(xs)).cuda()
    qcsim.qc_contract_slices_dev(plan, 0, 64, bits_dev, "c64", ws, out_d)
    torch.cuda.synchronize()
    assert torch.equal(out_h, out_d)
    o = out_d.cpu().numpy()
    check_amplitudes(o[:, 0] + 1j * o[:, 1], ref[:37], lat.n, TOL_C64)


# Split precisions: relative error <= 1e-4 for split FP16; split BF16 has no
# target of its own and is held to 1e-3.  They always run stepwise, and only
# GEMM steps with m and n multiples of 32 run on a split MFMA form.
TOL_SPLIT = {"split_fp16": 1e-4, "split_bf16": 1e-3}
SPLIT_KIND = {"split_fp16": "gemm_split_fp16", "split_bf16": "gemm_split_bf16"}


def _split_eligible_flops(plan, b, m):
    steps = qcsim.qc_plan_export_steps(plan, b, m)
    gemm = [s for s in steps if s["kind"] == 1]
    total = sum(s["flops"] for s in gemm)
    elig = sum(s["flops"] for s in gemm if not s["micro"] and s["m"] % 32 == 0 and s["n"] % 32 == 0)
    return elig, total


@pytest.mark.parametrize("prec", sorted(TOL_SPLIT))
def test_c2_split_precisions_match_statevector(c2_setup, prec):
    # The 5x5 depth-16 workload in a split precision (stepwise, 2^6 slices and
    # 64 bitstrings in flight): only its GEMM steps with m and n multiples of
    # 32 run on a split MFMA form (a small share of this program's flops; the
    # rest stays complex FP32), which the profile shows; the amplitudes meet
    # the split tolerance against the 2^25 state vector.  Split MFMA parity on
    # a program dominated by split steps is the 5x5 depth-28 test below.
    lat, circ, bs, plan, ref = c2_setup
    qcsim.qc_plan_set_exec(plan, "stepwise")
    try:
        elig, total = _split_eligible_flops(plan, 6, 6)
        say(f"c2 5x5 d16, 64 bitstrings x 64 slices, stepwise {prec} (split-eligible share {elig / total:.3f})")
        qcsim.qc_profile_read(plan)
        qcsim.qc_profile_enable(plan, True)
        got = _contract(plan, bs, 0, 64, prec=prec)
        qcsim.qc_profile_enable(plan, False)
        prof = qcsim.qc_profile_read(plan)
        assert (SPLIT_KIND[prec] in prof) == (elig > 0), prof
        info = check_amplitudes(got, ref, lat.n, TOL_SPLIT[prec])
        print("c2", prec, info, {kk: v[0] for kk, v in prof.items()})
    finally:
        qcsim.qc_plan_set_exec(plan, "auto")


@pytest.fixture(scope="module")
def deep5x5():
    # 5x5 grid at depth 1+28+1 (circuit seed 201, the 5x5 workload's seed):
    # about 90% of its program's flops sit in GEMM steps that a split MFMA
    # form runs, and its 2^25-entry state vector is still at hand.
    lat = synth.grid(5, 5)
    circ = synth.random_circuit(lat, 28, 201)
    xs = synth.random_bitstrings(lat.n, 16, 205)
    plan = qcsim.qc_plan_build(lat.n, circ, xs[0], log2_slices=2, greedy_trials=8, seed=1)
    qcsim.qc_plan_set_exec(plan, "stepwise")
    psi = oracle.statevector(lat.n, circ)
    ref = np.array([psi[oracle.index_of(x)] for x in xs])
    return lat, xs, plan, ref


@pytest.mark.parametrize("prec", ["c64", "split_fp16", "split_bf16"])
def test_deep5x5_split_mfma_matches_statevector(deep5x5, prec):
    lat, xs, plan, ref = deep5x5
    elig, total = _split_eligible_flops(plan, 2, 4)
    assert elig >= 0.5 * total, (elig, total)
    say(f"5x5 d28, 16 bitstrings x 4 slices, stepwise {prec}")
    qcsim.qc_profile_read(plan)
    qcsim.qc_profile_enable(plan, True)
    got = _contract(plan, xs, 0, 4, prec=prec)
    qcsim.qc_profile_enable(plan, False)
    prof = qcsim.qc_profile_read(plan)
    gemm_flops = sum(v[2] for kk, v in prof.items())
    if prec != "c64":
        kind = SPLIT_KIND[prec]
        assert kind in prof and prof[kind][0] > 0, prof
        # Most of the work ran on the split MFMA form.
        assert prof[kind][2] >= 0.5 * gemm_flops, prof
    info = check_amplitudes(got, ref, lat.n, TOL_C64 if prec == "c64" else TOL_SPLIT[prec])
    print("5x5 d28", prec, info, {kk: v[0] for kk, v in prof.items()})


def test_split_needs_stepwise(c2_setup):
    _lat, _circ, bs, plan, _ref = c2_setup
    qcsim.qc_plan_set_exec(plan, "fused")
    try:
        with pytest.raises(qcsim.QcError) as e:
            qcsim.qc_workspace_bytes(plan, 64, len(bs), "split_fp16")
        assert "complex FP32" in str(e.value)
    finally:
        qcsim.qc_plan_set_exec(plan, "auto")


@pytest.mark.parametrize("prec", ["c64", "split_fp16"])
def test_c3_sampled_slices_match_oracle(prec):
    # 7x7 depth 24: beyond the state vector, so slice values are compared
    # with the oracle's own sliced contraction (O3, slice list of the plan read
    # as data) on slices drawn from the seed + 2 stream; each oracle slice
    # takes ~16 s on the host, so two slices.  All 2^16 slices run in one
    # call (the measured configuration), per-slice values kept.
    lat, circ, bs, spec = synth.config("c3")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=16, log2_max_entries=30, greedy_trials=8, seed=1)
    k = qcsim.qc_plan_info(plan)["log2_slices"]
    segs = [tuple(int(v) for v in s) for s in qcsim.qc_plan_sliced_segments(plan)]
    picks = [int(s) for s in synth.random_slices(k, 2, spec["seed"] + 2)]
    say(f"c3 7x7 d24 all 2^{k} slices {prec}, oracle on slices {picks}")
    amp, ps = _contract(plan, bs[:1], 0, 1 << k, prec=prec, chunk=1 << k, per_slice=True)
    assert abs(ps[:, 0].sum() - amp[0]) <= 1e-12 * np.abs(ps).sum()
    scale = np.sqrt(np.mean(np.abs(ps[:, 0]) ** 2))
    tol = TOL_C64 if prec == "c64" else TOL_SPLIT[prec]
    for s in picks:
        v = oracle.sliced_value(lat.n, circ, bs[0], segs, s)
        assert abs(ps[s, 0] - v) <= tol * max(abs(v), scale), (s, ps[s, 0], v)


@pytest.mark.parametrize("prec", ["c64", "split_bf16"])
def test_c3_split_over_k_program_matches_o4(prec):
    # A coarse slicing of the 7x7 d24 circuit (the fewest slice bits, from 1
    # to 4, whose program holds a GEMM step split over k), one slice in
    # flight: every slice value against O4 along the same plan's tree, and
    # their sum against the sum of all 2^16 slices of the measured slicing.
    lat, circ, bs, _ = synth.config("c3")
    coarse = None
    for kc in (1, 2, 3, 4):
        p = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=kc, greedy_trials=4, seed=1)
        steps = qcsim.qc_plan_export_steps(p, 0, 0)
        if any(s["kind"] == 1 and not s["micro"] and qcsim.qc_gemm_kparts(s["nb"], s["m"], s["n"], s["k"]) > 1
               for s in steps):
            coarse = p
            break
    assert coarse is not None, "no coarse slicing with a step split over k"
    kc = qcsim.qc_plan_info(coarse)["log2_slices"]
    fine = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=16, log2_max_entries=30, greedy_trials=8, seed=1)
    say(f"c3 7x7 d24, {kc}-bit slicing one slice in flight ({prec}) vs O4 and the 16-bit slicing")
    a, ps_a = _contract(coarse, bs[:1], 0, 1 << kc, prec=prec, ws_bytes=qcsim.qc_workspace_bytes(coarse, 1, 1, prec),
                        per_slice=True)
    tree = qcsim.qc_plan_export_tree(coarse)
    segs = qcsim.qc_plan_sliced_segments(coarse)
    ref = np.array([oracle.hyper_value(lat.n, circ, bs[0], segs, s, tree) for s in range(1 << kc)])
    tol = TOL_C64 if prec == "c64" else TOL_SPLIT[prec]
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    assert (np.abs(ps_a[:, 0] - ref) <= tol * np.maximum(np.abs(ref), rms)).all(), (ps_a[:, 0], ref)
    b, ps_b = _contract(fine, bs[:1], 0, 1 << 16, prec="c64", chunk=1 << 16, per_slice=True)
    rms_b = np.sqrt(np.mean(np.abs(ps_b) ** 2))
    bound = tol * (2 * rms) + TOL_C64 * 256 * rms_b
    say(f"  |a - b| = {abs(a[0] - b[0]):.3e}, |b| = {abs(b[0]):.3e}, tol {bound:.3e}")
    assert abs(a[0] - b[0]) <= bound


def _butterfly_blocks(vals, lo, hi, base):
    # The reduction's arithmetic on the host: each aligned block of 64
    # slices summed by the xor butterfly (offsets 32, 16, ..., 1; lane 0's
    # value), blocks added in increasing order.
    acc = 0.0 + 0.0j
    first = (lo - base) // 64 * 64 + base
    for b0 in range(first, hi, 64):
        lane = np.zeros(64, dtype=np.complex128)
        for j in range(64):
            s = b0 + j
            if lo <= s < hi:
                lane[j] = vals[s - lo]
        for off in (32, 16, 8, 4, 2, 1):
            lane = lane + lane[np.arange(64) ^ off]
        acc += lane[0]
    return acc


@pytest.mark.parametrize("s0,s1,chunk", [(100, 9000, 1 << 13), (0, 64, 64), (3, 1000, 1 << 10)])
def test_reduction_order_is_the_fixed_butterfly(s0, s1, chunk):
    # The FP64 sum of slice values, bit for bit as the documented order (with
    # more than 64 blocks per super-chunk the block sums and their ordered
    # addition are separate launches).
    lat, circ, bs, _ = synth.config("c3")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=16, log2_max_entries=30, greedy_trials=8, seed=1)
    say(f"c3 slices [{s0}, {s1}), chunk {chunk}: reduction order")
    amp, ps = _contract(plan, bs[:1], s0, s1, chunk=chunk, per_slice=True)
    ref = _butterfly_blocks(ps[:, 0], s0, s1, s0 // chunk * chunk)
    assert amp[0] == ref, (amp[0], ref)


def test_fused_block_sums_compose_across_super_chunks():
    # 64-slice fused work items add their block sums to the output in the
    # launch; a range of several blocks runs one launch per 64-slice
    # super-chunk, so the blocks still arrive in increasing order: the result
    # equals the two-launch reduction's bits (b = 0 with the same blocks is a
    # different program, so that comparison is to rounding; the per-slice
    # values of b = 6 are checked through the butterfly re-computation).
    lat, circ, bs, _ = synth.config("c2")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=8, greedy_trials=2, seed=5)
    qcsim.qc_plan_set_exec(plan, "fused")
    qcsim.qc_plan_set_fused_slice_bits(plan, 6)
    xs = bs[:8]
    ws_bytes = qcsim.qc_workspace_bytes(plan, 64, len(xs))
    say("c2 circuit, 256 slices, 64-slice fused work items, block sums in the launch")
    whole, ps = _contract(plan, xs, 0, 256, ws_bytes=ws_bytes, per_slice=True)
    for j in range(len(xs)):
        assert whole[j] == _butterfly_blocks(ps[:, j], 0, 256, 0)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    out = torch.zeros(len(xs), 2, dtype=torch.float64, device="cuda")
    qcsim.qc_contract_slices(plan, 0, 128, xs, "c64", ws, out)
    qcsim.qc_contract_slices(plan, 128, 256, xs, "c64", ws, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert np.array_equal(o[:, 0] + 1j * o[:, 1], whole)
    plan0 = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=8, greedy_trials=2, seed=5)
    qcsim.qc_plan_set_exec(plan0, "fused")
    qcsim.qc_plan_set_fused_slice_bits(plan0, 0)
    b0 = _contract(plan0, xs, 0, 256, ws_bytes=qcsim.qc_workspace_bytes(plan0, 64, len(xs)))
    assert np.abs(b0 - whole).max() <= TOL_C64 * np.abs(whole).max()


def test_fused_program_with_many_levels():
    # A 1x220 chain at depth 1+10+1: the plan's tree is 69 levels deep, so
    # the fused kernel reads its level starts from memory (programs of 64
    # levels or more) instead of from lanes.  32 bitstrings in the fused
    # form against O4 (the oracle's network along the plan's tree).
    lat = synth.grid(1, 220)
    circ = synth.random_circuit(lat, 10, 5)
    plan = qcsim.qc_plan_build(lat.n, circ, None, log2_slices=2, greedy_trials=1, seed=1)
    desc = qcsim.qc_plan_describe(plan, 0, 0)
    lvl, deepest = {leaf["tensor"]: 0 for leaf in desc["leaves"]}, 0
    for op in desc["ops"]:
        if op["op"] == "gemm":
            lvl[op["c"]] = 1 + max(lvl[op["a_src"]], lvl[op["b_src"]])
            deepest = max(deepest, lvl[op["c"]])
    assert deepest >= 64
    qcsim.qc_plan_set_exec(plan, "fused")
    xs = synth.random_bitstrings(lat.n, 32, 6)
    say(f"fused program with {deepest} levels, 1x220 d10, 32 bitstrings")
    got = _contract(plan, xs, 0, 4)
    tree = qcsim.qc_plan_export_tree(plan)
    segs = qcsim.qc_plan_sliced_segments(plan)
    ref = np.array([sum(oracle.hyper_value(lat.n, circ, x, segs, s, tree) for s in range(4)) for x in xs])
    assert (np.abs(ref) > 0).sum() >= 8
    check_amplitudes(got, ref, lat.n, TOL_C64)
