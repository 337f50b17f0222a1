"""Open output qubits on the GPU: one contraction yields the 2^m amplitudes
of the bitstrings that differ only in the m open qubits (qc_plan_build_open),
checked against the FP64 state vector (O1) under the amplitude rule of
tests/gpu_util.check_amplitudes, and per slice against the CPU interpreter
of the same lowered program."""

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import check_amplitudes, say
from tests.plan_interp import sliced_amplitudes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1907_11217_amd import qcsim  # noqa: E402

TOL = {"c64": 1e-5, "split_fp16": 1e-4, "split_bf16": 1e-3}


def _sv_blocks(psi, xs, open_qubits):
    oq = sorted(open_qubits)
    m = len(oq)
    out = np.zeros((len(xs), 1 << m), dtype=np.complex128)
    for i, x in enumerate(xs):
        for o in range(1 << m):
            y = np.array(x, dtype=np.uint8).copy()
            for j, q in enumerate(oq):
                y[q] = (o >> (m - 1 - j)) & 1
            out[i, o] = psi[oracle.index_of(y)]
    return out


def _contract(plan, xs, s0, s1, prec="c64", chunk=None, per_slice=False):
    n_bs, A = len(xs), plan.n_amp
    chunk = chunk or min(s1 - s0, 1 << 12)
    ws = torch.empty(qcsim.qc_workspace_bytes(plan, chunk, n_bs, prec), dtype=torch.uint8, device="cuda")
    out = torch.zeros(n_bs, A, 2, dtype=torch.float64, device="cuda")
    ps = torch.zeros(s1 - s0, n_bs, A, 2, dtype=torch.float64, device="cuda") if per_slice else None
    qcsim.qc_contract_slices(plan, s0, s1, xs, prec, ws, out, ps)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    amps = o[..., 0] + 1j * o[..., 1]
    if per_slice:
        p = ps.cpu().numpy()
        return amps, p[..., 0] + 1j * p[..., 1]
    return amps


@pytest.mark.parametrize("prec", ["c64", "split_fp16", "split_bf16"])
def test_c2_open_six_qubits(prec):
    # 5x5 depth 1+16+1, 2^6 slices, six open qubits, four bitstrings:
    # 256 amplitudes against the state vector.
    lat, circ, bs, _ = synth.config("c2")
    oq = [0, 6, 12, 18, 20, 24]
    plan = qcsim.qc_plan_build(lat.n, circ, None, log2_slices=6, greedy_trials=4, seed=1, open_qubits=oq)
    xs = bs[:4]
    say(f"open outputs c2 6 qubits {prec}")
    got = _contract(plan, xs, 0, 64, prec)
    ref = _sv_blocks(oracle.statevector(lat.n, circ), xs, oq)
    info = check_amplitudes(got.reshape(-1), ref.reshape(-1), lat.n, TOL[prec])
    say(f"  {info}")


def test_all_outputs_open_state_vector_and_norm():
    # Every output of the 4x4 depth 1+10+1 circuit open: one sliced
    # contraction gives all 2^16 amplitudes; they must be the state vector and
    # their squares must sum to one (unitarity on the GPU).
    lat, circ, _bs, _ = synth.config("c1")
    plan = qcsim.qc_plan_build(lat.n, circ, None, log2_slices=3, greedy_trials=4, seed=1,
                               open_qubits=list(range(lat.n)))
    say("open outputs: all 16 qubits of the 4x4 workload")
    got = _contract(plan, np.zeros((1, lat.n), np.uint8), 0, 8)[0]
    psi = oracle.statevector(lat.n, circ)
    check_amplitudes(got, psi, lat.n, TOL["c64"])
    assert abs(np.sum(np.abs(got) ** 2) - 1.0) <= 1e-5


def test_open_per_slice_values_and_ranges_compose():
    # Per-slice values (layout [slice][bitstring][open]) against the CPU
    # interpreter of the same program, and two ranges adding up to the whole.
    lat, circ, _bs, _ = synth.config("c1")
    oq = [1, 5, 10, 14]
    plan = qcsim.qc_plan_build(lat.n, circ, None, log2_slices=4, greedy_trials=2, seed=3, open_qubits=oq)
    xs = synth.random_bitstrings(lat.n, 3, 77)
    say("open outputs: per-slice values, 4x4, 4 open qubits, 3 bitstrings")
    tot, per = _contract(plan, xs, 0, 16, per_slice=True, chunk=4)
    desc = qcsim.qc_plan_describe(plan, 0, 2)
    ref_tot, ref_per = sliced_amplitudes(desc, xs, 16)
    scale = np.sqrt(np.mean(np.abs(ref_per) ** 2))
    assert np.abs(per - ref_per).max() <= 1e-5 * scale
    assert np.abs(tot - ref_tot).max() <= 1e-5 * np.sqrt(np.mean(np.abs(ref_tot) ** 2))
    a = _contract(plan, xs, 0, 5)
    b = _contract(plan, xs, 5, 16)
    assert np.abs(a + b - tot).max() <= 1e-6 * np.abs(tot).max()


def test_open_amplitude_call():
    lat, circ, bs, _ = synth.config("c1")
    oq = [2, 9]
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=2, greedy_trials=2, seed=1, open_qubits=oq)
    say("open outputs: qc_amplitude, 2 open qubits")
    got = qcsim.qc_amplitude(plan, bs[0])
    ref = _sv_blocks(oracle.statevector(lat.n, circ), bs[:1], oq)[0]
    assert got.shape == (4,)
    assert np.abs(got - ref).max() <= 1e-5 * np.sqrt(np.mean(np.abs(ref) ** 2))


def test_open_plan_rejected_by_batch():
    lat, circ, bs, _ = synth.config("c1")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], open_qubits=[3])
    batch = qcsim.Batch([(plan, bs[0])])
    with pytest.raises(qcsim.QcError) as e:
        qcsim.qc_batch_workspace_bytes(batch)
    assert "open output" in str(e.value)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    out = torch.zeros(1, 2, dtype=torch.float64, device="cuda")
    tdone = torch.zeros(2, dtype=torch.int64, device="cuda")
    with pytest.raises(qcsim.QcError) as e:
        qcsim.qc_contract_batch(batch, "c64", ws, out, tdone)
    assert e.value.status == 5


def test_diamond70_open_outputs_vs_o4():
    # The 70-qubit depth 1+32+1 circuit with its last 12 outputs open (2^20
    # slices, cap 2^30): the per-slice values of one 16-slice chunk, complex
    # FP32 and split FP16, against O4 (the oracle's contraction of the
    # circuit's network along the plan's tree, the open qubits fixed to the
    # entry's bits) on the three largest entries and one drawn entry of the
    # chunk's first nonzero slice.
    lat, circ, bs, spec = synth.config("c4")
    oq = list(range(lat.n - 12, lat.n))
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=20, log2_max_entries=30, greedy_trials=64, seed=1,
                               open_qubits=oq)
    k = qcsim.qc_plan_info(plan)["log2_slices"]
    # Most slices of this plan are exactly zero: chunks around slices drawn
    # from the seed + 2 stream are tried in order until one holds a nonzero
    # slice.
    vals = {}
    for s0 in (int(s) for s in synth.random_slices(k, 64, spec["seed"] + 2)):
        c0 = s0 - s0 % 16
        say(f"70-qubit, 12 open outputs, slices [{c0}, {c0 + 16}) c64")
        _, vals["c64"] = _contract(plan, bs[:1], c0, c0 + 16, "c64", chunk=16, per_slice=True)
        v = vals["c64"][:, 0]
        nz = [j for j in range(16) if np.abs(v[j]).max() > 0]
        if nz:
            break
    assert nz, "every drawn chunk is zero"
    say(f"70-qubit, 12 open outputs, slices [{c0}, {c0 + 16}) split_fp16")
    _, vals["split_fp16"] = _contract(plan, bs[:1], c0, c0 + 16, "split_fp16", chunk=16, per_slice=True)
    j = nz[0]
    picks = list(np.argsort(-np.abs(v[j]))[:3]) + [int(synth.random_slices(12, 1, 7)[0])]
    tree = qcsim.qc_plan_export_tree(plan)
    segs = qcsim.qc_plan_sliced_segments(plan)
    ref = []
    for o in picks:
        y = bs[0].copy()
        for i, q in enumerate(oq):
            y[q] = (int(o) >> (11 - i)) & 1
        ref.append(oracle.hyper_value(lat.n, circ, y, segs, c0 + j, tree))
    ref = np.array(ref)
    rms = np.sqrt(np.mean(np.abs(v[j]) ** 2))
    for prec, tol in (("c64", 1e-5), ("split_fp16", 1e-4)):
        got = vals[prec][j, 0][picks]
        err = np.abs(got - ref) / np.maximum(np.abs(ref), rms)
        say(f"  {prec}: max err {err.max():.2e}")
        assert (err <= tol).all(), (prec, got, ref)
