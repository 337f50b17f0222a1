"""Parity of the HIP path with O4 where the state vector cannot reach: the
70-qubit diamond at depth 1+32+1, the 7x7 grid at depth 1+24+1 and the 6x6 /
7x7 requests of the uneven batch.

O4 (oracle/hyper.py) contracts the circuit's own hypergraph network in
complex128 along the plan's tree, read through qc_plan_export_tree as data
(any valid tree gives the same value), so each sampled slice value of the
GPU is compared with an FP64 value computed by code that shares nothing with
the library.  The paper's statement that subtask results add up to the
amplitude is what makes per-slice parity a check of the amplitude.

Slices are drawn from the workload's seed + 2 stream.  The per-slice rule:
|v - v_ref| <= tol * max(|v_ref|, rms), rms the RMS of the sampled reference
values (some slices are exactly zero); tol = 1e-5 complex FP32, 1e-4 split
FP16, 1e-3 split BF16 (reported, no target of its own).
"""

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1907_11217_amd import qcsim  # noqa: E402

TOL = {"c64": 1e-5, "split_fp16": 1e-4, "split_bf16": 1e-3}


def _plan(key, **over):
    lat, circ, bs, spec = synth.config(key)
    kw = dict(log2_slices=spec["log2_slices"], log2_max_entries=spec.get("log2_cap", 0),
              greedy_trials=spec["trials"], seed=spec["plan_seed"])
    kw.update(over)
    return lat, circ, bs, spec, qcsim.qc_plan_build(lat.n, circ, bs[0], **kw)


def _slice_values(plan, x, s0, s1, prec, chunk):
    ws = torch.empty(qcsim.qc_workspace_bytes(plan, chunk, 1, prec), dtype=torch.uint8, device="cuda")
    out = torch.zeros(1, 2, dtype=torch.float64, device="cuda")
    ps = torch.zeros(s1 - s0, 1, 2, dtype=torch.float64, device="cuda")
    qcsim.qc_contract_slices(plan, s0, s1, x[None, :], prec, ws, out, ps)
    torch.cuda.synchronize()
    p = ps.cpu().numpy()[:, 0]
    o = out.cpu().numpy()[0]
    del ws
    return p[:, 0] + 1j * p[:, 1], complex(o[0], o[1])


def _check_slices(got, ref, tol, what):
    ref = np.asarray(ref)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    assert rms > 0, f"{what}: every sampled reference slice is zero"
    err = np.abs(np.asarray(got) - ref)
    bound = tol * np.maximum(np.abs(ref), rms)
    say(f"  {what}: max err/bound {np.max(err / bound):.3e}, rms {rms:.3e}")
    assert (err <= bound).all(), (what, err.tolist(), ref.tolist())


# ------------------------------------------------ 70 qubits, depth 1+32+1
@pytest.fixture(scope="module")
def c4_full():
    """The measured 70-qubit plan (2^20 slices, cap 2^30) and O4 values of
    slices drawn in order from the seed + 2 stream until two are nonzero
    (about half of this plan's slices are exactly zero: a sliced value picks
    a zero row of a leaf, or an intermediate cancels), at most eight; each
    is ~1.1e12 flops in complex128 on the host."""
    import time
    lat, circ, bs, spec, plan = _plan("c4")
    k = qcsim.qc_plan_info(plan)["log2_slices"]
    tree = qcsim.qc_plan_export_tree(plan)
    segs = qcsim.qc_plan_sliced_segments(plan)
    picks, ref = [], {}
    for s in (int(v) for v in synth.random_slices(k, 8, spec["seed"] + 2)):
        t0 = time.perf_counter()
        ref[s] = oracle.hyper_value(lat.n, circ, bs[0], segs, s, tree)
        picks.append(s)
        say(f"c4 O4 slice {s}: {ref[s]} ({time.perf_counter() - t0:.1f} s)")
        if sum(1 for v in ref.values() if v != 0) == 2:
            break
    return lat, bs, spec, plan, picks, ref


@pytest.mark.parametrize("prec", ["c64", "split_fp16", "split_bf16"])
def test_c4_sampled_slices_match_o4(c4_full, prec):
    # Each sampled slice runs inside the chunk of `chunk` consecutive slices
    # the benchmark keeps in flight (the same lowered program and launches).
    lat, bs, spec, plan, picks, ref = c4_full
    chunk = spec["chunk"]
    got = []
    for s in picks:
        s0 = s - s % chunk
        say(f"c4 70q d32 slices [{s0}, {s0 + chunk}) {prec}")
        vals, total = _slice_values(plan, bs[0], s0, s0 + chunk, prec, chunk)
        assert abs(vals.sum() - total) <= 1e-12 * np.abs(vals).sum() + 1e-300
        got.append(vals[s - s0])
    _check_slices(got, [ref[s] for s in picks], TOL[prec], f"c4 {prec}")


@pytest.mark.parametrize("prec", ["c64", "split_fp16", "split_bf16"])
def test_c4_tuned_slices_match_o4(c4_full, prec):
    # The same slices with the GEMM forms the tuner picks (the benchmark's
    # configuration: streaming and tile forms, recorded maxima only where a
    # 16-bit form reads them).
    lat, bs, spec, plan, picks, ref = c4_full
    chunk = spec["chunk"]
    ws = torch.empty(qcsim.qc_workspace_bytes(plan, chunk, 1, prec), dtype=torch.uint8, device="cuda")
    say(f"c4 70q d32 qc_tune {prec}")
    qcsim.qc_tune(plan, chunk, 1, prec, ws)
    torch.cuda.synchronize()
    del ws
    got = []
    for s in picks:
        s0 = s - s % chunk
        say(f"c4 70q d32 tuned slices [{s0}, {s0 + chunk}) {prec}")
        vals, total = _slice_values(plan, bs[0], s0, s0 + chunk, prec, chunk)
        got.append(vals[s - s0])
    _check_slices(got, [ref[s] for s in picks], TOL[prec], f"c4 tuned {prec}")


@pytest.fixture(scope="module")
def c4_fine():
    """The same circuit under a finer slicing (cap 2^22: 32 slice bits, a
    different tree and program).  Most of this plan's slices are exactly
    zero (fixing many segments makes sums over the remaining ones cancel), so
    the slices are chosen from the GPU's values over the 64-slice blocks of
    slices drawn from the seed + 2 stream: up to four nonzero and four zero
    ones, all compared with O4 (so the GPU's zeros are checked as well)."""
    lat, circ, bs, spec, plan = _plan("c4", log2_slices=-1, log2_max_entries=22, greedy_trials=32)
    k = qcsim.qc_plan_info(plan)["log2_slices"]
    tree = qcsim.qc_plan_export_tree(plan)
    segs = qcsim.qc_plan_sliced_segments(plan)
    nonzero, zero = [], []
    for s in (int(v) for v in synth.random_slices(k, 8, spec["seed"] + 2)):
        b0 = s - s % 64
        say(f"c4 cap 2^22: GPU values of slices [{b0}, {b0 + 64})")
        vals, _ = _slice_values(plan, bs[0], b0, b0 + 64, "c64", 64)
        for j, v in enumerate(vals):
            (nonzero if v != 0 else zero).append(b0 + j)
        if len(nonzero) >= 4:
            break
    picks = nonzero[:4] + zero[:4]
    ref = [oracle.hyper_value(lat.n, circ, bs[0], segs, s, tree) for s in picks]
    return bs, plan, picks, ref


@pytest.mark.parametrize("prec", ["c64", "split_fp16"])
def test_c4_finer_slicing_matches_o4(c4_fine, prec):
    bs, plan, picks, ref = c4_fine
    say(f"c4 70q d32 cap 2^22, slices {picks} {prec}")
    got = [_slice_values(plan, bs[0], s, s + 1, prec, 1)[0][0] for s in picks]
    _check_slices(got, ref, TOL[prec], f"c4 cap22 {prec}")


# ----------------------------------------------- 7x7, depth 1+24+1
@pytest.fixture(scope="module")
def c3_o4():
    lat, circ, bs, spec, plan = _plan("c3")
    k = qcsim.qc_plan_info(plan)["log2_slices"]
    tree = qcsim.qc_plan_export_tree(plan)
    segs = qcsim.qc_plan_sliced_segments(plan)
    picks = [int(s) for s in synth.random_slices(k, spec["n_sampled"], spec["seed"] + 2)]
    ref = [oracle.hyper_value(lat.n, circ, bs[0], segs, s, tree) for s in picks]
    return bs, plan, k, picks, ref


@pytest.mark.parametrize("prec", ["c64", "split_fp16", "split_bf16"])
def test_c3_32_sampled_slices_match_o4(c3_o4, prec):
    # All 2^16 slices in one call (the measured configuration).
    bs, plan, k, picks, ref = c3_o4
    say(f"c3 7x7 d24 all 2^{k} slices {prec}, 32 sampled slices vs O4")
    vals, total = _slice_values(plan, bs[0], 0, 1 << k, prec, 1 << k)
    assert abs(vals.sum() - total) <= 1e-12 * np.abs(vals).sum()
    _check_slices(vals[picks], ref, TOL[prec], f"c3 {prec}")


# ------------------------------------- uneven batch: 6x6 and 7x7 requests
def test_batch_large_requests_match_o4():
    # The benchmark's request mix and per-request plans (2^24-entry cap, the
    # request's own slice count); three 6x6 d20 and three 7x7 d24 requests
    # run as one batch, each amplitude compared with O4 summed over all the
    # request's slices (the 7x7 ones are unsliced or lightly sliced: at most
    # a few hundred O4 slices of ~10^7 flops, or one of ~10^11).
    reqs = synth.request_mix(256, 501)
    picked = []
    for fam, kmax in (((6, 6, 20), 8), ((7, 7, 24), 2)):
        picked += [r for r in reqs if r["family"] == fam and r["log2_slices"] <= kmax][:3]
    items, refs = [], []
    for r in picked:
        lat = r["lattice"]
        plan = qcsim.qc_plan_build(lat.n, r["circuit"], r["bitstring"], log2_slices=r["log2_slices"],
                                   log2_max_entries=24, greedy_trials=32, seed=1)
        k = qcsim.qc_plan_info(plan)["log2_slices"]
        tree = qcsim.qc_plan_export_tree(plan)
        segs = qcsim.qc_plan_sliced_segments(plan)
        say(f"batch request {r['family']} k={k}: O4 over all slices")
        refs.append(sum(oracle.hyper_value(lat.n, r["circuit"], r["bitstring"], segs, s, tree) for s in range(1 << k)))
        items.append((plan, r["bitstring"], 0, 1 << k))
    batch = qcsim.Batch(items)
    for prec in ("c64", "split_fp16"):
        ws = torch.empty(qcsim.qc_batch_workspace_bytes(batch, prec), dtype=torch.uint8, device="cuda")
        out = torch.zeros(len(items), 2, dtype=torch.float64, device="cuda")
        t = torch.zeros(len(items) + 1, dtype=torch.int64, device="cuda")
        say(f"batch of {len(items)} 6x6/7x7 requests {prec}")
        qcsim.qc_contract_batch(batch, prec, ws, out, t)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        for i, r in enumerate(picked):
            n = r["lattice"].n
            got = complex(o[i, 0], o[i, 1])
            bound = TOL[prec] * max(abs(refs[i]), 2.0 ** (-n / 2))
            assert abs(got - refs[i]) <= bound, (i, r["family"], got, refs[i])
        del ws


# ------------------------------------------------ 72 qubits with degree-1 qubits
@pytest.mark.parametrize("prec", ["c64", "split_fp16"])
def test_diamond72_slices_vs_o4(prec):
    # The 72-qubit lattice whose corner qubits have one neighbour each, depth
    # 1+24+1, 2^12 slices of at most 2^20 entries: the 64-slice chunk around
    # a slice drawn from stream 413, every slice against O4.
    lat = synth.diamond72()
    circ = synth.random_circuit(lat, 24, 411)
    bs = synth.random_bitstrings(lat.n, 1, 412)
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=10, log2_max_entries=20, greedy_trials=8, seed=2)
    k = qcsim.qc_plan_info(plan)["log2_slices"]
    s0 = int(synth.random_slices(k, 1, 413)[0])
    c0 = s0 - s0 % 64
    say(f"72-qubit d24 slices [{c0}, {c0 + 64}) {prec}")
    got, _ = _slice_values(plan, bs[0], c0, c0 + 64, prec, 64)
    tree = qcsim.qc_plan_export_tree(plan)
    segs = qcsim.qc_plan_sliced_segments(plan)
    ref = [oracle.hyper_value(lat.n, circ, bs[0], segs, s, tree) for s in range(c0, c0 + 64)]
    _check_slices(got, ref, TOL[prec], f"72-qubit d24 {prec}")
