"""qc_contract_slices_noalloc (the entry point for callers that cannot
allocate device memory) against qc_contract_slices_dev on the same inputs.

Each case makes two no-alloc calls in a row, the second with a smaller input
(fewer bitstrings and slices), so the second runs on scratch that still
holds the first call's contents.  Tolerance: the complex FP32 bar of the
amplitude tests (1e-5 relative to max(|ref|, rms of the batch)), 1e-4 for
split FP16; the two entry points may keep different numbers of slices in
flight, which changes the rounding only.
"""

import numpy as np
import pytest

import synth
from tests.gpu_util import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1907_11217_amd import qcsim  # noqa: E402

TOL = {"c64": 1e-5, "split_fp16": 1e-4}


def _regular(plan, bits_dev, s0, s1, prec):
    n_bs = bits_dev.shape[0]
    ws = torch.empty(qcsim.qc_workspace_bytes(plan, min(s1 - s0, 4096), n_bs, prec), dtype=torch.uint8,
                     device="cuda")
    out = torch.zeros(n_bs, 2, dtype=torch.float64, device="cuda")
    ps = torch.zeros(s1 - s0, n_bs, 2, dtype=torch.float64, device="cuda")
    qcsim.qc_contract_slices_dev(plan, s0, s1, bits_dev, prec, ws, out, ps)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ps.cpu().numpy()


def _noalloc(plan, bits_dev, s0, s1, prec):
    n_bs = bits_dev.shape[0]
    out = torch.zeros(n_bs, 2, dtype=torch.float64, device="cuda")
    ps = torch.zeros(s1 - s0, n_bs, 2, dtype=torch.float64, device="cuda")
    qcsim.qc_contract_slices_noalloc(plan, s0, s1, bits_dev, prec, out, ps)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ps.cpu().numpy()


def _close(a, b, tol, what):
    a = a[..., 0] + 1j * a[..., 1]
    b = b[..., 0] + 1j * b[..., 1]
    rms = np.sqrt(np.mean(np.abs(b) ** 2))
    assert rms > 0, what
    err = np.abs(a - b)
    bound = tol * np.maximum(np.abs(b), rms)
    say(f"  {what}: max err/bound {np.max(err / bound):.2e}")
    assert (err <= bound).all(), what


def _two_calls(plan, bits, calls, prec):
    for n_bs, s0, s1 in calls:
        bd = torch.from_numpy(np.ascontiguousarray(bits[:n_bs])).cuda()
        say(f"no-alloc call: {n_bs} bitstrings, slices [{s0}, {s1}), {prec}")
        got_o, got_p = _noalloc(plan, bd, s0, s1, prec)
        ref_o, ref_p = _regular(plan, bd, s0, s1, prec)
        _close(got_o, ref_o, TOL[prec], f"amplitudes {n_bs}x[{s0},{s1})")
        _close(got_p, ref_p, TOL[prec], f"slice values {n_bs}x[{s0},{s1})")


def test_noalloc_fused_5x5_two_calls():
    # The 5x5 depth-16 workload (fused form): 64 bitstrings x 64 slices,
    # then 16 bitstrings x 16 slices.  The first regular call (inside the
    # helper, after the no-alloc one) times the fused shape; the second
    # no-alloc call then uses it.
    lat, circ, bs, spec = synth.config("c2")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=spec["log2_slices"], greedy_trials=spec["trials"],
                               seed=spec["plan_seed"])
    _two_calls(plan, bs, [(64, 0, 64), (16, 8, 24)], "c64")


@pytest.mark.parametrize("prec", ["c64", "split_fp16"])
def test_noalloc_stepwise_5x5_d24_two_calls(prec):
    # Stepwise form with GEMM steps on MFMA (split FP16 on the split MFMA
    # forms): 16 bitstrings x 4 slices, then 4 bitstrings x 2 slices.
    lat = synth.grid(5, 5)
    circ = synth.random_circuit(lat, 24, 201)
    xs = synth.random_bitstrings(lat.n, 16, 205)
    plan = qcsim.qc_plan_build(lat.n, circ, xs[0], log2_slices=2, greedy_trials=8, seed=1)
    qcsim.qc_plan_set_exec(plan, "stepwise")
    _two_calls(plan, xs, [(16, 0, 4), (4, 1, 3)], prec)


def test_noalloc_rejects_a_program_beyond_the_scratch():
    lat, circ, bs, spec = synth.config("c4")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=spec["log2_slices"],
                               log2_max_entries=spec["log2_cap"], greedy_trials=4, seed=1)
    bd = torch.from_numpy(np.ascontiguousarray(bs[:1])).cuda()
    out = torch.zeros(1, 2, dtype=torch.float64, device="cuda")
    with pytest.raises(qcsim.QcError) as e:
        qcsim.qc_contract_slices_noalloc(plan, 0, 1, bd, "c64", out)
    assert e.value.status == 3 and "64 MiB" in str(e.value)
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == 0).all()
