"""Uneven request batches (qc_contract_batch): every request's amplitude
equals its own qc_contract_slices result bit for bit (same kernels, same
fixed-order sums), the small ones equal the state-vector oracle, and the
completion stamps are ordered after the batch start."""

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import check_amplitudes, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1907_11217_amd import qcsim  # noqa: E402


def _single(plan, x, s0, s1, prec):
    ws = torch.empty(qcsim.qc_workspace_bytes(plan, min(s1 - s0, 4096), 1, prec), dtype=torch.uint8, device="cuda")
    out = torch.zeros(1, 2, dtype=torch.float64, device="cuda")
    qcsim.qc_contract_slices(plan, s0, s1, x[None, :], prec, ws, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()[0]


@pytest.mark.parametrize("prec", ["c64", "split_fp16"])
def test_batch_matches_single_requests(prec):
    reqs = synth.request_mix(24, 501)
    keep = [r for r in reqs if r["family"][0] <= 6][:10]
    fams = sorted({r["family"] for r in keep})
    assert len(fams) >= 3
    items = []
    for i, r in enumerate(keep):
        lat = r["lattice"]
        # 6x6 requests are sliced (stepwise, several chunks); small ones run
        # fused in complex FP32, one with a partial slice range.
        k = 3 if r["family"][0] == 6 else (2 if i % 2 else 0)
        plan = qcsim.qc_plan_build(lat.n, r["circuit"], r["bitstring"], log2_slices=k, greedy_trials=2, seed=1)
        # Batches run fused requests one slice per work item; pin the single
        # calls to the same so the two agree bit for bit.
        qcsim.qc_plan_set_fused_slice_bits(plan, 0)
        s1 = 1 << qcsim.qc_plan_info(plan)["log2_slices"]
        s0 = 1 if (k == 2 and i == 1) else 0
        items.append((plan, r["bitstring"], s0, s1))
    batch = qcsim.Batch(items)
    ws = torch.empty(qcsim.qc_batch_workspace_bytes(batch, prec), dtype=torch.uint8, device="cuda")
    out = torch.zeros(len(items), 2, dtype=torch.float64, device="cuda")
    t = torch.zeros(len(items) + 1, dtype=torch.int64, device="cuda")
    say(f"batch of {len(items)} requests {fams} {prec}")
    qcsim.qc_contract_batch(batch, prec, ws, out, t)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    stamps = t.cpu().numpy()
    assert np.all(stamps[:-1] >= stamps[-1]) and np.all(stamps > 0)
    for i, (plan, x, s0, s1) in enumerate(items):
        say(f"  request {i} single call")
        assert np.array_equal(got[i], _single(plan, x, s0, s1, prec)), i
    # The 4x4 and 5x5 requests with whole ranges against the oracle.
    for i, r in enumerate(keep):
        if r["family"][0] <= 5 and items[i][2] == 0:
            ref = oracle.amplitudes_sv(r["lattice"].n, r["circuit"], [r["bitstring"]])
            check_amplitudes([got[i, 0] + 1j * got[i, 1]], ref, r["lattice"].n, 1e-5 if prec == "c64" else 1e-4)


def test_batch_rejects_bad_requests():
    lat = synth.grid(2, 2)
    circ = synth.random_circuit(lat, 2, 1)
    plan = qcsim.qc_plan_build(lat.n, circ, None, log2_slices=0)
    with pytest.raises(qcsim.QcError) as e:
        qcsim.qc_batch_workspace_bytes(qcsim.Batch([(plan, np.zeros(lat.n, np.uint8), 0, 3)]))
    assert "out of bounds" in str(e.value)
    with pytest.raises(qcsim.QcError) as e:
        qcsim.qc_batch_workspace_bytes(qcsim.Batch([(plan, np.full(lat.n, 2, np.uint8), 0, 1)]))
    assert "0 or 1" in str(e.value)
