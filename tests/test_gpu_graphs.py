"""Graph replay of the contraction calls: every replay, with the caller's own
eager work and synchronisations between replays, must equal the directly
launched result bit for bit (same kernels, same arguments)."""

import numpy as np
import pytest

import synth
from tests.gpu_util import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1907_11217_amd import qcsim  # noqa: E402


def _calls(plan, xs, s0, s1, prec, graphs, reps):
    qcsim.qc_plan_set_graphs(plan, graphs)
    ws = torch.empty(qcsim.qc_workspace_bytes(plan, s1 - s0, len(xs), prec), dtype=torch.uint8, device="cuda")
    out = torch.zeros(len(xs), 2, dtype=torch.float64, device="cuda")
    ps = torch.zeros(s1 - s0, len(xs), 2, dtype=torch.float64, device="cuda")
    res = []
    for r in range(reps):
        out.zero_()
        ps.zero_()
        # Eager work of the caller's own between replays.
        junk = torch.randn(1 << 16, device="cuda").sum()
        qcsim.qc_contract_slices(plan, s0, s1, xs, prec, ws, out, ps)
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        res.append((out.cpu().numpy().copy(), ps.cpu().numpy().copy()))
    return res


@pytest.mark.parametrize("mode,prec", [("stepwise", "c64"), ("stepwise", "split_fp16"), ("stepwise", "split_bf16")])
def test_graph_replays_match_direct_launches(mode, prec):
    lat, circ, bs, spec = synth.config("c2")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=6, greedy_trials=4, seed=1)
    qcsim.qc_plan_set_exec(plan, mode)
    xs = bs[:16]
    say(f"graphs c2 {mode} {prec}: direct")
    direct = _calls(plan, xs, 0, 64, prec, False, 1)[0]
    say(f"graphs c2 {mode} {prec}: 4 replays")
    for o, p in _calls(plan, xs, 0, 64, prec, True, 4):
        assert np.array_equal(o, direct[0]) and np.array_equal(p, direct[1])
    # A different range is a different graph; the first one stays valid.
    say(f"graphs c2 {mode} {prec}: other range, then the first again")
    other = _calls(plan, xs, 0, 32, prec, True, 2)
    assert np.array_equal(other[0][0], other[1][0])
    again = _calls(plan, xs, 0, 64, prec, True, 2)
    for o, p in again:
        assert np.array_equal(o, direct[0]) and np.array_equal(p, direct[1])


def test_graph_large_program_7x7():
    # The 7x7 depth-24 program (hundreds of launches per chunk): replays of
    # one chunk of 4096 slices equal the direct launches.
    lat, circ, bs, spec = synth.config("c3")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=16, log2_max_entries=30, greedy_trials=8, seed=1)
    say("graphs c3 direct, slices [4096, 8192)")
    direct = _calls(plan, bs[:1], 4096, 8192, "c64", False, 1)[0]
    say("graphs c3 3 replays")
    for o, p in _calls(plan, bs[:1], 4096, 8192, "c64", True, 3):
        assert np.array_equal(o, direct[0]) and np.array_equal(p, direct[1])
