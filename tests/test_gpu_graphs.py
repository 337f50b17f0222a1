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


def test_multi_chunk_call_replays_one_graph():
    # The 7x7 depth-24 plan with a workspace for 4096 slices: one call over
    # all 2^16 slices runs 16 chunks, each replaying the same step graph
    # (one graph for the program however many chunks); it equals the direct
    # launches and 16 calls of one chunk each bit for bit (chunk boundaries
    # are multiples of 64, where the FP64 sums compose exactly).
    lat, circ, bs, spec = synth.config("c3")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=16, log2_max_entries=30, greedy_trials=8, seed=1)
    ws = torch.empty(qcsim.qc_workspace_bytes(plan, 4096, 1), dtype=torch.uint8, device="cuda")
    outs = []
    for graphs in (True, False):
        qcsim.qc_plan_set_graphs(plan, graphs)
        out = torch.zeros(1, 2, dtype=torch.float64, device="cuda")
        say(f"c3 one call over 16 chunks of 4096, graphs={graphs}")
        qcsim.qc_contract_slices(plan, 0, 1 << 16, bs[:1], "c64", ws, out)
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy().copy())
    assert np.array_equal(outs[0], outs[1])
    qcsim.qc_plan_set_graphs(plan, True)
    out = torch.zeros(1, 2, dtype=torch.float64, device="cuda")
    say("c3 16 calls of one chunk each")
    for c in range(16):
        qcsim.qc_contract_slices(plan, c * 4096, (c + 1) * 4096, bs[:1], "c64", ws, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), outs[0])
    assert qcsim.qc_plan_describe(plan, 12, 0)["n_graphs"] == 1


def test_multi_chunk_70_qubit_range():
    # 32 chunks of 64 slices of the 70-qubit plan in one call: one graph,
    # equal to the direct launches bit for bit, and to the per-chunk calls.
    lat, circ, bs, spec = synth.config("c4")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=spec["log2_slices"], log2_max_entries=spec["log2_cap"],
                               greedy_trials=spec["trials"], seed=spec["plan_seed"])
    chunk = spec["chunk"]
    ws = torch.empty(qcsim.qc_workspace_bytes(plan, chunk, 1), dtype=torch.uint8, device="cuda")
    s0, s1 = 5 * chunk, 37 * chunk
    res = []
    for graphs in (True, False):
        qcsim.qc_plan_set_graphs(plan, graphs)
        out = torch.zeros(1, 2, dtype=torch.float64, device="cuda")
        ps = torch.zeros(s1 - s0, 1, 2, dtype=torch.float64, device="cuda")
        say(f"c4 slices [{s0}, {s1}) in one call, graphs={graphs}")
        qcsim.qc_contract_slices(plan, s0, s1, bs[:1], "c64", ws, out, ps)
        torch.cuda.synchronize()
        res.append((out.cpu().numpy().copy(), ps.cpu().numpy().copy()))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    b = (chunk - 1).bit_length()
    assert qcsim.qc_plan_describe(plan, b, 0)["n_graphs"] == 1
