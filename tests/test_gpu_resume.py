"""Checkpoint and resume of a long slice range.

Slices are independent subtasks whose values add up to the amplitude (the
paper, Section "Benchmarking and the Experimental Setup", preprocessing
paragraph), and a range's FP64 partial sum is added to the output, with chunk
boundaries at multiples of 64 slices where the sums compose exactly.  So a
job over many slices can keep (next slice, partial sum) as its checkpoint:
a worker that dies loses only the chunk in flight, and a new process that
rebuilds the plan (the planner is deterministic) and resumes from the
checkpoint ends with the same bits as an uninterrupted run.  The failure is
forced from the host: the worker process exits on its own after its third
chunk, with its GPU work finished.
"""

import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

import synth
from tests.gpu_util import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1907_11217_amd import qcsim  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHUNK = 4096
N_CHUNKS = 16

WORKER = textwrap.dedent("""
    import os, sys
    import numpy as np
    sys.path.insert(0, ROOT)
    import torch
    import synth
    from paper_1907_11217_amd import qcsim
    lat, circ, bs, spec = synth.config("c3")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=16, log2_max_entries=30, greedy_trials=8, seed=1)
    ws = torch.empty(qcsim.qc_workspace_bytes(plan, CHUNK, 1), dtype=torch.uint8, device="cuda")
    out = torch.zeros(1, 2, dtype=torch.float64, device="cuda")
    for c in range(N_CHUNKS):
        qcsim.qc_contract_slices(plan, c * CHUNK, (c + 1) * CHUNK, bs[:1], "c64", ws, out)
        torch.cuda.synchronize()
        tmp = CKPT + ".tmp.npz"
        np.savez(tmp, cursor=np.int64((c + 1) * CHUNK), out=out.cpu().numpy())
        os.replace(tmp, CKPT)
        print(f"worker: chunk {c} done", flush=True)
        if c == 2:
            os._exit(17)
""")


def _plan():
    lat, circ, bs, spec = synth.config("c3")
    return qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=16, log2_max_entries=30, greedy_trials=8,
                               seed=1), bs


def test_resume_after_worker_death(tmp_path):
    plan, bs = _plan()
    ws = torch.empty(qcsim.qc_workspace_bytes(plan, CHUNK, 1), dtype=torch.uint8, device="cuda")
    ref = torch.zeros(1, 2, dtype=torch.float64, device="cuda")
    say("resume: uninterrupted reference over [0, 65536)")
    qcsim.qc_contract_slices(plan, 0, N_CHUNKS * CHUNK, bs[:1], "c64", ws, ref)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()

    ckpt = str(tmp_path / "job.npz")
    code = f"ROOT = {ROOT!r}\nCKPT = {ckpt!r}\nCHUNK = {CHUNK}\nN_CHUNKS = {N_CHUNKS}\n" + WORKER
    say("resume: worker process, exits after its third chunk")
    r = subprocess.run([sys.executable, "-u", "-c", code], capture_output=True, text=True, timeout=300)
    say(r.stdout.strip())
    assert r.returncode == 17, r.stderr[-4000:]
    assert "chunk 2 done" in r.stdout and "chunk 3 done" not in r.stdout

    # A new plan object (built again, as a new process would) resumes from
    # the checkpoint.
    del plan
    plan, bs = _plan()
    ck = np.load(ckpt)
    cursor = int(ck["cursor"])
    assert cursor == 3 * CHUNK
    out = torch.from_numpy(ck["out"].copy()).cuda()
    # A call the library rejects leaves the partial sum untouched.
    with pytest.raises(qcsim.QcError):
        qcsim.qc_contract_slices(plan, cursor, N_CHUNKS * CHUNK + 1, bs[:1], "c64", ws, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ck["out"])
    say(f"resume: slices [{cursor}, {N_CHUNKS * CHUNK}) in the test process")
    for c in range(cursor // CHUNK, N_CHUNKS):
        qcsim.qc_contract_slices(plan, c * CHUNK, (c + 1) * CHUNK, bs[:1], "c64", ws, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref)
