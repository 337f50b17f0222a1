"""GEMM kernel forms and the autotuner.

Every applicable form (the autotuner may choose any of them) is checked
against NumPy: the FP32 forms to FP32 accumulation error, the split forms to
the split error bound (see tests/test_gpu_split.py).  qc_tune is checked end
to end: tuned contractions still match the oracle, and a second tuning with
the same cache file times nothing."""

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import check_amplitudes, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1907_11217_amd import qcsim  # noqa: E402

U = {"c64": 2.0 ** -24, "split_fp16": 2.0 ** -22, "split_bf16": 2.0 ** -16}
FORM_SHAPES = [(1, 1, 256, 512), (2, 8, 64, 33), (1, 16, 128, 16), (3, 32, 32, 16), (1, 64, 128, 64),
               (2, 128, 128, 48), (1, 256, 384, 32), (4, 2, 2, 4096), (2, 512, 8, 64), (4, 16, 16, 2048),
               (1, 300, 16, 5)]


@pytest.mark.parametrize("prec", ["c64", "split_fp16", "split_bf16"])
@pytest.mark.parametrize("shape", FORM_SHAPES)
def test_every_applicable_form_matches_numpy(prec, shape):
    nb, m, n, k = shape
    rng = np.random.default_rng(nb + 3 * m + 7 * n + 11 * k)
    A = ((rng.standard_normal((nb, m, k)) + 1j * rng.standard_normal((nb, m, k))) * 2.0 ** -20).astype(np.complex64)
    B = (rng.standard_normal((nb, k, n)) + 1j * rng.standard_normal((nb, k, n))).astype(np.complex64)
    ref = np.matmul(A.astype(np.complex128), B.astype(np.complex128))
    dA = torch.from_numpy(A.reshape(-1)).cuda()
    dB = torch.from_numpy(B.reshape(-1)).cuda()
    amax = max(np.abs(A.real).max(), np.abs(A.imag).max())
    bmax = max(np.abs(B.real).max(), np.abs(B.imag).max())
    ran = 0
    for name, form in qcsim.GEMM_FORMS.items():
        dC = torch.full((nb * m * n,), float("nan"), dtype=torch.complex64, device="cuda")
        say(f"gemm form {name} {prec} {shape}")
        try:
            qcsim.qc_kernel_gemm(dA, dB, dC, nb, m, n, k, prec=prec, form=form)
        except qcsim.QcError as e:
            assert e.status == 5  # form does not apply
            continue
        torch.cuda.synchronize()
        got = dC.cpu().numpy().reshape(nb, m, n)
        # FP32 forms (and FP32 accumulation of the split forms).
        u = U[prec] if name.startswith("split") else U["c64"]
        assert np.abs(got - ref).max() <= 8.0 * k * u * amax * bmax, (name, np.abs(got - ref).max())
        ran += 1
    assert ran >= 2


def test_tune_c2_stepwise_matches_oracle(tmp_path):
    lat, circ, bs, spec = synth.config("c2")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=6, greedy_trials=4, seed=1)
    qcsim.qc_plan_set_exec(plan, "stepwise")
    ws = torch.empty(qcsim.qc_workspace_bytes(plan, 64, len(bs)), dtype=torch.uint8, device="cuda")
    cache = tmp_path / "tune.txt"
    say("qc_tune c2 stepwise, 64 slices x 64 bitstrings")
    n1 = qcsim.qc_tune(plan, 64, len(bs), "c64", ws, cache)
    assert n1 > 0 and cache.exists()
    lines = cache.read_text().split("\n")
    assert sum(1 for ln in lines if ln.strip()) >= n1
    out = torch.zeros(len(bs), 2, dtype=torch.float64, device="cuda")
    qcsim.qc_contract_slices(plan, 0, 64, bs, "c64", ws, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    psi = oracle.statevector(lat.n, circ)
    ref = np.array([psi[oracle.index_of(x)] for x in bs])
    check_amplitudes(o[:, 0] + 1j * o[:, 1], ref, lat.n, 1e-5)
    # A new plan of the same circuit finds every shape in the cache.
    plan2 = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=6, greedy_trials=4, seed=1)
    qcsim.qc_plan_set_exec(plan2, "stepwise")
    assert qcsim.qc_tune(plan2, 64, len(bs), "c64", ws, cache) == 0


@pytest.mark.parametrize("prec", ["c64", "split_fp16", "split_bf16"])
def test_tune_7x7_chunk_agrees_with_untuned(prec):
    lat, circ, bs, spec = synth.config("c3")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=16, log2_max_entries=30, greedy_trials=8, seed=1)
    ws = torch.empty(qcsim.qc_workspace_bytes(plan, 4096, 1, prec), dtype=torch.uint8, device="cuda")
    ps0 = torch.zeros(4096, 1, 2, dtype=torch.float64, device="cuda")
    ps1 = torch.zeros(4096, 1, 2, dtype=torch.float64, device="cuda")
    out = torch.zeros(1, 2, dtype=torch.float64, device="cuda")
    say(f"7x7 chunk of 4096 slices {prec}: untuned")
    qcsim.qc_contract_slices(plan, 0, 4096, bs[:1], prec, ws, out, ps0)
    say(f"7x7 chunk {prec}: qc_tune then tuned")
    assert qcsim.qc_tune(plan, 4096, 1, prec, ws) >= 1
    qcsim.qc_contract_slices(plan, 0, 4096, bs[:1], prec, ws, out, ps1)
    torch.cuda.synchronize()
    a, b = ps0.cpu().numpy(), ps1.cpu().numpy()
    scale = np.sqrt(np.mean(a ** 2))
    assert np.abs(a - b).max() <= {"c64": 1e-5, "split_fp16": 1e-4, "split_bf16": 1e-3}[prec] * scale
