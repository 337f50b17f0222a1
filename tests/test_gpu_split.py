"""Split-precision complex GEMM (hi/lo BF16 or FP16 operands, FP32
accumulation on MFMA, per-operand power-of-two scale) against NumPy FP64.

Pins:
  * exactness: when every operand value is x = h + l exactly (h, l in the
    16-bit type after the power-of-two scale), B needs no lo part, and every
    partial sum is a float32 integer multiple of one quantum, the split GEMM
    must return the FP64 product bit for bit (the dropped lo*lo term is zero
    and no rounding happens anywhere);
  * the same with operands of magnitude 2^-40 and 2^-20: FP16 would flush
    them to zero without the scale, so this pins the scale bookkeeping;
  * random operands: |C - C_exact| <= c K u max|A| max|B| elementwise with
    u = 2^-22 (FP16 split) or 2^-16 (BF16 split) and c = 8 (per real product
    the representation error of one operand is below u |x| and the dropped
    lo*lo term below u |x||y|; two real products per complex part; plus FP32
    accumulation over K);
  * scale slots: the call leaves the float bits of max(|re|,|im|) of A, B, C.
"""

import numpy as np
import pytest

from tests.gpu_util import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1907_11217_amd import qcsim  # noqa: E402

U = {"split_fp16": 2.0 ** -22, "split_bf16": 2.0 ** -16}
C_BOUND = 8.0
PRECS = ["split_fp16", "split_bf16"]


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x).reshape(-1)).cuda()


def _run(A, B, nb, m, n, k, a_km, b_nk, prec, scale_ws=None, form=-1):
    a_store = A.transpose(0, 2, 1) if a_km else A
    b_store = B.transpose(0, 2, 1) if b_nk else B
    dA, dB = _dev(a_store.astype(np.complex64)), _dev(b_store.astype(np.complex64))
    dC = torch.full((nb * m * n,), float("nan"), dtype=torch.complex64, device="cuda")
    say(f"gemm {prec} nb={nb} m={m} n={n} k={k} a_km={a_km} b_nk={b_nk} form={form}")
    if prec == "split_fp16" and scale_ws is None and form >= 0:
        scale_ws = torch.zeros(3, dtype=torch.int32, device="cuda")
    qcsim.qc_kernel_gemm(dA, dB, dC, nb, m, n, k, a_km, b_nk, prec=prec, scale_ws=scale_ws, form=form)
    torch.cuda.synchronize()
    return dC.cpu().numpy().reshape(nb, m, n)


def _exact_operands(rng, nb, m, n, k, sa, sb):
    # A: i 2^-5 with |i| < 2^12 (needs a lo part in both 16-bit types);
    # B: small integers (one 16-bit value, lo = 0).  |sum| < 2^12 * 8 * 2k
    # quanta of 2^-5 stays below 2^24 for k <= 256.
    ia = rng.integers(-(1 << 12) + 1, 1 << 12, size=(2, nb, m, k))
    ib = rng.integers(-8, 9, size=(2, nb, k, n))
    A = (ia[0] + 1j * ia[1]) * 2.0 ** -5 * sa
    B = (ib[0] + 1j * ib[1]) * sb
    return A, B


# 32-multiples take the 32/64-tile form, 128-multiples the large-tile form.
EXACT_SHAPES = [(1, 32, 32, 16), (2, 64, 64, 64), (3, 64, 32, 17), (4, 32, 64, 3), (1, 128, 128, 256), (2, 256, 128, 40),
                (1, 128, 384, 9)]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape", EXACT_SHAPES)
@pytest.mark.parametrize("a_km,b_nk", [(0, 0), (1, 1)])
@pytest.mark.parametrize("scale", [(1.0, 1.0), (2.0 ** -40, 2.0 ** -20)])
def test_split_gemm_exact(prec, shape, a_km, b_nk, scale):
    nb, m, n, k = shape
    rng = np.random.default_rng(m * 7 + n * 131 + k + nb * 17 + a_km)
    A, B = _exact_operands(rng, nb, m, n, k, *scale)
    got = _run(A, B, nb, m, n, k, a_km, b_nk, prec)
    ref = np.matmul(A, B)
    assert np.array_equal(got.astype(np.complex128), ref), np.abs(got - ref).max()


# The 128x64-tile form (m % 128 = 0, n % 64 = 0, k % 8 = 0), every operand layout.
BIG64_SHAPES = [(1, 128, 64, 16), (2, 256, 192, 40), (1, 128, 64, 256), (3, 384, 128, 8)]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape", BIG64_SHAPES)
@pytest.mark.parametrize("a_km,b_nk", [(0, 0), (1, 1), (1, 0), (0, 1)])
@pytest.mark.parametrize("scale", [(1.0, 1.0), (2.0 ** -40, 2.0 ** -20)])
def test_split_big64_exact(prec, shape, a_km, b_nk, scale):
    nb, m, n, k = shape
    rng = np.random.default_rng(m * 5 + n * 37 + k + nb * 19 + a_km + 2 * b_nk)
    A, B = _exact_operands(rng, nb, m, n, k, *scale)
    got = _run(A, B, nb, m, n, k, a_km, b_nk, prec, form=qcsim.GEMM_FORMS["split_big64"])
    ref = np.matmul(A, B)
    assert np.array_equal(got.astype(np.complex128), ref), np.abs(got - ref).max()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("a_km,b_nk", [(0, 0), (1, 0)])
def test_split_big64_error_bound(prec, a_km, b_nk):
    nb, m, n, k = 2, 256, 192, 1000 - 1000 % 8
    rng = np.random.default_rng(91 + a_km)
    A = (rng.standard_normal((nb, m, k)) + 1j * rng.standard_normal((nb, m, k))) * 2.0 ** -30
    B = (rng.standard_normal((nb, k, n)) + 1j * rng.standard_normal((nb, k, n))) * 2.0 ** 3
    A = A.astype(np.complex64).astype(np.complex128)
    B = B.astype(np.complex64).astype(np.complex128)
    got = _run(A, B, nb, m, n, k, a_km, b_nk, prec, form=qcsim.GEMM_FORMS["split_big64"])
    ref = np.matmul(A, B)
    amax = max(np.abs(A.real).max(), np.abs(A.imag).max())
    bmax = max(np.abs(B.real).max(), np.abs(B.imag).max())
    assert np.abs(got - ref).max() <= C_BOUND * k * U[prec] * amax * bmax


SHAPES = [(1, 32, 32, 16), (2, 64, 64, 128), (1, 128, 64, 1000), (8, 32, 32, 2), (1, 64, 128, 4096), (1, 256, 256, 1000),
          (3, 128, 128, 33), (1, 128, 256, 4096)]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("a_km,b_nk", [(0, 0), (1, 0), (0, 1)])
def test_split_gemm_error_bound(prec, shape, a_km, b_nk):
    nb, m, n, k = shape
    rng = np.random.default_rng(k * 3 + m + n * 5 + nb + 11 * a_km + 13 * b_nk)
    # Random circuit-like magnitudes: amplitudes far below FP16's range.
    A = (rng.standard_normal((nb, m, k)) + 1j * rng.standard_normal((nb, m, k))) * 2.0 ** -30
    B = (rng.standard_normal((nb, k, n)) + 1j * rng.standard_normal((nb, k, n))) * 2.0 ** 3
    A = A.astype(np.complex64).astype(np.complex128)
    B = B.astype(np.complex64).astype(np.complex128)
    got = _run(A, B, nb, m, n, k, a_km, b_nk, prec)
    ref = np.matmul(A, B)
    amax = max(np.abs(A.real).max(), np.abs(A.imag).max())
    bmax = max(np.abs(B.real).max(), np.abs(B.imag).max())
    err = np.abs(got - ref).max()
    bound = C_BOUND * k * U[prec] * amax * bmax
    say(f"  max err {err:.3e}, bound {bound:.3e}, fitted c = {err / (k * U[prec] * amax * bmax):.3e}")
    assert err <= bound


@pytest.mark.parametrize("prec", PRECS)
def test_split_gemm_small_shapes_use_fp32(prec):
    # Shapes below the 32x32 tile (or k = 1) take the FP32 vector-ALU form.
    rng = np.random.default_rng(5)
    for nb, m, n, k in [(4, 2, 4, 8), (16, 64, 64, 1), (1, 32, 2, 64), (2, 8, 512, 16)]:
        A = rng.standard_normal((nb, m, k)) + 1j * rng.standard_normal((nb, m, k))
        B = rng.standard_normal((nb, k, n)) + 1j * rng.standard_normal((nb, k, n))
        got = _run(A, B, nb, m, n, k, 0, 0, prec)
        ref = np.matmul(A.astype(np.complex64).astype(np.complex128), B.astype(np.complex64).astype(np.complex128))
        assert np.abs(got - ref).max() <= 1e-5 * np.sqrt(k)


@pytest.mark.parametrize("prec", PRECS + ["c64"])
@pytest.mark.parametrize("shape", [(2, 64, 32, 48), (1, 128, 256, 48)])
def test_scale_slots(prec, shape):
    nb, m, n, k = shape
    rng = np.random.default_rng(9)
    A = ((rng.standard_normal((nb, m, k)) + 1j * rng.standard_normal((nb, m, k))) * 2.0 ** -25).astype(np.complex64)
    B = ((rng.standard_normal((nb, k, n)) + 1j * rng.standard_normal((nb, k, n))) * 3.0).astype(np.complex64)
    slots = torch.full((3,), 12345, dtype=torch.int32, device="cuda")
    got = _run(A, B, nb, m, n, k, 0, 0, prec, scale_ws=slots).astype(np.complex64)
    s = slots.cpu().numpy().view(np.float32)

    def amax(x):
        return np.float32(max(np.abs(x.real).max(), np.abs(x.imag).max()))

    assert s[0] == amax(A) and s[1] == amax(B)
    # Every GEMM form records the maximum of its output when given a slot
    # (the FP32 forms too: a split program's step may run in FP32).
    assert s[2] == amax(got)


def test_split_gemm_zero_operand():
    # A zero tensor gets scale 0 and gives an exact zero product.
    nb, m, n, k = 1, 32, 32, 32
    A = np.zeros((nb, m, k), dtype=np.complex128)
    B = np.ones((nb, k, n), dtype=np.complex128)
    for prec in PRECS:
        got = _run(A, B, nb, m, n, k, 0, 0, prec)
        assert np.array_equal(got, np.zeros_like(got))
