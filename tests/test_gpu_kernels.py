"""Step kernels on the GPU against NumPy: the batched complex GEMM (MFMA and
VALU forms, all four operand layouts) and the bit-permuting transpose."""

import numpy as np
import pytest

from tests.gpu_util import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1907_11217_amd import qcsim  # noqa: E402


def _rand(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)


def fp32_sum_tol(k):
    """Bound on |C - C_exact| for FP32 sums of k products of unit-variance
    complex values.  Each real part of C sums 2k products of variance 1, so the
    partial sums grow like sqrt(2j) and a sequential FP32 sum's rounding error
    has a standard deviation of about 0.3 u k (u = 2^-23); blocked or split
    sums do better.  4 u k + 64 u sqrt(k) is at least 13 of those deviations
    at every k, yet at k = 2^20 it is 0.5, below the magnitude (about 2) of a
    single dropped or doubled product."""
    u = 2.0 ** -23
    return 4 * u * k + 64 * u * np.sqrt(k)


GEMM_SHAPES = [
    # nb, m, n, k          (MFMA needs m, n >= 32 and k >= 2)
    (1, 32, 32, 2), (3, 64, 64, 16), (2, 64, 32, 32), (1, 128, 64, 64), (5, 32, 64, 8),
    (2, 256, 128, 128), (1, 64, 64, 4),
    (4, 2, 4, 8), (7, 1, 16, 4), (1, 1, 1, 1024), (16, 64, 64, 1), (8, 16, 16, 16), (1, 32, 2, 64),
    # m <= 16 with n >= 256: the skinny form (one thread per column of C)
    (2, 1, 1024, 4), (1, 4, 4096, 64), (3, 16, 300, 7), (5, 8, 256, 1), (1, 2, 65536, 2),
    # a few outputs with k >= 4096: the dot form (one workgroup per output)
    (1, 1, 1, 1 << 20), (2, 2, 2, 5000), (1, 1, 3, 4096),
]


@pytest.mark.parametrize("shape", GEMM_SHAPES)
@pytest.mark.parametrize("a_km,b_nk", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_c64(shape, a_km, b_nk):
    nb, m, n, k = shape
    rng = np.random.default_rng(nb * 1000003 + m * 1009 + n * 31 + k + 7 * a_km + 13 * b_nk)
    A = _rand(rng, (nb, m, k))
    B = _rand(rng, (nb, k, n))
    a_store = A.transpose(0, 2, 1) if a_km else A
    b_store = B.transpose(0, 2, 1) if b_nk else B
    dA = torch.from_numpy(np.ascontiguousarray(a_store).reshape(-1)).cuda()
    dB = torch.from_numpy(np.ascontiguousarray(b_store).reshape(-1)).cuda()
    dC = torch.zeros(nb * m * n, dtype=torch.complex64, device="cuda")
    say(f"gemm c64 nb={nb} m={m} n={n} k={k} a_km={a_km} b_nk={b_nk}")
    qcsim.qc_kernel_gemm(dA, dB, dC, nb, m, n, k, a_km, b_nk)
    torch.cuda.synchronize()
    got = dC.cpu().numpy().reshape(nb, m, n)
    ref = np.matmul(A.astype(np.complex128), B.astype(np.complex128))
    assert np.abs(got - ref).max() <= fp32_sum_tol(k), (np.abs(got - ref).max(), fp32_sum_tol(k))


@pytest.mark.parametrize("rank", [0, 1, 3, 5, 8, 10, 11, 12, 13, 14, 18, 22, 24])
def test_transpose_exact(rank):
    rng = np.random.default_rng(rank)
    perm = rng.permutation(rank).astype(np.int32)
    x = _rand(rng, (1 << rank,))
    d_in = torch.from_numpy(x).cuda()
    d_out = torch.zeros(1 << rank, dtype=torch.complex64, device="cuda")
    say(f"transpose rank={rank}")
    qcsim.qc_kernel_transpose(d_in, d_out, rank, perm)
    torch.cuda.synchronize()
    got = d_out.cpu().numpy()
    # Reference: bit p of the input offset becomes bit perm[p] of the output.
    i = np.arange(1 << rank, dtype=np.int64)
    o = np.zeros_like(i)
    for p in range(rank):
        o |= ((i >> p) & 1) << int(perm[p])
    ref = np.zeros_like(x)
    ref[o] = x
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


def test_transpose_rejects_bad_perm():
    d = torch.zeros(8, dtype=torch.complex64, device="cuda")
    with pytest.raises(qcsim.QcError):
        qcsim.qc_kernel_transpose(d, d, 3, [0, 0, 1])


@pytest.mark.parametrize("kind", ["identity", "reverse", "low_fixed", "rotate"])
def test_transpose_structured(kind):
    # Permutations whose input-low and output-low bits overlap (the tile then
    # grows along both) or coincide entirely.
    rank = 20
    if kind == "identity":
        perm = np.arange(rank)
    elif kind == "reverse":
        perm = np.arange(rank)[::-1]
    elif kind == "low_fixed":
        perm = np.concatenate([np.arange(7), np.random.default_rng(3).permutation(np.arange(7, rank))])
    else:
        perm = (np.arange(rank) + 3) % rank
    perm = perm.astype(np.int32)
    rng = np.random.default_rng(11)
    x = _rand(rng, (1 << rank,))
    d_in = torch.from_numpy(x).cuda()
    d_out = torch.zeros(1 << rank, dtype=torch.complex64, device="cuda")
    say(f"transpose rank={rank} {kind}")
    qcsim.qc_kernel_transpose(d_in, d_out, rank, perm)
    torch.cuda.synchronize()
    i = np.arange(1 << rank, dtype=np.int64)
    o = np.zeros_like(i)
    for p in range(rank):
        o |= ((i >> p) & 1) << int(perm[p])
    ref = np.zeros_like(x)
    ref[o] = x
    assert np.array_equal(d_out.cpu().numpy().view(np.uint64), ref.view(np.uint64))


# Split over k: (nb, m, n, k, kparts); kparts 0 takes the library's rule.
KSPLIT_SHAPES = [(1, 128, 128, 1024, 4), (2, 256, 128, 2048, 8), (3, 128, 256, 512, 2), (1, 128, 384, 4096, 0),
                 (2, 128, 128, 8192, 64)]


@pytest.mark.parametrize("shape", KSPLIT_SHAPES)
@pytest.mark.parametrize("prec", ["c64", "split_bf16", "split_fp16"])
@pytest.mark.parametrize("a_km,b_nk", [(0, 0), (1, 1), (1, 0)])
def test_gemm_kparts(shape, prec, a_km, b_nk):
    _check_kparts(shape, prec, a_km, b_nk, "mfma_big" if prec == "c64" else "split_big")


# The 32- and 64-wide MFMA forms split over k: (nb, m, n, k, kparts, tile),
# tile = the form's 32-multiples in m and n.
KSPLIT_SMALL = [(1, 32, 64, 4096, 8, "12"), (2, 64, 64, 2048, 0, "22"), (3, 32, 32, 1024, 4, "11"),
                (1, 64, 32, 8192, 16, "21")]


@pytest.mark.parametrize("shape", KSPLIT_SMALL)
@pytest.mark.parametrize("prec", ["c64", "split_bf16", "split_fp16"])
@pytest.mark.parametrize("a_km,b_nk", [(0, 0), (1, 1), (1, 0)])
def test_gemm_kparts_small_forms(shape, prec, a_km, b_nk):
    *dims, tile = shape
    _check_kparts(tuple(dims), prec, a_km, b_nk, ("mfma" if prec == "c64" else "split") + tile)


def _check_kparts(shape, prec, a_km, b_nk, form_name):
    nb, m, n, k, kp = shape
    rng = np.random.default_rng(nb * 7 + m + n * 3 + k + kp + 5 * a_km + 11 * b_nk)
    A = _rand(rng, (nb, m, k)) * np.float32(2.0 ** -20)
    B = _rand(rng, (nb, k, n))
    a_store = A.transpose(0, 2, 1) if a_km else A
    b_store = B.transpose(0, 2, 1) if b_nk else B
    dA = torch.from_numpy(np.ascontiguousarray(a_store).reshape(-1)).cuda()
    dB = torch.from_numpy(np.ascontiguousarray(b_store).reshape(-1)).cuda()
    form = qcsim.GEMM_FORMS[form_name]
    parts = kp or qcsim.qc_gemm_kparts(nb, m, n, k)
    assert parts > 1
    scratch = torch.full((parts * nb * m * n,), float("nan"), dtype=torch.complex64, device="cuda")
    slots = torch.zeros(3, dtype=torch.int32, device="cuda")
    dC = torch.full((nb * m * n,), float("nan"), dtype=torch.complex64, device="cuda")
    dC1 = torch.full((nb * m * n,), float("nan"), dtype=torch.complex64, device="cuda")
    say(f"gemm {prec} {form_name} split over k: nb={nb} m={m} n={n} k={k} kparts={kp} a_km={a_km} b_nk={b_nk}")
    qcsim.qc_kernel_gemm(dA, dB, dC, nb, m, n, k, a_km, b_nk, prec=prec, scale_ws=slots, form=form, kparts=kp,
                         scratch=scratch)
    qcsim.qc_kernel_gemm(dA, dB, dC1, nb, m, n, k, a_km, b_nk, prec=prec, scale_ws=None if prec == "c64" else
                         torch.zeros(3, dtype=torch.int32, device="cuda"), form=form)
    torch.cuda.synchronize()
    got = dC.cpu().numpy().reshape(nb, m, n)
    whole = dC1.cpu().numpy().reshape(nb, m, n)
    ref = np.matmul(A.astype(np.complex128), B.astype(np.complex128))
    amax = max(np.abs(A.real).max(), np.abs(A.imag).max())
    bmax = max(np.abs(B.real).max(), np.abs(B.imag).max())
    # FP32 accumulation (plus the split's representation error) over k.
    u = {"c64": 2.0 ** -23, "split_fp16": 2.0 ** -22, "split_bf16": 2.0 ** -16}[prec]
    bound = 8.0 * k * u * amax * bmax
    assert np.abs(got - ref).max() <= bound, (np.abs(got - ref).max(), bound)
    assert np.abs(got - whole).max() <= 2 * bound
    # The sum kernel records max(|re|, |im|) of C.
    s = slots.cpu().numpy().view(np.float32)
    g32 = got.astype(np.complex64)
    assert s[2] == np.float32(max(np.abs(g32.real).max(), np.abs(g32.imag).max()))
    # Deterministic: the parts are summed in a fixed order.
    qcsim.qc_kernel_gemm(dA, dB, dC1, nb, m, n, k, a_km, b_nk, prec=prec, scale_ws=slots, form=form, kparts=kp,
                         scratch=scratch)
    torch.cuda.synchronize()
    assert np.array_equal(dC1.cpu().numpy().view(np.uint64), dC.cpu().numpy().view(np.uint64))


@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
def test_gemm_kparts_exact(prec):
    # Integer operands (A on a 2^-5 grid that needs a lo part): every partial
    # and every sum of parts is exact, so the split product equals the FP64 one.
    nb, m, n, k, kp = 2, 128, 256, 1024, 4
    rng = np.random.default_rng(21)
    ia = rng.integers(-(1 << 10) + 1, 1 << 10, size=(2, nb, m, k))
    ib = rng.integers(-4, 5, size=(2, nb, k, n))
    A = (ia[0] + 1j * ia[1]) * 2.0 ** -5
    B = (ib[0] + 1j * ib[1]) * 1.0
    dA = torch.from_numpy(A.astype(np.complex64).reshape(-1)).cuda()
    dB = torch.from_numpy(B.astype(np.complex64).reshape(-1)).cuda()
    dC = torch.zeros(nb * m * n, dtype=torch.complex64, device="cuda")
    say(f"gemm {prec} split over k, exact operands")
    qcsim.qc_kernel_gemm(dA, dB, dC, nb, m, n, k, 0, 0, prec=prec, form=qcsim.GEMM_FORMS["split_big"], kparts=kp,
                         scale_ws=torch.zeros(3, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    got = dC.cpu().numpy().reshape(nb, m, n).astype(np.complex128)
    assert np.array_equal(got, np.matmul(A, B))


def test_gemm_kparts_rejects_bad_arguments():
    nb, m, n, k = 1, 128, 128, 1024
    d = torch.zeros(nb * max(m, n) * k, dtype=torch.complex64, device="cuda")
    scratch = torch.zeros(128 * m * n, dtype=torch.complex64, device="cuda")
    # Not a power of two; parts of one k value, which the form does not take;
    # a form without a split over k.
    for form, kp, kk in [("mfma_big", 3, k), ("mfma22", 64, 64), ("valu", 2, k)]:
        with pytest.raises(qcsim.QcError):
            qcsim.qc_kernel_gemm(d, d, d, nb, m, n, kk, prec="c64", form=qcsim.GEMM_FORMS[form], kparts=kp,
                                 scratch=scratch)
    # The streaming forms do not split over k (n = 32, k = 64: the form and
    # each part of k = 32 would both apply).
    d32 = torch.zeros(128 * 64, dtype=torch.complex64, device="cuda")
    with pytest.raises(qcsim.QcError):
        qcsim.qc_kernel_gemm(d32, d32, d32, 1, 128, 32, 64, prec="c64", form=qcsim.GEMM_FORMS["stream"], kparts=2,
                             scratch=scratch)
    with pytest.raises(qcsim.QcError):  # 16 parts do not divide k = 24
        qcsim.qc_kernel_gemm(d, d, d, nb, m, n, 24, prec="c64", form=qcsim.GEMM_FORMS["mfma_big"], kparts=16,
                             scratch=scratch)


@pytest.mark.parametrize("shape", [(1, 1, 1, 1 << 20, 0), (2, 2, 2, 65536, 0), (1, 1, 3, 16384, 4), (3, 1, 1, 8192, 2)])
@pytest.mark.parametrize("a_km,b_nk", [(0, 0), (1, 1)])
def test_gemm_dot_kparts(shape, a_km, b_nk):
    nb, m, n, k, kp = shape
    rng = np.random.default_rng(k + nb + 3 * m + 5 * n + kp + a_km)
    A = _rand(rng, (nb, m, k))
    B = _rand(rng, (nb, k, n))
    a_store = A.transpose(0, 2, 1) if a_km else A
    b_store = B.transpose(0, 2, 1) if b_nk else B
    dA = torch.from_numpy(np.ascontiguousarray(a_store).reshape(-1)).cuda()
    dB = torch.from_numpy(np.ascontiguousarray(b_store).reshape(-1)).cuda()
    dC = torch.full((nb * m * n,), float("nan"), dtype=torch.complex64, device="cuda")
    parts = kp or qcsim.qc_gemm_kparts(nb, m, n, k)
    assert parts > 1
    say(f"gemm dot split over k: nb={nb} m={m} n={n} k={k} kparts={parts} a_km={a_km} b_nk={b_nk}")
    qcsim.qc_kernel_gemm(dA, dB, dC, nb, m, n, k, a_km, b_nk, form=qcsim.GEMM_FORMS["dot"], kparts=kp)
    torch.cuda.synchronize()
    got = dC.cpu().numpy().reshape(nb, m, n)
    ref = np.matmul(A.astype(np.complex128), B.astype(np.complex128))
    assert np.abs(got - ref).max() <= fp32_sum_tol(k), (np.abs(got - ref).max(), fp32_sum_tol(k))


def test_gemm_kparts_limit():
    nb, m, n, k = 1, 1, 1, 1 << 22
    d = torch.zeros(k, dtype=torch.complex64, device="cuda")
    with pytest.raises((qcsim.QcError, ValueError)):  # at most 1024 parts
        qcsim.qc_kernel_gemm(d, d, d, nb, m, n, k, form=qcsim.GEMM_FORMS["dot"], kparts=2048)


# Every complex FP32 form on integer operands small enough that every
# product and partial sum is an integer below 2^24: the result must equal the
# FP64 product bit for bit, so a dropped, repeated or misplaced term fails at
# any k (the random-operand tests above can only bound rounding).
# (form, nb, m, n, k, kparts); kparts 0 takes the library's rule.
EXACT_FORMS = [
    ("valu", 2, 3, 5, 7, 1), ("valu", 1, 1, 1, 1024, 1),
    ("skinny", 2, 4, 512, 33, 1), ("skinny", 1, 16, 300, 7, 1),
    ("skinny_t", 2, 512, 4, 33, 1), ("skinny_t", 3, 300, 16, 7, 1), ("skinny_t", 1, 256, 8, 64, 1),
    ("skinny_t", 1, 2048, 8, 12, 1), ("skinny_t", 2, 1024, 1, 5, 1), ("skinny", 2, 2, 1536, 9, 1),
    ("rows", 2, 512, 4, 33, 1), ("rows", 3, 300, 16, 7, 1), ("rows", 1, 256, 8, 4100, 1), ("rows", 2, 64, 1, 2, 1),
    ("rows", 1, 2048, 16, 24, 1), ("rows", 2, 768, 2, 9, 1),
    ("dot", 2, 2, 2, 5000, 1), ("dot", 1, 1, 1, 1 << 20, 0),
    ("dot_tile", 4, 16, 16, 4096, 1), ("dot_tile", 2, 32, 8, 2048, 1), ("dot_tile", 1, 1, 256, 300, 1),
    ("dot_tile", 3, 5, 7, 1000, 1), ("dot_tile", 2, 32, 8, 1 << 16, 0), ("dot_tile", 32, 16, 16, 16384, 0),
    ("mfma11", 2, 64, 64, 48, 1), ("mfma12", 1, 32, 64, 16, 1), ("mfma21", 3, 64, 32, 8, 1),
    ("mfma22", 1, 128, 64, 4, 1), ("mfma11", 1, 32, 32, 4096, 8),
    ("mfma_big", 1, 128, 256, 64, 1), ("mfma_big", 2, 128, 128, 8, 1), ("mfma_big", 1, 128, 128, 1024, 4),
    ("tile256x64", 2, 512, 64, 40, 1), ("tile64x256", 1, 64, 512, 16, 1), ("tile32x256", 3, 32, 256, 24, 1),
    ("tile256x32", 1, 256, 96, 64, 1), ("tile128x64", 2, 256, 64, 8, 1), ("tile64x128", 1, 128, 128, 512, 4),
    ("tile32x256", 1, 64, 512, 256, 8), ("tile128x32", 2, 256, 96, 32, 1), ("tile32x128", 1, 96, 256, 8, 1),
    ("tile128x32", 1, 128, 32, 2048, 4),
    ("mfma16", 2, 64, 16, 64, 1), ("mfma16", 1, 32, 8, 20, 1), ("mfma16", 3, 48, 32, 12, 1), ("mfma16", 1, 16, 16, 8, 1),
    ("mfma16", 4, 16, 16, 4096, 4), ("mfma16_t", 2, 16, 256, 64, 1), ("mfma16_t", 1, 8, 64, 36, 1),
    ("mfma16_t", 2, 32, 48, 4, 1),
    # Streaming form: every (n, k) instance; ranges of row blocks that cross
    # batch entries (B reloaded), and more row blocks than waves.
    ("stream", 2, 64, 32, 8, 1), ("stream", 1, 96, 32, 16, 1), ("stream", 3, 32, 32, 32, 1),
    ("stream", 2, 128, 64, 8, 1), ("stream", 5, 96, 64, 16, 1), ("stream", 1, 64, 64, 32, 1),
    ("stream", 3, 22400, 64, 16, 1), ("stream", 2, 40000, 32, 32, 1), ("stream", 2, 96, 32, 64, 1),
    ("stream", 3, 20000, 32, 64, 1), ("stream_t", 2, 32, 128, 64, 1),
    ("stream_t", 2, 32, 64, 8, 1), ("stream_t", 3, 64, 96, 32, 1), ("stream_t", 2, 32, 30016, 16, 1),
    ("stream16", 2, 64, 16, 64, 1), ("stream16", 1, 48, 8, 20, 1), ("stream16", 3, 32, 16, 12, 1),
    ("stream16", 1, 16, 8, 4, 1), ("stream16", 2, 96, 16, 44, 1), ("stream16", 3, 40000, 16, 32, 1),
    ("stream16", 2, 60000, 8, 64, 1), ("stream16", 5, 4096, 16, 8, 1),
]


@pytest.mark.parametrize("case", EXACT_FORMS, ids=lambda c: "-".join(str(v) for v in c))
@pytest.mark.parametrize("a_km,b_nk", [(0, 0), (1, 1), (1, 0), (0, 1)])
def test_fp32_forms_exact_on_integer_operands(case, a_km, b_nk):
    form, nb, m, n, k, kp = case
    r = max(1, int(np.sqrt((2.0 ** 23 - 1) / k)))
    rng = np.random.default_rng(nb + 7 * m + 13 * n + 17 * k + 3 * a_km + 5 * b_nk)
    ia = rng.integers(-r, r + 1, size=(2, nb, m, k))
    ib = rng.integers(-r, r + 1, size=(2, nb, k, n))
    A = (ia[0] + 1j * ia[1]).astype(np.complex64)
    B = (ib[0] + 1j * ib[1]).astype(np.complex64)
    a_store = A.transpose(0, 2, 1) if a_km else A
    b_store = B.transpose(0, 2, 1) if b_nk else B
    dA = torch.from_numpy(np.ascontiguousarray(a_store).reshape(-1)).cuda()
    dB = torch.from_numpy(np.ascontiguousarray(b_store).reshape(-1)).cuda()
    dC = torch.full((nb * m * n,), float("nan"), dtype=torch.complex64, device="cuda")
    say(f"gemm {form} exact: nb={nb} m={m} n={n} k={k} kparts={kp} a_km={a_km} b_nk={b_nk}")
    qcsim.qc_kernel_gemm(dA, dB, dC, nb, m, n, k, a_km, b_nk, form=qcsim.GEMM_FORMS[form], kparts=kp)
    torch.cuda.synchronize()
    got = dC.cpu().numpy().reshape(nb, m, n).astype(np.complex128)
    ref = np.matmul(A.astype(np.complex128), B.astype(np.complex128))
    assert np.abs(ref.real).max() < 2 ** 24 and np.abs(ref.imag).max() < 2 ** 24
    assert np.array_equal(got, ref), np.abs(got - ref).max()


def test_stream_records_output_max():
    # In a split FP16 program the streaming form (FP32) records max(|re|, |im|)
    # of its output for a later 16-bit step.
    nb, m, n, k = 2, 4096, 64, 32
    rng = np.random.default_rng(5)
    A = _rand(rng, (nb, m, k))
    B = _rand(rng, (nb, k, n))
    dA = torch.from_numpy(A.reshape(-1)).cuda()
    dB = torch.from_numpy(B.reshape(-1)).cuda()
    dC = torch.full((nb * m * n,), float("nan"), dtype=torch.complex64, device="cuda")
    slots = torch.zeros(3, dtype=torch.int32, device="cuda")
    say("gemm stream split_fp16 output max")
    qcsim.qc_kernel_gemm(dA, dB, dC, nb, m, n, k, prec="split_fp16", scale_ws=slots, form=qcsim.GEMM_FORMS["stream"])
    torch.cuda.synchronize()
    got = dC.cpu().numpy().reshape(nb, m, n)
    ref = np.matmul(A.astype(np.complex128), B.astype(np.complex128))
    assert np.abs(got - ref).max() <= fp32_sum_tol(k)
    s = slots.cpu().numpy().view(np.float32)
    assert s[2] == np.float32(max(np.abs(got.real).max(), np.abs(got.imag).max()))
