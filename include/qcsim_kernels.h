/*
 * Kernel-level entry points of libqcsim.so: one step kernel per call on
 * caller-owned device buffers, for unit tests and tuning.  Same error rules as
 * qcsim.h (status codes, qc_last_error, asynchronous on `stream`).
 *
 * Tensors are complex64, interleaved (re, im) float pairs.
 */
#ifndef QCSIM_KERNELS_H
#define QCSIM_KERNELS_H

#include <stdint.h>

#include "qcsim.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One pairwise contraction step as a batched complex GEMM (the step of the
 * contraction tree after its operands are grouped into batch, free and
 * contracted indices):
 *   C[b][i][j] = sum_l A[b][i][l] * B[b][l][j],  0 <= b < nb, i < m, j < n, l < k.
 * A is stored [nb][m][k] (a_km = 0) or [nb][k][m] (a_km = 1); B is stored
 * [nb][k][n] (b_nk = 0) or [nb][n][k] (b_nk = 1); C is [nb][m][n]; all are
 * caller-owned device buffers, extents >= 1.
 *
 * prec = QC_C64: complex FP32 (MFMA when m and n are multiples of 32 and k is
 * 2, 4, 8 or a multiple of 16; else the vector ALU).  prec = QC_SPLIT_BF16 or
 * QC_SPLIT_FP16: when m and n are multiples of 32 and k >= 2, each real
 * operand value x is written as x 2^-d = h + l (h = rn(x 2^-d), l = rn(x 2^-d
 * - h) in the 16-bit type), each real product is h h' + h l' + l h' with FP32
 * accumulation on MFMA, and C is complex FP32 scaled back by 2^(d_A + d_B);
 * d = 0 for BF16, d = floor(log2 max|x|) - 14 over the whole operand for FP16
 * (max over real and imaginary parts; d = 0 for a zero operand).  Other
 * shapes use the FP32 vector-ALU form.
 *
 * scale_ws: device buffer of 3 uint32, required for QC_SPLIT_FP16, optional
 * otherwise (NULL).  When given, the call overwrites it with the float bits
 * of max(|re|, |im|) over A, over B, and over the C it writes. */
qc_status qc_kernel_gemm(const void *A, const void *B, void *C, int64_t nb, int64_t m, int64_t n, int64_t k,
                         int32_t a_km, int32_t b_nk, qc_precision prec, void *scale_ws, void *stream);

/* qc_kernel_gemm with the kernel form fixed (the choices qc_tune times):
 *   0 vector ALU (any shape), 1 skinny (m in {1,2,4,8,16}, n >= 64),
 *   2 dot (k >= 256, nb m n <= 65536), 3..6 complex FP32 MFMA with block
 *   tiles 32x32, 32x64, 64x32, 64x64 (k in {2,4,8} or a multiple of 16),
 *   7 split 128x128 (split precisions, k a multiple of 8), 8..11 split 32x32,
 *   32x64, 64x32, 64x64 (split precisions, k >= 2), 12 complex FP32 MFMA
 *   128x128 (k a multiple of 8, m and n multiples of 128), 13 skinny on the
 *   transposed product (n in
 *   {1,2,4,8,16}, m >= 64), 14 dot tile (m n <= 256, k >= 64: one workgroup
 *   per batch entry's whole tile, k staged through LDS), 15 rows (n in
 *   {1,2,4,8,16}, m >= 64: one row of C per thread, B in LDS), 16..23
 *   complex FP32 MFMA with tall or wide tiles 256x64, 64x256, 32x256, 256x32,
 *   128x64, 64x128, 128x32, 32x128 (k a multiple of 8, m and n multiples of
 *   the tile: the
 *   128x128 form's double-buffered slabs for shapes with one short output
 *   dimension), 24 16-wide MFMA (n = 8 or a multiple of 16, m a multiple of
 *   16, k a multiple of 4: one 16x16 tile per wave on
 *   v_mfma_f32_16x16x4_f32, operands read straight into registers), 25 the
 *   same on the transposed product (m = 8 or a multiple of 16, n a multiple
 *   of 16), 26 streaming complex FP32 MFMA (n = 32 or 64 with k in {8,16,32},
 *   or n = 32 with k = 64, m a multiple of 32: B held in registers, 32-row
 *   blocks of A streamed into the MFMA operands), 27 the same on the
 *   transposed product (m = 32 or 64), 28 streaming 16-wide MFMA (n = 8 or
 *   16, k <= 64 a multiple of 4, m a multiple of 16); form -1 is the default
 *   choice.  Every form but 7..11 computes
 *   in complex FP32 for every
 *   precision.  QC_ERR_UNSUPPORTED if the form does not apply to the shape and
 *   precision. */
qc_status qc_kernel_gemm_form(const void *A, const void *B, void *C, int64_t nb, int64_t m, int64_t n, int64_t k,
                              int32_t a_km, int32_t b_nk, qc_precision prec, int32_t form, void *scale_ws,
                              void *stream);

/* qc_kernel_gemm_form split over k, as the stepwise contraction runs its
 * GEMM steps with few outputs: every MFMA form (3-12, 16-25; not the
 * streaming forms 26-28) and the dot forms (2, 14)
 * compute kparts partial products, part p over l in [p k/kparts,
 * (p+1) k/kparts), into `scratch`, then C = the parts summed in increasing p,
 * in FP32 (so the result is deterministic).  scratch: caller-owned device
 * buffer of kparts * nb * m * n complex64, contents afterwards unspecified.
 * kparts: a power of two dividing k, at most 1024; 0 takes
 * qc_gemm_kparts(nb, m, n, k); 1 is qc_kernel_gemm_form (scratch may then be
 * NULL).  QC_ERR_UNSUPPORTED when kparts > 1 and the form (given, or the
 * default) is none of these, kparts does not divide k, the form does not
 * apply to a part (k / kparts values of k), or scratch is NULL. */
qc_status qc_kernel_gemm_kparts(const void *A, const void *B, void *C, int64_t nb, int64_t m, int64_t n, int64_t k,
                                int32_t a_km, int32_t b_nk, qc_precision prec, int32_t form, int64_t kparts,
                                void *scratch, void *scale_ws, void *stream);

/* The number of k parts the stepwise contraction uses for a GEMM step of this
 * shape when it runs a form that splits: for m and n multiples of 128 with
 * fewer than 1024 tiles of 128x128, the smallest power of two p <= 64 with at
 * least 1024 tiles times p, while each part keeps at least 256 of k; else for
 * m and n multiples of 32 with fewer than 4096 tiles of 32x32, the smallest
 * power of two p <= 64 with at least 4096 tiles times p, while each part keeps
 * at least 256 of k; else for m n <= 256 and k >= 1024, the smallest power
 * of two p <= 1024 with nb p >= 1024, while each part keeps at least 256 of
 * k; else for at most 4096 outputs and k >= 8192, the smallest power of two p
 * with at least 1024 outputs times p, while each part keeps at least 4096 of
 * k; else 1.
 * The scratch for the largest such step is part of qc_workspace_bytes. */
int64_t qc_gemm_kparts(int64_t nb, int64_t m, int64_t n, int64_t k);

/* Bit-permuting transpose of a rank-r tensor (2^r complex64 values): the
 * value at input offset i goes to the output offset whose bit perm[p] equals
 * bit p of i, for p = 0..r-1 (bit 0 = least significant).  perm is a host
 * array, a permutation of 0..r-1; 0 <= r <= 40. */
qc_status qc_kernel_transpose(const void *in, void *out, int32_t rank, const int32_t *perm, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* QCSIM_KERNELS_H */
