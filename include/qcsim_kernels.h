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
 * [nb][k][n] (b_nk = 0) or [nb][n][k] (b_nk = 1); C is [nb][m][n].  All
 * extents >= 1.  prec selects complex FP32 or a split form (hi/lo BF16 or
 * FP16 operands with FP32 accumulation, per-call power-of-two scaling). */
qc_status qc_kernel_gemm(const void *A, const void *B, void *C, int64_t nb, int64_t m, int64_t n, int64_t k,
                         int32_t a_km, int32_t b_nk, qc_precision prec, void *stream);

/* Bit-permuting transpose of a rank-r tensor (2^r complex64 values): the
 * value at input offset i goes to the output offset whose bit perm[p] equals
 * bit p of i, for p = 0..r-1 (bit 0 = least significant).  perm is a host
 * array, a permutation of 0..r-1; 0 <= r <= 40. */
qc_status qc_kernel_transpose(const void *in, void *out, int32_t rank, const int32_t *perm, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* QCSIM_KERNELS_H */
