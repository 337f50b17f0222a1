// Device-side descriptors shared by the kernels and the runtime that fills
// them.  Plain structs, no torch types.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace qc {

constexpr int kLeafMaxRank = 40;
constexpr int kLeafMaxBase = 16;  // folded leaves carry up to 14 indices

// One leaf tensor to instantiate for a chunk of slices and bitstrings.
struct LeafDesc {
    int64_t out_off;             // complex64 element offset in the tensor region
    int32_t base_off;            // offset into the base-value table (complex double)
    int32_t r_out;               // output rank
    int32_t n_fix;               // base bits fixed by the chunk's slice id
    int32_t n_oq;                // base bits fixed by a qubit of the bitstring
    int32_t first_block;         // stepwise form: first block of this leaf in the launch
    int32_t amax_slot;           // stepwise form: max|x| slot of this leaf's tensor
    int8_t src[kLeafMaxRank];    // output bit p -> base bit, or 64 + bitstring bit
    int8_t fix_pos[kLeafMaxBase];
    int8_t fix_j[kLeafMaxBase];  // slice bit j (< 64)
    int8_t oq_pos[kLeafMaxBase];
    int16_t oq_q[kLeafMaxBase];
};

// Bit permutation out[perm(i)] = in[i] of a rank-r complex64 tensor, staged
// through LDS one tile at a time.  Tile bits = the input's lowest bits plus the
// output's lowest bits; the remaining bits enumerate tiles.
constexpr int kTransMaxTile = 12;    // tile bits of tensors of rank >= 12 (16-byte accesses)
constexpr int kTransSmallTile = 10;  // tile bits of smaller tensors (all of them up to rank 10)
struct TransposeDesc {
    const float2 *in;
    float2 *out;
    int32_t n_tile;                          // tile bits
    int32_t n_rest;                          // remaining bits (tile id)
    int64_t n_tiles;                         // 2^n_rest
    // Tile bits listed in input order (lowest input position first).
    int64_t tin_in[kTransMaxTile];           // input stride of tile bit i (input order)
    int64_t tin_out_lds[kTransMaxTile];      // unused (reserved)
    // Tile bits listed in output order.
    int64_t tout_out[kTransMaxTile];         // output stride
    int32_t tout_lds[kTransMaxTile];         // LDS stride (= 1 << rank in input order)
    int64_t rest_in[40];                     // input stride of rest bit j
    int64_t rest_out[40];                    // output stride of rest bit j
};

// Batched complex GEMM C[b][m][n] = sum_k A[b][m][k] B[b][k][n] (element
// strides, complex64 interleaved).
//
// Split precision (prec = 1 BF16, 2 FP16): every real operand value x is
// scaled by 2^-d of its tensor and split as h = rn(x 2^-d), l = rn(x 2^-d - h)
// in the 16-bit type; each real product is accumulated in FP32 as
// h h' + h l' + l h' and the result scaled back by 2^(d_A + d_B).  d = 0 for
// BF16 (FP32's exponent range); for FP16 d = floor(log2 max|x|) - 14, so the
// largest |x| 2^-d lies in [2^14, 2^15).  max|x| of each tensor comes from
// amax_* (the float bits of max(|re|, |im|) over the tensor, kept by the
// kernel that wrote it); a kernel that writes C with amax_c set folds its
// outputs in with atomicMax.
enum GemmPrec { kPrecC64 = 0, kPrecBF16 = 1, kPrecFP16 = 2 };
constexpr int kGemmMaxBits = 40;
struct GemmDesc {
    const float2 *A;
    const float2 *B;
    float2 *C;
    int64_t nb, m, n, k;
    int64_t sAb, sAm, sAk;
    int64_t sBb, sBk, sBn;
    int64_t sCb, sCm, sCn;
    int32_t prec;
    const uint32_t *amax_a, *amax_b;
    uint32_t *amax_c;
    // Split over k (the large-tile and dot forms only): with kparts > 1 and a
    // scratch buffer of kparts * nb * m * n complex64, the product runs as
    // nb * kparts partial products of k / kparts into the scratch, then a sum
    // over the parts in increasing order writes C.
    // Other forms ignore these fields.
    int64_t kparts = 1;
    float2 *kscratch = nullptr;
    int64_t sAp = 0, sBp = 0;   // operand offset between k parts (set by the launch)
    // Output scatter (cscatter = 1; nb, m, n powers of two): element (b, i, j)
    // of C has the flat index f = (b m + i) n + j, whose bits (cbn bits of j
    // least significant, then cbm of i, then cbb of b) go to bit positions
    // cpos[t] of the element's offset in C.  The strides sC* are then unused.
    int32_t cscatter = 0;
    int32_t cbb = 0, cbm = 0, cbn = 0;
    int8_t cpos[kGemmMaxBits] = {};
};

// Records max(|re|, |im|) of n values into *amax (atomicMax on float bits).
void launch_absmax(const float2 *x, int64_t n, uint32_t *amax, hipStream_t st);
// Sets n uint32 to zero (a fill kernel, so the op can sit in a captured graph).
void launch_zero_u32(uint32_t *p, int64_t n, hipStream_t st);
// dst[i] = src[i] for n complex64 values (a kernel, for the same reason).
void launch_copy(float2 *dst, const float2 *src, int64_t n, hipStream_t st);

// Fused form: one wavefront runs the whole program of (slice, bitstring)
// pairs with every tensor in LDS, contracting each step directly from the
// operands' own layouts (no transposes).  Steps are grouped into levels of
// the contraction tree (a step's level is one more than its operands'), and
// all outputs of one level are computed together, one per lane, with one
// wavefront-scope fence per level.  Each output is an item (int4):
//   x = out slot | nk << 16  (nk = number of contracted values)
//   y = a0 | b0 << 16        (operand slots of the first contracted value)
//   z = a1 | b1 << 16        (second value; the pair's zero slot when nk = 1)
//   w = pool index of the values past the fourth (count, then nk - 4 slot
//       pairs), or -1
// with a companion int2 (a2 | b2 << 16, a3 | b3 << 16) holding the third and
// fourth values when nk >= 4, read in the same round trip as the item.
// Slots are byte offsets inside one pair's LDS region (below 2^16, a region
// being at most 64 KiB).
constexpr int kFusedLdsBytes = 64 * 1024;

struct FusedParams {
    const int32_t *level_start;              // n_levels + 1 item offsets
    int32_t n_levels;
    const int4 *items;
    const int2 *items2;                      // third and fourth operand slots per item
    const int32_t *pool;
    const float2 *leaf_image;                // LDS [0, n_image): leaf values that do not depend on the pair
    int32_t n_image;
    const int4 *elems;                       // run-time leaf elements: (LDS slot, base index, dyn0, dyn1)
    int32_t n_elems;
    const double2 *base;
    const uint8_t *bits;                     // [n_bs][n_qubits]
    int32_t n_qubits;
    int32_t n_bs;
    int32_t m;                               // log2 padded bitstrings (rows of partial)
    int64_t first_slice, n_slices;           // chunks of 2^b slices, relative to sc
    uint64_t sc;                             // super-chunk base slice id
    int32_t b;                               // log2 slices per work item
    int32_t root_off;
    float2 *partial;                         // [slice - sc][2^m]
    int32_t lds_elems;
    // Set when each work item is exactly one 64-slice block (b = 6) and the
    // launch holds one block per bitstring: the kernel sums the block itself
    // (the reduction's butterfly and order) into out[bs] (and per_slice), for
    // slices in [lo, hi); partial is then not written.
    double *out = nullptr;
    double *per_slice = nullptr;
    uint64_t lo = 0, hi = 0, s_begin = 0;
};

// The scalar part of FusedParams, passed by value next to the tables (which
// go as separate read-only kernel arguments so that uniform reads of them
// become scalar loads).
struct FusedScalars {
    int32_t n_levels, n_image, n_elems, n_qubits, m, root_off, pair_elems, zero_slot;
    int32_t n_bs;                            // rows of bits; padded bitstrings reuse the last row
    int32_t b;                               // log2 slices per work item (in the program's layouts)
    int64_t first_slice, n_slices;           // in chunks of 2^b slices, relative to sc
    uint64_t sc;
    uint64_t lo, hi, s_begin;                // slice range (block sums in the kernel)
};

// Work-item shapes the fused kernel is built for, (work items per workgroup,
// wavefronts per work item): one wavefront running
// 1, 2 or 4 work items, or 2, 4, 8 or 16 wavefronts sharing one work item's levels.
// The runtime times them on first use of a program and keeps the fastest.
constexpr int kFusedShapes[][2] = {{1, 1}, {2, 1}, {4, 1}, {1, 2}, {1, 4}, {1, 8}, {1, 16}};
size_t fused_lds_bytes(int pairs, int pair_elems);
void launch_fused_pairs(const FusedParams &p, int pairs, int waves, int pair_elems, int zero_slot, hipStream_t st);

// One small GEMM step computed by the micro-step kernel straight from its
// operands' layouts: output element o (bit p of o = bit p of C's layout,
// least significant first) reads A at a + sum of sa[p] over set bits, B at
// b + sum of sb[p]; contracted value j adds ka[q], kb[q] for set bits q.
constexpr int kMicroRank = 12;
struct MicroStep {
    int64_t a, b, c;                         // element offsets in the tensor region
    int32_t rc, rk, out0, amax_slot;         // out0: first flat output of this step in its level
    int32_t sa[kMicroRank], sb[kMicroRank], ka[kMicroRank], kb[kMicroRank];
};
// Micro steps in groups of independent subtrees, one workgroup per group:
// group g runs levels [group_start[g], group_start[g + 1]) in order (a
// barrier between levels), level l holds steps [level_start[l],
// level_start[l + 1]) with level_outs[l] outputs in all; amax (or null) as
// for the GEMM epilogues.
constexpr int kMicroGroups = 1024;
void launch_micro(const MicroStep *steps, const int32_t *group_start, const int32_t *level_start,
                  const int32_t *level_outs, int n_groups, float2 *tensors, uint32_t *amax, hipStream_t st);

// Device descriptor of one request of a fused batch (one bitstring).  Its
// slice values go to partial[partial_off + (s - s_base)], s_base = s_begin
// rounded down to a multiple of 64.
struct BatchReq {
    const int32_t *level_start;
    const int4 *items;
    const int2 *items2;                      // third and fourth operand slots per item
    const int32_t *pool;
    const float2 *image;
    const int4 *elems;
    const double2 *base;
    const uint8_t *bits;                     // device copy of the bitstring
    int32_t n_levels, n_image, n_elems, root_off, zero_slot, out_index;  // out_index: position in the caller's array
    uint64_t s_begin, s_base;
    int64_t n_slices, item_off, partial_off;
};
void launch_fused_batch(const BatchReq *reqs, int n_reqs, int64_t n_items, int max_pair_elems, float2 *partial,
                        uint32_t *done, uint64_t *t_done, hipStream_t st);
void launch_reduce_batch(const BatchReq *reqs, int n_reqs, const float2 *partial, double *out, hipStream_t st);
// t[0] = the device wall clock (constant rate, hipDeviceAttributeWallClockRate kHz).
void launch_stamp(uint64_t *t, hipStream_t st);

// out[bs] += sum of partial over in-range slices of the super-chunk, in
// aligned blocks of 64 slices: a fixed butterfly within each block, blocks
// added in increasing order.  bsum: scratch of n_blocks * n_bs double2.
void launch_reduce64(const float2 *partial, int m, int n_bs, uint64_t sc, int64_t n_blocks, uint64_t lo, uint64_t hi,
                     uint64_t s_begin, double *out, double *per_slice, double2 *bsum, hipStream_t st);

// amax: per program tensor slots (indexed by leaf tensor id), or null.
void launch_leaves(const LeafDesc *descs, const int32_t *block_leaf, int n_blocks, const double2 *base,
                   float2 *tensors, const uint8_t *bits, int n_qubits, int n_bs, uint64_t chunk_base,
                   uint32_t *amax, hipStream_t st);
void launch_transpose(const TransposeDesc &d, hipStream_t st);
const char *launch_gemm(const GemmDesc &d, hipStream_t st);  // returns the form launched

// GEMM kernel forms (tuning choices).  Mfma/Split WM WN: complex FP32 or
// split 16-bit MFMA with a (32 WM) x (32 WN) block tile; SplitBig, MfmaBig:
// the 128 x 128 tiles; Skinny: m <= 16; Dot: few outputs, long k; Valu: any.
enum GemmVariant {
    kVarValu = 0, kVarSkinny, kVarDot, kVarMfma11, kVarMfma12, kVarMfma21, kVarMfma22,
    kVarSplitBig, kVarSplit11, kVarSplit12, kVarSplit21, kVarSplit22, kVarMfmaBig,
    kVarSkinnyT,   // the skinny form on the transposed problem (C^T = B^T A^T): n <= 16, wide m
    kVarDotTile,   // small output tile (m n <= 256 per batch), long k: A and B k-chunks through LDS
    kVarRows,      // n <= 16, tall m: B in LDS, one row of C per thread, A rows read once
    // Tall and wide tiles of the complex FP32 MFMA product (TM x TN):
    kVarT256x64, kVarT64x256, kVarT32x256, kVarT256x32, kVarT128x64, kVarT64x128, kVarT128x32, kVarT32x128,
    kVarMfma16,    // one 16x16 tile per wave on v_mfma_f32_16x16x4_f32 (n = 8 or n % 16 = 0), operands in registers
    kVarMfma16T,   // the same on the transposed product (m = 8 or m % 16 = 0)
    kVarStream,    // n = 32 or 64 with k = 8, 16 or 32, n = 32 with k = 64: B in registers, 32-row blocks of A streamed through MFMA
    kVarStreamT,   // the same on the transposed product (m = 32 or 64)
    kVarStream16,  // n = 8 or 16, k <= 64: the same scheme on v_mfma_f32_16x16x4_f32
    kVarSplitBig64,  // split 16-bit MFMA with a 128x64 tile (two waves per SIMD), m % 128 = n % 64 = 0
    kVarCount
};
bool gemm_variant_ok(const GemmDesc &d, int v);
int gemm_default_variant(const GemmDesc &d);
// Whether form v multiplies on 16-bit MFMA (and so reads its operands' recorded maxima).
bool gemm_variant_16bit(int v);
const char *launch_gemm_variant(const GemmDesc &d, int v, hipStream_t st);

}  // namespace qc
