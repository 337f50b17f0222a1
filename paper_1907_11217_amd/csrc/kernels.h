// Device-side descriptors shared by the kernels and the runtime that fills
// them.  Plain structs, no torch types.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace qc {

constexpr int kLeafMaxRank = 40;
constexpr int kLeafMaxBase = 8;

// One leaf tensor to instantiate for a chunk of slices and bitstrings.
struct LeafDesc {
    int64_t out_off;             // complex64 element offset in the tensor region
    int32_t base_off;            // offset into the base-value table (complex double)
    int32_t r_out;               // output rank
    int32_t n_fix;               // base bits fixed by the chunk's slice id
    int32_t n_oq;                // base bits fixed by a qubit of the bitstring
    int32_t pad0, pad1;
    int8_t src[kLeafMaxRank];    // output bit p -> base bit, or 64 + bitstring bit
    int8_t fix_pos[kLeafMaxBase];
    int8_t fix_j[kLeafMaxBase];  // slice bit j (< 64)
    int8_t oq_pos[kLeafMaxBase];
    int16_t oq_q[kLeafMaxBase];
};

// Bit permutation out[perm(i)] = in[i] of a rank-r complex64 tensor, staged
// through LDS one tile at a time.  Tile bits = the input's lowest bits plus the
// output's lowest bits; the remaining bits enumerate tiles.
constexpr int kTransMaxTile = 10;
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
struct GemmDesc {
    const float2 *A;
    const float2 *B;
    float2 *C;
    int64_t nb, m, n, k;
    int64_t sAb, sAm, sAk;
    int64_t sBb, sBk, sBn;
    int64_t sCb, sCm, sCn;
};

// Fused form: one wavefront runs a whole lowered program for one group of
// 2^bf slices x 2^mf bitstrings with every tensor in LDS, contracting each
// step directly from the operands' own layouts (no transposes).
constexpr int kFusedMaxRank = 16;
constexpr int kFusedMaxK = 12;
constexpr int kFusedLdsBytes = 64 * 1024;
struct FusedStep {
    int32_t a_off, b_off, c_off;             // LDS element offsets
    int32_t rc, rk;                          // log2 of C's size and of the contracted extent
    int32_t sA[kFusedMaxRank], sB[kFusedMaxRank];   // C bit p -> element stride in A / B (0 = absent)
    int32_t kA[kFusedMaxK], kB[kFusedMaxK];         // contracted bit j -> stride in A / B
};

struct FusedParams {
    const FusedStep *steps;
    int32_t n_steps;
    const LeafDesc *leaves;                  // out_off = LDS offset, pad1 = first flat element
    const int32_t *elem_leaf;                // flat leaf element -> leaf
    int32_t n_elems;
    const double2 *base;
    const uint8_t *bits;                     // [2^m][n_qubits]
    int32_t n_qubits;
    int32_t bf, mf;                          // log2 slices / bitstrings per group
    int32_t n_bs_groups;                     // 2^(m - mf)
    int64_t first_group, n_slice_groups;    // slice groups relative to sc
    uint64_t sc;                             // super-chunk base slice id
    int32_t root_off, root_rank;
    int8_t root_map[32];                     // root bit p -> slice bit j, or 64 + bitstring bit
    float2 *partial;                         // [slice - sc][2^m]
    int32_t m;
    int32_t lds_elems;
};

void launch_fused(const FusedParams &p, hipStream_t st);
// out[bs] += sum of partial over in-range slices of the super-chunk, in
// aligned blocks of 64 slices: a fixed butterfly within each block, blocks
// added in increasing order.
void launch_reduce64(const float2 *partial, int m, int n_bs, uint64_t sc, int64_t n_blocks, uint64_t lo, uint64_t hi,
                     uint64_t s_begin, double *out, double *per_slice, hipStream_t st);

void launch_leaves(const LeafDesc *descs, const int32_t *block_leaf, int n_blocks, const double2 *base,
                   float2 *tensors, const uint8_t *bits, int n_qubits, uint64_t chunk_base, hipStream_t st);
void launch_transpose(const TransposeDesc &d, hipStream_t st);
const char *launch_gemm(const GemmDesc &d, hipStream_t st);  // returns the form launched
void launch_reduce(const float2 *root, int b, int m, int n_bs, uint64_t chunk_base, uint64_t s_begin,
                   uint64_t s_end, double *out, double *per_slice, hipStream_t st);

}  // namespace qc
