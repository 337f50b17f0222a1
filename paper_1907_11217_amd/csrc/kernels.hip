// Step kernels for gfx950: leaf instantiation, LDS-staged bit-permuting
// transpose, complex batched GEMM (FP32 MFMA, split BF16/FP16 MFMA, and a VALU
// form for shapes below the MFMA tile), and the FP64 cross-slice reduction.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace qc {

// ------------------------------------------------------------------ leaves
// Each leaf is a base tensor (<= 8 binary indices, complex double) whose bits
// are either kept (summed indices, possibly in-flight slice bits), fixed by
// the chunk's slice id (sliced segments not in flight), or fixed by the
// bitstring (output segments); the bitstring bits of the batch become extra
// output bits.  One thread per output element.
// max(|re|, |im|) of the workgroup's values folded into *amax with one
// atomic per workgroup (uint32 order of non-negative floats is their numeric
// order).  Every thread of the workgroup must call it.
__device__ __forceinline__ void block_amax(float v, uint32_t *amax) {
    __shared__ float part[16];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < int(blockDim.x + 63) / 64; ++w) v = fmaxf(v, part[w]);
        atomicMax(amax, __float_as_uint(v));
    }
}

__global__ void __launch_bounds__(256) leaf_kernel(const LeafDesc *__restrict__ descs,
                                                   const int32_t *__restrict__ block_leaf,
                                                   const double2 *__restrict__ base, float2 *__restrict__ tensors,
                                                   const uint8_t *__restrict__ bits, int n_qubits, int n_bs,
                                                   uint64_t chunk_base, uint32_t *__restrict__ amax) {
    const int leaf = block_leaf[blockIdx.x];
    const LeafDesc &d = descs[leaf];
    const int64_t e = int64_t(blockIdx.x - d.first_block) * blockDim.x + threadIdx.x;
    float mx = 0.f;
    if (e < (int64_t(1) << d.r_out)) {
        int bs = 0, bidx = 0;
        for (int p = 0; p < d.r_out; ++p) {
            const int bit = int((e >> p) & 1);
            const int s = d.src[p];
            if (s >= 64) bs |= bit << (s - 64);
            else bidx |= bit << s;
        }
        bs = min(bs, n_bs - 1);  // padded bitstrings repeat the last one (their results are dropped)
        for (int i = 0; i < d.n_fix; ++i) bidx |= int((chunk_base >> d.fix_j[i]) & 1) << d.fix_pos[i];
        for (int i = 0; i < d.n_oq; ++i) bidx |= int(bits[int64_t(bs) * n_qubits + d.oq_q[i]] & 1) << d.oq_pos[i];
        const double2 v = base[d.base_off + bidx];
        const float2 f = make_float2(float(v.x), float(v.y));
        tensors[d.out_off + e] = f;
        mx = fmaxf(fabsf(f.x), fabsf(f.y));
    }
    if (amax) block_amax(mx, amax + d.amax_slot);
}

void launch_leaves(const LeafDesc *descs, const int32_t *block_leaf, int n_blocks, const double2 *base,
                   float2 *tensors, const uint8_t *bits, int n_qubits, int n_bs, uint64_t chunk_base,
                   uint32_t *amax, hipStream_t st) {
    if (n_blocks <= 0) return;
    hipLaunchKernelGGL(leaf_kernel, dim3(n_blocks), dim3(256), 0, st, descs, block_leaf, base, tensors, bits,
                       n_qubits, n_bs, chunk_base, amax);
}

// ------------------------------------------------------------ scale slots
__global__ void __launch_bounds__(256) absmax_kernel(const float2 *__restrict__ x, int64_t n, uint32_t *amax) {
    float mx = 0.f;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const float2 v = x[i];
        mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
    block_amax(mx, amax);
}

void launch_absmax(const float2 *x, int64_t n, uint32_t *amax, hipStream_t st) {
    int64_t grid = (n + 255) / 256;
    grid = grid < 1 ? 1 : (grid > 1024 ? 1024 : grid);
    hipLaunchKernelGGL(absmax_kernel, dim3((unsigned)grid), dim3(256), 0, st, x, n, amax);
}

__global__ void __launch_bounds__(256) zero_u32_kernel(uint32_t *p, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = 0u;
}

__global__ void __launch_bounds__(256) copy_kernel(float2 *__restrict__ dst, const float2 *__restrict__ src, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        dst[i] = src[i];
}

void launch_copy(float2 *dst, const float2 *src, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    int64_t grid = (n + 255) / 256;
    grid = grid > 4096 ? 4096 : grid;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)grid), dim3(256), 0, st, dst, src, n);
}

void launch_zero_u32(uint32_t *p, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    int64_t grid = (n + 255) / 256;
    grid = grid > 1024 ? 1024 : grid;
    hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)grid), dim3(256), 0, st, p, n);
}

// ------------------------------------------------------ GEMM output address
// Offset of the bits [first, first + nbits) of C's flat index, given as the
// value v of that bit group, under the output scatter (uniform loop: the
// positions are kernel arguments).
__device__ __forceinline__ int64_t scat_bits(const GemmDesc &d, uint64_t v, int first, int nbits) {
    int64_t o = 0;
    for (int t = 0; t < nbits; ++t) o += int64_t((v >> t) & 1) << d.cpos[first + t];
    return o;
}

// Offset of element (b, i, j) of C.
__device__ __forceinline__ int64_t c_off(const GemmDesc &d, int64_t bi, int64_t i, int64_t j) {
    if (!d.cscatter) return bi * d.sCb + i * d.sCm + j * d.sCn;
    return scat_bits(d, uint64_t(j), 0, d.cbn) + scat_bits(d, uint64_t(i), d.cbn, d.cbm) +
           scat_bits(d, uint64_t(bi), d.cbn + d.cbm, d.cbb);
}

// Addresses of a 32x32 MFMA output block with corner (row0, col0), both
// multiples of 32: accumulator entry v of a lane is row row0 + (v >> 2) * 8 +
// (lane >> 5) * 4 + (v & 3), column col0 + (lane & 31).  p is the lane's
// address for v = 0; the offsets of row bits 0, 1, 3 and 4 give the rest.
struct CBlock {
    float2 *p;
    int64_t r0, r1, r3, r4;
};

__device__ __forceinline__ CBlock c_block(const GemmDesc &d, int64_t bi, int64_t row0, int64_t col0, int lane) {
    CBlock o;
    if (!d.cscatter) {
        o.p = d.C + bi * d.sCb + (row0 + (lane >> 5) * 4) * d.sCm + (col0 + (lane & 31)) * d.sCn;
        o.r0 = d.sCm;
        o.r1 = 2 * d.sCm;
        o.r3 = 8 * d.sCm;
        o.r4 = 16 * d.sCm;
    } else {
        const int fm = d.cbn, fb = d.cbn + d.cbm;
        o.p = d.C + scat_bits(d, uint64_t(bi), fb, d.cbb) + scat_bits(d, uint64_t(row0), fm, d.cbm) +
              scat_bits(d, uint64_t(col0), 0, d.cbn) + scat_bits(d, uint64_t(lane & 31), 0, 5) +
              (int64_t(lane >> 5) << d.cpos[fm + 2]);
        o.r0 = int64_t(1) << d.cpos[fm];
        o.r1 = int64_t(1) << d.cpos[fm + 1];
        o.r3 = int64_t(1) << d.cpos[fm + 3];
        o.r4 = int64_t(1) << d.cpos[fm + 4];
    }
    return o;
}

__device__ __forceinline__ float2 *c_at(const CBlock &o, int v) {
    return o.p + ((v & 1) ? o.r0 : 0) + ((v & 2) ? o.r1 : 0) + ((v & 4) ? o.r3 : 0) + ((v & 8) ? o.r4 : 0);
}

// -------------------------------------------------------------- micro steps
// All small GEMM steps of a stepwise program in one launch: each workgroup
// runs one group of independent subtrees, its levels in order, the outputs of
// a level spread over the workgroup (steps of a level read only lower levels
// of the same subtree), the operands read in the layouts their producers
// wrote.  Every output is computed by one thread in a fixed order, so the
// result does not depend on the grouping.
__global__ void __launch_bounds__(1024) micro_kernel(const MicroStep *__restrict__ steps,
                                                     const int32_t *__restrict__ group_start,
                                                     const int32_t *__restrict__ level_start,
                                                     const int32_t *__restrict__ level_outs, float2 *tensors,
                                                     uint32_t *amax) {
    // Per-step maxima of a level gather in LDS first (one global atomic per
    // step); a level with more steps than fit uses global atomics directly.
    constexpr int kSlots = 1024;
    __shared__ uint32_t lmax[kSlots];
    for (int lv = group_start[blockIdx.x]; lv < group_start[blockIdx.x + 1]; ++lv) {
        const int s0 = level_start[lv], s1 = level_start[lv + 1];
        const bool local = amax && s1 - s0 <= kSlots;
        if (local) {
            for (int i = threadIdx.x; i < s1 - s0; i += blockDim.x) lmax[i] = 0u;
            __syncthreads();
        }
        for (int f = threadIdx.x; f < level_outs[lv]; f += blockDim.x) {
            int s = s0;
            while (s + 1 < s1 && steps[s + 1].out0 <= f) ++s;
            const MicroStep &M = steps[s];
            const int o = f - M.out0;
            int64_t oa = M.a, ob = M.b;
            for (int p = 0; p < M.rc; ++p)
                if ((o >> p) & 1) { oa += M.sa[p]; ob += M.sb[p]; }
            float re = 0.f, im = 0.f;
            for (int j = 0; j < (1 << M.rk); ++j) {
                int64_t xa = oa, xb = ob;
                for (int q = 0; q < M.rk; ++q)
                    if ((j >> q) & 1) { xa += M.ka[q]; xb += M.kb[q]; }
                const float2 x = tensors[xa], y = tensors[xb];
                re = fmaf(x.x, y.x, re);
                re = fmaf(-x.y, y.y, re);
                im = fmaf(x.x, y.y, im);
                im = fmaf(x.y, y.x, im);
            }
            tensors[M.c + o] = make_float2(re, im);
            const uint32_t mx = __float_as_uint(fmaxf(fabsf(re), fabsf(im)));
            if (local) atomicMax(&lmax[s - s0], mx);
            else if (amax) atomicMax(amax + M.amax_slot, mx);
        }
        __syncthreads();
        if (local) {
            for (int i = threadIdx.x; i < s1 - s0; i += blockDim.x) atomicMax(amax + steps[s0 + i].amax_slot, lmax[i]);
            __syncthreads();
        }
    }
}

void launch_micro(const MicroStep *steps, const int32_t *group_start, const int32_t *level_start,
                  const int32_t *level_outs, int n_groups, float2 *tensors, uint32_t *amax, hipStream_t st) {
    if (n_groups <= 0) return;
    hipLaunchKernelGGL(micro_kernel, dim3(n_groups), dim3(1024), 0, st, steps, group_start, level_start, level_outs,
                       tensors, amax);
}

// --------------------------------------------------------------- transpose
// A tile of 2^n_tile elements is read in input order (coalesced along the
// input's fastest bits), stored in LDS, then written in output order
// (coalesced along the output's fastest bits).  LDS rows of 32 complex values
// are padded by one entry to spread the strided phase-2 reads over banks.
// Every tile has the same shape, so each thread's element offsets inside a
// tile (at most four per thread) are computed once; per tile only the base
// offsets change, summed over the set bits of the tile id.
__device__ __forceinline__ int lds_pad(int t) { return t + (t >> 5); }

__global__ void __launch_bounds__(256) transpose_kernel(TransposeDesc d) {
    __shared__ float2 tile[(1 << kTransSmallTile) + (1 << kTransSmallTile) / 32];
    const int tsize = 1 << d.n_tile;
    constexpr int E = 4;  // (1 << kTransSmallTile) / 256, and 128 / 64 for the small form
    int64_t ioff[E], ooff[E];
    int ilds[E], olds[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int t = threadIdx.x + j * blockDim.x;
        int64_t io = 0, oo = 0;
        int l = 0;
        for (int i = 0; i < d.n_tile; ++i)
            if ((t >> i) & 1) { io += d.tin_in[i]; oo += d.tout_out[i]; l += d.tout_lds[i]; }
        ioff[j] = io;
        ilds[j] = lds_pad(t);
        ooff[j] = oo;
        olds[j] = lds_pad(l);
    }
    for (int64_t t_id = blockIdx.x; t_id < d.n_tiles; t_id += gridDim.x) {
        int64_t in_base = 0, out_base = 0;
        for (uint64_t rest = uint64_t(t_id); rest; rest &= rest - 1) {
            const int j = __builtin_ctzll(rest);
            in_base += d.rest_in[j];
            out_base += d.rest_out[j];
        }
#pragma unroll
        for (int j = 0; j < E; ++j)
            if (threadIdx.x + j * blockDim.x < tsize) tile[ilds[j]] = d.in[in_base + ioff[j]];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < E; ++j)
            if (threadIdx.x + j * blockDim.x < tsize) d.out[out_base + ooff[j]] = tile[olds[j]];
        __syncthreads();
    }
}

// Tiles of 2^12 elements (tensors of rank >= 12): both phases move pairs of
// elements with 16-byte accesses -- phase 1 pairs consecutive input elements
// (the tile holds input bit 0), phase 2 pairs consecutive output elements
// (the tile holds the input bit that becomes output bit 0) -- and each
// thread moves eight pairs per tile.  Pair j of thread t is element e = 2 t +
// 512 j of the tile in input order (phase 1) or output order (phase 2), so
// its offsets split into a per-thread part (bits 1..8) and a part shared by
// all threads (bits 9..11).
__global__ void __launch_bounds__(256) transpose_wide_kernel(TransposeDesc d) {
    constexpr int NT = 1 << kTransMaxTile, J = NT / 512;
    __shared__ float2 tile[NT + NT / 32];
    const int t = threadIdx.x;
    int64_t ilo = 0, olo = 0;
    int llo = 0;
#pragma unroll
    for (int i = 1; i < 9; ++i)
        if (((2 * t) >> i) & 1) { ilo += d.tin_in[i]; olo += d.tout_out[i]; llo += d.tout_lds[i]; }
    int64_t ihi[J], ohi[J];
    int lhi[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        ihi[j] = 0; ohi[j] = 0; lhi[j] = 0;
#pragma unroll
        for (int i = 9; i < kTransMaxTile; ++i)
            if (((512 * j) >> i) & 1) { ihi[j] += d.tin_in[i]; ohi[j] += d.tout_out[i]; lhi[j] += d.tout_lds[i]; }
    }
    const int l1 = d.tout_lds[0];  // input-order distance of the two elements of an output pair
    for (int64_t t_id = blockIdx.x; t_id < d.n_tiles; t_id += gridDim.x) {
        int64_t in_base = 0, out_base = 0;
        for (uint64_t rest = uint64_t(t_id); rest; rest &= rest - 1) {
            const int j = __builtin_ctzll(rest);
            in_base += d.rest_in[j];
            out_base += d.rest_out[j];
        }
        float4 v[J];
#pragma unroll
        for (int j = 0; j < J; ++j) v[j] = *(const float4 *)(d.in + in_base + ilo + ihi[j]);
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int e = 2 * t + 512 * j;
            tile[lds_pad(e)] = make_float2(v[j].x, v[j].y);
            tile[lds_pad(e + 1)] = make_float2(v[j].z, v[j].w);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int l = llo + lhi[j];
            const float2 a = tile[lds_pad(l)], b = tile[lds_pad(l + l1)];
            *(float4 *)(d.out + out_base + olo + ohi[j]) = make_float4(a.x, a.y, b.x, b.y);
        }
        __syncthreads();
    }
}

void launch_transpose(const TransposeDesc &d, hipStream_t st) {
    const int64_t grid = d.n_tiles < 65536 ? d.n_tiles : 65536;
    if (d.n_tile == kTransMaxTile) {
        hipLaunchKernelGGL(transpose_wide_kernel, dim3((unsigned)grid), dim3(256), 0, st, d);
        return;
    }
    // 256 threads for tiles of 256..1024 elements, 64 for smaller ones (at
    // most four elements per thread either way).
    const int threads = d.n_tile >= 8 ? 256 : 64;
    hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)grid), dim3(threads), 0, st, d);
}

// -------------------------------------------------------------- VALU GEMM
// One thread per output element; used when m or n is below the MFMA tile or
// k is 1.  FP32 complex accumulation in k order (also for the split
// precisions: these shapes gain nothing from 16-bit operands).
__global__ void __launch_bounds__(256) gemm_valu_kernel(GemmDesc d) {
    const int64_t total = d.nb * d.m * d.n;
    float mx = 0.f;
    for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < total;
         idx += int64_t(gridDim.x) * blockDim.x) {
        const int64_t ni = idx % d.n;
        const int64_t t = idx / d.n;
        const int64_t mi = t % d.m;
        const int64_t bi = t / d.m;
        const float2 *a = d.A + bi * d.sAb + mi * d.sAm;
        const float2 *b = d.B + bi * d.sBb + ni * d.sBn;
        float re = 0.f, im = 0.f;
        for (int64_t kk = 0; kk < d.k; ++kk) {
            const float2 x = a[kk * d.sAk];
            const float2 y = b[kk * d.sBk];
            re = fmaf(x.x, y.x, re);
            re = fmaf(-x.y, y.y, re);
            im = fmaf(x.x, y.y, im);
            im = fmaf(x.y, y.x, im);
        }
        d.C[c_off(d, bi, mi, ni)] = make_float2(re, im);
        mx = fmaxf(mx, fmaxf(fabsf(re), fabsf(im)));
    }
    if (d.amax_c) block_amax(mx, d.amax_c);
}

// Skinny form for m <= 16 with a wide n (a small tensor applied to a large
// one, HBM-bound): each thread owns two adjacent columns of C and reads
// B[b][:, j..j+1] once (16-byte loads, coalesced when n is B's fast axis),
// keeping all m outputs of both columns in registers; A's m x k values are
// staged in LDS as [k][m] (up to 32 KB per pass over k) and read as
// broadcasts.  Sums run over k in increasing order.
//
// Output: run on the transposed product (or with a scattered C) a thread's
// two columns are far from its neighbours', so for m <= 8, whole 512-column
// chunks and C offsets that are sums of per-bit offsets, the chunk's m x 512
// block is staged in LDS and written in the order of its offsets, as in the
// rows form below (bits ranked by their position in C; thread t writes the
// block's elements t, t + 256, ...).
template <int M>
__global__ void __launch_bounds__(256) gemm_skinny_kernel(GemmDesc d) {
    constexpr int KC = 4096 / M;
    constexpr int MB = M == 1 ? 0 : M == 2 ? 1 : M == 4 ? 2 : M == 8 ? 3 : 4;  // log2 M
    constexpr int RS = M + 1;                                                  // staged column stride (padded)
    constexpr bool kStage = M <= 8;
    constexpr int SM = kStage && 512 * RS > KC * M ? 512 * RS : KC * M;
    constexpr int NJ = 2 * M;                                                  // elements per thread
    __shared__ float2 sm[SM];
    __shared__ int hi_row[NJ], hi_col[NJ];
    __shared__ int64_t hi_off[NJ];
    __shared__ int s_pos[9 + MB], s_rank[9 + MB], s_ok;
    float2 *As = sm;
    const int64_t chunks = (d.n + 511) / 512;
    const int64_t total = d.nb * chunks;
    const bool bvec = d.sBn == 1 && d.sBk % 2 == 0 && d.sBb % 2 == 0 && (uintptr_t)d.B % 16 == 0;
    const bool cvec = !d.cscatter && d.sCn == 1 && d.sCm % 2 == 0 && d.sCb % 2 == 0 && (uintptr_t)d.C % 16 == 0;
    // Bit positions in C of the block's bits (column bits 0..8 of the chunk,
    // then the m row bits) and their ranks; a direct vector store (cvec) is
    // already coalesced and stays.
    const bool pow2 = d.sCn > 0 && d.sCm > 0 && (d.sCn & (d.sCn - 1)) == 0 && (d.sCm & (d.sCm - 1)) == 0;
    const bool can = kStage && !cvec && d.n % 512 == 0 && d.m == M && (d.cscatter || pow2);
    if (threadIdx.x == 0) s_ok = can;
    if (can && threadIdx.x < 9 + MB) {
        const int b = threadIdx.x;
        if (d.cscatter)
            s_pos[b] = b < 9 ? d.cpos[b] : d.cpos[d.cbn + b - 9];
        else
            s_pos[b] = b < 9 ? __builtin_ctzll(uint64_t(d.sCn)) + b : __builtin_ctzll(uint64_t(d.sCm)) + b - 9;
    }
    __syncthreads();
    if (can && threadIdx.x < 9 + MB) {
        const int b = threadIdx.x, p = s_pos[b];
        int r = 0;
        for (int c = 0; c < 9 + MB; ++c) {
            r += s_pos[c] < p;
            if (c != b && s_pos[c] == p) s_ok = 0;
        }
        s_rank[b] = r;
    }
    __syncthreads();
    const bool staged = s_ok;
    int lo_row = 0, lo_col = 0;
    int64_t lo_off = 0;
    if (staged) {
        for (int b = 0; b < 9 + MB; ++b) {
            const int r = s_rank[b];
            if (r < 8 && ((threadIdx.x >> r) & 1)) {
                if (b < 9) lo_col |= 1 << b; else lo_row |= 1 << (b - 9);
                lo_off += int64_t(1) << s_pos[b];
            }
        }
        if (threadIdx.x < NJ) {
            int hr = 0, hc = 0;
            int64_t ho = 0;
            for (int b = 0; b < 9 + MB; ++b) {
                const int r = s_rank[b];
                if (r >= 8 && ((threadIdx.x >> (r - 8)) & 1)) {
                    if (b < 9) hc |= 1 << b; else hr |= 1 << (b - 9);
                    ho += int64_t(1) << s_pos[b];
                }
            }
            hi_row[threadIdx.x] = hr;
            hi_col[threadIdx.x] = hc;
            hi_off[threadIdx.x] = ho;
        }
    }
    __syncthreads();
    float mx = 0.f;
    for (int64_t blk = blockIdx.x; blk < total; blk += gridDim.x) {
        const int64_t bi = blk / chunks;
        const int64_t j0 = (blk % chunks) * 512 + 2 * threadIdx.x;
        const bool ok0 = j0 < d.n, ok1 = j0 + 1 < d.n;
        const float2 *Ab = d.A + bi * d.sAb;
        const float2 *Bb = d.B + bi * d.sBb;
        float re0[M], im0[M], re1[M], im1[M];
#pragma unroll
        for (int i = 0; i < M; ++i) { re0[i] = 0.f; im0[i] = 0.f; re1[i] = 0.f; im1[i] = 0.f; }
        for (int64_t k0 = 0; k0 < d.k; k0 += KC) {
            const int kc = int(d.k - k0 < KC ? d.k - k0 : KC);
            __syncthreads();
            for (int e = threadIdx.x; e < kc * M; e += blockDim.x) {
                const int l = e / M, i = e - l * M;
                As[e] = Ab[i * d.sAm + (k0 + l) * d.sAk];
            }
            __syncthreads();
            for (int l0 = 0; l0 < kc; l0 += 8) {
                float2 y0[8], y1[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int64_t l = k0 + l0 + u;
                    y0[u] = make_float2(0.f, 0.f);
                    y1[u] = make_float2(0.f, 0.f);
                    if (l0 + u < kc) {
                        if (bvec && ok1) {
                            const float4 w = *(const float4 *)(Bb + l * d.sBk + j0);
                            y0[u] = make_float2(w.x, w.y);
                            y1[u] = make_float2(w.z, w.w);
                        } else {
                            if (ok0) y0[u] = Bb[l * d.sBk + j0 * d.sBn];
                            if (ok1) y1[u] = Bb[l * d.sBk + (j0 + 1) * d.sBn];
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (l0 + u >= kc) break;
#pragma unroll
                    for (int i = 0; i < M; ++i) {
                        const float2 x = As[(l0 + u) * M + i];
                        re0[i] = fmaf(x.x, y0[u].x, re0[i]);
                        re0[i] = fmaf(-x.y, y0[u].y, re0[i]);
                        im0[i] = fmaf(x.x, y0[u].y, im0[i]);
                        im0[i] = fmaf(x.y, y0[u].x, im0[i]);
                        re1[i] = fmaf(x.x, y1[u].x, re1[i]);
                        re1[i] = fmaf(-x.y, y1[u].y, re1[i]);
                        im1[i] = fmaf(x.x, y1[u].y, im1[i]);
                        im1[i] = fmaf(x.y, y1[u].x, im1[i]);
                    }
                }
            }
        }
        if constexpr (kStage) if (staged) {
            // The chunk's base: its batch entry and column bits 9 and up.
            const int64_t jc = j0 - 2 * threadIdx.x;
            const int64_t base = d.cscatter ? scat_bits(d, uint64_t(bi), d.cbn + d.cbm, d.cbb) +
                                                  scat_bits(d, uint64_t(jc), 0, d.cbn)
                                            : bi * d.sCb + jc * d.sCn;
            __syncthreads();  // A's values are no longer read
#pragma unroll
            for (int i = 0; i < M; ++i) {
                sm[(2 * threadIdx.x) * RS + i] = make_float2(re0[i], im0[i]);
                sm[(2 * threadIdx.x + 1) * RS + i] = make_float2(re1[i], im1[i]);
                mx = fmaxf(mx, fmaxf(fmaxf(fabsf(re0[i]), fabsf(im0[i])), fmaxf(fabsf(re1[i]), fabsf(im1[i]))));
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < NJ; ++j)
                d.C[base + lo_off + hi_off[j]] = sm[(lo_col + hi_col[j]) * RS + lo_row + hi_row[j]];
            continue;
        }
        float2 *Cb = d.C + bi * d.sCb;
        int64_t o0 = j0 * d.sCn, o1 = (j0 + 1) * d.sCn;
        if (d.cscatter) {
            Cb = d.C + scat_bits(d, uint64_t(bi), d.cbn + d.cbm, d.cbb);
            o0 = scat_bits(d, uint64_t(j0), 0, d.cbn);
            o1 = scat_bits(d, uint64_t(j0 + 1), 0, d.cbn);
        }
#pragma unroll
        for (int i = 0; i < M; ++i) {
            if (cvec && ok1) {
                *(float4 *)(Cb + i * d.sCm + j0) = make_float4(re0[i], im0[i], re1[i], im1[i]);
            } else {
                const int64_t oi = d.cscatter ? scat_bits(d, uint64_t(i), d.cbn, d.cbm) : i * d.sCm;
                if (ok0) Cb[oi + o0] = make_float2(re0[i], im0[i]);
                if (ok1) Cb[oi + o1] = make_float2(re1[i], im1[i]);
            }
            if (ok0) mx = fmaxf(mx, fmaxf(fabsf(re0[i]), fabsf(im0[i])));
            if (ok1) mx = fmaxf(mx, fmaxf(fabsf(re1[i]), fabsf(im1[i])));
        }
    }
    if (d.amax_c) block_amax(mx, d.amax_c);
}

// Dot form for a few outputs with a long k (the last steps of a tree often
// contract two large tensors to a handful of values): one workgroup of 1024
// threads per output, k strided over the threads (coalesced), then a fixed
// LDS tree, so the result does not depend on the launch.  Split over k, each
// workgroup takes one part of one output.
__global__ void __launch_bounds__(1024) gemm_dot_kernel(GemmDesc d) {
    __shared__ float2 part[1024];
    const int64_t total = d.nb * d.m * d.n;
    float mx = 0.f;
    for (int64_t o = blockIdx.x; o < total; o += gridDim.x) {
        const int64_t j = o % d.n, i = (o / d.n) % d.m, bi = o / (d.n * d.m);
        const int64_t bq = d.kparts == 1 ? bi : bi / d.kparts, bp = bi - bq * d.kparts;
        const float2 *a = d.A + bq * d.sAb + bp * d.sAp + i * d.sAm;
        const float2 *b = d.B + bq * d.sBb + bp * d.sBp + j * d.sBn;
        float re = 0.f, im = 0.f;
        for (int64_t l = threadIdx.x; l < d.k; l += blockDim.x) {
            const float2 x = a[l * d.sAk], y = b[l * d.sBk];
            re = fmaf(x.x, y.x, re);
            re = fmaf(-x.y, y.y, re);
            im = fmaf(x.x, y.y, im);
            im = fmaf(x.y, y.x, im);
        }
        part[threadIdx.x] = make_float2(re, im);
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if (int(threadIdx.x) < w) {
                const float2 u = part[threadIdx.x], v = part[threadIdx.x + w];
                part[threadIdx.x] = make_float2(u.x + v.x, u.y + v.y);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const float2 r = part[0];
            d.C[c_off(d, bi, i, j)] = r;
            mx = fmaxf(mx, fmaxf(fabsf(r.x), fabsf(r.y)));
        }
        __syncthreads();
    }
    if (d.amax_c) block_amax(mx, d.amax_c);
}

// Rows form for a small n (<= 16) with a tall m: B's k x n values are staged
// in LDS ([k][n], up to 2048 per pass, read as broadcasts) and each thread
// owns one row of C, keeping its n outputs in registers while it reads the
// row of A once -- with 16-byte loads along k when A is stored [m][k], or
// coalesced across the threads' rows when it is stored [k][m].  Sums run
// over k in increasing order.
//
// Output: a thread's n values of one row go to n places that are usually far
// from its neighbours' (rows are 8 n bytes apart or scattered), so direct
// stores touch 64 cache lines per instruction.  When every 256-row chunk is
// whole and C's element offset is a sum of per-bit offsets (a scattered
// output, or power-of-two strides), the chunk's 256 x n block is staged in
// LDS and written in the order of its offsets: the block's 8 + log2 n bits
// are ranked by their bit position in C, element e of the block takes bit r
// of e from the bit of rank r, and thread t writes elements t, t + 256, ...,
// so consecutive lanes write consecutive addresses as far as C keeps the
// block's bits together.
template <int N>
__global__ void __launch_bounds__(256) gemm_rows_kernel(GemmDesc d) {
    constexpr int KC = 2048 / N;
    constexpr int NB = N == 1 ? 0 : N == 2 ? 1 : N == 4 ? 2 : N == 8 ? 3 : 4;  // log2 N
    constexpr int RS = N + 1;                                                  // staged row stride (padded)
    constexpr int SM = 256 * RS > KC * N ? 256 * RS : KC * N;
    __shared__ float2 sm[SM];
    __shared__ int hi_row[N], hi_col[N];
    __shared__ int64_t hi_off[N];
    float2 *Bs = sm;
    const bool avec = d.sAk == 1 && d.sAm % 2 == 0 && d.sAb % 2 == 0 && (uintptr_t)d.A % 16 == 0;
    const int64_t chunks = (d.m + 255) / 256;
    const int64_t total = d.nb * chunks;
    // Bit positions in C of the block's bits (n bits 0..NB-1, then row bits
    // 0..7 of the chunk) and their ranks, worked out once by the first
    // NB + 8 threads; any two bits at one position leave the block unstaged.
    __shared__ int s_pos[NB + 8], s_rank[NB + 8], s_ok;
    const bool pow2 = d.sCn > 0 && d.sCm > 0 && (d.sCn & (d.sCn - 1)) == 0 && (d.sCm & (d.sCm - 1)) == 0;
    const bool can = d.m % 256 == 0 && d.n == N && (d.cscatter || pow2);
    if (threadIdx.x == 0) s_ok = can;
    if (can && threadIdx.x < NB + 8) {
        const int b = threadIdx.x;
        if (d.cscatter)
            s_pos[b] = b < NB ? d.cpos[b] : d.cpos[d.cbn + b - NB];
        else
            s_pos[b] = b < NB ? __builtin_ctzll(uint64_t(d.sCn)) + b : __builtin_ctzll(uint64_t(d.sCm)) + b - NB;
    }
    __syncthreads();
    if (can && threadIdx.x < NB + 8) {
        const int b = threadIdx.x, p = s_pos[b];
        int r = 0;
        for (int c = 0; c < NB + 8; ++c) {
            r += s_pos[c] < p;
            if (c != b && s_pos[c] == p) s_ok = 0;
        }
        s_rank[b] = r;
    }
    __syncthreads();
    const bool staged = s_ok;
    // This thread's element t: its row, column and offset from the bits of
    // rank < 8; elements t + 256 j add the parts of the bits of rank >= 8.
    int lo_row = 0, lo_col = 0;
    int64_t lo_off = 0;
    if (staged) {
        for (int b = 0; b < NB + 8; ++b) {
            const int r = s_rank[b];
            if (r < 8 && ((threadIdx.x >> r) & 1)) {
                if (b < NB) lo_col |= 1 << b; else lo_row |= 1 << (b - NB);
                lo_off += int64_t(1) << s_pos[b];
            }
        }
        if (threadIdx.x < N) {
            int hr = 0, hc = 0;
            int64_t ho = 0;
            for (int b = 0; b < NB + 8; ++b) {
                const int r = s_rank[b];
                if (r >= 8 && ((threadIdx.x >> (r - 8)) & 1)) {
                    if (b < NB) hc |= 1 << b; else hr |= 1 << (b - NB);
                    ho += int64_t(1) << s_pos[b];
                }
            }
            hi_row[threadIdx.x] = hr;
            hi_col[threadIdx.x] = hc;
            hi_off[threadIdx.x] = ho;
        }
    }
    __syncthreads();
    float mx = 0.f;
    for (int64_t blk = blockIdx.x; blk < total; blk += gridDim.x) {
        const int64_t bi = blk / chunks;
        const int64_t i = (blk % chunks) * 256 + threadIdx.x;
        const bool ok = i < d.m;
        const float2 *Ar = d.A + bi * d.sAb + (ok ? i : 0) * d.sAm;
        const float2 *Bb = d.B + bi * d.sBb;
        float re[N], im[N];
#pragma unroll
        for (int j = 0; j < N; ++j) { re[j] = 0.f; im[j] = 0.f; }
        for (int64_t k0 = 0; k0 < d.k; k0 += KC) {
            const int kc = int(d.k - k0 < KC ? d.k - k0 : KC);
            __syncthreads();
            for (int e = threadIdx.x; e < kc * N; e += blockDim.x) {
                const int l = e / N, j = e - l * N;
                Bs[e] = Bb[(k0 + l) * d.sBk + j * d.sBn];
            }
            __syncthreads();
            if (ok) {
                int l = 0;
                if (avec) {
                    for (; l + 1 < kc; l += 2) {
                        const float4 w = *(const float4 *)(Ar + k0 + l);
#pragma unroll
                        for (int j = 0; j < N; ++j) {
                            const float2 y0 = Bs[l * N + j], y1 = Bs[(l + 1) * N + j];
                            re[j] = fmaf(w.x, y0.x, re[j]);
                            re[j] = fmaf(-w.y, y0.y, re[j]);
                            im[j] = fmaf(w.x, y0.y, im[j]);
                            im[j] = fmaf(w.y, y0.x, im[j]);
                            re[j] = fmaf(w.z, y1.x, re[j]);
                            re[j] = fmaf(-w.w, y1.y, re[j]);
                            im[j] = fmaf(w.z, y1.y, im[j]);
                            im[j] = fmaf(w.w, y1.x, im[j]);
                        }
                    }
                }
                for (; l < kc; ++l) {
                    const float2 x = Ar[(k0 + l) * d.sAk];
#pragma unroll
                    for (int j = 0; j < N; ++j) {
                        const float2 y = Bs[l * N + j];
                        re[j] = fmaf(x.x, y.x, re[j]);
                        re[j] = fmaf(-x.y, y.y, re[j]);
                        im[j] = fmaf(x.x, y.y, im[j]);
                        im[j] = fmaf(x.y, y.x, im[j]);
                    }
                }
            }
        }
        if (staged) {
            // The chunk's base: its batch entry and row bits 8 and up.
            const int64_t i0 = i - threadIdx.x;
            const int64_t base = d.cscatter ? scat_bits(d, uint64_t(bi), d.cbn + d.cbm, d.cbb) +
                                                  scat_bits(d, uint64_t(i0), d.cbn, d.cbm)
                                            : bi * d.sCb + i0 * d.sCm;
            __syncthreads();  // B's values are no longer read
#pragma unroll
            for (int j = 0; j < N; ++j) {
                sm[threadIdx.x * RS + j] = make_float2(re[j], im[j]);
                mx = fmaxf(mx, fmaxf(fabsf(re[j]), fabsf(im[j])));
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < N; ++j)
                d.C[base + lo_off + hi_off[j]] = sm[(lo_row + hi_row[j]) * RS + lo_col + hi_col[j]];
        } else if (ok) {
            const int64_t ro = d.cscatter ? scat_bits(d, uint64_t(bi), d.cbn + d.cbm, d.cbb) +
                                                scat_bits(d, uint64_t(i), d.cbn, d.cbm)
                                          : bi * d.sCb + i * d.sCm;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                const int64_t co = d.cscatter ? scat_bits(d, uint64_t(j), 0, d.cbn) : j * d.sCn;
                d.C[ro + co] = make_float2(re[j], im[j]);
                mx = fmaxf(mx, fmaxf(fabsf(re[j]), fabsf(im[j])));
            }
        }
    }
    if (d.amax_c) block_amax(mx, d.amax_c);
}

// Dot-tile form for a small output tile (m n <= 256 per batch) with a long k:
// a workgroup owns one batch entry's whole m x n tile, thread t < m n one
// output (t / n, t % n); k runs in chunks whose A (m x kc) and B (kc x n)
// values are staged in LDS with loads coalesced along whichever index is
// contiguous, so every operand value is read from memory once per
// workgroup.  Sums run over k in increasing order.  Split over k, each
// workgroup takes one part of one batch entry.
__global__ void __launch_bounds__(256) gemm_dot_tile_kernel(GemmDesc d) {
    __shared__ float2 sm[4096];
    const int m = int(d.m), n = int(d.n), mn = m * n;
    int kc = 4096 / (m + n);
    kc = kc >= 64 ? 64 : kc;
    float2 *As = sm, *Bs = sm + m * kc;
    const bool a_k_fast = d.sAk == 1, b_k_fast = d.sBk == 1;
    const int t = threadIdx.x;
    const int oi = t / n, oj = t - (t / n) * n;
    float mx = 0.f;
    for (int64_t bi = blockIdx.x; bi < d.nb; bi += gridDim.x) {
        const int64_t bq = d.kparts == 1 ? bi : bi / d.kparts, bp = bi - bq * d.kparts;
        const float2 *a = d.A + bq * d.sAb + bp * d.sAp;
        const float2 *b = d.B + bq * d.sBb + bp * d.sBp;
        float re = 0.f, im = 0.f;
        for (int64_t l0 = 0; l0 < d.k; l0 += kc) {
            const int c = int(d.k - l0 < kc ? d.k - l0 : kc);
            __syncthreads();
            for (int e = t; e < m * c; e += blockDim.x) {
                int i, l;
                if (a_k_fast) { i = e / c; l = e - i * c; } else { l = e / m; i = e - l * m; }
                As[i * kc + l] = a[i * d.sAm + (l0 + l) * d.sAk];
            }
            for (int e = t; e < n * c; e += blockDim.x) {
                int j, l;
                if (b_k_fast) { j = e / c; l = e - j * c; } else { l = e / n; j = e - l * n; }
                Bs[l * n + j] = b[(l0 + l) * d.sBk + j * d.sBn];
            }
            __syncthreads();
            if (t < mn) {
                const float2 *ar = As + oi * kc;
                for (int l = 0; l < c; ++l) {
                    const float2 x = ar[l], y = Bs[l * n + oj];
                    re = fmaf(x.x, y.x, re);
                    re = fmaf(-x.y, y.y, re);
                    im = fmaf(x.x, y.y, im);
                    im = fmaf(x.y, y.x, im);
                }
            }
        }
        if (t < mn) {
            d.C[c_off(d, bi, oi, oj)] = make_float2(re, im);
            mx = fmaxf(mx, fmaxf(fabsf(re), fabsf(im)));
        }
    }
    if (d.amax_c) block_amax(mx, d.amax_c);
}

// -------------------------------------------------------------- MFMA GEMM
// Complex FP32 GEMM in the 4M form on v_mfma_f32_32x32x2_f32: each wave owns
// a 32x32 output tile with separate real and imaginary accumulators,
// Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br.  A block of WM x WN waves owns a
// (32 WM) x (32 WN) tile; K is staged through LDS in planar (re, im) slabs of
// KT values, laid out [k][m] and [k][n] so each MFMA operand fetch is a
// contiguous 32-float row.
typedef float floatx16 __attribute__((ext_vector_type(16)));

template <int WM, int WN, int KT>
__global__ void __launch_bounds__(64 * WM * WN) gemm_mfma_kernel(GemmDesc d) {
    constexpr int TM = 32 * WM, TN = 32 * WN, NT = 64 * WM * WN;
    __shared__ float As_re[KT][TM + 1], As_im[KT][TM + 1];
    __shared__ float Bs_re[KT][TN + 1], Bs_im[KT][TN + 1];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int64_t tiles_m = d.m / TM, tiles_n = d.n / TN;
    const int64_t n_tiles = d.nb * tiles_m * tiles_n;
    const bool a_k_fast = d.sAk == 1;
    const bool b_n_fast = d.sBn == 1;
    float mx = 0.f;  // max(|re|, |im|) written, folded into amax_c when the program tracks it
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t tn = tile % tiles_n;
        const int64_t tm = (tile / tiles_n) % tiles_m;
        const int64_t bi = tile / (tiles_n * tiles_m);
        // With a split over k, batch entry bi is part bp of entry bq.
        const int64_t bq = d.kparts == 1 ? bi : bi / d.kparts, bp = bi - bq * d.kparts;
        const float2 *Ab = d.A + bq * d.sAb + bp * d.sAp + tm * TM * d.sAm;
        const float2 *Bb = d.B + bq * d.sBb + bp * d.sBp + tn * TN * d.sBn;
        floatx16 acc_re, acc_im;
        for (int v = 0; v < 16; ++v) { acc_re[v] = 0.f; acc_im[v] = 0.f; }
        for (int64_t k0 = 0; k0 < d.k; k0 += KT) {
            for (int e = threadIdx.x; e < TM * KT; e += NT) {
                int i, kk;
                if (a_k_fast) { i = e / KT; kk = e % KT; } else { i = e % TM; kk = e / TM; }
                const float2 v = Ab[i * d.sAm + (k0 + kk) * d.sAk];
                As_re[kk][i] = v.x;
                As_im[kk][i] = v.y;
            }
            for (int e = threadIdx.x; e < TN * KT; e += NT) {
                int j, kk;
                if (b_n_fast) { j = e % TN; kk = e / TN; } else { j = e / KT; kk = e % KT; }
                const float2 v = Bb[(k0 + kk) * d.sBk + j * d.sBn];
                Bs_re[kk][j] = v.x;
                Bs_im[kk][j] = v.y;
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < KT; kk += 2) {
                const int kr = kk + (lane >> 5);
                const float ar = As_re[kr][wm * 32 + (lane & 31)];
                const float ai = As_im[kr][wm * 32 + (lane & 31)];
                const float br = Bs_re[kr][wn * 32 + (lane & 31)];
                const float bim = Bs_im[kr][wn * 32 + (lane & 31)];
                acc_re = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br, acc_re, 0, 0, 0);
                acc_re = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai, bim, acc_re, 0, 0, 0);
                acc_im = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, bim, acc_im, 0, 0, 0);
                acc_im = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, br, acc_im, 0, 0, 0);
            }
            __syncthreads();
        }
        const CBlock cb = c_block(d, bi, tm * TM + wm * 32, tn * TN + wn * 32, lane);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            *c_at(cb, v) = make_float2(acc_re[v], acc_im[v]);
            mx = fmaxf(mx, fmaxf(fabsf(acc_re[v]), fabsf(acc_im[v])));
        }
    }
    if (d.amax_c) block_amax(mx, d.amax_c);
}

// ------------------------------------------------ split-precision MFMA GEMM
// Operands stay complex64 in memory.  While a K slab of 16 complex values is
// staged into LDS, each real part x becomes x 2^-d = h + l (h, l in the 16-bit
// type, round to nearest even), stored in four planes per operand: hi re,
// hi im, lo re, lo im, each [row][16] so that one lane's MFMA operand (8
// consecutive k of one row) is a single 16-byte LDS read.  Each real product
// X Y is accumulated as Xh Yh + Xh Yl + Xl Yh on v_mfma_f32_32x32x16_{f16,bf16};
// the complex product takes four of them (4M), so 12 MFMAs per slab and wave.
// The product -Ai Bi uses Ai with flipped sign bits (exact).  K need not be a
// multiple of 16: the last slab is padded with zeros.
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx16 mfma16(half8 a, half8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx16 mfma16(bf16x8 a, bf16x8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
template <typename V> __device__ __forceinline__ V negate16(V v) {
    return __builtin_bit_cast(V, __builtin_bit_cast(u32x4, v) ^ 0x80008000u);
}

// Scale exponent of a tensor from its recorded max|x|: FP16 puts the largest
// magnitude in [2^14, 2^15); BF16 (FP32's exponent range) and zero, infinite
// or missing maxima use 0.
template <typename T> __device__ __forceinline__ int split_exp(const uint32_t *amax);
template <> __device__ __forceinline__ int split_exp<__bf16>(const uint32_t *) { return 0; }
template <> __device__ __forceinline__ int split_exp<_Float16>(const uint32_t *amax) {
    if (!amax) return 0;
    const float m = __uint_as_float(*amax);
    if (!(m > 0.f) || !(m <= 3.4028235e38f)) return 0;
    return ilogbf(m) - 14;
}

template <typename T, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN) gemm_split_kernel(GemmDesc d) {
    typedef T V __attribute__((ext_vector_type(8)));
    constexpr int TM = 32 * WM, TN = 32 * WN, NT = 64 * WM * WN, KT = 16;
    __shared__ __attribute__((aligned(16))) T As[4][TM][KT];
    __shared__ __attribute__((aligned(16))) T Bs[4][TN][KT];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int64_t tiles_m = d.m / TM, tiles_n = d.n / TN;
    const int64_t n_tiles = d.nb * tiles_m * tiles_n;
    const bool a_k_fast = d.sAk == 1;
    const bool b_n_fast = d.sBn == 1;
    const int ea = split_exp<T>(d.amax_a), eb = split_exp<T>(d.amax_b);
    float mx = 0.f;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t tn = tile % tiles_n;
        const int64_t tm = (tile / tiles_n) % tiles_m;
        const int64_t bi = tile / (tiles_n * tiles_m);
        // With a split over k, batch entry bi is part bp of entry bq.
        const int64_t bq = d.kparts == 1 ? bi : bi / d.kparts, bp = bi - bq * d.kparts;
        const float2 *Ab = d.A + bq * d.sAb + bp * d.sAp + tm * TM * d.sAm;
        const float2 *Bb = d.B + bq * d.sBb + bp * d.sBp + tn * TN * d.sBn;
        floatx16 acc_re, acc_im;
        for (int v = 0; v < 16; ++v) { acc_re[v] = 0.f; acc_im[v] = 0.f; }
        for (int64_t k0 = 0; k0 < d.k; k0 += KT) {
            for (int e = threadIdx.x; e < TM * KT; e += NT) {
                int i, kk;
                if (a_k_fast) { i = e / KT; kk = e % KT; } else { i = e % TM; kk = e / TM; }
                float2 v = make_float2(0.f, 0.f);
                if (k0 + kk < d.k) v = Ab[i * d.sAm + (k0 + kk) * d.sAk];
                const float xr = ldexpf(v.x, -ea), xi = ldexpf(v.y, -ea);
                const T hr = T(xr), hi = T(xi);
                As[0][i][kk] = hr;
                As[1][i][kk] = hi;
                As[2][i][kk] = T(xr - float(hr));
                As[3][i][kk] = T(xi - float(hi));
            }
            for (int e = threadIdx.x; e < TN * KT; e += NT) {
                int j, kk;
                if (b_n_fast) { j = e % TN; kk = e / TN; } else { j = e / KT; kk = e % KT; }
                float2 v = make_float2(0.f, 0.f);
                if (k0 + kk < d.k) v = Bb[(k0 + kk) * d.sBk + j * d.sBn];
                const float xr = ldexpf(v.x, -eb), xi = ldexpf(v.y, -eb);
                const T hr = T(xr), hi = T(xi);
                Bs[0][j][kk] = hr;
                Bs[1][j][kk] = hi;
                Bs[2][j][kk] = T(xr - float(hr));
                Bs[3][j][kk] = T(xi - float(hi));
            }
            __syncthreads();
            const int ra = wm * 32 + (lane & 31), rb = wn * 32 + (lane & 31), kq = (lane >> 5) * 8;
            const V arh = *(const V *)&As[0][ra][kq], aih = *(const V *)&As[1][ra][kq];
            const V arl = *(const V *)&As[2][ra][kq], ail = *(const V *)&As[3][ra][kq];
            const V brh = *(const V *)&Bs[0][rb][kq], bih = *(const V *)&Bs[1][rb][kq];
            const V brl = *(const V *)&Bs[2][rb][kq], bil = *(const V *)&Bs[3][rb][kq];
            const V naih = negate16(aih), nail = negate16(ail);
            acc_re = mfma16(arh, brh, acc_re);
            acc_re = mfma16(arh, brl, acc_re);
            acc_re = mfma16(arl, brh, acc_re);
            acc_re = mfma16(naih, bih, acc_re);
            acc_re = mfma16(naih, bil, acc_re);
            acc_re = mfma16(nail, bih, acc_re);
            acc_im = mfma16(arh, bih, acc_im);
            acc_im = mfma16(arh, bil, acc_im);
            acc_im = mfma16(arl, bih, acc_im);
            acc_im = mfma16(aih, brh, acc_im);
            acc_im = mfma16(aih, brl, acc_im);
            acc_im = mfma16(ail, brh, acc_im);
            __syncthreads();
        }
        const CBlock cb = c_block(d, bi, tm * TM + wm * 32, tn * TN + wn * 32, lane);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const float re = ldexpf(acc_re[v], ea + eb), im = ldexpf(acc_im[v], ea + eb);
            *c_at(cb, v) = make_float2(re, im);
            mx = fmaxf(mx, fmaxf(fabsf(re), fabsf(im)));
        }
    }
    if (d.amax_c) block_amax(mx, d.amax_c);
}

// Large-tile form for m, n multiples of 128: a 128x128 block tile, four
// waves each owning 64x64 (2x2 MFMA tiles, 8 accumulators), K slabs of 16
// double-buffered in LDS with one barrier per slab; the next slab's complex64
// operands are loaded into registers while the current slab is multiplied,
// then scaled, split and stored into the other buffer.  Each thread stages
// 8 consecutive k of one row of A and of B (one 16-byte LDS write per plane);
// the two 16-byte halves of a row swap places on every other group of 8 rows
// to spread the fragment reads over the LDS banks.  Tiles are numbered with n
// fastest and dealt to the eight XCDs in contiguous ranges, so the blocks of
// one XCD share A panels in that XCD's L2.
__device__ __forceinline__ int swz(int row, int half) { return (half ^ ((row >> 3) & 1)) * 8; }

template <typename T, int ROWS>
__device__ __forceinline__ void split_store(T (*plane)[ROWS][16], int row, int half, const float2 (&v)[8], int e) {
    typedef T V __attribute__((ext_vector_type(8)));
    V hr, hi, lr, li;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const float xr = ldexpf(v[q].x, -e), xi = ldexpf(v[q].y, -e);
        const T a = T(xr), b = T(xi);
        hr[q] = a;
        hi[q] = b;
        lr[q] = T(xr - float(a));
        li[q] = T(xi - float(b));
    }
    const int c = swz(row, half);
    *(V *)&plane[0][row][c] = hr;
    *(V *)&plane[1][row][c] = hi;
    *(V *)&plane[2][row][c] = lr;
    *(V *)&plane[3][row][c] = li;
}

// 8 consecutive k (from k0 + 8 half) of row `row` of an operand whose element
// (row, kk) sits at base[row * s_row + kk * s_k]; zero beyond k, which the
// forms using this require to be a multiple of 8 (a group is then entirely
// inside k or entirely past it: no per-element predicates, which would hold
// eight addresses live).  vec: k is the fast axis and every row start is
// 16-byte aligned (16-byte loads).
__device__ __forceinline__ void load8(float2 (&v)[8], const float2 *base, int64_t s_row, int64_t s_k, bool vec,
                                      int row, int64_t kk0, int64_t k) {
    const float2 *p = base + row * s_row + kk0 * s_k;
    if (kk0 < k) {
        if (vec) {
            const float4 *p4 = (const float4 *)p;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 w = p4[q];
                v[2 * q] = make_float2(w.x, w.y);
                v[2 * q + 1] = make_float2(w.z, w.w);
            }
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = p[q * s_k];
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = make_float2(0.f, 0.f);
    }
}

// JN = 2: the 128x128 tile above (each wave 64x64); JN = 1: a 128x64 tile
// (each wave 64x32, half the accumulators, two waves per SIMD), in which
// only the first 128 threads stage B.
template <typename T, int JN>
__global__ void __launch_bounds__(256, JN == 1 ? 2 : 1) gemm_split_big_kernel(GemmDesc d) {
    typedef T V __attribute__((ext_vector_type(8)));
    constexpr int TM = 128, TN = 64 * JN, KT = 16;
    __shared__ __attribute__((aligned(16))) T As[2][4][TM][KT];
    __shared__ __attribute__((aligned(16))) T Bs[2][4][TN][KT];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t tiles_m = d.m / TM, tiles_n = d.n / TN;
    const int64_t n_tiles = d.nb * tiles_m * tiles_n;
    // Staging roles: along k when k is the fast axis (64 contiguous bytes per
    // thread), else along the row (coalesced across the wavefront).
    const bool a_kc = d.sAk == 1, b_kc = d.sBk == 1;
    const int ar = a_kc ? (t >> 1) : (t & 127), ah = a_kc ? (t & 1) : (t >> 7);
    const int br = b_kc ? ((t >> 1) & (TN - 1)) : (t & (TN - 1)), bh = b_kc ? (t & 1) : ((t / TN) & 1);
    const bool bst = JN == 2 || t < 2 * TN;  // this thread stages a row half of B
    const bool a_vec = a_kc && d.sAm % 2 == 0 && d.sAb % 2 == 0 && d.sAp % 2 == 0 && (uintptr_t)d.A % 16 == 0;
    const bool b_vec = b_kc && d.sBn % 2 == 0 && d.sBb % 2 == 0 && d.sBp % 2 == 0 && (uintptr_t)d.B % 16 == 0;
    const int ea = split_exp<T>(d.amax_a), eb = split_exp<T>(d.amax_b);
    const int n_slabs = int((d.k + KT - 1) / KT);
    float mx = 0.f;
    // XCD-aware numbering (a permutation of the grid when it divides by 8).
    int64_t first = blockIdx.x;
    if (gridDim.x % 8 == 0) first = int64_t(blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    for (int64_t tile = first; tile < n_tiles; tile += gridDim.x) {
        const int64_t tn = tile % tiles_n;
        const int64_t tm = (tile / tiles_n) % tiles_m;
        const int64_t bi = tile / (tiles_n * tiles_m);
        const int64_t bq = d.kparts == 1 ? bi : bi / d.kparts, bp = bi - bq * d.kparts;
        const float2 *Ab = d.A + bq * d.sAb + bp * d.sAp + tm * TM * d.sAm;
        const float2 *Bb = d.B + bq * d.sBb + bp * d.sBp + tn * TN * d.sBn;
        floatx16 acc[2][JN][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < JN; ++j)
#pragma unroll
                for (int v = 0; v < 16; ++v) { acc[i][j][0][v] = 0.f; acc[i][j][1][v] = 0.f; }
        float2 ra[8], rb[8];
        load8(ra, Ab, d.sAm, d.sAk, a_vec, ar, 8 * ah, d.k);
        if (bst) load8(rb, Bb, d.sBn, d.sBk, b_vec, br, 8 * bh, d.k);
        split_store<T, TM>(As[0], ar, ah, ra, ea);
        if (bst) split_store<T, TN>(Bs[0], br, bh, rb, eb);
        __syncthreads();
        for (int s = 0; s < n_slabs; ++s) {
            const int buf = s & 1;
            // The next slab.  BF16 stages it unconditionally (zeros past the
            // end, into the buffer nobody reads again) so that the staging
            // shares the MFMAs' basic block and can be interleaved with them.
            constexpr bool kInterleave = __is_same(T, __bf16) && JN == 2;
            const bool more = kInterleave || s + 1 < n_slabs;
            if (more) {
                const int64_t k1 = int64_t(s + 1) * KT;
                load8(ra, Ab, d.sAm, d.sAk, a_vec, ar, k1 + 8 * ah, d.k);
                if (bst) load8(rb, Bb, d.sBn, d.sBk, b_vec, br, k1 + 8 * bh, d.k);
            }
            V a[2][4], b[JN][4], na[2][2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int row = wm * 64 + i * 32 + (lane & 31);
                const int c = swz(row, lane >> 5);
#pragma unroll
                for (int p = 0; p < 4; ++p) a[i][p] = *(const V *)&As[buf][p][row][c];
                na[i][0] = negate16(a[i][1]);
                na[i][1] = negate16(a[i][3]);
            }
#pragma unroll
            for (int j = 0; j < JN; ++j) {
                const int row = wn * 32 * JN + j * 32 + (lane & 31);
                const int c = swz(row, lane >> 5);
#pragma unroll
                for (int p = 0; p < 4; ++p) b[j][p] = *(const V *)&Bs[buf][p][row][c];
            }
            // Planes: 0 hi re, 1 hi im, 2 lo re, 3 lo im.  Consecutive MFMAs
            // go to different accumulators.
#define QC_MFMA_ALL(ROW_A, COL_B, RI)                                                    \
    _Pragma("unroll") for (int i = 0; i < 2; ++i) _Pragma("unroll") for (int j = 0; j < JN; ++j) \
        acc[i][j][RI] = mfma16(ROW_A, COL_B, acc[i][j][RI]);
            QC_MFMA_ALL(a[i][0], b[j][0], 0)
            QC_MFMA_ALL(a[i][0], b[j][1], 1)
            QC_MFMA_ALL(a[i][0], b[j][2], 0)
            QC_MFMA_ALL(a[i][0], b[j][3], 1)
            QC_MFMA_ALL(a[i][2], b[j][0], 0)
            QC_MFMA_ALL(a[i][2], b[j][1], 1)
            QC_MFMA_ALL(na[i][0], b[j][1], 0)
            QC_MFMA_ALL(a[i][1], b[j][0], 1)
            QC_MFMA_ALL(na[i][0], b[j][3], 0)
            QC_MFMA_ALL(a[i][1], b[j][2], 1)
            QC_MFMA_ALL(na[i][1], b[j][1], 0)
            QC_MFMA_ALL(a[i][3], b[j][0], 1)
#undef QC_MFMA_ALL
            if (more) {
                split_store<T, TM>(As[buf ^ 1], ar, ah, ra, ea);
                if (bst) split_store<T, TN>(Bs[buf ^ 1], br, bh, rb, eb);
            }
            // BF16: the fragment reads, then each of the 48 MFMAs with four
            // VALU instructions of the next slab's conversion and an LDS write
            // after every sixth, so the conversion hides under the matrix
            // pipe (measured faster).  FP16's conversion also scales and is
            // about twice as long; it is left to the compiler's order, which
            // measured faster for it.
            if constexpr (kInterleave) {
                __builtin_amdgcn_sched_group_barrier(0x100, 16, 0);
#pragma unroll
                for (int g = 0; g < 48; ++g) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);
                    if (g % 6 == 5) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < JN; ++j) {
                const CBlock cb = c_block(d, bi, tm * TM + wm * 64 + i * 32, tn * TN + wn * 32 * JN + j * 32, lane);
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const float re = ldexpf(acc[i][j][0][v], ea + eb), im = ldexpf(acc[i][j][1][v], ea + eb);
                    *c_at(cb, v) = make_float2(re, im);
                    mx = fmaxf(mx, fmaxf(fabsf(re), fabsf(im)));
                }
            }
    }
    if (d.amax_c) block_amax(mx, d.amax_c);
}

// Large-tile complex FP32 form for m, n multiples of 128: the split form's
// block structure (128x128 tile, four waves of 64x64, K slabs of 16 double
// buffered in LDS, next slab prefetched in registers, XCD-contiguous tile
// order) with FP32 operands stored [k][row] as (re, im) pairs, so one
// 8-byte LDS read gives a lane both parts of its v_mfma_f32_32x32x2_f32
// operand.  4M form: Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br.
__device__ __forceinline__ void store8_kmajor(float2 (*plane)[128], int row, int half, const float2 (&v)[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) plane[8 * half + q][row] = v[q];
}

// AMAX: also fold max(|re|, |im|) of the output into amax_c (split FP16
// programs, whose later steps derive scales from it; a separate instance, as
// the extra epilogue work costs the plain form its second wave per SIMD).
template <bool AMAX>
__global__ void __launch_bounds__(256) gemm_mfma_big_kernel(GemmDesc d) {
    constexpr int TM = 128, TN = 128, KT = 16;
    __shared__ __attribute__((aligned(16))) float2 As[2][KT][TM];
    __shared__ __attribute__((aligned(16))) float2 Bs[2][KT][TN];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t tiles_m = d.m / TM, tiles_n = d.n / TN;
    const int64_t n_tiles = d.nb * tiles_m * tiles_n;
    const bool a_kc = d.sAk == 1, b_kc = d.sBk == 1;
    const int ar = a_kc ? (t >> 1) : (t & 127), ah = a_kc ? (t & 1) : (t >> 7);
    const int br = b_kc ? (t >> 1) : (t & 127), bh = b_kc ? (t & 1) : (t >> 7);
    const bool a_vec = a_kc && d.sAm % 2 == 0 && d.sAb % 2 == 0 && d.sAp % 2 == 0 && (uintptr_t)d.A % 16 == 0;
    const bool b_vec = b_kc && d.sBn % 2 == 0 && d.sBb % 2 == 0 && d.sBp % 2 == 0 && (uintptr_t)d.B % 16 == 0;
    const int n_slabs = int((d.k + KT - 1) / KT);
    float mx = 0.f;  // max(|re|, |im|) written, folded into amax_c when the program tracks it
    int64_t first = blockIdx.x;
    if (gridDim.x % 8 == 0) first = int64_t(blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    for (int64_t tile = first; tile < n_tiles; tile += gridDim.x) {
        const int64_t tn = tile % tiles_n;
        const int64_t tm = (tile / tiles_n) % tiles_m;
        const int64_t bi = tile / (tiles_n * tiles_m);
        const int64_t bq = d.kparts == 1 ? bi : bi / d.kparts, bp = bi - bq * d.kparts;
        const float2 *Ab = d.A + bq * d.sAb + bp * d.sAp + tm * TM * d.sAm;
        const float2 *Bb = d.B + bq * d.sBb + bp * d.sBp + tn * TN * d.sBn;
        floatx16 acc[2][2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 16; ++v) { acc[i][j][0][v] = 0.f; acc[i][j][1][v] = 0.f; }
        float2 ra[8], rb[8];
        load8(ra, Ab, d.sAm, d.sAk, a_vec, ar, 8 * ah, d.k);
        load8(rb, Bb, d.sBn, d.sBk, b_vec, br, 8 * bh, d.k);
        store8_kmajor(As[0], ar, ah, ra);
        store8_kmajor(Bs[0], br, bh, rb);
        __syncthreads();
        for (int s = 0; s < n_slabs; ++s) {
            const int buf = s & 1;
            const bool more = s + 1 < n_slabs;
            if (more) {
                const int64_t k1 = int64_t(s + 1) * KT;
                load8(ra, Ab, d.sAm, d.sAk, a_vec, ar, k1 + 8 * ah, d.k);
                load8(rb, Bb, d.sBn, d.sBk, b_vec, br, k1 + 8 * bh, d.k);
            }
#pragma unroll
            for (int kk = 0; kk < KT; kk += 2) {
                const int kr = kk + (lane >> 5);
                float2 a[2], b[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) a[i] = As[buf][kr][wm * 64 + i * 32 + (lane & 31)];
#pragma unroll
                for (int j = 0; j < 2; ++j) b[j] = Bs[buf][kr][wn * 64 + j * 32 + (lane & 31)];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        acc[i][j][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].x, b[j].x, acc[i][j][0], 0, 0, 0);
                        acc[i][j][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].x, b[j].y, acc[i][j][1], 0, 0, 0);
                    }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        acc[i][j][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(-a[i].y, b[j].y, acc[i][j][0], 0, 0, 0);
                        acc[i][j][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].y, b[j].x, acc[i][j][1], 0, 0, 0);
                    }
            }
            if (more) {
                store8_kmajor(As[buf ^ 1], ar, ah, ra);
                store8_kmajor(Bs[buf ^ 1], br, bh, rb);
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const CBlock cb = c_block(d, bi, tm * TM + wm * 64 + i * 32, tn * TN + wn * 64 + j * 32, lane);
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    *c_at(cb, v) = make_float2(acc[i][j][0][v], acc[i][j][1][v]);
                    if (AMAX) mx = fmaxf(mx, fmaxf(fabsf(acc[i][j][0][v]), fabsf(acc[i][j][1][v])));
                }
            }
    }
    if (AMAX && d.amax_c) block_amax(mx, d.amax_c);
}

// Tall and wide tile forms of the complex FP32 MFMA product: the large-tile
// form's structure (four waves, K slabs of 16 double buffered in LDS as
// (re, im) pairs [k][row], the next slab prefetched in registers while the
// current one is multiplied, XCD-contiguous tile order) with a tile of
// TM x TN = (32 BM WGM) x (32 BN WGN): the waves in a WGM x WGN grid, each
// holding BM x BN output blocks of 32 x 32.  Shapes with one long and one
// short output dimension and a short k (a long panel streamed past a small
// operand) fill the chip with these tiles where 128 x 128 tiles do not fit.
// Each thread stages up to PA (PB) groups of 8 consecutive k of one row.
template <int BM, int BN, int WGM, int WGN, bool AMAX>
__global__ void __launch_bounds__(256) gemm_mfma_tile_kernel(GemmDesc d) {
    static_assert(WGM * WGN == 4, "four waves");
    constexpr int TM = 32 * BM * WGM, TN = 32 * BN * WGN, KT = 16;
    constexpr int PA = (2 * TM + 255) / 256, PB = (2 * TN + 255) / 256;
    __shared__ __attribute__((aligned(16))) float2 As[2][KT][TM];
    __shared__ __attribute__((aligned(16))) float2 Bs[2][KT][TN];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    const int64_t tiles_m = d.m / TM, tiles_n = d.n / TN;
    const int64_t n_tiles = d.nb * tiles_m * tiles_n;
    const bool a_kc = d.sAk == 1, b_kc = d.sBk == 1;
    const bool a_vec = a_kc && d.sAm % 2 == 0 && d.sAb % 2 == 0 && d.sAp % 2 == 0 && (uintptr_t)d.A % 16 == 0;
    const bool b_vec = b_kc && d.sBn % 2 == 0 && d.sBb % 2 == 0 && d.sBp % 2 == 0 && (uintptr_t)d.B % 16 == 0;
    // Staging pairs (row, half of the slab): along k when k is the fast axis
    // (two threads per row), else along the row (coalesced across lanes).
    int ar[PA], ah[PA], br[PB], bh[PB];
    bool a_on[PA], b_on[PB];
#pragma unroll
    for (int p = 0; p < PA; ++p) {
        const int q = t + 256 * p;
        a_on[p] = q < 2 * TM;
        ar[p] = a_kc ? (q >> 1) % TM : q % TM;
        ah[p] = a_kc ? (q & 1) : (q / TM) & 1;
    }
#pragma unroll
    for (int p = 0; p < PB; ++p) {
        const int q = t + 256 * p;
        b_on[p] = q < 2 * TN;
        br[p] = b_kc ? (q >> 1) % TN : q % TN;
        bh[p] = b_kc ? (q & 1) : (q / TN) & 1;
    }
    const int n_slabs = int((d.k + KT - 1) / KT);
    float mx = 0.f;  // max(|re|, |im|) written, folded into amax_c when the program tracks it
    // Operand panels of a tile (batch entry, rows, columns).
    auto panels = [&](int64_t tile, const float2 *&Ab, const float2 *&Bb, int64_t &bi, int64_t &tm, int64_t &tn) {
        tn = tile % tiles_n;
        tm = (tile / tiles_n) % tiles_m;
        bi = tile / (tiles_n * tiles_m);
        const int64_t bq = d.kparts == 1 ? bi : bi / d.kparts, bp = bi - bq * d.kparts;
        Ab = d.A + bq * d.sAb + bp * d.sAp + tm * TM * d.sAm;
        Bb = d.B + bq * d.sBb + bp * d.sBp + tn * TN * d.sBn;
    };
    float2 ra[PA][8], rb[PB][8];
    auto load_slab = [&](const float2 *Ab, const float2 *Bb, int64_t k0) {
#pragma unroll
        for (int p = 0; p < PA; ++p)
            if (a_on[p]) load8(ra[p], Ab, d.sAm, d.sAk, a_vec, ar[p], k0 + 8 * ah[p], d.k);
#pragma unroll
        for (int p = 0; p < PB; ++p)
            if (b_on[p]) load8(rb[p], Bb, d.sBn, d.sBk, b_vec, br[p], k0 + 8 * bh[p], d.k);
    };
    auto store_slab = [&](int buf) {
#pragma unroll
        for (int p = 0; p < PA; ++p)
            if (a_on[p])
#pragma unroll
                for (int q = 0; q < 8; ++q) As[buf][8 * ah[p] + q][ar[p]] = ra[p][q];
#pragma unroll
        for (int p = 0; p < PB; ++p)
            if (b_on[p])
#pragma unroll
                for (int q = 0; q < 8; ++q) Bs[buf][8 * bh[p] + q][br[p]] = rb[p][q];
    };
    // Persistent: a block takes tiles first, first + G, ... (G = grid size);
    // the first slab of its next tile is loaded while the last slab of the
    // current one is multiplied, so the loads overlap the MFMAs and the
    // output stores of the tile before.
    int64_t tile = blockIdx.x;
    if (gridDim.x % 8 == 0) tile = int64_t(blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    if (tile >= n_tiles) return;
    const float2 *Ab, *Bb;
    int64_t bi, tm, tn;
    panels(tile, Ab, Bb, bi, tm, tn);
    load_slab(Ab, Bb, 0);
    for (;;) {
        const int64_t next = tile + gridDim.x;
        floatx16 acc[BM][BN][2];
#pragma unroll
        for (int i = 0; i < BM; ++i)
#pragma unroll
            for (int j = 0; j < BN; ++j)
#pragma unroll
                for (int v = 0; v < 16; ++v) { acc[i][j][0][v] = 0.f; acc[i][j][1][v] = 0.f; }
        store_slab(0);
        __syncthreads();
        for (int s = 0; s < n_slabs; ++s) {
            const int buf = s & 1;
            const bool more = s + 1 < n_slabs;
            if (more) {
                load_slab(Ab, Bb, int64_t(s + 1) * KT);
            } else if (next < n_tiles) {
                // The next tile's panels (its indices are recomputed after
                // this tile's output is written).
                int64_t x0, x1, x2;
                panels(next, Ab, Bb, x0, x1, x2);
                load_slab(Ab, Bb, 0);
            }
#pragma unroll
            for (int kk = 0; kk < KT; kk += 2) {
                const int kr = kk + (lane >> 5);
                float2 a[BM], b[BN];
#pragma unroll
                for (int i = 0; i < BM; ++i) a[i] = As[buf][kr][wm * 32 * BM + i * 32 + (lane & 31)];
#pragma unroll
                for (int j = 0; j < BN; ++j) b[j] = Bs[buf][kr][wn * 32 * BN + j * 32 + (lane & 31)];
#pragma unroll
                for (int i = 0; i < BM; ++i)
#pragma unroll
                    for (int j = 0; j < BN; ++j) {
                        acc[i][j][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].x, b[j].x, acc[i][j][0], 0, 0, 0);
                        acc[i][j][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].x, b[j].y, acc[i][j][1], 0, 0, 0);
                    }
#pragma unroll
                for (int i = 0; i < BM; ++i)
#pragma unroll
                    for (int j = 0; j < BN; ++j) {
                        acc[i][j][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(-a[i].y, b[j].y, acc[i][j][0], 0, 0, 0);
                        acc[i][j][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].y, b[j].x, acc[i][j][1], 0, 0, 0);
                    }
            }
            if (more) store_slab(buf ^ 1);
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < BM; ++i)
#pragma unroll
            for (int j = 0; j < BN; ++j) {
                const CBlock cb = c_block(d, bi, tm * TM + wm * 32 * BM + i * 32, tn * TN + wn * 32 * BN + j * 32, lane);
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    *c_at(cb, v) = make_float2(acc[i][j][0][v], acc[i][j][1][v]);
                    if (AMAX) mx = fmaxf(mx, fmaxf(fabsf(acc[i][j][0][v]), fabsf(acc[i][j][1][v])));
                }
            }
        if (next >= n_tiles) break;
        tile = next;
        tn = tile % tiles_n;
        tm = (tile / tiles_n) % tiles_m;
        bi = tile / (tiles_n * tiles_m);
    }
    if (AMAX && d.amax_c) block_amax(mx, d.amax_c);
}

// 16-wide MFMA form for a short output dimension (n = 8 or a multiple of 16)
// with a long m -- through the transposed product also the reverse -- and
// for 16 x 16 tiles with a long k split into parts.  Each wave owns one
// 16 x 16 output tile and reads its operands straight into registers in the
// v_mfma_f32_16x16x4_f32 layout: lane l holds row (of A) and column (of B)
// l mod 16 and, of every chunk of 16 k, the four consecutive k from
// 4 (l / 16) -- 32 contiguous bytes per lane where k is the fast axis,
// 16-lane runs along the row or column otherwise -- and the chunk's four
// products pair A's and B's k lane group by lane group (4M complex form, 16
// MFMAs per chunk).  The next chunk is loaded while the current one is
// multiplied.  Tiles are dealt to the grid's waves in turn; with n = 8 the
// upper eight columns are zeros that are not stored.  No LDS, no barriers.
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

template <int NC>
__global__ void __launch_bounds__(256) gemm_mfma16_kernel(GemmDesc d) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, c = lane & 15;
    const bool bcol = NC == 16 || c < NC;
    const int64_t tiles_m = d.m / 16, tiles_n = NC == 16 ? d.n / 16 : 1;
    const int64_t n_tiles = d.nb * tiles_m * tiles_n;
    const int64_t waves = int64_t(gridDim.x) * (blockDim.x >> 6);
    const int n_chunks = int((d.k + 15) / 16);
    const bool a_vec = d.sAk == 1 && d.sAm % 2 == 0 && d.sAb % 2 == 0 && d.sAp % 2 == 0 && (uintptr_t)d.A % 16 == 0;
    const bool b_vec = d.sBk == 1 && d.sBn % 2 == 0 && d.sBb % 2 == 0 && d.sBp % 2 == 0 && (uintptr_t)d.B % 16 == 0;
    float mx = 0.f;
    for (int64_t tile = int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6); tile < n_tiles; tile += waves) {
        const int64_t tn = tile % tiles_n, tm = (tile / tiles_n) % tiles_m, bi = tile / (tiles_n * tiles_m);
        const int64_t bq = d.kparts == 1 ? bi : bi / d.kparts, bp = bi - bq * d.kparts;
        const float2 *Ar = d.A + bq * d.sAb + bp * d.sAp + (tm * 16 + c) * d.sAm;
        const float2 *Bc = d.B + bq * d.sBb + bp * d.sBp + (tn * 16 + (bcol ? c : 0)) * d.sBn;
        // Four consecutive k from 4 g of chunk ch (zero past k or past n).
        auto load = [&](int ch, float2 (&x)[4], float2 (&y)[4]) {
            const int64_t k0 = int64_t(ch) * 16 + 4 * g;
            if (k0 < d.k) {
                if (a_vec) {
                    const float4 u = *(const float4 *)(Ar + k0), w = *(const float4 *)(Ar + k0 + 2);
                    x[0] = make_float2(u.x, u.y); x[1] = make_float2(u.z, u.w);
                    x[2] = make_float2(w.x, w.y); x[3] = make_float2(w.z, w.w);
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) x[q] = Ar[(k0 + q) * d.sAk];
                }
                if (!bcol) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) y[q] = make_float2(0.f, 0.f);
                } else if (b_vec) {
                    const float4 u = *(const float4 *)(Bc + k0), w = *(const float4 *)(Bc + k0 + 2);
                    y[0] = make_float2(u.x, u.y); y[1] = make_float2(u.z, u.w);
                    y[2] = make_float2(w.x, w.y); y[3] = make_float2(w.z, w.w);
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) y[q] = Bc[(k0 + q) * d.sBk];
                }
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) { x[q] = make_float2(0.f, 0.f); y[q] = make_float2(0.f, 0.f); }
            }
        };
        floatx4 re = {0.f, 0.f, 0.f, 0.f}, im = {0.f, 0.f, 0.f, 0.f};
        float2 a[4], b[4], an[4], bn[4];
        load(0, a, b);
        for (int ch = 0; ch < n_chunks; ++ch) {
            if (ch + 1 < n_chunks) load(ch + 1, an, bn);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                re = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j].x, b[j].x, re, 0, 0, 0);
                im = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j].x, b[j].y, im, 0, 0, 0);
                re = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[j].y, b[j].y, re, 0, 0, 0);
                im = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j].y, b[j].x, im, 0, 0, 0);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) { a[q] = an[q]; b[q] = bn[q]; }
        }
        // Lane l holds rows 4 (l / 16) + v, column l mod 16.
        if (bcol) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                d.C[c_off(d, bi, tm * 16 + 4 * g + v, tn * 16 + c)] = make_float2(re[v], im[v]);
                mx = fmaxf(mx, fmaxf(fabsf(re[v]), fabsf(im[v])));
            }
        }
    }
    if (d.amax_c) block_amax(mx, d.amax_c);
}

// ------------------------------------------------ streaming MFMA form
// Tall products whose B operand (k x n per batch entry) is small: n = 32 or
// 64 with k = 8, 16 or 32, or n = 32 with k = 64.  Each wave keeps its batch entry's whole B in
// registers, in the v_mfma_f32_32x32x2_f32 operand layout, and streams 32-row
// blocks of A straight from memory into registers, loading the next block
// before multiplying the current one: no LDS and no barriers, so the output
// stores of one block overlap the next block's loads and MFMAs.  Row blocks
// are dealt to the waves in turn, so the waves in flight read and write
// neighbouring rows (B is reloaded where a wave's next block lies in another
// batch entry).  The k order inside an MFMA is free as long as
// both operands follow it: step s of lane half h (lane / 32) takes
// k = h (k / 2) + s, so a lane reads k / 2 consecutive values of its row of A
// (16-byte loads when k is A's fast axis, AKF).
template <int NB, int KK, bool AKF>
__global__ void __launch_bounds__(256, 2) gemm_mfma_stream_kernel(GemmDesc d) {
    constexpr int S = KK / 2;
    const int lane = threadIdx.x & 63, h = lane >> 5, r = lane & 31;
    const int64_t mb = d.m / 32, R = d.nb * mb;
    const int64_t W = int64_t(gridDim.x) * 4, w = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    float mx = 0.f;  // max(|re|, |im|) written, folded into amax_c when the program tracks it
    float bre[S][NB], bim[S][NB];
    float2 a[S], an[S];
    auto load_a = [&](float2 (&x)[S], int64_t rb) {
        const int64_t bi = rb / mb, tm = rb - bi * mb;
        const float2 *p = d.A + bi * d.sAb + (tm * 32 + r) * d.sAm + int64_t(h * S) * d.sAk;
        if constexpr (AKF) {
#pragma unroll
            for (int s = 0; s < S; s += 2) {
                const float4 q = *(const float4 *)(p + s);
                x[s] = make_float2(q.x, q.y);
                x[s + 1] = make_float2(q.z, q.w);
            }
        } else {
#pragma unroll
            for (int s = 0; s < S; ++s) x[s] = p[s * d.sAk];
        }
    };
    int64_t cur = -1;
    if (w < R) load_a(a, w);
    for (int64_t rb = w; rb < R; rb += W) {
        const int64_t bi = rb / mb, tm = rb - bi * mb;
        if (bi != cur) {
            cur = bi;
            const float2 *q = d.B + bi * d.sBb + int64_t(h * S) * d.sBk + r * d.sBn;
#pragma unroll
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const float2 v = q[s * d.sBk + j * 32 * d.sBn];
                    bre[s][j] = v.x;
                    bim[s][j] = v.y;
                }
        }
        if (rb + W < R) load_a(an, rb + W);
        floatx16 acc[NB][2];
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) { acc[j][0][v] = 0.f; acc[j][1][v] = 0.f; }
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                acc[j][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s].x, bre[s][j], acc[j][0], 0, 0, 0);
                acc[j][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(-a[s].y, bim[s][j], acc[j][0], 0, 0, 0);
                acc[j][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s].x, bim[s][j], acc[j][1], 0, 0, 0);
                acc[j][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s].y, bre[s][j], acc[j][1], 0, 0, 0);
            }
        // Nontemporal stores: the block is not read again by this launch
        // (measured 3-17% faster on the 70-qubit chunk's streaming steps).
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const CBlock cb = c_block(d, bi, tm * 32, j * 32, lane);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                f32x2 y;
                y.x = acc[j][0][v];
                y.y = acc[j][1][v];
                __builtin_nontemporal_store(y, (f32x2 *)c_at(cb, v));
            }
            if (d.amax_c)
#pragma unroll
                for (int v = 0; v < 16; ++v) mx = fmaxf(mx, fmaxf(fabsf(acc[j][0][v]), fabsf(acc[j][1][v])));
        }
#pragma unroll
        for (int s = 0; s < S; ++s) a[s] = an[s];
    }
    if (d.amax_c) block_amax(mx, d.amax_c);
}

// The same streaming scheme on v_mfma_f32_16x16x4_f32 for n = 8 or 16 and
// k <= 64 (a multiple of 4): the batch entry's B (KC chunks of 16 k) in
// registers, 16-row blocks of A dealt to the waves in turn, each block's
// whole k loaded into registers one block ahead.  Operand layout as in the
// 16-wide form above (lane l: row / column l mod 16, four consecutive k from
// 4 (l / 16) of each 16-k chunk; groups past k are zeros).
template <int NC, int KC, bool AV>
__global__ void __launch_bounds__(256) gemm_mfma16_stream_kernel(GemmDesc d) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, c = lane & 15;
    const bool bcol = NC == 16 || c < NC;
    const int64_t mb = d.m / 16, R = d.nb * mb;
    const int64_t W = int64_t(gridDim.x) * 4, w = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    float mx = 0.f;  // max(|re|, |im|) written, folded into amax_c when the program tracks it
    float2 b[KC][4], a[KC][4], an[KC][4];
    auto load_a = [&](float2 (&x)[KC][4], int64_t rb) {
        const int64_t bi = rb / mb, tm = rb - bi * mb;
        const float2 *Ar = d.A + bi * d.sAb + (tm * 16 + c) * d.sAm;
#pragma unroll
        for (int ch = 0; ch < KC; ++ch) {
            const int64_t k0 = int64_t(ch) * 16 + 4 * g;
            if (k0 < d.k) {
                if constexpr (AV) {
                    const float4 u = *(const float4 *)(Ar + k0), v = *(const float4 *)(Ar + k0 + 2);
                    x[ch][0] = make_float2(u.x, u.y); x[ch][1] = make_float2(u.z, u.w);
                    x[ch][2] = make_float2(v.x, v.y); x[ch][3] = make_float2(v.z, v.w);
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) x[ch][q] = Ar[(k0 + q) * d.sAk];
                }
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) x[ch][q] = make_float2(0.f, 0.f);
            }
        }
    };
    int64_t cur = -1;
    if (w < R) load_a(a, w);
    for (int64_t rb = w; rb < R; rb += W) {
        const int64_t bi = rb / mb, tm = rb - bi * mb;
        if (bi != cur) {
            cur = bi;
            const float2 *Bc = d.B + bi * d.sBb + (bcol ? c : 0) * d.sBn;
#pragma unroll
            for (int ch = 0; ch < KC; ++ch) {
                const int64_t k0 = int64_t(ch) * 16 + 4 * g;
#pragma unroll
                for (int q = 0; q < 4; ++q) b[ch][q] = (bcol && k0 < d.k) ? Bc[(k0 + q) * d.sBk] : make_float2(0.f, 0.f);
            }
        }
        if (rb + W < R) load_a(an, rb + W);
        floatx4 re = {0.f, 0.f, 0.f, 0.f}, im = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ch = 0; ch < KC; ++ch)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                re = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ch][j].x, b[ch][j].x, re, 0, 0, 0);
                im = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ch][j].x, b[ch][j].y, im, 0, 0, 0);
                re = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[ch][j].y, b[ch][j].y, re, 0, 0, 0);
                im = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ch][j].y, b[ch][j].x, im, 0, 0, 0);
            }
        // Lane l holds rows 4 (l / 16) + v, column l mod 16 (nontemporal
        // stores, as in the 32-wide streaming form).
        if (bcol) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                f32x2 y;
                y.x = re[v];
                y.y = im[v];
                __builtin_nontemporal_store(y, (f32x2 *)(d.C + c_off(d, bi, tm * 16 + 4 * g + v, c)));
                mx = fmaxf(mx, fmaxf(fabsf(re[v]), fabsf(im[v])));
            }
        }
#pragma unroll
        for (int ch = 0; ch < KC; ++ch)
#pragma unroll
            for (int q = 0; q < 4; ++q) a[ch][q] = an[ch][q];
    }
    if (d.amax_c) block_amax(mx, d.amax_c);
}

static int device_cus();
namespace {
GemmDesc transposed(const GemmDesc &d);
}

// Whether the streaming form applies to d as it is (n and k fixed by the
// instances; no split over k).
static bool stream_ok(const GemmDesc &d) {
    return d.kparts == 1 && d.m % 32 == 0 && d.m >= 32 &&
           (((d.n == 32 || d.n == 64) && (d.k == 8 || d.k == 16 || d.k == 32)) || (d.n == 32 && d.k == 64));
}

static bool stream16_ok(const GemmDesc &d) {
    return d.kparts == 1 && d.m % 16 == 0 && d.m >= 16 && (d.n == 16 || d.n == 8) && d.k % 4 == 0 && d.k >= 4 &&
           d.k <= 64;
}

static void launch_stream16(const GemmDesc &d, hipStream_t st) {
    const int kc = int((d.k + 15) / 16);
    // Workgroups per compute unit as the instance's registers allow.
    const int per_cu = kc == 1 ? 6 : kc == 2 ? 4 : 3;
    const int64_t blocks = (d.nb * (d.m / 16) + 3) / 4, cap = per_cu * int64_t(device_cus());
    const unsigned g = (unsigned)(blocks < cap ? blocks : cap);
    const bool av = d.sAk == 1 && d.sAm % 2 == 0 && d.sAb % 2 == 0 && (uintptr_t)d.A % 16 == 0;
#define QC_S16(NC, KC)                                                                                    \
    do {                                                                                                  \
        if (av)                                                                                           \
            hipLaunchKernelGGL((gemm_mfma16_stream_kernel<NC, KC, true>), dim3(g), dim3(256), 0, st, d);  \
        else                                                                                              \
            hipLaunchKernelGGL((gemm_mfma16_stream_kernel<NC, KC, false>), dim3(g), dim3(256), 0, st, d); \
    } while (0)
    if (d.n == 16) {
        if (kc == 1) QC_S16(16, 1);
        else if (kc == 2) QC_S16(16, 2);
        else if (kc == 3) QC_S16(16, 3);
        else QC_S16(16, 4);
    } else {
        if (kc == 1) QC_S16(8, 1);
        else if (kc == 2) QC_S16(8, 2);
        else if (kc == 3) QC_S16(8, 3);
        else QC_S16(8, 4);
    }
#undef QC_S16
}

static void launch_stream(const GemmDesc &d, hipStream_t st) {
    // Workgroups per compute unit as the instance's registers allow.
    const int per_cu = d.n == 32 ? (d.k <= 16 ? 4 : d.k == 32 ? 3 : 2) : (d.k == 8 ? 3 : 2);
    const int64_t blocks = (d.nb * (d.m / 32) + 3) / 4, cap = per_cu * int64_t(device_cus());
    const unsigned g = (unsigned)(blocks < cap ? blocks : cap);
    const bool akf = d.sAk == 1 && d.sAm % 2 == 0 && d.sAb % 2 == 0 && (uintptr_t)d.A % 16 == 0;
#define QC_STREAM(NB, KK)                                                                                 \
    do {                                                                                                  \
        if (akf)                                                                                          \
            hipLaunchKernelGGL((gemm_mfma_stream_kernel<NB, KK, true>), dim3(g), dim3(256), 0, st, d);         \
        else                                                                                              \
            hipLaunchKernelGGL((gemm_mfma_stream_kernel<NB, KK, false>), dim3(g), dim3(256), 0, st, d);        \
    } while (0)
    if (d.n == 32) {
        if (d.k == 8) QC_STREAM(1, 8);
        else if (d.k == 16) QC_STREAM(1, 16);
        else if (d.k == 32) QC_STREAM(1, 32);
        else QC_STREAM(1, 64);
    } else {
        if (d.k == 8) QC_STREAM(2, 8);
        else if (d.k == 16) QC_STREAM(2, 16);
        else QC_STREAM(2, 32);
    }
#undef QC_STREAM
}

// ----------------------------------------------------------- GEMM variants
// Every kernel form a GEMM step can run as.  gemm_variant_ok says whether a
// form applies to a shape (tile divisibility, k, precision); the default
// choice follows fixed rules, the autotuner may pick another applicable one.
// Compute units of the current device (looked up once per device).
static int device_cus() {
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cus[dev] = n;
    }
    return cus[dev];
}

// Tile of a tall or wide FP32 MFMA form.
static void tile_dims(int v, int &tm, int &tn) {
    switch (v) {
        case kVarT256x64: tm = 256; tn = 64; break;
        case kVarT64x256: tm = 64; tn = 256; break;
        case kVarT32x256: tm = 32; tn = 256; break;
        case kVarT256x32: tm = 256; tn = 32; break;
        case kVarT128x64: tm = 128; tn = 64; break;
        case kVarT64x128: tm = 64; tn = 128; break;
        case kVarT128x32: tm = 128; tn = 32; break;
        default: tm = 32; tn = 128; break;
    }
}

bool gemm_variant_ok(const GemmDesc &d, int v) {
    const bool split = d.prec != kPrecC64;
    const int64_t kt = d.k >= 16 ? 16 : d.k;
    const bool k_fp32 = (kt == 2 || kt == 4 || kt == 8 || kt == 16) && d.k % kt == 0;
    const bool m_pow2_16 = d.m == 1 || d.m == 2 || d.m == 4 || d.m == 8 || d.m == 16;
    switch (v) {
        case kVarValu: return true;
        case kVarSkinny: return d.n >= 64 && m_pow2_16;
        case kVarSkinnyT: return d.m >= 64 && (d.n == 1 || d.n == 2 || d.n == 4 || d.n == 8 || d.n == 16);
        case kVarDotTile: return d.m * d.n <= 256 && d.k >= 64;
        case kVarRows: return d.m >= 64 && (d.n == 1 || d.n == 2 || d.n == 4 || d.n == 8 || d.n == 16);
        // 16-wide MFMA (FP32 for every precision, like the other small-shape forms).
        case kVarMfma16: return (d.n % 16 == 0 || d.n == 8) && d.m % 16 == 0 && d.k % 4 == 0 && d.k >= 4;
        case kVarMfma16T: return (d.m % 16 == 0 || d.m == 8) && d.n % 16 == 0 && d.k % 4 == 0 && d.k >= 4;
        // Streaming form (FP32 for every precision): B in registers, A streamed.
        case kVarStream: return stream_ok(d);
        case kVarStreamT: return stream_ok(transposed(d));
        case kVarStream16: return stream16_ok(d);
        case kVarDot: return d.k >= 256 && d.nb * d.m * d.n <= 65536;
        // Complex FP32 MFMA forms (any precision: a split program's step may
        // run in FP32 where the tuner measured it faster).
        case kVarMfma11: case kVarMfma12: case kVarMfma21: case kVarMfma22: {
            const int wm = (v == kVarMfma21 || v == kVarMfma22) ? 2 : 1, wn = (v == kVarMfma12 || v == kVarMfma22) ? 2 : 1;
            return k_fp32 && d.m % (32 * wm) == 0 && d.n % (32 * wn) == 0;
        }
        // The large-tile and tile forms stage k in groups of 8 (load8).
        case kVarSplitBig: return split && d.k % 8 == 0 && d.m % 128 == 0 && d.n % 128 == 0;
        case kVarSplitBig64: return split && d.k % 8 == 0 && d.m % 128 == 0 && d.n % 64 == 0;
        case kVarMfmaBig: return d.k % 8 == 0 && d.m % 128 == 0 && d.n % 128 == 0;
        case kVarT256x64: case kVarT64x256: case kVarT32x256: case kVarT256x32: case kVarT128x64: case kVarT64x128:
        case kVarT128x32: case kVarT32x128: {
            int tm = 0, tn = 0;
            tile_dims(v, tm, tn);
            return d.k % 8 == 0 && d.m % tm == 0 && d.n % tn == 0;
        }
        case kVarSplit11: case kVarSplit12: case kVarSplit21: case kVarSplit22: {
            const int wm = (v == kVarSplit21 || v == kVarSplit22) ? 2 : 1, wn = (v == kVarSplit12 || v == kVarSplit22) ? 2 : 1;
            return split && d.k >= 2 && d.m % (32 * wm) == 0 && d.n % (32 * wn) == 0;
        }
        default: return false;
    }
}

bool gemm_variant_16bit(int v) {
    return v == kVarSplitBig || v == kVarSplitBig64 || v == kVarSplit11 || v == kVarSplit12 || v == kVarSplit21 ||
           v == kVarSplit22;
}

int gemm_default_variant(const GemmDesc &d) {
    if (d.prec != kPrecC64 && gemm_variant_ok(d, kVarSplitBig)) return kVarSplitBig;
    if (d.prec == kPrecC64 && gemm_variant_ok(d, kVarMfmaBig)) return kVarMfmaBig;
    // Tall or wide shapes with a 32- or 64-wide side (measured fastest on
    // such steps of the 70-qubit workload).
    if (d.prec == kPrecC64 && d.m >= 1024) {
        if (d.n == 64 && gemm_variant_ok(d, kVarT128x64)) return kVarT128x64;
        if (d.n == 32 && gemm_variant_ok(d, kVarT128x32)) return kVarT128x32;
    }
    if (d.prec == kPrecC64 && d.n >= 1024 && d.m == 32 && gemm_variant_ok(d, kVarT32x128)) return kVarT32x128;
    // A 16-wide side with a long other one: one 16x16 MFMA tile per wave.
    if (d.n == 16 && d.m >= 256 && gemm_variant_ok(d, kVarMfma16)) return kVarMfma16;
    if (d.m == 16 && d.n >= 256 && gemm_variant_ok(d, kVarMfma16T)) return kVarMfma16T;
    const int wm = d.m % 64 == 0 ? 2 : 1, wn = d.n % 64 == 0 ? 2 : 1;
    if (d.prec != kPrecC64) {
        const int v = wm == 2 ? (wn == 2 ? kVarSplit22 : kVarSplit21) : (wn == 2 ? kVarSplit12 : kVarSplit11);
        if (gemm_variant_ok(d, v)) return v;
    } else {
        const int v = wm == 2 ? (wn == 2 ? kVarMfma22 : kVarMfma21) : (wn == 2 ? kVarMfma12 : kVarMfma11);
        if (gemm_variant_ok(d, v)) return v;
    }
    if (d.k >= 1024 && gemm_variant_ok(d, kVarDotTile)) return kVarDotTile;
    if (d.k >= 4096 && d.nb * d.m * d.n <= 4096) return kVarDot;
    if (d.n >= 256 && gemm_variant_ok(d, kVarSkinny)) return kVarSkinny;
    if (d.m >= 256 && gemm_variant_ok(d, kVarRows)) return kVarRows;
    return kVarValu;
}

// Sum of the k parts of a split product: element (b, i, j) of C = sum over p
// in increasing order of the parts' values (FP32), read from the scratch
// P[b][p][i][j]; the maximum of |re|, |im| of C is recorded.
__global__ void __launch_bounds__(256) ksum_kernel(GemmDesc d) {
    float mx = 0.f;
    const int64_t mn = d.m * d.n, total = d.nb * mn;
    for (int64_t f = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; f < total; f += int64_t(gridDim.x) * blockDim.x) {
        const int64_t b = f / mn, r = f - b * mn;
        const float2 *src = d.kscratch + b * d.kparts * mn + r;
        float2 acc = src[0];
        for (int64_t p = 1; p < d.kparts; ++p) {
            const float2 v = src[p * mn];
            acc.x += v.x;
            acc.y += v.y;
        }
        const int64_t i = r / d.n;
        d.C[c_off(d, b, i, r - i * d.n)] = acc;
        mx = fmaxf(mx, fmaxf(fabsf(acc.x), fabsf(acc.y)));
    }
    if (d.amax_c) block_amax(mx, d.amax_c);
}

namespace {
template <int WM, int WN>
void launch_mfma(const GemmDesc &d, hipStream_t st) {
    const int64_t tiles = d.nb * (d.m / (32 * WM)) * (d.n / (32 * WN));
    const unsigned grid = (unsigned)(tiles < 1048576 ? tiles : 1048576);
    switch (d.k >= 16 ? 16 : int(d.k)) {
        case 2: hipLaunchKernelGGL((gemm_mfma_kernel<WM, WN, 2>), dim3(grid), dim3(64 * WM * WN), 0, st, d); break;
        case 4: hipLaunchKernelGGL((gemm_mfma_kernel<WM, WN, 4>), dim3(grid), dim3(64 * WM * WN), 0, st, d); break;
        case 8: hipLaunchKernelGGL((gemm_mfma_kernel<WM, WN, 8>), dim3(grid), dim3(64 * WM * WN), 0, st, d); break;
        default: hipLaunchKernelGGL((gemm_mfma_kernel<WM, WN, 16>), dim3(grid), dim3(64 * WM * WN), 0, st, d); break;
    }
}

template <int WM, int WN>
void launch_split(const GemmDesc &d, hipStream_t st) {
    const int64_t tiles = d.nb * (d.m / (32 * WM)) * (d.n / (32 * WN));
    const unsigned grid = (unsigned)(tiles < 1048576 ? tiles : 1048576);
    if (d.prec == kPrecFP16)
        hipLaunchKernelGGL((gemm_split_kernel<_Float16, WM, WN>), dim3(grid), dim3(64 * WM * WN), 0, st, d);
    else
        hipLaunchKernelGGL((gemm_split_kernel<__bf16, WM, WN>), dim3(grid), dim3(64 * WM * WN), 0, st, d);
}
void launch_skinny(const GemmDesc &d, hipStream_t st) {
    // Fewer workgroups when each folds a maximum into one slot.
    const int64_t blocks = d.nb * ((d.n + 511) / 512), cap = d.amax_c ? 2048 : 8192;
    const unsigned g = (unsigned)(blocks < cap ? blocks : cap);
    switch (d.m) {
        case 1: hipLaunchKernelGGL(gemm_skinny_kernel<1>, dim3(g), dim3(256), 0, st, d); break;
        case 2: hipLaunchKernelGGL(gemm_skinny_kernel<2>, dim3(g), dim3(256), 0, st, d); break;
        case 4: hipLaunchKernelGGL(gemm_skinny_kernel<4>, dim3(g), dim3(256), 0, st, d); break;
        case 8: hipLaunchKernelGGL(gemm_skinny_kernel<8>, dim3(g), dim3(256), 0, st, d); break;
        default: hipLaunchKernelGGL(gemm_skinny_kernel<16>, dim3(g), dim3(256), 0, st, d); break;
    }
}

// The same product as C^T = B^T A^T: operands swapped and transposed through
// their strides, C's index roles swapped (strides, or the scatter positions
// of its row and column bits).
GemmDesc transposed(const GemmDesc &d) {
    GemmDesc t = d;
    t.A = d.B; t.B = d.A;
    t.m = d.n; t.n = d.m;
    t.sAb = d.sBb; t.sAm = d.sBn; t.sAk = d.sBk;
    t.sBb = d.sAb; t.sBk = d.sAk; t.sBn = d.sAm;
    t.sCb = d.sCb; t.sCm = d.sCn; t.sCn = d.sCm;
    t.sAp = d.sBp; t.sBp = d.sAp;
    t.amax_a = d.amax_b; t.amax_b = d.amax_a;
    if (d.cscatter) {
        t.cbm = d.cbn;
        t.cbn = d.cbm;
        for (int q = 0; q < d.cbm; ++q) t.cpos[q] = d.cpos[d.cbn + q];
        for (int q = 0; q < d.cbn; ++q) t.cpos[d.cbm + q] = d.cpos[q];
    }
    return t;
}

void launch_dot(const GemmDesc &d, hipStream_t st) {
    const int64_t outs = d.nb * d.m * d.n;
    const unsigned g = (unsigned)(outs < 65536 ? outs : 65536);
    hipLaunchKernelGGL(gemm_dot_kernel, dim3(g), dim3(1024), 0, st, d);
}

// The forms that can run split over k (large-tile and dot) as they are, then
// split over k.
const char *launch_big(const GemmDesc &d, int v, hipStream_t st) {
    if (v == kVarDot) {
        launch_dot(d, st);
        return "gemm_dot";
    }
    if (v == kVarDotTile) {
        const unsigned g = (unsigned)(d.nb < 65536 ? d.nb : 65536);
        hipLaunchKernelGGL(gemm_dot_tile_kernel, dim3(g), dim3(256), 0, st, d);
        return "gemm_dot_tile";
    }
    if (v == kVarMfma16 || v == kVarMfma16T) {
        const GemmDesc e = v == kVarMfma16T ? transposed(d) : d;
        const int64_t tiles = e.nb * (e.m / 16) * (e.n % 16 == 0 ? e.n / 16 : 1);
        const int64_t blocks = (tiles + 3) / 4, cap = 8 * int64_t(device_cus());
        const unsigned gb = (unsigned)(blocks < cap ? blocks : cap);
        if (e.n % 16 == 0)
            hipLaunchKernelGGL(gemm_mfma16_kernel<16>, dim3(gb), dim3(256), 0, st, e);
        else
            hipLaunchKernelGGL(gemm_mfma16_kernel<8>, dim3(gb), dim3(256), 0, st, e);
        return "gemm_mfma";
    }
    if (v >= kVarT256x64 && v <= kVarT32x128) {
        int tm = 0, tn = 0;
        tile_dims(v, tm, tn);
        // Persistent blocks, two per compute unit.
        const int64_t tiles = d.nb * (d.m / tm) * (d.n / tn), cap = 2 * int64_t(device_cus());
        const unsigned gt = (unsigned)(tiles < cap ? tiles : cap);
#define QC_TILE(BM, BN, WGM, WGN)                                                                          \
    do {                                                                                                   \
        if (d.amax_c)                                                                                      \
            hipLaunchKernelGGL((gemm_mfma_tile_kernel<BM, BN, WGM, WGN, true>), dim3(gt), dim3(256), 0, st, d);  \
        else                                                                                               \
            hipLaunchKernelGGL((gemm_mfma_tile_kernel<BM, BN, WGM, WGN, false>), dim3(gt), dim3(256), 0, st, d); \
    } while (0)
        switch (v) {
            case kVarT256x64: QC_TILE(2, 2, 4, 1); break;
            case kVarT64x256: QC_TILE(2, 2, 1, 4); break;
            case kVarT32x256: QC_TILE(1, 2, 1, 4); break;
            case kVarT256x32: QC_TILE(2, 1, 4, 1); break;
            case kVarT128x64: QC_TILE(2, 1, 2, 2); break;
            case kVarT64x128: QC_TILE(1, 2, 2, 2); break;
            case kVarT128x32: QC_TILE(1, 1, 4, 1); break;
            default: QC_TILE(1, 1, 1, 4); break;
        }
#undef QC_TILE
        return "gemm_mfma";
    }
    const int64_t t128 = d.nb * (d.m / 128) * (d.n / 128);
    const unsigned g = (unsigned)(t128 < 1048576 ? t128 : 1048576);
    if (v == kVarMfmaBig) {
        if (d.amax_c)
            hipLaunchKernelGGL(gemm_mfma_big_kernel<true>, dim3(g), dim3(256), 0, st, d);
        else
            hipLaunchKernelGGL(gemm_mfma_big_kernel<false>, dim3(g), dim3(256), 0, st, d);
        return "gemm_mfma";
    }
    if (v == kVarSplitBig64) {
        const int64_t t64 = d.nb * (d.m / 128) * (d.n / 64);
        const unsigned g64 = (unsigned)(t64 < 1048576 ? t64 : 1048576);
        if (d.prec == kPrecFP16)
            hipLaunchKernelGGL((gemm_split_big_kernel<_Float16, 1>), dim3(g64), dim3(256), 0, st, d);
        else
            hipLaunchKernelGGL((gemm_split_big_kernel<__bf16, 1>), dim3(g64), dim3(256), 0, st, d);
        return d.prec == kPrecFP16 ? "gemm_split_fp16" : "gemm_split_bf16";
    }
    if (d.prec == kPrecFP16)
        hipLaunchKernelGGL((gemm_split_big_kernel<_Float16, 2>), dim3(g), dim3(256), 0, st, d);
    else
        hipLaunchKernelGGL((gemm_split_big_kernel<__bf16, 2>), dim3(g), dim3(256), 0, st, d);
    return d.prec == kPrecFP16 ? "gemm_split_fp16" : "gemm_split_bf16";
}

// Callers guarantee: kparts a power of two dividing k, kscratch holding
// kparts * nb * m * n values.
const char *launch_gemm_kparts(const GemmDesc &d, int v, hipStream_t st) {
    GemmDesc e = d;
    e.nb = d.nb * d.kparts;
    e.k = d.k / d.kparts;
    e.sAp = e.k * d.sAk;
    e.sBp = e.k * d.sBk;
    e.C = d.kscratch;
    e.sCb = d.m * d.n; e.sCm = d.n; e.sCn = 1;
    e.cscatter = 0;
    e.amax_c = nullptr;
    const char *split_name = d.prec == kPrecFP16 ? "gemm_split_fp16" : "gemm_split_bf16";
    const char *name = "gemm_mfma";
    switch (v) {
        case kVarMfma11: launch_mfma<1, 1>(e, st); break;
        case kVarMfma12: launch_mfma<1, 2>(e, st); break;
        case kVarMfma21: launch_mfma<2, 1>(e, st); break;
        case kVarMfma22: launch_mfma<2, 2>(e, st); break;
        case kVarSplit11: launch_split<1, 1>(e, st); name = split_name; break;
        case kVarSplit12: launch_split<1, 2>(e, st); name = split_name; break;
        case kVarSplit21: launch_split<2, 1>(e, st); name = split_name; break;
        case kVarSplit22: launch_split<2, 2>(e, st); name = split_name; break;
        default: name = launch_big(e, v, st); break;
    }
    const int64_t total = d.nb * d.m * d.n;
    int64_t grid = (total + 255) / 256;
    grid = grid > 2048 ? 2048 : grid;
    hipLaunchKernelGGL(ksum_kernel, dim3((unsigned)grid), dim3(256), 0, st, d);
    return name;
}
}  // namespace

const char *launch_gemm_variant(const GemmDesc &d, int v, hipStream_t st) {
    const char *split_name = d.prec == kPrecFP16 ? "gemm_split_fp16" : "gemm_split_bf16";
    switch (v) {
        case kVarMfma11: case kVarMfma12: case kVarMfma21: case kVarMfma22:
        case kVarSplit11: case kVarSplit12: case kVarSplit21: case kVarSplit22:
            if (d.kparts > 1) return launch_gemm_kparts(d, v, st);
            switch (v) {
                case kVarMfma11: launch_mfma<1, 1>(d, st); return "gemm_mfma";
                case kVarMfma12: launch_mfma<1, 2>(d, st); return "gemm_mfma";
                case kVarMfma21: launch_mfma<2, 1>(d, st); return "gemm_mfma";
                case kVarMfma22: launch_mfma<2, 2>(d, st); return "gemm_mfma";
                case kVarSplit11: launch_split<1, 1>(d, st); return split_name;
                case kVarSplit12: launch_split<1, 2>(d, st); return split_name;
                case kVarSplit21: launch_split<2, 1>(d, st); return split_name;
                default: launch_split<2, 2>(d, st); return split_name;
            }
        case kVarMfmaBig: case kVarSplitBig: case kVarSplitBig64:
        case kVarT256x64: case kVarT64x256: case kVarT32x256: case kVarT256x32: case kVarT128x64: case kVarT64x128:
        case kVarT128x32: case kVarT32x128: case kVarMfma16: case kVarMfma16T:
            if (d.kparts > 1) return launch_gemm_kparts(d, v, st);
            return launch_big(d, v, st);
        case kVarDot: case kVarDotTile:
            if (d.kparts > 1) return launch_gemm_kparts(d, v, st);
            return launch_big(d, v, st);
        case kVarSkinny:
            launch_skinny(d, st);
            return "gemm_skinny";
        case kVarSkinnyT:
            launch_skinny(transposed(d), st);
            return "gemm_skinny_t";
        case kVarStream:
            launch_stream(d, st);
            return "gemm_mfma";
        case kVarStreamT:
            launch_stream(transposed(d), st);
            return "gemm_mfma";
        case kVarStream16:
            launch_stream16(d, st);
            return "gemm_mfma";
        case kVarRows: {
            const int64_t blocks = d.nb * ((d.m + 255) / 256), cap = d.amax_c ? 2048 : 65536;
            const unsigned g = (unsigned)(blocks < cap ? blocks : cap);
            switch (d.n) {
                case 1: hipLaunchKernelGGL(gemm_rows_kernel<1>, dim3(g), dim3(256), 0, st, d); break;
                case 2: hipLaunchKernelGGL(gemm_rows_kernel<2>, dim3(g), dim3(256), 0, st, d); break;
                case 4: hipLaunchKernelGGL(gemm_rows_kernel<4>, dim3(g), dim3(256), 0, st, d); break;
                case 8: hipLaunchKernelGGL(gemm_rows_kernel<8>, dim3(g), dim3(256), 0, st, d); break;
                default: hipLaunchKernelGGL(gemm_rows_kernel<16>, dim3(g), dim3(256), 0, st, d); break;
            }
            return "gemm_rows";
        }
        default: {
            const int64_t total = d.nb * d.m * d.n;
            int64_t g = (total + 255) / 256;
            if (g > 8192) g = 8192;
            hipLaunchKernelGGL(gemm_valu_kernel, dim3((unsigned)g), dim3(256), 0, st, d);
            return "gemm_valu";
        }
    }
}

const char *launch_gemm(const GemmDesc &d, hipStream_t st) { return launch_gemm_variant(d, gemm_default_variant(d), st); }

// ------------------------------------------------------------------ fused
// One work item = one chunk of 2^b slices (the program's in-flight slice bits,
// b = 0 for one slice) with one bitstring, one wavefront.  Leaves are written
// into LDS from the base table (each element picks its base entry from its
// own index plus up to four bits taken from the chunk's slice id or the
// bitstring), then every step computes its outputs from table-driven LDS
// offsets, and the lanes store the root's 2^b slice values.
// A run-time bit of a leaf element, 16-bit code: base bit position in the low
// 3 bits, source above it (slice bit j < 64, or 64 + qubit of the bitstring);
// 0xffff = none.  Two codes per 32-bit word.
__device__ __forceinline__ int dyn_bit(uint32_t code, uint64_t slice, const uint8_t *row) {
    if (code == 0xffffu) return 0;
    const int src = int(code >> 3);
    const int bit = src < 64 ? int((slice >> src) & 1) : int(row[src - 64] & 1);
    return bit << (code & 7u);
}

__device__ __forceinline__ int dyn_bits(int z, int w, uint64_t slice, const uint8_t *row) {
    return dyn_bit(uint32_t(z) & 0xffffu, slice, row) + dyn_bit(uint32_t(z) >> 16, slice, row) +
           dyn_bit(uint32_t(w) & 0xffffu, slice, row) + dyn_bit(uint32_t(w) >> 16, slice, row);
}

// The same with the bitstring given as bit masks (qubit q is bit q & 63 of
// qm[q >> 6]), uniform over the wavefront.
__device__ __forceinline__ int dyn_bit_m(uint32_t code, uint64_t slice, const uint64_t (&qm)[4]) {
    if (code == 0xffffu) return 0;
    const int src = int(code >> 3);
    uint64_t word = slice;
    int sh = src;
    if (src >= 64) {
        const int q = src - 64;
        word = q < 64 ? qm[0] : q < 128 ? qm[1] : q < 192 ? qm[2] : qm[3];
        sh = q & 63;
    }
    return int((word >> sh) & 1) << (code & 7u);
}

__device__ __forceinline__ int dyn_bits_m(int z, int w, uint64_t slice, const uint64_t (&qm)[4]) {
    return dyn_bit_m(uint32_t(z) & 0xffffu, slice, qm) + dyn_bit_m(uint32_t(z) >> 16, slice, qm) +
           dyn_bit_m(uint32_t(w) & 0xffffu, slice, qm) + dyn_bit_m(uint32_t(w) >> 16, slice, qm);
}

// The fused kernel's workgroup is a single wavefront, whose LDS accesses are
// performed in issue order.  Between levels it is therefore enough that the
// compiler keeps LDS accesses on their side of the boundary (a wavefront-scope
// fence); a workgroup barrier would also wait for outstanding global loads.
__device__ __forceinline__ void wave_step_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One output of a level: the sum over its contracted values of the products
// of LDS operands, in table order (it: first two values; it2: the third and
// fourth when there are four or more; pool: the rest, counted by pool[it.w]).
// Slots are byte offsets from L.
__device__ __forceinline__ const float2 &lds_at(const float2 *L, uint32_t byte_off) {
    return *reinterpret_cast<const float2 *>(reinterpret_cast<const char *>(L) + byte_off);
}

__device__ __forceinline__ void item_acc(const float2 *L, uint32_t w, float &re, float &im) {
    const float2 xa = lds_at(L, w & 0xffffu), yb = lds_at(L, w >> 16);
    re = fmaf(xa.x, yb.x, re);
    re = fmaf(-xa.y, yb.y, re);
    im = fmaf(xa.x, yb.y, im);
    im = fmaf(xa.y, yb.x, im);
}

// Operands of two values are read together, before the products.
__device__ __forceinline__ void item_acc2(const float2 *L, uint32_t u, uint32_t v, float &re, float &im) {
    const float2 x0 = lds_at(L, u & 0xffffu), y0 = lds_at(L, u >> 16);
    const float2 x1 = lds_at(L, v & 0xffffu), y1 = lds_at(L, v >> 16);
    re = fmaf(x0.x, y0.x, re);
    re = fmaf(-x0.y, y0.y, re);
    im = fmaf(x0.x, y0.y, im);
    im = fmaf(x0.y, y0.x, im);
    re = fmaf(x1.x, y1.x, re);
    re = fmaf(-x1.y, y1.y, re);
    im = fmaf(x1.x, y1.y, im);
    im = fmaf(x1.y, y1.x, im);
}

__device__ __forceinline__ float2 item_value(const float2 *L, int4 it, int2 it2, const int32_t *__restrict__ pool) {
    float re = 0.f, im = 0.f;
    item_acc2(L, uint32_t(it.y), uint32_t(it.z), re, im);
    if ((uint32_t(it.x) >> 16) > 2u) {
        item_acc2(L, uint32_t(it2.x), uint32_t(it2.y), re, im);
        if (it.w >= 0) {
            // Values past the fourth: their count is nk - 4 (also stored at
            // pool[it.w]); four slot pairs are loaded at a time, together.
            const int extra = int(uint32_t(it.x) >> 16) - 4;
            // Indexes past the last value repeat it (never used), so every
            // load is issued and consumed on every path.
            for (int j0 = 0; j0 < extra; j0 += 4) {
                uint32_t w[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) w[j] = uint32_t(pool[it.w + 1 + min(j0 + j, extra - 1)]);
                asm volatile("" ::"v"(w[0]), "v"(w[1]), "v"(w[2]), "v"(w[3]));
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (j0 + j < extra) item_acc(L, w[j], re, im);
            }
        }
    }
    return make_float2(re, im);
}

// One wavefront runs PAIRS (slice, bitstring) pairs, each in its own LDS
// region of pair_elems values (the last one, zero_slot, holds 0), level by
// level: every item of a level reads only tensors of lower levels, so a level
// needs no synchronisation inside it.
template <int PAIRS, int W>
__global__ void __launch_bounds__(64 * W)
fused_kernel(const int32_t *__restrict__ level_start, const int4 *__restrict__ items,
             const int2 *__restrict__ items2, const int32_t *__restrict__ pool, const float2 *__restrict__ image, const int4 *__restrict__ elems,
             const double2 *__restrict__ base, const uint8_t *__restrict__ bits, float2 *__restrict__ partial,
             double *__restrict__ out, double *__restrict__ per_slice, FusedScalars S) {
    extern __shared__ float2 lds[];
    constexpr int NT = 64 * W;  // threads per work item
    const int tid = threadIdx.x, lane = tid & 63;
    // Between levels: a wavefront-scope fence for one wavefront, a barrier
    // for several.
    auto step_sync = [] {
        if constexpr (W == 1) wave_step_sync();
        else __syncthreads();
    };
    const int n_bs = 1 << S.m;
    const int64_t n_pairs = S.n_slices << S.m;
    const int64_t n_groups = (n_pairs + PAIRS - 1) / PAIRS;
    // The level starts, one per lane (read back with readlane, no memory
    // round trip per level, up to 63 levels).  The table has n_levels + 1 >= 1
    // entries; lanes past its end repeat the last, and lane 0 is read here on
    // every path, so the load is known to be complete before the loops.
    const bool ls_in_lanes = S.n_levels < 64;
    const int ls_lane = level_start[min(lane, S.n_levels)];
    auto lstart = [&](int l) { return ls_in_lanes ? __builtin_amdgcn_readlane(ls_lane, l) : level_start[l]; };
    const int first_item = __builtin_amdgcn_readlane(ls_lane, 0);
    // Sixteen wavefronts per work item rotate three register sets of
    // prefetched items (below); fewer wavefronts, for which that bookkeeping
    // costs more than it hides, load each thread's next item one pass ahead,
    // starting with its first item, loaded here (all work items are alike).
    constexpr bool kRotate = W >= 16;
    int a1_first = 0;
    int4 cur_first = make_int4(0, 0, 0, -1);
    int2 cur2_first = make_int2(0, 0);
    if constexpr (!kRotate) {
        if (S.n_levels > 0) a1_first = lstart(1);
        if (first_item + tid < a1_first) {
            cur_first = items[first_item + tid];
            cur2_first = items2[first_item + tid];
        }
    }
    // The levels run as a sequence of passes of NT items each; a level's last
    // pass ends with a synchronisation.  take() loads the next pass's items
    // (cursor: level cl, first item cs) and run() computes a loaded pass.
    struct Pass {
        int4 it;
        int2 it2;
        int i, end;
        bool last, valid;
    };
    int cl = 0, cs = 0;
    // take() has no branch on the cursor: past the last level it loads the
    // last item again and marks the pass invalid.  Levels are never empty, so
    // a thread past its level's end loads the level's last item (unused).
    // Plans without levels never load.
    const bool has_levels = S.n_levels > 0;
    auto take = [&](Pass &f) {
        f.valid = cl < S.n_levels;
        const int e = lstart(min(cl + 1, S.n_levels));
        f.i = cs + tid;
        f.end = e;
        f.last = cs + NT >= e;
        if (has_levels) {
            const int ii = min(f.i, e - 1);
            f.it = items[ii];
            f.it2 = items2[ii];
        }
        cl = f.valid && f.last ? cl + 1 : cl;
        cs = !f.valid ? cs : f.last ? e : cs + NT;
    };
    auto run = [&](const Pass &f) {
        // An empty statement that reads the pass's registers on every path,
        // so their loads are complete here even in a wavefront without an
        // item in this pass (the next load into the same registers then has
        // nothing of theirs to wait for).
        asm volatile("" ::"v"(f.it.x), "v"(f.it.y), "v"(f.it.z), "v"(f.it.w), "v"(f.it2.x), "v"(f.it2.y));
        if (f.i < f.end) {
#pragma unroll
            for (int p = 0; p < PAIRS; ++p)
                const_cast<float2 &>(lds_at(lds + p * S.pair_elems, uint32_t(f.it.x) & 0xffffu)) =
                    item_value(lds + p * S.pair_elems, f.it, f.it2, pool);
        }
        if (f.last) step_sync();
    };
    for (int64_t g = blockIdx.x; g < n_groups; g += gridDim.x) {
        // With rotation, the first two passes' items are loaded before the
        // leaves, so that their latency overlaps them.
        Pass A, B, C;
        if constexpr (kRotate) {
            cl = 0;
            cs = first_item;
            take(A);
            take(B);
        }
        // Leaves of every pair: the pair-independent values in one coalesced
        // copy, then the elements whose base entry depends on slice or
        // bitstring bits.  A group past the last pair repeats the last pair.
        for (int p = 0; p < PAIRS; ++p) {
            float2 *L = lds + p * S.pair_elems;
            for (int e = tid; e < S.n_image; e += NT) L[e] = image[e];
            if (tid == 0) L[S.zero_slot] = make_float2(0.f, 0.f);
        }
        step_sync();
        for (int p = 0; p < PAIRS; ++p) {
            const int64_t pair = min(g * PAIRS + p, n_pairs - 1);
            const uint64_t slice = S.sc + (uint64_t(S.first_slice + (pair >> S.m)) << S.b);
            const uint8_t *row = bits + int64_t(min(int(pair & (n_bs - 1)), S.n_bs - 1)) * S.n_qubits;
            // The bitstring as four 64-bit masks (one load per lane and word).
            uint64_t qm[4] = {0, 0, 0, 0};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int q = j * 64 + lane;
                qm[j] = __ballot(q < S.n_qubits && (row[q < S.n_qubits ? q : 0] & 1));
            }
            float2 *L = lds + p * S.pair_elems;
            // Eight element descriptors per lane in flight, then their base
            // values, then the stores.
            for (int e0 = tid; e0 < S.n_elems; e0 += 8 * NT) {
                int4 t[8];
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    if (e0 + j * NT < S.n_elems) t[j] = elems[e0 + j * NT];
                double2 v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    if (e0 + j * NT < S.n_elems) v[j] = base[t[j].y + dyn_bits_m(t[j].z, t[j].w, slice, qm)];
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    if (e0 + j * NT < S.n_elems) L[t[j].x] = make_float2(float(v[j].x), float(v[j].y));
            }
        }
        step_sync();
        // Levels.  With rotation, three passes rotate through the register
        // sets A, B, C: a pass's items are loaded two passes before they are
        // used and read where they were loaded, so their latency overlaps two
        // passes and their synchronisations.
        if constexpr (kRotate) {
            while (true) {
                if (!A.valid) break;
                take(C);
                run(A);
                if (!B.valid) break;
                take(A);
                run(B);
                if (!C.valid) break;
                take(B);
                run(C);
            }
        } else {
            // Each thread's next item (the next stretch of this level, or the
            // first of the next level) is loaded before the current one is
            // computed.  Levels are never empty, so the clamped index is in
            // range; a thread past the end loads the level's last item.
            int a0 = first_item, a1 = a1_first;
            int4 cur = cur_first;
            int2 cur2 = cur2_first;
            for (int lv = 0; lv < S.n_levels; ++lv) {
                const int i0 = a0, i1 = a1;
                const int b1 = lv + 2 <= S.n_levels ? lstart(lv + 2) : i1;
                const int n_it = (i1 - i0 + NT - 1) / NT;
                for (int t = 0; t < n_it; ++t) {
                    const int i = i0 + t * NT + tid;
                    const int nx = t + 1 < n_it ? i + NT : i1 + tid;
                    const int nx_end = t + 1 < n_it ? i1 : b1;
                    const int nxc = min(nx, nx_end - 1);
                    const int4 nxt = items[nxc];
                    const int2 nxt2 = items2[nxc];
                    if (i < i1) {
#pragma unroll
                        for (int p = 0; p < PAIRS; ++p)
                            const_cast<float2 &>(lds_at(lds + p * S.pair_elems, uint32_t(cur.x) & 0xffffu)) =
                                item_value(lds + p * S.pair_elems, cur, cur2, pool);
                    }
                    cur = nxt;
                    cur2 = nxt2;
                }
                step_sync();
                a0 = i1;
                a1 = b1;
            }
        }
        if (out) {
            // The work item is one 64-slice block: its in-range values summed
            // by the reduction's fixed butterfly in FP64 and added to out.
            if (tid < 64) {
                const int64_t pair = g * PAIRS;
                const int bsi = int(pair & (n_bs - 1));
                const uint64_t s = S.sc + (uint64_t(S.first_slice + (pair >> S.m)) << S.b) + uint64_t(tid);
                double re = 0.0, im = 0.0;
                if (s >= S.lo && s < S.hi) {
                    const float2 v = lds[S.root_off + tid];
                    re = double(v.x);
                    im = double(v.y);
                    if (per_slice && bsi < S.n_bs) {
                        double *ps = per_slice + 2 * (int64_t(s - S.s_begin) * S.n_bs + bsi);
                        ps[0] = re;
                        ps[1] = im;
                    }
                }
                re = wave_sum(re);
                im = wave_sum(im);
                if (tid == 0 && bsi < S.n_bs) {
                    out[2 * bsi] += re;
                    out[2 * bsi + 1] += im;
                }
            }
            step_sync();
            continue;
        }
        // A work item's root holds its 2^b slice values in slice order.
        for (int q = tid; q < (PAIRS << S.b); q += NT) {
            const int p = q >> S.b, sl = q & ((1 << S.b) - 1);
            const int64_t pair = g * PAIRS + p;
            if (pair < n_pairs) {
                const int64_t s_rel = ((S.first_slice + (pair >> S.m)) << S.b) + sl;
                partial[(s_rel << S.m) + (pair & (n_bs - 1))] = lds[p * S.pair_elems + S.root_off + sl];
            }
        }
        step_sync();
    }
}


// ---------------------------------------------------------- fused batches
// Many independent requests (each its own plan and bitstring) in one
// launch: a work item is one (request, slice) pair, taken by one wavefront
// in grid-stride order; the request is found by binary search over the
// requests' first items.  Each request keeps its own tables; the workgroup
// allocates the largest pair region among them.  The wavefront that writes
// a request's last slice value stamps the request's completion time
// (done[] counts finished slices per request, in batch order; t_done[] is
// indexed by the request's position in the caller's array).
__global__ void __launch_bounds__(64) fused_batch_kernel(const BatchReq *__restrict__ reqs, int n_reqs,
                                                         int64_t n_items, float2 *__restrict__ partial,
                                                         uint32_t *__restrict__ done, uint64_t *__restrict__ t_done) {
    extern __shared__ float2 lds[];
    const int lane = threadIdx.x;
    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        int lo = 0, hi = n_reqs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (reqs[mid].item_off <= item) lo = mid;
            else hi = mid - 1;
        }
        const BatchReq &R = reqs[lo];
        const int64_t sl = item - R.item_off;
        const uint64_t slice = R.s_begin + uint64_t(sl);
        for (int e = lane; e < R.n_image; e += 64) lds[e] = R.image[e];
        if (lane == 0) lds[R.zero_slot] = make_float2(0.f, 0.f);
        wave_step_sync();
        for (int e = lane; e < R.n_elems; e += 64) {
            const int4 t = R.elems[e];
            const double2 v = R.base[t.y + dyn_bits(t.z, t.w, slice, R.bits)];
            lds[t.x] = make_float2(float(v.x), float(v.y));
        }
        wave_step_sync();
        for (int lv = 0; lv < R.n_levels; ++lv) {
            const int i0 = R.level_start[lv], i1 = R.level_start[lv + 1];
            for (int i = i0 + lane; i < i1; i += 64) {
                const int4 it = R.items[i];
                const int2 it2 = R.items2[i];
                const_cast<float2 &>(lds_at(lds, uint32_t(it.x) & 0xffffu)) = item_value(lds, it, it2, R.pool);
            }
            wave_step_sync();
        }
        if (lane == 0) {
            partial[R.partial_off + (int64_t(slice) - int64_t(R.s_base))] = lds[R.root_off];
            __threadfence();
            if (atomicAdd(&done[lo], 1u) + 1u == uint32_t(R.n_slices)) t_done[R.out_index] = wall_clock64();
        }
        wave_step_sync();
    }
}

void launch_fused_batch(const BatchReq *reqs, int n_reqs, int64_t n_items, int max_pair_elems, float2 *partial,
                        uint32_t *done, uint64_t *t_done, hipStream_t st) {
    if (n_items <= 0) return;
    const unsigned grid = (unsigned)(n_items < 1048576 ? n_items : 1048576);
    hipLaunchKernelGGL(fused_batch_kernel, dim3(grid), dim3(64), size_t(max_pair_elems) * sizeof(float2), st, reqs,
                       n_reqs, n_items, partial, done, t_done);
}

// One workgroup per request: its slice values summed as the single-request
// reduction does (aligned 64-slice blocks, fixed butterfly, blocks in order)
// and added to out[2 r].
__global__ void __launch_bounds__(64) reduce_batch_kernel(const BatchReq *__restrict__ reqs,
                                                          const float2 *__restrict__ partial,
                                                          double *__restrict__ out) {
    const BatchReq &R = reqs[blockIdx.x];
    const int lane = threadIdx.x;
    double acc_re = out[2 * R.out_index], acc_im = out[2 * R.out_index + 1];
    const uint64_t lo = R.s_begin, hi = R.s_begin + uint64_t(R.n_slices);
    for (uint64_t b0 = R.s_base; b0 < hi; b0 += 64) {
        const uint64_t s = b0 + lane;
        double re = 0.0, im = 0.0;
        if (s >= lo && s < hi) {
            const float2 v = partial[R.partial_off + int64_t(s - R.s_base)];
            re = double(v.x);
            im = double(v.y);
        }
        acc_re += wave_sum(re);
        acc_im += wave_sum(im);
    }
    if (lane == 0) {
        out[2 * R.out_index] = acc_re;
        out[2 * R.out_index + 1] = acc_im;
    }
}

void launch_reduce_batch(const BatchReq *reqs, int n_reqs, const float2 *partial, double *out, hipStream_t st) {
    if (n_reqs <= 0) return;
    hipLaunchKernelGGL(reduce_batch_kernel, dim3(n_reqs), dim3(64), 0, st, reqs, partial, out);
}

__global__ void stamp_kernel(uint64_t *t) {
    if (threadIdx.x == 0) t[0] = wall_clock64();
}

void launch_stamp(uint64_t *t, hipStream_t st) { hipLaunchKernelGGL(stamp_kernel, dim3(1), dim3(64), 0, st, t); }

size_t fused_lds_bytes(int pairs, int pair_elems) { return size_t(pairs) * pair_elems * sizeof(float2); }

void launch_fused_pairs(const FusedParams &p, int pairs, int waves, int pair_elems, int zero_slot, hipStream_t st) {
    const int64_t n_pairs = p.n_slices << p.m;
    if (n_pairs <= 0) return;
    const int64_t groups = (n_pairs + pairs - 1) / pairs;
    const unsigned grid = (unsigned)(groups < 1048576 ? groups : 1048576);
    FusedScalars S;
    S.n_levels = p.n_levels;
    S.zero_slot = zero_slot;
    S.n_image = p.n_image;
    S.n_elems = p.n_elems;
    S.n_qubits = p.n_qubits;
    S.m = p.m;
    S.root_off = p.root_off;
    S.pair_elems = pair_elems;
    S.n_bs = p.n_bs;
    S.b = p.b;
    S.first_slice = p.first_slice;
    S.n_slices = p.n_slices;
    S.sc = p.sc;
    S.lo = p.lo;
    S.hi = p.hi;
    S.s_begin = p.s_begin;
    const size_t lds = fused_lds_bytes(pairs, pair_elems);
#define QC_FUSED_CASE(N, WV)                                                                                   \
    case N * 16 + WV:                                                                                         \
        hipLaunchKernelGGL((fused_kernel<N, WV>), dim3(grid), dim3(64 * WV), lds, st, p.level_start, p.items,  \
                           p.items2, p.pool, p.leaf_image, p.elems, p.base, p.bits, p.partial, p.out,         \
                           p.per_slice, S);                                                                    \
        break;
    switch (pairs * 16 + waves) {
        QC_FUSED_CASE(1, 1)
        QC_FUSED_CASE(2, 1)
        QC_FUSED_CASE(4, 1)
        QC_FUSED_CASE(1, 2)
        QC_FUSED_CASE(1, 4)
        QC_FUSED_CASE(1, 8)
        QC_FUSED_CASE(1, 16)
    default: break;
    }
#undef QC_FUSED_CASE
}

// --------------------------------------------------------------- reduce64

// Two launches.  Block sums: one wavefront per (block of 64 slices,
// bitstring) overlapping [lo, hi), the fixed butterfly over the block's
// in-range slice values in FP64 (spread over the whole chip; a wavefront
// sum's cross-lane moves go through each compute unit's LDS crossbar).
__global__ void __launch_bounds__(1024) block_sum_kernel(const float2 *__restrict__ partial, int m, int n_bs,
                                                         uint64_t sc, int64_t n_blocks, int64_t groups, uint64_t lo,
                                                         uint64_t hi, uint64_t s_begin, double2 *__restrict__ bsum,
                                                         double *__restrict__ per_slice) {
    const int lane = threadIdx.x & 63;
    const int bs = int(blockIdx.x / groups);
    const int64_t j = (blockIdx.x % groups) * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (j >= n_blocks) return;
    const uint64_t b0 = sc + uint64_t(j) * 64;
    if (b0 + 64 <= lo || b0 >= hi) return;
    const uint64_t s = b0 + lane;
    double re = 0.0, im = 0.0;
    if (s >= lo && s < hi) {
        const float2 v = partial[(int64_t(s - sc) << m) + bs];
        re = double(v.x);
        im = double(v.y);
        if (per_slice) {
            double *p = per_slice + 2 * (int64_t(s - s_begin) * n_bs + bs);
            p[0] = re;
            p[1] = im;
        }
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) bsum[int64_t(bs) * n_blocks + j] = make_double2(re, im);
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo32 = __builtin_amdgcn_readlane(int(b & 0xffffffffll), l);
    const int hi32 = __builtin_amdgcn_readlane(int(b >> 32), l);
    return __longlong_as_double((long long)(uint32_t(lo32)) | ((long long)hi32 << 32));
}

// Then one wavefront per bitstring adds the block sums to out[bs] in
// increasing block order: 64 at a time are loaded across the lanes and read
// back one by one, so the result is bitwise the same as adding the blocks one
// after another.
__global__ void __launch_bounds__(64) block_add_kernel(const double2 *__restrict__ bsum, int64_t n_blocks, uint64_t sc,
                                                       uint64_t lo, uint64_t hi, double *__restrict__ out) {
    const int bs = blockIdx.x, lane = threadIdx.x;
    double acc_re = out[2 * bs], acc_im = out[2 * bs + 1];
    const int64_t j0 = int64_t(lo - sc) / 64, j1 = (int64_t(hi - sc) + 63) / 64;
    for (int64_t c = j0; c < j1; c += 64) {
        const double2 v = c + lane < j1 ? bsum[int64_t(bs) * n_blocks + c + lane] : make_double2(0.0, 0.0);
        const int cnt = int(j1 - c < 64 ? j1 - c : 64);
        for (int l = 0; l < cnt; ++l) {
            acc_re += readlane_f64(v.x, l);
            acc_im += readlane_f64(v.y, l);
        }
    }
    if (lane == 0) {
        out[2 * bs] = acc_re;
        out[2 * bs + 1] = acc_im;
    }
}

// One workgroup per bitstring.  Its waves (one, four or sixteen, by the number
// of blocks) form the 64-slice block sums (fixed butterfly) of up to 256 blocks
// at a time into LDS; then one thread adds them to the running total in
// increasing block order, so the result is bitwise the same as adding the
// blocks one after another.
constexpr int kReduceBatch = 1024;

__global__ void __launch_bounds__(1024) reduce64_kernel(const float2 *__restrict__ partial, int m, int n_bs,
                                                       uint64_t sc, int64_t n_blocks, uint64_t lo, uint64_t hi,
                                                       uint64_t s_begin, double *__restrict__ out,
                                                       double *__restrict__ per_slice) {
    __shared__ double2 bsum[kReduceBatch];
    __shared__ int valid[kReduceBatch];
    const int bs = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double acc_re = 0.0, acc_im = 0.0;
    if (threadIdx.x == 0) { acc_re = out[2 * bs]; acc_im = out[2 * bs + 1]; }
    for (int64_t first = 0; first < n_blocks; first += kReduceBatch) {
        const int nb = int(n_blocks - first < kReduceBatch ? n_blocks - first : kReduceBatch);
        for (int j = wave; j < nb; j += int(blockDim.x) / 64) {
            const uint64_t b0 = sc + uint64_t(first + j) * 64;
            const bool in = !(b0 + 64 <= lo || b0 >= hi);
            double re = 0.0, im = 0.0;
            const uint64_t s = b0 + lane;
            if (in && s >= lo && s < hi) {
                const float2 v = partial[(int64_t(s - sc) << m) + bs];
                re = double(v.x);
                im = double(v.y);
                if (per_slice) {
                    double *p = per_slice + 2 * (int64_t(s - s_begin) * n_bs + bs);
                    p[0] = re;
                    p[1] = im;
                }
            }
            re = wave_sum(re);
            im = wave_sum(im);
            if (lane == 0) {
                bsum[j] = make_double2(re, im);
                valid[j] = in;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0)
            for (int j = 0; j < nb; ++j)
                if (valid[j]) { acc_re += bsum[j].x; acc_im += bsum[j].y; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * bs] = acc_re;
        out[2 * bs + 1] = acc_im;
    }
}

// A few blocks per bitstring (up to 64): one launch, one workgroup per
// bitstring forming the block sums and adding them.  More blocks: the two
// launches above.  Both give the same bits.
void launch_reduce64(const float2 *partial, int m, int n_bs, uint64_t sc, int64_t n_blocks, uint64_t lo, uint64_t hi,
                     uint64_t s_begin, double *out, double *per_slice, double2 *bsum, hipStream_t st) {
    if (n_blocks <= 64) {
        const int threads = n_blocks >= 16 ? 1024 : (n_blocks >= 4 ? 256 : 64);
        hipLaunchKernelGGL(reduce64_kernel, dim3(n_bs), dim3(threads), 0, st, partial, m, n_bs, sc, n_blocks, lo, hi,
                           s_begin, out, per_slice);
        return;
    }
    const int waves = n_blocks >= 16 ? 16 : int(n_blocks);
    const int64_t groups = (n_blocks + waves - 1) / waves;
    hipLaunchKernelGGL(block_sum_kernel, dim3((unsigned)(groups * n_bs)), dim3(64 * waves), 0, st, partial, m, n_bs, sc,
                       n_blocks, groups, lo, hi, s_begin, bsum, per_slice);
    hipLaunchKernelGGL(block_add_kernel, dim3(n_bs), dim3(64), 0, st, bsum, n_blocks, sc, lo, hi, out);
}

}  // namespace qc
