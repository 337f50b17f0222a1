// Step kernels for gfx950: leaf instantiation, LDS-staged bit-permuting
// transpose, complex batched GEMM (FP32 MFMA and a VALU form for shapes below
// the MFMA tile), and the FP64 cross-slice reduction.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace qc {

// ------------------------------------------------------------------ leaves
// Each leaf is a base tensor (<= 8 binary indices, complex double) whose bits
// are either kept (summed indices, possibly in-flight slice bits), fixed by
// the chunk's slice id (sliced segments not in flight), or fixed by the
// bitstring (output segments); the bitstring bits of the batch become extra
// output bits.  One thread per output element.
__global__ void __launch_bounds__(256) leaf_kernel(const LeafDesc *__restrict__ descs,
                                                   const int32_t *__restrict__ block_leaf,
                                                   const double2 *__restrict__ base, float2 *__restrict__ tensors,
                                                   const uint8_t *__restrict__ bits, int n_qubits,
                                                   uint64_t chunk_base) {
    const int leaf = block_leaf[blockIdx.x];
    const LeafDesc &d = descs[leaf];
    const int64_t e = int64_t(blockIdx.x - d.pad0) * blockDim.x + threadIdx.x;
    if (e >= (int64_t(1) << d.r_out)) return;
    int bs = 0, bidx = 0;
    for (int p = 0; p < d.r_out; ++p) {
        const int bit = int((e >> p) & 1);
        const int s = d.src[p];
        if (s >= 64) bs |= bit << (s - 64);
        else bidx |= bit << s;
    }
    for (int i = 0; i < d.n_fix; ++i) bidx |= int((chunk_base >> d.fix_j[i]) & 1) << d.fix_pos[i];
    for (int i = 0; i < d.n_oq; ++i) bidx |= int(bits[int64_t(bs) * n_qubits + d.oq_q[i]] & 1) << d.oq_pos[i];
    const double2 v = base[d.base_off + bidx];
    tensors[d.out_off + e] = make_float2(float(v.x), float(v.y));
}

void launch_leaves(const LeafDesc *descs, const int32_t *block_leaf, int n_blocks, const double2 *base,
                   float2 *tensors, const uint8_t *bits, int n_qubits, uint64_t chunk_base, hipStream_t st) {
    if (n_blocks <= 0) return;
    hipLaunchKernelGGL(leaf_kernel, dim3(n_blocks), dim3(256), 0, st, descs, block_leaf, base, tensors, bits,
                       n_qubits, chunk_base);
}

// --------------------------------------------------------------- transpose
// A tile of 2^n_tile elements is read in input order (coalesced along the
// input's fastest bits), stored in LDS, then written in output order
// (coalesced along the output's fastest bits).  LDS rows of 32 complex values
// are padded by one entry to spread the strided phase-2 reads over banks.
__device__ __forceinline__ int lds_pad(int t) { return t + (t >> 5); }

__global__ void __launch_bounds__(256) transpose_kernel(TransposeDesc d) {
    __shared__ float2 tile[(1 << kTransMaxTile) + (1 << kTransMaxTile) / 32];
    const int tsize = 1 << d.n_tile;
    for (int64_t t_id = blockIdx.x; t_id < d.n_tiles; t_id += gridDim.x) {
        int64_t in_base = 0, out_base = 0;
        for (int j = 0; j < d.n_rest; ++j)
            if ((t_id >> j) & 1) { in_base += d.rest_in[j]; out_base += d.rest_out[j]; }
        for (int t = threadIdx.x; t < tsize; t += blockDim.x) {
            int64_t off = in_base;
            for (int i = 0; i < d.n_tile; ++i)
                if ((t >> i) & 1) off += d.tin_in[i];
            tile[lds_pad(t)] = d.in[off];
        }
        __syncthreads();
        for (int t = threadIdx.x; t < tsize; t += blockDim.x) {
            int64_t off = out_base;
            int l = 0;
            for (int i = 0; i < d.n_tile; ++i)
                if ((t >> i) & 1) { off += d.tout_out[i]; l += d.tout_lds[i]; }
            d.out[off] = tile[lds_pad(l)];
        }
        __syncthreads();
    }
}

void launch_transpose(const TransposeDesc &d, hipStream_t st) {
    const int64_t grid = d.n_tiles < 65536 ? d.n_tiles : 65536;
    const int threads = d.n_tile >= 8 ? 256 : (d.n_tile >= 6 ? 64 : 64);
    hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)grid), dim3(threads), 0, st, d);
}

// -------------------------------------------------------------- VALU GEMM
// One thread per output element; used when m or n is below the MFMA tile or
// k is 1.  FP32 complex accumulation in k order.
__global__ void __launch_bounds__(256) gemm_valu_kernel(GemmDesc d) {
    const int64_t total = d.nb * d.m * d.n;
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
        d.C[bi * d.sCb + mi * d.sCm + ni * d.sCn] = make_float2(re, im);
    }
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
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t tn = tile % tiles_n;
        const int64_t tm = (tile / tiles_n) % tiles_m;
        const int64_t bi = tile / (tiles_n * tiles_m);
        const float2 *Ab = d.A + bi * d.sAb + tm * TM * d.sAm;
        const float2 *Bb = d.B + bi * d.sBb + tn * TN * d.sBn;
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
        float2 *Cb = d.C + bi * d.sCb + (tm * TM + wm * 32) * d.sCm + (tn * TN + wn * 32) * d.sCn;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int row = (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
            const int col = lane & 31;
            Cb[row * d.sCm + col * d.sCn] = make_float2(acc_re[v], acc_im[v]);
        }
    }
}

const char *launch_gemm(const GemmDesc &d, hipStream_t st) {
    // The MFMA form needs whole 32x32 tiles and a K that the LDS slab divides.
    const int64_t kt_try = d.k >= 16 ? 16 : d.k;
    const bool k_ok = (kt_try == 2 || kt_try == 4 || kt_try == 8 || kt_try == 16) && d.k % kt_try == 0;
    const bool mfma = k_ok && d.m % 32 == 0 && d.n % 32 == 0;
    if (!mfma) {
        const int64_t total = d.nb * d.m * d.n;
        int64_t grid = (total + 255) / 256;
        if (grid > 262144) grid = 262144;
        hipLaunchKernelGGL(gemm_valu_kernel, dim3((unsigned)grid), dim3(256), 0, st, d);
        return "gemm_valu";
    }
    const int wm = d.m % 64 == 0 ? 2 : 1, wn = d.n % 64 == 0 ? 2 : 1;
    const int64_t tiles = d.nb * (d.m / (32 * wm)) * (d.n / (32 * wn));
    const unsigned grid = (unsigned)(tiles < 1048576 ? tiles : 1048576);
    const int kt = d.k >= 16 ? 16 : (int)d.k;
#define QC_GEMM_CASE(WM, WN, KT)                                                                        \
    if (wm == WM && wn == WN && kt == KT) {                                                               \
        hipLaunchKernelGGL((gemm_mfma_kernel<WM, WN, KT>), dim3(grid), dim3(64 * WM * WN), 0, st, d);     \
        return "gemm_mfma";                                                                              \
    }
#define QC_GEMM_KTS(WM, WN) QC_GEMM_CASE(WM, WN, 2) QC_GEMM_CASE(WM, WN, 4) QC_GEMM_CASE(WM, WN, 8) QC_GEMM_CASE(WM, WN, 16)
    QC_GEMM_KTS(1, 1)
    QC_GEMM_KTS(1, 2)
    QC_GEMM_KTS(2, 1)
    QC_GEMM_KTS(2, 2)
#undef QC_GEMM_KTS
#undef QC_GEMM_CASE
    return "gemm_none";
}

// ------------------------------------------------------------------ fused
__global__ void __launch_bounds__(64) fused_kernel(FusedParams P) {
    extern __shared__ float2 lds[];
    const int lane = threadIdx.x;
    const int64_t n_items = P.n_slice_groups * P.n_bs_groups;
    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int64_t gsl = P.first_group + item / P.n_bs_groups;
        const int gb = int(item % P.n_bs_groups);
        const uint64_t slice0 = P.sc + (uint64_t(gsl) << P.bf);
        const uint8_t *bits = P.bits + (int64_t(gb) << P.mf) * P.n_qubits;
        for (int e = lane; e < P.n_elems; e += 64) {
            const LeafDesc &d = P.leaves[P.elem_leaf[e]];
            const int local = e - d.pad1;
            int bs = 0, bidx = 0;
            for (int p = 0; p < d.r_out; ++p) {
                const int bit = (local >> p) & 1;
                const int s = d.src[p];
                if (s >= 64) bs |= bit << (s - 64);
                else bidx |= bit << s;
            }
            for (int i = 0; i < d.n_fix; ++i) bidx |= int((slice0 >> d.fix_j[i]) & 1) << d.fix_pos[i];
            for (int i = 0; i < d.n_oq; ++i) bidx |= int(bits[bs * P.n_qubits + d.oq_q[i]] & 1) << d.oq_pos[i];
            const double2 v = P.base[d.base_off + bidx];
            lds[d.out_off + local] = make_float2(float(v.x), float(v.y));
        }
        __syncthreads();
        for (int s = 0; s < P.n_steps; ++s) {
            const FusedStep &st = P.steps[s];
            const int nc = 1 << st.rc, nk = 1 << st.rk;
            for (int c = lane; c < nc; c += 64) {
                int a = st.a_off, b = st.b_off;
                for (int p = 0; p < st.rc; ++p)
                    if ((c >> p) & 1) { a += st.sA[p]; b += st.sB[p]; }
                float re = 0.f, im = 0.f;
                for (int kk = 0; kk < nk; ++kk) {
                    int ka = a, kb = b;
                    for (int j = 0; j < st.rk; ++j)
                        if ((kk >> j) & 1) { ka += st.kA[j]; kb += st.kB[j]; }
                    const float2 x = lds[ka], y = lds[kb];
                    re = fmaf(x.x, y.x, re);
                    re = fmaf(-x.y, y.y, re);
                    im = fmaf(x.x, y.y, im);
                    im = fmaf(x.y, y.x, im);
                }
                lds[st.c_off + c] = make_float2(re, im);
            }
            __syncthreads();
        }
        const int nr = 1 << P.root_rank;
        for (int c = lane; c < nr; c += 64) {
            int64_t s_low = 0;
            int bs_low = 0;
            for (int p = 0; p < P.root_rank; ++p) {
                const int bit = (c >> p) & 1;
                const int code = P.root_map[p];
                if (code >= 64) bs_low |= bit << (code - 64);
                else s_low |= int64_t(bit) << code;
            }
            const int64_t s_rel = (gsl << P.bf) + s_low;
            const int64_t bs = (int64_t(gb) << P.mf) + bs_low;
            P.partial[(s_rel << P.m) + bs] = lds[P.root_off + c];
        }
        __syncthreads();
    }
}

void launch_fused(const FusedParams &p, hipStream_t st) {
    const int64_t items = p.n_slice_groups * p.n_bs_groups;
    if (items <= 0) return;
    const unsigned grid = (unsigned)(items < 1048576 ? items : 1048576);
    hipLaunchKernelGGL(fused_kernel, dim3(grid), dim3(64), size_t(p.lds_elems) * sizeof(float2), st, p);
}

// --------------------------------------------------------------- reduce64
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ void __launch_bounds__(64) reduce64_kernel(const float2 *__restrict__ partial, int m, int n_bs,
                                                      uint64_t sc, int64_t n_blocks, uint64_t lo, uint64_t hi,
                                                      uint64_t s_begin, double *__restrict__ out,
                                                      double *__restrict__ per_slice) {
    const int bs = blockIdx.x;
    const int lane = threadIdx.x;
    if (bs >= n_bs) return;
    double acc_re = out[2 * bs], acc_im = out[2 * bs + 1];
    for (int64_t blk = 0; blk < n_blocks; ++blk) {
        const uint64_t b0 = sc + uint64_t(blk) * 64;
        if (b0 + 64 <= lo || b0 >= hi) continue;
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
        acc_re += wave_sum(re);
        acc_im += wave_sum(im);
    }
    if (lane == 0) {
        out[2 * bs] = acc_re;
        out[2 * bs + 1] = acc_im;
    }
}

void launch_reduce64(const float2 *partial, int m, int n_bs, uint64_t sc, int64_t n_blocks, uint64_t lo, uint64_t hi,
                     uint64_t s_begin, double *out, double *per_slice, hipStream_t st) {
    hipLaunchKernelGGL(reduce64_kernel, dim3(n_bs), dim3(64), 0, st, partial, m, n_bs, sc, n_blocks, lo, hi, s_begin,
                       out, per_slice);
}

// ---------------------------------------------------------------- reduce
// out[bs] += sum over in-range slices of root[s_low][bs], in FP64.  One block
// per bitstring; thread t sums s_low = t, t + 256, ... in order, then a fixed
// LDS tree combines the 256 partial sums, so the result does not depend on
// timing.
__global__ void __launch_bounds__(256) reduce_kernel(const float2 *__restrict__ root, int b, int m, int n_bs,
                                                     uint64_t chunk_base, uint64_t s_begin, uint64_t s_end,
                                                     double *__restrict__ out, double *__restrict__ per_slice) {
    __shared__ double sre[256], sim[256];
    const int bs = blockIdx.x;
    if (bs >= n_bs) return;
    double re = 0, im = 0;
    const int64_t ns = int64_t(1) << b;
    for (int64_t sl = threadIdx.x; sl < ns; sl += blockDim.x) {
        const uint64_t s = chunk_base + uint64_t(sl);
        if (s < s_begin || s >= s_end) continue;
        const float2 v = root[(sl << m) + bs];
        re += double(v.x);
        im += double(v.y);
        if (per_slice) {
            double *p = per_slice + 2 * (int64_t(s - s_begin) * n_bs + bs);
            p[0] = double(v.x);
            p[1] = double(v.y);
        }
    }
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sre[threadIdx.x] += sre[threadIdx.x + w];
            sim[threadIdx.x] += sim[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * bs] += sre[0];
        out[2 * bs + 1] += sim[0];
    }
}

void launch_reduce(const float2 *root, int b, int m, int n_bs, uint64_t chunk_base, uint64_t s_begin,
                   uint64_t s_end, double *out, double *per_slice, hipStream_t st) {
    hipLaunchKernelGGL(reduce_kernel, dim3(n_bs), dim3(256), 0, st, root, b, m, n_bs, chunk_base, s_begin, s_end,
                       out, per_slice);
}

}  // namespace qc
