// Device side of the C ABI: program constants, workspace layout and the
// slice loop of qc_contract_slices.
//
// A call covers [s_begin, s_end) in aligned super-chunks of P slices (P a
// power of two >= 64).  Per super-chunk the slice values of every bitstring
// are written to a partial buffer, then added to out_dev in aligned blocks of
// 64 slices (fixed butterfly per block, blocks in increasing order), so any
// split of a range at multiples of 64 gives bitwise the same sums.
//
// Two ways to produce the slice values:
//  * fused: when every tensor of one (slice, bitstring) group fits in LDS, a
//    single launch runs the whole program per wavefront (leaves, all steps,
//    root) -- one launch per super-chunk;
//  * stepwise: leaves, then per step an LDS-staged transpose (if the operand
//    layout needs one) and a batched complex GEMM on MFMA, over 2^b slices
//    and all bitstrings in flight in global memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <mutex>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.h"
#include "plan.h"
#include "qcsim_kernels.h"

using qc::set_error;

namespace qc {

namespace {

int ceil_log2(int64_t v) {
    int r = 0;
    while ((int64_t(1) << r) < v) ++r;
    return r;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

#define QC_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            err = std::string(#call) + ": " + hipGetErrorString(e_);                  \
            return false;                                                             \
        }                                                                             \
    } while (0)

// How one call executes: which program, fused or not, and the super-chunk.
struct Exec {
    Program *prog = nullptr;
    bool fused = false;
    int m = 0;          // log2 bitstrings (padded)
    int mo = 0;         // open output qubits: 2^mo values per (slice, bitstring)
    int lp = 6;         // log2 super-chunk slices
    int prec = kPrecC64;
    const DevConsts *dc = nullptr;  // device constants (nullptr: the program's own)
    int pairs = 0, waves = 0;       // fused work-item shape (0: the plan's, timed on first use)
    void *steps_graph = nullptr;    // hipGraphExec_t of the chunk's step sequence (stepwise form), or null
};

// Workspace: bitstrings (when handed over from the host), the super-chunk's
// slice values and their 64-slice block sums, per-tensor max|x| slots (split
// FP16 scale bookkeeping), the stepwise program's tensor region, and the
// scratch of GEMM steps split over k.
struct WsLayout {
    size_t bits_off, partial_off, bsum_off, amax_off, tensor_off, ksplit_off, total;
};

WsLayout ws_layout(const Exec &x, int n_qubits) {
    WsLayout w;
    w.bits_off = 0;
    w.partial_off = align256(size_t(n_qubits) << x.m);
    w.bsum_off = w.partial_off + align256((size_t(1) << (x.lp + x.m + x.mo)) * sizeof(float2));
    w.amax_off = w.bsum_off + align256((size_t(1) << (x.lp - 6 + x.m + x.mo)) * sizeof(double2));
    w.tensor_off = w.amax_off + (x.fused ? 0 : align256(x.prog->tensors.size() * sizeof(uint32_t)));
    w.ksplit_off = w.tensor_off + (x.fused ? 0 : align256(size_t(x.prog->tensor_elems) * sizeof(float2)));
    w.total = w.ksplit_off + (x.fused ? 0 : align256(size_t(x.prog->ksplit_elems) * sizeof(float2)));
    return w;
}

// The fused form runs a (b slices, 0 bitstring bits) program, b <= 6: every
// tensor of one work item in LDS (offsets then fit in 16 bits) and a root of
// the b in-flight slice bits; each leaf may take at most four bits from the
// chunk's slice id and the bitstring (of at most 256 qubits, held as masks).
// b is chosen by timing per plan.
constexpr int kFusedMaxSliceBits = 6;
// A work item's LDS region: the program's tensors, then one slot holding zero.
int64_t pair_elems64(const Program &prog) { return (prog.lds_elems + 2) & ~int64_t(1); }
int zero_slot_of(const Program &prog) { return int(prog.lds_elems); }
int pair_elems_of(const Program &prog) { return int(pair_elems64(prog)); }  // only once fused_fits holds

bool fused_fits_uncached(const qc_plan *plan, const Program &p) {
    if (p.m != 0 || p.b > kFusedMaxSliceBits || plan->net.n_qubits > 256) return false;
    if (!plan->open_qubits.empty()) return false;  // a work item yields one value per slice
    if (pair_elems64(p) * int64_t(sizeof(float2)) > kFusedLdsBytes) return false;
    if ((int)p.tensors[p.root].layout.size() != p.b) return false;
    std::vector<char> sliced(plan->net.n_index(), 0);  // fixed per work item
    for (size_t j = p.b; j < plan->sliced.size(); ++j) sliced[plan->sliced[j]] = 1;
    for (const LeafOp &lo : p.leaves) {
        int dyn = 0;
        for (int e : plan->net.leaves[lo.leaf].idx) dyn += sliced[e] || plan->net.out_qubit[e] >= 0;
        if (dyn > 4) return false;
    }
    return true;
}

// The answer depends on the lowered program only; it is kept with it.
bool fused_fits(const qc_plan *plan, const Program &p) {
    const int known = p.fused_fit.load(std::memory_order_relaxed);
    if (known >= 0) return known == 1;
    const bool fits = fused_fits_uncached(plan, p);
    p.fused_fit.store(fits ? 1 : 0, std::memory_order_relaxed);
    return fits;
}

// Picks the execution for a range of n_range slices with 2^m bitstrings that
// fits ws_bytes (ws_bytes = 0: no limit, used by the workspace query with the
// caller's chunk size in `want_lp`).
// The split precisions run stepwise: the fused form computes its small dot
// products on the vector ALU in FP32.
bool choose_exec(qc_plan *plan, int m, int want_lp, int prec, size_t ws_bytes, Exec &x, std::string &err) {
    const int k = (int)plan->sliced.size();
    const int nq = plan->net.n_qubits;
    x.m = m;
    x.mo = (int)plan->open_qubits.size();
    x.prec = prec;
    Program *pf = get_program(plan, 0, 0, err);
    if (!pf) return false;
    const bool fits = prec == kPrecC64 && fused_fits(plan, *pf);
    if (plan->exec_mode == QC_EXEC_FUSED && !fits) {
        err = prec == kPrecC64 ? "the fused form does not fit in LDS for this plan"
                               : "the fused form runs complex FP32 only";
        return false;
    }
    if (fits && plan->exec_mode != QC_EXEC_STEPWISE) {
        x.prog = pf;
        x.fused = true;
        for (int lp = std::max(6, want_lp); lp >= 6; --lp) {
            x.lp = lp;
            if (ws_bytes == 0 || ws_layout(x, nq).total <= ws_bytes) return true;
        }
        err = "workspace too small for one block of 64 slices";
        return false;
    }
    x.fused = false;
    for (int b = std::min(k, want_lp); b >= 0; --b) {
        Program *p = get_program(plan, b, m, err);
        if (!p) return false;
        x.prog = p;
        x.lp = std::max(b, 6);
        if (ws_bytes == 0 || ws_layout(x, nq).total <= ws_bytes) return true;
    }
    err = "workspace too small for one slice";
    return false;
}

// Keeps the host image of device constant `id` of a program.
bool stage(Program &prog, int id, const void *src, size_t bytes) {
    prog.const_host[id].assign((const char *)src, (const char *)src + bytes);
    return true;
}

// The constants each form reads.
bool const_needed(const Program &prog, bool fused, int id) {
    if (id == kCBase) return true;
    if (fused) return id >= kCFusedImage;
    if (id == kCMicro || id == kCMicroLevels) return prog.n_micro_levels > 0;
    return id == kCLeafDesc || id == kCLeafBlock;
}

// Leaf table of a program; lds = true gives LDS offsets (fused form).
void leaf_table(const qc_plan *plan, const Program &prog, bool lds, std::vector<LeafDesc> &descs,
                std::vector<int32_t> &block_or_elem, std::vector<double2> &base, std::string &err) {
    const Network &net = plan->net;
    std::vector<char> fixed(net.n_index(), 0);
    std::vector<int> slice_bit(net.n_index(), -1);
    for (size_t j = 0; j < plan->sliced.size(); ++j) {
        slice_bit[plan->sliced[j]] = (int)j;
        if ((int)j >= prog.b) fixed[plan->sliced[j]] = 1;
    }
    for (size_t li = 0; li < prog.leaves.size(); ++li) {
        const Tensor &T = net.leaves[prog.leaves[li].leaf];
        const int tid = prog.leaves[li].tensor;
        const ProgTensor &pt = prog.tensors[tid];
        LeafDesc d;
        std::memset(&d, 0, sizeof(d));
        const int rb = (int)T.idx.size();
        const int ro = (int)pt.layout.size();
        if (rb > kLeafMaxBase || ro > kLeafMaxRank) { err = "leaf too large for the device table"; return; }
        d.out_off = lds ? prog.lds_offset[tid] : pt.offset;
        d.base_off = (int32_t)base.size();
        d.r_out = ro;
        auto base_pos = [&](int e) {
            for (int j = 0; j < rb; ++j)
                if (T.idx[j] == e) return rb - 1 - j;
            return -1;
        };
        for (int p = 0; p < ro; ++p) {
            const int e = pt.layout[ro - 1 - p];
            d.src[p] = (int8_t)(e >= kBsBase ? 64 + (e - kBsBase) : base_pos(e));
        }
        for (int j = 0; j < rb; ++j) {
            const int e = T.idx[j];
            if (net.fixed_out(e)) {
                d.oq_pos[d.n_oq] = (int8_t)(rb - 1 - j);
                d.oq_q[d.n_oq] = (int16_t)net.out_qubit[e];
                ++d.n_oq;
            } else if (fixed[e]) {
                d.fix_pos[d.n_fix] = (int8_t)(rb - 1 - j);
                d.fix_j[d.n_fix] = (int8_t)slice_bit[e];
                ++d.n_fix;
            }
        }
        for (const cplx &v : T.data) base.push_back(make_double2(v.real(), v.imag()));
        if (lds) {
            for (int64_t e = 0; e < (int64_t(1) << ro); ++e) block_or_elem.push_back((int32_t)li);
        } else {
            d.first_block = (int32_t)block_or_elem.size();
            d.amax_slot = tid;
            const int64_t nblk = ((int64_t(1) << ro) + 255) / 256;
            for (int64_t b = 0; b < nblk; ++b) block_or_elem.push_back((int32_t)li);
        }
        descs.push_back(d);
    }
}

// Strides of index e in a layout (0 if absent).
int32_t stride_in(const std::vector<int> &layout, int e) {
    const int r = (int)layout.size();
    for (int i = 0; i < r; ++i)
        if (layout[i] == e) return int32_t(1) << (r - 1 - i);
    return 0;
}

// Uploads the program's constants to the current device (once).
// Host images of the device constants of one form (built once; host work only).
bool build_consts(const qc_plan *plan, Program &prog, bool fused, std::string &err) {
    if (!fused && !prog.built_stepwise) {
        std::vector<LeafDesc> descs;
        std::vector<int32_t> blocks;
        std::vector<double2> base;
        leaf_table(plan, prog, false, descs, blocks, base, err);
        if (!err.empty()) return false;
        stage(prog, kCLeafBlock, blocks.data(), blocks.size() * 4);
        stage(prog, kCBase, base.data(), base.size() * sizeof(double2));
        stage(prog, kCLeafDesc, descs.data(), descs.size() * sizeof(LeafDesc));
        prog.n_leaf_blocks = (int)blocks.size();
        // Micro steps.  They form independent subtrees (a micro step reads
        // leaves and outputs of micro steps only); each subtree runs in a
        // workgroup of its own, level by level (leaves are level 0).  With
        // more subtrees than kMicroGroups, subtrees are dealt to groups by
        // decreasing work, each to the least loaded group.
        std::vector<int> lvl(prog.tensors.size(), 0), comp_of(prog.tensors.size(), -1);
        std::vector<int> parent;  // union-find over subtrees
        auto find = [&](int x) {
            while (parent[x] != x) x = parent[x] = parent[parent[x]];
            return x;
        };
        std::vector<MicroStep> all;
        std::vector<int> all_lv, all_comp;
        std::vector<double> all_work;
        for (size_t i = 0; i < prog.ops.size(); ++i) {
            if (prog.op_micro.empty() || !prog.op_micro[i] || prog.ops[i].kind != Op::GEMM) continue;
            const GemmOp &g = prog.gemms[prog.ops[i].index];
            const auto &LA = prog.tensors[g.a_src].layout, &LB = prog.tensors[g.b_src].layout;
            const auto &LC = prog.tensors[g.c].layout;
            const int lv = 1 + std::max(lvl[g.a_src], lvl[g.b_src]);
            lvl[g.c] = lv;
            int c = -1;
            for (int src : {g.a_src, g.b_src}) {
                if (comp_of[src] < 0) continue;
                const int r = find(comp_of[src]);
                if (c < 0) c = r;
                else if (r != c) parent[r] = c;
            }
            if (c < 0) {
                c = (int)parent.size();
                parent.push_back(c);
            }
            comp_of[g.c] = c;
            MicroStep M;
            std::memset(&M, 0, sizeof(M));
            M.a = prog.tensors[g.a_src].offset;
            M.b = prog.tensors[g.b_src].offset;
            M.c = prog.tensors[g.c].offset;
            M.rc = (int)LC.size();
            M.amax_slot = g.c;
            if (M.rc > kMicroRank) { err = "micro step rank too large"; return false; }
            for (int p = 0; p < M.rc; ++p) {
                const int e = LC[M.rc - 1 - p];
                M.sa[p] = stride_in(LA, e);
                M.sb[p] = stride_in(LB, e);
            }
            std::vector<int> ks;  // summed indices: in A or B, not in C
            for (const auto *Lx : {&LA, &LB})
                for (int e : *Lx)
                    if (std::find(LC.begin(), LC.end(), e) == LC.end() && std::find(ks.begin(), ks.end(), e) == ks.end())
                        ks.push_back(e);
            if ((int)ks.size() > kMicroRank) { err = "micro step contraction too large"; return false; }
            M.rk = (int)ks.size();
            for (int q = 0; q < M.rk; ++q) {
                M.ka[q] = stride_in(LA, ks[q]);
                M.kb[q] = stride_in(LB, ks[q]);
            }
            all.push_back(M);
            all_lv.push_back(lv);
            all_comp.push_back(c);
            all_work.push_back(std::ldexp(1.0, M.rc + M.rk));
        }
        // Subtree -> group.
        std::vector<int> root_id(parent.size(), -1);
        std::vector<double> comp_work;
        for (size_t i = 0; i < all.size(); ++i) {
            int &r = root_id[find(all_comp[i])];
            if (r < 0) { r = (int)comp_work.size(); comp_work.push_back(0.0); }
            comp_work[r] += all_work[i];
        }
        const int n_comp = (int)comp_work.size();
        const int n_groups = std::min(n_comp, kMicroGroups);
        std::vector<int> group_of_comp(n_comp);
        {
            std::vector<int> order(n_comp);
            for (int i = 0; i < n_comp; ++i) order[i] = i;
            std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return comp_work[x] > comp_work[y]; });
            std::vector<double> load(n_groups, 0.0);
            for (int c : order) {
                const int gi = int(std::min_element(load.begin(), load.end()) - load.begin());
                group_of_comp[c] = gi;
                load[gi] += comp_work[c];
            }
        }
        // Steps ordered by (group, level, program order); one level entry per
        // (group, level) pair.
        std::vector<int> idx(all.size());
        for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
        auto grp = [&](int i) { return group_of_comp[root_id[find(all_comp[i])]]; };
        std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
            return grp(x) != grp(y) ? grp(x) < grp(y) : all_lv[x] < all_lv[y];
        });
        std::vector<MicroStep> steps;
        std::vector<int32_t> group_start(1, 0), starts(1, 0), outs;
        for (size_t j = 0; j < idx.size(); ++j) {
            const int i = idx[j];
            const bool new_group = j == 0 || grp(i) != grp(idx[j - 1]);
            const bool new_level = new_group || all_lv[i] != all_lv[idx[j - 1]];
            if (j > 0 && new_level) {
                starts.push_back((int32_t)steps.size());
                if (new_group) group_start.push_back((int32_t)outs.size());
            }
            if (new_level) outs.push_back(0);
            MicroStep M = all[i];
            M.out0 = outs.back();
            outs.back() += 1 << M.rc;
            steps.push_back(M);
        }
        if (!steps.empty()) {
            starts.push_back((int32_t)steps.size());
            group_start.push_back((int32_t)outs.size());
        }
        prog.n_micro_levels = (int)outs.size();
        prog.n_micro_groups = (int)group_start.size() - 1;
        if (prog.n_micro_levels > 0) {
            // Table: group starts (G + 1 level entries), level starts (L + 1
            // steps), outputs per level (L).
            std::vector<int32_t> lv_tab(group_start);
            lv_tab.insert(lv_tab.end(), starts.begin(), starts.end());
            lv_tab.insert(lv_tab.end(), outs.begin(), outs.end());
            stage(prog, kCMicro, steps.data(), steps.size() * sizeof(MicroStep));
            stage(prog, kCMicroLevels, lv_tab.data(), lv_tab.size() * 4);
        }
        prog.built_stepwise = true;
    }
    if (fused && !prog.built_fused) {
        std::vector<LeafDesc> descs;
        std::vector<int32_t> unused;
        std::vector<double2> base;
        leaf_table(plan, prog, true, descs, unused, base, err);
        if (!err.empty()) return false;
        // Leaf elements: LDS slot, base index from the element's own bits,
        // and up to four bits taken at run time from the slice id (16-bit
        // code pos | j << 3) or the bitstring (pos | (64 + q) << 3).
        // Elements without run-time bits go into the LDS image instead.
        std::vector<int4> elems;
        std::vector<float2> image;
        for (const LeafDesc &d : descs) {
            std::vector<uint32_t> dyn;
            for (int i = 0; i < d.n_fix; ++i) dyn.push_back(uint32_t(d.fix_pos[i]) | (uint32_t(d.fix_j[i]) << 3));
            for (int i = 0; i < d.n_oq; ++i) dyn.push_back(uint32_t(d.oq_pos[i]) | (uint32_t(64 + d.oq_q[i]) << 3));
            if (dyn.size() > 4) { err = "a leaf has more than four run-time bits"; return false; }
            while (dyn.size() < 4) dyn.push_back(0xffffu);
            const bool is_dyn = dyn[0] != 0xffffu;
            const int z = int(dyn[0] | (dyn[1] << 16)), w = int(dyn[2] | (dyn[3] << 16));
            for (int64_t e = 0; e < (int64_t(1) << d.r_out); ++e) {
                int idx = d.base_off;
                for (int p = 0; p < d.r_out; ++p)
                    if ((e >> p) & 1) idx += 1 << d.src[p];
                const int64_t slot = d.out_off + e;
                if ((int64_t)image.size() <= slot) image.resize(slot + 1, make_float2(0.f, 0.f));
                if (!is_dyn) image[slot] = make_float2(float(base[idx].x), float(base[idx].y));
                else elems.push_back(make_int4(int(slot), idx, z, w));
            }
        }
        // Items: one per output of every step, grouped by tree level (a
        // step's level is one more than its operands'; leaves are level 0).
        const int zero = zero_slot_of(prog);
        std::vector<int> level(prog.tensors.size(), 0);
        int n_levels = 0;
        for (const GemmOp &g : prog.gemms) {
            level[g.c] = 1 + std::max(level[g.a_src], level[g.b_src]);
            n_levels = std::max(n_levels, level[g.c]);
        }
        std::vector<std::vector<int4>> by_level(n_levels);
        std::vector<std::vector<int2>> by_level2(n_levels);
        std::vector<int32_t> pool;
        // Operand and output slots are stored as LDS byte offsets inside a
        // pair's region (below 2^16, the region being at most 64 KiB).
        auto pack = [](int64_t a, int64_t b) {
            return int32_t(uint32_t(a * int64_t(sizeof(float2))) | (uint32_t(b * int64_t(sizeof(float2))) << 16));
        };
        for (const GemmOp &g : prog.gemms) {
            const auto &LA = prog.tensors[g.a_src].layout, &LB = prog.tensors[g.b_src].layout;
            const auto &LC = prog.tensors[g.c].layout;
            const int rc = (int)LC.size();
            std::vector<int32_t> sA, sB, kA, kB;
            for (int p = 0; p < rc; ++p) {
                const int e = LC[rc - 1 - p];
                sA.push_back(stride_in(LA, e));
                sB.push_back(stride_in(LB, e));
            }
            for (int e : LA)
                if (std::find(LC.begin(), LC.end(), e) == LC.end()) {
                    kA.push_back(stride_in(LA, e));
                    kB.push_back(stride_in(LB, e));
                }
            const int rk = (int)kA.size();
            const int64_t nk = int64_t(1) << rk;
            std::vector<int64_t> ka(nk, 0), kb(nk, 0);
            for (int64_t kk = 0; kk < nk; ++kk)
                for (int j = 0; j < rk; ++j)
                    if ((kk >> j) & 1) { ka[kk] += kA[j]; kb[kk] += kB[j]; }
            const int64_t a0 = prog.lds_offset[g.a_src], b0 = prog.lds_offset[g.b_src];
            for (int64_t c = 0; c < (int64_t(1) << rc); ++c) {
                int64_t a = a0, b = b0;
                for (int p = 0; p < rc; ++p)
                    if ((c >> p) & 1) { a += sA[p]; b += sB[p]; }
                int4 it;
                it.x = int(uint32_t((prog.lds_offset[g.c] + c) * int64_t(sizeof(float2))) | (uint32_t(nk) << 16));
                it.y = pack(a, b);
                it.z = nk > 1 ? pack(a + ka[1], b + kb[1]) : pack(zero, zero);
                it.w = -1;
                int2 it2 = make_int2(0, 0);
                if (nk > 2) it2 = make_int2(pack(a + ka[2], b + kb[2]), pack(a + ka[3], b + kb[3]));
                if (nk > 4) {
                    it.w = (int)pool.size();
                    pool.push_back(int32_t(nk - 4));
                    for (int64_t kk = 4; kk < nk; ++kk) pool.push_back(pack(a + ka[kk], b + kb[kk]));
                }
                by_level[level[g.c] - 1].push_back(it);
                by_level2[level[g.c] - 1].push_back(it2);
            }
        }
        std::vector<int4> items;
        std::vector<int2> items2;
        std::vector<int32_t> level_start(1, 0);
        for (int l = 0; l < n_levels; ++l) {
            items.insert(items.end(), by_level[l].begin(), by_level[l].end());
            items2.insert(items2.end(), by_level2[l].begin(), by_level2[l].end());
            level_start.push_back((int32_t)items.size());
        }
        stage(prog, kCFusedImage, image.data(), image.size() * sizeof(float2));
        stage(prog, kCFusedElems, elems.data(), elems.size() * sizeof(int4));
        stage(prog, kCFusedPool, pool.data(), pool.size() * 4);
        stage(prog, kCBase, base.data(), base.size() * sizeof(double2));
        stage(prog, kCFusedItems, items.data(), items.size() * sizeof(int4));
        stage(prog, kCFusedItems2, items2.data(), items2.size() * sizeof(int2));
        stage(prog, kCFusedLevels, level_start.data(), level_start.size() * 4);
        prog.n_leaf_elems = (int)elems.size();
        prog.n_image = (int)image.size();
        prog.n_pool = (int)pool.size();
        prog.n_levels = n_levels;
        prog.built_fused = true;
    }
    return true;
}

// Device constants of one form in plan-owned buffers on the current device
// (allocated and copied on first use).
bool ensure_device(const qc_plan *plan, Program &prog, bool fused, std::string &err) {
    int dev = 0;
    QC_HIP(hipGetDevice(&dev));
    if (prog.device >= 0 && prog.device != dev) { err = "plan was first used on another device"; return false; }
    if (!build_consts(plan, prog, fused, err)) return false;
    prog.device = dev;
    for (int id = 0; id < kNumConst; ++id) {
        if (!const_needed(prog, fused, id) || prog.dc.p[id]) continue;
        const std::vector<char> &h = prog.const_host[id];
        QC_HIP(hipMalloc(&prog.dc.p[id], std::max<size_t>(h.size(), 16)));
        if (!h.empty()) QC_HIP(hipMemcpy(prog.dc.p[id], h.data(), h.size(), hipMemcpyHostToDevice));
    }
    return true;
}

// Bytes the constants of one form take when packed at 256-byte boundaries.
size_t packed_const_bytes(const Program &prog, bool fused) {
    size_t total = 0;
    for (int id = 0; id < kNumConst; ++id)
        if (const_needed(prog, fused, id)) total += (std::max<size_t>(prog.const_host[id].size(), 16) + 255) & ~size_t(255);
    return total;
}

// Copies the constants of one form into dst (device memory of at least
// packed_const_bytes) on stream st, and points dc at the copies.
bool place_consts(const Program &prog, bool fused, char *dst, hipStream_t st, DevConsts &dc, std::string &err) {
    size_t off = 0;
    for (int id = 0; id < kNumConst; ++id) {
        if (!const_needed(prog, fused, id)) continue;
        const std::vector<char> &h = prog.const_host[id];
        dc.p[id] = dst + off;
        if (!h.empty()) QC_HIP(hipMemcpyAsync(dst + off, h.data(), h.size(), hipMemcpyHostToDevice, st));
        off += (std::max<size_t>(h.size(), 16) + 255) & ~size_t(255);
    }
    return true;
}

// Times each pairs-per-wavefront option once on the caller's stream (the
// launches write the same partial values the real launch then overwrites)
// and keeps the fastest.  Runs once per program.
constexpr int kFusedTuneReps = 10;   // timed launches per work-item shape and round
constexpr int kFusedTuneRounds = 3;  // interleaved timing rounds over the shapes

bool tune_fused(Program &prog, const FusedParams &fp, hipStream_t st, std::string &err) {
    const int pe = pair_elems_of(prog), zero = zero_slot_of(prog);
    hipEvent_t e0, e1;
    QC_HIP(hipEventCreate(&e0));
    QC_HIP(hipEventCreate(&e1));
    // Every shape that fits is timed in kFusedTuneRounds interleaved rounds
    // (so that a shape timed while the clocks change is timed again at
    // another moment) and keeps its best round.
    std::vector<std::array<float, 3>> tuned;
    for (const auto &shape : kFusedShapes)
        if (fused_lds_bytes(shape[0], pe) <= size_t(kFusedLdsBytes))
            tuned.push_back({float(shape[0]), float(shape[1]), -1.f});
    for (int round = 0; round < kFusedTuneRounds; ++round)
        for (auto &t : tuned) {
            const int pairs = int(t[0]), waves = int(t[1]);
            launch_fused_pairs(fp, pairs, waves, pe, zero, st);  // warm-up
            QC_HIP(hipEventRecord(e0, st));
            for (int r = 0; r < kFusedTuneReps; ++r) launch_fused_pairs(fp, pairs, waves, pe, zero, st);
            QC_HIP(hipEventRecord(e1, st));
            QC_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            QC_HIP(hipEventElapsedTime(&ms, e0, e1));
            ms /= kFusedTuneReps;
            if (t[2] < 0.f || ms < t[2]) t[2] = ms;
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    QC_HIP(hipGetLastError());
    for (const auto &t : tuned) {
        prog.fused_tuning.push_back(t);
        if (prog.fused_pairs == 0 || t[2] < prog.fused_tuning[prog.fused_best][2]) {
            prog.fused_best = (int)prog.fused_tuning.size() - 1;
            prog.fused_pairs = int(t[0]);
            prog.fused_waves = int(t[1]);
        }
    }
    if (prog.fused_pairs == 0) { err = "no fused form fits in LDS"; return false; }
    return true;
}

// perm[p] = output bit position of input bit p.
TransposeDesc make_transpose_desc(const float2 *in, float2 *out, int r, const std::vector<int> &perm) {
    TransposeDesc d;
    std::memset(&d, 0, sizeof(d));
    d.in = in;
    d.out = out;
    // Tile bits: the input's lowest bits and the output's lowest bits, taken
    // alternately until the tile has kTransMaxTile bits (rank >= 12: the
    // 16-byte form, whose pairs need input bit 0 and the input bit of output
    // bit 0, the first two taken) or kTransSmallTile bits (all bits of a
    // tensor of rank <= 10), so reads and writes both run along contiguous
    // stretches.
    const int nt = r >= kTransMaxTile ? kTransMaxTile : kTransSmallTile;
    std::vector<char> in_tile(r, r <= nt ? 1 : 0);
    if (r > nt) {
        std::vector<int> inv(r);
        for (int p = 0; p < r; ++p) inv[perm[p]] = p;
        int a = 0, c = 0, n = 0;
        while (n < nt) {
            const int p = a <= c ? a++ : inv[c++];
            if (!in_tile[p]) { in_tile[p] = 1; ++n; }
        }
    }
    std::vector<int> tile, rest;  // input bit positions
    for (int p = 0; p < r; ++p) (in_tile[p] ? tile : rest).push_back(p);
    std::vector<int> tin = tile, tout = tile;
    std::sort(tin.begin(), tin.end());
    std::sort(tout.begin(), tout.end(), [&](int x, int y) { return perm[x] < perm[y]; });
    d.n_tile = (int)tile.size();
    d.n_rest = (int)rest.size();
    d.n_tiles = int64_t(1) << d.n_rest;
    for (size_t i = 0; i < tin.size(); ++i) d.tin_in[i] = int64_t(1) << tin[i];
    for (size_t i = 0; i < tout.size(); ++i) {
        d.tout_out[i] = int64_t(1) << perm[tout[i]];
        const int rank_in = (int)(std::find(tin.begin(), tin.end(), tout[i]) - tin.begin());
        d.tout_lds[i] = 1 << rank_in;
    }
    for (size_t j = 0; j < rest.size(); ++j) {
        d.rest_in[j] = int64_t(1) << rest[j];
        d.rest_out[j] = int64_t(1) << perm[rest[j]];
    }
    return d;
}

TransposeDesc make_transpose(const Program &prog, const TransposeOp &t, float2 *tensors) {
    const auto &src = prog.tensors[t.src].layout;
    const auto &dst = prog.tensors[t.dst].layout;
    const int r = (int)src.size();
    std::vector<int> perm(r);
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < r; ++j)
            if (dst[j] == src[i]) perm[r - 1 - i] = r - 1 - j;
    return make_transpose_desc(tensors + prog.tensors[t.src].offset, tensors + prog.tensors[t.dst].offset, r, perm);
}

// amax: per-tensor max|x| slots (split FP16) or null; slot[t] maps a
// transposed tensor to the slot of the tensor it was copied from; need_c, if
// given, says which slots a later step reads (the output maximum is recorded
// only for those).
GemmDesc make_gemm(const Program &prog, const GemmOp &g, float2 *tensors, int prec, uint32_t *amax,
                   const std::vector<int> &slot, float2 *kscratch, const std::vector<char> *need_c = nullptr) {
    GemmDesc d;
    d.kparts = kscratch ? gemm_kparts(g.nb, g.m, g.n, g.k) : 1;
    if (d.kparts > 1) d.kscratch = kscratch;
    d.prec = prec;
    d.amax_a = amax ? amax + slot[g.a] : nullptr;
    d.amax_b = amax ? amax + slot[g.b] : nullptr;
    d.amax_c = amax && (!need_c || (*need_c)[slot[g.c]]) ? amax + slot[g.c] : nullptr;
    d.A = tensors + prog.tensors[g.a].offset;
    d.B = tensors + prog.tensors[g.b].offset;
    d.C = tensors + prog.tensors[g.c].offset;
    d.nb = g.nb; d.m = g.m; d.n = g.n; d.k = g.k;
    d.sAb = g.m * g.k;
    if (g.a_km) { d.sAk = g.m; d.sAm = 1; } else { d.sAm = g.k; d.sAk = 1; }
    d.sBb = g.k * g.n;
    if (g.b_nk) { d.sBn = g.k; d.sBk = 1; } else { d.sBk = g.n; d.sBn = 1; }
    d.sCb = g.m * g.n; d.sCm = g.n; d.sCn = 1;
    if (g.c_nat >= 0 && g.c_nat != g.c) {
        // C goes straight into its consumer's layout: bit t of the natural
        // flat index (least significant first) is index nat[r - 1 - t].
        const auto &nat = prog.tensors[g.c_nat].layout, &lay = prog.tensors[g.c].layout;
        const int r = (int)nat.size();
        d.cscatter = 1;
        d.cbb = g.cls_b; d.cbm = g.cls_m; d.cbn = g.cls_n;
        for (int t = 0; t < r; ++t) {
            const int e = nat[r - 1 - t];
            const int at = int(std::find(lay.begin(), lay.end(), e) - lay.begin());
            d.cpos[t] = (int8_t)(r - 1 - at);
        }
    }
    return d;
}

// Algorithmic real flops of a GEMM step (8 per complex multiply-add) and its
// algorithmic bytes (complex64 operands read and the result written once).
double gemm_flops(const GemmOp &g) { return 8.0 * double(g.nb) * double(g.m) * double(g.n) * double(g.k); }
double gemm_bytes(const GemmOp &g) {
    return 8.0 * double(g.nb) * (double(g.m) * double(g.k) + double(g.k) * double(g.n) + double(g.m) * double(g.n));
}

// Event pair around each launch while the plan's kernel timing is on.
struct Prof {
    qc_plan *plan;
    hipStream_t st;
    void *e0 = nullptr;
    void *event() {
        if (!plan->prof_pool.empty()) {
            void *e = plan->prof_pool.back();
            plan->prof_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        hipEventCreate(&e);
        return (void *)e;
    }
    void begin() {
        if (!plan->profiling) return;
        e0 = event();
        hipEventRecord((hipEvent_t)e0, st);
    }
    void end(const char *kind, double flops = 0, double bytes = 0) {
        if (!plan->profiling) return;
        void *e1 = event();
        hipEventRecord((hipEvent_t)e1, st);
        plan->prof_pending.push_back({kind, e0, e1, flops, bytes});
    }
};

// The scale slot of each tensor of a stepwise program (a transpose's output
// shares its input's).
std::vector<int> scale_slots(const Program &prog) {
    std::vector<int> slot(prog.tensors.size());
    for (size_t t = 0; t < slot.size(); ++t) slot[t] = (int)t;
    for (const Op &op : prog.ops)
        if (op.kind == Op::TRANSPOSE) slot[prog.transposes[op.index].dst] = slot[prog.transposes[op.index].src];
    return slot;
}

// The launches of one chunk of the stepwise form that do not depend on the
// chunk's position: the micro-step launch, then every GEMM and transpose op on
// the chunk's tensors.  This sequence is what a graph captures.
void launch_steps(qc_plan *plan, const Exec &x, const DevConsts &dc, float2 *tensors, float2 *kscratch,
                  uint32_t *amax, const std::vector<int> &slot, hipStream_t st, Prof &prof) {
    const Program &prog = *x.prog;
    // Split FP16: a GEMM step records its output's maximum only where a step
    // reading that tensor (directly or through a transpose) multiplies on a
    // 16-bit form, which derives its operand scale from it; elsewhere the
    // complex FP32 forms run their instances without the recording epilogue.
    std::vector<char> need;
    if (amax) {
        need.assign(prog.tensors.size(), 0);
        for (size_t gi = 0; gi < prog.gemms.size(); ++gi) {
            if (prog.gemm_micro[gi]) continue;
            const GemmOp &g = prog.gemms[gi];
            const GemmDesc gd = make_gemm(prog, g, tensors, x.prec, amax, slot, kscratch);
            const int v = g.variant[x.prec];
            if (gemm_variant_16bit(v >= 0 && gemm_variant_ok(gd, v) ? v : gemm_default_variant(gd)))
                need[slot[g.a]] = need[slot[g.b]] = 1;
        }
    }
    if (prog.n_micro_levels > 0) {
        const int32_t *lt = (const int32_t *)dc.p[kCMicroLevels];
        prof.begin();
        const int32_t *ls = lt + prog.n_micro_groups + 1;
        launch_micro((const MicroStep *)dc.p[kCMicro], lt, ls, ls + prog.n_micro_levels + 1, prog.n_micro_groups,
                     tensors, amax, st);
        double mf = 0, mb = 0;
        if (plan->profiling)
            for (size_t gi = 0; gi < prog.gemms.size(); ++gi)
                if (prog.gemm_micro[gi]) {
                    mf += gemm_flops(prog.gemms[gi]);
                    mb += gemm_bytes(prog.gemms[gi]);
                }
        prof.end("micro", mf, mb);
    }
    for (size_t oi = 0; oi < prog.ops.size(); ++oi) {
        const Op &op = prog.ops[oi];
        if (prog.op_micro[oi]) continue;
        prof.begin();
        if (op.kind == Op::TRANSPOSE) {
            const TransposeOp &t = prog.transposes[op.index];
            launch_transpose(make_transpose(prog, t, tensors), st);
            // Algorithmic bytes: every element read once and written once.
            prof.end("transpose", 0, 16.0 * double(int64_t(1) << prog.tensors[t.src].layout.size()));
        } else {
            const GemmOp &g = prog.gemms[op.index];
            const GemmDesc gd = make_gemm(prog, g, tensors, x.prec, amax, slot, kscratch, amax ? &need : nullptr);
            const int v = g.variant[x.prec];
            prof.end(v >= 0 && gemm_variant_ok(gd, v) ? launch_gemm_variant(gd, v, st) : launch_gemm(gd, st),
                     gemm_flops(g), gemm_bytes(g));
        }
    }
}

// A fused launch whose work items are exactly 64-slice blocks, one item per
// workgroup, with one block of [lo, hi) per bitstring, adds its block sums to
// the output itself (same butterfly and order as the reduction launch).
bool block_sums_in_fused(const Program &prog, int pairs, uint64_t sc, uint64_t lo, uint64_t hi) {
    return prog.b == 6 && pairs == 1 && ((lo - sc) >> 6) == ((hi - 1 - sc) >> 6);
}

// The work-item shape a fused launch of prog uses: the caller's, if set, else
// the timed one.
int fused_pairs_of(const qc_plan *plan, const Program &prog) {
    return plan->fused_force_pairs > 0 ? plan->fused_force_pairs : prog.fused_pairs;
}
int fused_waves_of(const qc_plan *plan, const Program &prog) {
    return plan->fused_force_pairs > 0 ? plan->fused_force_waves : prog.fused_waves;
}

// Kernel parameters of the fused form for slices [lo, hi) of super-chunk sc.
FusedParams fused_params(const qc_plan *plan, const Program &prog, const Exec &x, uint64_t sc, uint64_t lo,
                         uint64_t hi, const uint8_t *bits, int n_bs, float2 *partial) {
    FusedParams fp;
    std::memset(&fp, 0, sizeof(fp));
    const DevConsts &dc = x.dc ? *x.dc : prog.dc;
    fp.level_start = (const int32_t *)dc.p[kCFusedLevels];
    fp.n_levels = prog.n_levels;
    fp.items = (const int4 *)dc.p[kCFusedItems];
    fp.items2 = (const int2 *)dc.p[kCFusedItems2];
    fp.pool = (const int32_t *)dc.p[kCFusedPool];
    fp.leaf_image = (const float2 *)dc.p[kCFusedImage];
    fp.n_image = prog.n_image;
    fp.elems = (const int4 *)dc.p[kCFusedElems];
    fp.n_elems = prog.n_leaf_elems;
    fp.base = (const double2 *)dc.p[kCBase];
    fp.bits = bits;
    fp.n_qubits = plan->net.n_qubits;
    fp.n_bs = n_bs;
    fp.m = x.m;
    fp.b = prog.b;
    fp.first_slice = int64_t(lo - sc) >> prog.b;
    fp.n_slices = ((int64_t(hi - sc) + (int64_t(1) << prog.b) - 1) >> prog.b) - fp.first_slice;
    fp.sc = sc;
    fp.root_off = (int32_t)prog.lds_offset[prog.root];
    fp.partial = partial;
    fp.lds_elems = (int32_t)prog.lds_elems;
    return fp;
}

// The launches of one call, on stream st, bitstrings already in device
// memory: for each super-chunk either the fused kernel or the stepwise
// sequence (scale-slot reset, leaves, transposes and GEMMs per chunk, root
// copy), then the FP64 reduction.  Only kernel launches (and, with prof,
// event records), so the sequence can be captured as a graph.
bool launch_all(qc_plan *plan, const Exec &x, uint64_t s_begin, uint64_t s_end, const uint8_t *bits, int n_bs,
                void *ws, hipStream_t st, double *out_dev, double *per_slice_dev, bool profile, std::string &err) {
    Program &prog = *x.prog;
    const DevConsts &dc = x.dc ? *x.dc : prog.dc;
    Prof prof{plan, st};
    const bool saved = plan->profiling;
    plan->profiling = profile;
    const int nq = plan->net.n_qubits;
    const WsLayout w = ws_layout(x, nq);
    float2 *partial = (float2 *)((char *)ws + w.partial_off);
    float2 *tensors = (float2 *)((char *)ws + w.tensor_off);
    float2 *kscratch = (float2 *)((char *)ws + w.ksplit_off);
    // Scale bookkeeping only where a scale is derived from it (FP16).
    uint32_t *amax = (!x.fused && x.prec == kPrecFP16) ? (uint32_t *)((char *)ws + w.amax_off) : nullptr;
    const std::vector<int> slot = x.fused ? std::vector<int>() : scale_slots(prog);
    const uint64_t P = uint64_t(1) << x.lp;
    for (uint64_t sc = s_begin & ~(P - 1); sc < s_end; sc += P) {
        const uint64_t lo = std::max(s_begin, sc), hi = std::min(s_end, sc + P);
        bool summed = false;  // block sums already added to out by the fused launch
        if (x.fused) {
            FusedParams fp = fused_params(plan, prog, x, sc, lo, hi, bits, n_bs, partial);
            if (x.pairs == 0 && prog.fused_pairs == 0 && !tune_fused(prog, fp, st, err)) {
                plan->profiling = saved;
                return false;
            }
            const int pairs = x.pairs > 0 ? x.pairs : fused_pairs_of(plan, prog);
            const int waves = x.pairs > 0 ? x.waves : fused_waves_of(plan, prog);
            if (fused_lds_bytes(pairs, pair_elems_of(prog)) > size_t(kFusedLdsBytes)) {
                err = "the fused work-item shape set for this plan does not fit in LDS";
                plan->profiling = saved;
                return false;
            }
            summed = block_sums_in_fused(prog, pairs, sc, lo, hi);
            if (summed) {
                fp.out = out_dev;
                fp.per_slice = per_slice_dev;
                fp.lo = lo;
                fp.hi = hi;
                fp.s_begin = s_begin;
            }
            prof.begin();
            launch_fused_pairs(fp, pairs, waves, pair_elems_of(prog), zero_slot_of(prog), st);
            prof.end("fused");
        } else {
            const uint64_t chunk = uint64_t(1) << prog.b;
            for (uint64_t cb = lo & ~(chunk - 1); cb < hi; cb += chunk) {
                prof.begin();
                if (amax) launch_zero_u32(amax, (int64_t)slot.size(), st);
                launch_leaves((const LeafDesc *)dc.p[kCLeafDesc], (const int32_t *)dc.p[kCLeafBlock],
                              prog.n_leaf_blocks, (const double2 *)dc.p[kCBase], tensors, bits, nq, n_bs, cb, amax,
                              st);
                prof.end("leaves");
                if (!x.steps_graph) {
                    launch_steps(plan, x, dc, tensors, kscratch, amax, slot, st, prof);
                } else if (hipGraphLaunch((hipGraphExec_t)x.steps_graph, st) != hipSuccess) {
                    err = std::string("hipGraphLaunch: ") + hipGetErrorString(hipGetLastError());
                    plan->profiling = saved;
                    return false;
                }
                launch_copy(partial + ((cb - sc) << (x.m + x.mo)), tensors + prog.tensors[prog.root].offset,
                            int64_t(1) << (prog.b + x.m + x.mo), st);
            }
        }
        if (!summed) {
            prof.begin();
            // Open outputs: the root holds [bitstring][open bits], so the sums
            // run over n_bs << mo values per slice in the same layout.
            launch_reduce64(partial, x.m + x.mo, n_bs << x.mo, sc, int64_t(P / 64), lo, hi, s_begin, out_dev,
                            per_slice_dev, (double2 *)((char *)ws + w.bsum_off), st);
            prof.end("reduce64");
        }
    }
    plan->profiling = saved;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) { err = std::string("kernel launch: ") + hipGetErrorString(e); return false; }
    return true;
}

// The graph of a stepwise program's per-chunk step sequence for one
// configuration (precision, slices and bitstrings in flight, workspace):
// captured once on the plan's capture stream and kept (at most 8 per program;
// dropping one waits for the device to drain).  Every chunk of every call with
// that configuration replays it, whatever the slice range, so host memory and
// capture work stay bounded however many chunks a call holds.  Returns null
// with err empty if capture is not possible (the caller then launches
// directly).
void *steps_graph(qc_plan *plan, const Exec &x, void *ws, std::string &err) {
    Program &prog = *x.prog;
    const std::vector<uint64_t> key = {uint64_t(x.prec), uint64_t(x.lp), uint64_t(x.m), uint64_t(prog.b),
                                       uint64_t(uintptr_t(ws))};
    for (auto &g : prog.graphs)
        if (g.first == key) return g.second;
    if (!plan->capture_stream) {
        hipStream_t cs = nullptr;
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
            err = "hipStreamCreateWithFlags failed";
            return nullptr;
        }
        plan->capture_stream = (void *)cs;
    }
    hipStream_t cs = (hipStream_t)plan->capture_stream;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    const WsLayout w = ws_layout(x, plan->net.n_qubits);
    float2 *tensors = (float2 *)((char *)ws + w.tensor_off);
    float2 *kscratch = (float2 *)((char *)ws + w.ksplit_off);
    uint32_t *amax = x.prec == kPrecFP16 ? (uint32_t *)((char *)ws + w.amax_off) : nullptr;
    Prof none{plan, cs};
    const bool saved = plan->profiling;
    plan->profiling = false;
    launch_steps(plan, x, prog.dc, tensors, kscratch, amax, scale_slots(prog), cs, none);
    plan->profiling = saved;
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    hipGraphExec_t exec = nullptr;
    const bool inst = ec == hipSuccess && graph && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
    if (graph) (void)hipGraphDestroy(graph);
    if (!inst) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (prog.graphs.size() >= 8) {
        if (hipDeviceSynchronize() != hipSuccess) {
            err = "hipDeviceSynchronize failed";
            (void)hipGraphExecDestroy(exec);
            return nullptr;
        }
        (void)hipGraphExecDestroy((hipGraphExec_t)prog.graphs.front().second);
        prog.graphs.erase(prog.graphs.begin());
    }
    prog.graphs.push_back({key, (void *)exec});
    return (void *)exec;
}

// Slices in flight per fused work item: a program with b in-flight slice bits
// shares the work that does not depend on them among its 2^b slices, but has
// 2^b times fewer work items.  Each b whose program fits is timed once per
// plan (with its best pairs per wavefront) on a whole super-chunk starting at
// the call's first one, with the call's bitstrings; the fastest is kept.
// Only the super-chunk's slice values in the workspace are written.
bool choose_fused_b(qc_plan *plan, const Exec &x, uint64_t s_begin, const uint8_t *bits, int n_bs, void *ws,
                    hipStream_t st, std::string &err) {
    const int k = (int)plan->sliced.size();
    const uint64_t P = uint64_t(1) << x.lp;
    const uint64_t sc = s_begin & ~(P - 1);
    const uint64_t hi = std::min(sc + P, uint64_t(1) << k);
    float2 *partial = (float2 *)((char *)ws + ws_layout(x, plan->net.n_qubits).partial_off);
    // The separate reduction launch, timed once on the super-chunk's slice
    // values into scratch (the block-sum region), is added to every b whose
    // launch does not sum the blocks itself.
    const WsLayout w = ws_layout(x, plan->net.n_qubits);
    float reduce_ms = 0.f;
    {
        hipEvent_t e0, e1;
        QC_HIP(hipEventCreate(&e0));
        QC_HIP(hipEventCreate(&e1));
        double *scratch = (double *)((char *)ws + w.bsum_off);
        QC_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < 3; ++r)
            launch_reduce64(partial, x.m, n_bs, sc, int64_t(P / 64), sc, hi, sc, scratch, nullptr, (double2 *)scratch, st);
        QC_HIP(hipEventRecord(e1, st));
        QC_HIP(hipEventSynchronize(e1));
        QC_HIP(hipEventElapsedTime(&reduce_ms, e0, e1));
        reduce_ms /= 3;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    int best_b = 0;
    float best_ms = -1.f;
    for (int b = 0; b <= std::min(k, kFusedMaxSliceBits); ++b) {
        Program *p = get_program(plan, b, 0, err);
        if (!p) return false;
        if (!fused_fits(plan, *p) || (uint64_t(1) << b) > P) continue;
        if (!ensure_device(plan, *p, true, err)) return false;
        const FusedParams fp = fused_params(plan, *p, x, sc, sc, hi, bits, n_bs, partial);
        if (p->fused_pairs == 0 && !tune_fused(*p, fp, st, err)) return false;
        float ms = -1.f;
        for (auto &t : p->fused_tuning)
            if (ms < 0 || t[2] < ms) ms = t[2];
        if (!block_sums_in_fused(*p, fused_pairs_of(plan, *p), sc, sc, hi)) ms += reduce_ms;
        if (best_ms < 0 || ms < best_ms) { best_ms = ms; best_b = b; }
    }
    plan->fused_b = best_b;
    return true;
}

// bits_in: host bitstrings (copied into the workspace) or, with bits_on_device,
// the caller's device array (read in place).
bool enqueue(qc_plan *plan, const Exec &x, uint64_t s_begin, uint64_t s_end, const uint8_t *bits_in,
             bool bits_on_device, int n_bs, void *ws, hipStream_t st, double *out_dev, double *per_slice_dev,
             std::string &err) {
    std::lock_guard<std::mutex> lk(plan->dev_mu);
    Exec y = x;
    if (!ensure_device(plan, *y.prog, y.fused, err)) return false;
    const WsLayout w = ws_layout(y, plan->net.n_qubits);
    const uint8_t *bits = bits_in;
    if (!bits_on_device) {
        uint8_t *dst = (uint8_t *)ws + w.bits_off;
        QC_HIP(hipMemcpyAsync(dst, bits_in, size_t(n_bs) * plan->net.n_qubits, hipMemcpyHostToDevice, st));
        bits = dst;
    }
    if (y.fused) {
        if (plan->fused_b < 0 && !choose_fused_b(plan, y, s_begin, bits, n_bs, ws, st, err)) return false;
        if (plan->fused_b > 0) {
            y.prog = get_program(plan, plan->fused_b, 0, err);
            if (!y.prog || !ensure_device(plan, *y.prog, true, err)) return false;
        }
    }
    // Graphs pay off for the stepwise form's long launch sequences; the fused
    // form is two launches per super-chunk, which replay no faster.
    if (plan->use_graphs && !plan->profiling && !y.fused) {
        y.steps_graph = steps_graph(plan, y, ws, err);
        if (!y.steps_graph && !err.empty()) return false;
    }
    return launch_all(plan, y, s_begin, s_end, bits, n_bs, ws, st, out_dev, per_slice_dev, plan->profiling, err);
}

// ------------------------------------------------------------------ tuning
// Process-wide choice of GEMM kernel form per (device architecture,
// precision, shape, operand layouts), filled by qc_tune from timings or a
// cache file of lines "arch prec nb m n k a_km b_nk variant ms".
std::mutex g_tune_mu;
std::map<std::string, std::pair<int, float>> g_tune;

std::string tune_key(const std::string &arch, const GemmDesc &d, bool a_km, bool b_nk) {
    return arch + " " + std::to_string(d.prec) + " " + std::to_string(d.nb) + " " + std::to_string(d.m) + " " +
           std::to_string(d.n) + " " + std::to_string(d.k) + " " + std::to_string(int(a_km)) + " " +
           std::to_string(int(b_nk));
}

void tune_load(const char *path) {
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char arch[64];
    int prec, a_km, b_nk, v;
    long long nb, m, n, k;
    float ms;
    while (std::fscanf(f, "%63s %d %lld %lld %lld %lld %d %d %d %f", arch, &prec, &nb, &m, &n, &k, &a_km, &b_nk, &v,
                       &ms) == 10) {
        if (v < 0 || v >= kVarCount) continue;
        GemmDesc d{};
        d.prec = prec; d.nb = nb; d.m = m; d.n = n; d.k = k;
        g_tune[tune_key(arch, d, a_km, b_nk)] = {v, ms};
    }
    std::fclose(f);
}

bool tune_save(const char *path, std::string &err) {
    if (!path) return true;
    FILE *f = std::fopen(path, "w");
    if (!f) { err = std::string("cannot write ") + path; return false; }
    for (auto &kv : g_tune) std::fprintf(f, "%s %d %.6f\n", kv.first.c_str(), kv.second.first, kv.second.second);
    std::fclose(f);
    return true;
}

}  // namespace

void free_program_device(Program &prog) {
    if (prog.device < 0) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(prog.device);
    for (auto &g : prog.graphs) (void)hipGraphExecDestroy((hipGraphExec_t)g.second);
    prog.graphs.clear();
    for (void *&p : prog.dc.p) {
        if (p) (void)hipFree(p);
        p = nullptr;
    }
    (void)hipSetDevice(cur);
}

}  // namespace qc

static bool check_bitstrings(const qc_plan *plan, const uint8_t *bits, int n_bs) {
    const int nq = plan->net.n_qubits;
    for (int64_t i = 0; i < int64_t(n_bs) * nq; ++i)
        if (bits[i] > 1) return false;
    return true;
}

static bool valid_prec(qc_precision p) { return p == QC_C64 || p == QC_SPLIT_BF16 || p == QC_SPLIT_FP16; }

namespace qc {
int prec_code(qc_precision p) { return p == QC_SPLIT_FP16 ? kPrecFP16 : (p == QC_SPLIT_BF16 ? kPrecBF16 : kPrecC64); }
}  // namespace qc

extern "C" size_t qc_workspace_bytes(qc_plan *plan, int64_t chunk_slices, int32_t n_bs, qc_precision prec) {
    if (!plan || chunk_slices < 1 || n_bs < 1 || n_bs > (1 << qc::kMaxBsBits) || !valid_prec(prec)) {
        set_error("qc_workspace_bytes: invalid argument");
        return 0;
    }
    const int b = qc::ceil_log2(chunk_slices);
    if (b > (int)plan->sliced.size()) { set_error("qc_workspace_bytes: more slices than the plan has"); return 0; }
    std::string err;
    qc::Exec x;
    if (!qc::choose_exec(plan, qc::ceil_log2(n_bs), b, qc::prec_code(prec), 0, x, err)) {
        set_error("qc_workspace_bytes: " + err);
        return 0;
    }
    return qc::ws_layout(x, plan->net.n_qubits).total;
}

static qc_status contract_common(const char *fn, qc_plan *plan, uint64_t s_begin, uint64_t s_end,
                                 const uint8_t *bitstrings, bool bits_on_device, int32_t n_bs, qc_precision prec,
                                 void *ws, size_t ws_bytes, void *stream, double *out_dev, double *per_slice_dev) {
    if (!plan || !bitstrings || !ws || !out_dev) { set_error(std::string(fn) + ": NULL argument"); return QC_ERR_INVALID_ARG; }
    if (!valid_prec(prec)) { set_error(std::string(fn) + ": invalid precision"); return QC_ERR_INVALID_ARG; }
    if (n_bs < 1 || n_bs > (1 << qc::kMaxBsBits) || (int64_t(n_bs) << plan->open_qubits.size()) > (int64_t(1) << 20)) {
        set_error(std::string(fn) + ": n_bs out of range");
        return QC_ERR_RANGE;
    }
    const int k = (int)plan->sliced.size();
    const uint64_t n_slices = k >= 64 ? ~uint64_t(0) : (uint64_t(1) << k);
    if (s_begin > s_end || s_end > n_slices) { set_error(std::string(fn) + ": slice range out of bounds"); return QC_ERR_RANGE; }
    if (!bits_on_device && !check_bitstrings(plan, bitstrings, n_bs)) {
        set_error(std::string(fn) + ": bitstring entries must be 0 or 1");
        return QC_ERR_INVALID_ARG;
    }
    if (s_begin == s_end) return QC_OK;
    std::string err;
    qc::Exec x;
    const int want = std::min(k, qc::ceil_log2((int64_t)(s_end - s_begin)));
    if (!qc::choose_exec(plan, qc::ceil_log2(n_bs), want, qc::prec_code(prec), ws_bytes, x, err)) {
        set_error(std::string(fn) + ": " + err);
        return err.find("workspace") != std::string::npos ? QC_ERR_NOMEM : QC_ERR_UNSUPPORTED;
    }
    if (!qc::enqueue(plan, x, s_begin, s_end, bitstrings, bits_on_device, n_bs, ws, (hipStream_t)stream, out_dev,
                     per_slice_dev, err)) {
        set_error(std::string(fn) + ": " + err);
        return QC_ERR_DEVICE;
    }
    return QC_OK;
}

extern "C" qc_status qc_contract_slices(qc_plan *plan, uint64_t s_begin, uint64_t s_end, const uint8_t *bitstrings,
                                        int32_t n_bs, qc_precision prec, void *ws, size_t ws_bytes, void *stream,
                                        double *out_dev, double *per_slice_dev) {
    return contract_common("qc_contract_slices", plan, s_begin, s_end, bitstrings, false, n_bs, prec, ws, ws_bytes,
                           stream, out_dev, per_slice_dev);
}

extern "C" qc_status qc_contract_slices_dev(qc_plan *plan, uint64_t s_begin, uint64_t s_end,
                                            const uint8_t *bitstrings_dev, int32_t n_bs, qc_precision prec, void *ws,
                                            size_t ws_bytes, void *stream, double *out_dev, double *per_slice_dev) {
    return contract_common("qc_contract_slices_dev", plan, s_begin, s_end, bitstrings_dev, true, n_bs, prec, ws,
                           ws_bytes, stream, out_dev, per_slice_dev);
}

// ------------------------------------------------------------------ no allocation
// Scratch of qc_contract_slices_noalloc: the lowered program's constants
// followed by its workspace.  Each device holds its own copy until the
// process ends; every call on a device shares it.
namespace qc {
constexpr size_t kNoAllocBytes = size_t(64) << 20;
}  // namespace qc

static __device__ __align__(256) unsigned char scratch[qc::kNoAllocBytes];

// Device address of `scratch` on the current device, looked up once per
// device (the array's host-side name is not a device address).
static bool scratch_address(int dev, char **out, std::string &err) {
    static std::mutex mu;
    static std::map<int, char *> addr;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return false;
        }
        it = addr.emplace(dev, (char *)ptr).first;
    }
    *out = it->second;
    return true;
}

extern "C" qc_status qc_contract_slices_noalloc(qc_plan *plan, uint64_t s_begin, uint64_t s_end,
                                                const uint8_t *bitstrings_dev, int32_t n_bs, qc_precision prec,
                                                void *stream, double *out_dev, double *per_slice_dev) {
    const std::string fn = "qc_contract_slices_noalloc";
    if (!plan || !bitstrings_dev || !out_dev) { set_error(fn + ": NULL argument"); return QC_ERR_INVALID_ARG; }
    if (!valid_prec(prec)) { set_error(fn + ": invalid precision"); return QC_ERR_INVALID_ARG; }
    if (n_bs < 1 || n_bs > (1 << qc::kMaxBsBits) || (int64_t(n_bs) << plan->open_qubits.size()) > (int64_t(1) << 20)) {
        set_error(fn + ": n_bs out of range");
        return QC_ERR_RANGE;
    }
    const int k = (int)plan->sliced.size();
    const uint64_t n_slices = k >= 64 ? ~uint64_t(0) : (uint64_t(1) << k);
    if (s_begin > s_end || s_end > n_slices) { set_error(fn + ": slice range out of bounds"); return QC_ERR_RANGE; }
    if (s_begin == s_end) return QC_OK;
    std::string err;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { set_error(fn + ": no current device"); return QC_ERR_DEVICE; }
    char *base = nullptr;
    if (!scratch_address(dev, &base, err)) { set_error(fn + ": " + err); return QC_ERR_DEVICE; }
    std::lock_guard<std::mutex> lk(plan->dev_mu);
    // The form and program qc_contract_slices_dev would choose with a
    // workspace of what the constants leave of the scratch.
    const int want = std::min(k, qc::ceil_log2((int64_t)(s_end - s_begin)));
    const int m = qc::ceil_log2(n_bs);
    const int pc = qc::prec_code(prec);
    qc::Exec x;
    size_t cap = qc::kNoAllocBytes, cbytes = 0;
    bool ok = false;
    for (int iter = 0; iter < 8 && !ok; ++iter) {
        if (!qc::choose_exec(plan, m, want, pc, cap, x, err)) {
            set_error(fn + ": " + err + " (the scratch of this entry point holds " +
                      std::to_string(qc::kNoAllocBytes >> 20) + " MiB)");
            return err.find("workspace") != std::string::npos ? QC_ERR_NOMEM : QC_ERR_UNSUPPORTED;
        }
        if (x.fused) {
            // The plan's slice bits and shape if timed before, else b = 0 and
            // one work item on four wavefronts (nothing is timed here).
            const int fb = plan->fused_b > 0 ? plan->fused_b : 0;
            if (fb > 0 && !(x.prog = qc::get_program(plan, fb, 0, err))) { set_error(fn + ": " + err); return QC_ERR_DEVICE; }
            if (plan->fused_force_pairs > 0) { x.pairs = plan->fused_force_pairs; x.waves = plan->fused_force_waves; }
            else if (x.prog->fused_pairs > 0) { x.pairs = x.prog->fused_pairs; x.waves = x.prog->fused_waves; }
            else { x.pairs = 1; x.waves = 4; }
        }
        if (!qc::build_consts(plan, *x.prog, x.fused, err)) { set_error(fn + ": " + err); return QC_ERR_DEVICE; }
        cbytes = qc::packed_const_bytes(*x.prog, x.fused);
        const size_t need = cbytes + qc::ws_layout(x, plan->net.n_qubits).total;
        if (need <= qc::kNoAllocBytes) { ok = true; break; }
        if (cbytes >= qc::kNoAllocBytes || cap <= qc::kNoAllocBytes - cbytes) break;
        cap = qc::kNoAllocBytes - cbytes;
    }
    if (!ok) {
        set_error(fn + ": the program's constants and workspace need more than the " +
                  std::to_string(qc::kNoAllocBytes >> 20) + " MiB of this entry point's scratch");
        return QC_ERR_NOMEM;
    }
    qc::DevConsts dc;
    hipStream_t st = (hipStream_t)stream;
    if (!qc::place_consts(*x.prog, x.fused, base, st, dc, err)) { set_error(fn + ": " + err); return QC_ERR_DEVICE; }
    x.dc = &dc;
    if (!qc::launch_all(plan, x, s_begin, s_end, bitstrings_dev, n_bs, base + cbytes, st, out_dev, per_slice_dev,
                        false, err)) {
        set_error(fn + ": " + err);
        return QC_ERR_DEVICE;
    }
    return QC_OK;
}

extern "C" qc_status qc_amplitude(qc_plan *plan, const uint8_t *bitstring, qc_precision prec, double out_host[2]) {
    if (!plan || !out_host) { set_error("qc_amplitude: NULL argument"); return QC_ERR_INVALID_ARG; }
    const uint8_t *bits = bitstring ? bitstring : (plan->default_bitstring.empty() ? nullptr : plan->default_bitstring.data());
    if (!bits) { set_error("qc_amplitude: no bitstring given and the plan has none"); return QC_ERR_INVALID_ARG; }
    const int k = (int)plan->sliced.size();
    const size_t cap = size_t(8) << 30;
    int b = std::min(k, 12);
    size_t need = 0;
    for (; b >= 0; --b) {
        need = qc_workspace_bytes(plan, int64_t(1) << b, 1, prec);
        if (need == 0) return QC_ERR_UNSUPPORTED;
        if (need <= cap) break;
    }
    if (b < 0) need = qc_workspace_bytes(plan, 1, 1, prec);
    // 2^n_open amplitudes for a plan with open outputs.
    const size_t n_out = size_t(2) << plan->open_qubits.size();
    void *ws = nullptr, *out = nullptr;
    if (hipMalloc(&ws, need) != hipSuccess) { set_error("qc_amplitude: workspace allocation failed"); return QC_ERR_NOMEM; }
    if (hipMalloc(&out, n_out * sizeof(double)) != hipSuccess) { hipFree(ws); set_error("qc_amplitude: allocation failed"); return QC_ERR_NOMEM; }
    qc_status st = QC_OK;
    std::vector<double> res(n_out, 0.0);
    if (hipMemset(out, 0, n_out * sizeof(double)) != hipSuccess) st = QC_ERR_DEVICE;
    if (st == QC_OK) {
        const uint64_t n_slices = uint64_t(1) << k;
        st = qc_contract_slices(plan, 0, n_slices, bits, 1, prec, ws, need, nullptr, (double *)out, nullptr);
    }
    if (st == QC_OK) {
        if (hipDeviceSynchronize() != hipSuccess ||
            hipMemcpy(res.data(), out, n_out * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
            set_error(std::string("qc_amplitude: ") + hipGetErrorString(hipGetLastError()));
            st = QC_ERR_DEVICE;
        }
    }
    hipFree(ws);
    hipFree(out);
    if (st == QC_OK) std::copy(res.begin(), res.end(), out_host);
    return st;
}

// ------------------------------------------------------------------ batches
namespace qc {
namespace {
constexpr int kBatchStreams = 8;

struct BatchLayout {
    size_t desc_off, bits_off, done_off, partial_off, steps_off, part_bytes, total;
    std::vector<int> fused;                   // request indices run by the fused batch kernel
    std::vector<int> stepwise;                // the others
    std::vector<Exec> exec;                   // per request
    std::vector<int> want;                    // per request: log2 slices wanted in flight
    int64_t n_items = 0, partial_elems = 0;
    int max_pair_elems = 0, bits_stride = 16;
};

bool batch_layout(const qc_request *reqs, int n, int prec, size_t ws_bytes, BatchLayout &L, std::string &err) {
    L.exec.assign(n, Exec());
    L.want.assign(n, 0);
    L.part_bytes = 0;
    for (int r = 0; r < n; ++r) {
        const qc_request &q = reqs[r];
        const int k = (int)q.plan->sliced.size();
        const uint64_t range = q.s_end - q.s_begin;
        L.bits_stride = std::max(L.bits_stride, (q.plan->net.n_qubits + 15) & ~15);
        const int want = std::min({k, 12, ceil_log2((int64_t)std::max<uint64_t>(range, 1))});
        Exec x;
        if (!choose_exec(q.plan, 0, want, prec, 0, x, err)) return false;
        L.exec[r] = x;
        L.want[r] = want;
        if (range == 0) continue;
        if (x.fused) {
            L.fused.push_back(r);
            L.n_items += int64_t(range);
            const uint64_t base = q.s_begin & ~uint64_t(63);
            L.partial_elems += int64_t((q.s_end - base + 63) & ~uint64_t(63));
            L.max_pair_elems = std::max(L.max_pair_elems, pair_elems_of(*x.prog));
        } else {
            L.stepwise.push_back(r);
            L.part_bytes = std::max(L.part_bytes, ws_layout(x, q.plan->net.n_qubits).total);
        }
    }
    const size_t nf = L.fused.size();
    L.desc_off = 0;
    L.bits_off = align256(nf * sizeof(BatchReq));
    L.done_off = L.bits_off + align256(nf * size_t(L.bits_stride));
    L.partial_off = L.done_off + align256(nf * sizeof(uint32_t));
    L.steps_off = L.partial_off + align256(size_t(L.partial_elems) * sizeof(float2));
    const int streams = std::min<int>(kBatchStreams, (int)L.stepwise.size());
    L.total = L.steps_off + size_t(streams) * align256(L.part_bytes);
    if (ws_bytes && L.total > ws_bytes) { err = "workspace too small for the batch"; return false; }
    return true;
}

std::mutex g_stream_mu;
std::map<int, std::vector<hipStream_t>> g_streams;

bool batch_streams(int dev, std::vector<hipStream_t> &out, std::string &err) {
    std::lock_guard<std::mutex> lk(g_stream_mu);
    auto &v = g_streams[dev];
    while ((int)v.size() < kBatchStreams) {
        hipStream_t s = nullptr;
        QC_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        v.push_back(s);
    }
    out = v;
    return true;
}
}  // namespace
}  // namespace qc

static qc_status check_requests(const char *fn, const qc_request *reqs, int32_t n, qc_precision prec) {
    const std::string f(fn);
    if (!reqs || n < 1 || !valid_prec(prec)) { set_error(f + ": invalid argument"); return QC_ERR_INVALID_ARG; }
    for (int32_t r = 0; r < n; ++r) {
        const qc_request &q = reqs[r];
        if (!q.plan || !q.bitstring) { set_error(f + ": request with NULL plan or bitstring"); return QC_ERR_INVALID_ARG; }
        if (!q.plan->open_qubits.empty()) {
            set_error(f + ": plans with open output qubits are not accepted in a batch");
            return QC_ERR_UNSUPPORTED;
        }
        const int k = (int)q.plan->sliced.size();
        const uint64_t n_slices = k >= 64 ? ~uint64_t(0) : (uint64_t(1) << k);
        if (q.s_begin > q.s_end || q.s_end > n_slices) {
            set_error(f + ": request slice range out of bounds");
            return QC_ERR_RANGE;
        }
        if (!check_bitstrings(q.plan, q.bitstring, 1)) {
            set_error(f + ": bitstring entries must be 0 or 1");
            return QC_ERR_INVALID_ARG;
        }
    }
    return QC_OK;
}

extern "C" size_t qc_batch_workspace_bytes(const qc_request *reqs, int32_t n, qc_precision prec) {
    if (check_requests("qc_batch_workspace_bytes", reqs, n, prec) != QC_OK) return 0;
    qc::BatchLayout L;
    std::string err;
    if (!qc::batch_layout(reqs, n, qc::prec_code(prec), 0, L, err)) {
        set_error("qc_batch_workspace_bytes: " + err);
        return 0;
    }
    return std::max<size_t>(L.total, 256);
}

extern "C" qc_status qc_contract_batch(const qc_request *reqs, int32_t n, qc_precision prec, void *ws, size_t ws_bytes,
                                       void *stream, double *out_dev, uint64_t *t_done_dev) {
    const qc_status cs = check_requests("qc_contract_batch", reqs, n, prec);
    if (cs != QC_OK) return cs;
    if (!ws || !out_dev || !t_done_dev) { set_error("qc_contract_batch: NULL argument"); return QC_ERR_INVALID_ARG; }
    qc::BatchLayout L;
    std::string err;
    if (!qc::batch_layout(reqs, n, qc::prec_code(prec), ws_bytes, L, err)) {
        set_error("qc_contract_batch: " + err);
        return err.find("workspace") != std::string::npos ? QC_ERR_NOMEM : QC_ERR_UNSUPPORTED;
    }
    const hipStream_t st = (hipStream_t)stream;
    char *w = (char *)ws;
    hipEvent_t fork = nullptr;
    auto fail = [&](const std::string &m) {
        if (fork) (void)hipEventDestroy(fork);
        set_error("qc_contract_batch: " + m);
        return QC_ERR_DEVICE;
    };
    // Batch start, and requests with an empty range complete at once.
    qc::launch_stamp(t_done_dev + n, st);
    for (int32_t r = 0; r < n; ++r)
        if (reqs[r].s_begin == reqs[r].s_end) qc::launch_stamp(t_done_dev + r, st);
    // Stepwise requests run on internal streams (each with its own workspace
    // part) that start after the caller's prior work, marked here, before the
    // fused launch, which they therefore do not wait for; the caller's stream
    // waits for them at the end.
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail("no device");
    if (!L.stepwise.empty()) {
        if (!qc::batch_streams(dev, streams, err)) return fail(err);
        if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess || hipEventRecord(fork, st) != hipSuccess)
            return fail("event");
    }
    // Fused requests: one launch over every (request, slice) pair, enqueued
    // before the stepwise requests so that the device starts these short
    // requests first instead of queueing them behind long ones.
    if (!L.fused.empty()) {
        std::vector<qc::BatchReq> desc(L.fused.size());
        std::vector<uint8_t> bits(L.fused.size() * size_t(L.bits_stride), 0);
        int64_t item = 0, poff = 0;
        for (size_t j = 0; j < L.fused.size(); ++j) {
            const int r = L.fused[j];
            const qc_request &q = reqs[r];
            qc::Program &prog = *L.exec[r].prog;
            {
                std::lock_guard<std::mutex> lk(q.plan->dev_mu);
                if (!qc::ensure_device(q.plan, prog, true, err)) return fail(err);
            }
            std::memcpy(bits.data() + j * L.bits_stride, q.bitstring, q.plan->net.n_qubits);
            qc::BatchReq &d = desc[j];
            std::memset(&d, 0, sizeof(d));
            d.level_start = (const int32_t *)prog.dc.p[qc::kCFusedLevels];
            d.items = (const int4 *)prog.dc.p[qc::kCFusedItems];
            d.items2 = (const int2 *)prog.dc.p[qc::kCFusedItems2];
            d.pool = (const int32_t *)prog.dc.p[qc::kCFusedPool];
            d.image = (const float2 *)prog.dc.p[qc::kCFusedImage];
            d.elems = (const int4 *)prog.dc.p[qc::kCFusedElems];
            d.base = (const double2 *)prog.dc.p[qc::kCBase];
            d.bits = (const uint8_t *)(w + L.bits_off) + j * L.bits_stride;
            d.n_levels = prog.n_levels;
            d.n_image = prog.n_image;
            d.n_elems = prog.n_leaf_elems;
            d.root_off = (int32_t)prog.lds_offset[prog.root_pre];
            d.zero_slot = qc::zero_slot_of(prog);
            d.out_index = r;
            d.s_begin = q.s_begin;
            d.s_base = q.s_begin & ~uint64_t(63);
            d.n_slices = int64_t(q.s_end - q.s_begin);
            d.item_off = item;
            d.partial_off = poff;
            item += d.n_slices;
            poff += int64_t((q.s_end - d.s_base + 63) & ~uint64_t(63));
        }
        if (hipMemcpyAsync(w + L.desc_off, desc.data(), desc.size() * sizeof(qc::BatchReq), hipMemcpyHostToDevice, st) !=
                hipSuccess ||
            hipMemcpyAsync(w + L.bits_off, bits.data(), bits.size(), hipMemcpyHostToDevice, st) != hipSuccess)
            return fail("copy");
        uint32_t *done = (uint32_t *)(w + L.done_off);
        float2 *partial = (float2 *)(w + L.partial_off);
        qc::launch_zero_u32(done, (int64_t)L.fused.size(), st);
        qc::launch_fused_batch((const qc::BatchReq *)(w + L.desc_off), (int)L.fused.size(), L.n_items,
                               L.max_pair_elems, partial, done, t_done_dev, st);
        qc::launch_reduce_batch((const qc::BatchReq *)(w + L.desc_off), (int)L.fused.size(), partial, out_dev, st);
    }
    if (!L.stepwise.empty()) {
        const int used = std::min<int>(qc::kBatchStreams, (int)L.stepwise.size());
        for (int i = 0; i < used; ++i)
            if (hipStreamWaitEvent(streams[i], fork, 0) != hipSuccess) return fail("stream wait");
        (void)hipEventDestroy(fork);
        fork = nullptr;
        // Dealt round-robin in order of increasing work (the lowered program's
        // flops times its chunks), so that light requests do not wait behind
        // heavy ones on the same stream.
        std::vector<std::pair<double, int>> order;
        for (const int r : L.stepwise) {
            const int b = L.exec[r].prog->b;
            const double chunks = double(((reqs[r].s_end - reqs[r].s_begin) + (uint64_t(1) << b) - 1) >> b);
            order.push_back({L.exec[r].prog->flops * chunks, r});
        }
        std::stable_sort(order.begin(), order.end(),
                         [](const std::pair<double, int> &x, const std::pair<double, int> &y) { return x.first < y.first; });
        for (size_t j = 0; j < order.size(); ++j) {
            const int r = order[j].second;
            const int i = int(j % used);
            void *part = w + L.steps_off + size_t(i) * qc::align256(L.part_bytes);
            qc::Exec x;
            if (!qc::choose_exec(reqs[r].plan, 0, L.want[r], qc::prec_code(prec), L.part_bytes, x, err)) return fail(err);
            if (!qc::enqueue(reqs[r].plan, x, reqs[r].s_begin, reqs[r].s_end, reqs[r].bitstring, false, 1, part,
                             streams[i], out_dev + 2 * r, nullptr, err))
                return fail(err);
            qc::launch_stamp(t_done_dev + r, streams[i]);
        }
    }
    // The caller's stream waits for the internal streams (after its own
    // fused work, which overlaps them).
    const int used = std::min<int>(qc::kBatchStreams, (int)L.stepwise.size());
    for (int i = 0; i < used; ++i) {
        hipEvent_t join = nullptr;
        if (hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(join, streams[i]) != hipSuccess || hipStreamWaitEvent(st, join, 0) != hipSuccess)
            return fail("event");
        events.push_back(join);
    }
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(hipGetErrorString(e));
    return QC_OK;
}

extern "C" qc_status qc_wall_clock_khz(int32_t *khz) {
    int dev = 0;
    if (!khz) { set_error("qc_wall_clock_khz: NULL argument"); return QC_ERR_INVALID_ARG; }
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) {
        set_error("qc_wall_clock_khz: device query failed");
        return QC_ERR_DEVICE;
    }
    return QC_OK;
}

extern "C" qc_status qc_plan_set_graphs(qc_plan *plan, int32_t on) {
    if (!plan) { set_error("qc_plan_set_graphs: NULL plan"); return QC_ERR_INVALID_ARG; }
    std::lock_guard<std::mutex> lk(plan->dev_mu);
    plan->use_graphs = on != 0;
    return QC_OK;
}

extern "C" qc_status qc_plan_set_fused_slice_bits(qc_plan *plan, int32_t b) {
    if (!plan || b < -1 || b > qc::kFusedMaxSliceBits) {
        set_error("qc_plan_set_fused_slice_bits: invalid argument");
        return QC_ERR_INVALID_ARG;
    }
    if (b > (int)plan->sliced.size()) {
        set_error("qc_plan_set_fused_slice_bits: more slice bits than the plan has");
        return QC_ERR_RANGE;
    }
    std::string err;
    if (b > 0) {
        qc::Program *p = qc::get_program(plan, b, 0, err);
        if (!p) { set_error("qc_plan_set_fused_slice_bits: " + err); return QC_ERR_UNSUPPORTED; }
        if (!qc::fused_fits(plan, *p)) {
            set_error("qc_plan_set_fused_slice_bits: the fused program with these slice bits does not fit in LDS");
            return QC_ERR_UNSUPPORTED;
        }
    }
    std::lock_guard<std::mutex> lk(plan->dev_mu);
    plan->fused_b = b;
    return QC_OK;
}

extern "C" qc_status qc_plan_set_fused_shape(qc_plan *plan, int32_t items_per_workgroup, int32_t waves_per_item) {
    bool ok = items_per_workgroup == 0 && waves_per_item == 0;
    for (const auto &shape : qc::kFusedShapes)
        ok = ok || (shape[0] == items_per_workgroup && shape[1] == waves_per_item);
    if (!plan || !ok) {
        set_error("qc_plan_set_fused_shape: invalid argument");
        return QC_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(plan->dev_mu);
    plan->fused_force_pairs = items_per_workgroup;
    plan->fused_force_waves = waves_per_item;
    return QC_OK;
}

extern "C" qc_status qc_tune(qc_plan *plan, int64_t chunk_slices, int32_t n_bs, qc_precision prec, void *ws,
                             size_t ws_bytes, void *stream, const char *cache_path, int32_t *n_timed) {
    if (!plan || !ws || chunk_slices < 1 || n_bs < 1 || n_bs > (1 << qc::kMaxBsBits) || !valid_prec(prec)) {
        set_error("qc_tune: invalid argument");
        return QC_ERR_INVALID_ARG;
    }
    const int k = (int)plan->sliced.size();
    const int b = qc::ceil_log2(chunk_slices);
    if (b > k) { set_error("qc_tune: more slices than the plan has"); return QC_ERR_RANGE; }
    std::string err;
    qc::Exec x;
    if (!qc::choose_exec(plan, qc::ceil_log2(n_bs), b, qc::prec_code(prec), ws_bytes, x, err)) {
        set_error("qc_tune: " + err);
        return err.find("workspace") != std::string::npos ? QC_ERR_NOMEM : QC_ERR_UNSUPPORTED;
    }
    int32_t timed = 0;
    if (!x.fused) {
        std::lock_guard<std::mutex> lk(plan->dev_mu);
        qc::Program &prog = *x.prog;
        const hipStream_t st = (hipStream_t)stream;
        if (!qc::ensure_device(plan, prog, false, err)) { set_error("qc_tune: " + err); return QC_ERR_DEVICE; }
        int dev = 0;
        hipDeviceProp_t props;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&props, dev) != hipSuccess) {
            set_error("qc_tune: device query failed");
            return QC_ERR_DEVICE;
        }
        const std::string arch = std::string(props.gcnArchName).substr(0, std::string(props.gcnArchName).find(':'));
        std::lock_guard<std::mutex> tl(qc::g_tune_mu);
        qc::tune_load(cache_path);
        const qc::WsLayout w = qc::ws_layout(x, plan->net.n_qubits);
        float2 *tensors = (float2 *)((char *)ws + w.tensor_off);
        float2 *kscratch = (float2 *)((char *)ws + w.ksplit_off);
        uint32_t *amax = x.prec == qc::kPrecFP16 ? (uint32_t *)((char *)ws + w.amax_off) : nullptr;
        std::vector<int> slot(prog.tensors.size());
        for (size_t t = 0; t < slot.size(); ++t) slot[t] = (int)t;
        for (const qc::Op &op : prog.ops)
            if (op.kind == qc::Op::TRANSPOSE) slot[prog.transposes[op.index].dst] = slot[prog.transposes[op.index].src];
        if (amax) qc::launch_zero_u32(amax, (int64_t)slot.size(), st);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            set_error("qc_tune: event creation failed");
            return QC_ERR_DEVICE;
        }
        qc_status status = QC_OK;
        // Operands are the program's own workspace regions: their contents do
        // not matter for timing, and every access stays inside the tensors.
        for (size_t gi = 0; gi < prog.gemms.size(); ++gi) {
            qc::GemmOp &g = prog.gemms[gi];
            if (prog.gemm_micro[gi]) continue;  // run by the micro-step kernel
            const qc::GemmDesc d = qc::make_gemm(prog, g, tensors, x.prec, amax, slot, kscratch);
            const std::string key = qc::tune_key(arch, d, g.a_km, g.b_nk);
            auto it = qc::g_tune.find(key);
            if (it == qc::g_tune.end()) {
                int best = -1;
                float best_ms = 0.f;
                // The one-thread-per-output vector form is not timed on large
                // steps that an MFMA form can take (it is far slower there).
                bool mfma_ok = false;
                for (int v = qc::kVarMfma11; v < qc::kVarCount; ++v) mfma_ok |= qc::gemm_variant_ok(d, v);
                const double flops = 8.0 * double(d.nb) * double(d.m) * double(d.n) * double(d.k);
                for (int v = 0; v < qc::kVarCount; ++v) {
                    if (!qc::gemm_variant_ok(d, v)) continue;
                    if (mfma_ok && flops > 1e8 && v == qc::kVarValu) continue;
                    qc::launch_gemm_variant(d, v, st);  // warm-up
                    float ms = 0.f;
                    if (hipEventRecord(e0, st) != hipSuccess) { status = QC_ERR_DEVICE; break; }
                    for (int r = 0; r < 3; ++r) qc::launch_gemm_variant(d, v, st);
                    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                        status = QC_ERR_DEVICE;
                        break;
                    }
                    if (best < 0 || ms < best_ms) { best = v; best_ms = ms; }
                }
                if (status != QC_OK || best < 0) break;
                it = qc::g_tune.insert({key, {best, best_ms / 3}}).first;
                ++timed;
            }
            g.variant[x.prec] = it->second.first;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (status == QC_OK && hipGetLastError() != hipSuccess) status = QC_ERR_DEVICE;
        if (status != QC_OK) { set_error("qc_tune: a timing launch failed"); return status; }
        // Captured graphs hold the previous forms.
        if (!prog.graphs.empty()) {
            if (hipDeviceSynchronize() != hipSuccess) { set_error("qc_tune: synchronize failed"); return QC_ERR_DEVICE; }
            for (auto &gr : prog.graphs) (void)hipGraphExecDestroy((hipGraphExec_t)gr.second);
            prog.graphs.clear();
        }
        if (!qc::tune_save(cache_path, err)) { set_error("qc_tune: " + err); return QC_ERR_INVALID_ARG; }
    }
    if (n_timed) *n_timed = timed;
    return QC_OK;
}

extern "C" qc_status qc_profile_enable(qc_plan *plan, int32_t on) {
    if (!plan) { set_error("qc_profile_enable: NULL plan"); return QC_ERR_INVALID_ARG; }
    plan->profiling = on != 0;
    return QC_OK;
}

extern "C" qc_status qc_profile_read(qc_plan *plan, qc_kernel_stat_t *out, int32_t cap, int32_t *n) {
    if (!plan || !n || cap < 0 || (cap > 0 && !out)) { set_error("qc_profile_read: invalid argument"); return QC_ERR_INVALID_ARG; }
    std::vector<qc_kernel_stat_t> stats;
    qc_status st = QC_OK;
    for (auto &pe : plan->prof_pending) {
        float ms = 0.f;
        if (hipEventSynchronize((hipEvent_t)pe.e1) != hipSuccess ||
            hipEventElapsedTime(&ms, (hipEvent_t)pe.e0, (hipEvent_t)pe.e1) != hipSuccess) {
            set_error("qc_profile_read: event query failed");
            st = QC_ERR_DEVICE;
        }
        qc_kernel_stat_t *s = nullptr;
        for (auto &x : stats)
            if (pe.kind == x.kind) s = &x;
        if (!s) {
            stats.push_back(qc_kernel_stat_t{});
            s = &stats.back();
            std::strncpy(s->kind, pe.kind.c_str(), sizeof(s->kind) - 1);
        }
        s->launches += 1;
        s->total_ms += ms;
        s->flops += pe.flops;
        s->bytes += pe.bytes;
        plan->prof_pool.push_back(pe.e0);
        plan->prof_pool.push_back(pe.e1);
    }
    plan->prof_pending.clear();
    *n = (int32_t)stats.size();
    for (int32_t i = 0; i < std::min<int32_t>(cap, *n); ++i) out[i] = stats[i];
    return st;
}

extern "C" void qc_plan_destroy(qc_plan *plan) {
    if (!plan) return;
    for (auto &pe : plan->prof_pending) plan->prof_pool.push_back(pe.e0), plan->prof_pool.push_back(pe.e1);
    for (void *e : plan->prof_pool) hipEventDestroy((hipEvent_t)e);
    for (auto &kv : plan->programs) qc::free_program_device(*kv.second);
    if (plan->capture_stream) (void)hipStreamDestroy((hipStream_t)plan->capture_stream);
    delete plan;
}

extern "C" int64_t qc_gemm_kparts(int64_t nb, int64_t m, int64_t n, int64_t k) {
    if (nb < 1 || m < 1 || n < 1 || k < 1) return 1;
    return qc::gemm_kparts(nb, m, n, k);
}

extern "C" qc_status qc_kernel_gemm_kparts(const void *A, const void *B, void *C, int64_t nb, int64_t m, int64_t n,
                                           int64_t k, int32_t a_km, int32_t b_nk, qc_precision prec, int32_t form,
                                           int64_t kparts, void *scratch, void *scale_ws, void *stream) {
    if (!A || !B || !C || nb < 1 || m < 1 || n < 1 || k < 1 || !valid_prec(prec) || form < -1 ||
        form >= qc::kVarCount || kparts < 0 || kparts > 1024 || (kparts & (kparts - 1)) != 0) {
        set_error("qc_kernel_gemm: invalid argument");
        return QC_ERR_INVALID_ARG;
    }
    if (prec == QC_SPLIT_FP16 && !scale_ws) {
        set_error("qc_kernel_gemm: split FP16 needs scale_ws");
        return QC_ERR_INVALID_ARG;
    }
    const hipStream_t st = (hipStream_t)stream;
    uint32_t *amax = (uint32_t *)scale_ws;
    qc::GemmDesc d;
    d.A = (const float2 *)A; d.B = (const float2 *)B; d.C = (float2 *)C;
    d.nb = nb; d.m = m; d.n = n; d.k = k;
    d.sAb = m * k;
    if (a_km) { d.sAk = m; d.sAm = 1; } else { d.sAm = k; d.sAk = 1; }
    d.sBb = k * n;
    if (b_nk) { d.sBn = k; d.sBk = 1; } else { d.sBk = n; d.sBn = 1; }
    d.sCb = m * n; d.sCm = n; d.sCn = 1;
    d.prec = qc::prec_code(prec);
    d.amax_a = amax;
    d.amax_b = amax ? amax + 1 : nullptr;
    d.amax_c = amax ? amax + 2 : nullptr;
    if (form >= 0 && !qc::gemm_variant_ok(d, form)) {
        set_error("qc_kernel_gemm_form: the form does not apply to this shape and precision");
        return QC_ERR_UNSUPPORTED;
    }
    const int v = form >= 0 ? form : qc::gemm_default_variant(d);
    if (kparts == 0) kparts = qc::gemm_kparts(nb, m, n, k);
    // Every MFMA form but the streaming ones, and the dot form, split over
    // k; each part must itself be a product the form applies to.
    const bool splits = v != qc::kVarValu && v != qc::kVarSkinny && v != qc::kVarSkinnyT && v != qc::kVarRows &&
                        v != qc::kVarStream && v != qc::kVarStreamT && v != qc::kVarStream16;
    qc::GemmDesc part = d;
    if (kparts > 1) part.k = k / kparts;
    if (kparts > 1 && (!splits || k % kparts != 0 || !scratch || !qc::gemm_variant_ok(part, v))) {
        set_error("qc_kernel_gemm_kparts: a split over k needs an MFMA or dot form, kparts dividing k with each "
                  "part a product the form applies to, and a scratch buffer");
        return QC_ERR_UNSUPPORTED;
    }
    if (kparts > 1) {
        d.kparts = kparts;
        d.kscratch = (float2 *)scratch;
    }
    if (amax) {
        qc::launch_zero_u32(amax, 3, st);
        qc::launch_absmax(d.A, nb * m * k, amax, st);
        qc::launch_absmax(d.B, nb * k * n, amax + 1, st);
    }
    qc::launch_gemm_variant(d, v, st);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error(std::string("qc_kernel_gemm: ") + hipGetErrorString(e)); return QC_ERR_DEVICE; }
    return QC_OK;
}

extern "C" qc_status qc_kernel_gemm_form(const void *A, const void *B, void *C, int64_t nb, int64_t m, int64_t n,
                                         int64_t k, int32_t a_km, int32_t b_nk, qc_precision prec, int32_t form,
                                         void *scale_ws, void *stream) {
    return qc_kernel_gemm_kparts(A, B, C, nb, m, n, k, a_km, b_nk, prec, form, 1, nullptr, scale_ws, stream);
}

extern "C" qc_status qc_kernel_gemm(const void *A, const void *B, void *C, int64_t nb, int64_t m, int64_t n, int64_t k,
                                    int32_t a_km, int32_t b_nk, qc_precision prec, void *scale_ws, void *stream) {
    return qc_kernel_gemm_form(A, B, C, nb, m, n, k, a_km, b_nk, prec, -1, scale_ws, stream);
}

extern "C" qc_status qc_kernel_transpose(const void *in, void *out, int32_t rank, const int32_t *perm, void *stream) {
    if (!in || !out || rank < 0 || rank > 40 || (rank > 0 && !perm)) { set_error("qc_kernel_transpose: invalid argument"); return QC_ERR_INVALID_ARG; }
    std::vector<int> p(perm, perm + rank), seen(rank, 0);
    for (int v : p) {
        if (v < 0 || v >= rank || seen[v]++) { set_error("qc_kernel_transpose: perm is not a permutation"); return QC_ERR_INVALID_ARG; }
    }
    qc::launch_transpose(qc::make_transpose_desc((const float2 *)in, (float2 *)out, rank, p), (hipStream_t)stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error(std::string("qc_kernel_transpose: ") + hipGetErrorString(e)); return QC_ERR_DEVICE; }
    return QC_OK;
}
