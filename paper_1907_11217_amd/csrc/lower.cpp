// Lowering of a contraction tree to a device program for 2^b slices and 2^m
// bitstrings in flight.
//
// In-flight slice bits are the first b sliced segments left open (never
// summed); bitstring bits are extra open indices carried by every leaf that
// touches a fixed output segment; the output segments of open output qubits
// are open indices of their own.  All of them behave like hyper-edges: in a step
// where both operands hold them they are batch indices, otherwise free
// indices.  Each step C = A (x) B is classified per index as batch (in both,
// still needed later), contracted (in both, needed nowhere else), free-A or
// free-B, and run as a batched GEMM C[b][m][n] = sum_k A[b][m][k] B[b][k][n]
// after at most one bit-permuting transpose per operand.
#include <algorithm>
#include <climits>
#include <cstring>
#include <sstream>

#include "plan.h"

namespace qc {

namespace {

enum Cls { CB = 0, CM = 1, CN = 2, CK = 3 };

// True if `layout` is [first-class run][x run][y run] with x, y the two other
// classes of this operand, each run contiguous (runs may be empty).
bool groupable(const std::vector<int> &layout, const std::vector<int> &cls, int other_a, int other_b,
               bool &a_first) {
    // Sequence of classes with runs collapsed.
    std::vector<int> runs;
    for (size_t i = 0; i < layout.size(); ++i)
        if (runs.empty() || runs.back() != cls[i]) runs.push_back(cls[i]);
    std::vector<int> seen;
    for (int r : runs) {
        if (std::count(seen.begin(), seen.end(), r)) return false;
        seen.push_back(r);
    }
    // Batch must come first if present.
    size_t pos = 0;
    if (!runs.empty() && runs[0] == CB) pos = 1;
    for (size_t i = pos; i < runs.size(); ++i)
        if (runs[i] == CB) return false;
    a_first = true;
    for (size_t i = pos; i < runs.size(); ++i) {
        if (runs[i] == other_a) { a_first = true; break; }
        if (runs[i] == other_b) { a_first = false; break; }
    }
    return true;
}

std::vector<int> of_class(const std::vector<int> &layout, const std::vector<int> &cls, int c) {
    std::vector<int> out;
    for (size_t i = 0; i < layout.size(); ++i)
        if (cls[i] == c) out.push_back(layout[i]);
    return out;
}

std::vector<int> cat(std::initializer_list<std::vector<int>> parts) {
    std::vector<int> out;
    for (auto &p : parts) out.insert(out.end(), p.begin(), p.end());
    return out;
}

// Best-fit offset allocator over a growing arena (units: complex64 elements).
struct Arena {
    std::vector<std::pair<int64_t, int64_t>> free_;  // (offset, size), sorted by offset
    int64_t end = 0;
    int64_t granule = 32;  // allocation unit (elements), a power of two
    int64_t align(int64_t v) const { return (v + granule - 1) & ~(granule - 1); }
    int64_t alloc(int64_t n) {
        n = align(std::max<int64_t>(n, 1));
        int best = -1;
        for (size_t i = 0; i < free_.size(); ++i)
            if (free_[i].second >= n && (best < 0 || free_[i].second < free_[best].second)) best = (int)i;
        if (best >= 0) {
            const int64_t off = free_[best].first;
            free_[best].first += n;
            free_[best].second -= n;
            if (free_[best].second == 0) free_.erase(free_.begin() + best);
            return off;
        }
        // Extend, absorbing a free block that touches the end.
        if (!free_.empty() && free_.back().first + free_.back().second == end) {
            const int64_t off = free_.back().first;
            free_.pop_back();
            end = off + n;
            return off;
        }
        const int64_t off = end;
        end += n;
        return off;
    }
    void release(int64_t off, int64_t n) {
        n = align(std::max<int64_t>(n, 1));
        free_.push_back({off, n});
        std::sort(free_.begin(), free_.end());
        std::vector<std::pair<int64_t, int64_t>> merged;
        for (auto &f : free_) {
            if (!merged.empty() && merged.back().first + merged.back().second == f.first) merged.back().second += f.second;
            else merged.push_back(f);
        }
        free_ = std::move(merged);
    }
};

}  // namespace

static bool lower(const qc_plan *plan, int b, int m, Program &prog, std::string &err) {
    const Network &net = plan->net;
    const int n_idx = net.n_index();
    const int L = (int)net.leaves.size();
    prog.b = b;
    prog.m = m;
    const int k = (int)plan->sliced.size();
    if (b < 0 || b > k) { err = "in-flight slice bits out of range"; return false; }
    if (m < 0 || m > kMaxBsBits) { err = "in-flight bitstring bits out of range"; return false; }
    std::vector<char> fixed(n_idx, 0), open(n_idx, 0);
    for (int j = 0; j < k; ++j) (j < b ? open : fixed)[plan->sliced[j]] = 1;
    for (int e = 0; e < n_idx; ++e)
        if (net.open_out[e]) open[e] = 1;   // open outputs: indices of the result

    std::vector<int> bs_bits;  // major -> minor
    for (int i = m - 1; i >= 0; --i) bs_bits.push_back(kBsBase + i);

    // Leaf layouts: [bitstring bits][summed indices in base order].
    std::vector<std::vector<int>> layout;   // per program tensor
    std::vector<int> total(n_idx, 0);
    for (int t = 0; t < L; ++t) {
        const Tensor &T = net.leaves[t];
        bool has_out = false;
        std::vector<int> lay;
        for (int e : T.idx) {
            if (net.fixed_out(e)) has_out = true;
            else if (!fixed[e]) { lay.push_back(e); ++total[e]; }
        }
        if (has_out) lay.insert(lay.begin(), bs_bits.begin(), bs_bits.end());
        if ((int)lay.size() > kMaxRank) { err = "leaf rank exceeds the device limit"; return false; }
        layout.push_back(lay);
        prog.leaves.push_back(LeafOp{t, t});
    }
    auto is_open = [&](int e) { return e >= kBsBase || open[e]; };
    // Per tensor: how many of each index's leaves it covers.
    std::vector<std::vector<std::pair<int, int>>> counts(L);
    for (int t = 0; t < L; ++t)
        for (int e : layout[t])
            if (e < kBsBase) counts[t].push_back({e, 1});
    for (auto &c : counts) std::sort(c.begin(), c.end());

    std::vector<int> tensor_of(L);  // tree node id -> program tensor id
    for (int t = 0; t < L; ++t) tensor_of[t] = t;
    auto new_tensor = [&](std::vector<int> lay) {
        layout.push_back(std::move(lay));
        return (int)layout.size() - 1;
    };
    auto emit_transpose = [&](int src, std::vector<int> dst_layout) {
        const int dst = new_tensor(std::move(dst_layout));
        prog.transposes.push_back(TransposeOp{src, dst});
        prog.ops.push_back(Op{Op::TRANSPOSE, (int)prog.transposes.size() - 1});
        prog.transpose_bytes += 16.0 * std::ldexp(1.0, (int)layout[src].size());
        return dst;
    };

    for (size_t s = 0; s < plan->tree.size(); ++s) {
        const int ta = tensor_of[plan->tree[s].a], tb = tensor_of[plan->tree[s].b];
        const std::vector<int> LA = layout[ta], LB = layout[tb];
        // Merge counts.
        const auto &ca = counts[plan->tree[s].a], &cb = counts[plan->tree[s].b];
        std::vector<std::pair<int, int>> cc;
        {
            size_t x = 0, y = 0;
            while (x < ca.size() || y < cb.size()) {
                if (y == cb.size() || (x < ca.size() && ca[x].first < cb[y].first)) cc.push_back(ca[x++]);
                else if (x == ca.size() || cb[y].first < ca[x].first) cc.push_back(cb[y++]);
                else { cc.push_back({ca[x].first, ca[x].second + cb[y].second}); ++x; ++y; }
            }
        }
        auto count_of = [&](int e) {
            auto it = std::lower_bound(cc.begin(), cc.end(), std::make_pair(e, INT_MIN));
            return (it != cc.end() && it->first == e) ? it->second : 0;
        };
        auto in = [](const std::vector<int> &v, int e) { return std::find(v.begin(), v.end(), e) != v.end(); };
        std::vector<int> clsA(LA.size()), clsB(LB.size());
        for (size_t i = 0; i < LA.size(); ++i) {
            const int e = LA[i];
            if (in(LB, e)) clsA[i] = (!is_open(e) && count_of(e) == total[e]) ? CK : CB;
            else clsA[i] = CM;
        }
        for (size_t i = 0; i < LB.size(); ++i) {
            const int e = LB[i];
            if (in(LA, e)) clsB[i] = (!is_open(e) && count_of(e) == total[e]) ? CK : CB;
            else clsB[i] = CN;
        }
        bool a_mfirst = true, b_kfirst = true;
        const bool a_ok = groupable(LA, clsA, CM, CK, a_mfirst);
        const bool b_ok = groupable(LB, clsB, CK, CN, b_kfirst);
        std::vector<int> Ab = of_class(LA, clsA, CB), Am = of_class(LA, clsA, CM), Ak = of_class(LA, clsA, CK);
        std::vector<int> Bb = of_class(LB, clsB, CB), Bk = of_class(LB, clsB, CK), Bn = of_class(LB, clsB, CN);
        int opA = ta, opB = tb;
        bool a_km = !a_mfirst, b_nk = !b_kfirst;
        const int64_t szA = int64_t(1) << LA.size(), szB = int64_t(1) << LB.size();
        // A reordered operand is written by its producer straight into the
        // new layout (see the folding below).  Its writes stay coalesced when
        // the new layout's lowest bits are the producer's own lowest output
        // bits in order, so among the valid layouts (batch outermost, the
        // other two groups in either order, free indices in the producer's
        // order) the one keeping the longest such run is taken; leaves and
        // small tensors cost nothing.
        auto by_nat = [](std::vector<int> v, const std::vector<int> &nat) {
            std::stable_sort(v.begin(), v.end(), [&](int x, int y) {
                return std::find(nat.begin(), nat.end(), x) < std::find(nat.begin(), nat.end(), y);
            });
            return v;
        };
        auto write_cost = [&](int t, const std::vector<int> &lay) {
            const std::vector<int> &nat = layout[t];
            if (t < L || nat.size() <= 12) return 0.0;
            size_t q = 0;
            while (q < nat.size() && lay[lay.size() - 1 - q] == nat[nat.size() - 1 - q]) ++q;
            return std::ldexp(1.0, (int)nat.size()) * (q >= 4 ? 0.0 : (4.0 - double(q)) / 4.0);
        };
        if (!(a_ok && b_ok && Ab == Bb && Ak == Bk)) {
            // Candidates: reorder B only (A as it is), A only, or both.
            struct Cand {
                int kind = -1;  // 0 B only, 1 A only, 2 both
                double cost = 0;
                std::vector<int> la, lb, b_, k_, m_, n_;
                bool km = false, nk = false;
            } best;
            auto offer = [&](Cand c) {
                if (best.kind < 0 || c.cost < best.cost) best = std::move(c);
            };
            const std::vector<int> m_ = by_nat(Am, LA), n_ = by_nat(Bn, LB);
            if (a_ok) {
                for (int nk = 0; nk < 2; ++nk) {
                    Cand c;
                    c.kind = 0;
                    c.lb = nk ? cat({Ab, n_, Ak}) : cat({Ab, Ak, n_});
                    c.cost = write_cost(tb, c.lb);
                    c.b_ = Ab; c.k_ = Ak; c.m_ = Am; c.n_ = n_;
                    c.km = a_km; c.nk = nk;
                    offer(std::move(c));
                }
            }
            if (b_ok) {
                for (int km = 0; km < 2; ++km) {
                    Cand c;
                    c.kind = 1;
                    c.la = km ? cat({Bb, Bk, m_}) : cat({Bb, m_, Bk});
                    c.cost = write_cost(ta, c.la);
                    c.b_ = Bb; c.k_ = Bk; c.m_ = m_; c.n_ = Bn;
                    c.km = km; c.nk = b_nk;
                    offer(std::move(c));
                }
            }
            for (int bsel = 0; bsel < 2; ++bsel)
                for (int ksel = 0; ksel < 2; ++ksel)
                    for (int km = 0; km < 2; ++km)
                        for (int nk = 0; nk < 2; ++nk) {
                            Cand c;
                            c.kind = 2;
                            c.b_ = by_nat(Ab, bsel ? LB : LA);
                            c.k_ = by_nat(Ak, ksel ? LB : LA);
                            c.m_ = m_; c.n_ = n_;
                            c.la = km ? cat({c.b_, c.k_, m_}) : cat({c.b_, m_, c.k_});
                            c.lb = nk ? cat({c.b_, n_, c.k_}) : cat({c.b_, c.k_, n_});
                            c.cost = write_cost(ta, c.la) + write_cost(tb, c.lb);
                            c.km = km; c.nk = nk;
                            offer(std::move(c));
                        }
            if (best.kind != 1) opB = emit_transpose(tb, best.lb);
            if (best.kind != 0) opA = emit_transpose(ta, best.la);
            Ab = Bb = best.b_; Ak = Bk = best.k_; Am = best.m_; Bn = best.n_;
            a_km = best.km; b_nk = best.nk;
        }
        const int tc = new_tensor(cat({Ab, Am, Bn}));
        GemmOp g;
        g.a_src = ta; g.b_src = tb;
        g.a = opA; g.b = opB; g.c = g.c_nat = tc;
        g.cls_b = (int)Ab.size(); g.cls_m = (int)Am.size(); g.cls_n = (int)Bn.size(); g.cls_k = (int)Ak.size();
        g.nb = int64_t(1) << g.cls_b; g.m = int64_t(1) << g.cls_m; g.n = int64_t(1) << g.cls_n; g.k = int64_t(1) << g.cls_k;
        g.a_km = a_km && g.m > 1 && g.k > 1;
        g.b_nk = b_nk && g.n > 1 && g.k > 1;
        if ((int)layout[tc].size() > kMaxRank) { err = "intermediate rank exceeds the device limit"; return false; }
        prog.gemms.push_back(g);
        prog.ops.push_back(Op{Op::GEMM, (int)prog.gemms.size() - 1});
        prog.flops += 8.0 * double(g.nb) * double(g.m) * double(g.n) * double(g.k);
        prog.bytes += 8.0 * double(g.nb) * double(g.m * g.k + g.k * g.n + g.m * g.n);
        // Counts of C: drop contracted indices.
        std::vector<std::pair<int, int>> keep;
        for (auto &v : cc)
            if (in(layout[tc], v.first)) keep.push_back(v);
        counts.push_back(std::move(keep));
        tensor_of.push_back(tc);
    }
    int root = tensor_of.back();
    prog.root_pre = root;
    std::vector<int> want;  // [slice bits][bitstring bits][open outputs, first qubit most significant]
    for (int j = b - 1; j >= 0; --j) want.push_back(plan->sliced[j]);
    want.insert(want.end(), bs_bits.begin(), bs_bits.end());
    for (int q : plan->open_qubits)
        for (int e = 0; e < n_idx; ++e)
            if (net.open_out[e] && net.out_qubit[e] == q) want.push_back(e);
    {
        std::vector<int> a = layout[root], w = want;
        std::sort(a.begin(), a.end());
        std::sort(w.begin(), w.end());
        if (a != w) { err = "internal: root indices are not the open indices"; return false; }
    }
    if (layout[root] != want) root = emit_transpose(root, want);
    prog.root = root;

    // Transposes are folded into the producer of their source (each tensor
    // has exactly one consumer): a leaf is instantiated directly in the
    // transposed layout, and a GEMM step writes its output in that layout
    // (its natural [batch][m][n] order stays recorded as c_nat, and the
    // kernels scatter the output bits accordingly).  Consumers then read the
    // producer's tensor as is.  Exception: a large GEMM output whose new
    // layout keeps fewer than kMinWriteRun of its natural lowest bits lowest
    // would be written in scattered 8- or 16-byte pieces; it is written in
    // natural order and moved by the LDS-staged transpose kernel instead
    // (coalesced on both sides, two more passes over the tensor, cheaper
    // than writes a sixteenth or an eighth as efficient).
    {
        std::vector<int> producer(layout.size(), -1), rename(layout.size());
        for (size_t i = 0; i < prog.gemms.size(); ++i) producer[prog.gemms[i].c] = (int)i;
        for (size_t t = 0; t < rename.size(); ++t) rename[t] = (int)t;
        std::vector<char> keep(prog.transposes.size(), 0);
        for (size_t ti = 0; ti < prog.transposes.size(); ++ti) {
            const TransposeOp &t = prog.transposes[ti];
            if (t.src < L) {
                layout[t.src] = layout[t.dst];
                rename[t.dst] = t.src;
            } else {
                GemmOp &g = prog.gemms[producer[t.src]];
                std::vector<int> x = layout[t.src], y = layout[t.dst];
                std::sort(x.begin(), x.end());
                std::sort(y.begin(), y.end());
                if (x != y || (int)x.size() != g.cls_b + g.cls_m + g.cls_n) {
                    err = "internal: a folded transpose is not a permutation of its step's output";
                    return false;
                }
                const std::vector<int> &nat = layout[t.src], &lay = layout[t.dst];
                size_t q = 0;
                while (q < nat.size() && lay[lay.size() - 1 - q] == nat[nat.size() - 1 - q]) ++q;
                if ((int)nat.size() >= kTransposeMinLog2 && (int)q < kMinWriteRun) {
                    keep[ti] = 1;
                    continue;
                }
                g.c = t.dst;
                rename[t.src] = t.dst;
            }
        }
        for (GemmOp &g : prog.gemms) {
            g.a = g.a_src = rename[g.a];
            g.b = g.b_src = rename[g.b];
        }
        prog.root = rename[prog.root];
        std::vector<Op> ops;
        std::vector<TransposeOp> kept;
        prog.transpose_bytes = 0;
        for (const Op &op : prog.ops) {
            if (op.kind == Op::GEMM) {
                ops.push_back(op);
            } else if (keep[op.index]) {
                kept.push_back(prog.transposes[op.index]);
                ops.push_back(Op{Op::TRANSPOSE, (int)kept.size() - 1});
                prog.transpose_bytes += 16.0 * std::ldexp(1.0, (int)layout[kept.back().src].size());
            }
        }
        prog.ops = std::move(ops);
        prog.transposes = std::move(kept);
        prog.root_pre = prog.root;
    }

    // Lifetimes and offsets.  Leaves are born before op 0; each op's output is
    // allocated before its inputs are released.
    const int nt = (int)layout.size();
    std::vector<int> death(nt, -1);
    for (size_t i = 0; i < prog.ops.size(); ++i) {
        const Op &op = prog.ops[i];
        if (op.kind == Op::TRANSPOSE) death[prog.transposes[op.index].src] = (int)i;
        else { death[prog.gemms[op.index].a] = (int)i; death[prog.gemms[op.index].b] = (int)i; }
    }
    prog.tensors.resize(nt);
    for (int t = 0; t < nt; ++t) prog.tensors[t].layout = layout[t];
    Arena arena;
    for (int t = 0; t < L; ++t) prog.tensors[t].offset = arena.alloc(prog.tensors[t].size());
    for (size_t i = 0; i < prog.ops.size(); ++i) {
        const Op &op = prog.ops[i];
        const int out = op.kind == Op::TRANSPOSE ? prog.transposes[op.index].dst : prog.gemms[op.index].c;
        prog.tensors[out].offset = arena.alloc(prog.tensors[out].size());
        for (int t = 0; t < nt; ++t)
            if (death[t] == (int)i) arena.release(prog.tensors[t].offset, prog.tensors[t].size());
    }
    prog.tensor_elems = arena.end;

    // Micro steps: GEMM steps whose output and (untransposed) operands have at
    // most 2^kMicroMaxLog2 entries and whose operands are leaves or outputs of
    // micro steps.  They run together in one kernel right after the leaves,
    // reading their operands as produced, so the transposes that fed them are
    // skipped.  Being computed before their turn, their outputs get a region
    // of their own after the arena.
    {
        std::vector<char> avail(nt, 0);
        std::vector<int> producer(nt, -1);
        for (int t = 0; t < L; ++t) avail[t] = 1;
        for (size_t i = 0; i < prog.ops.size(); ++i) {
            const Op &op = prog.ops[i];
            producer[op.kind == Op::TRANSPOSE ? prog.transposes[op.index].dst : prog.gemms[op.index].c] = (int)i;
        }
        prog.op_micro.assign(prog.ops.size(), 0);
        prog.gemm_micro.assign(prog.gemms.size(), 0);
        const int64_t cap = int64_t(1) << kMicroMaxLog2;
        int64_t extra = 0;
        for (size_t i = 0; i < prog.ops.size(); ++i) {
            const Op &op = prog.ops[i];
            if (op.kind != Op::GEMM) continue;
            const GemmOp &g = prog.gemms[op.index];
            if (!avail[g.a_src] || !avail[g.b_src] || prog.tensors[g.c].size() > cap ||
                prog.tensors[g.a_src].size() > cap || prog.tensors[g.b_src].size() > cap)
                continue;
            prog.op_micro[i] = 1;
            prog.gemm_micro[op.index] = 1;
            avail[g.c] = 1;
            if (g.a != g.a_src) prog.op_micro[producer[g.a]] = 1;
            if (g.b != g.b_src) prog.op_micro[producer[g.b]] = 1;
            prog.tensors[g.c].offset = arena.end + extra;
            extra += (prog.tensors[g.c].size() + 31) & ~int64_t(31);
        }
        prog.tensor_elems = arena.end + extra;
    }
    // Scratch of the GEMM steps that run split over k (steps run one after
    // another, so the largest one).
    prog.ksplit_elems = 0;
    for (size_t i = 0; i < prog.gemms.size(); ++i) {
        const GemmOp &g = prog.gemms[i];
        const int64_t p = gemm_kparts(g.nb, g.m, g.n, g.k);
        if (!prog.gemm_micro[i] && p > 1) prog.ksplit_elems = std::max(prog.ksplit_elems, p * g.nb * g.m * g.n);
    }

    // Fused form: GEMM steps read their operands as produced (no transposes)
    // and run level by level (a step's level is one more than its operands'),
    // all steps of a level at once.  Offsets come from a separate arena sized
    // for LDS, filled in level order: the outputs of level l are placed
    // first, and only then are the operands read at level l released, so a
    // slot is reused only by a later level.
    {
        const int ng = (int)prog.gemms.size();
        std::vector<int> level(nt, 0);
        int n_levels = 0;
        for (const GemmOp &g : prog.gemms) {
            level[g.c] = 1 + std::max(level[g.a_src], level[g.b_src]);
            n_levels = std::max(n_levels, level[g.c]);
        }
        prog.lds_offset.assign(nt, -1);
        Arena la;
        la.granule = 2;
        for (int t = 0; t < L; ++t) prog.lds_offset[t] = la.alloc(prog.tensors[t].size());
        for (int lv = 1; lv <= n_levels; ++lv) {
            for (int i = 0; i < ng; ++i) {
                const int c = prog.gemms[i].c;
                if (level[c] == lv) prog.lds_offset[c] = la.alloc(prog.tensors[c].size());
            }
            for (int i = 0; i < ng; ++i) {
                const GemmOp &g = prog.gemms[i];
                if (level[g.c] != lv) continue;
                la.release(prog.lds_offset[g.a_src], prog.tensors[g.a_src].size());
                la.release(prog.lds_offset[g.b_src], prog.tensors[g.b_src].size());
            }
        }
        prog.lds_elems = la.end;
    }
    return true;
}

Program *get_program(qc_plan *plan, int b, int m, std::string &err) {
    std::lock_guard<std::mutex> lk(plan->mu);
    auto key = std::make_pair(b, m);
    auto it = plan->programs.find(key);
    if (it != plan->programs.end()) return it->second.get();
    auto prog = std::make_unique<Program>();
    if (!lower(plan, b, m, *prog, err)) return nullptr;
    Program *raw = prog.get();
    plan->programs[key] = std::move(prog);
    return raw;
}

static void json_ints(std::ostringstream &o, const std::vector<int> &v) {
    o << '[';
    for (size_t i = 0; i < v.size(); ++i) o << (i ? "," : "") << v[i];
    o << ']';
}

std::string describe_program(const qc_plan *plan, const Program &prog) {
    const Network &net = plan->net;
    std::ostringstream o;
    o.precision(17);
    o << "{\"b\":" << prog.b << ",\"m\":" << prog.m << ",\"bs_base\":" << kBsBase;
    o << ",\"n_graphs\":" << prog.graphs.size();
    o << ",\"n_qubits\":" << net.n_qubits;
    o << ",\"segments\":[";
    for (int e = 0; e < net.n_index(); ++e)
        o << (e ? "," : "") << '[' << net.seg_q[e] << ',' << net.seg_ord[e] << ',' << net.out_qubit[e] << ']';
    o << "],\"sliced\":";
    json_ints(o, plan->sliced);
    o << ",\"open_qubits\":";
    json_ints(o, plan->open_qubits);
    o << ",\"leaves\":[";
    for (size_t t = 0; t < net.leaves.size(); ++t) {
        const Tensor &T = net.leaves[t];
        o << (t ? "," : "") << "{\"idx\":";
        json_ints(o, T.idx);
        o << ",\"re\":[";
        for (size_t i = 0; i < T.data.size(); ++i) o << (i ? "," : "") << T.data[i].real();
        o << "],\"im\":[";
        for (size_t i = 0; i < T.data.size(); ++i) o << (i ? "," : "") << T.data[i].imag();
        o << "],\"tensor\":" << prog.leaves[t].tensor << '}';
    }
    o << "],\"tensors\":[";
    for (size_t t = 0; t < prog.tensors.size(); ++t) {
        o << (t ? "," : "") << "{\"layout\":";
        json_ints(o, prog.tensors[t].layout);
        o << ",\"offset\":" << prog.tensors[t].offset;
        if (t < prog.lds_offset.size()) o << ",\"lds\":" << prog.lds_offset[t];
        o << '}';
    }
    o << "],\"ops\":[";
    for (size_t i = 0; i < prog.ops.size(); ++i) {
        const Op &op = prog.ops[i];
        o << (i ? "," : "");
        if (op.kind == Op::TRANSPOSE) {
            const TransposeOp &t = prog.transposes[op.index];
            o << "{\"op\":\"transpose\",\"src\":" << t.src << ",\"dst\":" << t.dst
              << ",\"micro\":" << int(prog.op_micro.empty() ? 0 : prog.op_micro[i]) << '}';
        } else {
            const GemmOp &g = prog.gemms[op.index];
            o << "{\"op\":\"gemm\",\"a\":" << g.a << ",\"b\":" << g.b << ",\"a_src\":" << g.a_src
              << ",\"b_src\":" << g.b_src << ",\"c\":" << g.c << ",\"c_nat\":" << g.c_nat << ",\"nb\":" << g.nb
              << ",\"m\":" << g.m << ",\"n\":" << g.n << ",\"k\":" << g.k << ",\"a_km\":" << (g.a_km ? 1 : 0)
              << ",\"b_nk\":" << (g.b_nk ? 1 : 0) << ",\"micro\":" << int(prog.op_micro.empty() ? 0 : prog.op_micro[i])
              << '}';
        }
    }
    o << "],\"fused_pairs\":" << prog.fused_pairs << ",\"fused_waves\":" << prog.fused_waves << ",\"fused_slice_bits\":" << plan->fused_b
      << ",\"fused_shape_set\":[" << plan->fused_force_pairs << ',' << plan->fused_force_waves << ']'
      << ",\"fused_tuning\":[";
    for (size_t i = 0; i < prog.fused_tuning.size(); ++i)
        o << (i ? "," : "") << '[' << prog.fused_tuning[i][0] << ',' << prog.fused_tuning[i][1] << ','
          << prog.fused_tuning[i][2] << ']';
    o << "],\"root\":" << prog.root << ",\"tensor_elems\":" << prog.tensor_elems << ",\"lds_elems\":" << prog.lds_elems
      << ",\"flops\":" << prog.flops
      << ",\"bytes\":" << prog.bytes << ",\"transpose_bytes\":" << prog.transpose_bytes << '}';
    return o.str();
}

}  // namespace qc
