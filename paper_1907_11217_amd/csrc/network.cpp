// Circuit -> hypergraph tensor network, and its simplification.
//
// Each qubit's wire is cut at every non-diagonal gate (H, sqrt X, sqrt Y);
// each piece (segment) is one binary running index.  A non-diagonal gate is
// the 2x2 tensor U[new segment][old segment]; a T is the vector (1, e^{i pi/4})
// on the segment it acts on, and a CZ the 2x2 tensor [[1, 1], [1, -1]] on its
// two qubits' current segments -- diagonal gates add no index, which is what
// makes the running indices hyper-edges (the paper's refactored network:
// nodes hold tensors, hyper-edges are running indices).  The input segment of
// every qubit carries the vector e_0 = (1, 0); the output segment is left as
// an index, fixed to x[q] when the leaves are instantiated for a bitstring --
// or, for the qubits the caller leaves open, kept as an index of the result,
// so that one contraction gives the amplitudes of all 2^m settings of them.
#include <algorithm>
#include <cmath>
#include <set>

#include "plan.h"

namespace qc {

int Network::find_segment(int q, int ord) const {
    for (int i = 0; i < n_index(); ++i)
        if (seg_q[i] == q && seg_ord[i] == ord) return i;
    return -1;
}

static void gate_2x2(int kind, cplx u[2][2]) {
    const double r = 1.0 / std::sqrt(2.0);
    const cplx h(0.5, 0.5);      // (1 + i) / 2
    const cplx hc(0.5, -0.5);    // (1 - i) / 2
    switch (kind) {
    case QC_GATE_H: u[0][0] = r; u[0][1] = r; u[1][0] = r; u[1][1] = -r; break;
    case QC_GATE_SQRT_X: u[0][0] = h; u[0][1] = hc; u[1][0] = hc; u[1][1] = h; break;
    case QC_GATE_SQRT_Y: u[0][0] = h; u[0][1] = -h; u[1][0] = h; u[1][1] = h; break;
    default: u[0][0] = 1; u[0][1] = 0; u[1][0] = 0; u[1][1] = std::polar(1.0, M_PI / 4); break;
    }
}

bool build_network(const qc_circuit &c, const std::vector<int> &open, Network &net, std::string &err) {
    const int n = c.n_qubits;
    net = Network();
    net.n_qubits = n;
    net.n_cut.assign(n, 0);
    std::vector<int> cur(n);
    auto new_index = [&](int q, int ord) {
        net.seg_q.push_back(q);
        net.seg_ord.push_back(ord);
        net.out_qubit.push_back(-1);
        net.open_out.push_back(0);
        return (int)net.seg_q.size() - 1;
    };
    for (int q = 0; q < n; ++q) {
        cur[q] = new_index(q, 0);
        net.leaves.push_back(Tensor{{cur[q]}, {cplx(1), cplx(0)}});
        net.origin.push_back({q});
    }
    for (int g = 0; g < c.n_gates; ++g) {
        const qc_gate &gt = c.gates[g];
        if (gt.q0 < 0 || gt.q0 >= n) { err = "gate " + std::to_string(g) + ": qubit out of range"; return false; }
        switch (gt.kind) {
        case QC_GATE_H: case QC_GATE_SQRT_X: case QC_GATE_SQRT_Y: {
            cplx u[2][2];
            gate_2x2(gt.kind, u);
            const int old = cur[gt.q0];
            const int nw = new_index(gt.q0, ++net.n_cut[gt.q0]);
            cur[gt.q0] = nw;
            net.leaves.push_back(Tensor{{nw, old}, {u[0][0], u[0][1], u[1][0], u[1][1]}});
            break;
        }
        case QC_GATE_T: {
            cplx u[2][2];
            gate_2x2(QC_GATE_T, u);
            net.leaves.push_back(Tensor{{cur[gt.q0]}, {u[0][0], u[1][1]}});
            break;
        }
        case QC_GATE_CZ:
            if (gt.q1 < 0 || gt.q1 >= n || gt.q1 == gt.q0) {
                err = "gate " + std::to_string(g) + ": bad CZ qubits";
                return false;
            }
            net.leaves.push_back(Tensor{{cur[gt.q0], cur[gt.q1]}, {cplx(1), cplx(1), cplx(1), cplx(-1)}});
            break;
        default:
            err = "gate " + std::to_string(g) + ": unknown kind " + std::to_string(gt.kind);
            return false;
        }
        net.origin.push_back({n + g});
    }
    net.n_orig = n + c.n_gates;
    for (int q = 0; q < n; ++q) net.out_qubit[cur[q]] = q;
    for (int q : open) {
        if (q < 0 || q >= n) { err = "open output qubit out of range"; return false; }
        net.open_out[cur[q]] = 1;
    }
    return true;
}

// C = sum over `contracted` of A * B, with C's indices in the order given.
Tensor contract_host(const Tensor &A, const Tensor &B, const std::vector<int> &c_idx,
                            const std::vector<int> &contracted) {
    std::vector<int> all = c_idx;
    all.insert(all.end(), contracted.begin(), contracted.end());
    const int r = (int)all.size();
    auto pos_in = [&](const Tensor &T, int e) {
        for (size_t i = 0; i < T.idx.size(); ++i)
            if (T.idx[i] == e) return (int)(T.idx.size() - 1 - i);
        return -1;
    };
    std::vector<int> pa(r), pb(r);
    for (int i = 0; i < r; ++i) { pa[i] = pos_in(A, all[i]); pb[i] = pos_in(B, all[i]); }
    Tensor C;
    C.idx = c_idx;
    C.data.assign(size_t(1) << c_idx.size(), cplx(0));
    const int rc = (int)c_idx.size();
    for (uint64_t v = 0; v < (uint64_t(1) << r); ++v) {
        // bit of all[i] is bit (r - 1 - i) of v; C's offset is the top rc bits.
        uint64_t oa = 0, ob = 0;
        for (int i = 0; i < r; ++i) {
            const uint64_t bit = (v >> (r - 1 - i)) & 1;
            if (pa[i] >= 0) oa |= bit << pa[i];
            if (pb[i] >= 0) ob |= bit << pb[i];
        }
        C.data[v >> (r - rc)] += A.data[oa] * B.data[ob];
    }
    return C;
}

// Merge pairs of tensors that share an index whenever the result is no larger
// than the larger of the two (this absorbs vectors, collapses chains of 2x2
// tensors and folds tensors whose indices are a subset of a neighbour's).
// Output segments and the indices in `keep` (caller-chosen slices) are never
// summed here.  Sizes are counted without the fixed output segments, which
// are fixed per bitstring when leaves are instantiated (open ones count); a
// merged tensor keeps at most kMaxLeafBase indices in all.  Exact in FP64.
void simplify_network(Network &net, const std::vector<int> &keep) {
    auto eff = [&](const std::vector<int> &idx) {
        int r = 0;
        for (int f : idx) r += !net.fixed_out(f);
        return r;
    };
    std::vector<Tensor> &T = net.leaves;
    std::vector<char> alive(T.size(), 1);
    std::vector<std::set<int>> holders(net.n_index());
    for (size_t t = 0; t < T.size(); ++t)
        for (int e : T[t].idx) holders[e].insert((int)t);
    bool changed = true;
    while (changed) {
        changed = false;
        for (size_t a = 0; a < T.size(); ++a) {
            if (!alive[a]) continue;
            bool merged = false;
            for (int e : std::vector<int>(T[a].idx)) {
                for (int b : std::vector<int>(holders[e].begin(), holders[e].end())) {
                    if (b == (int)a || !alive[b]) continue;
                    std::vector<int> c_idx, contracted;
                    std::set<int> seen;
                    for (const Tensor *X : {&T[a], &T[b]})
                        for (int f : X->idx) {
                            if (!seen.insert(f).second) continue;
                            const bool in_a = std::count(T[a].idx.begin(), T[a].idx.end(), f) > 0;
                            const bool in_b = std::count(T[b].idx.begin(), T[b].idx.end(), f) > 0;
                            const bool closes = in_a && in_b && holders[f].size() == 2 && net.out_qubit[f] < 0 &&
                                                std::find(keep.begin(), keep.end(), f) == keep.end();
                            (closes ? contracted : c_idx).push_back(f);
                        }
                    if (eff(c_idx) > std::max(eff(T[a].idx), eff(T[b].idx)) || (int)c_idx.size() > kMaxLeafBase)
                        continue;
                    Tensor C = contract_host(T[a], T[b], c_idx, contracted);
                    for (int f : T[a].idx) holders[f].erase((int)a);
                    for (int f : T[b].idx) holders[f].erase(b);
                    alive[b] = 0;
                    T[a] = std::move(C);
                    net.origin[a].insert(net.origin[a].end(), net.origin[b].begin(), net.origin[b].end());
                    net.origin[b].clear();
                    for (int f : T[a].idx) holders[f].insert((int)a);
                    merged = changed = true;
                    break;
                }
                if (merged) break;
            }
            if (merged) --a;  // revisit the merged tensor
        }
    }
    std::vector<Tensor> out;
    std::vector<std::vector<int>> origin;
    for (size_t t = 0; t < T.size(); ++t)
        if (alive[t]) {
            out.push_back(std::move(T[t]));
            std::sort(net.origin[t].begin(), net.origin[t].end());
            origin.push_back(std::move(net.origin[t]));
        }
    T = std::move(out);
    net.origin = std::move(origin);
}

}  // namespace qc

extern "C" qc_status qc_gate_matrix(int32_t kind, double *out) {
    if (!out) { qc::set_error("qc_gate_matrix: out is NULL"); return QC_ERR_INVALID_ARG; }
    if (kind == QC_GATE_CZ) {
        for (int i = 0; i < 32; ++i) out[i] = 0;
        for (int d = 0; d < 4; ++d) out[2 * (5 * d)] = d == 3 ? -1.0 : 1.0;
        return QC_OK;
    }
    if (kind < QC_GATE_H || kind > QC_GATE_T) { qc::set_error("qc_gate_matrix: unknown kind"); return QC_ERR_INVALID_ARG; }
    qc::cplx u[2][2];
    qc::gate_2x2(kind, u);
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) { out[2 * (2 * i + j)] = u[i][j].real(); out[2 * (2 * i + j) + 1] = u[i][j].imag(); }
    return QC_OK;
}
