// C ABI: plan construction and inspection (host only).  The device entry
// points (qc_workspace_bytes, qc_contract_slices, qc_amplitude) live in
// runtime.hip.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>

#include "plan.h"

namespace qc {
bool search_plan(qc_plan *plan, const qc_slice_spec *spec, std::string &err);

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }
}  // namespace qc

using qc::set_error;

extern "C" const char *qc_last_error(void) { return qc::g_last_error.c_str(); }

extern "C" qc_status qc_plan_build(const qc_circuit *circuit, const uint8_t *bitstring,
                                   const qc_slice_spec *spec, qc_plan **out) {
    return qc_plan_build_open(circuit, bitstring, spec, 0, nullptr, out);
}

extern "C" qc_status qc_plan_build_open(const qc_circuit *circuit, const uint8_t *bitstring,
                                        const qc_slice_spec *spec, int32_t n_open, const int32_t *open_qubits,
                                        qc_plan **out) {
    if (!circuit || !out) { set_error("qc_plan_build: NULL argument"); return QC_ERR_INVALID_ARG; }
    if (n_open < 0 || n_open > QC_MAX_OPEN_QUBITS || (n_open > 0 && !open_qubits)) {
        set_error("qc_plan_build: n_open must be in [0, " + std::to_string(QC_MAX_OPEN_QUBITS) + "]");
        return QC_ERR_INVALID_ARG;
    }
    std::vector<int> open(open_qubits, open_qubits + n_open);
    std::sort(open.begin(), open.end());
    for (size_t i = 0; i < open.size(); ++i)
        if (open[i] < 0 || open[i] >= circuit->n_qubits || (i > 0 && open[i] == open[i - 1])) {
            set_error("qc_plan_build: open qubits must be distinct qubits of the circuit");
            return QC_ERR_INVALID_ARG;
        }
    if (circuit->n_qubits < 1 || circuit->n_qubits > 4096 || circuit->n_gates < 0 ||
        (circuit->n_gates > 0 && !circuit->gates)) {
        set_error("qc_plan_build: invalid circuit");
        return QC_ERR_INVALID_ARG;
    }
    if (spec && (spec->log2_slices < -1 || spec->log2_slices > 62 || spec->n_explicit < 0 ||
                 (spec->n_explicit > 0 && !spec->explicit_segments) || spec->greedy_trials < 0)) {
        set_error("qc_plan_build: invalid slice spec");
        return QC_ERR_INVALID_ARG;
    }
    if (bitstring)
        for (int q = 0; q < circuit->n_qubits; ++q)
            if (bitstring[q] > 1) { set_error("qc_plan_build: bitstring entries must be 0 or 1"); return QC_ERR_INVALID_ARG; }
    const auto t0 = std::chrono::steady_clock::now();
    qc_plan *plan = new (std::nothrow) qc_plan();
    if (!plan) { set_error("qc_plan_build: out of host memory"); return QC_ERR_NOMEM; }
    std::string err;
    try {
        plan->open_qubits = open;
        if (!qc::build_network(*circuit, open, plan->net, err)) {
            delete plan;
            set_error("qc_plan_build: " + err);
            return QC_ERR_INVALID_ARG;
        }
        std::vector<int> keep;
        if (spec)
            for (int i = 0; i < spec->n_explicit; ++i) {
                const int e = plan->net.find_segment(spec->explicit_segments[2 * i], spec->explicit_segments[2 * i + 1]);
                if (e >= 0) keep.push_back(e);
            }
        qc::simplify_network(plan->net, keep);
        plan->prob.n_index = plan->net.n_index();
        for (const auto &T : plan->net.leaves) {
            std::vector<int> s;
            for (int e : T.idx)
                if (!plan->net.fixed_out(e)) s.push_back(e);
            plan->prob.leaf_idx.push_back(s);
        }
        if (!open.empty()) plan->prob.keep = plan->net.open_out;
        if (!qc::search_plan(plan, spec, err)) {
            delete plan;
            set_error("qc_plan_build: " + err);
            return QC_ERR_INFEASIBLE;
        }
    } catch (const std::bad_alloc &) {
        delete plan;
        set_error("qc_plan_build: out of host memory");
        return QC_ERR_NOMEM;
    }
    if (bitstring) plan->default_bitstring.assign(bitstring, bitstring + circuit->n_qubits);
    int n_sum = 0;
    for (int e = 0; e < plan->net.n_index(); ++e) {
        if (plan->prob.kept(e)) continue;
        bool used = false;
        for (const auto &li : plan->prob.leaf_idx)
            for (int f : li) used |= f == e;
        n_sum += used;
    }
    plan->info.n_qubits = circuit->n_qubits;
    plan->info.n_open = (int32_t)open.size();
    plan->info.n_indices = n_sum;
    plan->info.n_leaves = (int)plan->net.leaves.size();
    plan->info.n_steps = (int)plan->tree.size();
    plan->info.plan_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = plan;
    return QC_OK;
}

extern "C" qc_status qc_plan_info(const qc_plan *plan, qc_plan_info_t *info) {
    if (!plan || !info) { set_error("qc_plan_info: NULL argument"); return QC_ERR_INVALID_ARG; }
    *info = plan->info;
    return QC_OK;
}

extern "C" qc_status qc_plan_sliced_segments(const qc_plan *plan, int32_t *out_pairs) {
    if (!plan || (!out_pairs && !plan->sliced.empty())) { set_error("qc_plan_sliced_segments: NULL argument"); return QC_ERR_INVALID_ARG; }
    for (size_t j = 0; j < plan->sliced.size(); ++j) {
        out_pairs[2 * j] = plan->net.seg_q[plan->sliced[j]];
        out_pairs[2 * j + 1] = plan->net.seg_ord[plan->sliced[j]];
    }
    return QC_OK;
}

extern "C" qc_status qc_plan_slice_assignment(const qc_plan *plan, uint64_t s, uint8_t *out) {
    if (!plan || (!out && !plan->sliced.empty())) { set_error("qc_plan_slice_assignment: NULL argument"); return QC_ERR_INVALID_ARG; }
    const int k = (int)plan->sliced.size();
    if (k < 64 && s >= (uint64_t(1) << k)) { set_error("qc_plan_slice_assignment: slice id out of range"); return QC_ERR_RANGE; }
    for (int j = 0; j < k; ++j) out[j] = (uint8_t)((s >> j) & 1);
    return QC_OK;
}

extern "C" qc_status qc_plan_describe(qc_plan *plan, int32_t log2_batch_slices, int32_t log2_batch_bs,
                                      qc_precision prec, char *buf, size_t cap, size_t *len) {
    if (!plan || !len) { set_error("qc_plan_describe: NULL argument"); return QC_ERR_INVALID_ARG; }
    if (prec != QC_C64 && prec != QC_SPLIT_BF16 && prec != QC_SPLIT_FP16) { set_error("qc_plan_describe: bad precision"); return QC_ERR_INVALID_ARG; }
    std::string err;
    qc::Program *prog = qc::get_program(plan, log2_batch_slices, log2_batch_bs, err);
    if (!prog) { set_error("qc_plan_describe: " + err); return QC_ERR_RANGE; }
    const std::string s = qc::describe_program(plan, *prog);
    *len = s.size();
    if (buf && cap > 0) {
        const size_t n = std::min(cap - 1, s.size());
        std::memcpy(buf, s.data(), n);
        buf[n] = 0;
    }
    return QC_OK;
}

extern "C" qc_status qc_plan_export_steps(qc_plan *plan, int32_t log2_batch_slices, int32_t log2_batch_bs,
                                          qc_step_t *out, int32_t cap, int32_t *n) {
    if (!plan || !n || cap < 0 || (cap > 0 && !out)) {
        set_error("qc_plan_export_steps: invalid argument");
        return QC_ERR_INVALID_ARG;
    }
    std::string err;
    qc::Program *prog = qc::get_program(plan, log2_batch_slices, log2_batch_bs, err);
    if (!prog) { set_error("qc_plan_export_steps: " + err); return QC_ERR_RANGE; }
    *n = (int32_t)prog->ops.size();
    for (int32_t i = 0; i < std::min<int32_t>(cap, *n); ++i) {
        const qc::Op &op = prog->ops[i];
        qc_step_t r{};
        if (op.kind == qc::Op::TRANSPOSE) {
            const qc::TransposeOp &t = prog->transposes[op.index];
            r.kind = 0;
            r.a = t.src;
            r.b = -1;
            r.c = t.dst;
            r.m = prog->tensors[t.src].size();
        } else {
            const qc::GemmOp &g = prog->gemms[op.index];
            r.kind = 1;
            r.a = g.a;
            r.b = g.b;
            r.c = g.c;
            r.nb = g.nb; r.m = g.m; r.n = g.n; r.k = g.k;
            r.a_km = g.a_km;
            r.b_nk = g.b_nk;
            r.flops = 8.0 * double(g.nb) * double(g.m) * double(g.n) * double(g.k);
        }
        r.micro = prog->op_micro.empty() ? 0 : prog->op_micro[i];
        out[i] = r;
    }
    return QC_OK;
}

extern "C" qc_status qc_plan_export_tree(const qc_plan *plan, int32_t *n_leaves, int32_t *n_tensors,
                                         int32_t *origin_offsets, int32_t *origin_ids, int32_t *merges) {
    if (!plan || !n_leaves || !n_tensors) { set_error("qc_plan_export_tree: NULL argument"); return QC_ERR_INVALID_ARG; }
    const int L = (int)plan->origin_full.size();
    *n_leaves = L;
    *n_tensors = plan->net.n_orig;
    if (origin_offsets && origin_ids) {
        int32_t off = 0;
        for (int t = 0; t < L; ++t) {
            origin_offsets[t] = off;
            for (int g : plan->origin_full[t]) origin_ids[off++] = g;
        }
        origin_offsets[L] = off;
    }
    if (merges)
        for (size_t i = 0; i < plan->tree_full.size(); ++i) {
            merges[2 * i] = plan->tree_full[i].a;
            merges[2 * i + 1] = plan->tree_full[i].b;
        }
    return QC_OK;
}

extern "C" qc_status qc_plan_set_exec(qc_plan *plan, int32_t mode) {
    if (!plan || mode < QC_EXEC_AUTO || mode > QC_EXEC_STEPWISE) {
        set_error("qc_plan_set_exec: invalid argument");
        return QC_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(plan->mu);
    plan->exec_mode = mode;
    return QC_OK;
}

extern "C" void qc_plan_destroy(qc_plan *plan);
