// Device side of the C ABI: program constants, workspace layout and the
// chunk loop of qc_contract_slices (leaves -> steps -> FP64 reduction).
#include <hip/hip_runtime.h>

#include <algorithm>
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

struct WsLayout {
    size_t bits_off, bits_bytes, tensor_off, total;
};

WsLayout ws_layout(const Program &prog, int n_qubits) {
    WsLayout w;
    w.bits_off = 0;
    w.bits_bytes = align256(size_t(n_qubits) << prog.m);
    w.tensor_off = w.bits_bytes;
    w.total = w.tensor_off + align256(size_t(prog.tensor_elems) * sizeof(float2));
    return w;
}

#define QC_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            err = std::string(#call) + ": " + hipGetErrorString(e_);                  \
            return false;                                                             \
        }                                                                             \
    } while (0)

// Uploads the program's leaf table and base values to the current device.
bool ensure_device(const qc_plan *plan, Program &prog, std::string &err) {
    int dev = 0;
    QC_HIP(hipGetDevice(&dev));
    if (prog.d_leaf_desc) {
        if (prog.device != dev) { err = "plan was first used on another device"; return false; }
        return true;
    }
    const Network &net = plan->net;
    std::vector<char> fixed(net.n_index(), 0);
    std::vector<int> slice_bit(net.n_index(), -1);
    for (size_t j = 0; j < plan->sliced.size(); ++j) {
        slice_bit[plan->sliced[j]] = (int)j;
        if ((int)j >= prog.b) fixed[plan->sliced[j]] = 1;
    }
    std::vector<LeafDesc> descs;
    std::vector<int32_t> block_leaf;
    std::vector<double2> base;
    for (size_t li = 0; li < prog.leaves.size(); ++li) {
        const Tensor &T = net.leaves[prog.leaves[li].leaf];
        const ProgTensor &pt = prog.tensors[prog.leaves[li].tensor];
        LeafDesc d;
        std::memset(&d, 0, sizeof(d));
        const int rb = (int)T.idx.size();
        const int ro = (int)pt.layout.size();
        if (rb > kLeafMaxBase || ro > kLeafMaxRank) { err = "leaf too large for the device table"; return false; }
        d.out_off = pt.offset;
        d.base_off = (int32_t)base.size();
        d.r_out = ro;
        auto base_pos = [&](int e) {
            for (int j = 0; j < rb; ++j)
                if (T.idx[j] == e) return rb - 1 - j;
            return -1;
        };
        for (int p = 0; p < ro; ++p) {
            const int e = pt.layout[ro - 1 - p];
            if (e >= kBsBase) d.src[p] = (int8_t)(64 + (e - kBsBase));
            else d.src[p] = (int8_t)base_pos(e);
        }
        for (int j = 0; j < rb; ++j) {
            const int e = T.idx[j];
            if (net.out_qubit[e] >= 0) {
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
        d.pad0 = (int32_t)block_leaf.size();
        const int64_t nblk = ((int64_t(1) << ro) + 255) / 256;
        for (int64_t b = 0; b < nblk; ++b) block_leaf.push_back((int32_t)li);
        descs.push_back(d);
    }
    void *a = nullptr, *b = nullptr, *c = nullptr;
    QC_HIP(hipMalloc(&a, std::max<size_t>(1, descs.size() * sizeof(LeafDesc))));
    if (hipMalloc(&b, std::max<size_t>(1, block_leaf.size() * sizeof(int32_t))) != hipSuccess ||
        hipMalloc(&c, std::max<size_t>(1, base.size() * sizeof(double2))) != hipSuccess) {
        hipFree(a);
        if (b) hipFree(b);
        err = "hipMalloc of program constants failed";
        return false;
    }
    if (hipMemcpy(a, descs.data(), descs.size() * sizeof(LeafDesc), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b, block_leaf.data(), block_leaf.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c, base.data(), base.size() * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(a); hipFree(b); hipFree(c);
        err = "upload of program constants failed";
        return false;
    }
    prog.d_leaf_desc = a;
    prog.d_leaf_block = b;
    prog.d_base = c;
    prog.n_leaf_blocks = (int)block_leaf.size();
    prog.device = dev;
    return true;
}

// perm[p] = output bit position of input bit p.
TransposeDesc make_transpose_desc(const float2 *in, float2 *out, int r, const std::vector<int> &perm) {
    TransposeDesc d;
    std::memset(&d, 0, sizeof(d));
    d.in = in;
    d.out = out;
    const int a = std::min(r, 5), c = std::min(r, 5);
    std::vector<int> tile, rest;  // input bit positions
    for (int p = 0; p < r; ++p) {
        if (r <= kTransMaxTile || p < a || perm[p] < c) tile.push_back(p);
        else rest.push_back(p);
    }
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

GemmDesc make_gemm(const Program &prog, const GemmOp &g, float2 *tensors) {
    GemmDesc d;
    d.A = tensors + prog.tensors[g.a].offset;
    d.B = tensors + prog.tensors[g.b].offset;
    d.C = tensors + prog.tensors[g.c].offset;
    d.nb = g.nb; d.m = g.m; d.n = g.n; d.k = g.k;
    d.sAb = g.m * g.k;
    if (g.a_km) { d.sAk = g.m; d.sAm = 1; } else { d.sAm = g.k; d.sAk = 1; }
    d.sBb = g.k * g.n;
    if (g.b_nk) { d.sBn = g.k; d.sBk = 1; } else { d.sBk = g.n; d.sBn = 1; }
    d.sCb = g.m * g.n; d.sCm = g.n; d.sCn = 1;
    return d;
}

}  // namespace

void free_program_device(Program &prog) {
    if (!prog.d_leaf_desc) return;
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(prog.device);
    hipFree(prog.d_leaf_desc);
    hipFree(prog.d_leaf_block);
    hipFree(prog.d_base);
    hipSetDevice(cur);
    prog.d_leaf_desc = prog.d_leaf_block = prog.d_base = nullptr;
}

static bool enqueue(qc_plan *plan, Program &prog, uint64_t s_begin, uint64_t s_end, const uint8_t *bits_host,
                    int n_bs, void *ws, size_t ws_bytes, hipStream_t st, double *out_dev, double *per_slice_dev,
                    std::string &err) {
    if (!ensure_device(plan, prog, err)) return false;
    const int nq = plan->net.n_qubits;
    const WsLayout w = ws_layout(prog, nq);
    if (w.total > ws_bytes) { err = "workspace too small"; return false; }
    uint8_t *bits = (uint8_t *)ws + w.bits_off;
    float2 *tensors = (float2 *)((char *)ws + w.tensor_off);
    const size_t used = size_t(n_bs) * nq;
    QC_HIP(hipMemcpyAsync(bits, bits_host, used, hipMemcpyHostToDevice, st));
    if ((size_t(nq) << prog.m) > used)
        QC_HIP(hipMemsetAsync(bits + used, 0, (size_t(nq) << prog.m) - used, st));
    const uint64_t chunk = uint64_t(1) << prog.b;
    for (uint64_t cb = s_begin & ~(chunk - 1); cb < s_end; cb += chunk) {
        launch_leaves((const LeafDesc *)prog.d_leaf_desc, (const int32_t *)prog.d_leaf_block, prog.n_leaf_blocks,
                      (const double2 *)prog.d_base, tensors, bits, nq, cb, st);
        for (const Op &op : prog.ops) {
            if (op.kind == Op::TRANSPOSE) launch_transpose(make_transpose(prog, prog.transposes[op.index], tensors), st);
            else launch_gemm(make_gemm(prog, prog.gemms[op.index], tensors), st);
        }
        launch_reduce(tensors + prog.tensors[prog.root].offset, prog.b, prog.m, n_bs, cb, s_begin, s_end, out_dev,
                      per_slice_dev, st);
        QC_HIP(hipGetLastError());
    }
    return true;
}

}  // namespace qc

static bool check_bitstrings(const qc_plan *plan, const uint8_t *bits, int n_bs) {
    const int nq = plan->net.n_qubits;
    for (int64_t i = 0; i < int64_t(n_bs) * nq; ++i)
        if (bits[i] > 1) return false;
    return true;
}

extern "C" size_t qc_workspace_bytes(qc_plan *plan, int64_t chunk_slices, int32_t n_bs, qc_precision prec) {
    if (!plan || chunk_slices < 1 || n_bs < 1 || n_bs > (1 << qc::kMaxBsBits) ||
        (prec != QC_C64 && prec != QC_SPLIT_BF16 && prec != QC_SPLIT_FP16)) {
        set_error("qc_workspace_bytes: invalid argument");
        return 0;
    }
    const int b = qc::ceil_log2(chunk_slices);
    if (b > (int)plan->sliced.size()) { set_error("qc_workspace_bytes: more slices than the plan has"); return 0; }
    std::string err;
    qc::Program *prog = qc::get_program(plan, b, qc::ceil_log2(n_bs), err);
    if (!prog) { set_error("qc_workspace_bytes: " + err); return 0; }
    return qc::ws_layout(*prog, plan->net.n_qubits).total;
}

extern "C" qc_status qc_contract_slices(qc_plan *plan, uint64_t s_begin, uint64_t s_end, const uint8_t *bitstrings,
                                        int32_t n_bs, qc_precision prec, void *ws, size_t ws_bytes, void *stream,
                                        double *out_dev, double *per_slice_dev) {
    if (!plan || !bitstrings || !ws || !out_dev) { set_error("qc_contract_slices: NULL argument"); return QC_ERR_INVALID_ARG; }
    if (prec != QC_C64 && prec != QC_SPLIT_BF16 && prec != QC_SPLIT_FP16) {
        set_error("qc_contract_slices: invalid precision");
        return QC_ERR_INVALID_ARG;
    }
    if (prec != QC_C64) { set_error("qc_contract_slices: split precision is not built yet"); return QC_ERR_UNSUPPORTED; }
    if (n_bs < 1 || n_bs > (1 << qc::kMaxBsBits)) { set_error("qc_contract_slices: n_bs out of range"); return QC_ERR_RANGE; }
    const int k = (int)plan->sliced.size();
    const uint64_t n_slices = k >= 64 ? ~uint64_t(0) : (uint64_t(1) << k);
    if (s_begin > s_end || s_end > n_slices) { set_error("qc_contract_slices: slice range out of bounds"); return QC_ERR_RANGE; }
    if (!check_bitstrings(plan, bitstrings, n_bs)) { set_error("qc_contract_slices: bitstring entries must be 0 or 1"); return QC_ERR_INVALID_ARG; }
    if (s_begin == s_end) return QC_OK;
    const int m = qc::ceil_log2(n_bs);
    std::string err;
    qc::Program *prog = nullptr;
    for (int b = std::min(k, qc::ceil_log2((int64_t)(s_end - s_begin))); b >= 0; --b) {
        qc::Program *p = qc::get_program(plan, b, m, err);
        if (!p) { set_error("qc_contract_slices: " + err); return QC_ERR_UNSUPPORTED; }
        if (qc::ws_layout(*p, plan->net.n_qubits).total <= ws_bytes) { prog = p; break; }
    }
    if (!prog) { set_error("qc_contract_slices: workspace too small for one slice"); return QC_ERR_NOMEM; }
    if (!qc::enqueue(plan, *prog, s_begin, s_end, bitstrings, n_bs, ws, ws_bytes, (hipStream_t)stream, out_dev,
                     per_slice_dev, err)) {
        set_error("qc_contract_slices: " + err);
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
    if (b < 0) b = 0;
    need = qc_workspace_bytes(plan, int64_t(1) << b, 1, prec);
    void *ws = nullptr, *out = nullptr;
    if (hipMalloc(&ws, need) != hipSuccess) { set_error("qc_amplitude: workspace allocation failed"); return QC_ERR_NOMEM; }
    if (hipMalloc(&out, 2 * sizeof(double)) != hipSuccess) { hipFree(ws); set_error("qc_amplitude: allocation failed"); return QC_ERR_NOMEM; }
    qc_status st = QC_OK;
    double res[2] = {0, 0};
    if (hipMemset(out, 0, 2 * sizeof(double)) != hipSuccess) st = QC_ERR_DEVICE;
    if (st == QC_OK) {
        const uint64_t n_slices = uint64_t(1) << k;
        st = qc_contract_slices(plan, 0, n_slices, bits, 1, prec, ws, need, nullptr, (double *)out, nullptr);
    }
    if (st == QC_OK) {
        if (hipDeviceSynchronize() != hipSuccess ||
            hipMemcpy(res, out, sizeof(res), hipMemcpyDeviceToHost) != hipSuccess) {
            set_error(std::string("qc_amplitude: ") + hipGetErrorString(hipGetLastError()));
            st = QC_ERR_DEVICE;
        }
    }
    hipFree(ws);
    hipFree(out);
    if (st == QC_OK) { out_host[0] = res[0]; out_host[1] = res[1]; }
    return st;
}

extern "C" void qc_plan_destroy(qc_plan *plan) {
    if (!plan) return;
    for (auto &kv : plan->programs) qc::free_program_device(*kv.second);
    delete plan;
}

extern "C" qc_status qc_kernel_gemm(const void *A, const void *B, void *C, int64_t nb, int64_t m, int64_t n, int64_t k,
                                    int32_t a_km, int32_t b_nk, qc_precision prec, void *stream) {
    if (!A || !B || !C || nb < 1 || m < 1 || n < 1 || k < 1) { set_error("qc_kernel_gemm: invalid argument"); return QC_ERR_INVALID_ARG; }
    if (prec != QC_C64) { set_error("qc_kernel_gemm: split precision is not built yet"); return QC_ERR_UNSUPPORTED; }
    qc::GemmDesc d;
    d.A = (const float2 *)A; d.B = (const float2 *)B; d.C = (float2 *)C;
    d.nb = nb; d.m = m; d.n = n; d.k = k;
    d.sAb = m * k;
    if (a_km) { d.sAk = m; d.sAm = 1; } else { d.sAm = k; d.sAk = 1; }
    d.sBb = k * n;
    if (b_nk) { d.sBn = k; d.sBk = 1; } else { d.sBk = n; d.sBn = 1; }
    d.sCb = m * n; d.sCm = n; d.sCn = 1;
    qc::launch_gemm(d, (hipStream_t)stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error(std::string("qc_kernel_gemm: ") + hipGetErrorString(e)); return QC_ERR_DEVICE; }
    return QC_OK;
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
