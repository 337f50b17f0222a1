// Host-side planner: circuit -> hypergraph tensor network -> simplified
// leaves -> greedy pairwise order -> sliced segments -> lowered programs.
//
// The network follows the paper's refactored form (Section "Benchmarking and
// the Experimental Setup"): each node holds a tensor and each hyper-edge is a
// running index.  Running indices are wire segments: a qubit's wire is cut at
// every non-diagonal gate, and diagonal gates (T, CZ) attach to the segment
// they act on, so one index can join many tensors.
#pragma once

#include <atomic>
#include <array>
#include <complex>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "qcsim.h"

namespace qc {

using cplx = std::complex<double>;

constexpr int kMaxRank = 40;       // largest tensor rank a program may hold
constexpr int kMaxLeafBase = 4;    // indices of a simplified leaf, output segments included
constexpr int kMaxBsBits = 16;     // bitstrings in flight <= 65536

// A tensor over binary indices; data is row-major with idx[0] the most
// significant bit of the flat offset.
struct Tensor {
    std::vector<int> idx;
    std::vector<cplx> data;
};

struct Network {
    int n_qubits = 0;
    std::vector<int> seg_q, seg_ord;    // per index: its segment (q, ordinal)
    std::vector<int> out_qubit;         // per index: q if it is q's output segment, else -1
    std::vector<char> open_out;         // per index: an output segment left open (never fixed or summed)
    std::vector<int> n_cut;             // per qubit: non-diagonal gate count
    std::vector<Tensor> leaves;         // simplified tensors
    // Per leaf: the circuit's tensors merged into it, numbered t < n_qubits for
    // qubit t's input state and n_qubits + g for gate g.
    std::vector<std::vector<int>> origin;
    int n_orig = 0;                     // n_qubits + number of gates
    int n_index() const { return (int)seg_q.size(); }
    int find_segment(int q, int ord) const;
    // An output segment fixed to the bitstring's bit (not an open one).
    bool fixed_out(int e) const { return out_qubit[e] >= 0 && !open_out[e]; }
};

// Builds the hypergraph network of <x|C|0^n> with output segments left as
// indices (fixed per bitstring at instantiation, except those of the qubits in
// `open`, which stay open to the end) and input segments fixed to 0.
bool build_network(const qc_circuit &c, const std::vector<int> &open, Network &net, std::string &err);
void simplify_network(Network &net, const std::vector<int> &keep);
// C = sum over `contracted` of A * B, with C's indices in the order c_idx (FP64, host).
Tensor contract_host(const Tensor &A, const Tensor &B, const std::vector<int> &c_idx,
                     const std::vector<int> &contracted);

// One pairwise merge: tensors a, b -> a new tensor (ids: leaves first, then
// merges in order).
struct Merge { int a, b; };

struct TreeCost {
    double max_log2 = 0;     // largest intermediate (log2 entries)
    double flops = 0;        // real flops (8 per complex MAC)
    double bytes = 0;        // complex64 operand bytes
    double peak_live = 0;    // peak live complex64 bytes (sequential execution)
};

// Index sets of all tree nodes given removed (sliced) indices; used by the
// order search and slicing.
struct OrderProblem {
    int n_index = 0;
    std::vector<std::vector<int>> leaf_idx;   // summed and open-output indices per leaf (not fixed outputs)
    std::vector<char> keep;                   // per index: never summed (open outputs); empty = none
    bool kept(int e) const { return !keep.empty() && keep[e]; }
    // Weight of an element moved against a complex multiply-add in the
    // search's step cost (see order.cpp).
    double move_per_mac = 20.0;
};

std::vector<Merge> greedy_order(const OrderProblem &p, const std::vector<char> &removed,
                                uint64_t seed, double temperature);
std::vector<Merge> greedy_order_phased(const OrderProblem &p, const std::vector<char> &removed, uint64_t seed,
                                       double temperature, const std::vector<char> *dynamic, int const_cap);
TreeCost tree_cost(const OrderProblem &p, const std::vector<Merge> &tree,
                   const std::vector<char> &removed);

// ------------------------------------------------------------ lowering
// Index ids inside a program: segment ids, then kBsBase + i for bitstring bit i.
constexpr int kBsBase = 1 << 20;
constexpr int kMicroMaxLog2 = 12;  // micro steps: output and operands of at most 2^12 entries
constexpr int kTransposeMinLog2 = 20;  // GEMM outputs from 2^20 entries may keep an explicit transpose
constexpr int kMinWriteRun = 2;        // ... when fewer natural lowest bits than this stay lowest

struct ProgTensor {
    std::vector<int> layout;   // major -> minor
    int64_t offset = 0;        // element offset in the tensor region of ws
    int64_t size() const { return int64_t(1) << layout.size(); }
};

struct LeafOp {
    int leaf;                  // network leaf id
    int tensor;                // program tensor id
};

struct TransposeOp {
    int src, dst;
};

// The number of k parts for a GEMM shape: large-tile shapes whose 128x128
// tiles number fewer than 1024 (four per compute unit) are split into up to
// 64 power-of-two parts, each of at least 256 k; other shapes with m and n
// multiples of 32 (the 32- and 64-wide MFMA forms) likewise while their
// 32x32 tiles number fewer than 4096; shapes with small output tiles (m n
// <= 256, the dot-tile form's) and k >= 1024 into the smallest power of two
// giving 1024 (batch, part) workgroups, each part keeping at least 256 k;
// other shapes of at most 4096 outputs with k >= 8192 (the dot form's) into
// the smallest power of two giving 1024 (output, part) workgroups, each part
// keeping at least 4096 k.
inline int64_t gemm_kparts(int64_t nb, int64_t m, int64_t n, int64_t k) {
    int64_t p = 1;
    if (m % 128 == 0 && n % 128 == 0) {
        const int64_t tiles = nb * (m / 128) * (n / 128);
        while (tiles * p < 1024 && p < 64 && k % (2 * p) == 0 && k / (2 * p) >= 256) p *= 2;
    } else if (m % 32 == 0 && n % 32 == 0) {
        const int64_t tiles = nb * (m / 32) * (n / 32);
        while (tiles * p < 4096 && p < 64 && k % (2 * p) == 0 && k / (2 * p) >= 256) p *= 2;
    } else if (m * n <= 256 && k >= 1024) {
        while (nb * p < 1024 && p < 1024 && k % (2 * p) == 0 && k / (2 * p) >= 256) p *= 2;
    } else if (nb * m * n <= 4096 && k >= 8192) {
        const int64_t outs = nb * m * n;
        while (outs * p < 1024 && k % (2 * p) == 0 && k / (2 * p) >= 4096) p *= 2;
    }
    return p;
}

struct GemmOp {
    int a_src, b_src;          // operand tensors as produced (before transposes)
    int a, b, c;               // program tensor ids after transposes
    int c_nat = -1;            // tensor holding C's natural [b][m][n] layout (c_nat != c: C is written scattered into c's layout)
    int64_t nb, m, n, k;       // C[b][m][n] = sum_k A . B
    bool a_km;                 // A stored [b][k][m] (else [b][m][k])
    bool b_nk;                 // B stored [b][n][k] (else [b][k][n])
    int cls_b, cls_m, cls_n, cls_k;  // log2 extents
    int variant[3] = {-1, -1, -1};   // GEMM kernel form per precision chosen by qc_tune (-1: default rules)
};

// Device constants of a lowered program, by id.
enum ConstId {
    kCLeafDesc,      // leaf descriptors (stepwise form)
    kCLeafBlock,     // leaf blocks (stepwise form)
    kCBase,          // leaf base values, complex double (both forms)
    kCMicro,         // micro-step table (stepwise form)
    kCMicroLevels,   // group and level starts of the micro-step table
    kCFusedImage,    // leaf values that do not depend on the (slice, bitstring) pair
    kCFusedElems,    // run-time leaf elements: LDS slot, base index, dynamic bits
    kCFusedPool,     // operand slots of items with more than four contracted values
    kCFusedItems,    // one item per output of every step, grouped by tree level
    kCFusedItems2,   // third and fourth operand slots of each item
    kCFusedLevels,   // item offsets of the levels
    kNumConst
};

struct DevConsts {
    void *p[kNumConst] = {};
};

struct Op {
    enum Kind { TRANSPOSE, GEMM } kind;
    int index;                 // into transposes / gemms
};

struct Program {
    int b = 0, m = 0;                     // log2 slices / bitstrings in flight
    std::vector<ProgTensor> tensors;
    std::vector<LeafOp> leaves;
    std::vector<TransposeOp> transposes;
    std::vector<GemmOp> gemms;
    std::vector<Op> ops;
    std::vector<char> op_micro;           // per op: run by the micro-step kernel (GEMM) or skipped (its transpose)
    std::vector<char> gemm_micro;         // per GEMM step: run by the micro-step kernel
    int root = -1;                        // tensor holding [slice bits][bs bits]
    int root_pre = -1;                    // the tree's last tensor
    int64_t tensor_elems = 0;             // tensor region size (complex64 elements)
    int64_t ksplit_elems = 0;             // scratch of the GEMM steps split over k (complex64 elements)
    double flops = 0, bytes = 0, transpose_bytes = 0;
    // Fused form: the same steps without transposes, every tensor in LDS.
    std::vector<int64_t> lds_offset;      // per program tensor (-1 if not used by the fused form)
    int64_t lds_elems = 0;
    mutable std::atomic<int> fused_fit{-1};  // whether the fused form fits (-1: not known yet)
    // Device constants.  Their host images are built once (build_consts);
    // dc holds the plan-owned device copies, created lazily on the device
    // current at first use (a call that may not allocate copies the images
    // into the library's static scratch instead).
    int device = -1;
    bool built_stepwise = false, built_fused = false;
    std::vector<char> const_host[kNumConst];
    DevConsts dc;
    int n_leaf_blocks = 0;
    int n_micro_levels = 0;
    int n_micro_groups = 0;               // workgroups of the micro-step launch
    int n_image = 0;
    int n_leaf_elems = 0;
    int n_levels = 0;
    int n_pool = 0;
    int fused_pairs = 0;                  // work items per workgroup chosen by timing (0 = not tuned yet)
    int fused_waves = 1;                  // wavefronts per work item chosen by timing
    int fused_best = 0;                   // entry of fused_tuning chosen
    std::vector<std::array<float, 3>> fused_tuning;  // (work items, wavefronts, ms) measured when tuning
    // Launch sequences captured as HIP graphs, keyed by everything the
    // captured kernel arguments depend on (buffers, range, batch, precision).
    std::vector<std::pair<std::vector<uint64_t>, void *>> graphs;  // (key, hipGraphExec_t)
};

}  // namespace qc

struct qc_plan {
    qc::Network net;
    qc::OrderProblem prob;
    std::vector<qc::Merge> tree;
    std::vector<int> sliced;              // index ids in slice-bit order
    std::vector<int> open_qubits;         // qubits whose output segment stays open (ascending)
    // The chosen tree before host folding of pair-invariant subtrees, over the
    // simplified leaves it was searched on (qc_plan_export_tree).
    std::vector<qc::Merge> tree_full;
    std::vector<std::vector<int>> origin_full;
    std::vector<uint8_t> default_bitstring;
    qc_plan_info_t info{};
    int exec_mode = QC_EXEC_AUTO;
    // Kernel timing (qc_profile_enable): pending event pairs and their kind.
    bool profiling = false;
    struct ProfEntry {
        std::string kind;
        void *e0, *e1;
        double flops;             // algorithmic flops of the launch (GEMM and micro steps; 0 otherwise)
        double bytes;             // algorithmic bytes: complex64 operands read and written once
    };
    std::vector<ProfEntry> prof_pending;
    std::vector<void *> prof_pool;
    std::mutex mu;
    std::map<std::pair<int, int>, std::unique_ptr<qc::Program>> programs;
    // Device-side state of the contraction calls (constants, tuning, graphs,
    // profiling events) is updated under dev_mu.
    std::mutex dev_mu;
    bool use_graphs = true;
    int fused_b = -1;                     // slices in flight per fused work item (log2; -1: not timed yet)
    int fused_force_pairs = 0;            // work-item shape set by the caller (0: the timed one)
    int fused_force_waves = 0;
    void *capture_stream = nullptr;       // hipStream_t used only to capture graphs
};

namespace qc {
// Lowers the plan for 2^b slices and 2^m bitstrings in flight (cached).
Program *get_program(qc_plan *plan, int b, int m, std::string &err);
std::string describe_program(const qc_plan *plan, const Program &prog);
void set_error(const std::string &msg);
}  // namespace qc
