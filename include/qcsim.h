/*
 * qcsim -- single output amplitudes <x|C|0^n> of random 2D-lattice circuits
 * by sliced tensor-network contraction on one MI355X (gfx950).
 *
 * The method (the paper, Sections "Benchmarking and the Experimental Setup"
 * and "Benchmarking Results"): the circuit is a tensor network whose nodes
 * hold tensors and whose hyper-edges are running indices; a preprocessing
 * step splits the contraction of one amplitude into N_s subtasks of equal
 * cost that share no data, and the subtask results add up to the amplitude.
 * Here the subtasks are *slices*: k binary indices (wire segments) are fixed
 * to the bits of a slice id s in [0, 2^k), every slice is contracted along
 * the same pairwise order, and the amplitude is the FP64 sum over slices.
 *
 * Conventions
 *   - Qubit q of a bitstring x is the byte x[q] in {0, 1}; batches of
 *     bitstrings are row-major uint8 [n_bs][n_qubits].
 *   - Gate matrices are indexed U[out][in]; H = (1/sqrt2)[[1,1],[1,-1]],
 *     sqrt X = 1/2[[1+i,1-i],[1-i,1+i]], sqrt Y = 1/2[[1+i,-1-i],[1+i,1+i]],
 *     T = diag(1, e^{i pi/4}), CZ = diag(1,1,1,-1) (qc_gate_matrix exports them).
 *   - A segment (q, o) is the piece of qubit q's wire after its o-th
 *     non-diagonal gate (H, sqrt X, sqrt Y); o = 0 is the input piece (fixed
 *     to 0) and the last one is the output piece (fixed to x[q]); neither can
 *     be sliced.  Slice s gives the j-th sliced segment the bit (s >> j) & 1.
 *
 * Errors: every call returns a qc_status; on error the outputs are left
 * untouched, nothing of the failed call stays enqueued on the stream, and
 * qc_last_error() (per thread) holds a message.  The library never aborts.
 *
 * Threads: a plan is immutable after qc_plan_build except for its caches
 * (lowered programs and device constants), which are guarded by a mutex.
 * Concurrent qc_contract_slices calls need separate workspaces.
 */
#ifndef QCSIM_H
#define QCSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QC_OK = 0,
    QC_ERR_INVALID_ARG = 1,  /* a pointer, size or value is invalid */
    QC_ERR_RANGE = 2,        /* a slice range or batch is out of bounds */
    QC_ERR_NOMEM = 3,        /* host or device allocation failed, or ws too small */
    QC_ERR_DEVICE = 4,       /* a HIP call failed (message in qc_last_error) */
    QC_ERR_UNSUPPORTED = 5,  /* valid request this build does not handle */
    QC_ERR_INFEASIBLE = 6    /* the slice count and the size cap cannot both be met */
} qc_status;

enum {
    QC_GATE_H = 0,
    QC_GATE_SQRT_X = 1,
    QC_GATE_SQRT_Y = 2,
    QC_GATE_T = 3,
    QC_GATE_CZ = 4
};

/* One gate; gates are given in application order.  q1 = -1 for one-qubit
 * gates.  moment is informational (not used for ordering). */
typedef struct {
    int32_t kind;
    int32_t q0;
    int32_t q1;
    int32_t moment;
} qc_gate;

typedef struct {
    int32_t n_qubits;        /* 1 .. 4096 */
    int32_t n_gates;
    const qc_gate *gates;    /* host pointer, n_gates entries; copied by qc_plan_build */
} qc_circuit;

/* Arithmetic of the contraction steps.  Tensors are always stored as
 * interleaved complex64.  QC_C64: complex FP32 steps (FP32 MFMA or vector ALU).
 * QC_SPLIT_BF16 / QC_SPLIT_FP16: GEMM steps with m and n multiples of 32 read
 * each real operand value x as x 2^-d = hi + lo in BF16 or FP16 (round to
 * nearest even) and accumulate hi*hi + hi*lo + lo*hi in FP32 on MFMA; the
 * power-of-two scale d is 0 for BF16 and, for FP16, floor(log2 max|x|) - 14
 * over the tensor instance of the current chunk, with max|x| recorded by the
 * kernel that wrote the tensor.  Smaller steps stay complex FP32, and after
 * qc_tune any step may run in complex FP32 where that form measured faster
 * (never less accurate; the kernel statistics name each launch's form).  The split
 * forms always run stepwise (see qc_plan_set_exec).  The cross-slice sum is
 * FP64 in every case. */
typedef enum {
    QC_C64 = 0,
    QC_SPLIT_BF16 = 1,
    QC_SPLIT_FP16 = 2
} qc_precision;

/* How to slice.  The planner picks k segments (in slice-bit order) so that the
 * largest intermediate of one (slice, bitstring) contraction has at most
 * 2^log2_max_entries entries and k >= log2_slices. */
typedef struct {
    int32_t log2_slices;             /* k wanted; -1 = the smallest k that meets the cap */
    double log2_max_entries;         /* cap on the largest intermediate; <= 0 = no cap */
    int32_t n_explicit;              /* number of caller-chosen sliced segments (taken first) */
    const int32_t *explicit_segments;/* n_explicit (q, ordinal) pairs, host pointer, or NULL */
    uint64_t seed;                   /* seed of the randomised greedy restarts */
    int32_t greedy_trials;           /* restarts of the order search (>= 1) */
    int32_t quick;                   /* 0: full search (greedy restarts refined by subtree
                                        reconfiguration); 1: greedy restarts and slicing only,
                                        much faster, for many small plans */
} qc_slice_spec;

typedef struct qc_plan qc_plan;

typedef struct {
    int32_t n_qubits;
    int32_t log2_slices;        /* k */
    int32_t n_indices;          /* summed binary indices of the simplified network */
    int32_t n_leaves;           /* tensors after simplification */
    int32_t n_steps;            /* pairwise contraction steps (n_leaves - 1) */
    double log2_max_entries;    /* largest intermediate, one slice and one bitstring */
    double flops_per_slice;     /* algorithmic real flops, one slice, one bitstring (8 per complex MAC) */
    double bytes_per_slice;     /* algorithmic bytes, complex64 operands read/written once */
    double flops_unsliced;      /* same order, no slicing */
    double peak_live_bytes;     /* peak live complex64 bytes, one slice, one bitstring */
    double plan_seconds;        /* host time spent in qc_plan_build */
    int32_t n_folded_steps;     /* steps whose value is the same for every slice and bitstring,
                                   computed once in qc_plan_build (not counted in n_steps or
                                   flops_per_slice) */
    int32_t n_open;             /* output qubits left open (qc_plan_build_open); 0 otherwise */
    double flops_folded;        /* algorithmic flops of those steps (FP64 on the host, once per plan) */
} qc_plan_info_t;

/* circuit + bitstring + slice set -> contraction plan (host only).
 * The paper's preprocessing (Section "Benchmarking and the Experimental
 * Setup", preprocessing paragraph): the network of the amplitude is refactored
 * into a hypergraph (refactoring paragraph: nodes hold tensors, hyper-edges are
 * running indices) and split into subtasks of equal cost that share no data;
 * it is done once and not counted in the running time.
 *   bitstring: optional default bitstring (n_qubits bytes) or NULL.
 *   spec: slicing request (NULL = no slicing, one greedy trial).
 * Builds the hypergraph network (diagonal gates share the wire's index),
 * simplifies it, searches a greedy pairwise order with randomised restarts,
 * picks the sliced segments and returns an opaque plan owned by the caller
 * (free with qc_plan_destroy).  QC_ERR_INFEASIBLE if the cap cannot be met
 * with the requested k (the message states the achievable size). */
qc_status qc_plan_build(const qc_circuit *circuit, const uint8_t *bitstring,
                        const qc_slice_spec *spec, qc_plan **out);

/* Largest number of open output qubits (2^20 amplitudes per bitstring). */
#define QC_MAX_OPEN_QUBITS 20

/* qc_plan_build with the output segments of the qubits open_qubits[0 ..
 * n_open - 1] left open: those indices are never fixed to a bitstring bit nor
 * summed, the order search keeps them to the end, and every contraction of the
 * plan yields, per bitstring x, the 2^n_open amplitudes <y|C|0^n> of the
 * bitstrings y that equal x outside the open qubits -- many amplitudes from one
 * contraction, the regime where the paper computes many amplitudes of one
 * circuit (Section "Benchmarking Results", N_a paragraph; Porter-Thomas
 * paragraph).  The bits x[q] of the open qubits are ignored.  Result entry o in
 * [0, 2^n_open) sets open qubit open_qubits_sorted[i] to bit (n_open - 1 - i)
 * of o: the open qubits in increasing order, the first one the most
 * significant, as in the bitstring index of the state vector.
 *   n_open: 0 .. QC_MAX_OPEN_QUBITS; open_qubits: distinct qubits (any order,
 *   host pointer, copied), or NULL when n_open = 0.
 * Plans with open outputs always run stepwise and are not accepted by
 * qc_contract_batch (QC_ERR_UNSUPPORTED); every output buffer of the
 * contraction calls has 2^n_open entries per bitstring (below).  Errors as
 * qc_plan_build; QC_ERR_INVALID_ARG for a bad open qubit list. */
qc_status qc_plan_build_open(const qc_circuit *circuit, const uint8_t *bitstring, const qc_slice_spec *spec,
                             int32_t n_open, const int32_t *open_qubits, qc_plan **out);

/* The plan's sizes and costs (the quantities of the paper's prediction from
 * subtask cost, Section "Benchmarking Results", prediction paragraph). */
qc_status qc_plan_info(const qc_plan *plan, qc_plan_info_t *info);

/* The k sliced segments as (q, ordinal) pairs in slice-bit order: out_pairs
 * must hold 2k int32.  (The split into subtasks of the preprocessing
 * paragraph; which indices are fixed is this library's choice.) */
qc_status qc_plan_sliced_segments(const qc_plan *plan, int32_t *out_pairs);

/* Bit values of slice s: out[j] = (s >> j) & 1 for j < k; QC_ERR_RANGE if
 * s >= 2^k. */
qc_status qc_plan_slice_assignment(const qc_plan *plan, uint64_t s, uint8_t *out);

/* JSON description of the program lowered for 2^log2_batch_slices slices and
 * 2^log2_batch_bs bitstrings in flight: leaves (indices, base values),
 * steps (operands, layouts, GEMM shapes; c_nat names the tensor holding a
 * step's natural [batch][m][n] order when it writes its output scattered
 * into the layout of c) and per-step algorithmic flops/bytes, and the fused
 * form's state: fused_pairs and fused_waves (the timed work-item shape, 0
 * before the first fused call), fused_slice_bits, fused_shape_set (the shape
 * set by qc_plan_set_fused_shape, [0,0] if none) and fused_tuning (items,
 * wavefronts, ms per timed shape).  Writes at most cap bytes to buf (NUL
 * terminated when it fits) and the full length to *len. */
qc_status qc_plan_describe(qc_plan *plan, int32_t log2_batch_slices, int32_t log2_batch_bs,
                           qc_precision prec, char *buf, size_t cap, size_t *len);

/* The same lowered program's operations as a table, in execution order.
 * kind 1 = GEMM step (a, b = operand tensors, c = result; C[nb][m][n] =
 * sum_k A B with A stored [nb][k][m] if a_km else [nb][m][k], B stored
 * [nb][n][k] if b_nk else [nb][k][n]; C is written in c's layout, which may
 * be a bit permutation of [nb][m][n]).  kind 0 = bit-permuting transpose
 * (a = source, c = destination, m = its number of complex64 elements): the
 * current lowering folds every transpose into the producer of its source
 * and emits none.  Tensor ids match qc_plan_describe.  Writes min(cap,
 * count) rows to out (out may be NULL when cap is 0) and the count to *n;
 * QC_ERR_RANGE if the batch sizes exceed the plan.  micro = 1 marks the
 * small steps (output and operands of at most 2^12 entries, fed only by
 * leaves and other small steps) that the stepwise form runs together in one
 * launch right after the leaves. */
typedef struct {
    int32_t kind;
    int32_t a, b, c;                 /* b = -1 for a transpose */
    int64_t nb, m, n, k;
    int32_t a_km, b_nk;
    double flops;                    /* 8 nb m n k for a GEMM step, 0 for a transpose */
    int32_t micro, reserved;
} qc_step_t;
qc_status qc_plan_export_steps(qc_plan *plan, int32_t log2_batch_slices, int32_t log2_batch_bs, qc_step_t *out,
                               int32_t cap, int32_t *n);

/* The plan's pairwise contraction tree in the circuit's own terms, so that
 * it can be followed by code that shares nothing with this library (the
 * tree is data: any valid tree gives the same value, up to rounding, since
 * the value of a network does not depend on the order of its pairwise
 * contractions).  The circuit's tensors are numbered t < n_qubits for qubit
 * t's input state <0| ... |0> factor and n_qubits + g for gate g of the
 * circuit as given to qc_plan_build (H, sqrt X, sqrt Y: U[new][old] between
 * consecutive segments; T: a vector on its segment; CZ: a 2x2 tensor on two
 * segments).  Output segments are fixed to x[q] and sliced segments to the
 * slice's bits; they are not tensors here.
 *   *n_leaves: L, the number of simplified tensors the order was chosen on;
 *   *n_tensors: n_qubits + number of gates;
 *   origin_offsets (optional, L + 1 int32) and origin_ids (optional,
 *     *n_tensors int32): leaf l consists of the circuit tensors
 *     origin_ids[origin_offsets[l] .. origin_offsets[l + 1]) (every circuit
 *     tensor in exactly one leaf);
 *   merges (optional, 2 (L - 1) int32): merge i combines nodes merges[2 i]
 *     and merges[2 i + 1], where nodes < L are leaves and node L + i is the
 *     result of merge i; the last merge yields the slice value.
 * This is the tree before the plan evaluates its pair-invariant subtrees on
 * the host (those subtrees are part of it).  Call with NULL arrays first to
 * learn the sizes.  Host only; QC_ERR_INVALID_ARG on NULL plan or counts. */
qc_status qc_plan_export_tree(const qc_plan *plan, int32_t *n_leaves, int32_t *n_tensors,
                              int32_t *origin_offsets, int32_t *origin_ids, int32_t *merges);

/* How qc_contract_slices runs the program:
 *   QC_EXEC_AUTO (default): fused when one (slice, bitstring) contraction
 *     fits in LDS and prec is QC_C64, else stepwise;
 *   QC_EXEC_FUSED: one launch per super-chunk, each wavefront contracting a
 *     whole program for a chunk of 2^b slices (b in-flight slice bits, see
 *     qc_plan_set_fused_slice_bits) and one bitstring in LDS in complex FP32
 *     (QC_ERR_UNSUPPORTED later if it does not fit or prec is split);
 *   QC_EXEC_STEPWISE: one batched complex GEMM per pairwise step, with
 *     slices and bitstrings in flight as batch indices in global memory; each
 *     step writes its output directly in the layout its consumer reads (no
 *     separate transposes), and small steps run together in one launch.
 * Call before qc_workspace_bytes (the workspace depends on the mode). */
enum { QC_EXEC_AUTO = 0, QC_EXEC_FUSED = 1, QC_EXEC_STEPWISE = 2 };
qc_status qc_plan_set_exec(qc_plan *plan, int32_t mode);

/* Graph replay of the stepwise form (on by default).  The launches of one
 * chunk that do not depend on its position (the micro-step launch and every
 * GEMM or transpose step) are captured once per configuration (precision,
 * slices and bitstrings in flight, workspace) as a HIP graph on a private
 * stream, with no memset nodes; every chunk of every call with that
 * configuration replays it on the caller's stream, between the chunk's leaf
 * launch and its slice-value copy, whatever the slice range -- so a call over
 * any number of chunks holds one graph.  Up to 8 graphs are kept per lowered
 * program; evicting one waits for the device to drain.  Calls with kernel
 * timing on, and the fused form, launch directly.  on = 0 launches every
 * kernel directly. */
qc_status qc_plan_set_graphs(qc_plan *plan, int32_t on);

/* In-flight slice bits b of the fused form: each work item contracts 2^b
 * slices at once, sharing the work that does not depend on those slice bits
 * (the program is lowered with them as open indices), at the price of 2^b
 * times fewer work items (each run by 1 to 16 wavefronts, as timed).  With
 * b = 6 a work item is one 64-slice block and, when a launch holds one block
 * per bitstring, it adds its block sum to out_dev itself (no separate
 * reduction launch; same bits).  b = -1 (default): the first fused call times
 * every b in 0..6 whose program fits in LDS (with its best work-item shape,
 * plus the reduction launch where one is needed) on one super-chunk and keeps
 * the fastest for the plan's lifetime; b in 0..6 fixes it (for b > 0,
 * QC_ERR_UNSUPPORTED if that program does not fit; QC_ERR_RANGE if b exceeds
 * the plan's slice bits).  Slice values depend on b at the
 * rounding level only; calls with the same b are bitwise reproducible.  The
 * fused requests of qc_contract_batch always run b = 0.  The choice is
 * reported as "fused_slice_bits" by qc_plan_describe. */
qc_status qc_plan_set_fused_slice_bits(qc_plan *plan, int32_t b);

/* Work-item shape of the fused form: items_per_workgroup work items, each
 * run by waves_per_item wavefronts, one of (1,1), (2,1), (4,1), (1,2),
 * (1,4), (1,8), (1,16); (0,0) (default) uses the shape timed on first use
 * for each lowered program.  The shape changes the kernel's schedule, not
 * what it computes (same bits), and is used by every later fused launch of
 * the plan; a launch whose shape does not fit in LDS (more items per
 * workgroup than the program's LDS region allows) fails with QC_ERR_DEVICE
 * and a message.  QC_ERR_INVALID_ARG for any other pair.  The in-launch
 * block sums of b = 6 need one item per workgroup.  The requests of
 * qc_contract_batch are not affected. */
qc_status qc_plan_set_fused_shape(qc_plan *plan, int32_t items_per_workgroup, int32_t waves_per_item);

/* Autotuning (untimed preparation, like qc_plan_build).  Lowers the plan
 * for chunk_slices slices and n_bs bitstrings in flight (as
 * qc_contract_slices would with this workspace) and, for every GEMM step of
 * the stepwise program, times each applicable kernel form (MFMA tile shapes,
 * the split 128 x 128 and 128 x 64 tiles, the streaming MFMA forms, the
 * skinny, rows, dot and vector-ALU forms) on the
 * caller's workspace (contents are overwritten) and stream, and keeps the
 * fastest for this plan and precision.  Choices are shared process-wide per
 * (device architecture, precision, shape, operand layout); cache_path (or
 * NULL) names a text file that is read first, so known shapes are not timed
 * again, and rewritten afterwards.  *n_timed (optional) receives the number
 * of shapes timed.  Synchronous.  Fused programs time their own launch forms
 * on first use and are left alone here. */
qc_status qc_tune(qc_plan *plan, int64_t chunk_slices, int32_t n_bs, qc_precision prec, void *ws,
                  size_t ws_bytes, void *stream, const char *cache_path, int32_t *n_timed);

/* Kernel timing.  While enabled, qc_contract_slices records a pair of HIP
 * events on its stream around every kernel it launches.  qc_profile_read
 * waits for the recorded events, then reports per kernel kind the launch
 * count, the summed event-to-event milliseconds and the summed algorithmic
 * flops and bytes of those launches (8 nb m n k flops and 8 nb (m k + k n +
 * m n) bytes per GEMM step, the micro launch's steps likewise; 0 for kinds
 * that do no GEMM work) since the last read, and clears them.  kinds:
 * "fused", "leaves", "micro", "transpose", "gemm_mfma", "gemm_split_bf16",
 * "gemm_split_fp16", "gemm_skinny", "gemm_skinny_t", "gemm_rows", "gemm_dot",
 * "gemm_dot_tile", "gemm_valu", "reduce64" (a GEMM step split over k counts its
 * partial products and their sum under its form's kind), so the kinds show
 * which form -- and for split precisions whether a split MFMA form or a
 * complex FP32 one -- ran each step.  Launches replayed from a graph are not
 * timed (calls with timing on launch directly).  Not thread-safe across
 * concurrent calls on one plan. */
typedef struct {
    char kind[16];
    int64_t launches;
    double total_ms;
    double flops;
    double bytes;      /* algorithmic bytes of those launches: 8 nb (m k + k n + m n) per GEMM step */
} qc_kernel_stat_t;
qc_status qc_profile_enable(qc_plan *plan, int32_t on);
qc_status qc_profile_read(qc_plan *plan, qc_kernel_stat_t *out, int32_t cap, int32_t *n);

/* Device workspace (bytes) that qc_contract_slices needs to keep
 * chunk_slices slices (rounded up to a power of two) and n_bs bitstrings in
 * flight.  0 on invalid arguments.
 *
 * Open outputs: for a plan with n_open > 0, every per-bitstring output below
 * holds A = 2^n_open amplitudes (entry o as in qc_plan_build_open): out_dev is
 * double [n_bs][A][2], per_slice_dev [s_end - s_begin][n_bs][A][2], out_host
 * of qc_amplitude [A][2].  n_bs * A must not exceed 2^20. */
size_t qc_workspace_bytes(qc_plan *plan, int64_t chunk_slices, int32_t n_bs, qc_precision prec);

/* plan + slice range -> partial amplitudes, asynchronously on `stream`
 * The subtasks of the paper (Section "Benchmarking Results", subtask
 * paragraph: equal cost, no shared data, any share of them per worker) are the
 * slices; their results add up to the amplitude (Section "Benchmarking and the
 * Experimental Setup", preprocessing paragraph), so a range's partial sum is
 * added to out_dev and ranges compose.
 * (a hipStream_t, or NULL for the null stream) of the current device.
 *   bitstrings: host uint8 [n_bs][n_qubits], 1 <= n_bs <= 65536; copied.
 *   ws, ws_bytes: device workspace owned by the caller; the largest
 *     power-of-two number of slices in flight that fits is used (at least
 *     one slice must fit, else QC_ERR_NOMEM).
 *   out_dev: device double [n_bs][2] (re, im); the sum over s in
 *     [s_begin, s_end) of each slice value is ADDED to it, so consecutive
 *     ranges compose.  Slices are summed in increasing s within fixed-size
 *     chunks, in FP64, so the result is bitwise reproducible for the same
 *     range and workspace size.
 *   per_slice_dev: optional device double [s_end - s_begin][n_bs][2]
 *     receiving each slice's value, or NULL.
 * The call returns once the work is enqueued; synchronise the stream before
 * reading out_dev. */
qc_status qc_contract_slices(qc_plan *plan, uint64_t s_begin, uint64_t s_end,
                             const uint8_t *bitstrings, int32_t n_bs, qc_precision prec,
                             void *ws, size_t ws_bytes, void *stream,
                             double *out_dev, double *per_slice_dev);

/* qc_contract_slices with the bitstrings already resident in device memory:
 * bitstrings_dev is a device uint8 [n_bs][n_qubits] array owned by the
 * caller, entries 0 or 1 (not checked), read by the kernels of this call, so
 * it must stay unchanged until the stream reaches them.  Nothing is copied
 * from the host; otherwise identical semantics and errors. */
qc_status qc_contract_slices_dev(qc_plan *plan, uint64_t s_begin, uint64_t s_end,
                                 const uint8_t *bitstrings_dev, int32_t n_bs, qc_precision prec,
                                 void *ws, size_t ws_bytes, void *stream,
                                 double *out_dev, double *per_slice_dev);

/* qc_contract_slices_dev for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): it calls no hipMalloc, hipFree or allocating library routine.
 * Instead of a caller workspace it uses the library's own scratch, a static
 * device array of 64 MiB that each GPU the library runs on holds until the
 * process ends: the lowered program's constants are copied into it on
 * `stream` (hipMemcpyAsync from plan-owned host memory) and the rest serves as
 * the workspace.  Same arguments, semantics and errors as
 * qc_contract_slices_dev otherwise (out_dev accumulates; per_slice_dev
 * optional), with these differences:
 *   - QC_ERR_NOMEM if the program's constants plus the workspace for one
 *     slice (or one 64-slice block of the fused form) in flight exceed the
 *     64 MiB; the message says so.  Fewer slices are kept in flight than a
 *     larger caller workspace would allow, so results may differ from
 *     qc_contract_slices_dev in rounding (the FP64 sum's chunking, and for
 *     the fused form the slice bits per work item), never beyond the
 *     precision's tolerance.
 *   - Nothing is timed and no graph is captured: the fused form uses the
 *     plan's in-flight slice bits and work-item shape if an earlier call
 *     timed them, else b = 0 and one work item on four wavefronts; kernel
 *     timing (qc_profile_enable) is ignored.
 *   - Every call on one GPU shares that GPU's scratch, which keeps the last
 *     call's contents: calls that overlap on one GPU (different streams or
 *     threads without ordering between them) race and give wrong results.
 *     Calls ordered on one stream are safe. */
qc_status qc_contract_slices_noalloc(qc_plan *plan, uint64_t s_begin, uint64_t s_end,
                                     const uint8_t *bitstrings_dev, int32_t n_bs, qc_precision prec,
                                     void *stream, double *out_dev, double *per_slice_dev);

/* All slices of one amplitude, synchronously; allocates and frees its own
 * workspace on the current device.  out_host[0..1] = (re, im).  The
 * amplitude <x|C|0^n> is the sum of all subtask results (Section
 * "Benchmarking and the Experimental Setup", preprocessing paragraph). */
qc_status qc_amplitude(qc_plan *plan, const uint8_t *bitstring, qc_precision prec,
                       double out_host[2]);

/* Many amplitude requests, each with its own plan, bitstring and slice
 * range, in one call (asynchronous on `stream`): the paper's many-amplitude
 * batches (Section "Benchmarking Results", N_a paragraph: time per amplitude
 * falls as more amplitudes share the machine).  Requests whose plan runs
 * fused (complex FP32, the program fits in LDS) share one launch whose
 * wavefronts take (request, slice) pairs in turn; the others run stepwise on
 * eight internal streams (default priority) that start after the caller's
 * earlier work and that the caller's stream waits for.  Per request r: out_dev[2 r .. 2 r + 1] +=
 * its sum over slices [s_begin, s_end) (same fixed-order FP64 sum as
 * qc_contract_slices); t_done_dev[r] = device wall-clock time (see
 * hipDeviceAttributeWallClockRate) at which its last slice value was
 * written (fused) or its sum was formed (stepwise); t_done_dev[n] = the
 * time the batch started.  ws: at least qc_batch_workspace_bytes. */
typedef struct {
    qc_plan *plan;
    const uint8_t *bitstring;    /* host uint8 [n_qubits] of this plan's circuit, copied */
    uint64_t s_begin, s_end;     /* slice range of this request */
} qc_request;
size_t qc_batch_workspace_bytes(const qc_request *reqs, int32_t n, qc_precision prec);
/* Rate of the device wall clock used by the completion stamps (kHz). */
qc_status qc_wall_clock_khz(int32_t *khz);
qc_status qc_contract_batch(const qc_request *reqs, int32_t n, qc_precision prec, void *ws, size_t ws_bytes,
                            void *stream, double *out_dev, uint64_t *t_done_dev);

/* The library's gate matrix as row-major (re, im) pairs: 2x2 (8 doubles)
 * for one-qubit kinds, 4x4 (32 doubles) for CZ; out must hold 32 doubles. */
qc_status qc_gate_matrix(int32_t kind, double *out);

/* Frees the plan and its device constants (NULL-safe). */
void qc_plan_destroy(qc_plan *plan);

/* Message of the last failed call on this thread ("" if none). */
const char *qc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QCSIM_H */
