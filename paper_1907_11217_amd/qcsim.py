"""Thin ctypes binding of libqcsim.so (argument marshalling only).

Every function here has the name of the C entry point it calls (see
include/qcsim.h).  Device buffers are torch tensors on the current device
(``data_ptr()``) and the stream is torch's current stream; all contraction
work runs in the library's HIP kernels.  If the library is missing, every
call raises: there is no fallback path.
"""

from __future__ import annotations

import ctypes
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqcsim.so")

QC_OK = 0
QC_C64, QC_SPLIT_BF16, QC_SPLIT_FP16 = 0, 1, 2
PRECISIONS = {"c64": QC_C64, "split_bf16": QC_SPLIT_BF16, "split_fp16": QC_SPLIT_FP16}
STATUS_NAMES = {0: "QC_OK", 1: "QC_ERR_INVALID_ARG", 2: "QC_ERR_RANGE", 3: "QC_ERR_NOMEM",
                4: "QC_ERR_DEVICE", 5: "QC_ERR_UNSUPPORTED", 6: "QC_ERR_INFEASIBLE"}

EXPORTED = (
    "qc_plan_build", "qc_plan_info", "qc_plan_sliced_segments", "qc_plan_slice_assignment",
    "qc_plan_describe", "qc_workspace_bytes", "qc_contract_slices", "qc_amplitude",
    "qc_gate_matrix", "qc_plan_destroy", "qc_last_error", "qc_kernel_gemm", "qc_kernel_transpose",
    "qc_plan_set_exec", "qc_profile_enable", "qc_profile_read", "qc_contract_slices_dev", "qc_plan_set_graphs",
    "qc_tune", "qc_kernel_gemm_form", "qc_batch_workspace_bytes", "qc_contract_batch", "qc_wall_clock_khz",
    "qc_plan_export_steps", "qc_kernel_gemm_kparts", "qc_gemm_kparts", "qc_plan_set_fused_slice_bits",
    "qc_plan_set_fused_shape", "qc_plan_export_tree", "qc_contract_slices_noalloc", "qc_plan_build_open",
)
EXEC_MODES = {"auto": 0, "fused": 1, "stepwise": 2}


class QcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class qc_gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("q0", ctypes.c_int32), ("q1", ctypes.c_int32),
                ("moment", ctypes.c_int32)]


class qc_circuit(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_gates", ctypes.c_int32),
                ("gates", ctypes.POINTER(qc_gate))]


class qc_step_t(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("a", ctypes.c_int32), ("b", ctypes.c_int32), ("c", ctypes.c_int32),
                ("nb", ctypes.c_int64), ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
                ("a_km", ctypes.c_int32), ("b_nk", ctypes.c_int32), ("flops", ctypes.c_double),
                ("micro", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class qc_request(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("bitstring", ctypes.POINTER(ctypes.c_uint8)),
                ("s_begin", ctypes.c_uint64), ("s_end", ctypes.c_uint64)]


class qc_slice_spec(ctypes.Structure):
    _fields_ = [("log2_slices", ctypes.c_int32), ("log2_max_entries", ctypes.c_double),
                ("n_explicit", ctypes.c_int32), ("explicit_segments", ctypes.POINTER(ctypes.c_int32)),
                ("seed", ctypes.c_uint64), ("greedy_trials", ctypes.c_int32), ("quick", ctypes.c_int32)]


class qc_plan_info_t(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("log2_slices", ctypes.c_int32),
                ("n_indices", ctypes.c_int32), ("n_leaves", ctypes.c_int32), ("n_steps", ctypes.c_int32),
                ("log2_max_entries", ctypes.c_double), ("flops_per_slice", ctypes.c_double),
                ("bytes_per_slice", ctypes.c_double), ("flops_unsliced", ctypes.c_double),
                ("peak_live_bytes", ctypes.c_double), ("plan_seconds", ctypes.c_double),
                ("n_folded_steps", ctypes.c_int32), ("n_open", ctypes.c_int32), ("flops_folded", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class qc_kernel_stat_t(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_char * 16), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


_lib = None


def load(path: str | None = None):
    """Loads libqcsim.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(p)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    lib.qc_plan_build.argtypes = [ctypes.POINTER(qc_circuit), vp, ctypes.POINTER(qc_slice_spec), ctypes.POINTER(vp)]
    lib.qc_plan_build_open.argtypes = [ctypes.POINTER(qc_circuit), vp, ctypes.POINTER(qc_slice_spec), ctypes.c_int32,
                                       vp, ctypes.POINTER(vp)]
    lib.qc_plan_build_open.restype = ctypes.c_int
    lib.qc_plan_info.argtypes = [vp, ctypes.POINTER(qc_plan_info_t)]
    lib.qc_plan_sliced_segments.argtypes = [vp, vp]
    lib.qc_plan_slice_assignment.argtypes = [vp, ctypes.c_uint64, vp]
    lib.qc_plan_describe.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, vp, sz, ctypes.POINTER(sz)]
    lib.qc_gate_matrix.argtypes = [ctypes.c_int32, vp]
    lib.qc_plan_set_exec.argtypes = [vp, ctypes.c_int32]
    lib.qc_plan_set_exec.restype = ctypes.c_int
    lib.qc_plan_destroy.argtypes = [vp]
    lib.qc_plan_destroy.restype = None
    lib.qc_last_error.restype = ctypes.c_char_p
    for name in ("qc_plan_build", "qc_plan_info", "qc_plan_sliced_segments", "qc_plan_slice_assignment",
                 "qc_plan_describe", "qc_gate_matrix"):
        getattr(lib, name).restype = ctypes.c_int
    if hasattr(lib, "qc_contract_slices"):
        lib.qc_workspace_bytes.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int]
        lib.qc_workspace_bytes.restype = sz
        lib.qc_contract_slices.argtypes = [vp, ctypes.c_uint64, ctypes.c_uint64, vp, ctypes.c_int32, ctypes.c_int,
                                           vp, sz, vp, vp, vp]
        lib.qc_contract_slices.restype = ctypes.c_int
        lib.qc_contract_slices_dev.argtypes = lib.qc_contract_slices.argtypes
        lib.qc_contract_slices_dev.restype = ctypes.c_int
        lib.qc_amplitude.argtypes = [vp, vp, ctypes.c_int, vp]
        lib.qc_amplitude.restype = ctypes.c_int
        i64 = ctypes.c_int64
        lib.qc_kernel_gemm.argtypes = [vp, vp, vp, i64, i64, i64, i64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, vp,
                                       vp]
        lib.qc_kernel_gemm.restype = ctypes.c_int
        lib.qc_kernel_gemm_form.argtypes = [vp, vp, vp, i64, i64, i64, i64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int,
                                            ctypes.c_int32, vp, vp]
        lib.qc_kernel_gemm_form.restype = ctypes.c_int
        lib.qc_kernel_gemm_kparts.argtypes = [vp, vp, vp, i64, i64, i64, i64, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_int, ctypes.c_int32, i64, vp, vp, vp]
        lib.qc_kernel_gemm_kparts.restype = ctypes.c_int
        lib.qc_gemm_kparts.argtypes = [i64, i64, i64, i64]
        lib.qc_gemm_kparts.restype = i64
        lib.qc_kernel_transpose.argtypes = [vp, vp, ctypes.c_int32, vp, vp]
        lib.qc_kernel_transpose.restype = ctypes.c_int
        lib.qc_tune.argtypes = [vp, i64, ctypes.c_int32, ctypes.c_int, vp, ctypes.c_size_t, vp, ctypes.c_char_p,
                                ctypes.POINTER(ctypes.c_int32)]
        lib.qc_tune.restype = ctypes.c_int
        lib.qc_batch_workspace_bytes.argtypes = [ctypes.POINTER(qc_request), ctypes.c_int32, ctypes.c_int]
        lib.qc_batch_workspace_bytes.restype = ctypes.c_size_t
        lib.qc_contract_batch.argtypes = [ctypes.POINTER(qc_request), ctypes.c_int32, ctypes.c_int, vp, ctypes.c_size_t,
                                          vp, vp, vp]
        lib.qc_contract_batch.restype = ctypes.c_int
        lib.qc_plan_export_steps.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(qc_step_t),
                                             ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        lib.qc_plan_export_steps.restype = ctypes.c_int
        lib.qc_contract_slices_noalloc.argtypes = [vp, ctypes.c_uint64, ctypes.c_uint64, vp, ctypes.c_int32,
                                                   ctypes.c_int, vp, vp, vp]
        lib.qc_contract_slices_noalloc.restype = ctypes.c_int
        pi32 = ctypes.POINTER(ctypes.c_int32)
        lib.qc_plan_export_tree.argtypes = [vp, pi32, pi32, pi32, pi32, pi32]
        lib.qc_plan_export_tree.restype = ctypes.c_int
        lib.qc_wall_clock_khz.argtypes = [ctypes.POINTER(ctypes.c_int32)]
        lib.qc_wall_clock_khz.restype = ctypes.c_int
        lib.qc_plan_set_graphs.argtypes = [vp, ctypes.c_int32]
        lib.qc_plan_set_graphs.restype = ctypes.c_int
        lib.qc_plan_set_fused_slice_bits.argtypes = [vp, ctypes.c_int32]
        lib.qc_plan_set_fused_slice_bits.restype = ctypes.c_int
        lib.qc_plan_set_fused_shape.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
        lib.qc_plan_set_fused_shape.restype = ctypes.c_int
        lib.qc_profile_enable.argtypes = [vp, ctypes.c_int32]
        lib.qc_profile_enable.restype = ctypes.c_int
        lib.qc_profile_read.argtypes = [vp, ctypes.POINTER(qc_kernel_stat_t), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32)]
        lib.qc_profile_read.restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def qc_last_error() -> str:
    return load().qc_last_error().decode()


def _check(status: int, lib=None):
    if status != QC_OK:
        raise QcError(status, (lib or load()).qc_last_error().decode())


def _prec(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


class Plan:
    """Owns a qc_plan*; freed by qc_plan_destroy when garbage collected."""

    def __init__(self, handle, lib, n_qubits, n_open=0):
        self._h = handle
        self._lib = lib
        self.n_qubits = n_qubits
        self.n_open = n_open            # open output qubits: 2^n_open amplitudes per bitstring

    @property
    def n_amp(self):
        return 1 << self.n_open

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.qc_plan_destroy(self._h)
            self._h = None


def qc_plan_build(n_qubits: int, circuit, bitstring=None, log2_slices: int = 0,
                  log2_max_entries: float = 0.0, explicit_segments=None, seed: int = 0,
                  greedy_trials: int = 1, open_qubits=None, quick: bool = False, lib=None) -> Plan:
    """Calls qc_plan_build, or qc_plan_build_open when ``open_qubits`` (a
    list of qubits whose outputs stay open) is given and not empty; ``quick``
    skips the subtree reconfiguration of the order search."""
    lib = lib or load()
    circ = np.ascontiguousarray(np.asarray(circuit, dtype=np.int32).reshape(-1, 4))
    gates = (qc_gate * max(1, len(circ)))()
    ctypes.memmove(gates, circ.ctypes.data, circ.nbytes)
    c = qc_circuit(int(n_qubits), len(circ), gates)
    ex = None
    n_ex = 0
    if explicit_segments is not None and len(explicit_segments):
        ex_arr = np.ascontiguousarray(np.asarray(explicit_segments, dtype=np.int32).reshape(-1, 2))
        n_ex = len(ex_arr)
        ex = (ctypes.c_int32 * (2 * n_ex))(*ex_arr.reshape(-1).tolist())
    spec = qc_slice_spec(int(log2_slices), float(log2_max_entries), n_ex,
                         ctypes.cast(ex, ctypes.POINTER(ctypes.c_int32)) if ex is not None else None,
                         int(seed), int(greedy_trials), int(bool(quick)))
    bsp = None
    if bitstring is not None:
        bs = np.ascontiguousarray(np.asarray(bitstring, dtype=np.uint8).reshape(-1))
        bsp = bs.ctypes.data
    h = ctypes.c_void_p()
    if open_qubits is not None and len(open_qubits):
        oq = np.ascontiguousarray(np.asarray(open_qubits, dtype=np.int32).reshape(-1))
        _check(lib.qc_plan_build_open(ctypes.byref(c), bsp, ctypes.byref(spec), len(oq), oq.ctypes.data,
                                      ctypes.byref(h)), lib)
        return Plan(h, lib, int(n_qubits), len(oq))
    _check(lib.qc_plan_build(ctypes.byref(c), bsp, ctypes.byref(spec), ctypes.byref(h)), lib)
    return Plan(h, lib, int(n_qubits))


def qc_plan_info(plan: Plan) -> dict:
    info = qc_plan_info_t()
    _check(plan._lib.qc_plan_info(plan.handle, ctypes.byref(info)), plan._lib)
    return info.as_dict()


def qc_plan_sliced_segments(plan: Plan) -> np.ndarray:
    k = qc_plan_info(plan)["log2_slices"]
    out = np.zeros((max(k, 1), 2), dtype=np.int32)
    _check(plan._lib.qc_plan_sliced_segments(plan.handle, out.ctypes.data), plan._lib)
    return out[:k]


def qc_plan_slice_assignment(plan: Plan, s: int) -> np.ndarray:
    k = qc_plan_info(plan)["log2_slices"]
    out = np.zeros(max(k, 1), dtype=np.uint8)
    _check(plan._lib.qc_plan_slice_assignment(plan.handle, ctypes.c_uint64(int(s)), out.ctypes.data), plan._lib)
    return out[:k]


def qc_plan_describe(plan: Plan, log2_batch_slices: int = 0, log2_batch_bs: int = 0, prec="c64") -> dict:
    n = ctypes.c_size_t()
    _check(plan._lib.qc_plan_describe(plan.handle, log2_batch_slices, log2_batch_bs, _prec(prec), None, 0,
                                      ctypes.byref(n)), plan._lib)
    buf = ctypes.create_string_buffer(n.value + 1)
    _check(plan._lib.qc_plan_describe(plan.handle, log2_batch_slices, log2_batch_bs, _prec(prec), buf,
                                      n.value + 1, ctypes.byref(n)), plan._lib)
    return json.loads(buf.value.decode())


def qc_plan_set_exec(plan: Plan, mode) -> None:
    m = EXEC_MODES[mode] if isinstance(mode, str) else int(mode)
    _check(plan._lib.qc_plan_set_exec(plan.handle, m), plan._lib)


def qc_tune(plan: Plan, chunk_slices: int, n_bs: int, prec, ws, cache_path=None, stream=None) -> int:
    """Times the GEMM kernel forms of the stepwise program for this chunk and
    keeps the fastest; returns the number of shapes timed (0 when the cache
    file already held them all)."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    n = ctypes.c_int32(0)
    _check(plan._lib.qc_tune(plan.handle, int(chunk_slices), int(n_bs), _prec(prec), ws.data_ptr(),
                             ws.numel() * ws.element_size(), st.cuda_stream,
                             None if cache_path is None else str(cache_path).encode(), ctypes.byref(n)), plan._lib)
    return n.value


class Batch:
    """A request array for qc_contract_batch: (plan, bitstring, s_begin, s_end)
    tuples; keeps the plans and bitstrings alive."""

    def __init__(self, requests):
        self.plans = [r[0] for r in requests]
        self.bits = [np.ascontiguousarray(np.asarray(r[1], dtype=np.uint8)) for r in requests]
        self.array = (qc_request * len(requests))()
        for i, (p, b, r) in enumerate(zip(self.plans, self.bits, requests)):
            s0 = r[2] if len(r) > 2 else 0
            s1 = r[3] if len(r) > 3 else (1 << qc_plan_info(p)["log2_slices"])
            self.array[i] = qc_request(p.handle, b.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), s0, s1)
        self.lib = self.plans[0]._lib

    def __len__(self):
        return len(self.plans)


def qc_batch_workspace_bytes(batch: Batch, prec="c64") -> int:
    n = int(batch.lib.qc_batch_workspace_bytes(batch.array, len(batch), _prec(prec)))
    if n == 0:
        raise QcError(1, batch.lib.qc_last_error().decode())
    return n


def qc_contract_batch(batch: Batch, prec, ws, out_dev, t_done_dev, stream=None):
    """Enqueues every request; out_dev float64 [n, 2] (accumulated into),
    t_done_dev int64 [n + 1] (completion wall-clock stamps, then the start)."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(batch.lib.qc_contract_batch(batch.array, len(batch), _prec(prec), ws.data_ptr(),
                                       ws.numel() * ws.element_size(), st.cuda_stream, out_dev.data_ptr(),
                                       t_done_dev.data_ptr()), batch.lib)


def qc_plan_export_steps(plan: Plan, log2_batch_slices: int = 0, log2_batch_bs: int = 0):
    """The lowered program's operations as a list of dicts (execution order)."""
    n = ctypes.c_int32(0)
    _check(plan._lib.qc_plan_export_steps(plan.handle, log2_batch_slices, log2_batch_bs, None, 0, ctypes.byref(n)),
           plan._lib)
    rows = (qc_step_t * max(1, n.value))()
    _check(plan._lib.qc_plan_export_steps(plan.handle, log2_batch_slices, log2_batch_bs, rows, n.value,
                                          ctypes.byref(n)), plan._lib)
    return [{f: getattr(rows[i], f) for f, _ in qc_step_t._fields_} for i in range(n.value)]


def qc_plan_export_tree(plan: Plan):
    """The plan's contraction tree in circuit terms: (groups, merges), groups[l]
    the circuit tensor ids of leaf l (t < n_qubits: input of qubit t; n_qubits
    + g: gate g), merges an int32 [L - 1, 2] array of node ids (leaves first,
    then merge results)."""
    L, T = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(plan._lib.qc_plan_export_tree(plan.handle, ctypes.byref(L), ctypes.byref(T), None, None, None), plan._lib)
    offs = np.zeros(L.value + 1, dtype=np.int32)
    ids = np.zeros(max(1, T.value), dtype=np.int32)
    merges = np.zeros((max(1, L.value - 1), 2), dtype=np.int32)
    i32p = ctypes.POINTER(ctypes.c_int32)
    _check(plan._lib.qc_plan_export_tree(plan.handle, ctypes.byref(L), ctypes.byref(T), offs.ctypes.data_as(i32p),
                                         ids.ctypes.data_as(i32p), merges.ctypes.data_as(i32p)), plan._lib)
    groups = [ids[offs[i]:offs[i + 1]].tolist() for i in range(L.value)]
    return groups, merges[:max(0, L.value - 1)]


def qc_wall_clock_khz() -> int:
    lib = load()
    k = ctypes.c_int32(0)
    _check(lib.qc_wall_clock_khz(ctypes.byref(k)), lib)
    return k.value


def qc_plan_set_graphs(plan: Plan, on: bool = True) -> None:
    """Replay captured HIP graphs for repeated call configurations (default on)."""
    _check(plan._lib.qc_plan_set_graphs(plan.handle, int(bool(on))), plan._lib)


def qc_plan_set_fused_slice_bits(plan: Plan, b: int = -1) -> None:
    """In-flight slice bits of the fused form (0..6), or -1 to time them on
    the first fused call."""
    _check(plan._lib.qc_plan_set_fused_slice_bits(plan.handle, int(b)), plan._lib)


def qc_plan_set_fused_shape(plan: Plan, items_per_workgroup: int = 0, waves_per_item: int = 0) -> None:
    """Work-item shape of the fused form: (items per workgroup, wavefronts
    per item), one of (1,1), (2,1), (4,1), (1,2), (1,4), (1,8), (1,16);
    (0, 0) returns to the shape timed on first use."""
    _check(plan._lib.qc_plan_set_fused_shape(plan.handle, int(items_per_workgroup), int(waves_per_item)),
           plan._lib)


def qc_profile_enable(plan: Plan, on: bool = True) -> None:
    _check(plan._lib.qc_profile_enable(plan.handle, int(bool(on))), plan._lib)


def qc_profile_read(plan: Plan) -> dict:
    """{kind: (launches, total_ms, algorithmic flops, algorithmic bytes)} since
    the last read (waits for the events)."""
    stats = (qc_kernel_stat_t * 32)()
    n = ctypes.c_int32()
    _check(plan._lib.qc_profile_read(plan.handle, stats, 32, ctypes.byref(n)), plan._lib)
    return {stats[i].kind.decode(): (int(stats[i].launches), float(stats[i].total_ms), float(stats[i].flops),
                                     float(stats[i].bytes))
            for i in range(n.value)}


def qc_gate_matrix(kind: int, lib=None) -> np.ndarray:
    lib = lib or load()
    out = np.zeros(32, dtype=np.float64)
    _check(lib.qc_gate_matrix(int(kind), out.ctypes.data), lib)
    c = out[0::2] + 1j * out[1::2]
    return c.reshape(4, 4) if int(kind) == 4 else c[:4].reshape(2, 2)


def qc_workspace_bytes(plan: Plan, chunk_slices: int, n_bs: int, prec="c64") -> int:
    n = int(plan._lib.qc_workspace_bytes(plan.handle, int(chunk_slices), int(n_bs), _prec(prec)))
    if n == 0:
        raise QcError(1, plan._lib.qc_last_error().decode())
    return n


def _check_outputs(plan: Plan, n_bs: int, n_range: int, out_dev, per_slice_dev):
    import torch
    a = plan.n_amp
    if out_dev.dtype != torch.float64 or out_dev.numel() < 2 * n_bs * a or not out_dev.is_contiguous():
        raise ValueError("out_dev must be a contiguous float64 device tensor of n_bs x 2^n_open x 2")
    if per_slice_dev is not None and (per_slice_dev.dtype != torch.float64 or not per_slice_dev.is_contiguous() or
                                      per_slice_dev.numel() < 2 * n_bs * a * n_range):
        raise ValueError("per_slice_dev must be contiguous float64 with (s_end - s_begin) x n_bs x 2^n_open x 2 "
                         "entries")


def qc_contract_slices(plan: Plan, s_begin: int, s_end: int, bitstrings, prec, ws, out_dev,
                       per_slice_dev=None, stream=None):
    """Enqueues the slice range on ``stream`` (default: torch's current
    stream); ``ws``, ``out_dev`` and ``per_slice_dev`` are torch device
    tensors (out_dev float64 [n_bs, 2], accumulated into)."""
    import torch
    bs = np.ascontiguousarray(np.atleast_2d(np.asarray(bitstrings, dtype=np.uint8)))
    if bs.shape[1] != plan.n_qubits:
        raise ValueError("bitstrings must be [n_bs, n_qubits]")
    _check_outputs(plan, bs.shape[0], s_end - s_begin, out_dev, per_slice_dev)
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(plan._lib.qc_contract_slices(
        plan.handle, ctypes.c_uint64(int(s_begin)), ctypes.c_uint64(int(s_end)), bs.ctypes.data, bs.shape[0],
        _prec(prec), ws.data_ptr(), ws.numel() * ws.element_size(), st.cuda_stream, out_dev.data_ptr(),
        per_slice_dev.data_ptr() if per_slice_dev is not None else None), plan._lib)


def qc_contract_slices_dev(plan: Plan, s_begin: int, s_end: int, bits_dev, prec, ws, out_dev, per_slice_dev=None,
                           stream=None):
    """As qc_contract_slices, with ``bits_dev`` a contiguous uint8 device
    tensor [n_bs, n_qubits] already on the GPU (entries 0/1, not checked)."""
    import torch
    if bits_dev.dtype != torch.uint8 or bits_dev.dim() != 2 or bits_dev.shape[1] != plan.n_qubits \
            or not bits_dev.is_contiguous() or not bits_dev.is_cuda:
        raise ValueError("bits_dev must be a contiguous uint8 device tensor [n_bs, n_qubits]")
    n_bs = bits_dev.shape[0]
    _check_outputs(plan, n_bs, s_end - s_begin, out_dev, per_slice_dev)
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(plan._lib.qc_contract_slices_dev(
        plan.handle, ctypes.c_uint64(int(s_begin)), ctypes.c_uint64(int(s_end)), bits_dev.data_ptr(), n_bs,
        _prec(prec), ws.data_ptr(), ws.numel() * ws.element_size(), st.cuda_stream, out_dev.data_ptr(),
        per_slice_dev.data_ptr() if per_slice_dev is not None else None), plan._lib)


def qc_contract_slices_noalloc(plan: Plan, s_begin: int, s_end: int, bits_dev, prec, out_dev, per_slice_dev=None,
                               stream=None):
    """As qc_contract_slices_dev without a workspace: the library's static
    device scratch (64 MiB per GPU) serves instead, and nothing is allocated."""
    import torch
    if bits_dev.dtype != torch.uint8 or bits_dev.dim() != 2 or bits_dev.shape[1] != plan.n_qubits \
            or not bits_dev.is_contiguous() or not bits_dev.is_cuda:
        raise ValueError("bits_dev must be a contiguous uint8 device tensor [n_bs, n_qubits]")
    n_bs = bits_dev.shape[0]
    _check_outputs(plan, n_bs, s_end - s_begin, out_dev, per_slice_dev)
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(plan._lib.qc_contract_slices_noalloc(
        plan.handle, ctypes.c_uint64(int(s_begin)), ctypes.c_uint64(int(s_end)), bits_dev.data_ptr(), n_bs,
        _prec(prec), st.cuda_stream, out_dev.data_ptr(),
        per_slice_dev.data_ptr() if per_slice_dev is not None else None), plan._lib)


GEMM_FORMS = {"valu": 0, "skinny": 1, "dot": 2, "mfma11": 3, "mfma12": 4, "mfma21": 5, "mfma22": 6,
              "split_big": 7, "split11": 8, "split12": 9, "split21": 10, "split22": 11, "mfma_big": 12,
              "skinny_t": 13, "dot_tile": 14, "rows": 15, "tile256x64": 16, "tile64x256": 17, "tile32x256": 18,
              "tile256x32": 19, "tile128x64": 20, "tile64x128": 21, "tile128x32": 22, "tile32x128": 23, "mfma16": 24,
              "mfma16_t": 25, "stream": 26, "stream_t": 27, "stream16": 28,
              "split_big64": 29}


def qc_kernel_gemm(A, B, C, nb: int, m: int, n: int, k: int, a_km: bool = False, b_nk: bool = False,
                   prec="c64", scale_ws=None, stream=None, form=-1, kparts=1, scratch=None):
    """One batched complex GEMM step on torch complex64 device tensors.
    scale_ws: optional int32 device tensor of >= 3 entries (required for
    split_fp16); afterwards it holds the float bits of max(|re|,|im|) of A, B
    and C.  form: a GEMM_FORMS value fixes the kernel form (-1: default).
    kparts: split over k (MFMA and dot forms; 0 = the library's rule for the
    shape) with `scratch` a complex64 device tensor of kparts * nb * m * n
    values (allocated here when not given)."""
    import torch
    lib = load()
    for t in (A, B, C):
        if t.dtype != torch.complex64 or not t.is_contiguous():
            raise ValueError("operands must be contiguous complex64 device tensors")
    if A.numel() < nb * m * k or B.numel() < nb * k * n or C.numel() < nb * m * n:
        raise ValueError("operand too small for the GEMM shape")
    if scale_ws is not None and (scale_ws.numel() < 3 or scale_ws.element_size() != 4):
        raise ValueError("scale_ws must hold at least 3 32-bit entries")
    if scale_ws is None and _prec(prec) == PRECISIONS["split_fp16"]:
        scale_ws = torch.zeros(3, dtype=torch.int32, device=A.device)
    st = stream if stream is not None else torch.cuda.current_stream()
    if kparts == 1:
        _check(lib.qc_kernel_gemm_form(A.data_ptr(), B.data_ptr(), C.data_ptr(), nb, m, n, k, int(bool(a_km)),
                                       int(bool(b_nk)), _prec(prec), int(form),
                                       None if scale_ws is None else scale_ws.data_ptr(), st.cuda_stream), lib)
        return
    parts = kparts if kparts > 0 else int(lib.qc_gemm_kparts(nb, m, n, k))
    if scratch is None:
        scratch = torch.empty(max(1, parts * nb * m * n), dtype=torch.complex64, device=A.device)
    if scratch.dtype != torch.complex64 or scratch.numel() < parts * nb * m * n:
        raise ValueError("scratch must hold kparts * nb * m * n complex64 values")
    _check(lib.qc_kernel_gemm_kparts(A.data_ptr(), B.data_ptr(), C.data_ptr(), nb, m, n, k, int(bool(a_km)),
                                     int(bool(b_nk)), _prec(prec), int(form), int(kparts), scratch.data_ptr(),
                                     None if scale_ws is None else scale_ws.data_ptr(), st.cuda_stream), lib)


def qc_gemm_kparts(nb: int, m: int, n: int, k: int) -> int:
    """k parts the stepwise contraction uses for a GEMM step of this shape."""
    return int(load().qc_gemm_kparts(nb, m, n, k))


def qc_kernel_transpose(inp, out, rank: int, perm, stream=None):
    """Bit-permuting transpose: input bit p goes to output bit perm[p]."""
    import torch
    lib = load()
    if inp.dtype != torch.complex64 or out.dtype != torch.complex64 or inp.numel() < (1 << rank) \
            or out.numel() < (1 << rank):
        raise ValueError("operands must be complex64 device tensors of 2^rank entries")
    p = np.ascontiguousarray(np.asarray(perm, dtype=np.int32))
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib.qc_kernel_transpose(inp.data_ptr(), out.data_ptr(), int(rank), p.ctypes.data, st.cuda_stream), lib)


def qc_amplitude(plan: Plan, bitstring, prec="c64"):
    """The amplitude (complex), or for a plan with open outputs the 2^n_open
    amplitudes (complex128 array, entry o as in qc_plan_build_open)."""
    bs = np.ascontiguousarray(np.asarray(bitstring, dtype=np.uint8).reshape(-1))
    out = np.zeros(2 * plan.n_amp, dtype=np.float64)
    _check(plan._lib.qc_amplitude(plan.handle, bs.ctypes.data, _prec(prec), out.ctypes.data), plan._lib)
    if plan.n_open == 0:
        return complex(out[0], out[1])
    return out[0::2] + 1j * out[1::2]
