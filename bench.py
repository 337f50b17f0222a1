#!/usr/bin/env python3
"""Throughput of the sliced tensor-network amplitude path on one MI355X.

Headline workload: the 70-qubit diamond lattice at depth 1+32+1 (seed 401,
one bitstring), sliced into 2^20 slices of at most 2^30 entries.  One step =
one qc_contract_slices_dev call over a chunk of consecutive slices (64 in
flight): leaf instantiation, every pairwise contraction step, the FP64
cross-slice sum, inputs resident on the device.  A whole amplitude is 2^20
such slices; as in the paper's own extrapolation from subtask times, the
amplitude rate is projected as slices/s / 2^20 (every slice has the same
program and cost).

Prints ONE JSON line: projected amplitudes/s (value) and slices/s in complex
FP32, the same for split FP16 and split BF16 beside it (speedup), the
roofline of the dominant kernel (its algorithmic flops per launch / its
average launch time, from HIP events the library records on the call's
stream), the error of the timed chunk's slice values against the FP64 oracle
(O4), and the oracle's own CPU rate on the host cores (per-slice time on the
same slices, projected to 2^20 slices).  The other workloads (4x4, 5x5, 7x7,
the request batch) follow as extra keys.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "amplitudes/sec and contraction TFLOP/s vs MFMA peak, FP32 vs split-FP16 at stated rel err"
PEAK_FP32_TFLOPS = 157.3      # MI355X FP32 (vector and matrix)
PEAK_MFMA_TFLOPS = {"c64": PEAK_FP32_TFLOPS, "split_bf16": 2500.0, "split_fp16": 2500.0}
HW_PER_ALG = {"c64": 1.0, "split_bf16": 3.0, "split_fp16": 3.0}   # hardware flops per algorithmic flop
PEAK_HBM_GBS = 8000.0
TOL = {"c64": 1e-5, "split_fp16": 1e-4, "split_bf16": 1e-3}
MFMA_KINDS = {"gemm_mfma", "gemm_split_fp16", "gemm_split_bf16"}


def _say(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _events_ms(stream, fn, reps):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _kernels_hash():
    src = open(os.path.join(ROOT, "paper_1907_11217_amd", "csrc", "kernels.hip"), "rb").read()
    return hashlib.sha256(src).hexdigest()[:16]


def _traffic(kind, workload, prec):
    """HBM bytes per launch of `kind` from the committed counter runs
    (profiles/traffic.json: FETCH_SIZE and WRITE_SIZE per launch, each scaled
    by the same counter on a plain copy), or None if they were taken on
    another workload or precision, or before the kernel source last changed."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[f"{kind}|{workload}|{prec}"]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("kernels_hip_sha256_16") != _kernels_hash():
        return None
    return 1024.0 * (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"])


def _roofline(prof, prec, workload):
    """The dominant kernel kind (most time) of a profiled loop: its algorithmic
    flops and bytes as the library counts them per launch, over the summed
    launch time (HIP events on the call's stream).  It is MFMA-bound when its
    flops at the dtype's MFMA peak take longer than its bytes at the HBM
    peak, else HBM-bound; `frac` is the achieved rate over that peak."""
    dom = max(prof, key=lambda kk: prof[kk][1])
    launches, total_ms, flops, nbytes = prof[dom]
    # The 16-bit kinds multiply three hardware products per algorithmic one
    # against the 16-bit peak; every other kind (the complex FP32 MFMA forms
    # included, also inside a split program) computes in FP32.
    hw = HW_PER_ALG[prec] if dom.startswith("gemm_split") else 1.0
    peak_f = PEAK_MFMA_TFLOPS[prec] if dom.startswith("gemm_split") else PEAK_FP32_TFLOPS
    t_f = flops * hw / (peak_f * 1e12)
    t_b = nbytes / (PEAK_HBM_GBS * 1e9)
    sec = total_ms * 1e-3
    if t_f >= t_b:
        r = {"bound": "mfma" if dom in MFMA_KINDS else "alu", "achieved": flops * hw / sec / 1e12, "peak": peak_f,
             "unit": "TFLOP/s"}
    else:
        r = {"bound": "hbm", "achieved": nbytes / sec / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    r["frac"] = r["achieved"] / r["peak"]
    r.update({"traffic": _traffic(dom, workload, prec), "kernel": dom, "launches": launches,
              "avg_launch_ms": total_ms / launches, "flops_per_launch": flops / launches,
              "bytes_per_launch": nbytes / launches, "tflops_alg": flops / sec / 1e12, "gbs_alg": nbytes / sec / 1e9,
              "roofline_time_frac": max(t_f, t_b) / sec,
              "flops_counted": "hardware (3 per algorithmic) for split forms" if hw > 1
              else "algorithmic (8 per complex multiply-add)"})
    return r


def _hbm_kind(prof, kind):
    """Achieved algorithmic HBM rate of one kernel kind (bytes each launch must
    read and write, over its HIP-event time) against the 8 TB/s peak."""
    if kind not in prof or prof[kind][1] <= 0 or prof[kind][3] <= 0:
        return None
    launches, total_ms, _, nbytes = prof[kind]
    gbs = nbytes / (total_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": kind, "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": gbs / PEAK_HBM_GBS, "launches": launches, "bytes_per_launch": nbytes / launches,
            "avg_launch_ms": total_ms / launches}


def _kernel_table(prof, steps):
    return {kk: {"launches_per_step": v[0] / steps, "ms_per_step": v[1] / steps,
                 "tflops_alg": (v[2] / (v[1] * 1e-3) / 1e12) if v[1] > 0 and v[2] > 0 else None,
                 "gbs_alg": (v[3] / (v[1] * 1e-3) / 1e9) if v[1] > 0 and v[3] > 0 else None}
            for kk, v in prof.items()}


def _split_share(prof):
    """Share of the GEMM steps' algorithmic flops that ran on 16-bit MFMA
    (split kinds); the rest ran in complex FP32 (smaller steps, and steps the
    tuner measured faster in FP32)."""
    gemm = sum(v[2] for kk, v in prof.items() if kk.startswith("gemm") or kk == "micro")
    split = sum(v[2] for kk, v in prof.items() if kk.startswith("gemm_split"))
    return split / gemm if gemm > 0 else None


def _cpu_info():
    import torch
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cores": torch.get_num_threads(), "cpu_model": model}


def _slice_errors(got, ref, tol):
    """Per-slice error rule of the parity tests: |v - v_ref| / max(|v_ref|, rms)
    over the slices, rms of the nonzero reference values."""
    import numpy as np
    got, ref = np.asarray(got), np.asarray(ref)
    nz = np.abs(ref) > 0
    if not nz.any():
        return None
    rms = np.sqrt(np.mean(np.abs(ref[nz]) ** 2))
    e = np.abs(got - ref) / np.maximum(np.abs(ref), rms)
    return {"max": float(e.max()), "tol": tol, "nonzero_slices": int(nz.sum()), "slices": int(len(ref))}


# ---------------------------------------------------------------- headline
def diamond_leg(steps, warmup, precs, chunk=None, cpu=True, tune_cache=None):
    """The 70-qubit depth 1+32+1 workload: a chunk of consecutive slices per
    step, each precision timed over `steps` steps after `warmup` (the first
    call of a configuration captures its graph), then `min(steps, 5)` steps
    again with kernel timing on for the roofline."""
    import numpy as np
    import torch

    import synth
    from paper_1907_11217_amd import qcsim

    lat, circ, bs, spec = synth.config("c4")
    chunk = chunk or spec["chunk"]
    t0 = time.perf_counter()
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=spec["log2_slices"],
                               log2_max_entries=spec["log2_cap"], greedy_trials=spec["trials"],
                               seed=spec["plan_seed"])
    plan_s = time.perf_counter() - t0
    info = qcsim.qc_plan_info(plan)
    k = info["log2_slices"]
    _say(f"70-qubit plan: 2^{k} slices, {info['flops_per_slice']:.3e} flops per slice ({plan_s:.1f} s)")
    stream = torch.cuda.current_stream()
    bits = torch.from_numpy(np.ascontiguousarray(bs[:1])).cuda()
    out = torch.zeros(1, 2, dtype=torch.float64, device="cuda")
    ps = torch.zeros(chunk, 1, 2, dtype=torch.float64, device="cuda")
    # The timed chunk: among the chunks holding slices drawn from the seed + 2
    # stream, the first with a nonzero slice value (about half of this plan's
    # slices are exactly zero; the time per slice does not depend on values).
    ws = torch.empty(qcsim.qc_workspace_bytes(plan, chunk, 1, "c64"), dtype=torch.uint8, device="cuda")
    c0 = None
    for s in synth.random_slices(k, 8, spec["seed"] + 2):
        c = int(s) - int(s) % chunk
        out.zero_()
        qcsim.qc_contract_slices_dev(plan, c, c + chunk, bits, "c64", ws, out, ps, stream=stream)
        torch.cuda.synchronize()
        if c0 is None:
            c0 = c
        if ps.abs().max().item() > 0:
            c0 = c
            break
    del ws
    leg = {"workload": (f"{spec['name']}: {lat.n}-qubit diamond (8x9 grid without two corners), depth 1+"
                        f"{spec['depth']}+1, circuit seed {spec['seed']}, bitstring seed {spec['seed'] + 1}; "
                        f"2^{k} slices (cap 2^{spec['log2_cap']} entries), {chunk} slices [{c0}, {c0 + chunk}) "
                        f"per step"),
           "log2_slices": k, "slices_per_step": chunk, "chunk_start": c0, "plan_seconds": plan_s,
           "log2_max_entries": info["log2_max_entries"], "flops_per_slice": info["flops_per_slice"],
           "flops_per_amplitude": info["flops_per_slice"] * float(1 << k),
           "flops_unsliced": info["flops_unsliced"],
           "slicing_overhead": info["flops_per_slice"] * float(1 << k) / max(info["flops_unsliced"], 1.0),
           "folded_steps": info["n_folded_steps"], "flops_folded_once": info["flops_folded"],
           "per_prec": {}}
    vals = {}
    for prec in precs:
        ws = torch.empty(qcsim.qc_workspace_bytes(plan, chunk, 1, prec), dtype=torch.uint8, device="cuda")
        t1 = time.perf_counter()
        n_timed = qcsim.qc_tune(plan, chunk, 1, prec, ws, cache_path=tune_cache, stream=stream)   # untimed
        torch.cuda.synchronize()
        tune_s = time.perf_counter() - t1

        def step():
            qcsim.qc_contract_slices_dev(plan, c0, c0 + chunk, bits, prec, ws, out, stream=stream)

        for _ in range(max(1, warmup)):
            step()
        ms = _events_ms(stream, step, steps)
        qcsim.qc_profile_read(plan)
        qcsim.qc_profile_enable(plan, True)
        n_prof = min(steps, 5)
        ms_prof = _events_ms(stream, step, n_prof)
        qcsim.qc_profile_enable(plan, False)
        prof = qcsim.qc_profile_read(plan)
        out.zero_()
        qcsim.qc_contract_slices_dev(plan, c0, c0 + chunk, bits, prec, ws, out, ps, stream=stream)
        torch.cuda.synchronize()
        p = ps.cpu().numpy()[:, 0]
        vals[prec] = p[:, 0] + 1j * p[:, 1]
        flops_step = info["flops_per_slice"] * chunk
        leg["per_prec"][prec] = {
            "ms_per_step": ms, "slices_per_s": chunk / (ms * 1e-3),
            "projected_amplitudes_per_s": chunk / (ms * 1e-3) / float(1 << k),
            "projected_s_per_amplitude": ms * 1e-3 * float(1 << k) / chunk,
            "tflops_alg": flops_step / (ms * 1e-3) / 1e12, "ms_per_step_profiled": ms_prof,
            "kernels": _kernel_table(prof, n_prof), "roofline": _roofline(prof, prec, "diamond70_d32"),
            "transpose_hbm": _hbm_kind(prof, "transpose"), "gemm_flop_share_16bit": _split_share(prof),
            "tune_seconds": tune_s, "shapes_timed": n_timed}
        _say(f"70-qubit {prec}: {ms:.2f} ms per {chunk} slices")
        del ws
    c64 = leg["per_prec"].get("c64")
    for prec in precs:
        if prec != "c64" and c64:
            leg["per_prec"][prec]["speedup_over_c64"] = c64["ms_per_step"] / leg["per_prec"][prec]["ms_per_step"]
            leg["per_prec"][prec]["slice_diff_vs_c64"] = _slice_errors(vals[prec], vals["c64"], TOL[prec])
    if cpu:
        # The oracle (O4: the hypergraph network along this plan's tree, read
        # as data, complex128 on the host cores) on the timed chunk's slices:
        # the reference for the slice errors and the CPU baseline.
        import oracle
        tree = qcsim.qc_plan_export_tree(plan)
        segs = qcsim.qc_plan_sliced_segments(plan)
        ref, secs = [], []
        for s in range(c0, c0 + chunk):
            t1 = time.perf_counter()
            ref.append(oracle.hyper_value(lat.n, circ, bs[0], segs, s, tree))
            secs.append(time.perf_counter() - t1)
        for prec in precs:
            leg["per_prec"][prec]["slice_err_vs_oracle"] = _slice_errors(vals[prec], ref, TOL[prec])
        med = float(np.median(secs))
        _say(f"70-qubit oracle: {med:.2f} s per slice")
        # One host thread, for a per-core figure (the paper quotes per-vCPU
        # work): two slices of the same chunk.
        n_threads = torch.get_num_threads()
        torch.set_num_threads(1)
        t1 = time.perf_counter()
        for s in range(c0, c0 + 2):
            oracle.hyper_value(lat.n, circ, bs[0], segs, s, tree)
        one = (time.perf_counter() - t1) / 2
        torch.set_num_threads(n_threads)
        _say(f"70-qubit oracle, one thread: {one:.2f} s per slice")
        leg["cpu_oracle"] = dict(seconds_per_slice=med, projected_s_per_amplitude=med * float(1 << k), **_cpu_info(),
                                 seconds_per_slice_one_thread=one,
                                 projected_core_s_per_amplitude=one * float(1 << k),
                                 sample=f"O4 on the {chunk} slices of the timed chunk ({sum(secs):.1f} s); one "
                                        f"thread: 2 of them")
    return leg


# ------------------------------------------------------------ extra legs
def open_leg(steps=3, warmup=1, precs=("c64", "split_fp16"), cpu=True):
    """The 70-qubit depth 1+32+1 circuit with its last 16 output qubits left
    open (qc_plan_build_open): every slice contraction yields 2^16 amplitude
    contributions, so one pass over the 2^20 slices gives 65536 amplitudes
    (the bitstrings that differ from the drawn one only in those qubits).
    One step = one call over a chunk of consecutive slices; amplitudes/s is
    projected as 2^16 x slices/s / 2^20.  Checked against O4 on the two
    largest entries of the chunk's first nonzero slice (the oracle fixes the
    open qubits to those entries' bits)."""
    import numpy as np
    import torch

    import synth
    from paper_1907_11217_amd import qcsim

    lat, circ, bs, spec = synth.config("c4o")
    oq, chunk, m = spec["open_qubits"], spec["chunk"], spec["n_open"]
    t0 = time.perf_counter()
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=spec["log2_slices"], log2_max_entries=spec["log2_cap"],
                               greedy_trials=spec["trials"], seed=spec["plan_seed"], open_qubits=oq)
    plan_s = time.perf_counter() - t0
    info = qcsim.qc_plan_info(plan)
    k = info["log2_slices"]
    _say(f"70-qubit open: 2^{k} slices, {info['flops_per_slice']:.3e} flops per slice ({plan_s:.1f} s)")
    stream = torch.cuda.current_stream()
    bits = torch.from_numpy(np.ascontiguousarray(bs[:1])).cuda()
    A = 1 << m
    out = torch.zeros(1, A, 2, dtype=torch.float64, device="cuda")
    ps = torch.zeros(chunk, 1, A, 2, dtype=torch.float64, device="cuda")
    # The timed chunk: the first chunk around a slice drawn from the seed + 2
    # stream that holds a nonzero slice (most slices of this plan are exact
    # zeros; the time does not depend on the values).
    ws = torch.empty(qcsim.qc_workspace_bytes(plan, chunk, 1, "c64"), dtype=torch.uint8, device="cuda")
    c0 = None
    for s in synth.random_slices(k, 16, spec["seed"] + 2):
        c = int(s) - int(s) % chunk
        qcsim.qc_contract_slices_dev(plan, c, c + chunk, bits, "c64", ws, out, ps, stream=stream)
        torch.cuda.synchronize()
        c0 = c if c0 is None else c0
        if ps.abs().max().item() > 0:
            c0 = c
            break
    del ws
    leg = {"workload": (f"{spec['name']}: the 70-qubit diamond at depth 1+{spec['depth']}+1 (seed {spec['seed']}, "
                        f"bitstring seed {spec['seed'] + 1}) with the outputs of qubits {oq[0]}..{oq[-1]} open; "
                        f"2^{k} slices (cap 2^{spec['log2_cap']}), {chunk} slices [{c0}, {c0 + chunk}) per step, "
                        f"2^{m} amplitudes per contraction"),
           "open_qubits": len(oq), "log2_slices": k, "slices_per_step": chunk, "plan_seconds": plan_s,
           "log2_max_entries": info["log2_max_entries"], "flops_per_slice": info["flops_per_slice"],
           "flops_per_amplitude": info["flops_per_slice"] * float(1 << k) / A, "per_prec": {}}
    vals = {}
    for prec in precs:
        ws = torch.empty(qcsim.qc_workspace_bytes(plan, chunk, 1, prec), dtype=torch.uint8, device="cuda")
        qcsim.qc_tune(plan, chunk, 1, prec, ws, stream=stream)   # untimed

        def step():
            qcsim.qc_contract_slices_dev(plan, c0, c0 + chunk, bits, prec, ws, out, stream=stream)

        for _ in range(max(1, warmup)):
            step()
        ms = _events_ms(stream, step, steps)
        qcsim.qc_profile_read(plan)
        qcsim.qc_profile_enable(plan, True)
        ms_prof = _events_ms(stream, step, 1)
        qcsim.qc_profile_enable(plan, False)
        prof = qcsim.qc_profile_read(plan)
        out.zero_()
        qcsim.qc_contract_slices_dev(plan, c0, c0 + chunk, bits, prec, ws, out, ps, stream=stream)
        torch.cuda.synchronize()
        p = ps.cpu().numpy()[:, 0]
        vals[prec] = p[..., 0] + 1j * p[..., 1]
        leg["per_prec"][prec] = {
            "ms_per_step": ms, "slices_per_s": chunk / (ms * 1e-3),
            "projected_amplitudes_per_s": A * chunk / (ms * 1e-3) / float(1 << k),
            "projected_s_per_amplitude": ms * 1e-3 * float(1 << k) / chunk / A,
            "tflops_alg": info["flops_per_slice"] * chunk / (ms * 1e-3) / 1e12, "ms_per_step_profiled": ms_prof,
            "kernels": _kernel_table(prof, 1), "roofline": _roofline(prof, prec, "diamond70_d32_open16"),
            "gemm_flop_share_16bit": _split_share(prof)}
        _say(f"70-qubit open {prec}: {ms:.1f} ms per {chunk} slices")
        del ws
    c64 = leg["per_prec"].get("c64")
    for prec in precs:
        if prec != "c64" and c64:
            leg["per_prec"][prec]["speedup_over_c64"] = c64["ms_per_step"] / leg["per_prec"][prec]["ms_per_step"]
            leg["per_prec"][prec]["slice_diff_vs_c64"] = _slice_errors(vals[prec].reshape(-1),
                                                                       vals["c64"].reshape(-1), TOL[prec])
    if cpu:
        import oracle
        v = vals[precs[0]]
        nz = [j for j in range(chunk) if np.abs(v[j]).max() > 0]
        if nz:
            j = nz[0]
            top = np.argsort(-np.abs(v[j]))[:2]
            tree = qcsim.qc_plan_export_tree(plan)
            segs = qcsim.qc_plan_sliced_segments(plan)
            ref, secs = [], []
            for o in top:
                y = bs[0].copy()
                for i, q in enumerate(oq):
                    y[q] = (int(o) >> (m - 1 - i)) & 1
                t1 = time.perf_counter()
                ref.append(oracle.hyper_value(lat.n, circ, y, segs, c0 + j, tree))
                secs.append(time.perf_counter() - t1)
            rms = float(np.sqrt(np.mean(np.abs(v[j]) ** 2)))
            for prec in precs:
                got = vals[prec][j][top]
                leg["per_prec"][prec]["err_vs_oracle"] = {
                    "max_rel": float(np.max(np.abs(got - np.array(ref)) / np.abs(np.array(ref)))),
                    "values": 2, "slice": c0 + j, "tol": TOL[prec], "slice_rms": rms}
            med = float(np.median(secs))
            _say(f"70-qubit open oracle: {med:.1f} s per value")
            leg["cpu_oracle"] = dict(seconds_per_value=med, projected_s_per_amplitude=med * float(1 << k),
                                     **_cpu_info(), sample="O4 on 2 entries of one slice (one open setting each)")
    return leg


def fused_leg(steps=50, warmup=10, cpu=True):
    """The 5x5 depth 1+16+1 workload: every one of its 2^6 slices for all 64
    bitstrings per step, fused form (one launch per call plus the sums)."""
    import numpy as np
    import torch

    import synth
    from paper_1907_11217_amd import qcsim

    lat, circ, bs, spec = synth.config("c2")
    n_bs = len(bs)
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=spec["log2_slices"], greedy_trials=spec["trials"],
                               seed=spec["plan_seed"], quick=spec.get("quick", False))
    n_slices = 1 << qcsim.qc_plan_info(plan)["log2_slices"]
    ws = torch.empty(qcsim.qc_workspace_bytes(plan, n_slices, n_bs), dtype=torch.uint8, device="cuda")
    out = torch.zeros(n_bs, 2, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    bits = torch.from_numpy(np.ascontiguousarray(bs)).cuda()

    def step():
        qcsim.qc_contract_slices_dev(plan, 0, n_slices, bits, "c64", ws, out, stream=stream)

    for _ in range(warmup):
        step()
    ms = _events_ms(stream, step, steps)
    n_prof = 10
    qcsim.qc_profile_read(plan)
    qcsim.qc_profile_enable(plan, True)
    _events_ms(stream, step, n_prof)
    qcsim.qc_profile_enable(plan, False)
    prof = qcsim.qc_profile_read(plan)
    out.zero_()
    step()
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    amps = o[:, 0] + 1j * o[:, 1]
    fb = max(qcsim.qc_plan_describe(plan, 0, 0)["fused_slice_bits"], 0)
    item = qcsim.qc_plan_describe(plan, fb, 0)
    leg = {"workload": f"{spec['name']}: {lat.n} qubits, depth 1+{spec['depth']}+1, 2^6 slices, {n_bs} bitstrings",
           "ms_per_step": ms, "amplitudes_per_s": n_bs / (ms * 1e-3), "slices_per_s": n_slices * n_bs / (ms * 1e-3),
           "fused_slice_bits": fb, "fused_items_per_workgroup": item["fused_pairs"],
           "fused_waves_per_item": item["fused_waves"], "fused_flops_per_item": item["flops"],
           "kernels": {kk: {"launches_per_step": v[0] / n_prof, "avg_ms": v[1] / v[0]} for kk, v in prof.items()}}
    if "fused" in prof:
        launches, total_ms = prof["fused"][:2]
        items_per_launch = (n_slices >> fb) * n_bs
        ach = item["flops"] * items_per_launch / (total_ms / launches * 1e-3) / 1e12
        leg["fused_roofline"] = {"bound": "alu", "achieved": ach, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                                 "frac": ach / PEAK_FP32_TFLOPS, "avg_launch_ms": total_ms / launches}
    if cpu:
        import oracle
        t0 = time.perf_counter()
        psi = oracle.statevector(lat.n, circ)
        cpu_s = time.perf_counter() - t0
        ref = np.array([psi[oracle.index_of(x)] for x in bs])
        mask = (1 << lat.n) * np.abs(ref) ** 2 >= 1e-2
        leg["rel_err"] = {"max_rel": float((np.abs(amps - ref)[mask] / np.abs(ref[mask])).max()),
                          "norm_rel": float(np.linalg.norm(amps - ref) / np.linalg.norm(ref)), "tol": 1e-5}
        leg["cpu_oracle"] = {"seconds": cpu_s, "amplitudes_per_s": n_bs / cpu_s,
                             "sample": f"one FP64 state-vector run (2^{lat.n} entries, OpenMP C)",
                             "threads": int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))}
    return leg


def small_leg(reps=200):
    """The 4x4 depth-10 workload: one amplitude (no slicing), latency per call
    with the bitstring resident, against the oracle's state vector (timed
    with the host's threads, and in NumPy on one thread)."""
    import numpy as np
    import torch

    import oracle
    import synth
    from paper_1907_11217_amd import qcsim

    lat, circ, bs, spec = synth.config("c1")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=0, greedy_trials=spec["trials"],
                               seed=spec["plan_seed"])
    dbits = torch.from_numpy(np.ascontiguousarray(bs[:1], dtype=np.uint8)).cuda()
    ws = torch.empty(qcsim.qc_workspace_bytes(plan, 1, 1), dtype=torch.uint8, device="cuda")
    out = torch.zeros(1, 2, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        qcsim.qc_contract_slices_dev(plan, 0, 1, dbits, "c64", ws, out, stream=stream)

    step()  # the first fused call times the work-item shapes (untimed preparation)
    ms = _events_ms(stream, step, reps)
    out.zero_()
    step()
    torch.cuda.synchronize()
    got = complex(*out.cpu().numpy()[0])
    t1 = time.perf_counter()
    ref = complex(oracle.amplitudes_sv(lat.n, circ, bs[:1])[0])
    cpu_s = time.perf_counter() - t1
    t1 = time.perf_counter()
    oracle.statevector(lat.n, circ, impl="numpy")
    cpu_1 = time.perf_counter() - t1
    return {"workload": f"{spec['name']}: {lat.n} qubits, depth 1+{spec['depth']}+1, no slicing, 1 bitstring",
            "us_per_amplitude": ms * 1e3, "amplitudes_per_s": 1.0 / (ms * 1e-3),
            "abs_err": abs(got - ref), "abs_ref": abs(ref),
            "cpu_oracle": {"seconds": cpu_s, "seconds_one_thread_numpy": cpu_1,
                           "sample": "one state-vector run of the same circuit"}}


def grid7_leg(precs, reps=5, cpu=True):
    """The 7x7 depth 1+24+1 workload: every one of its 2^16 slices of one
    amplitude per step (one chunk), per precision, against O4 on the 32
    sampled slices of the seed + 2 stream."""
    import numpy as np
    import torch

    import synth
    from paper_1907_11217_amd import qcsim

    lat, circ, bs, spec = synth.config("c3")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=spec["log2_slices"], log2_max_entries=spec["log2_cap"],
                               greedy_trials=spec["trials"], seed=spec["plan_seed"])
    info = qcsim.qc_plan_info(plan)
    k = info["log2_slices"]
    n = 1 << k
    stream = torch.cuda.current_stream()
    bits = torch.from_numpy(np.ascontiguousarray(bs[:1])).cuda()
    out = torch.zeros(1, 2, dtype=torch.float64, device="cuda")
    ps = torch.zeros(n, 1, 2, dtype=torch.float64, device="cuda")
    picks = [int(s) for s in synth.random_slices(k, spec["n_sampled"], spec["seed"] + 2)]
    leg = {"workload": f"{spec['name']}: {lat.n} qubits, depth 1+{spec['depth']}+1, all 2^{k} slices of one amplitude",
           "flops_per_amplitude": info["flops_per_slice"] * n, "flops_unsliced": info["flops_unsliced"],
           "folded_steps": info["n_folded_steps"], "flops_folded_once": info["flops_folded"], "per_prec": {}}
    vals = {}
    for prec in precs:
        ws = torch.empty(qcsim.qc_workspace_bytes(plan, n, 1, prec), dtype=torch.uint8, device="cuda")
        qcsim.qc_tune(plan, n, 1, prec, ws, stream=stream)

        def step():
            qcsim.qc_contract_slices_dev(plan, 0, n, bits, prec, ws, out, stream=stream)

        step()
        ms = _events_ms(stream, step, reps)
        qcsim.qc_profile_read(plan)
        qcsim.qc_profile_enable(plan, True)
        _events_ms(stream, step, 2)
        qcsim.qc_profile_enable(plan, False)
        prof = qcsim.qc_profile_read(plan)
        qcsim.qc_contract_slices_dev(plan, 0, n, bits, prec, ws, out, ps, stream=stream)
        torch.cuda.synchronize()
        p = ps.cpu().numpy()[:, 0]
        vals[prec] = p[:, 0] + 1j * p[:, 1]
        leg["per_prec"][prec] = {"ms_per_amplitude": ms, "slices_per_s": n / (ms * 1e-3),
                                 "tflops_alg": info["flops_per_slice"] * n / (ms * 1e-3) / 1e12,
                                 "kernels": _kernel_table(prof, 2), "roofline": _roofline(prof, prec, "grid7x7_d24")}
        del ws
    for prec in precs:
        if prec != "c64" and "c64" in leg["per_prec"]:
            leg["per_prec"][prec]["speedup_over_c64"] = (leg["per_prec"]["c64"]["ms_per_amplitude"] /
                                                         leg["per_prec"][prec]["ms_per_amplitude"])
    if cpu:
        import oracle
        tree = qcsim.qc_plan_export_tree(plan)
        segs = qcsim.qc_plan_sliced_segments(plan)
        ref, secs = [], []
        for s in picks:
            t1 = time.perf_counter()
            ref.append(oracle.hyper_value(lat.n, circ, bs[0], segs, s, tree))
            secs.append(time.perf_counter() - t1)
        for prec in precs:
            leg["per_prec"][prec]["slice_err_vs_oracle"] = _slice_errors(vals[prec][picks], ref, TOL[prec])
        med = float(np.median(secs))
        leg["cpu_oracle"] = {"seconds_per_slice": med, "projected_s_per_amplitude": med * n,
                             "sample": f"O4 on {len(picks)} sampled slices"}
    return leg


def batch_leg(n_req=256, seed=501, cap=24, reps=3, n_oracle=6, trials=32, precs=("c64", "split_fp16")):
    """Uneven batch of requests (4x4 d12, 5x5 d16, 6x6 d20, 7x7 d24 drawn
    uniformly), each with its own plan (its drawn slice count 2^0..2^12, more
    where the 2^cap-entry cap needs it) and bitstring, in one
    qc_contract_batch call per step; the stepwise requests' GEMM forms are
    tuned beforehand (untimed, like the plan build)."""
    import numpy as np
    import torch

    import synth
    from paper_1907_11217_amd import qcsim

    from concurrent.futures import ThreadPoolExecutor

    reqs = synth.request_mix(n_req, seed)
    t0 = time.perf_counter()

    def build(r):
        lat = r["lattice"]
        # Orders from the greedy restarts alone (quick search): the full
        # search's subtree reconfiguration costs ~20 core-seconds per 7x7
        # plan, which for 256 plans would dominate the run.
        return qcsim.qc_plan_build(lat.n, r["circuit"], r["bitstring"], log2_slices=r["log2_slices"],
                                   log2_max_entries=cap, greedy_trials=trials, seed=1, quick=True)

    # Plans are independent host work (untimed): eight at a time, each
    # call releasing the interpreter while the library searches.
    plans = []
    with ThreadPoolExecutor(max_workers=8) as pool:
        for i, plan in enumerate(pool.map(build, reqs)):
            plans.append(plan)
            if (i + 1) % 64 == 0:
                _say(f"request batch: {i + 1} of {n_req} plans built")
    ks = [qcsim.qc_plan_info(p)["log2_slices"] for p in plans]
    items = [(p, r["bitstring"]) for p, r in zip(plans, reqs)]
    plan_s = time.perf_counter() - t0
    batch = qcsim.Batch(items)
    stream = torch.cuda.current_stream()
    khz = qcsim.qc_wall_clock_khz()
    leg = {"workload": (f"{n_req} requests drawn uniformly from 4x4 d12 / 5x5 d16 / 6x6 d20 / 7x7 d24 "
                        f"(seed {seed}), one bitstring each, 2^0..2^12 slices each (drawn), plans capped at 2^{cap} "
                        f"entries, quick order search ({trials} greedy restarts, no reconfiguration)"),
           "plan_seconds": plan_s, "per_prec": {}}
    fam_of = ["%dx%d_d%d" % r["family"] for r in reqs]
    leg["families"] = {f: {"count": fam_of.count(f), "k": sorted({k for g, k in zip(fam_of, ks) if g == f})}
                       for f in sorted(set(fam_of))}
    ref = None
    for prec in precs:
        t1 = time.perf_counter()
        chunk = [1 << min(k, 12) for k in ks]
        tws = torch.empty(max(qcsim.qc_workspace_bytes(p, c, 1, prec) for (p, _), c in zip(items, chunk)),
                          dtype=torch.uint8, device="cuda")
        n_timed = sum(qcsim.qc_tune(p, c, 1, prec, tws, stream=stream) for (p, _), c in zip(items, chunk))
        torch.cuda.synchronize()
        del tws
        tune_s = time.perf_counter() - t1
        ws = torch.empty(qcsim.qc_batch_workspace_bytes(batch, prec), dtype=torch.uint8, device="cuda")
        out = torch.zeros(n_req, 2, dtype=torch.float64, device="cuda")
        tdone = torch.zeros(n_req + 1, dtype=torch.int64, device="cuda")
        qcsim.qc_contract_batch(batch, prec, ws, out, tdone, stream=stream)  # first call: graphs
        torch.cuda.synchronize()
        o = out.cpu().numpy().copy()
        amps = o[:, 0] + 1j * o[:, 1]

        def step():
            qcsim.qc_contract_batch(batch, prec, ws, out, tdone, stream=stream)

        ms = _events_ms(stream, step, reps)
        step()
        torch.cuda.synchronize()
        t = tdone.cpu().numpy()
        done_ms = (t[:-1] - t[-1]) / khz
        r = {"ms_per_batch": ms, "amplitudes_per_s": n_req / (ms * 1e-3), "tune_seconds": tune_s,
             "shapes_timed": n_timed,
             "completion_ms": {"p50": float(np.percentile(done_ms, 50)), "p99": float(np.percentile(done_ms, 99)),
                               "max": float(done_ms.max())},
             "family_max_completion_ms": {f: float(max(d for g, d in zip(fam_of, done_ms) if g == f))
                                          for f in sorted(set(fam_of))}}
        if ref is None:
            ref = amps
            import oracle
            errs = []
            for i, q in enumerate(reqs):
                if len(errs) >= n_oracle:
                    break
                if q["family"][0] <= 5:
                    a = oracle.amplitudes_sv(q["lattice"].n, q["circuit"], [q["bitstring"]])[0]
                    errs.append(abs(amps[i] - a) / abs(a))
            r["oracle_rel_err_small_requests"] = {"n": len(errs), "max": float(max(errs))}
        else:
            n_q = np.array([q["lattice"].n for q in reqs], dtype=float)
            gate = np.exp2(n_q) * np.abs(ref) ** 2 >= 1e-2
            r["max_rel_diff_vs_c64"] = float((np.abs(amps - ref)[gate] / np.abs(ref[gate])).max())
        leg["per_prec"][prec] = r
        del ws
    return leg


def _headline_program(prec):
    """The 70-qubit plan and its 64-slice program's step list (host only)."""
    import synth
    from paper_1907_11217_amd import qcsim

    lat, circ, bs, spec = synth.config("c4")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=spec["log2_slices"], log2_max_entries=spec["log2_cap"],
                               greedy_trials=spec["trials"], seed=spec["plan_seed"])
    b = spec["chunk"].bit_length() - 1
    return qcsim.qc_plan_export_steps(plan, b, 0), qcsim.qc_plan_describe(plan, b, 0, prec)


def trace_summary(path, prec):
    """Per-step table of the last complete 64-slice call in a rocprofv3
    kernel trace (CSV) of the 70-qubit workload: each launch matched to its
    step in program order, with the step's shape, kernel, time and the time
    its algorithmic flops and bytes take at the chip's peaks."""
    import csv
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Start_Timestamp"]))
    names = [r["Kernel_Name"] for r in rows]
    i0 = max(i for i, nm in enumerate(names) if "leaf_kernel" in nm)
    if i0 > 0 and "zero_u32" in names[i0 - 1]:
        i0 -= 1
    i1 = next(i for i in range(i0, len(names)) if "reduce64" in names[i] or "block_add" in names[i])
    call = rows[i0:i1 + 1]
    steps, desc = _headline_program(prec)
    peak_f = PEAK_MFMA_TFLOPS[prec] * 1e12
    dur = lambda r: (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
    k = next(i for i, r in enumerate(call) if "micro_kernel" in r["Kernel_Name"]) + 1
    lines, tot, roof_tot = [], 0.0, 0.0
    for i, st in enumerate(steps):
        if st["micro"]:
            continue
        r = call[k]
        k += 1
        t = dur(r)
        if k < len(call) and "ksum" in call[k]["Kernel_Name"]:
            t += dur(call[k])
            k += 1
        if st["kind"] == 0:
            by = 16.0 * st["m"]
            roof = by / (PEAK_HBM_GBS * 1e9) * 1e6
            shape = f"transpose 2^{st['m'].bit_length() - 1}"
        else:
            nb, m, n, kk = st["nb"], st["m"], st["n"], st["k"]
            f = 8.0 * nb * m * n * kk
            by = 8.0 * nb * (m * kk + kk * n + m * n)
            hw = HW_PER_ALG[prec] if "split" in r["Kernel_Name"] else 1.0
            pf = peak_f if "split" in r["Kernel_Name"] or prec == "c64" else PEAK_FP32_TFLOPS * 1e12
            roof = max(f * hw / pf, by / (PEAK_HBM_GBS * 1e9)) * 1e6
            op = desc["ops"][i]
            shape = f"{nb}x{m}x{n}x{kk}{' scat' if op['c_nat'] != op['c'] else ''}"
        name = r["Kernel_Name"].replace("void ", "").replace("qc::", "").split("(")[0]
        lines.append(f"  {i:4d} {shape:32s} {name[:44]:44s} {t:9.1f} us  roof {roof:8.1f} us  {roof / t:6.1%}")
        tot += t
        roof_tot += roof
    span = (int(call[-1]["End_Timestamp"]) - int(call[0]["Start_Timestamp"])) * 1e-3
    print(f"  step shape (nb x m x n x k)               kernel                                        time        "
          f"roofline (peaks: {PEAK_MFMA_TFLOPS[prec]:.1f} TFLOP/s, {PEAK_HBM_GBS / 1e3:.0f} TB/s)")
    print("\n".join(lines))
    print(f"  steps {tot / 1e3:.2f} ms, their roofline {roof_tot / 1e3:.2f} ms ({roof_tot / tot:.1%}); "
          f"whole call {span / 1e3:.2f} ms")


def _kernel_name(raw):
    """Readable kernel name: the trace's demangled form without the argument
    list, or, for names the profiler left mangled (templates over the 16-bit
    float types), the name with its template arguments spelled out."""
    import re
    m = re.match(r"_ZN2qc(\d+)", raw)
    if not m:
        return raw.replace("void ", "").replace("qc::", "").split("(")[0]
    n = int(m.group(1))
    name = raw[m.end():m.end() + n]
    rest = raw[m.end() + n:]
    args = []
    if rest.startswith("I"):
        for t in re.finditer(r"DF16_|DF16b|Li(\d+)E", rest):
            args.append({"DF16_": "_Float16", "DF16b": "__bf16"}.get(t.group(0), t.group(1)))
    return name + (f"<{', '.join(args)}>" if args else "")


def trace_kernels(path):
    """Per-kernel launches and time of the last complete contraction call in a
    rocprofv3 kernel trace (CSV) of any workload: from its leaf launch to its
    slice reduction."""
    import csv
    from collections import defaultdict
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Start_Timestamp"]))
    names = [r["Kernel_Name"] for r in rows]
    ends = [i for i, nm in enumerate(names) if "reduce64" in nm or "block_add" in nm]
    i1 = ends[-1]
    i0 = max(i for i in range(i1) if "leaf_kernel" in names[i])
    if i0 > 0 and "zero_u32" in names[i0 - 1]:
        i0 -= 1
    call = rows[i0:i1 + 1]
    agg = defaultdict(lambda: [0, 0.0])
    for r in call:
        nm = _kernel_name(r["Kernel_Name"])
        agg[nm][0] += 1
        agg[nm][1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
    span = (int(call[-1]["End_Timestamp"]) - int(call[0]["Start_Timestamp"])) * 1e-3
    busy = sum(v[1] for v in agg.values())
    print(f"  last complete call: {len(call)} launches, {span / 1e3:.3f} ms from first start to last end, "
          f"kernels busy {busy / 1e3:.3f} ms")
    print(f"  {'kernel':52s} {'launches':>8s} {'total us':>11s} {'avg us':>9s} {'% busy':>7s}")
    for nm, (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        print(f"  {nm[:52]:52s} {n:8d} {t:11.1f} {t / n:9.1f} {t / busy:7.1%}")


def pmc_summary(path, calls):
    """Per-kernel sums of every counter in a rocprofv3 counter-collection CSV,
    divided by the number of contraction calls in the traced process."""
    import csv
    from collections import defaultdict
    agg = defaultdict(lambda: defaultdict(float))
    n = defaultdict(set)
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"].replace("void ", "").replace("qc::", "").split("(")[0]
        agg[name][r["Counter_Name"]] += float(r["Counter_Value"])
        n[name].add(r["Dispatch_Id"])
    for name in sorted(agg, key=lambda x: -len(n[x])):
        vals = ", ".join(f"{c} {v / calls:.6g}" for c, v in sorted(agg[name].items()))
        print(f"  {name[:48]:48s} dispatches/call {len(n[name]) / calls:7.2f}  per call: {vals}")


def gemm_form_probe(spec):
    """Four launches of one GEMM kernel form on one shape (random complex64
    operands, A stored [k][m] when AKM, B stored [n][k] when BNK); the split
    FP16 form gets a scale workspace.  Returns the last launch's event time."""
    import torch
    from paper_1907_11217_amd import qcsim
    form, prec, nb, m, n, k, akm, bnk = spec.split(":")
    nb, m, n, k, akm, bnk = (int(v) for v in (nb, m, n, k, akm, bnk))
    A = torch.randn(nb * m * k, dtype=torch.complex64, device="cuda")
    B = torch.randn(nb * k * n, dtype=torch.complex64, device="cuda")
    C = torch.empty(nb * m * n, dtype=torch.complex64, device="cuda")
    slots = torch.zeros(3, dtype=torch.int32, device="cuda") if prec != "c64" else None
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(4):
        e0.record()
        qcsim.qc_kernel_gemm(A, B, C, nb, m, n, k, akm, bnk, prec=prec, scale_ws=slots, form=qcsim.GEMM_FORMS[form])
        e1.record()
        torch.cuda.synchronize()
    flops = 8.0 * nb * m * n * k
    return {"form": form, "prec": prec, "shape": [nb, m, n, k], "a_km": akm, "b_nk": bnk,
            "ms_last": e0.elapsed_time(e1), "tflops_alg": flops / (e0.elapsed_time(e1) * 1e-3) / 1e12}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="c64", choices=["c64", "split_fp16", "split_bf16"],
                    help="precision of the headline value (the others are reported beside it)")
    ap.add_argument("--chunk", type=int, default=0, help="slices per step of the 70-qubit workload (default 64)")
    ap.add_argument("--tune-cache", default=None,
                    help="text file of GEMM form choices read before and written after tuning the 70-qubit "
                         "workload (a profiling run then times no forms)")
    ap.add_argument("--only-prec", action="store_true", help="time only --prec on the 70-qubit workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the 4x4, 5x5, 7x7 and request-batch legs")
    ap.add_argument("--leg", choices=["grid5x5_d16", "grid7x7_d24", "request_batch", "diamond70_d32_open16"],
                    help="run only this leg and print its JSON (for profiling runs)")
    ap.add_argument("--trace-summary", metavar="CSV",
                    help="print the per-step table of a rocprofv3 kernel trace of the 70-qubit workload "
                         "(host only: rebuilds the plan to match launches to steps) and exit")
    ap.add_argument("--trace-kernels", metavar="CSV",
                    help="print per-kernel time of the last complete contraction call in a rocprofv3 kernel trace")
    ap.add_argument("--pmc-summary", metavar="CSV",
                    help="print per-kernel counter sums of a rocprofv3 counter-collection CSV, divided by "
                         "--calls, and exit")
    ap.add_argument("--calls", type=int, default=1, help="contraction calls in the traced process (--pmc-summary)")
    ap.add_argument("--gemm", metavar="FORM:PREC:NB:M:N:K:AKM:BNK", action="append", default=[],
                    help="only time GEMM kernel forms (qcsim.GEMM_FORMS names) on one shape each, four launches "
                         "apiece (for counter runs on a single kernel), and print one JSON line per form")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB device to device 5 times (the plain-copy reference of the "
                         "FETCH_SIZE / WRITE_SIZE counter runs)")
    args = ap.parse_args()
    if args.trace_summary:
        trace_summary(args.trace_summary, args.prec)
        return
    if args.trace_kernels:
        trace_kernels(args.trace_kernels)
        return
    if args.pmc_summary:
        pmc_summary(args.pmc_summary, args.calls)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}): it measures one "
              "GPU's share; more GPUs would take independent slice ranges of the same plan", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": src.numel() * 4}), flush=True)
        return
    if args.gemm:
        for spec in args.gemm:
            print(json.dumps(gemm_form_probe(spec)), flush=True)
        return
    if args.leg:
        leg = {"grid5x5_d16": lambda: fused_leg(cpu=False),
               "grid7x7_d24": lambda: grid7_leg(["c64", "split_fp16", "split_bf16"], cpu=False),
               "request_batch": batch_leg,
               "diamond70_d32_open16": lambda: open_leg(cpu=False)}[args.leg]()
        print(json.dumps(leg), flush=True)
        return

    precs = [args.prec] if args.only_prec else \
        [args.prec] + [p for p in ("c64", "split_fp16", "split_bf16") if p != args.prec]
    head = diamond_leg(args.steps, args.warmup, precs, chunk=args.chunk or None, cpu=not args.no_cpu_baseline,
                       tune_cache=args.tune_cache)
    main_prec = head["per_prec"][args.prec]
    result = {
        "metric": METRIC,
        "value": main_prec["projected_amplitudes_per_s"],
        "unit": "amplitudes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_prec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"c64": "complex-f32", "split_fp16": "f16-split-f32acc", "split_bf16": "bf16-split-f32acc"}[args.prec],
        "data": "synthetic",
        "config": {"workload": head["workload"],
                   "value_is": (f"projected amplitudes/s = slices/s / 2^{head['log2_slices']} (every slice runs the "
                                f"same program; one step = {head['slices_per_step']} slices)")},
        "slices_per_s": main_prec["slices_per_s"],
        "projected_s_per_amplitude": main_prec["projected_s_per_amplitude"],
        "tflops": main_prec["tflops_alg"],
        "roofline": main_prec["roofline"],
        "transpose_hbm": main_prec["transpose_hbm"],
        "diamond70_d32": head,
    }
    if "cpu_oracle" in head:
        c = head["cpu_oracle"]
        result["cpu_baseline"] = {"value": 1.0 / c["projected_s_per_amplitude"], "unit": "amplitudes/s",
                                  "cores": c["cores"], "kind": "oracle", "cpu_model": c["cpu_model"],
                                  "one_thread_value": 1.0 / (c["seconds_per_slice_one_thread"] * float(1 << head["log2_slices"])),
                                  "sample": c["sample"] + f", median {c['seconds_per_slice']:.2f} s per slice x "
                                                          f"2^{head['log2_slices']} slices (projection)"}
    for prec, r in head["per_prec"].items():
        result[f"{prec}_amplitudes_per_s"] = r["projected_amplitudes_per_s"]
        if "speedup_over_c64" in r:
            result[f"{prec}_speedup_over_c64"] = r["speedup_over_c64"]
        if r.get("slice_err_vs_oracle"):
            result[f"{prec}_slice_rel_err_vs_oracle"] = r["slice_err_vs_oracle"]["max"]
    if not args.no_extra:
        result["grid4x4_d10"] = small_leg()
        _say("4x4 done")
        result["grid5x5_d16"] = fused_leg(cpu=not args.no_cpu_baseline)
        _say("5x5 done")
        result["grid7x7_d24"] = grid7_leg(["c64", "split_fp16", "split_bf16"], cpu=not args.no_cpu_baseline)
        _say("7x7 done")
        result["request_batch"] = batch_leg()
        _say("request batch done")
        result["diamond70_d32_open16"] = open_leg(cpu=not args.no_cpu_baseline)
        _say("70-qubit open outputs done")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
