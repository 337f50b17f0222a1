#!/usr/bin/env python3
"""Throughput of the sliced tensor-network amplitude path on one MI355X.

One step = one qc_contract_slices call over every slice of the workload for
its whole bitstring batch (leaf instantiation, all pairwise contraction
steps, FP64 cross-slice reduction), inputs resident on the device.  Default
workload: 5x5 grid, depth 1+16+1, 2^6 slices, 64 bitstrings.

Prints ONE JSON line: amplitudes/s (value), slices/s, algorithmic TFLOP/s,
relative error against the FP64 oracle, the roofline of the dominant kernel
(per-launch algorithmic work / average launch time from HIP events recorded
by the library on the call's stream during the timed steps) and the oracle's
own CPU throughput on the host cores.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "amplitudes/sec and contraction TFLOP/s vs MFMA peak, FP32 vs split-FP16 at stated rel err"
PEAK_FP32_TFLOPS = 157.3      # MI355X FP32 (vector and matrix)
PEAK_HBM_GBS = 8000.0
WORKLOADS = {"grid5x5_d16": "c2", "grid4x4_d10": "c1"}


def _workload_text(key, lat, spec, k, n_bs):
    return (f"{spec['name']}: {lat.n} qubits on a {spec['lattice'][0]}x{spec['lattice'][1]} grid, depth 1+"
            f"{spec['depth']}+1, 2^{k} slices, {n_bs} bitstrings (seeds {spec['seed']}/{spec['seed'] + 1})")


def _traffic(kind, workload):
    """HBM bytes per launch of `kind` from the committed counter runs
    (profiles/traffic.json: FETCH_SIZE and WRITE_SIZE, each scaled by the same
    counter on a plain copy), or None if they were taken on another workload
    or before the kernel source last changed."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[kind]
    except (OSError, KeyError, ValueError):
        return None
    src = open(os.path.join(ROOT, "paper_1907_11217_amd", "csrc", "kernels.hip"), "rb").read()
    if rec.get("workload") != workload or hashlib.sha256(src).hexdigest()[:16] != rec.get("kernels_hip_sha256_16"):
        return None
    return 1024.0 * (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"])


def _gemm_form(op, prec="c64"):
    """Kernel kind the library launches for a GEMM step (its dispatch rule)."""
    k, m, n = op["k"], op["m"], op["n"]
    if prec != "c64" and m % 32 == 0 and n % 32 == 0 and k >= 2:
        return f"gemm_{prec}"
    kt = 16 if k >= 16 else k
    ok = kt in (2, 4, 8, 16) and k % kt == 0
    if prec == "c64" and ((ok and m % 32 == 0 and n % 32 == 0) or (k >= 2 and m % 128 == 0 and n % 128 == 0)):
        return "gemm_mfma"
    if k >= 4096 and op["nb"] * m * n <= 4096:
        return "gemm_dot"
    return "gemm_skinny" if n >= 256 and m in (1, 2, 4, 8, 16) else "gemm_valu"


PEAK_MFMA_TFLOPS = {"c64": PEAK_FP32_TFLOPS, "split_bf16": 2500.0, "split_fp16": 2500.0}
HW_PER_ALG = {"c64": 1.0, "split_bf16": 3.0, "split_fp16": 3.0}   # hardware flops per algorithmic flop


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


def batch_leg(n_req=256, seed=501, cap=24, reps=3, n_oracle=6, trials=32, precs=("c64", "split_fp16")):
    """Uneven batch of requests (4x4 d12, 5x5 d16, 6x6 d20, 7x7 d24 drawn
    uniformly), each with its own plan (its drawn slice count 2^0..2^12, more
    where the 2^cap-entry cap needs it) and bitstring, in one qc_contract_batch call per step; the
    stepwise requests' GEMM forms are tuned beforehand (untimed, like the plan
    build)."""
    import numpy as np
    import torch

    import synth
    from paper_1907_11217_amd import qcsim

    reqs = synth.request_mix(n_req, seed)
    t0 = time.perf_counter()
    items, ks = [], []
    for r in reqs:
        lat = r["lattice"]
        plan = qcsim.qc_plan_build(lat.n, r["circuit"], r["bitstring"], log2_slices=r["log2_slices"],
                                   log2_max_entries=cap, greedy_trials=trials, seed=1)
        ks.append(qcsim.qc_plan_info(plan)["log2_slices"])
        items.append((plan, r["bitstring"]))
    plan_s = time.perf_counter() - t0
    batch = qcsim.Batch(items)
    stream = torch.cuda.current_stream()
    khz = qcsim.qc_wall_clock_khz()
    leg = {"workload": (f"{n_req} requests drawn uniformly from 4x4 d12 / 5x5 d16 / 6x6 d20 / 7x7 d24 "
                        f"(seed {seed}), one bitstring each, 2^0..2^12 slices each (drawn), plans capped at 2^{cap} "
                        f"entries"),
           "plan_seconds": plan_s, "per_prec": {}}
    fam_of = ["%dx%d_d%d" % r["family"] for r in reqs]
    leg["families"] = {f: {"count": fam_of.count(f), "k": sorted({k for g, k in zip(fam_of, ks) if g == f})}
                       for f in sorted(set(fam_of))}
    ref = None
    for prec in precs:
        # Untimed preparation, like the plan build: the GEMM forms of each
        # stepwise request's program are timed (qc_tune keeps its choices per
        # shape for the process, so a shape met again is not timed again).
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


def _plan_trials():
    import synth
    return {k: v["trials"] for k, v in synth.CONFIGS.items()}


PLAN_TRIALS = _plan_trials()   # greedy restarts of the order search (untimed)


def first_nonzero_slice(key, candidates):
    """The first candidate slice of the 70-qubit plan whose value is not exactly
    zero (found with one split-BF16 contraction each)."""
    import torch

    import synth
    from paper_1907_11217_amd import qcsim

    lat, circ, bs, spec = synth.config(key)
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=spec["log2_slices"],
                               log2_max_entries=spec.get("log2_cap", 0), greedy_trials=PLAN_TRIALS[key], seed=1)
    k = qcsim.qc_plan_info(plan)["log2_slices"]
    ws = torch.empty(qcsim.qc_workspace_bytes(plan, 1, 1, "split_bf16"), dtype=torch.uint8, device="cuda")
    out = torch.zeros(1, 2, dtype=torch.float64, device="cuda")
    tried = []
    for s in candidates(k):
        out.zero_()
        qcsim.qc_contract_slices(plan, s, s + 1, bs[:1], "split_bf16", ws, out)
        torch.cuda.synchronize()
        tried.append(s)
        if out.abs().max().item() > 0:
            return s, tried
    return tried[-1], tried


def big_leg(key, precs, reps, s_range, oracle_slices=(), tune=False):
    """One large configuration on the stepwise path: every precision runs the
    same slice range for one bitstring; reports time, algorithmic TFLOP/s,
    the GEMM kernels' achieved MFMA rate against their dtype's peak, and the
    agreement with the complex FP32 result (and with the oracle on sampled
    slices, when asked)."""
    import numpy as np
    import torch

    import synth
    from paper_1907_11217_amd import qcsim

    lat, circ, bs, spec = synth.config(key)
    t0 = time.perf_counter()
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=spec["log2_slices"],
                               log2_max_entries=spec.get("log2_cap", 0), greedy_trials=PLAN_TRIALS[key], seed=1)
    plan_s = time.perf_counter() - t0
    info = qcsim.qc_plan_info(plan)
    k = info["log2_slices"]
    s0, s1 = s_range(k)
    n_sl = s1 - s0
    x = bs[:1]
    stream = torch.cuda.current_stream()
    out = torch.zeros(1, 2, dtype=torch.float64, device="cuda")
    b = (n_sl - 1).bit_length()
    steps = qcsim.qc_plan_export_steps(plan, b, 0)
    chunks = max(1, n_sl >> b)
    leg = {"workload": (f"{spec['name']}: {lat.n} qubits, depth 1+{spec['depth']}+1, 2^{k} slices (cap 2^"
                        f"{spec.get('log2_cap', 0)} entries), slices [{s0}, {s1}) for bitstring seed "
                        f"{spec['seed'] + 1}"),
           "log2_slices": k, "slices_per_step": n_sl, "plan_seconds": plan_s,
           "flops_per_slice_b0": info["flops_per_slice"], "per_prec": {}}
    ref = None
    per_slice_ref = None
    for prec in precs:
        ws = torch.empty(qcsim.qc_workspace_bytes(plan, n_sl, 1, prec), dtype=torch.uint8, device="cuda")
        ps = torch.zeros(n_sl, 1, 2, dtype=torch.float64, device="cuda")

        def step():
            qcsim.qc_contract_slices(plan, s0, s1, x, prec, ws, out, stream=stream)

        tune_s = None
        if tune:
            # Untimed preparation, like the plan build.
            t1 = time.perf_counter()
            qcsim.qc_tune(plan, n_sl, 1, prec, ws, stream=stream)
            tune_s = time.perf_counter() - t1

        out.zero_()
        qcsim.qc_contract_slices(plan, s0, s1, x, prec, ws, out, ps, stream=stream)
        torch.cuda.synchronize()
        val = complex(*out.cpu().numpy()[0])
        psv = ps.cpu().numpy()[:, 0, 0] + 1j * ps.cpu().numpy()[:, 0, 1]
        out.zero_()
        step()  # the timed configuration's first call captures its graph (untimed)
        ms = _events_ms(stream, step, reps)
        qcsim.qc_profile_read(plan)
        qcsim.qc_profile_enable(plan, True)
        step()
        torch.cuda.synchronize()
        qcsim.qc_profile_enable(plan, False)
        prof = qcsim.qc_profile_read(plan)
        # Algorithmic flops of the step's GEMMs, per kernel kind.
        per_kind = {}
        for op in steps:
            if op["kind"] == 1:
                f = "micro" if op["micro"] else _gemm_form(op, prec)
                per_kind[f] = per_kind.get(f, 0.0) + op["flops"] * chunks
        flops = sum(per_kind.values())
        r = {"ms_per_step": ms, "value": val.real, "value_im": val.imag, "tflops": flops / (ms * 1e-3) / 1e12,
             "tune_seconds": tune_s,
             "kernels": {kk: {"launches": v[0], "ms": v[1]} for kk, v in prof.items()}}
        mf = "gemm_mfma" if prec == "c64" else f"gemm_{prec}"
        if mf in prof and mf in per_kind:
            ach = per_kind[mf] / (prof[mf][1] * 1e-3) / 1e12
            r["mfma_gemm"] = {"kernel": mf, "achieved_tflops_alg": ach,
                              "achieved_tflops_hw": ach * HW_PER_ALG[prec], "peak_tflops": PEAK_MFMA_TFLOPS[prec],
                              "frac": ach * HW_PER_ALG[prec] / PEAK_MFMA_TFLOPS[prec],
                              "flop_share": per_kind[mf] / flops}
        if ref is None:
            ref, per_slice_ref = val, psv
        else:
            r["rel_diff_vs_c64"] = abs(val - ref) / abs(ref) if ref != 0 else None
            scale = np.sqrt(np.mean(np.abs(per_slice_ref) ** 2))
            r["per_slice_max_diff_vs_c64_over_rms"] = float(np.abs(psv - per_slice_ref).max() / scale)
        leg["per_prec"][prec] = r
        del ws
    if "c64" in leg["per_prec"] and n_sl < (1 << k):
        leg["projected_s_per_amplitude_c64"] = leg["per_prec"]["c64"]["ms_per_step"] * 1e-3 * (1 << k) / n_sl
    for p in precs[1:]:
        leg[f"speedup_{p}_over_c64"] = leg["per_prec"]["c64"]["ms_per_step"] / leg["per_prec"][p]["ms_per_step"]
    leg["flops_unsliced"] = info["flops_unsliced"]
    leg["slicing_overhead"] = info["flops_per_slice"] * float(1 << k) / max(info["flops_unsliced"], 1.0)
    if oracle_slices:
        import oracle
        segs = [tuple(int(v) for v in sg) for sg in qcsim.qc_plan_sliced_segments(plan)]
        errs, secs = [], []
        for s in oracle_slices:
            t1 = time.perf_counter()
            v = oracle.sliced_value(lat.n, circ, x[0], segs, s0 + s)
            secs.append(time.perf_counter() - t1)
            errs.append(abs(per_slice_ref[s] - v) / abs(v))
        leg["oracle_per_slice_rel_err_c64"] = {"slices": [s0 + s for s in oracle_slices], "max": float(max(errs))}
        # The oracle beside the GPU: its per-slice time (NumPy FP64 pairwise
        # contraction, the host's BLAS threads) projected to all 2^k slices.
        med = sorted(secs)[len(secs) // 2]
        leg["cpu_oracle"] = {"seconds_per_slice": med, "projected_s_per_amplitude": med * float(1 << k),
                             "cores": len(os.sched_getaffinity(0)), "kind": "oracle",
                             "sample": f"{len(secs)} sampled slice(s) of the same plan"}
    return leg


def small_leg(reps=200):
    """The 4x4 depth-10 workload: one amplitude (no slicing), latency per call
    with the bitstring resident, against the oracle's state vector."""
    import numpy as np
    import torch

    import oracle
    import synth
    from paper_1907_11217_amd import qcsim

    lat, circ, bs, spec = synth.config("c1")
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=0, greedy_trials=PLAN_TRIALS["c1"], seed=1)
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
    return {"workload": f"{spec['name']}: {lat.n} qubits, depth 1+{spec['depth']}+1, no slicing, 1 bitstring "
                        f"(seeds {spec['seed']}/{spec['seed'] + 1})",
            "us_per_amplitude": ms * 1e3, "amplitudes_per_s": 1.0 / (ms * 1e-3),
            "abs_err": abs(got - ref), "abs_ref": abs(ref),
            "cpu_oracle": {"seconds": cpu_s, "amplitudes_per_s": 1.0 / cpu_s, "kind": "oracle",
                           "sample": "one state-vector run of the same circuit"}}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="grid5x5_d16", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default="c64", choices=["c64", "split_bf16", "split_fp16"])
    ap.add_argument("--exec", default="auto", choices=["auto", "fused", "stepwise"])
    ap.add_argument("--fused-slice-bits", type=int, default=-1,
                    help="slices per fused work item (log2); default: timed by the library on the first call")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 7x7 depth-24, 70-qubit depth-32 and request-batch reports")
    ap.add_argument("--leg", choices=["grid7x7_d24", "diamond70_d32", "request_batch"],
                    help="run only this report and print its JSON (for profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB device to device 5 times (the plain-copy reference of the "
                         "FETCH_SIZE / WRITE_SIZE counter runs)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the slice ranges of a multi-GPU run would be independent per GPU, see DESIGN.md", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        import torch
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": src.numel() * 4}), flush=True)
        return
    if args.leg:
        import torch
        torch.cuda.set_device(0)
        precs = ["c64", "split_fp16", "split_bf16"]
        if args.leg == "grid7x7_d24":
            leg = big_leg("c3", precs, 5, lambda k: (0, 1 << k), oracle_slices=(), tune=True)
        elif args.leg == "diamond70_d32":
            s4, _ = first_nonzero_slice("c4", lambda k: [(1 << k) - 1 - j for j in range(16)])
            leg = big_leg("c4", precs, 2, lambda k: (s4, s4 + 1))
        else:
            leg = batch_leg()
        print(json.dumps(leg), flush=True)
        return

    import numpy as np
    import torch

    import synth
    from paper_1907_11217_amd import qcsim

    key = WORKLOADS[args.workload]
    lat, circ, bs, spec = synth.config(key)
    n_bs = len(bs)
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    plan = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=spec["log2_slices"],
                               log2_max_entries=spec.get("log2_cap", 0), greedy_trials=PLAN_TRIALS[key], seed=1)
    plan_s = time.perf_counter() - t0
    qcsim.qc_plan_set_exec(plan, args.exec)
    if args.fused_slice_bits >= 0:
        qcsim.qc_plan_set_fused_slice_bits(plan, args.fused_slice_bits)
    info = qcsim.qc_plan_info(plan)
    k = info["log2_slices"]
    n_slices = 1 << k
    ws = torch.empty(qcsim.qc_workspace_bytes(plan, n_slices, n_bs, args.prec), dtype=torch.uint8, device="cuda")
    out = torch.zeros(n_bs, 2, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    bits_dev = torch.from_numpy(np.ascontiguousarray(bs)).cuda()

    def step():
        # Inputs resident on the device: the bitstrings are read in place.
        qcsim.qc_contract_slices_dev(plan, 0, n_slices, bits_dev, args.prec, ws, out, stream=stream)

    def step_host_bits():
        qcsim.qc_contract_slices(plan, 0, n_slices, bs, args.prec, ws, out, stream=stream)

    for _ in range(args.warmup):
        step()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / args.steps

    # The timed region: K steps back to back on `stream`.
    ms = timed(step)
    # The same K steps again with the library's kernel timing on (an event
    # pair around each of its kernels, on `stream`) for the per-kernel
    # roofline; kept out of `value` because the extra events add host work.
    qcsim.qc_profile_read(plan)
    qcsim.qc_profile_enable(plan, True)
    ms_profiled = timed(step)
    qcsim.qc_profile_enable(plan, False)
    prof = qcsim.qc_profile_read(plan)
    # The same steps with the bitstrings handed over from host memory (the
    # host-to-device copy included), reported beside the resident rate.
    ms_host_bits = timed(step_host_bits)

    # Result of one clean step, for the error report.
    out.zero_()
    step()
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    amps = o[:, 0] + 1j * o[:, 1]

    # Algorithmic work (the lowered program's own per-step shapes).
    fused = "fused" in prof
    result_extra = {}
    if fused:
        # A fused work item is a chunk of 2^fb slices (the slice bits the
        # plan's first call chose by timing) with one bitstring; its work is
        # the flops of the program lowered with those fb open slice bits.
        fb = qcsim.qc_plan_describe(plan, 0, 0)["fused_slice_bits"]
        fb = max(fb, 0)
        desc = qcsim.qc_plan_describe(plan, fb, 0)
        items_per_launch = ((n_slices + (1 << fb) - 1) >> fb) * (1 << max(0, int(np.ceil(np.log2(n_bs)))))
        result_extra = {"fused_slice_bits": fb, "fused_items_per_workgroup": desc["fused_pairs"],
                        "fused_waves_per_item": desc["fused_waves"],
                        "fused_tuning_items_waves_ms": desc["fused_tuning"], "fused_flops_per_item": desc["flops"],
                        "flops_per_pair_one_slice_program": qcsim.qc_plan_describe(plan, 0, 0)["flops"]}
        flops_step = desc["flops"] * ((n_slices + (1 << fb) - 1) >> fb) * n_bs
        kind_work = {"fused": (desc["flops"] * items_per_launch, "alu")}
    else:
        b = min(k, 12)
        desc = None
        kind_work = {}
        flops_step = 0.0
        for bb in range(min(k, 12), -1, -1):
            try:
                desc = qcsim.qc_plan_describe(plan, bb, int(np.ceil(np.log2(n_bs))))
                b = bb
                break
            except qcsim.QcError:
                continue
        chunks = max(1, n_slices >> b)
        per = {"gemm_mfma": 0.0, "gemm_valu": 0.0, "gemm_skinny": 0.0, "gemm_dot": 0.0, "micro": 0.0,
               "transpose": 0.0}
        for op in desc["ops"]:
            if op["op"] == "gemm":
                per["micro" if op.get("micro") else _gemm_form(op)] += 8.0 * op["nb"] * op["m"] * op["n"] * op["k"]
            elif not op.get("micro"):
                per["transpose"] += 16.0 * (1 << len(desc["tensors"][op["src"]]["layout"]))
        flops_step = (per["gemm_mfma"] + per["gemm_valu"] + per["gemm_skinny"] + per["gemm_dot"] + per["micro"]) * \
            chunks * n_bs / (1 << desc["m"])
        kind_work = {"gemm_mfma": (per["gemm_mfma"] * chunks, "mfma"),
                     "gemm_valu": (per["gemm_valu"] * chunks, "alu"),
                     "gemm_skinny": (per["gemm_skinny"] * chunks, "alu"),
                     "gemm_dot": (per["gemm_dot"] * chunks, "alu"),
                     "micro": (per["micro"] * chunks, "alu"),
                     "transpose": (per["transpose"] * chunks, "hbm")}
    dom = max(prof, key=lambda kk: prof[kk][1])
    launches, total_ms = prof[dom]
    avg_ms = total_ms / launches
    roof = None
    if dom in kind_work:
        work_total, bound = kind_work[dom]
        per_launch = work_total * args.steps / launches
        if bound == "hbm":
            achieved = per_launch / (avg_ms * 1e-3) / 1e9
            roof = dict(bound="hbm", achieved=achieved, peak=PEAK_HBM_GBS, unit="GB/s", frac=achieved / PEAK_HBM_GBS)
        else:
            achieved = per_launch / (avg_ms * 1e-3) / 1e12
            roof = dict(bound=bound, achieved=achieved, peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                        frac=achieved / PEAK_FP32_TFLOPS)
        roof.update(kernel=dom, avg_launch_ms=avg_ms, launches_per_step=launches / args.steps,
                    traffic=_traffic(dom, args.workload))

    result = {
        "metric": METRIC,
        "value": n_bs / (ms * 1e-3),
        "unit": "amplitudes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": _workload_text(key, lat, spec, k, n_bs), "n_qubits": lat.n, "depth": spec["depth"],
                   "log2_slices": k, "n_bitstrings": n_bs, "exec": "fused" if fused else "stepwise"},
        "slices_per_s": n_slices * n_bs / (ms * 1e-3),
        "host_bitstrings_value": n_bs / (ms_host_bits * 1e-3),
        "ms_per_step_profiled": ms_profiled,
        "tflops": flops_step / (ms * 1e-3) / 1e12,
        "flops_per_step": flops_step,
        "plan_seconds": plan_s,
        "kernels": {kk: {"launches_per_step": v[0] / args.steps, "avg_ms": v[1] / v[0]} for kk, v in prof.items()},
        "roofline": roof,
    }
    result.update(result_extra)

    if not args.no_large:
        precs = ["c64", "split_fp16", "split_bf16"]
        # 7x7 depth 24: every slice of one amplitude per step.
        result["grid4x4_d10"] = small_leg()
        result["grid7x7_d24"] = big_leg("c3", precs, 5, lambda k: (0, 1 << k), oracle_slices=(0,), tune=True)
        # 70 qubits depth 32: one slice per step; the amplitude is projected
        # as slice time x 2^k.  Many slices of this plan are exactly zero (a
        # leaf or an intermediate vanishes for their sliced values); the
        # precisions are compared on the first nonzero one counting down from
        # the last slice (the time per slice does not depend on the values).
        s4, tried = first_nonzero_slice("c4", lambda k: [(1 << k) - 1 - j for j in range(16)])
        result["diamond70_d32"] = big_leg("c4", precs, 2, lambda k: (s4, s4 + 1))
        result["diamond70_d32"]["zero_slices_skipped"] = len(tried) - 1
        result["request_batch"] = batch_leg()

    if not args.no_cpu_baseline:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
        t0 = time.perf_counter()
        psi = oracle.statevector(lat.n, circ)
        cpu_s = time.perf_counter() - t0
        ref = np.array([psi[oracle.index_of(x)] for x in bs])
        mask = (1 << lat.n) * np.abs(ref) ** 2 >= 1e-2
        rel = np.abs(amps - ref)[mask] / np.abs(ref[mask])
        result["rel_err"] = {"max_rel": float(rel.max()), "norm_rel": float(np.linalg.norm(amps - ref) /
                                                                             np.linalg.norm(ref)),
                             "gate": "N|a|^2 >= 1e-2", "tol": 1e-5 if args.prec == "c64" else 1e-4}
        result["cpu_baseline"] = {"value": n_bs / cpu_s, "unit": "amplitudes/s", "cores": threads, "kind": "oracle",
                                  "sample": f"one FP64 state-vector run of the same circuit (2^{lat.n} entries, "
                                            f"OpenMP C) giving all {n_bs} requested amplitudes, {cpu_s:.2f} s"}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
