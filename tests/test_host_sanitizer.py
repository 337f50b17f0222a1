"""The host planner (network, order search, lowering, C ABI) under
AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

The four host sources are compiled with g++ -fsanitize=address,undefined
(no recovery: the first finding aborts) and linked with the regular HIP
objects into a separate library; a child process with the ASan runtime
preloaded builds plans of several workloads through the Python binding
(greedy and refined order search on its worker threads, slicing, open
outputs, the 72-qubit lattice), lowers and describes them, exports steps and
trees, drives the argument-checking error paths, and destroys every plan.
Nothing here touches a GPU.
"""

import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1907_11217_amd")
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
OUT_DIR = os.path.join(BUILD, "sanitize")
SOURCES = ["network.cpp", "order.cpp", "lower.cpp", "capi.cpp"]
DEVICE_OBJS = ["kernels.hip.o", "runtime.hip.o"]
FLAGS = ["-O1", "-g", "-std=c++17", "-fPIC", "-pthread", "-fno-omit-frame-pointer",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _runtime(name):
    r = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True)
    p = r.stdout.strip()
    return p if r.returncode == 0 and os.path.isabs(p) and os.path.exists(p) else None


def _build():
    for o in DEVICE_OBJS:
        if not os.path.exists(os.path.join(BUILD, o)):
            pytest.skip("the HIP objects are not built (run __graft_entry__.build())")
    os.makedirs(OUT_DIR, exist_ok=True)
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(OUT_DIR, src + ".o")
        objs.append(obj)
        procs.append(subprocess.Popen(["g++", *FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for p in procs:
        out, err = p.communicate()
        assert p.returncode == 0, err
    lib = os.path.join(OUT_DIR, "libqcsim_sanitized.so")
    r = subprocess.run(["g++", "-shared", *FLAGS, *objs, *[os.path.join(BUILD, o) for o in DEVICE_OBJS],
                        "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-o", lib],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return lib


CHILD = textwrap.dedent("""
    import sys
    import numpy as np
    sys.path.insert(0, ROOT)
    import synth
    from paper_1907_11217_amd import qcsim
    qcsim.LIB_PATH = LIB

    def exercise(plan, b=0, m=0):
        qcsim.qc_plan_info(plan)
        segs = qcsim.qc_plan_sliced_segments(plan)
        k = qcsim.qc_plan_info(plan)["log2_slices"]
        for s in (0, (1 << k) - 1):
            qcsim.qc_plan_slice_assignment(plan, s)
        qcsim.qc_plan_describe(plan, b, m)
        qcsim.qc_plan_describe(plan, b, m, "split_fp16")
        qcsim.qc_plan_export_steps(plan, b, m)
        qcsim.qc_plan_export_tree(plan)
        return segs

    lat, circ, bs, spec = synth.config("c1")
    p = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=2, greedy_trials=8, seed=1)
    exercise(p, 2, 0)
    exercise(p, 0, 3)
    # A cap of two entries: met by slicing nearly every index.
    p = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_max_entries=1.0, log2_slices=2)
    exercise(p, 0, 0)
    del p
    lat, circ, bs, spec = synth.config("c2")
    p = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=6, greedy_trials=8, seed=1, quick=True)
    exercise(p, 6, 6)
    p = qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=3, greedy_trials=4, seed=3, open_qubits=[0, 7, 24])
    exercise(p, 2, 0)
    del p
    lat = synth.diamond70()
    circ = synth.random_circuit(lat, 12, 7)
    p = qcsim.qc_plan_build(lat.n, circ, synth.random_bitstrings(lat.n, 1, 8)[0], log2_slices=8,
                            log2_max_entries=16, greedy_trials=16, seed=2)
    exercise(p, 3, 0)
    del p
    lat = synth.diamond72()
    circ = synth.random_circuit(lat, 10, 9)
    p = qcsim.qc_plan_build(lat.n, circ, synth.random_bitstrings(lat.n, 1, 10)[0], log2_slices=4,
                            log2_max_entries=18, greedy_trials=4, seed=4)
    exercise(p, 2, 0)
    del p
    # Error paths: each must fail with a status, not crash.
    lat, circ, bs, spec = synth.config("c1")
    bad = np.array(circ).copy()
    bad[0, 1] = 99
    cases = [
        lambda: qcsim.qc_plan_build(lat.n, bad, bs[0]),
        lambda: qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=40),
        lambda: qcsim.qc_plan_build(lat.n, circ, bs[0], log2_slices=-7),
        lambda: qcsim.qc_plan_build(lat.n, circ, bs[0], open_qubits=[3, 3]),
        lambda: qcsim.qc_plan_build(lat.n, circ, bs[0], open_qubits=[lat.n]),
        lambda: qcsim.qc_plan_build(lat.n, circ, bs[0], explicit_segments=[[10**6, 0]]),
    ]
    for f in cases:
        try:
            f()
        except qcsim.QcError:
            continue
        raise SystemExit("an invalid plan request was accepted")
    maps = open("/proc/self/maps").read()
    if "libasan" not in maps or "libqcsim_sanitized" not in maps:
        raise SystemExit("the sanitized library or the ASan runtime is not the one loaded")
    print("sanitized planner runs: ok", flush=True)
""")


def test_planner_under_asan_and_ubsan():
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("g++ has no AddressSanitizer runtime")
    lib = _build()
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan
    # Leaks are not checked: the interpreter's own allocations would be
    # reported at exit.
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    code = f"ROOT = {ROOT!r}\nLIB = {lib!r}\n" + CHILD
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    report = r.stdout[-4000:] + r.stderr[-8000:]
    assert r.returncode == 0, report
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
    assert "sanitized planner runs: ok" in r.stdout, report
