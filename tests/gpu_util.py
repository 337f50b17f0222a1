"""Helpers shared by the GPU tests (tolerances, device buffers)."""

import sys

import numpy as np


def say(msg: str):
    """Names the case before a GPU step, flushed, so a failing run shows it."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def check_amplitudes(got, ref, n_qubits, tol):
    """The amplitude tolerance: relative error |a - a_ref| / |a_ref| at most
    ``tol`` over the bitstrings with N |a_ref|^2 >= 1e-2 (Porter-Thomas puts
    ~1% of them below that, where relative error is meaningless), the batch's
    relative 2-norm error at most ``tol``, and every absolute error at most
    ``tol`` times the batch's RMS amplitude."""
    got = np.asarray(got, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    N = 2.0 ** n_qubits
    err = np.abs(got - ref)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    mask = N * np.abs(ref) ** 2 >= 1e-2
    rel = err[mask] / np.abs(ref[mask]) if mask.any() else np.zeros(0)
    norm_rel = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
    info = dict(max_rel=float(rel.max(initial=0.0)), norm_rel=float(norm_rel),
                max_abs_over_rms=float(err.max() / max(rms, 1e-300)), n_gated=int(mask.sum()))
    assert info["max_rel"] <= tol, info
    assert info["norm_rel"] <= tol, info
    assert info["max_abs_over_rms"] <= tol, info
    return info
