"""Loader for the C build of O1 (``sv.c``); test infrastructure only.

``build()`` compiles sv.c with gcc into ``_oracle_sv.so`` beside it.  It is
called by the top-level build step and, if the library is missing, on first
use here.
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sv.c")
_LIB = os.path.join(_HERE, "_oracle_sv.so")
_lib = None


def build() -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu11", _SRC, "-o", _LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_statevector.restype = ctypes.c_int
        lib.oracle_statevector.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def statevector_c(n_qubits: int, circuit) -> np.ndarray:
    circ = np.ascontiguousarray(np.asarray(circuit, dtype=np.int32).reshape(-1, 4))
    psi = np.empty(1 << int(n_qubits), dtype=np.complex128)
    rc = _load().oracle_statevector(int(n_qubits), circ.shape[0], circ.ctypes.data, psi.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_statevector: invalid gate in circuit")
    return psi
