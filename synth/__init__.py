"""Seeded synthetic inputs shared by the GPU path and the oracle.

This package draws random circuits and bitstrings and nothing else: it holds
no gate matrix, no amplitude arithmetic and no contraction logic, so both the
CPU oracle and the HIP path can take their inputs from it without sharing any
of the method's arithmetic.
"""

from .rng import SplitMix64
from .circuits import (
    GATE_H, GATE_SQRT_X, GATE_SQRT_Y, GATE_T, GATE_CZ, GATE_NAMES,
    Lattice, grid, diamond70, diamond72, cz_patterns, random_circuit, random_bitstrings,
    random_slices, config, request_mix, CONFIGS,
)

__all__ = [
    "SplitMix64", "GATE_H", "GATE_SQRT_X", "GATE_SQRT_Y", "GATE_T", "GATE_CZ",
    "GATE_NAMES", "Lattice", "grid", "diamond70", "diamond72", "cz_patterns",
    "random_circuit", "random_bitstrings", "random_slices", "config",
    "request_mix", "CONFIGS",
]
