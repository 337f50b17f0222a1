"""FP64 CPU oracle for single amplitudes <x|C|0^n> -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything from here.  The library (``libqcsim.so``
and the ``paper_1907_11217_amd`` package) never imports, links or runs it,
and nothing here imports from the library: the two share no code.  Inputs
(circuits, bitstrings, sampled slice ids) come from the ``synth`` package,
which holds no arithmetic of the method.

What it computes (all in complex128):

* ``statevector``  -- the definition: psi = U_L ... U_1 e_0, amp(x) = psi[idx(x)]
  with qubit 0 the most significant bit of idx (O1).
* ``pathsum``      -- the same amplitude as an explicit sum over all values of
  the circuit's wire segments (brute force, tiny circuits only).
* ``tn``           -- a plain tensor network with one tensor per gate and two
  tensors per index (no hyper-edges), contracted pairwise with numpy einsum
  in an order this module chooses itself; ``sliced_value`` fixes the wire
  indices of chosen segments to the bits of a slice id, so that the values
  of all slices add up to the amplitude (the paper's statement that subtask
  results add up to the amplitude, Section "Benchmarking and the Experimental
  Setup").

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, brute force and invariants; see the test docstrings.
"""

from .gates import gate_matrix, ORACLE_GATES
from .statevector import statevector, amplitudes_sv, index_of
from .pathsum import pathsum_amplitude
from .hyper import hyper_network, hyper_value, contract_tree, contract_greedy, validate_tree
from .tn import (
    build_plain_network, contract_network, tn_amplitude, sliced_value,
    segment_counts,
)

__all__ = [
    "gate_matrix", "ORACLE_GATES", "statevector", "amplitudes_sv", "index_of",
    "pathsum_amplitude", "build_plain_network", "contract_network",
    "tn_amplitude", "sliced_value", "segment_counts", "hyper_network", "hyper_value",
    "contract_tree", "contract_greedy", "validate_tree",
]
