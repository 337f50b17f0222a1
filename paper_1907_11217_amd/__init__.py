"""MI355X-native engine for single amplitudes <x|C|0^n> of random 2D-lattice
circuits by sliced tensor-network contraction (arXiv:1907.11217's hot path).

The compute path is libqcsim.so (hand-written HIP for gfx950 behind the C ABI
in include/qcsim.h); ``qcsim`` is its ctypes binding.  Importing this package
does not load the library; the first call does, and fails loudly if it has
not been built.
"""

from . import qcsim  # noqa: F401
