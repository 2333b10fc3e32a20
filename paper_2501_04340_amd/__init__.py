"""MI355X (gfx950) tree-cotree gauged IETI-DP solver for 3D magnetostatics.

The solver lives in the C-ABI library ``lib/libietidp.so`` (declared in
``include/ietidp.h``); :mod:`paper_2501_04340_amd.ietidp` is its ctypes
binding.  Importing this package does not load the library.
"""
from .ietidp import NN, IetiError, Solver, load_library, library_path  # noqa: F401
