"""MI355X (gfx950) phase-field FEM step library: Python side.

The computation lives in libpfhip.so (HIP kernels for gfx950 behind the C ABI
in include/pf.h).  This package only marshals arguments (``solver``), builds
the library (``build``) and draws synthetic inputs (``inputs``).  Importing it
does not load the library; the first call does, and fails loudly if it is not
built.
"""
from . import _abi  # noqa: F401

__all__ = ["solver", "inputs", "_abi"]
