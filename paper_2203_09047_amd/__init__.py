"""MI355X-native third-order gas-kinetic scheme on hybrid unstructured meshes.

The solver (``gks``) is a thin ctypes binding over ``libgks.so``: a C-ABI
library of hand-written gfx950 HIP kernels (WENO reconstruction, BGK face
flux, two-stage fourth-order update) plus a C++ host preprocessor.  The
``inputs`` module builds seeded synthetic meshes and cell-averaged fields.
"""
from . import inputs  # noqa: F401

__all__ = ["inputs", "gks"]
