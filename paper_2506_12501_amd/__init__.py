"""mdx: batched McMurchie-Davidson electron-repulsion integrals for MI355X.

The compute path is the native library ``libmdx.so`` (HIP kernels for gfx950
behind a C ABI, see ``include/mdx.h``); this package only marshals arguments.
Importing the package does not load the library; the first call that needs
it does, and raises if it is missing.
"""
from .workloads import Basis  # noqa: F401

__all__ = ["Basis"]
