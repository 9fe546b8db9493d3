"""spk: CSR SpMV and Jacobi-preconditioned CG for AMD MI355X (gfx950).

The compute path is the HIP library ``libspk.so`` behind the C ABI declared in
``include/spk.h``; ``paper_2011_00715_amd.spk`` is its ctypes binding.
PyTorch only supplies device memory and streams.
"""

import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libspk.so")


def load():
    """Import the binding (raises if the HIP library is not built)."""
    from . import spk

    return spk
