"""Python binding of liblfmm (include/lfmm.h): the lattice FMM on MI355X.

Thin ctypes layer: it checks tensor shapes/dtypes/devices and passes raw device pointers and
the current HIP stream to the C ABI.  Every step of the computation runs in the library's
HIP kernels; there is no Python or CPU fallback, and importing fails loudly when the
library has not been built (``python paper_1105_3505_amd/build.py``).
"""
from __future__ import annotations

from ._lib import (  # noqa: F401
    LfmmError,
    LfmmWarning,
    Context,
    Plan,
    Server,
    Inclusions,
    Dirichlet,
    HostOperators,
    host_phi,
    library_path,
    exported_symbols,
    PRECISIONS,
)

__all__ = ["LfmmError", "LfmmWarning", "Context", "Plan", "Server", "Inclusions", "Dirichlet", "HostOperators", "host_phi", "library_path",
           "exported_symbols", "PRECISIONS"]
