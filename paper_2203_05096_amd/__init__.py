"""CSR-k sparse matrix-vector multiplication for AMD Instinct MI355X (gfx950).

The compute lives in ``lib/libcsrk.so`` (host preprocessing in C++, products
in hand-written HIP kernels) behind the C ABI of ``include/csrk.h``.  This
package is its Python binding:

* ``paper_2203_05096_amd._capi``  — one function per C entry point (ctypes);
* ``CsrkMatrix`` / ``CsrkSpMV`` / ``CsrkBatch`` — torch tensors in and out.

Importing the package does not load the library; the first call does, and
fails loudly if it has not been built (``python -m paper_2203_05096_amd.build``).
"""

from . import _capi  # noqa: F401
from ._capi import CsrkError, csrk_tune  # noqa: F401


def __getattr__(name):
    if name in ("CsrkMatrix", "CsrkSpMV", "CsrkBatch"):
        from . import matrix
        return getattr(matrix, name)
    raise AttributeError(name)
