"""MI355X (gfx950) altGDmin: Python binding of the HIP library libaltgdmin.so.

The binding only marshals arguments: every step of the reconstruction runs
in the library's HIP kernels.  PyTorch provides device memory and the
stream.  Layouts (see include/altgdmin.h) as torch tensors:

* coils   complex64 (nc, n)             s_c(p), p = x + nx*y
* mask    int32     (q, L_max) lines / (q, m_max) flat indices
* m_k     int32     (q,)                samples per coil per frame
* y       complex64 (q, nc, m_max)      padded measurements
* U       complex64 (r, n)              row j is the basis column u_j
* B       complex64 (q, r)              row k is b_k
* X       complex64 (q, n)              row k is the frame x_k

There is no CPU path: constructing a context without the built library, or
with tensors not on a GPU, raises.
"""
from ._lib import (AltGDmin, AltGDminError, Params, Stats, MASK_LINES, MASK_INDEX, FP32, MIXED,  # noqa: F401
                   TIMED_KERNELS, WsInit, lib_path, load_library)
