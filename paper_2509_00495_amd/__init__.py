"""MI355X-native mixed-precision Jacobi eigensolver (libjacobi + binding).

The solver itself is the HIP library ``libjacobi.so`` (built from ``csrc/``
by ``paper_2509_00495_amd.build``); this package only marshals torch GPU
tensors into its C ABI.
"""
from .jacobi import (  # noqa: F401
    DEGENERATE, DEVICE, NOCONV, NONFINITE, NOTSYM, OK, WORKSPACE,
    Info, JacobiError, Opts, Workspace, declared_functions, device_summary,
    eigh, eigh_autograd, eigh_backward, eigh_batched, eigh_batched_noalloc, eigh_mixed, make_opts,
    workspace_bytes, EighFn, LIB_PATH,
)
