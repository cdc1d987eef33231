"""MI355X (gfx950) tall & skinny matrix products: TSMTTSM C = A^T B and TSMM B = A C.

The products run in the HIP kernels of ``libtsgemm.so`` (C ABI in
include/tsgemm.h); this package only marshals torch tensors into that ABI.
Importing the torch API requires the built library.
"""


def __getattr__(name):
    if name in ("tsmttsm", "tsmm", "kernel_name", "OrthPlan", "orth_batched"):
        from . import api
        return getattr(api, name)
    if name == "TSMTTSM":
        from . import autograd
        return autograd.TSMTTSM
    raise AttributeError(name)
