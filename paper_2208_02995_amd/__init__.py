"""MI355X energy-minimization prolongation (arXiv 2208.02995).

The restricted preconditioned CG of the paper runs in hand-written HIP
kernels for gfx950 behind the C ABI of include/emin.h; ``emin`` is the ctypes
binding with the C names, ``api`` a small convenience layer that moves host
matrices to the device.  The shared library is required: there is no CPU
fallback.
"""

from . import emin  # noqa: F401

__all__ = ["emin", "api"]
