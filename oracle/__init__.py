"""CPU FP64 oracle for the energy-minimization RCG.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  Independent of the
HIP library (no shared code, headers, tables or helpers).
"""

from . import rcg  # noqa: F401
from . import adjoint  # noqa: F401
from . import sgs  # noqa: F401
from . import ptent  # noqa: F401
from .rcg import (  # noqa: F401
    pattern_expand,
    pattern_contains,
    emin_setup,
    project,
    masked_product,
    energy,
    constraint_error,
    jacobi,
    block_jacobi,
    block_jacobi_shared,
    rcg as rcg_solve,
    solve,
    values_on_pattern,
    row_ids,
)
