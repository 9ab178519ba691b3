"""CPU complex128 oracle for the Jac-PCG RZF precoder (Xu et al., "Jac-PCG Based
Low-Complexity Precoding for Extremely Large-Scale MIMO Systems").

TEST INFRASTRUCTURE ONLY. This package is the slow, plain reference that the GPU
path is checked against. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it. It shares no code with the
HIP path (``paper_2305_13925_amd``) and imports nothing from it.

Everything is computed in complex128 / float64 with NumPy; matrix products are
used as library primitives, nothing is blocked, fused or reordered.

Parity pins (see ``tests/test_oracle_*.py``): every function here is pinned
against something other than itself -- exact rational arithmetic, the Krylov
optimality of the t-th CG iterate, SciPy's CG, LAPACK inverses, closed forms
and invariants of the method.
"""

from .rzf import (  # noqa: F401
    OK,
    NOT_CONVERGED,
    BREAKDOWN,
    gram,
    cholesky_lower,
    lower_inverse,
    chol_inverse,
    gauss_jordan_inverse,
    jacpcg,
    cg_on_jacobi_scaled_operator,
    precoder,
    rzf,
    block_slices,
    block_rzf,
    direct_rzf,
    sinr,
    sum_rate,
)
